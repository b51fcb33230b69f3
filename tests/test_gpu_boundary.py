"""GPU parity on bounded meshes (traction-free and absorbing boundary faces)
against the oracle, through the C ABI: the operator at every degree, stepping
with a source, the traction-free standing wave against its exact solution,
the locally implicit step, and the refusals of the periodic-only paths.
Bars as for periodic meshes: relative L2 1e-12 (FP64), 1e-5 (FP32).
"""
import numpy as np
import pytest
import torch  # noqa: F401  (imported at collection, outside the per-test time limit)

from test_oracle_boundary import _standing, bounded_case

pytestmark = pytest.mark.gpu

TOL = {64: 1e-12, 32: 1e-5}
SRC = dict(xs=[0.05, -0.10, 0.15], direction=[0.2, -0.3, 0.9], amp=1.7, f0=5.0, t0=0.2)


def _ctx(N, prec, EToV, VXYZ, mat, bc):
    import paper_1711_01175_amd as P
    c = P.Context(N, prec)
    c.set_mesh(EToV, VXYZ, boundary=bc)
    c.bind_workspace()
    c.set_material(*mat)
    return c


def _report(name, **kw):
    print(name, " ".join(f"{k}={v:.3e}" if isinstance(v, float) else f"{k}={v}" for k, v in kw.items()),
          flush=True)


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("bc", ["free", "absorbing"])
@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 7])
def test_bounded_rhs_parity(N, bc, prec):
    op, EToV, VXYZ, xyz, mat = bounded_case(N, 3, bc, shuffle_seed=N, jump_seed=40 + N)
    c = _ctx(N, prec, EToV, VXYZ, mat, bc)
    fq = np.random.default_rng(N).standard_normal((op.K, 9, op.Nq))
    c.set_source(SRC["xs"], SRC["direction"], SRC["amp"], SRC["f0"], SRC["t0"])
    op.set_source(SRC["xs"], SRC["direction"], SRC["amp"])
    from oracle.timestep import ricker
    t = 0.23
    got = c.eval_quadrature(c.rhs(t, c.project_quadrature(torch.from_numpy(fq)))).cpu().numpy()
    ref = op.to_q(op.rhs(op.project_q(fq), src_value=ricker(t, SRC["f0"], SRC["t0"])))
    err = op.l2_q(got - ref) / op.l2_q(ref)
    _report("bounded rhs", N=N, bc=bc, prec=prec, rel_l2=err)
    assert err <= TOL[prec]


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("bc", ["free", "absorbing"])
@pytest.mark.parametrize("N", [2, 4, 5])
def test_bounded_step_parity(N, bc, prec):
    """20 LSRK steps with the source from a random state: the in-stage
    projection and the boundary gathers of the stepping kernel."""
    from oracle import timestep
    op, EToV, VXYZ, xyz, mat = bounded_case(N, 3, bc, shuffle_seed=10 + N, jump_seed=50 + N)
    c = _ctx(N, prec, EToV, VXYZ, mat, bc)
    fq = np.random.default_rng(60 + N).standard_normal((op.K, 9, op.Nq))
    src = timestep.Source(**SRC)
    c.set_source(src.xs, src.direction, src.amp, src.f0, src.t0)
    t0 = 0.1
    c.set_state(c.project_quadrature(torch.from_numpy(fq)), t0)
    dt = c.cfl_dt(0.5)
    c.step(dt, 20)
    got = c.eval_quadrature().cpu().numpy()
    cT, T, _ = timestep.run(op, op.project_q(fq), dt, 20, t=t0, source=src)
    ref = op.to_q(cT)
    err = op.l2_q(got - ref) / op.l2_q(ref)
    E_gpu, E_ref = c.energy(), op.energy(cT)
    _report("bounded step", N=N, bc=bc, prec=prec, rel_l2=err, E_gpu=E_gpu, E_ref=E_ref)
    assert err <= TOL[prec]
    assert abs(E_gpu - E_ref) <= TOL[prec] * E_ref


def test_traction_free_standing_wave_on_the_gpu():
    """lambda = 0: the standing P-wave is an exact traction-free solution;
    FP64 GPU against the exact wave after half a time unit (n = 4, N = 3)."""
    from helpers import quad_points
    from oracle.dg import Elastic
    from oracle.reference import stroud_rule
    from workloads.mesh import kuhn_box_mesh
    N, n = 3, 4
    EToV, VXYZ = kuhn_box_mesh(n)
    xq, _ = stroud_rule(N)
    xyz = quad_points(VXYZ, xq)
    one = np.ones(xyz.shape[:2])
    op = Elastic(N, VXYZ, one, 0 * one, one, boundary="free")
    c = _ctx(N, 64, EToV, VXYZ, (one, 0 * one, one), "free")
    c.set_state(c.project_quadrature(torch.from_numpy(_standing(op, xyz, 0.0))), 0.0)
    dt = c.cfl_dt(0.5)
    steps = int(round(0.5 / dt))
    c.step(dt, steps)
    got = c.eval_quadrature().cpu().numpy()
    ex = _standing(op, xyz, c.time())
    err = op.l2_q(got - ex) / op.l2_q(ex)
    _report("standing wave", rel_l2=err, t=c.time())
    assert err < 2e-3


def test_bounded_implicit_step_parity():
    """Crank-Nicolson at CFL 2 on the traction-free box: the implicit set-up
    probes the boundary operator through the same kernels."""
    from oracle.ihdg import ImplicitStep, l2_norm
    N = 2
    op, EToV, VXYZ, xyz, mat = bounded_case(N, 3, "free", shuffle_seed=7, jump_seed=8)
    c = _ctx(N, 64, EToV, VXYZ, mat, "free")
    c.bind_implicit_workspace()
    dt = c.cfl_dt(2.0)
    c.implicit_setup(dt, 0.5)
    fq = np.random.default_rng(9).standard_normal((op.K, 9, op.Nq))
    c.set_state(c.project_quadrature(torch.from_numpy(fq)), 0.0)
    c0 = op.project_q(fq)
    tol = 1e-11 * l2_norm(op, c0)
    iters, _ = c.implicit_step(2, tol, 200)
    S = ImplicitStep(op, dt, 0.5)
    cc, counts = c0, []
    for s in range(2):
        cc, it, _ = S.step(cc, s * dt, tol=tol)
        counts.append(it)
    got = c.eval_quadrature().cpu().numpy()
    ref = op.to_q(cc)
    err = op.l2_q(got - ref) / op.l2_q(ref)
    _report("bounded implicit", rel_l2=err, iters=list(iters), oracle=counts)
    assert err <= 1e-11 and list(iters) == counts


def test_periodic_only_paths_refuse_bounded_meshes():
    import paper_1711_01175_amd as P
    op, EToV, VXYZ, xyz, mat = bounded_case(2, 3, "absorbing")
    c = _ctx(2, 32, EToV, VXYZ, mat, "absorbing")
    with pytest.raises(P.EwdgError):
        c.bind_adjoint_workspace(10, 5)
    table = torch.empty(P.batch_table_bytes(1), dtype=torch.uint8, device="cuda")
    with pytest.raises(P.EwdgError):
        P.step_batch([c], [1e-3], 1, table)
