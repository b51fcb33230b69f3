"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

States are exchanged as values at the Stroud quadrature points, which both
sides compute independently: the GPU projects them to its nodal basis, the
oracle to its modal basis, and results are compared at the same points.
Tolerances: relative L2 <= 1e-12 in FP64, <= 1e-5 in FP32.
"""
import numpy as np
import pytest
import torch  # noqa: F401  (imported at collection, outside the per-test time limit)

from helpers import oracle_case

pytestmark = pytest.mark.gpu

TOL = {64: 1e-12, 32: 1e-5}


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch


def _ctx(N, prec, EToV, VXYZ, mat, max_rec=0, max_steps=0):
    import paper_1711_01175_amd as P
    c = P.Context(N, prec)
    c.set_mesh(EToV, VXYZ)
    c.bind_workspace(max_rec, max_steps)
    c.set_material(*mat)
    return c


def _rel_l2(op, a, b):
    return op.l2_q(a - b) / op.l2_q(b)


def _report(name, **kw):
    print(name, " ".join(f"{k}={v:.3e}" if isinstance(v, float) else f"{k}={v}" for k, v in kw.items()),
          flush=True)


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 7])
def test_rhs_parity(N, prec):
    torch = _torch()
    op, EToV, VXYZ, xyz, mat = oracle_case(N, 3, shuffle_seed=N, jump_seed=100 + N)
    c = _ctx(N, prec, EToV, VXYZ, mat)
    rng = np.random.default_rng(N)
    fq = rng.standard_normal((op.K, 9, op.Nq))
    src = dict(xs=[0.05, -0.10, 0.15], direction=[0.2, -0.3, 0.9], amp=1.7, f0=5.0, t0=0.2)
    c.set_source(src["xs"], src["direction"], src["amp"], src["f0"], src["t0"])
    op.set_source(src["xs"], src["direction"], src["amp"])
    t = 0.23
    from oracle.timestep import ricker
    q = c.project_quadrature(torch.from_numpy(fq))
    got = c.eval_quadrature(c.rhs(t, q)).cpu().numpy()
    ref = op.to_q(op.rhs(op.project_q(fq), src_value=ricker(t, src["f0"], src["t0"])))
    err = _rel_l2(op, got, ref)
    _report("rhs", N=N, prec=prec, rel_l2=err)
    assert err <= TOL[prec]


def _pwave(xyz, t):
    cp = np.sqrt(3.0)
    ph = np.pi * (xyz[..., 0] - cp * t)
    out = np.zeros(xyz.shape[:-1] + (9,))
    out[..., 0] = np.cos(ph)
    out[..., 3] = -np.cos(ph) / cp
    return np.moveaxis(out, -1, 1)


@pytest.mark.parametrize("prec", [64, 32])
def test_periodic_cube_pwave_200_steps(prec):
    """Homogeneous periodic cube, 384 tets, N=3, P-plane wave, 200 LSRK
    steps at CFL 0.5: GPU state vs oracle state, and both vs the exact wave."""
    torch = _torch()
    from oracle import timestep
    N, n, steps = 3, 4, 200
    op, EToV, VXYZ, xyz, mat = oracle_case(N, n, medium="homogeneous")
    c = _ctx(N, prec, EToV, VXYZ, mat)
    dt = c.cfl_dt(0.5)
    assert abs(dt - timestep.cfl_dt(op, 0.5)) <= 1e-13 * dt
    f0 = _pwave(xyz, 0.0)
    c.set_state(c.project_quadrature(torch.from_numpy(f0)), 0.0)
    c.step(dt, steps)
    got = c.eval_quadrature().cpu().numpy()
    cT, T, _ = timestep.run(op, op.project_q(f0), dt, steps)
    ref = op.to_q(cT)
    err = _rel_l2(op, got, ref)
    exact = _pwave(xyz, T)
    _report("pwave", prec=prec, rel_l2=err, disc_err=_rel_l2(op, ref, exact), t=T)
    assert abs(c.time() - T) < 1e-14
    assert err <= TOL[prec]
    assert _rel_l2(op, got, exact) < 2e-3


@pytest.mark.parametrize("prec", [64, 32])
def test_receivers_energy_source(prec):
    """Heterogeneous medium with element jumps, Ricker source, receivers and
    energy over 30 steps."""
    torch = _torch()
    from oracle import timestep
    N = 3
    op, EToV, VXYZ, xyz, mat = oracle_case(N, 3, shuffle_seed=9, jump_seed=9)
    rec = np.array([[0.1, 0.1, 0.1], [-0.5, 0.3, 0.77], [0.9, -0.9, 0.0], [0.0, 0.0, 0.0]])
    c = _ctx(N, prec, EToV, VXYZ, mat, max_rec=len(rec), max_steps=40)
    src = timestep.Source([0.05, -0.10, 0.15], [0.0, 0.0, 1.0], 1.0, 5.0, 0.2)
    c.set_source(src.xs, src.direction, src.amp, src.f0, src.t0)
    c.set_receivers(rec)
    dt = c.cfl_dt(0.5)
    # start after the wavelet's onset so that it carries signal
    t0 = 0.1
    c.set_state(torch.zeros((op.K, 9, op.Np), dtype=torch.float64), t0)
    c.step(dt, 30)
    got = c.eval_quadrature().cpu().numpy()
    cT, T, traces = timestep.run(op, np.zeros((op.K, 9, op.Np)), dt, 30, t=t0, source=src, receivers=rec)
    ref = op.to_q(cT)
    err = _rel_l2(op, got, ref)
    tr = c.receivers()
    terr = np.abs(tr - traces).max() / np.abs(traces).max()
    E_gpu, E_ref = c.energy(), op.energy(cT)
    _report("src", prec=prec, rel_l2=err, trace_err=terr, E_gpu=E_gpu, E_ref=E_ref)
    assert tr.shape == traces.shape
    assert err <= TOL[prec] and terr <= 10 * TOL[prec]
    assert abs(E_gpu - E_ref) <= 10 * TOL[prec] * E_ref


def test_determinism_and_element_permutation():
    """Two identical runs are bitwise equal; relabelling elements permutes
    the result bitwise (each element's arithmetic does not depend on where it
    sits in memory)."""
    torch = _torch()
    N = 4
    op, EToV, VXYZ, xyz, mat = oracle_case(N, 3, shuffle_seed=4, jump_seed=4)
    fq = np.random.default_rng(3).standard_normal((op.K, 9, op.Nq))
    outs = []
    for _ in range(2):
        c = _ctx(N, 64, EToV, VXYZ, mat)
        c.set_state(c.project_quadrature(torch.from_numpy(fq)), 0.0)
        c.step(c.cfl_dt(0.5), 5)
        outs.append(c.get_state().cpu().numpy())
    assert np.array_equal(outs[0], outs[1])
    perm = np.random.default_rng(0).permutation(op.K)
    mat_p = tuple(m[perm] for m in mat)
    c = _ctx(N, 64, EToV[perm], VXYZ[perm], mat_p)
    c.set_state(c.project_quadrature(torch.from_numpy(fq[perm])), 0.0)
    c.step(c.cfl_dt(0.5), 5)
    assert np.array_equal(c.get_state().cpu().numpy(), outs[0][perm])


@pytest.mark.parametrize("prec", [64, 32])
def test_constant_state_is_steady(prec):
    """Degenerate case: a constant state in a homogeneous medium has zero
    right-hand side (no gradients, no jumps)."""
    torch = _torch()
    from workloads import media
    from workloads.mesh import kuhn_periodic_mesh
    EToV, VXYZ = kuhn_periodic_mesh(3, shuffle_seed=5)
    import paper_1711_01175_amd as P
    c = P.Context(4, prec)
    c.set_mesh(EToV, VXYZ)
    c.bind_workspace()
    c.set_material(*media.homogeneous(c.quadrature_points(), 1.3, 0.7, 1.1))
    vals = np.array([0.3, -1.2, 0.5, 0.2, -0.1, 0.4, 0.15, -0.25, 0.05])
    fq = torch.from_numpy(np.broadcast_to(vals[None, :, None], (c.K, 9, c.Nq)).copy())
    q = c.project_quadrature(fq)
    r = c.rhs(0.0, q)
    # the exact value is 0; what remains is rounding of derivative and lift
    # sums, of size eps * (operator scale) * |q|, the operator scale taken as
    # |L x| / |x| for a random state x
    x = torch.randn_like(q)
    op_scale = float(c.rhs(0.0, x).abs().max() / x.abs().max())
    scale = float(q.abs().max())
    eps = 2.2e-16 if prec == 64 else 1.2e-7
    _report("steady", prec=prec, max_rhs=float(r.abs().max()), scale=scale, op_scale=op_scale)
    assert float(r.abs().max()) <= 1000 * eps * op_scale * scale


def test_zero_steps_and_error_paths():
    torch = _torch()
    import paper_1711_01175_amd as P
    from workloads import media
    from workloads.mesh import kuhn_periodic_mesh
    EToV, VXYZ = kuhn_periodic_mesh(3)
    c = P.Context(3, 32)
    c.set_mesh(EToV, VXYZ)
    c.bind_workspace(max_receivers=1, max_record_steps=2)
    c.set_material(*media.smooth(c.quadrature_points()))
    q0 = torch.randn((c.K, 9, c.Np), dtype=torch.float32, device="cuda",
                     generator=torch.Generator(device="cuda").manual_seed(3))
    c.set_state(q0, 0.25)
    dt = c.cfl_dt(0.5)
    c.step(dt, 0)
    assert torch.equal(c.get_state(), q0) and c.time() == 0.25
    for bad in ((0.0, 1), (-dt, 1), (dt, -1)):
        with pytest.raises(P.EwdgError) as e:
            c.step(*bad)
        assert e.value.code == P.ewdg.EWDG_EINVAL
    with pytest.raises(P.EwdgError) as e:
        c.set_receivers(np.zeros((2, 3)))                  # more than the workspace holds
    assert e.value.code == P.ewdg.EWDG_ENOMEM
    with pytest.raises(P.EwdgError) as e:
        c.set_receivers(np.array([[3.0, 0.0, 0.0]]))       # outside the cube
    assert e.value.code == P.ewdg.EWDG_EPOINT
    c.set_receivers(np.array([[0.1, 0.2, 0.3]]))
    c.step(dt, 2)
    with pytest.raises(P.EwdgError) as e:
        c.step(dt, 1)                                      # record capacity exhausted
    assert e.value.code == P.ewdg.EWDG_ENOMEM
    assert c.receivers().shape == (2, 1, 3)
