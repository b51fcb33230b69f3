"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

States are exchanged as values at the Stroud quadrature points, which both
sides compute independently: the GPU projects them to its nodal basis, the
oracle to its modal basis, and results are compared at the same points.
Tolerances: relative L2 <= 1e-12 in FP64, <= 1e-5 in FP32, for states,
right-hand sides, receiver traces (max-norm relative to the largest trace
value) and the energy alike.
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
    # Both sides take the Sec. 4.4 scaling dt = CFL min_K r_K / (max_q c_p (N+1)^2)
    # from the same material values, but the inradius 3|K|/|dK| through
    # different arithmetic (a determinant on the host, cross products in the
    # oracle): about ten rounded operations each, so a few ulps apart.  The
    # bound is 20 ulps of the result.
    assert abs(dt - timestep.cfl_dt(op, 0.5)) <= 20 * np.finfo(float).eps * dt
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
    assert err <= TOL[prec] and terr <= TOL[prec]
    assert abs(E_gpu - E_ref) <= TOL[prec] * E_ref


STEP_SRC = dict(xs=[0.05, -0.10, 0.15], direction=[0.2, -0.3, 0.9], amp=1.7, f0=5.0, t0=0.2)


def _elem_rel_max(op, a, b):
    """Largest per-element relative L2_Q error (localises a wrong element)."""
    w = op.ref.wq[None, None, :] * op.mesh.J[:, None, None]
    num = np.sqrt(np.sum(w * (a - b) ** 2, axis=(1, 2)))
    den = np.sqrt(np.sum(w * b ** 2, axis=(1, 2)))
    return float(np.max(num / np.maximum(den, 1e-300)))


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("N", [1, 2, 3, 4, 5, 7])
def test_step_parity(N, prec):
    """LSRK stepping through the stage kernel (update, mass inverse, source,
    and the in-stage stress projection of every new state) against the
    oracle: shuffled n=3 mesh (all six face orientations), smooth media with
    +-20 % element jumps, Ricker source, random initial state, 30 steps
    (20 at N=7)."""
    torch = _torch()
    from oracle import timestep
    nsteps = 20 if N == 7 else 30
    op, EToV, VXYZ, xyz, mat = oracle_case(N, 3, shuffle_seed=10 + N, jump_seed=200 + N)
    c = _ctx(N, prec, EToV, VXYZ, mat)
    src = timestep.Source(STEP_SRC["xs"], STEP_SRC["direction"], STEP_SRC["amp"], STEP_SRC["f0"], STEP_SRC["t0"])
    c.set_source(src.xs, src.direction, src.amp, src.f0, src.t0)
    fq = np.random.default_rng(50 + N).standard_normal((op.K, 9, op.Nq))
    t0 = 0.1
    c.set_state(c.project_quadrature(torch.from_numpy(fq)), t0)
    dt = c.cfl_dt(0.5)
    c.step(dt, nsteps)
    got = c.eval_quadrature().cpu().numpy()
    cT, T, _ = timestep.run(op, op.project_q(fq), dt, nsteps, t=t0, source=src)
    ref = op.to_q(cT)
    err = _rel_l2(op, got, ref)
    emax = _elem_rel_max(op, got, ref)
    _report("step", N=N, prec=prec, steps=nsteps, rel_l2=err, elem_max=emax)
    assert abs(c.time() - T) <= 1e-14
    assert err <= TOL[prec]
    assert emax <= 10 * TOL[prec]


def _owners(op, x, tol=1e-12):
    """Elements whose closure holds x (all barycentric coordinates >= -tol)."""
    M = op.mesh
    rh = np.einsum('kij,kj->ki', M.rk_x, np.asarray(x, float)[None, :] - M.X[:, 0]) - 1.0
    lam = np.stack([-(rh.sum(axis=1) + 1.0) / 2.0, (rh[:, 0] + 1) / 2, (rh[:, 1] + 1) / 2,
                    (rh[:, 2] + 1) / 2], axis=1)
    return np.nonzero(np.all(lam >= -tol, axis=1))[0]


@pytest.mark.parametrize("prec", [64, 32])
def test_source_and_receivers_on_shared_points(prec):
    """A point on a shared vertex, edge or face belongs to the lowest-index
    element that holds it.  The fields are discontinuous there, so a
    different owner on either side shows up in the traces and (for the
    source) in the state.  Source on a mesh vertex; receivers on a vertex, a
    hexahedron face, an inner Kuhn face and an edge of the n=4 shuffled cube
    (grid spacing 0.5, exact in binary)."""
    torch = _torch()
    from oracle import timestep
    N = 3
    op, EToV, VXYZ, xyz, mat = oracle_case(N, 4, shuffle_seed=21, jump_seed=21)
    xs = [0.0, 0.5, -0.5]
    rec = np.array([[0.5, 0.5, 0.5], [0.25, 0.0, 0.1], [0.1, 0.1, 0.3], [0.5, -0.5, 0.2]])
    for x in [xs] + list(rec):
        assert len(_owners(op, x)) >= 2, x      # every point is shared
    c = _ctx(N, prec, EToV, VXYZ, mat, max_rec=len(rec), max_steps=30)
    src = timestep.Source(xs, [0.3, 0.4, -0.8], 1.0, 5.0, 0.2)
    c.set_source(src.xs, src.direction, src.amp, src.f0, src.t0)
    c.set_receivers(rec)
    dt = c.cfl_dt(0.5)
    t0 = 0.1
    c.set_state(torch.zeros((op.K, 9, op.Np), dtype=torch.float64), t0)
    c.step(dt, 25)
    got = c.eval_quadrature().cpu().numpy()
    cT, T, traces = timestep.run(op, np.zeros((op.K, 9, op.Np)), dt, 25, t=t0, source=src, receivers=rec)
    ref = op.to_q(cT)
    err = _rel_l2(op, got, ref)
    tr = c.receivers()
    terr = np.abs(tr - traces).max() / np.abs(traces).max()
    _report("shared-points", prec=prec, rel_l2=err, trace_err=terr, owners=[len(_owners(op, x)) for x in rec])
    assert err <= TOL[prec] and terr <= TOL[prec]
    assert np.abs(traces).max() > 0


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


def test_context_on_its_own_stream():
    """A context whose stream is not torch's current stream: states,
    projections and right-hand sides passed in and out as device tensors are
    ordered against torch's stream by the binding.  Every result must equal
    bitwise that of a context on torch's current stream."""
    torch = _torch()
    N = 4
    op, EToV, VXYZ, xyz, mat = oracle_case(N, 4, shuffle_seed=6, jump_seed=6)
    fq = np.random.default_rng(11).standard_normal((op.K, 9, op.Nq))
    side = torch.cuda.Stream()
    outs = []
    for stream in (None, side.cuda_stream):
        import paper_1711_01175_amd as P
        c = P.Context(N, 32, stream=stream)
        c.set_mesh(EToV, VXYZ)
        c.bind_workspace()
        c.set_material(*mat)
        # inputs produced on torch's stream right before the calls
        q = c.project_quadrature(torch.from_numpy(fq).cuda() * 1.0)
        r = c.rhs(0.1, q * 1.0)
        c.set_state(q * 1.0, 0.0)
        c.step(c.cfl_dt(0.5), 7)
        s1 = c.get_state()
        s1 = s1 + 0.0                     # consumed on torch's stream at once
        e = c.eval_quadrature()
        outs.append([x.cpu().numpy() for x in (q, r, s1, e)])
        c.close()
    for a, b in zip(*outs):
        assert np.array_equal(a, b)


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
