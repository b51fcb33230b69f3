"""GPU parity of the locally implicit step (theta scheme solved by iHDG-II)
against the oracle's iHDG-II, through the C ABI.

Both sides run the same iteration from the same initial guess: the GPU on
its nodal basis with local inverses probed through its own operator kernels,
the oracle on its modal basis.  Iterates are the same functions up to
rounding, so in FP64 the iteration counts agree exactly and the states to
rounding (bar 1e-11 relative L2 at the quadrature points, after the
stopping tolerance of 1e-11 relative to the initial state).  In FP32 the
stopping test sees rounding of about 1e-7 of the state, so the tolerance is
1e-6 relative, counts may differ by one iteration and the states are held to
1e-5.
"""
import numpy as np
import pytest
import torch  # noqa: F401  (imported at collection, outside the per-test time limit)

from helpers import oracle_case

pytestmark = pytest.mark.gpu

TOL = {64: 1e-11, 32: 1e-5}
STOP = {64: 1e-11, 32: 1e-6}
SRC = dict(xs=(0.05, -0.10, 0.15), direction=(0.2, -0.3, 0.9), amp=1.7, f0=5.0, t0=0.2)
_CASES = {}


def _case(N):
    """Oracle operator, its local matrices and the seeded initial values."""
    if N not in _CASES:
        from oracle.ihdg import local_matrices
        op, EToV, VXYZ, xyz, mat = oracle_case(N, 3, shuffle_seed=N, jump_seed=200 + N)
        fq = np.random.default_rng(300 + N).standard_normal((op.K, 9, op.Nq))
        _CASES[N] = (op, EToV, VXYZ, mat, fq, local_matrices(op))
    return _CASES[N]


def _ctx(N, prec, EToV, VXYZ, mat, max_rec=0, max_steps=0):
    import paper_1711_01175_amd as P
    c = P.Context(N, prec)
    c.set_mesh(EToV, VXYZ)
    c.bind_workspace(max_rec, max_steps)
    c.set_material(*mat)
    c.bind_implicit_workspace()
    return c


def _report(name, **kw):
    print(name, " ".join(f"{k}={v:.3e}" if isinstance(v, float) else f"{k}={v}" for k, v in kw.items()),
          flush=True)


def _oracle_steps(op, A, c0, t0, dt, theta, nsteps, tol, receivers=None):
    from oracle import timestep
    from oracle.ihdg import ImplicitStep
    S = ImplicitStep(op, dt, theta, A=A)
    src = timestep.Source(**SRC)
    c, counts, last, traces = c0, [], [], []
    for s in range(nsteps):
        c, it, norms = S.step(c, t0 + s * dt, source=src, tol=tol, max_iters=200)
        counts.append(it)
        last.append(norms)
        if receivers is not None:
            traces.append(op.eval_points(c, receivers)[:, 0:3])
    return c, counts, last, (np.array(traces) if receivers is not None else None)


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("theta", [1.0, 0.5])
@pytest.mark.parametrize("N", [1, 2, 3, 4])
def test_implicit_step_parity(N, theta, prec):
    """Three steps at CFL 2 with a Ricker source on the jump medium of 162
    shuffled tets: states, iteration counts and final changes."""
    op, EToV, VXYZ, mat, fq, A = _case(N)
    from oracle.ihdg import l2_norm
    c = _ctx(N, prec, EToV, VXYZ, mat)
    c.set_source(SRC["xs"], SRC["direction"], SRC["amp"], SRC["f0"], SRC["t0"])
    dt = c.cfl_dt(2.0)
    c.implicit_setup(dt, theta)
    t0 = 0.1
    c.set_state(c.project_quadrature(torch.from_numpy(fq)), t0)
    c0 = op.project_q(fq)
    tol = STOP[prec] * l2_norm(op, c0)
    iters, change = c.implicit_step(3, tol, 200)
    got = c.eval_quadrature().cpu().numpy()
    cT, counts, norms, _ = _oracle_steps(op, A, c0, t0, dt, theta, 3, tol)
    ref = op.to_q(cT)
    err = op.l2_q(got - ref) / op.l2_q(ref)
    _report("implicit", N=N, theta=theta, prec=prec, rel_l2=err, iters=list(iters), oracle=counts)
    assert abs(c.time() - (t0 + 3 * dt)) < 1e-14
    assert np.all(change < tol) and np.all(iters < 200)
    assert err <= TOL[prec]
    if prec == 64:
        # a count could only differ if a change fell within rounding of tol
        margin = min(min(abs(x / tol - 1.0) for x in nr[-2:]) for nr in norms)
        if margin > 1e-6:
            assert list(iters) == counts
        # the last change is ~1e-11 of the state, so rounding of the state
        # (~1e-16 of it) is ~1e-5 of the change
        assert np.allclose(change, [nr[-1] for nr in norms], rtol=1e-3, atol=0)
    else:
        assert np.all(np.abs(np.array(iters) - np.array(counts)) <= 1)


@pytest.mark.parametrize("prec", [64, 32])
def test_implicit_receivers_energy_and_explicit_continuation(prec):
    """Crank-Nicolson at CFL 4 for 6 steps with receivers (recorded after
    every implicit step), then 5 explicit LSRK steps from the implicit state:
    traces, energy and the final state against the oracle."""
    from oracle import timestep
    from oracle.ihdg import l2_norm
    N = 3
    op, EToV, VXYZ, mat, fq, A = _case(N)
    rec = np.array([[0.1, 0.1, 0.1], [-0.5, 0.3, 0.77], [0.05, -0.10, 0.15]])
    c = _ctx(N, prec, EToV, VXYZ, mat, max_rec=len(rec), max_steps=16)
    c.set_source(SRC["xs"], SRC["direction"], SRC["amp"], SRC["f0"], SRC["t0"])
    c.set_receivers(rec)
    dt = c.cfl_dt(4.0)
    c.implicit_setup(dt, 0.5)
    assert c.implicit_dt() == (dt, 0.5)
    t0 = 0.05
    c.set_state(c.project_quadrature(torch.from_numpy(fq)), t0)
    c0 = op.project_q(fq)
    tol = STOP[prec] * l2_norm(op, c0)
    iters, _ = c.implicit_step(6, tol, 200)
    E_imp = c.energy()
    dte = c.cfl_dt(0.5)
    c.step(dte, 5)
    got = c.eval_quadrature().cpu().numpy()
    cI, counts, _, traces = _oracle_steps(op, A, c0, t0, dt, 0.5, 6, tol, receivers=rec)
    E_ref = op.energy(cI)
    cT, _, tr2 = timestep.run(op, cI, dte, 5, t=t0 + 6 * dt, source=timestep.Source(**SRC), receivers=rec)
    ref = op.to_q(cT)
    err = op.l2_q(got - ref) / op.l2_q(ref)
    tr = c.receivers()
    want = np.concatenate([traces, tr2])
    terr = np.abs(tr - want).max() / np.abs(want).max()
    _report("implicit+explicit", prec=prec, rel_l2=err, trace_err=terr, E=E_imp, E_ref=E_ref,
            iters=list(iters), oracle=counts)
    assert tr.shape == want.shape
    assert err <= TOL[prec] and terr <= TOL[prec]
    assert abs(E_imp - E_ref) <= TOL[prec] * E_ref


def test_implicit_call_order_errors():
    import paper_1711_01175_amd as P
    op, EToV, VXYZ, mat, fq, A = _case(1)
    c = P.Context(1, 64)
    c.set_mesh(EToV, VXYZ)
    assert c.implicit_workspace_bytes() > 0
    c.bind_workspace()
    c.set_material(*mat)
    with pytest.raises(P.EwdgError):
        c.implicit_setup(1e-3, 1.0)           # no implicit workspace yet
    c.bind_implicit_workspace()
    with pytest.raises(P.EwdgError):
        c.implicit_step(1, 1e-10, 10)          # no set-up yet
    for dt, th in ((0.0, 1.0), (1e-3, 0.0), (1e-3, 1.5)):
        with pytest.raises(P.EwdgError):
            c.implicit_setup(dt, th)
    c.implicit_setup(c.cfl_dt(1.0), 1.0)
    c.set_state(c.project_quadrature(torch.from_numpy(fq)), 0.0)
    iters, change = c.implicit_step(1, 1e-300, 2)   # capped: keeps the last iterate
    assert list(iters) == [2] and change[0] > 0
    c.set_material(*mat)                           # new material: set-up again
    with pytest.raises(P.EwdgError):
        c.implicit_step(1, 1e-10, 10)
