"""Pins for the oracle's iHDG-II solution of the implicit (theta-scheme) step.

Each test checks the iteration against something other than itself: a
Krylov solve of the global implicit system (no element splitting, no local
matrices), exact discrete energy identities of the theta scheme, its order of
accuracy against the pinned explicit integrator, direct single-element
evaluations of the operator, and the stopping rule of Sec. 6.1.
"""
import numpy as np
import pytest
from scipy.sparse.linalg import LinearOperator, gmres

from helpers import oracle_case
from oracle import timestep
from oracle.ihdg import ImplicitStep, greedy_colouring, l2_norm, local_matrices


def _random_state(op, seed):
    return np.random.default_rng(seed).standard_normal((op.K, 9, op.Np))


@pytest.fixture(scope="module")
def case_n1():
    op, *_ = oracle_case(1, 3, shuffle_seed=3, jump_seed=11)
    return op, local_matrices(op)


def test_colouring_separates_neighbours(case_n1):
    op, _ = case_n1
    col = greedy_colouring(op.mesh.nbr)
    for f in range(4):
        assert np.all(col != col[op.mesh.nbr[:, f]])


def test_local_matrix_is_the_operator_on_one_element(case_n1):
    """Column j of A_K is L applied to the state that is the j-th unit
    coefficient on K alone, evaluated element by element (no colouring)."""
    op, A = case_n1
    n = 9 * op.Np
    for k in (0, 17, op.K - 1):
        for j in (0, 5, n - 1):
            c = np.zeros((op.K, 9, op.Np))
            c[k, j // op.Np, j % op.Np] = 1.0
            col = op.rhs(c, 0.0, elems=[k]).reshape(n)
            assert np.allclose(A[k, :, j], col, rtol=0, atol=1e-13 * np.abs(col).max())


@pytest.mark.parametrize("theta", [1.0, 0.5])
def test_fixed_point_is_the_global_implicit_step(case_n1, theta):
    """Converged iHDG-II equals the solution of the coupled system
    (I - theta dt L) c^{m+1} = c^m + (1 - theta) dt L c^m + dt s_theta,
    solved here by GMRES on the operator as a whole, with a point source."""
    op, A = case_n1
    dt = timestep.cfl_dt(op, 2.0)
    src = timestep.Source((0.05, -0.1, 0.15), (0.3, 0.0, 1.0), 2.0, 5.0, 0.2)
    c0 = _random_state(op, 1)
    t0 = 0.15
    c1, iters, _ = ImplicitStep(op, dt, theta, A=A).step(c0, t0, source=src, tol=1e-13 * l2_norm(op, c0))
    op.set_source(src.xs, src.direction, src.amp)
    s_now = timestep.ricker(t0, src.f0, src.t0)
    s_next = timestep.ricker(t0 + dt, src.f0, src.t0)
    zero = np.zeros_like(c0)
    b = c0 + (1 - theta) * dt * op.rhs(c0, s_now) + theta * dt * op.rhs(zero, s_next)
    M = LinearOperator((c0.size, c0.size), matvec=lambda x: x - theta * dt * op.rhs(x.reshape(c0.shape)).ravel())
    x, info = gmres(M, b.ravel(), rtol=1e-14, atol=0, restart=200, maxiter=50)
    assert info == 0
    assert iters > 2
    assert np.linalg.norm(c1.ravel() - x) <= 1e-12 * np.linalg.norm(x)


@pytest.mark.parametrize("flux", ["upwind", "central"])
@pytest.mark.parametrize("theta", [1.0, 0.5])
def test_theta_scheme_energy_identity(flux, theta):
    """With c_th = theta c^{m+1} + (1 - theta) c^m the scheme reads
    c^{m+1} - c^m = dt L c_th, so in the energy inner product
    E^{m+1} - E^m = dt (L c_th, c_th)_E - (2 theta - 1) E(c^{m+1} - c^m),
    where (L c, c)_E is the closed-form face dissipation (upwind) or zero
    (central, Sec. 2 weighted norms).  Crank-Nicolson with the central flux
    conserves energy exactly."""
    op, *_ = oracle_case(2, 3, shuffle_seed=5, jump_seed=13, flux=flux)
    c0 = _random_state(op, 2)
    dt = timestep.cfl_dt(op, 2.0)
    c1, _, _ = ImplicitStep(op, dt, theta).step(c0, 0.0, tol=1e-14 * l2_norm(op, c0), max_iters=500)
    cth = theta * c1 + (1 - theta) * c0
    rate = op.face_dissipation(cth) if flux == "upwind" else 0.0
    expect = dt * rate - (2 * theta - 1) * op.energy(c1 - c0)
    E0 = op.energy(c0)
    assert abs((op.energy(c1) - E0) - expect) <= 1e-12 * E0
    if flux == "upwind":
        assert op.energy(c1) < E0


def test_theta_scheme_order():
    """Implicit Euler is first order and Crank-Nicolson second order in time:
    halving dt over a fixed interval divides the error against a fine
    LSRK(5,4) run by 2 and by 4."""
    op, _, VXYZ, xyz, _ = oracle_case(2, 3)
    A = local_matrices(op)
    from oracle.reference import stroud_rule
    xq, _ = stroud_rule(2)
    from helpers import quad_points
    pq = quad_points(VXYZ, xq)
    x, y, z = pq[..., 0], pq[..., 1], pq[..., 2]
    fq = np.zeros((op.K, 9, op.Nq))
    fq[:, 0] = np.sin(np.pi * x) * np.cos(np.pi * y)
    fq[:, 1] = np.cos(np.pi * z)
    fq[:, 5] = 0.3 * np.sin(np.pi * (x + y + z))
    c0 = op.project_q(fq)
    dt0 = timestep.cfl_dt(op, 1.0)
    ref, _, _ = timestep.run(op, c0, dt0 / 64, 8 * 64)
    for theta, order in ((1.0, 1), (0.5, 2)):
        errs = []
        for m in (1, 2, 4):
            S = ImplicitStep(op, dt0 / m, theta, A=A)
            c = c0.copy()
            for s in range(8 * m):
                c, _, _ = S.step(c, s * dt0 / m, tol=1e-13, max_iters=500)
            errs.append(l2_norm(op, c - ref))
        for a, b in zip(errs, errs[1:]):
            assert abs(np.log2(a / b) - order) < 0.1, (theta, errs)


def test_stopping_rule_and_growth_with_dt(case_n1):
    """Iteration k reports ||c^k - c^{k-1}||; the loop ends at the first value
    below tol (Sec. 6.1), the differences contract, and a longer step needs
    more iterations (the locally implicit trade-off of Sec. 4.3)."""
    op, A = case_n1
    c0 = _random_state(op, 3)
    tol = 1e-10 * l2_norm(op, c0)
    counts = []
    for cfl in (0.5, 1.0, 2.0, 4.0):
        c1, iters, norms = ImplicitStep(op, timestep.cfl_dt(op, cfl), 1.0, A=A).step(c0, 0.0, tol=tol)
        assert iters == len(norms)
        assert norms[-1] < tol and np.all(norms[:-1] >= tol)
        assert np.all(norms[1:] < norms[:-1])
        counts.append(iters)
    assert counts == sorted(counts) and counts[-1] > counts[0]
    # max_iters caps the loop; one iteration is the locally implicit step
    _, iters, norms = ImplicitStep(op, timestep.cfl_dt(op, 1.0), 1.0, A=A).step(c0, 0.0, tol=tol, max_iters=1)
    assert iters == 1 and norms[0] > tol
