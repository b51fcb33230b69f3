"""Pins for the oracle's semi-discrete operator L(q).

Each test checks the oracle against something other than itself: the
closed-form energy dissipation of the upwind interface state, the paper's
eliminated upwind HDG flux built from an eigendecomposition of A(n),
conservation laws, exact polynomial states and a mesh symmetry.
"""
import numpy as np
import pytest

from helpers import oracle_case, quad_points
from oracle.dg import VOIGT
from workloads.mesh import hex_translation_permutation


def _random_state(op, seed):
    return np.random.default_rng(seed).standard_normal((op.K, 9, op.Np))


@pytest.mark.parametrize("N,n", [(1, 3), (2, 3), (3, 3), (4, 3), (7, 3)])
def test_energy_rate_equals_face_dissipation(N, n):
    """dE/dt = -sum_faces int sum_modes ([T]^2 + Z^-Z^+[v]^2)/(Z^-+Z^+),
    derived by hand from the interface states; holds for any state and any
    positive impedances, here with per-element material jumps."""
    op, *_ = oracle_case(N, n, shuffle_seed=3, jump_seed=11)
    c = _random_state(op, 1)
    rate = op.energy_rate(c, op.rhs(c))
    closed = op.face_dissipation(c)
    assert closed < 0
    assert abs(rate - closed) <= 1e-12 * abs(closed)


@pytest.mark.parametrize("N", [1, 3])
def test_central_flux_conserves_energy(N):
    op, *_ = oracle_case(N, 3, shuffle_seed=4, jump_seed=12, flux="central")
    c = _random_state(op, 2)
    rate = op.energy_rate(c, op.rhs(c))
    assert abs(rate) <= 1e-13 * op.energy(c)


def test_momentum_conserved_and_source_impulse():
    op, *_ = oracle_case(3, 3, shuffle_seed=5, jump_seed=13)
    c = _random_state(op, 3)
    P0 = op.momentum(op.rhs(c))
    scale = np.abs(op.rhs(c)).max()
    assert np.abs(P0).max() < 1e-12 * scale
    op.set_source([0.05, -0.10, 0.15], [0.3, -0.2, 0.9], amp=2.5)
    P1 = op.momentum(op.rhs(c, src_value=0.7))
    assert np.allclose(P1 - P0, 0.7 * 2.5 * np.array([0.3, -0.2, 0.9]), rtol=0, atol=1e-11)


def test_constant_states_are_steady():
    op, *_ = oracle_case(2, 3, medium="homogeneous", shuffle_seed=6)
    c = np.zeros((op.K, 9, op.Np))
    # the constant function 1 has coefficients project_q(1)
    one = op.project_q(np.ones(op.Nq))
    rng = np.random.default_rng(5)
    vals = rng.standard_normal(9)
    c[:] = vals[None, :, None] * one[None, None, :]
    assert np.abs(op.rhs(c)).max() < 1e-12
    # heterogeneous medium: constant velocity with zero strain is steady
    op2, *_ = oracle_case(2, 3, jump_seed=9)
    c2 = np.zeros((op2.K, 9, op2.Np))
    c2[:, 0:3] = vals[None, 0:3, None] * one[None, None, :]
    assert np.abs(op2.rhs(c2)).max() < 1e-12


def _monomials(deg, count, rng):
    """count distinct exponent triples (a, b, c) with a + b + c <= deg,
    always including every monomial of total degree exactly deg along one
    axis so that the top degree is exercised."""
    allm = [(a, b, c) for a in range(deg + 1) for b in range(deg + 1 - a) for c in range(deg + 1 - a - b)]
    pick = [allm[i] for i in rng.choice(len(allm), size=min(count, len(allm)), replace=False)]
    for top in ((deg, 0, 0), (0, deg, 0), (0, 0, deg), (deg - 1, 1, 0) if deg > 1 else (1, 0, 0)):
        if top not in pick:
            pick.append(top)
    return pick


@pytest.mark.parametrize("N,deg", [(3, 2), (3, 3), (4, 4), (7, 7)])
def test_polynomial_states_give_the_pde_operator(N, deg):
    """A global polynomial state of degree <= N is continuous, so away from
    the periodic seam every jump vanishes and L equals the PDE operator
    exactly (the derivatives of a degree-N polynomial are exact on P_N)."""
    n = 4
    op, EToV, VXYZ, xyz, (rho, lam, mu) = oracle_case(N, n, medium="homogeneous")
    rng = np.random.default_rng(8 + N + deg)
    mons = _monomials(deg, 8, rng)
    Cq = rng.standard_normal((9, len(mons)))

    def basis(x, dk=None):
        cols = []
        for (a, b, c) in mons:
            e = [a, b, c]
            coef = 1.0
            if dk is not None:
                coef = e[dk]
                e[dk] = max(e[dk] - 1, 0)
            cols.append(coef * x[..., 0] ** e[0] * x[..., 1] ** e[1] * x[..., 2] ** e[2])
        return np.stack(cols, -1)

    fields = np.einsum('kqb,fb->kfq', basis(xyz), Cq)
    c = op.project_q(fields)
    L = op.rhs(c)
    grads = np.stack([np.einsum('kqb,fb->kfq', basis(xyz, k), Cq) for k in range(3)], 2)
    # exact: v_t = div(C e) / rho, e_t = sym grad v (rho = lambda = mu = 1)
    de = grads[:, 3:9]                          # d_k e_m
    dtr = de[:, 0] + de[:, 1] + de[:, 2]        # [K][3 dir][Nq]
    vt = np.zeros((op.K, 3, op.Nq))
    for m, (i, j) in enumerate(VOIGT):
        if i == j:
            vt[:, i] += 2.0 * de[:, m, i]
        else:
            vt[:, i] += 2.0 * de[:, m, j]
            vt[:, j] += 2.0 * de[:, m, i]
    for i in range(3):
        vt[:, i] += dtr[:, i]
    gv = grads[:, 0:3]                          # [K][comp][dir][Nq]
    et = np.stack([0.5 * (gv[:, i, j] + gv[:, j, i]) for (i, j) in VOIGT], 1)
    exact = op.project_q(np.concatenate([vt, et], axis=1))
    interior = np.all(np.abs(VXYZ) < 1 - 1e-12, axis=(1, 2))
    assert interior.sum() > 0
    err = np.abs(L[interior] - exact[interior]).max()
    # at the seam the polynomial jumps, so some boundary element must differ
    # (the check is not vacuous)
    assert np.abs(L[~interior] - exact[~interior]).max() > 1e-6 * np.abs(exact).max()
    assert err < 1e-11 * np.abs(exact).max()


def test_translation_symmetry():
    """Shifting the state by one hexahedron shifts L(q) the same way."""
    N, n = 2, 3
    op, EToV, VXYZ, xyz, _ = oracle_case(N, n, medium="homogeneous")
    h = 2.0 / n

    def field(x):
        k = np.pi * np.array([1.0, 2.0, -1.0])
        ph = x @ k
        return np.stack([np.cos(ph + m) for m in range(9)], axis=1)

    c = op.project_q(field(xyz))
    c_shift = op.project_q(field(xyz - np.array([h, 0, 0])))
    perm = hex_translation_permutation(n, (1, 0, 0))
    L = op.rhs(c)
    Ls = op.rhs(c_shift)
    assert np.abs(Ls[perm] - L).max() < 1e-12 * np.abs(L).max()


def _flux_jacobian(nvec, rho, lam, mu):
    """A(n) = sum_k n_k A_k for u = (v, e_Voigt) written as
    du/dt + sum_k d_k (A_k u) = 0 (Sec. 2, eq. LPDE, C = 0)."""
    A = np.zeros((9, 9))
    for col in range(9):
        u = np.zeros(9)
        u[col] = 1.0
        v, e6 = u[:3], u[3:]
        eps = np.zeros((3, 3))
        for m, (i, j) in enumerate(VOIGT):
            eps[i, j] = eps[j, i] = e6[m]
        sig = lam * np.trace(eps) * np.eye(3) + 2 * mu * eps
        out = np.zeros(9)
        out[:3] = -(sig @ nvec) / rho
        sym = 0.5 * (np.outer(v, nvec) + np.outer(nvec, v))
        out[3:] = [-sym[i, j] for (i, j) in VOIGT]
        A[:, col] = out
    return A


def test_interface_state_is_the_upwind_hdg_flux():
    """With equal materials the correction (T*-T^-)/rho, sym(n (x) (v*-v^-))
    equals F(u^-).n - F^.n with F^.n = 1/2 A (u^- + u^+) + 1/2 |A| (u^- - u^+),
    |A| = R |S| R^-1 from a numerical eigendecomposition (Sec. 2, eq.
    RiemannFluxBoth with u^ from eq. HDGeqn)."""
    op, *_ = oracle_case(1, 3)
    rng = np.random.default_rng(21)
    rho, lam, mu = 1.3, 2.1, 0.7
    zp, zs = np.sqrt(rho * (lam + 2 * mu)), np.sqrt(rho * mu)
    for trial in range(20):
        nvec = rng.standard_normal(3)
        nvec /= np.linalg.norm(nvec)
        um, up = rng.standard_normal(9), rng.standard_normal(9)

        def traction(u):
            eps = np.zeros((3, 3))
            for m, (i, j) in enumerate(VOIGT):
                eps[i, j] = eps[j, i] = u[3 + m]
            return (lam * np.trace(eps) * np.eye(3) + 2 * mu * eps) @ nvec

        Tm, Tp = traction(um), traction(up)
        Ts, vs = op._riemann(um[:3], Tm, up[:3], Tp, nvec, zp, zp, zs, zs)
        w = vs - um[:3]
        got = np.concatenate([(Ts - Tm) / rho,
                              [0.5 * (nvec[i] * w[j] + nvec[j] * w[i]) for (i, j) in VOIGT]])
        A = _flux_jacobian(nvec, rho, lam, mu)
        S, Rm = np.linalg.eig(A)
        absA = np.real(Rm @ np.diag(np.abs(S)) @ np.linalg.inv(Rm))
        Fhat = 0.5 * A @ (um + up) + 0.5 * absA @ (um - up)
        ref = A @ um - Fhat
        assert np.abs(got - ref).max() < 1e-12 * max(1, np.abs(ref).max())
    # the eigenvalues are the wave speeds +-c_p, +-c_s (twice) and 0 (three times)
    ev = np.sort(np.real(np.linalg.eigvals(_flux_jacobian(np.array([0, 0, 1.0]), rho, lam, mu))))
    cp, cs = np.sqrt((lam + 2 * mu) / rho), np.sqrt(mu / rho)
    assert np.allclose(ev, np.sort([-cp, -cs, -cs, 0, 0, 0, cs, cs, cp]))


def test_riemann_picks_upstream_state():
    op, *_ = oracle_case(1, 3)
    rng = np.random.default_rng(3)
    n = np.array([0.0, 0.6, 0.8])
    z = 1.7
    vm, vp = rng.standard_normal(3), rng.standard_normal(3)
    Tm, Tp = -z * vm, -z * vp                     # purely right-going (along +n) waves
    Ts, vs = op._riemann(vm, Tm, vp, Tp, n, z, z, z, z)
    assert np.allclose(Ts, Tm) and np.allclose(vs, vm)
    Ts, vs = op._riemann(vm, z * vm, vm, z * vm, n, 1.0, 3.0, 0.5, 2.0)
    assert np.allclose(Ts, z * vm) and np.allclose(vs, vm)   # no jump, no correction


def test_energy_non_increasing_over_steps():
    from oracle import timestep
    op, *_ = oracle_case(2, 3, shuffle_seed=2, jump_seed=5)
    c = 1e-3 * _random_state(op, 9)
    dt = timestep.cfl_dt(op, 0.5)
    energies = []
    timestep.run(op, c, dt, 12, callback=lambda i, t, cc: energies.append(op.energy(cc)))
    e0 = op.energy(c)
    seq = np.array([e0] + energies)
    assert np.all(np.diff(seq) <= 1e-14 * e0)


def test_energy_closed_forms():
    """Constant state in a homogeneous medium: E = 1/2 |cube| (rho |v|^2 +
    lambda tr(e)^2 + 2 mu e:e) with |cube| = 8 (energy density of the
    velocity-strain system).  Constant velocity, zero strain and a density
    linear in x (integrated exactly by Q_N): E = 1/2 |v|^2 * 8 * mean(rho)."""
    from workloads import media
    op, EToV, VXYZ, xyz, _ = oracle_case(2, 3, medium="homogeneous", shuffle_seed=4)
    rho, lam, mu = 1.3, 0.7, 1.1
    from oracle.dg import Elastic
    op = Elastic(2, VXYZ, *media.homogeneous(xyz, rho, lam, mu))
    one = op.project_q(np.ones(op.Nq))
    v = np.array([0.3, -1.2, 0.5])
    e6 = np.array([0.2, -0.1, 0.4, 0.15, -0.25, 0.05])      # xx yy zz yz xz xy
    c = np.zeros((op.K, 9, op.Np))
    c[:, 0:3] = v[None, :, None] * one
    c[:, 3:9] = e6[None, :, None] * one
    ee = np.sum(e6[:3] ** 2) + 2.0 * np.sum(e6[3:] ** 2)
    E = 0.5 * 8.0 * (rho * v @ v + lam * np.sum(e6[:3]) ** 2 + 2.0 * mu * ee)
    assert abs(op.energy(c) - E) <= 1e-12 * E
    r_lin = 1.0 + 0.3 * xyz[..., 0] - 0.2 * xyz[..., 2]
    op2 = Elastic(2, VXYZ, r_lin, np.full_like(r_lin, lam), np.full_like(r_lin, mu))
    c2 = np.zeros_like(c)
    c2[:, 0:3] = v[None, :, None] * one
    assert abs(op2.energy(c2) - 0.5 * 8.0 * (v @ v)) <= 1e-12 * (v @ v)


def test_point_values_reproduce_polynomials():
    """The projection of a global degree-N polynomial is exact in every
    element, so its value at any point equals the polynomial's."""
    N = 3
    op, EToV, VXYZ, xyz, _ = oracle_case(N, 3, shuffle_seed=2)
    rng = np.random.default_rng(12)
    cf = rng.standard_normal((9, 4))

    def poly(p):
        x, y, z = p[..., 0], p[..., 1], p[..., 2]
        basis = np.stack([np.ones_like(x), x * y * z, x ** 3 - y, y * z ** 2], axis=-1)
        return basis @ cf.T

    c = op.project_q(np.moveaxis(poly(xyz), -1, 1))
    pts = rng.uniform(-0.99, 0.99, size=(25, 3))
    got = op.eval_points(c, pts)
    assert np.abs(got - poly(pts)).max() <= 1e-12


def test_point_values_on_the_singular_edge_of_the_collapsed_map():
    """Values at mesh vertices, on edges and on faces, which in the owning
    element's reference coordinates include the vertex t = 1 and the edge
    s + t = 0 where the collapsed map is singular: the projection of a global
    degree-N polynomial must still give the polynomial's value (the
    singularity is removable for values), at N = 2, 3 and 4."""
    from oracle.reference import Basis
    rng = np.random.default_rng(13)
    for N in (2, 3, 4):
        # reference vertices and points on the singular edge (r = -1, s + t = 0)
        B = Basis(N)
        edge = np.array([[-1.0, -1.0, 1.0], [-1.0, 1.0, -1.0], [1.0, -1.0, -1.0], [-1.0, -1.0, -1.0],
                         [-1.0, 0.4, -0.4], [-1.0, -0.2, 0.2], [-1.0, 0.0, 0.0]])
        assert np.all(np.isfinite(B.eval(edge)))
        # the values at the singular points are limits of nearby interior ones
        inner = edge + 1e-8 * (np.array([-0.5, -0.5, -0.5]) - edge)      # towards the centroid
        assert np.abs(B.eval(edge) - B.eval(inner)).max() <= 1e-5
        op, EToV, VXYZ, xyz, _ = oracle_case(N, 4, shuffle_seed=30 + N)
        cf = rng.standard_normal((9, 4))

        def poly(p):
            x, y, z = p[..., 0], p[..., 1], p[..., 2]
            basis = np.stack([np.ones_like(x), x * y - z, x ** N + y, y * z ** (N - 1)], axis=-1)
            return basis @ cf.T

        c = op.project_q(np.moveaxis(poly(xyz), -1, 1))
        pts = np.array([[0.0, 0.5, -0.5], [0.5, 0.5, 0.5], [0.25, 0.0, 0.1], [0.1, 0.1, 0.3],
                        [0.5, -0.5, 0.2], [-0.5, -0.5, -0.5], [0.0, 0.0, 0.0]])
        got = op.eval_points(c, pts)
        assert np.abs(got - poly(pts)).max() <= 1e-11, N
