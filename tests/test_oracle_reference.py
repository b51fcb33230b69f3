"""Pins for the oracle's reference element, quadrature and mesh geometry.

Every check compares against a closed form (Dirichlet simplex integrals,
analytic derivatives of random polynomials, the Kuhn tetrahedron's inradius)
rather than against the oracle itself.
"""
import itertools
from math import factorial

import numpy as np
import pytest

from oracle.mesh import Mesh
from oracle.reference import Reference, stroud_rule, triangle_rule
from workloads.mesh import kuhn_periodic_mesh

NS = [1, 2, 3, 4, 5, 7]


def _tet_monomial(a, b, c):
    """Closed form of the integral of (1+r)^a (1+s)^b (1+t)^c over T^."""
    return 8.0 * 2.0 ** (a + b + c) * factorial(a) * factorial(b) * factorial(c) \
        / factorial(a + b + c + 3)


@pytest.mark.parametrize("N", NS)
def test_stroud_exact_to_2N_plus_1(N):
    x, w = stroud_rule(N)
    assert len(w) == (N + 1) ** 3 and np.all(w > 0)
    inside = (x >= -1 - 1e-14).all(1) & (x.sum(1) <= -1 + 1e-14)
    assert inside.all()
    deg = 2 * N + 1
    worst = 0.0
    for a, b, c in itertools.product(range(deg + 1), repeat=3):
        if a + b + c > deg:
            continue
        f = (1 + x[:, 0]) ** a * (1 + x[:, 1]) ** b * (1 + x[:, 2]) ** c
        ex = _tet_monomial(a, b, c)
        worst = max(worst, abs(w @ f - ex) / ex)
    assert worst < 1e-13
    # and not exact one degree higher (the rule is not over-specified)
    a = 2 * N + 2
    f = (1 + x[:, 2]) ** a
    assert abs(w @ f - _tet_monomial(0, 0, a)) / _tet_monomial(0, 0, a) > 1e-10


@pytest.mark.parametrize("N", NS)
def test_triangle_rule_exact(N):
    bary, w = triangle_rule(N)
    assert abs(w.sum() - 1.0) < 1e-14
    deg = 2 * N + 1
    for a in range(deg + 1):
        for b in range(deg + 1 - a):
            f = bary[:, 1] ** a * bary[:, 2] ** b
            # integral over the unit triangle divided by its area 1/2
            ex = 2.0 * factorial(a) * factorial(b) / factorial(a + b + 2)
            assert abs(w @ f - ex) < 1e-14 * max(1.0, ex) + 1e-15


@pytest.mark.parametrize("N", NS)
def test_basis_orthonormal(N):
    R = Reference(N)
    G = R.Psi_q.T @ (R.wq[:, None] * R.Psi_q)
    assert np.abs(G - np.eye(R.Np)).max() < 1e-12


@pytest.mark.parametrize("N", NS)
def test_derivative_matrices_exact_on_PN(N):
    """D_k maps the coefficients of a random degree-N polynomial to those of
    its exact derivative (compared pointwise with the analytic derivative)."""
    R = Reference(N)
    rng = np.random.default_rng(N)
    exps = [(a, b, c) for a in range(N + 1) for b in range(N + 1 - a)
            for c in range(N + 1 - a - b)]
    coef = rng.standard_normal(len(exps))

    def p(x):
        return sum(cf * x[:, 0] ** a * x[:, 1] ** b * x[:, 2] ** c
                   for cf, (a, b, c) in zip(coef, exps))

    def dp(x, k):
        out = np.zeros(len(x))
        for cf, e in zip(coef, exps):
            if e[k] == 0:
                continue
            e2 = list(e)
            e2[k] -= 1
            out += cf * e[k] * x[:, 0] ** e2[0] * x[:, 1] ** e2[1] * x[:, 2] ** e2[2]
        return out

    c = R.project_q(p(R.xq))
    # random interior test points
    lam = rng.dirichlet(np.ones(4), size=50)
    from oracle.reference import REF_VERTS
    pts = lam @ REF_VERTS
    psi = R.basis.eval(pts)
    assert np.abs(psi @ c - p(pts)).max() < 1e-11 * max(1, np.abs(p(pts)).max())
    for k in range(3):
        got = psi @ (R.D[k] @ c)
        ex = dp(pts, k)
        assert np.abs(got - ex).max() < 1e-10 * max(1.0, np.abs(ex).max())


@pytest.mark.parametrize("N", [1, 3, 4])
def test_sbp_identity(N):
    """Integration by parts on T^: D_k + D_k^T = sum_f n_k,f |f| E_f^T W_f E_f
    in the orthonormal basis (the discrete analogue of the identity used in
    the energy arguments of Sec. 4.1)."""
    from oracle.reference import FACE_VERTS, REF_VERTS
    R = Reference(N)
    for k in range(3):
        S = np.zeros((R.Np, R.Np))
        for tri in FACE_VERTS:
            V = REF_VERTS[list(tri)]
            opp = REF_VERTS[list({0, 1, 2, 3} - set(tri))[0]]
            cr = np.cross(V[1] - V[0], V[2] - V[0])
            area = 0.5 * np.linalg.norm(cr)
            nrm = cr / np.linalg.norm(cr)
            if nrm @ (opp - V[0]) > 0:
                nrm = -nrm
            psi = R.face_psi(tri)
            S += nrm[k] * area * psi.T @ (R.face_w[:, None] * psi)
        assert np.abs(R.D[k] + R.D[k].T - S).max() < 1e-12


@pytest.mark.parametrize("n", [3, 4])
def test_kuhn_mesh_geometry(n):
    EToV, VXYZ = kuhn_periodic_mesh(n, shuffle_seed=7)
    M = Mesh(VXYZ)
    h = 2.0 / n
    assert M.K == 6 * n ** 3
    assert abs(M.volume.sum() - 8.0) < 1e-12
    assert np.allclose(M.volume, h ** 3 / 6.0)
    # Kuhn tetrahedron inradius h / (2 (1 + sqrt 2)) in closed form
    assert np.allclose(M.inradius, h / (2.0 * (1.0 + np.sqrt(2.0))))
    # partners have opposite normals and equal areas
    for f in range(4):
        nb, fb = M.nbr[:, f], M.nbr_face[:, f]
        assert np.allclose(M.normal[nb, fb], -M.normal[:, f])
        assert np.allclose(M.area[nb, fb], M.area[:, f])
    bary, _ = triangle_rule(3)
    assert M.check_face_points(bary) < 1e-13


def test_locate_lowest_index_on_ties():
    EToV, VXYZ = kuhn_periodic_mesh(3)
    M = Mesh(VXYZ)
    x = VXYZ[10, 0].copy()           # a vertex shared by many elements
    k, _ = M.locate(x)
    owners = [e for e in range(M.K)
              if np.any(np.all(np.abs(VXYZ[e] - x) < 1e-14, axis=1))]
    assert k == min(owners)
