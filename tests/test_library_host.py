"""Host-side checks of the C-ABI library (no GPU needed).

The library's reference-element operators are checked against closed forms
(exact differentiation, interpolation, the discrete integration-by-parts
identity) and its quadrature against the oracle's, which is an independent
implementation (scipy Gauss-Jacobi vs the library's Golub-Welsch).
"""
import os
import re

import numpy as np
import pytest

import paper_1711_01175_amd as P
from paper_1711_01175_amd import ewdg as B
from workloads.mesh import kuhn_periodic_mesh

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
NS = [1, 2, 3, 4, 5, 7]


def test_exports_every_declared_symbol():
    lib = B.load()
    hdr = open(os.path.join(ROOT, "include", "ewdg.h")).read()
    declared = set(re.findall(r"\b(ewdg_[a-z_0-9]+)\s*\(", hdr))
    assert len(declared) >= 20
    for name in declared:
        assert hasattr(lib, name), name
    assert declared == set(B.SIGNATURES), declared ^ set(B.SIGNATURES)


def test_rejects_bad_arguments():
    with pytest.raises(B.EwdgError):
        P.Context(6, 64)
    with pytest.raises(B.EwdgError):
        P.Context(3, 16)


def test_rejects_non_periodic_or_degenerate_meshes():
    c = P.Context(2, 64)
    EToV, VXYZ = kuhn_periodic_mesh(3)
    bad = VXYZ.copy()
    bad[5, [2, 3]] = bad[5, [3, 2]]          # negative orientation
    with pytest.raises(B.EwdgError) as e:
        c.set_mesh(EToV, bad)
    assert e.value.code == B.EWDG_EMESH
    with pytest.raises(B.EwdgError) as e:
        c.set_mesh(EToV[:-6], VXYZ[:-6])     # unmatched faces
    assert e.value.code == B.EWDG_EMESH
    E2, X2 = kuhn_periodic_mesh(2)           # 2 hexes per period: faces not unique
    with pytest.raises(B.EwdgError) as e:
        c.set_mesh(E2, X2)
    assert e.value.code == B.EWDG_EMESH
    with pytest.raises(B.EwdgError) as e:
        c.step(1e-3, 1)                       # no mesh bound
    assert e.value.code == B.EWDG_ESTATE


@pytest.mark.parametrize("N", NS)
def test_quadrature_matches_oracle(N):
    from oracle.reference import stroud_rule
    from helpers import quad_points
    c = P.Context(N, 64)
    EToV, VXYZ = kuhn_periodic_mesh(3, shuffle_seed=2)
    c.set_mesh(EToV, VXYZ)
    xq, wq = stroud_rule(N)
    assert np.abs(c.reference_operator(8) - wq).max() < 1e-15
    assert np.abs(c.quadrature_points() - quad_points(VXYZ, xq)).max() < 1e-14


def _poly(N, seed):
    rng = np.random.default_rng(seed)
    exps = [(a, b, cc) for a in range(N + 1) for b in range(N + 1 - a) for cc in range(N + 1 - a - b)]
    coef = rng.standard_normal(len(exps))

    def f(x):
        return sum(k * x[:, 0] ** a * x[:, 1] ** b * x[:, 2] ** cc for k, (a, b, cc) in zip(coef, exps))

    def df(x, d):
        out = np.zeros(len(x))
        for k, e in zip(coef, exps):
            if e[d]:
                e2 = list(e)
                e2[d] -= 1
                out += k * e[d] * x[:, 0] ** e2[0] * x[:, 1] ** e2[1] * x[:, 2] ** e2[2]
        return out
    return f, df


@pytest.mark.parametrize("N", NS)
def test_reference_operators_exact(N):
    from oracle.reference import stroud_rule
    c = P.Context(N, 64)
    nodes = c.reference_operator(7)
    f, df = _poly(N, N)
    u = f(nodes)
    scale = max(1.0, np.abs(u).max())
    for d in range(3):
        D = c.reference_operator(d)
        assert np.abs(D @ u - df(nodes, d)).max() < 1e-10 * scale * (N + 1) ** 2
    xq, wq = stroud_rule(N)
    Vq, Pq = c.reference_operator(4), c.reference_operator(5)
    assert np.abs(Vq @ u - f(xq)).max() < 1e-11 * scale
    assert np.abs(Pq @ Vq - np.eye(c.Np)).max() < 1e-11
    M = c.reference_operator(6)
    assert np.abs(M - Vq.T @ (wq[:, None] * Vq)).max() < 1e-12


@pytest.mark.parametrize("N", NS)
def test_lift_integration_by_parts(N):
    """M D_k + D_k^T M = sum_f n_k,f sJ_f E_f^T M_f E_f, with the face
    blocks read off M LIFT (= E^T M_f); reference faces t=-1, s=-1,
    r+s+t=-1, r=-1 with sJ = 1, 1, sqrt3, 1."""
    c = P.Context(N, 64)
    nodes = c.reference_operator(7)
    M = c.reference_operator(6)
    ML = M @ c.reference_operator(3)
    L = np.array([0.5 * (1 + nodes[:, 0]), 0.5 * (1 + nodes[:, 1]), 0.5 * (1 + nodes[:, 2])])
    lam = np.vstack([-(L.sum(0) - 0.5) * 0 + (-0.5 * (1 + nodes.sum(1))), L])  # l0..l3
    opp = [3, 2, 0, 1]
    normals = [np.array([0, 0, -1.0]), np.array([0, -1.0, 0]), np.ones(3) / np.sqrt(3), np.array([-1.0, 0, 0])]
    sJ = [1.0, 1.0, np.sqrt(3.0), 1.0]
    Nfp = c.Nfp
    for k in range(3):
        D = c.reference_operator(k)
        lhs = M @ D + D.T @ M
        rhs = np.zeros_like(lhs)
        for f in range(4):
            fm = np.nonzero(np.abs(lam[opp[f]]) < 1e-10)[0]
            assert len(fm) == Nfp
            blk = ML[:, f * Nfp:(f + 1) * Nfp]            # E^T M_f (rows: volume nodes)
            rhs[:, fm] += normals[f][k] * sJ[f] * blk
        assert np.abs(lhs - rhs).max() < 1e-10 * np.abs(lhs).max()


@pytest.mark.parametrize("N", [2, 4, 7])
def test_warp_blend_edges_are_gauss_lobatto(N):
    from scipy.special import roots_jacobi
    c = P.Context(N, 64)
    nodes = c.reference_operator(7)
    edge = nodes[(np.abs(nodes[:, 1] + 1) < 1e-12) & (np.abs(nodes[:, 2] + 1) < 1e-12)][:, 0]
    lgl = np.concatenate([[-1.0], roots_jacobi(N - 1, 1, 1)[0] if N > 1 else [], [1.0]])
    assert np.allclose(np.sort(edge), np.sort(lgl), atol=1e-13)


def test_cfl_dt_needs_material():
    c = P.Context(3, 64)
    EToV, VXYZ = kuhn_periodic_mesh(3)
    c.set_mesh(EToV, VXYZ)
    with pytest.raises(B.EwdgError) as e:
        c.cfl_dt(0.5)
    assert e.value.code == B.EWDG_ESTATE


def test_empty_and_oversized_meshes_are_rejected():
    """K = 0 and K >= 2^26 (the connectivity packs neighbour * 32 into int32)
    are refused before any array is read."""
    import ctypes
    lib = B.load()
    c = P.Context(2, 32)
    one = np.zeros((1, 4), dtype=np.int64)
    xyz = np.zeros((1, 4, 3))
    for K in (0, -1, 1 << 26):
        rc = lib.ewdg_set_mesh(c.h, ctypes.c_int64(K), one.ctypes.data_as(ctypes.c_void_p),
                               xyz.ctypes.data_as(ctypes.c_void_p))
        assert rc == B.EWDG_EINVAL, (K, rc)


@pytest.mark.parametrize("N,K", [(1, 1 << 23), (4, 6_900_000), (7, 2_000_000), (5, 4_300_000)])
def test_meshes_beyond_32bit_offsets_are_rejected(N, K):
    """Meshes whose element data would overflow the kernels' 32-bit offsets
    (K 9 Np >= 2^31, or K >= 2^23 for the packed neighbour index) are refused
    with EWDG_EINVAL before any array is read (the arrays passed hold one
    element)."""
    import ctypes
    lib = B.load()
    c = P.Context(N, 32)
    one = np.zeros((1, 4), dtype=np.int64)
    xyz = np.zeros((1, 4, 3))
    rc = lib.ewdg_set_mesh(c.h, ctypes.c_int64(K), one.ctypes.data_as(ctypes.c_void_p),
                           xyz.ctypes.data_as(ctypes.c_void_p))
    assert rc == B.EWDG_EINVAL
    assert b"32-bit" in lib.ewdg_last_error(c.h)


def test_empty_batch_and_null_arguments():
    import ctypes
    lib = B.load()
    size = ctypes.c_size_t()
    assert lib.ewdg_batch_table_bytes(0, ctypes.byref(size)) == B.EWDG_OK and size.value > 0
    assert lib.ewdg_batch_table_bytes(-1, ctypes.byref(size)) == B.EWDG_EINVAL
    assert lib.ewdg_step_batch(None, 0, None, 5, None, 0, None) == B.EWDG_OK
    assert lib.ewdg_step_batch(None, 2, None, 5, None, 0, None) == B.EWDG_EINVAL
    assert lib.ewdg_create(4, 32, None, None) == B.EWDG_EINVAL
    c = P.Context(3, 64)
    assert lib.ewdg_workspace_bytes(c.h, 0, 0, ctypes.byref(size)) == B.EWDG_ESTATE   # no mesh yet
    EToV, VXYZ = kuhn_periodic_mesh(3)
    c.set_mesh(EToV, VXYZ)
    assert lib.ewdg_workspace_bytes(c.h, -1, 0, ctypes.byref(size)) == B.EWDG_EINVAL
    assert lib.ewdg_adjoint_workspace_bytes(c.h, 10, 5, ctypes.byref(size)) == B.EWDG_ESTATE  # not bound
    assert lib.ewdg_adjoint_workspace_bytes_overlapped(c.h, 10, 5, ctypes.byref(size)) == B.EWDG_ESTATE
    assert lib.ewdg_adjoint_workspace_bytes_overlapped(None, 10, 5, ctypes.byref(size)) != B.EWDG_OK


@pytest.mark.parametrize("d,p,n", [(2, 1, 3), (2, 4, 2), (3, 2, 2), (3, 4, 1)])
def test_transport_points_follow_the_documented_numbering(d, p, n):
    """The library's volume and face points, in the numbering include/ewdg.h
    states, against the oracle's (an independent construction: numpy
    Gauss-Legendre vs the library's Golub-Welsch)."""
    from oracle.transport import Transport as OT
    beta = (1.0, -0.8, 0.6)
    T = P.Transport(d, p, n, beta)
    o = OT(d, p, n, beta)
    assert (T.E, T.Np, T.Nq, T.Nqf) == (n ** d, (p + 1) ** d, (p + 3) ** d, (p + 3) ** (d - 1))
    xv, xf = T.points()
    assert np.abs(xv - o.volume_points()).max() < 1e-15
    for a in range(d):
        for s in (0, 1):
            assert np.abs(xf[:, 2 * a + s] - o.face_points(a, s)).max() < 1e-15
    assert T.workspace_bytes() > 0


def test_transport_rejects_bad_arguments():
    for args in ((1, 2, 4, (1, 1, 1)), (2, 0, 4, (1, 1, 1)), (2, 5, 4, (1, 1, 1)), (3, 2, 0, (1, 1, 1)),
                 (2, 2, 4, (1, 0, 1)), (3, 2, 4, (1, 1, 0))):
        with pytest.raises(B.EwdgError):
            P.Transport(*args)
    with pytest.raises(B.EwdgError):
        P.Transport(2, 2, 4, (1, 1), precision=16)
    T = P.Transport(2, 2, 4, (1.0, 1.0))
    with pytest.raises(B.EwdgError):      # no workspace, no problem
        T.solve()
    with pytest.raises(B.EwdgError):
        T.set_problem(np.zeros((T.E, T.Nq)), np.zeros((T.E, 4, T.Nqf)))


def test_bounded_meshes_mark_boundary_faces():
    """A box mesh (no periodic wrap) is refused as periodic; with a boundary
    condition its 12 n^2 boundary faces point at their own element."""
    from workloads.mesh import kuhn_box_mesh
    n = 3
    EToV, VXYZ = kuhn_box_mesh(n, shuffle_seed=2)
    c = P.Context(2, 64)
    with pytest.raises(B.EwdgError):
        c.set_mesh(EToV, VXYZ)
    for bc in ("free", "absorbing"):
        c = P.Context(2, 64)
        c.set_mesh(EToV, VXYZ, boundary=bc)
        conn = c.connectivity()
        nb = conn >> 5
        selfref = nb == np.arange(c.K)[:, None]
        assert selfref.sum() == 12 * n * n
        # interior faces still point back
        for k, f in zip(*np.nonzero(~selfref)):
            g = (conn[k, f] & 31) // 6
            assert conn[nb[k, f], g] >> 5 == k
    with pytest.raises(B.EwdgError):
        P.Context(2, 64).set_mesh(EToV, VXYZ, boundary="nonsense")
