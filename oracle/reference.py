"""Reference tetrahedron, quadrature rules and an orthonormal modal basis of P_N.

Reference element T^ = {r, s, t >= -1, r + s + t <= -1} with vertices
v0 = (-1,-1,-1), v1 = (1,-1,-1), v2 = (-1,1,-1), v3 = (-1,-1,1).  Element k
of a mesh is the affine image sending v_i to its i-th vertex.

The polynomial space is P_N on each element (Sec. 2, the discontinuous
spaces V_h).  The paper works on tensor-product elements; on simplices the
same construction uses total-degree polynomials.

Quadrature Q_N is the Stroud conical-product rule: Gauss-Jacobi points in the
three collapsed directions with weights (1-x)^0, (1-x)^1, (1-x)^2, N+1 points
each, exact for total degree 2N+1.  Points are ordered with the first
collapsed index fastest: q = i + (N+1) * (j + (N+1) * k).  This rule defines
the material-weighted integrals, so the ordering is part of the interface
with the GPU library.  Gauss-Jacobi nodes come from scipy (a library routine;
the GPU library computes them independently by Golub-Welsch).
"""
import numpy as np
from scipy.special import eval_jacobi, gammaln, roots_jacobi

REF_VERTS = np.array([[-1.0, -1.0, -1.0],
                      [1.0, -1.0, -1.0],
                      [-1.0, 1.0, -1.0],
                      [-1.0, -1.0, 1.0]])
REF_VOLUME = 4.0 / 3.0

# Faces as ordered vertex triples of the reference element.
FACE_VERTS = ((0, 1, 2), (0, 1, 3), (1, 2, 3), (0, 2, 3))


def n_modes(N):
    return (N + 1) * (N + 2) * (N + 3) // 6


def stroud_rule(N):
    """Conical-product rule on T^, (N+1)^3 points, exact to degree 2N+1.

    Returns points [Nq][3] (r,s,t) and weights [Nq] (summing to 4/3).
    """
    m = N + 1
    a, wa = roots_jacobi(m, 0.0, 0.0)
    b, wb = roots_jacobi(m, 1.0, 0.0)
    c, wc = roots_jacobi(m, 2.0, 0.0)
    A = a[None, None, :]
    B = b[None, :, None]
    C = c[:, None, None]
    r = (1.0 + A) * (1.0 - B) * (1.0 - C) / 4.0 - 1.0
    s = (1.0 + B) * (1.0 - C) / 2.0 - 1.0 + 0.0 * A
    t = C + 0.0 * A * B
    w = wa[None, None, :] * wb[None, :, None] * wc[:, None, None] / 8.0
    pts = np.stack([r, s, t], axis=-1).reshape(-1, 3)
    return pts, w.reshape(-1)


def triangle_rule(N):
    """Collapsed Gauss-Jacobi rule on a triangle, exact to degree 2N+1.

    Returns barycentric coordinates [Nfq][3] (with respect to the triangle's
    three vertices in order) and weights [Nfq] summing to one, so that the
    integral over a face of area |f| is |f| * sum(w * g(points)).
    """
    m = N + 1
    a, wa = roots_jacobi(m, 0.0, 0.0)
    b, wb = roots_jacobi(m, 1.0, 0.0)
    u = (1.0 + a[None, :]) * (1.0 - b[:, None]) / 2.0 - 1.0
    v = b[:, None] + 0.0 * a[None, :]
    w = wa[None, :] * wb[:, None] / 2.0          # sums to 2 = area of (u,v) triangle
    l1 = (u + 1.0) / 2.0
    l2 = (v + 1.0) / 2.0
    l0 = 1.0 - l1 - l2
    bary = np.stack([l0, l1, l2], axis=-1).reshape(-1, 3)
    return bary, (w / 2.0).reshape(-1)


class Basis:
    """Orthonormal basis psi_m of P_N on T^ (integral of psi_m psi_n = delta).

    The Dubiner (Proriol-Koornwinder) basis in collapsed coordinates
        a = 2(1+r)/(-s-t) - 1,  b = 2(1+s)/(1-t) - 1,  c = t,
        psi_ijk = sqrt(8) P_i^(0,0)(a) P_j^(2i+1,0)(b) (1-b)^i
                          P_k^(2i+2j+2,0)(c) (1-c)^(i+j),   i+j+k <= N,
    with P^(alpha,beta) the Jacobi polynomials normalised to unit norm under
    their weight.  Jacobi values come from scipy.special.eval_jacobi.  The
    collapsed map is singular on the edge s+t=0 and at the vertex t=1.  For
    values the singularity is removable: on s+t=0 the factor (1-b)^i is zero
    for i > 0 and P_0 is constant, so any a gives the same value (a = -1 is
    taken); at t=1 likewise (1-c)^(i+j) vanishes unless i = j = 0 (b = -1 is
    taken).  Gradients are only asked for away from that edge (quadrature
    and face-rule points), and there the map is smooth.
    """

    def __init__(self, N):
        self.N = N
        self.Np = n_modes(N)
        self.idx = [(i, j, k) for i in range(N + 1) for j in range(N + 1 - i)
                    for k in range(N + 1 - i - j)]
        assert len(self.idx) == self.Np

    @staticmethod
    def _jac(n, al, be, x):
        """Orthonormal Jacobi polynomial and its derivative."""
        lognorm = ((al + be + 1.0) * np.log(2.0) - np.log(2.0 * n + al + be + 1.0)
                   + gammaln(n + al + 1.0) + gammaln(n + be + 1.0)
                   - gammaln(n + al + be + 1.0) - gammaln(n + 1.0))
        h = np.exp(-0.5 * lognorm)
        p = eval_jacobi(n, al, be, x) * h
        if n == 0:
            dp = np.zeros_like(x)
        else:
            dp = 0.5 * (n + al + be + 1.0) * eval_jacobi(n - 1, al + 1.0, be + 1.0, x) * h
        return p, dp

    @staticmethod
    def _collapse(x, singular_ok=False):
        r, s, t = x[:, 0], x[:, 1], x[:, 2]
        den_a = -s - t
        den_b = 1.0 - t
        sa = den_a <= 1e-12
        sb = den_b <= 1e-12
        if not singular_ok and (np.any(sa) or np.any(sb)):
            raise ValueError("point on the singular edge of the collapsed map")
        a = np.where(sa, -1.0, 2.0 * (1.0 + r) / np.where(sa, 1.0, den_a) - 1.0)
        b = np.where(sb, -1.0, 2.0 * (1.0 + s) / np.where(sb, 1.0, den_b) - 1.0)
        return r, s, t, a, b, t.copy(), den_a, den_b

    def _eval(self, x, grad):
        x = np.asarray(x, dtype=np.float64).reshape(-1, 3)
        r, s, t, a, b, c, den_a, den_b = self._collapse(x, singular_ok=not grad)
        n = x.shape[0]
        P = np.empty((n, self.Np))
        if grad:
            Pr = np.empty((n, self.Np))
            Ps = np.empty((n, self.Np))
            Pt = np.empty((n, self.Np))
            da_dr = 2.0 / den_a
            da_ds = 2.0 * (1.0 + r) / den_a ** 2
            db_ds = 2.0 / den_b
            db_dt = 2.0 * (1.0 + s) / den_b ** 2
        sq8 = np.sqrt(8.0)
        for m, (i, j, k) in enumerate(self.idx):
            fa, dfa = self._jac(i, 0.0, 0.0, a)
            pb, dpb = self._jac(j, 2.0 * i + 1.0, 0.0, b)
            pc, dpc = self._jac(k, 2.0 * i + 2.0 * j + 2.0, 0.0, c)
            fb = pb * (1.0 - b) ** i
            fc = pc * (1.0 - c) ** (i + j)
            P[:, m] = sq8 * fa * fb * fc
            if grad:
                dfb = dpb * (1.0 - b) ** i
                if i > 0:
                    dfb = dfb - i * pb * (1.0 - b) ** (i - 1)
                dfc = dpc * (1.0 - c) ** (i + j)
                if i + j > 0:
                    dfc = dfc - (i + j) * pc * (1.0 - c) ** (i + j - 1)
                Pr[:, m] = sq8 * dfa * fb * fc * da_dr
                Ps[:, m] = sq8 * (dfa * fb * fc * da_ds + fa * dfb * fc * db_ds)
                Pt[:, m] = sq8 * (dfa * fb * fc * da_ds + fa * dfb * fc * db_dt
                                  + fa * fb * dfc)
        if grad:
            return Pr, Ps, Pt
        return P

    def eval(self, x):
        """psi_m at points x [n][3] -> [n][Np]."""
        return self._eval(x, False)

    def grad(self, x):
        """(d/dr, d/ds, d/dt) psi_m at points x -> three [n][Np] arrays."""
        return self._eval(x, True)


class Reference:
    """All reference-element data the oracle needs for degree N."""

    def __init__(self, N):
        self.N = N
        self.basis = Basis(N)
        self.Np = self.basis.Np
        self.xq, self.wq = stroud_rule(N)
        self.Nq = len(self.wq)
        self.Psi_q = self.basis.eval(self.xq)                  # [Nq][Np]
        g = self.basis.grad(self.xq)
        # Modal derivative matrices D_k[m][n] = (psi_m, d_k psi_n) on T^.
        # The integrand has degree 2N-1, so Q_N integrates it exactly.
        self.D = [self.Psi_q.T @ (self.wq[:, None] * gk) for gk in g]
        self.face_bary, self.face_w = triangle_rule(N)
        self.Nfq = len(self.face_w)
        self._face_cache = {}

    def face_points(self, triple):
        """Reference points of the face rule placed on the ordered vertex triple."""
        V = REF_VERTS[list(triple)]                           # [3][3]
        return self.face_bary @ V

    def face_psi(self, triple):
        """psi at the face-rule points laid on reference vertices `triple`."""
        key = tuple(int(i) for i in triple)
        if key not in self._face_cache:
            self._face_cache[key] = self.basis.eval(self.face_points(key))
        return self._face_cache[key]

    def project_q(self, fq):
        """L2_Q projection: values at Q_N points [..., Nq] -> modal [..., Np]."""
        return np.einsum('q,qm,...q->...m', self.wq, self.Psi_q, fq)

    def to_q(self, c):
        """Modal coefficients [..., Np] -> values at Q_N points [..., Nq]."""
        return np.einsum('qm,...m->...q', self.Psi_q, c)
