"""Steady transport by upwind HDG on a structured grid, solved by iHDG-II (oracle).

TEST INFRASTRUCTURE ONLY, like the rest of this package.

Problem (Sec. 4.1, eq. transport): beta . grad u = f in the unit square or
cube, u = g on the inflow boundary (beta . n < 0), with a constant velocity
beta.  The grid is n^d squares or cubes of side h = 1/n, and each element
carries the tensor-product space Q_p.

Discretisation.  The upwind HDG local equation (Sec. 4.1) on element K,
    -(u, div(beta v))_K + <beta.n u + |beta.n|(u - u^), v>_dK = (f, v)_K,
with the trace u^ eliminated by the weighted-trace equation of Sec. 4.1, is
the upwind flux: on an outflow face (beta.n > 0) the element's own trace,
on an inflow face the exterior trace (the neighbour's, or g on the boundary).

iHDG-II (Sec. 4.1 with Algorithm 1 of Sec. 3).  Iteration k+1 solves every
element's local equation with its own unknowns at k+1 and the exterior
traces of its inflow faces at iteration k:
    A_K u_K^{k+1} = (f, phi)_K - sum over inflow faces of <beta.n u_ext^k, phi>_f.
The initial guess is u^0 = 0.  Theorem 1 (Sec. 4.1): the iteration marches
the flow and is exact after finitely many iterations.

Stopping rule (Sec. 6.1): with the exact solution, stop at the first k with
| ||u^k - u^e|| - ||u^{k-1} - u^e|| | < tol (eq. tolerancecriteria, tol
1e-10); without it, ||u^k - u^{k-1}|| < tol.

Basis: Lagrange polynomials at the p+1 Gauss-Legendre points of each
direction (so the mass matrix is diagonal and every bilinear form of Q_p
polynomials is integrated exactly by that rule); right-hand side and error
norms with p+3 Gauss points per direction.
"""
import itertools

import numpy as np
from numpy.polynomial import legendre as npleg


def gauss(m):
    """Gauss-Legendre points and weights on [-1, 1]."""
    return npleg.leggauss(m)


def lagrange(nodes, x):
    """Values L[i][q] and derivatives D[i][q] of the Lagrange basis on nodes at x."""
    m = len(nodes)
    L = np.ones((m, len(x)))
    D = np.zeros((m, len(x)))
    for i in range(m):
        for j in range(m):
            if j == i:
                continue
            L[i] *= (x - nodes[j]) / (nodes[i] - nodes[j])
        # derivative by the product rule
        for k in range(m):
            if k == i:
                continue
            term = np.full(len(x), 1.0 / (nodes[i] - nodes[k]))
            for j in range(m):
                if j != i and j != k:
                    term = term * (x - nodes[j]) / (nodes[i] - nodes[j])
            D[i] += term
    return L, D


class Transport:
    """Upwind HDG for beta . grad u = f on [0,1]^d with n^d elements of degree p."""

    def __init__(self, d, p, n, beta):
        if d not in (2, 3):
            raise ValueError("d must be 2 or 3")
        self.d, self.p, self.n = d, p, n
        self.beta = np.asarray(beta, dtype=float)[:d]
        if np.any(self.beta == 0.0):
            raise ValueError("every component of beta must be nonzero")
        self.h = 1.0 / n
        self.E = n ** d
        m = p + 1
        self.nodes, self.w = gauss(m)
        self.Np = m ** d
        # element multi-indices (i_0 fastest) and their node multi-indices
        self.eidx = np.array(list(itertools.product(range(n), repeat=d)))[:, ::-1]
        self.nidx = np.array(list(itertools.product(range(m), repeat=d)))[:, ::-1]
        self._operators()

    # ------------------------------------------------------------ reference
    def _operators(self):
        d, m, h = self.d, self.p + 1, self.h
        x, w = self.nodes, self.w
        L, D = lagrange(x, x)            # L = identity at the nodes
        L1, _ = lagrange(x, np.array([-1.0, 1.0]))   # traces at the two ends [i][end]
        # volume form  -(phi_j, beta . grad phi_i)_K  on the physical element
        # (h/2)^d w_q  times  (2/h) beta_a d/dxi_a
        A = np.zeros((self.Np, self.Np))
        for a in range(d):
            # d phi_i / d xi_a at node q (tensor product)
            for I, ni in enumerate(self.nidx):
                for J, nj in enumerate(self.nidx):
                    # integrand phi_j(x_q) dphi_i/dxi_a(x_q) w_q: phi_j is 1 only at node nj
                    other = all(ni[b] == nj[b] for b in range(d) if b != a)
                    if not other:
                        continue
                    wq = np.prod([w[nj[b]] for b in range(d)])
                    A[I, J] -= (h / 2) ** (d - 1) * self.beta[a] * D[ni[a], nj[a]] * wq
        # outflow faces: + beta.n <phi_j, phi_i>_f
        self.faces = []      # (axis, side, beta.n)
        for a in range(d):
            for side in (0, 1):
                bn = self.beta[a] * (1.0 if side == 1 else -1.0)
                self.faces.append((a, side, bn))
        self.face_mass = {}
        for (a, side, bn) in self.faces:
            # <phi_j, phi_i>_f on face xi_a = -1 / +1 of the own element
            Mf = np.zeros((self.Np, self.Np))
            for I, ni in enumerate(self.nidx):
                for J, nj in enumerate(self.nidx):
                    if any(ni[b] != nj[b] for b in range(d) if b != a):
                        continue
                    wq = np.prod([w[nj[b]] for b in range(d) if b != a])
                    Mf[I, J] = (h / 2) ** (d - 1) * wq * L1[ni[a], side] * L1[nj[a], side]
            self.face_mass[(a, side)] = Mf
            if bn > 0:
                A += bn * Mf
        self.A = A
        self.Ainv = np.linalg.inv(A)
        # coupling to the exterior across face (a, side): the neighbour's face is (a, 1 - side)
        self.couple = {}
        for (a, side, bn) in self.faces:
            C = np.zeros((self.Np, self.Np))
            for I, ni in enumerate(self.nidx):
                for J, nj in enumerate(self.nidx):
                    if any(ni[b] != nj[b] for b in range(d) if b != a):
                        continue
                    wq = np.prod([w[nj[b]] for b in range(d) if b != a])
                    C[I, J] = (h / 2) ** (d - 1) * wq * L1[ni[a], side] * L1[nj[a], 1 - side]
            self.couple[(a, side)] = C
        # fine rule for right-hand sides and norms
        mq = self.p + 3
        self.xq, self.wq = gauss(mq)
        Lq, _ = lagrange(x, self.xq)                  # [node][fine point]
        self.qidx = np.array(list(itertools.product(range(mq), repeat=d)))[:, ::-1]
        self.Vq = np.ones((len(self.qidx), self.Np))   # nodal -> fine points
        for Q, qi in enumerate(self.qidx):
            for I, ni in enumerate(self.nidx):
                self.Vq[Q, I] = np.prod([Lq[ni[b], qi[b]] for b in range(d)])
        self.Wq = np.array([np.prod([self.wq[qi[b]] for b in range(d)]) for qi in self.qidx])
        # fine points on face (a, side) of the reference element, and face basis traces
        self.fidx = np.array(list(itertools.product(range(mq), repeat=d - 1)))[:, ::-1]
        self.Wf = np.array([np.prod([self.wq[k] for k in fi]) for fi in self.fidx])
        self.face_trace = {}
        for (a, side, bn) in self.faces:
            T = np.zeros((len(self.fidx), self.Np))
            for F, fi in enumerate(self.fidx):
                free = [b for b in range(d) if b != a]
                for I, ni in enumerate(self.nidx):
                    v = L1[ni[a], side]
                    for k, b in enumerate(free):
                        v *= Lq[ni[b], fi[k]]
                    T[F, I] = v
            self.face_trace[(a, side)] = T

    # ---------------------------------------------------------------- points
    def volume_points(self):
        """Physical fine points [E][Nq][d]."""
        ref = (self.xq[self.qidx] + 1.0) / 2.0 * self.h           # [Nq][d]
        return self.eidx[:, None, :] * self.h + ref[None, :, :]

    def face_points(self, a, side):
        """Physical fine points of face (a, side) of every element [E][Nf][d]."""
        d = self.d
        free = [b for b in range(d) if b != a]
        ref = np.zeros((len(self.fidx), d))
        ref[:, a] = float(side)
        for k, b in enumerate(free):
            ref[:, b] = (self.xq[self.fidx[:, k]] + 1.0) / 2.0
        return (self.eidx[:, None, :] + ref[None, :, :]) * self.h

    def neighbour(self, a, side):
        """Element across face (a, side) of every element, -1 on the boundary."""
        step = np.zeros(self.d, dtype=int)
        step[a] = 1 if side == 1 else -1
        nb = self.eidx + step
        inside = np.all((nb >= 0) & (nb < self.n), axis=1)
        flat = np.zeros(self.E, dtype=np.int64)
        mult = self.n ** np.arange(self.d)
        flat[inside] = nb[inside] @ mult
        flat[~inside] = -1
        return flat

    # --------------------------------------------------------------- problem
    def load(self, f, g):
        """(f, phi)_K minus the boundary inflow terms, for callables f(x), g(x)
        on points [..., d]; returns [E][Np]."""
        J = (self.h / 2) ** self.d
        fq = f(self.volume_points())                                # [E][Nq]
        b = J * (fq * self.Wq) @ self.Vq                           # [E][Np]
        Jf = (self.h / 2) ** (self.d - 1)
        for (a, side, bn) in self.faces:
            if bn >= 0:
                continue
            nb = self.neighbour(a, side)
            bd = nb < 0
            if not np.any(bd):
                continue
            gq = g(self.face_points(a, side)[bd])                   # [B][Nf]
            b[bd] -= bn * Jf * (gq * self.Wf) @ self.face_trace[(a, side)]
        return b

    def sweep(self, u, b):
        """One iHDG-II iteration: every element's local solve with the inflow
        traces of the previous iterate u."""
        rhs = b.copy()
        for (a, side, bn) in self.faces:
            if bn >= 0:
                continue
            nb = self.neighbour(a, side)
            ins = nb >= 0
            rhs[ins] -= bn * u[nb[ins]] @ self.couple[(a, side)].T
        return rhs @ self.Ainv.T

    def error(self, u, ue):
        """L2 distance from the exact solution callable ue."""
        J = (self.h / 2) ** self.d
        diff = u @ self.Vq.T - ue(self.volume_points())
        return float(np.sqrt(J * np.sum(diff ** 2 * self.Wq)))

    def solve(self, f, g, ue=None, tol=1e-10, max_iters=100000):
        """iHDG-II from u^0 = 0.  Returns (u, iterations, history) where
        history holds ||u^k - u^e|| (with ue) or ||u^k - u^{k-1}|| per k."""
        b = self.load(f, g)
        u = np.zeros((self.E, self.Np))
        J = (self.h / 2) ** self.d
        hist = [self.error(u, ue)] if ue is not None else []
        for k in range(1, max_iters + 1):
            new = self.sweep(u, b)
            if ue is not None:
                hist.append(self.error(new, ue))
                done = abs(hist[-1] - hist[-2]) < tol
            else:
                # nodal basis with the diagonal Gauss mass matrix
                wn = np.array([np.prod([self.w[i] for i in ni]) for ni in self.nidx])
                hist.append(float(np.sqrt(J * np.sum((new - u) ** 2 * wn))))
                done = hist[-1] < tol
            u = new
            if done:
                return u, k, np.array(hist)
        return u, max_iters, np.array(hist)

    def global_solve(self, f, g):
        """The coupled upwind HDG system solved directly (sparse LU)."""
        import scipy.sparse as sp
        import scipy.sparse.linalg as spla
        Np, E = self.Np, self.E
        blocks = sp.kron(sp.identity(E), sp.csr_matrix(self.A), format="lil")
        for (a, side, bn) in self.faces:
            if bn >= 0:
                continue
            nb = self.neighbour(a, side)
            C = bn * self.couple[(a, side)]
            for e in np.nonzero(nb >= 0)[0]:
                blocks[e * Np:(e + 1) * Np, nb[e] * Np:(nb[e] + 1) * Np] = C
        b = self.load(f, g).ravel()
        return spla.spsolve(blocks.tocsc(), b).reshape(E, Np)
