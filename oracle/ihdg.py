"""iHDG-II solution of the implicit time step of the elastic operator (oracle).

TEST INFRASTRUCTURE ONLY, like the rest of this package.

Time discretisation.  The semi-discrete upwind DG system of dg.py,
dc/dt = L c + s(t), is advanced by the theta scheme
    (c^{m+1} - c^m) / dt = theta (L c^{m+1} + s^{m+1}) + (1 - theta)(L c^m + s^m).
theta = 1 is the implicit Euler scheme of Sec. 4.3 (eq. implicitHDG, there
for transport) written for this system; theta = 1/2 is the Crank-Nicolson
scheme used for the linearised shallow-water system in Sec. 6.

Solver.  The coupled system is solved by iHDG-II (Sec. 3, Algorithm 1).  On
iteration k+1 every element solves its local equation (eq. iHDGlocal) in
which the interface state, the weighted trace of eq. iHDGtrace, is formed
from the element's own unknowns at the new iterate and the neighbours'
unknowns at the old iterate k.  The interface state of dg.py is linear in the
traces of both sides, so the local equation of element K is the linear system
    (I - theta dt A_K) c_K^{k+1}
        = c_K^m + (1 - theta) dt (L c^m + s^m)_K + theta dt (s^{m+1} + N_K(c^k))
with A_K the operator L restricted to K's own unknowns (every other element
zero) and N_K(c^k) = (L c^k)_K - A_K c_K^k the contribution that the
neighbours' old iterate makes through the traces.  Elements are independent
within an iteration.  The initial guess is c^m, so the first iteration is the
locally implicit step of Sec. 4.3.

Stopping rule: the second criterion of Sec. 6.1 (no exact solution),
||c^k - c^{k-1}||_{L2(Omega)} < tol over all nine fields; with the orthonormal
modal basis ||u||^2_{L2(K)} = J_K sum c^2.

A_K is probed column by column: a unit value of one coefficient on every
element of a colour class (elements of one class share no face) makes the
operator's output on each member of the class that member's column of A_K.
"""
import numpy as np


def greedy_colouring(nbr):
    """Colour the face-adjacency graph so that no two neighbours share a colour."""
    K = nbr.shape[0]
    colour = np.full(K, -1, dtype=np.int64)
    for k in range(K):
        if np.any(nbr[k] == k):
            raise ValueError("element %d is its own neighbour" % k)
        used = {int(colour[j]) for j in nbr[k] if j >= 0 and colour[j] >= 0}
        c = 0
        while c in used:
            c += 1
        colour[k] = c
    return colour


def local_matrices(op):
    """A_K for every element: [K][9 Np][9 Np] acting on c_K flattened as [9][Np]."""
    K, Np = op.K, op.Np
    n = 9 * Np
    colour = greedy_colouring(op.mesh.nbr)
    A = np.zeros((K, n, n))
    for col in range(int(colour.max()) + 1):
        members = np.nonzero(colour == col)[0]
        for j in range(n):
            c = np.zeros((K, 9, Np))
            c[members, j // Np, j % Np] = 1.0
            A[members, :, j] = op.rhs(c, 0.0, elems=members).reshape(len(members), n)
    return A


def l2_norm(op, c):
    """L2(Omega) norm of all nine fields of the modal state c [K][9][Np]."""
    return float(np.sqrt(np.sum(op.mesh.J[:, None, None] * c ** 2)))


class ImplicitStep:
    """The theta scheme with step dt for operator op, solved by iHDG-II."""

    def __init__(self, op, dt, theta=1.0, A=None):
        if not (0.0 < theta <= 1.0):
            raise ValueError("theta must lie in (0, 1]")
        self.op, self.dt, self.theta = op, float(dt), float(theta)
        self.n = 9 * op.Np
        self.A = local_matrices(op) if A is None else A
        self.local_inv = np.linalg.inv(np.eye(self.n)[None] - self.theta * self.dt * self.A)

    def _own(self, c):
        """A_K c_K for every element (the element's own part of L c)."""
        K = self.op.K
        return (self.A @ c.reshape(K, self.n, 1)).reshape(c.shape)

    def step(self, c, t, source=None, tol=1e-10, max_iters=1000):
        """One step from (c^m, t^m).  Returns (c^{m+1}, iterations, norms) with
        norms[k] = ||c^{k+1} - c^k||; iterations = len(norms)."""
        from .timestep import ricker
        op, dt, th = self.op, self.dt, self.theta
        K, n = op.K, self.n
        s_now = 0.0 if source is None else ricker(t, source.f0, source.t0)
        s_next = 0.0 if source is None else ricker(t + dt, source.f0, source.t0)
        if source is not None:
            op.set_source(source.xs, source.direction, source.amp)
        # the fixed part of every local equation's right-hand side
        fixed = c + (1.0 - th) * dt * op.rhs(c, s_now)
        if source is not None:
            fixed = fixed + th * dt * op.rhs(np.zeros_like(c), s_next)
        ck = c.copy()
        norms = []
        for _ in range(max_iters):
            nbr_part = op.rhs(ck, 0.0) - self._own(ck)             # N_K(c^k)
            b = fixed + th * dt * nbr_part
            new = (self.local_inv @ b.reshape(K, n, 1)).reshape(c.shape)
            norms.append(l2_norm(op, new - ck))
            ck = new
            if norms[-1] < tol:
                break
        return ck, len(norms), np.array(norms)
