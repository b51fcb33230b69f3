"""Time integration, source wavelet, receivers and time step (oracle).

The paper's explicit HDG update (Sec. 4.3) advances each element
independently with forward Euler.  Here forward Euler is replaced by the
five-stage, fourth-order, two-register (2N-storage) Runge-Kutta scheme of
Carpenter and Kennedy (NASA TM-109112, 1994):
    res <- a_i res + dt L(q, t + c_i dt);   q <- q + b_i res,   i = 1..5.
With a single stage (a_1 = 0, b_1 = 1) this is exactly forward Euler.

Time step: dt = CFL * min_K (r_K / max_q c_p) / (N+1)^2, following the
explicit step scaling dt = O(h / (p^2 c)) quoted in Sec. 4.4 and the
(p+1)(p+2)/h growth of the inverse trace constant there; r_K is the
inradius 3|K|/|dK|.
"""
from fractions import Fraction as Fr

import numpy as np

# Carpenter-Kennedy (5,4) 2N-storage coefficients, as published.
RK_A = [Fr(0), Fr(-567301805773, 1357537059087), Fr(-2404267990393, 2016746695238),
        Fr(-3550918686646, 2091501179385), Fr(-1275806237668, 842570457699)]
RK_B = [Fr(1432997174477, 9575080441755), Fr(5161836677717, 13612068292357),
        Fr(1720146321549, 2090206949498), Fr(3134564353537, 4481467310338),
        Fr(2277821191437, 14882151754819)]
RK_C = [Fr(0), Fr(1432997174477, 9575080441755), Fr(2526269341429, 6820363962896),
        Fr(2006345519317, 3224310063776), Fr(2802321613138, 2924317926251)]
A = [float(x) for x in RK_A]
B = [float(x) for x in RK_B]
C = [float(x) for x in RK_C]


def ricker(t, f0, t0):
    """Ricker wavelet (1 - 2 pi^2 f0^2 (t-t0)^2) exp(-pi^2 f0^2 (t-t0)^2)."""
    a = (np.pi * f0 * (t - t0)) ** 2
    return (1.0 - 2.0 * a) * np.exp(-a)


def cfl_dt(op, cfl):
    cp = np.sqrt((op.lam_q + 2.0 * op.mu_q) / op.rho_q).max(axis=1)
    return float(cfl * np.min(op.mesh.inradius / cp) / (op.N + 1) ** 2)


class Source:
    def __init__(self, xs, direction, amp, f0, t0):
        self.xs = np.asarray(xs, float)
        self.direction = np.asarray(direction, float)
        self.amp = float(amp)
        self.f0 = float(f0)
        self.t0 = float(t0)


def run(op, c, dt, nsteps, t=0.0, source=None, receivers=None, callback=None):
    """Advance modal state c by nsteps LSRK(5,4) steps.

    Receivers record v at the given physical points after every full step.
    Returns (c, t, traces[nsteps][nr][3] or None).
    """
    c = np.asarray(c)
    c = c.astype(np.result_type(c.dtype, np.float64), copy=True)
    res = np.zeros_like(c)
    if source is not None:
        op.set_source(source.xs, source.direction, source.amp)
    rec_loc = None
    if receivers is not None:
        rec_loc = [op.locate(x) for x in np.atleast_2d(receivers)]
        rec_phi = [op.ref.basis.eval(rh[None, :])[0] for (_, rh) in rec_loc]
        traces = np.zeros((nsteps, len(rec_loc), 3), dtype=c.dtype)
    for n in range(nsteps):
        for i in range(5):
            ts = t + C[i] * dt
            sv = 0.0 if source is None else ricker(ts, source.f0, source.t0)
            L = op.rhs(c, sv)
            res = A[i] * res + dt * L
            c = c + B[i] * res
        t = t + dt
        if rec_loc is not None:
            for r, (k, _) in enumerate(rec_loc):
                traces[n, r] = c[k, 0:3] @ rec_phi[r]
        if callback is not None:
            callback(n, t, c)
    return c, t, (traces if rec_loc is not None else None)
