"""Receiver misfit and its exact discrete gradient (oracle).

Misfit of the fully discrete solution (LSRK(5,4) steps of the upwind DG
operator) against data d at receivers, after every step n = 1..nsteps:
    J(theta) = 1/2 dt sum_n sum_r |v_h(x_r, t_n) - d_r(t_n)|^2 .
Parameters are per-element multipliers theta_e = (s_rho, s_lambda, s_mu)
of the quadrature-sampled fields (value 1 at the reference medium).

The oracle's gradient is taken by the complex-step method: J is evaluated
with theta_e[k] = 1 + i h for one (element, field) pair, and dJ/dtheta =
Im J / h holds to rounding for any h small enough (no subtractive
cancellation).  This is the exact derivative of the oracle's own discrete J,
independent of any hand-written adjoint.
"""
import numpy as np

from . import timestep
from .dg import Elastic

FIELDS = ("rho", "lam", "mu")


def misfit(N, VXYZ, rho_q, lam_q, mu_q, c0, dt, nsteps, source, receivers, data, t0=0.0):
    """J and the receiver traces for the given (possibly complex) material."""
    op = Elastic(N, VXYZ, rho_q, lam_q, mu_q)
    dtype = np.result_type(op.rho_q.dtype, np.float64)
    _, _, traces = timestep.run(op, np.asarray(c0, dtype=dtype), dt, nsteps, t=t0, source=source,
                                receivers=receivers)
    r = traces - data
    return 0.5 * dt * np.sum(r * r), traces


def complex_step_gradient(N, VXYZ, rho_q, lam_q, mu_q, c0, dt, nsteps, source, receivers, data,
                          elems, h=1e-30, t0=0.0):
    """dJ/dtheta for the listed elements, shape [len(elems)][3]."""
    g = np.zeros((len(elems), 3))
    base = [np.asarray(x, dtype=np.complex128) for x in (rho_q, lam_q, mu_q)]
    for a, e in enumerate(elems):
        for k in range(3):
            mats = [b.copy() for b in base]
            mats[k][e] *= (1.0 + 1j * h)
            J, _ = misfit(N, VXYZ, *mats, c0, dt, nsteps, source, receivers, data, t0=t0)
            g[a, k] = J.imag / h
    return g
