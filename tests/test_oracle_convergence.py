"""Plane-wave convergence pins for the oracle (exact solutions of the PDE).

P and S plane waves in a homogeneous periodic cube (rho = lambda = mu = 1,
c_p = sqrt 3, c_s = 1) are exact solutions of the velocity-strain system;
the L2 error at a fixed time must fall at the rate expected of a degree-N
upwind DG method (about N+1, required >= N+1/2).
"""
import numpy as np
import pytest

from helpers import oracle_case
from oracle import timestep


def plane_wave(xyz, t, d, pol, c, k):
    """v = pol cos(k (d.x - c t)), e = -(1/c) sym(d (x) pol) cos(...)."""
    ph = k * (xyz @ d - c * t)
    cs = np.cos(ph)
    out = np.zeros(xyz.shape[:-1] + (9,))
    out[..., 0:3] = pol * cs[..., None]
    sym = 0.5 * (np.outer(d, pol) + np.outer(pol, d))
    for m, (i, j) in enumerate(((0, 0), (1, 1), (2, 2), (1, 2), (0, 2), (0, 1))):
        out[..., 3 + m] = -sym[i, j] / c * cs
    return np.moveaxis(out, -1, 1)                  # [K][9][Nq]


def _error(N, n, T, d, pol, c, k):
    op, EToV, VXYZ, xyz, _ = oracle_case(N, n, medium="homogeneous")
    c0 = op.project_q(plane_wave(xyz, 0.0, d, pol, c, k))
    dt = timestep.cfl_dt(op, 0.5)
    ns = int(np.ceil(T / dt))
    cT, _, _ = timestep.run(op, c0, T / ns, ns)
    ex = plane_wave(xyz, T, d, pol, c, k)
    return op.l2_q(op.to_q(cT) - ex) / op.l2_q(ex)


CASES = {
    "P_x": (np.array([1.0, 0, 0]), np.array([1.0, 0, 0]), np.sqrt(3.0), np.pi),
    "S_x": (np.array([1.0, 0, 0]), np.array([0, 1.0, 0]), 1.0, np.pi),
    "P_oblique": (np.array([1.0, 1.0, 0]) / np.sqrt(2), np.array([1.0, 1.0, 0]) / np.sqrt(2),
                  np.sqrt(3.0), np.pi * np.sqrt(2)),
}


@pytest.mark.parametrize("N,case", [(1, "P_x"), (2, "P_x"), (2, "S_x"), (1, "P_oblique")])
def test_plane_wave_convergence(N, case):
    d, pol, c, k = CASES[case]
    T = 0.1
    e1 = _error(N, 3, T, d, pol, c, k)
    e2 = _error(N, 6, T, d, pol, c, k)
    rate = np.log2(e1 / e2)
    assert rate >= N + 0.5, (e1, e2, rate)
