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


@pytest.mark.parametrize("N,case,n1,n2", [(1, "P_x", 3, 6), (2, "P_x", 3, 6), (2, "S_x", 3, 6),
                                          (1, "P_oblique", 3, 6), (3, "P_x", 3, 4), (3, "P_oblique", 3, 4),
                                          (4, "S_x", 3, 4)])
def test_plane_wave_convergence(N, case, n1, n2):
    """Observed order between meshes of n1^3 and n2^3 hexahedra (at N = 3, 4
    the finer mesh is n = 4 so that the error stays far above rounding)."""
    d, pol, c, k = CASES[case]
    T = 0.1
    e1 = _error(N, n1, T, d, pol, c, k)
    e2 = _error(N, n2, T, d, pol, c, k)
    rate = np.log(e1 / e2) / np.log(n2 / n1)
    assert rate >= N + 0.5, (e1, e2, rate)
