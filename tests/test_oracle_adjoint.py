"""Pins for the oracle's misfit gradient (complex step) against central
finite differences of its real-valued misfit."""
import numpy as np

from helpers import oracle_case
from oracle import adjoint, timestep


def test_complex_step_matches_central_differences():
    N, n = 2, 3
    op, EToV, VXYZ, xyz, (rho, lam, mu) = oracle_case(N, n, shuffle_seed=1, jump_seed=3)
    src = timestep.Source([0.05, -0.10, 0.15], [0.0, 0.0, 1.0], 1.0, 5.0, 0.2)
    rec = np.array([[0.3, -0.2, 0.1], [-0.4, 0.5, -0.6]])
    dt = timestep.cfl_dt(op, 0.5)
    c0 = np.zeros((op.K, 9, op.Np))
    nsteps = 15
    data = np.zeros((nsteps, 2, 3))
    _, tr = adjoint.misfit(N, VXYZ, rho, lam, mu, c0, dt, nsteps, src, rec, data, t0=0.1)
    data = 0.7 * tr[::-1]                      # data that leave a nonzero misfit
    elems = [0, 17, op.mesh.locate(src.xs)[0]]
    g = adjoint.complex_step_gradient(N, VXYZ, rho, lam, mu, c0, dt, nsteps, src, rec, data, elems, t0=0.1)
    hh = 1e-5
    for a, e in enumerate(elems):
        for k in range(3):
            mats_p = [rho.copy(), lam.copy(), mu.copy()]
            mats_m = [rho.copy(), lam.copy(), mu.copy()]
            mats_p[k][e] *= 1 + hh
            mats_m[k][e] *= 1 - hh
            Jp, _ = adjoint.misfit(N, VXYZ, *mats_p, c0, dt, nsteps, src, rec, data, t0=0.1)
            Jm, _ = adjoint.misfit(N, VXYZ, *mats_m, c0, dt, nsteps, src, rec, data, t0=0.1)
            fd = (Jp - Jm) / (2 * hh)
            assert abs(fd - g[a, k]) <= 1e-6 * np.abs(g).max() + 1e-14, (e, k, fd, g[a, k])
    assert np.abs(g).max() > 0
