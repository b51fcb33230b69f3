"""Seeded inputs of the misfit-gradient workload (receiver-misfit adjoint).

Periodic cube of n^3 hexahedra x 6 tetrahedra (n = 12: 10,368 tets), smooth
reference medium, "observed" traces from the same medium with
mu * (1 + 0.1 exp(-|x|^2 / (2 0.15^2))), a Ricker point force (f0 = 8,
t0 = 1/f0, direction z) at (-0.10, 0, 0) and 16 receivers on the plane
x = +0.10 at y, z in {-0.15, -0.05, 0.05, 0.15}.  At CFL 0.5 (dt ~ 2.7e-4)
the 800 steps span T ~ 0.21, long enough for the main lobe to cross the
0.2 gap.  Only inputs are built here; no step of the method.
"""
import numpy as np

from . import media

SOURCE = dict(xs=(-0.10, 0.0, 0.0), direction=(0.0, 0.0, 1.0), amp=1.0, f0=8.0, t0=0.125)
ANOMALY = dict(center=(0.0, 0.0, 0.0), amp=0.1, width=0.15)


def receiver_grid():
    """16 receivers on x = 0.10, y and z in {-0.15, -0.05, 0.05, 0.15}."""
    g = np.array([-0.15, -0.05, 0.05, 0.15])
    Y, Z = np.meshgrid(g, g, indexing="ij")
    return np.stack([np.full(16, 0.10), Y.ravel(), Z.ravel()], axis=-1)


def media_pair(xyz):
    """(reference rho, lam, mu), (true rho, lam, mu): the true medium has
    mu * (1 + amp exp(-|x - c|^2 / (2 width^2)))."""
    rho, lam, mu = media.smooth(xyz)
    a = ANOMALY
    return (rho, lam, mu), (rho, lam, media.gaussian_mu_anomaly(xyz, mu, amp=a["amp"], width=a["width"],
                                                                center=a["center"]))


def fd_elements(g, count=20, seed=5, floor=1e-2):
    """count distinct elements drawn with numpy.random.default_rng(seed)
    among those whose gradient norm over (rho, lambda, mu) is at least
    floor times the largest one (elements the misfit is sensitive to)."""
    nrm = np.linalg.norm(np.asarray(g).reshape(-1, 3), axis=1)
    pool = np.flatnonzero(nrm >= floor * nrm.max())
    return np.sort(np.random.default_rng(seed).choice(pool, size=min(count, len(pool)), replace=False))
