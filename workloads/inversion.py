"""Seeded inputs of the misfit-gradient workload (receiver-misfit adjoint).

Periodic cube of n^3 hexahedra x 6 tetrahedra, smooth reference medium,
"observed" traces from the same medium with a Gaussian bump in mu between
source and receivers, a vertical Ricker point source (f0 = 10) below the
centre and a 4 x 4 receiver grid above it, close enough that the P front
reaches the receivers within 800 steps at CFL 0.5 on the 12^3 mesh.  Only
inputs are built here; no step of the method.
"""
import numpy as np

from . import media

SOURCE = dict(xs=(0.05, -0.10, -0.15), direction=(0.0, 0.0, 1.0), amp=1.0, f0=10.0, t0=0.1)
ANOMALY = dict(center=(0.0, 0.0, 0.0), amp=0.1, width=0.15)


def receiver_grid(m=4, z=0.15, extent=0.3):
    """m x m receivers on the plane z, x and y evenly spaced in [-extent, extent]."""
    g = np.linspace(-extent, extent, m)
    X, Y = np.meshgrid(g, g, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), np.full(m * m, z)], axis=-1)


def media_pair(xyz):
    """(reference rho, lam, mu), (true rho, lam, mu): the true medium has
    mu * (1 + amp exp(-|x - c|^2 / (2 width^2)))."""
    rho, lam, mu = media.smooth(xyz)
    a = ANOMALY
    return (rho, lam, mu), (rho, lam, media.gaussian_mu_anomaly(xyz, mu, amp=a["amp"], width=a["width"],
                                                                center=a["center"]))


def sensitive_elements(VXYZ, count=20, seed=5, radius=0.3):
    """count distinct elements drawn with numpy.random.default_rng(seed)
    among those whose centroid lies within radius of the midpoint between
    the source and the receiver plane (where the misfit is sensitive)."""
    cen = VXYZ.mean(axis=1)
    mid = np.array([0.0, 0.0, 0.5 * (SOURCE["xs"][2] + 0.15)])
    pool = np.flatnonzero(np.linalg.norm(cen - mid, axis=1) <= radius)
    return np.sort(np.random.default_rng(seed).choice(pool, size=count, replace=False))
