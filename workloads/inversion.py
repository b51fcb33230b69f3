"""Seeded inputs of the misfit-gradient workload (receiver-misfit adjoint).

Periodic cube of n^3 hexahedra x 6 tetrahedra, smooth reference medium,
"observed" traces from the same medium with a Gaussian bump in mu, a
vertical Ricker point source below the centre and a 4 x 4 receiver grid
above it.  Only inputs are built here; no step of the method.
"""
import numpy as np

from . import media

SOURCE = dict(xs=(0.05, -0.10, -0.45), direction=(0.0, 0.0, 1.0), amp=1.0, f0=5.0, t0=0.2)


def receiver_grid(m=4, z=0.45, extent=0.6):
    """m x m receivers on the plane z, x and y evenly spaced in [-extent, extent]."""
    g = np.linspace(-extent, extent, m)
    X, Y = np.meshgrid(g, g, indexing="ij")
    return np.stack([X.ravel(), Y.ravel(), np.full(m * m, z)], axis=-1)


def media_pair(xyz, amp=0.1, width=0.25):
    """(reference rho, lam, mu), (true rho, lam, mu): the true medium has
    mu * (1 + amp exp(-|x|^2 / (2 width^2)))."""
    rho, lam, mu = media.smooth(xyz)
    return (rho, lam, mu), (rho, lam, media.gaussian_mu_anomaly(xyz, mu, amp=amp, width=width))


def random_elements(K, count=20, seed=5):
    """Distinct element indices drawn with numpy.random.default_rng(seed)."""
    return np.sort(np.random.default_rng(seed).choice(K, size=count, replace=False))
