"""Material fields (rho, lambda, mu) as closed-form functions of position.

All functions take xyz with shape [..., 3] (for example the physical
quadrature points [K][Nq][3]) and return arrays of shape [...].  smooth also
takes a torch tensor and then returns torch tensors (the same formula).  The smooth
fields are 1-periodic, hence periodic on [-1,1]^3.
"""
import numpy as np

TWO_PI = 2.0 * np.pi


def homogeneous(xyz, rho=1.0, lam=1.0, mu=1.0):
    shp = xyz.shape[:-1]
    return (np.full(shp, rho), np.full(shp, lam), np.full(shp, mu))


def smooth(xyz, phases=(0.0, 0.0, 0.0, 0.0, 0.0), amps=(1.0, 1.0, 1.0)):
    """Smooth heterogeneous medium varying inside elements.

    mu  = 1 + 0.5 a_mu  sin(2 pi x + p0) cos(2 pi y + p1)
    lam = 2 + 0.5 a_lam cos(2 pi z + p2)
    rho = 1 + 0.3 a_rho sin(2 pi (x + y + z) + p3)
    Default phases 0 and amplitude factors 1 give the reference medium.
    """
    xp = np if isinstance(xyz, np.ndarray) else _array_module(xyz)
    x, y, z = xyz[..., 0], xyz[..., 1], xyz[..., 2]
    p0, p1, p2, p3 = phases[:4]
    a_rho, a_lam, a_mu = amps
    mu = 1.0 + 0.5 * a_mu * xp.sin(TWO_PI * x + p0) * xp.cos(TWO_PI * y + p1)
    lam = 2.0 + 0.5 * a_lam * xp.cos(TWO_PI * z + p2)
    rho = 1.0 + 0.3 * a_rho * xp.sin(TWO_PI * (x + y + z) + p3)
    return rho, lam, mu


def _array_module(a):
    """numpy, or torch for a torch tensor (its CPU kernels run on several
    threads: the server samples large media that way)."""
    import torch
    return torch if isinstance(a, torch.Tensor) else np


def perturb_per_element(rho, lam, mu, seed, frac=0.1):
    """Multiply each element's fields by (1 + frac*u), u ~ U[-1,1] i.i.d.

    One u per element and per field (rho, lambda, mu), drawn with
    numpy.random.default_rng(seed); fields have shape [K][Nq].
    """
    rng = np.random.default_rng(seed)
    K = rho.shape[0]
    u = rng.uniform(-1.0, 1.0, size=(3, K, 1))
    return (rho * (1.0 + frac * u[0]), lam * (1.0 + frac * u[1]),
            mu * (1.0 + frac * u[2]))


def gaussian_mu_anomaly(xyz, mu, amp=0.1, width=0.15, center=(0.0, 0.0, 0.0)):
    """mu * (1 + amp exp(-|x-c|^2 / (2 width^2)))."""
    d = xyz - np.asarray(center)
    r2 = np.sum(d * d, axis=-1)
    return mu * (1.0 + amp * np.exp(-r2 / (2.0 * width ** 2)))
