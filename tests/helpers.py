"""Shared test helpers: build seeded inputs and oracle operators."""
import numpy as np

from workloads import media
from workloads.mesh import kuhn_periodic_mesh


def quad_points(VXYZ, xq):
    """Physical positions of reference points xq [Nq][3] in every element."""
    X0 = VXYZ[:, 0]
    A = np.stack([VXYZ[:, 1] - X0, VXYZ[:, 2] - X0, VXYZ[:, 3] - X0], axis=-1) / 2.0
    return np.einsum('qd,kjd->kqj', xq + 1.0, A) + X0[:, None, :]


def oracle_case(N, n, medium="smooth", shuffle_seed=None, jump_seed=None, flux="upwind"):
    from oracle.dg import Elastic
    from oracle.reference import stroud_rule
    EToV, VXYZ = kuhn_periodic_mesh(n, shuffle_seed=shuffle_seed)
    xq, _ = stroud_rule(N)
    xyz = quad_points(VXYZ, xq)
    if medium == "homogeneous":
        rho, lam, mu = media.homogeneous(xyz)
    else:
        rho, lam, mu = media.smooth(xyz)
    if jump_seed is not None:
        rho, lam, mu = media.perturb_per_element(rho, lam, mu, jump_seed, frac=0.2)
    op = Elastic(N, VXYZ, rho, lam, mu, flux=flux)
    return op, EToV, VXYZ, xyz, (rho, lam, mu)
