"""Pins for the oracle's weight-adjusted mass inverse (M_rho^-1 replaced by
M^-1 M_{1/rho} M^-1).

Against the mathematics: it is exact when rho is constant on every element,
the semi-discrete energy rate in the metric it inverts equals the closed-form
face dissipation, and its departure from the exact inverse shrinks at order
N + 1 (or faster) under refinement for a smooth density.
"""
import numpy as np
import pytest

from helpers import oracle_case, quad_points
from oracle.dg import Elastic
from oracle.reference import stroud_rule
from workloads import media
from workloads.mesh import kuhn_periodic_mesh


@pytest.mark.parametrize("N", [1, 3, 4])
def test_exact_for_elementwise_constant_density(N):
    op, EToV, VXYZ, xyz, _ = oracle_case(N, 3, medium="homogeneous", shuffle_seed=2)
    rho, lam, mu = media.perturb_per_element(*media.homogeneous(xyz), 7, frac=0.3)
    ex = Elastic(N, VXYZ, rho, lam, mu)
    wa = Elastic(N, VXYZ, rho, lam, mu, mass="wadg")
    c = np.random.default_rng(N).standard_normal((ex.K, 9, ex.Np))
    a, b = ex.rhs(c), wa.rhs(c)
    assert np.linalg.norm(a - b) <= 1e-13 * np.linalg.norm(a)


@pytest.mark.parametrize("N", [1, 3, 4])
def test_energy_rate_in_the_weight_adjusted_metric(N):
    op, EToV, VXYZ, xyz, mat = oracle_case(N, 3, shuffle_seed=3, jump_seed=11)
    wa = Elastic(N, VXYZ, *mat, mass="wadg")
    c = np.random.default_rng(1).standard_normal((wa.K, 9, wa.Np))
    rate = wa.energy_rate(c, wa.rhs(c))
    closed = wa.face_dissipation(c)
    assert abs(rate - closed) <= 1e-12 * abs(closed)


@pytest.mark.parametrize("N", [1, 2])
def test_departure_from_the_exact_inverse_shrinks(N):
    """For rho = 1 + 0.3 sin(pi (x + y + z)) the weight-adjusted velocity
    update of a smooth residual approaches the exact one at order >= N + 1."""
    errs = []
    for n in (3, 6):
        EToV, VXYZ = kuhn_periodic_mesh(n)
        xq, _ = stroud_rule(N)
        xyz = quad_points(VXYZ, xq)
        s = xyz.sum(axis=-1)
        rho = 1.0 + 0.3 * np.sin(np.pi * s)
        one = np.ones_like(rho)
        ex = Elastic(N, VXYZ, rho, one, one)
        wa = Elastic(N, VXYZ, rho, one, one, mass="wadg")
        f = np.zeros((ex.K, 9, ex.Nq))
        f[:, 3] = np.cos(np.pi * xyz[..., 0])     # a strain whose stress divergence is smooth
        c = ex.project_q(f)
        a, b = ex.rhs(c)[:, 0:3], wa.rhs(c)[:, 0:3]
        errs.append(np.sqrt(np.sum(ex.mesh.J[:, None, None] * (a - b) ** 2) / np.sum(ex.mesh.J[:, None, None] * a ** 2)))
    assert np.log2(errs[0] / errs[1]) > N + 0.5, errs
