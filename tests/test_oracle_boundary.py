"""Pins for the oracle's boundary faces (traction-free and absorbing).

Against the mathematics: the semi-discrete energy rate equals the closed
forms derived by hand for the boundary faces' exterior states, a standing
P-wave that is an exact traction-free solution (lambda = 0) is approximated
at the expected order, the boundary face count of the bounded Kuhn mesh, and
energy never grows.
"""
import numpy as np
import pytest

from helpers import quad_points
from oracle import timestep
from oracle.dg import Elastic
from oracle.reference import stroud_rule
from workloads import media
from workloads.mesh import kuhn_box_mesh


def bounded_case(N, n, bc, shuffle_seed=None, jump_seed=None):
    EToV, VXYZ = kuhn_box_mesh(n, shuffle_seed=shuffle_seed)
    xq, _ = stroud_rule(N)
    xyz = quad_points(VXYZ, xq)
    rho, lam, mu = media.smooth(xyz)
    if jump_seed is not None:
        rho, lam, mu = media.perturb_per_element(rho, lam, mu, jump_seed, frac=0.2)
    return Elastic(N, VXYZ, rho, lam, mu, boundary=bc), EToV, VXYZ, xyz, (rho, lam, mu)


def test_boundary_face_count():
    for n in (2, 3):
        op, *_ = bounded_case(1, n, "free")
        assert op.mesh.boundary.sum() == 12 * n * n
        assert np.all((op.mesh.nbr < 0) == op.mesh.boundary)


@pytest.mark.parametrize("bc", ["free", "absorbing"])
@pytest.mark.parametrize("N", [1, 3, 4])
def test_energy_rate_with_boundary_faces(bc, N):
    """dE/dt = interior face dissipation + the boundary closed form:
    -(T_n^2/Z_p + |T_t|^2/Z_s) (traction-free) or
    -(Z_p v_n^2 + T_n^2/Z_p + Z_s |v_t|^2 + |T_t|^2/Z_s)/2 (absorbing)."""
    op, *_ = bounded_case(N, 3, bc, shuffle_seed=3, jump_seed=11)
    c = np.random.default_rng(1).standard_normal((op.K, 9, op.Np))
    rate = op.energy_rate(c, op.rhs(c))
    closed = op.face_dissipation(c)
    assert closed < 0
    assert abs(rate - closed) <= 1e-12 * abs(closed)


def _standing(op, xyz, t):
    """lambda = 0, rho = mu = 1: v_x = c cos(a(x+1)) sin(c a t),
    e_xx = sin(a(x+1)) cos(c a t), a = pi/2, c = sqrt(2): sigma_xx = 0 at
    x = +-1 and sigma_yy = sigma_zz = 0 everywhere, so every face of the box
    is traction-free."""
    cp, a = np.sqrt(2.0), np.pi / 2
    f = np.zeros((op.K, 9, op.Nq))
    x = xyz[..., 0]
    f[:, 0] = cp * np.cos(a * (x + 1)) * np.sin(cp * a * t)
    f[:, 3] = np.sin(a * (x + 1)) * np.cos(cp * a * t)
    return f


@pytest.mark.parametrize("N", [1, 2])
def test_traction_free_standing_wave_converges(N):
    errs = []
    for n in (2, 4):
        EToV, VXYZ = kuhn_box_mesh(n)
        xq, _ = stroud_rule(N)
        xyz = quad_points(VXYZ, xq)
        one = np.ones(xyz.shape[:2])
        op = Elastic(N, VXYZ, one, 0 * one, one, boundary="free")
        dt = timestep.cfl_dt(op, 0.5)
        steps = int(round(0.5 / dt))
        c, T, _ = timestep.run(op, op.project_q(_standing(op, xyz, 0.0)), dt, steps)
        ex = _standing(op, xyz, T)
        errs.append(op.l2_q(op.to_q(c) - ex) / op.l2_q(ex))
    assert np.log2(errs[0] / errs[1]) > N + 0.5, errs


@pytest.mark.parametrize("bc", ["free", "absorbing"])
def test_energy_does_not_grow(bc):
    op, *_ = bounded_case(2, 3, bc, jump_seed=5)
    c = np.random.default_rng(2).standard_normal((op.K, 9, op.Np))
    dt = timestep.cfl_dt(op, 0.5)
    E = [op.energy(c)]
    for _ in range(5):
        c, _, _ = timestep.run(op, c, dt, 1)
        E.append(op.energy(c))
    assert np.all(np.diff(E) < 0)
