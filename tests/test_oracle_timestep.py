"""Pins for the oracle's time integration, source wavelet and time step."""
from fractions import Fraction as Fr

import numpy as np
import pytest

from helpers import oracle_case
from oracle import timestep


def _butcher():
    """Butcher tableau of the 2N-storage scheme, in exact rationals.

    With k_i = L(q_{i-1}): res_i = sum_{j<=i} (prod_{m=j+1..i} a_m) dt k_j and
    q_i = q_0 + sum_{l<=i} b_l res_l, so the stage matrix is
    A_ij = sum_{l=j..i-1} b_l prod_{m=j+1..l} a_m and the weights are
    B_j = sum_{l=j..5} b_l prod_{m=j+1..l} a_m."""
    a, b = timestep.RK_A, timestep.RK_B
    s = 5

    def prod(lo, hi):
        p = Fr(1)
        for m in range(lo, hi + 1):
            p *= a[m]
        return p

    A = [[Fr(0)] * s for _ in range(s)]
    for i in range(s):
        for j in range(i):
            A[i][j] = sum((b[l] * prod(j + 1, l) for l in range(j, i)), Fr(0))
    B = [sum((b[l] * prod(j + 1, l) for l in range(j, s)), Fr(0)) for j in range(s)]
    return A, B


def test_order_conditions():
    A, B = _butcher()
    c = [sum(row) for row in A]
    # the published c equal the row sums of the stage matrix
    for ci, cp in zip(c, timestep.RK_C):
        assert abs(float(ci - cp)) < 1e-15
    s = range(5)
    conds = [
        (sum(B), Fr(1)),
        (sum(B[i] * c[i] for i in s), Fr(1, 2)),
        (sum(B[i] * c[i] ** 2 for i in s), Fr(1, 3)),
        (sum(B[i] * A[i][j] * c[j] for i in s for j in s), Fr(1, 6)),
        (sum(B[i] * c[i] ** 3 for i in s), Fr(1, 4)),
        (sum(B[i] * c[i] * A[i][j] * c[j] for i in s for j in s), Fr(1, 8)),
        (sum(B[i] * A[i][j] * c[j] ** 2 for i in s for j in s), Fr(1, 12)),
        (sum(B[i] * A[i][j] * A[j][k] * c[k] for i in s for j in s for k in s), Fr(1, 24)),
    ]
    for got, want in conds:
        assert abs(float(got - want)) < 1e-15


class _Scalar:
    """A scalar linear 'operator' L(c) = lam c to drive the oracle's stepper."""

    def __init__(self, lam):
        self.lam = lam

    def rhs(self, c, src_value=0.0):
        return self.lam * c


def test_stability_polynomial():
    """One step on y' = z y multiplies by 1+z+z^2/2+z^3/6+z^4/24+z^5/200."""
    for z in [-0.3, -1.7, 0.5j, -2.0 + 1.0j, -4.0]:
        c, _, _ = timestep.run(_Scalar(z), np.array([1.0 + 0j]), 1.0, 1)
        poly = 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24 + z ** 5 / 200
        assert abs(c[0] - poly) < 1e-14 * max(1, abs(poly))


def test_temporal_order_four():
    lam = -1.0 + 3.0j
    errs = []
    for nsteps in [10, 20, 40]:
        c, _, _ = timestep.run(_Scalar(lam), np.array([1.0 + 0j]), 1.0 / nsteps, nsteps)
        errs.append(abs(c[0] - np.exp(lam)))
    rates = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert np.all(rates > 3.8)


def test_ricker():
    f0, t0 = 5.0, 0.2
    assert timestep.ricker(t0, f0, t0) == 1.0
    # zeros at t0 +- 1/(sqrt(2) pi f0)
    tz = t0 + 1.0 / (np.sqrt(2.0) * np.pi * f0)
    assert abs(timestep.ricker(tz, f0, t0)) < 1e-15


def test_cfl_dt_closed_form():
    """Homogeneous cube, n=4, N=3: r = h/(2(1+sqrt2)), c_p = sqrt3."""
    op, *_ = oracle_case(3, 4, medium="homogeneous")
    h = 0.5
    expect = 0.5 * (h / (2 * (1 + np.sqrt(2)))) / np.sqrt(3.0) / 16
    assert abs(timestep.cfl_dt(op, 0.5) - expect) < 1e-16
    assert abs(expect - 1.868e-3) < 1e-6


def test_receivers_sampled_after_each_full_step():
    """Receiver n holds v(x_r) at t_{n+1} = t0 + (n+1) dt, after the n-th
    full step (not at a stage time, not before the update).  Pinned to the
    exact P-plane wave: the discretisation error at the receivers is far
    below the change of v over one step, so sampling one step early (the
    state before the update) or one step late fails."""
    N, n, steps = 3, 4, 20
    op, EToV, VXYZ, xyz, _ = oracle_case(N, n, medium="homogeneous")
    cp, k = np.sqrt(3.0), np.pi

    def wave(x, t):
        ph = k * (x[..., 0] - cp * t)
        out = np.zeros(x.shape[:-1] + (9,))
        out[..., 0] = np.cos(ph)
        out[..., 3] = -np.cos(ph) / cp
        return out

    rec = np.array([[0.13, -0.41, 0.27], [-0.62, 0.35, -0.08], [0.71, 0.52, 0.66]])
    dt = timestep.cfl_dt(op, 0.5)
    t_start = 0.05
    c0 = op.project_q(np.moveaxis(wave(xyz, t_start), -1, 1))
    cT, T, traces = timestep.run(op, c0, dt, steps, t=t_start, receivers=rec)
    assert traces.shape == (steps, len(rec), 3)
    times = t_start + dt * np.arange(1, steps + 1)
    exact = np.stack([wave(rec, t)[:, 0:3] for t in times])            # [steps][nr][3]
    early = np.stack([wave(rec, t - dt)[:, 0:3] for t in times])
    late = np.stack([wave(rec, t + dt)[:, 0:3] for t in times])
    err = np.abs(traces - exact).max()
    assert err < 2e-3
    assert np.abs(traces - early).max() > 5 * err
    assert np.abs(traces - late).max() > 5 * err
    # the last record is the value of the final state at the receivers
    assert np.abs(traces[-1] - op.eval_points(cT, rec)[:, 0:3]).max() < 1e-14
    assert abs(T - times[-1]) < 1e-14
