"""GPU parity of the steady transport solver (iHDG-II, ewdg_transport_*)
against the oracle, and the paper's Table 1 iteration counts on the GPU.

The GPU uses a modal orthonormal Legendre basis, the oracle a nodal basis at
Gauss points; solutions are compared at the volume points both evaluate.
Bars: iteration counts equal (the iteration marches the flow, so once an
element is exact it is recomputed bitwise identically and the stopping test
sees an exact zero change, in either precision); values within 1e-12 (FP64)
and 1e-5 (FP32) relative L2.
"""
import os

import numpy as np
import pytest
import torch  # noqa: F401  (imported at collection, outside the per-test time limit)

from test_oracle_transport import BETA, smooth, table1

pytestmark = pytest.mark.gpu


def _gpu(d, p, n, prec, with_exact=True):
    import paper_1711_01175_amd as P
    ue, f, b = smooth(d)
    T = P.Transport(d, p, n, b, precision=prec)
    T.bind_workspace()
    xv, xf = T.points()
    T.set_problem(f(xv), ue(xf), ue(xv) if with_exact else None)
    return T, ue, xv


def _report(name, **kw):
    print(name, " ".join(f"{k}={v:.3e}" if isinstance(v, float) else f"{k}={v}" for k, v in kw.items()),
          flush=True)


@pytest.mark.parametrize("prec", [64, 32])
@pytest.mark.parametrize("d,p,n", [(2, 1, 8), (2, 3, 6), (2, 4, 5), (3, 1, 4), (3, 2, 4), (3, 4, 3)])
def test_transport_parity(d, p, n, prec):
    from oracle.transport import Transport as OT
    T, ue, xv = _gpu(d, p, n, prec)
    iters, hist = T.solve(1e-10, 1000)
    got = T.values()
    _, f, b = smooth(d)
    o = OT(d, p, n, b)
    u, oi, oh = o.solve(f, ue, ue, tol=1e-10)
    ref = u @ o.Vq.T
    err = np.sqrt(np.sum((got - ref) ** 2 * o.Wq)) / np.sqrt(np.sum(ref ** 2 * o.Wq))
    _report("transport", d=d, p=p, n=n, prec=prec, iters=iters, oracle=oi, rel_l2=err)
    assert iters == oi == d * (n - 1) + 2
    assert err <= (1e-12 if prec == 64 else 1e-5)
    # the error history: ||u^k - u^e|| after every iteration
    tolh = 1e-12 if prec == 64 else 1e-5
    assert np.allclose(hist, oh, rtol=tolh, atol=tolh * oh[0])


@pytest.mark.parametrize("prec", [64, 32])
def test_table1_iteration_counts_on_the_gpu(prec):
    """Every count of the paper's Table 1 (Sec. 6.1), on the GPU: exactly
    d (n - 1) + 2 for our problem and within 2 of the printed count."""
    rows = []
    for d, n, p, paper in table1():
        T, _, _ = _gpu(d, p, n, prec)
        iters, _ = T.solve(1e-10, 1000)
        rows.append((d, n, p, paper, iters))
        T.close()
    _report("table1", prec=prec, counts=[r[4] for r in rows])
    for d, n, p, paper, iters in rows:
        assert iters == d * (n - 1) + 2, (d, n, p, iters)
        assert abs(iters - paper) <= 2, (d, n, p, iters, paper)


def test_stopping_on_the_change_without_exact_solution():
    """Without the exact solution the rule is ||u^k - u^{k-1}|| < tol: zero
    once the last layer is exact, so the same count, and the same solution."""
    T, ue, xv = _gpu(3, 2, 5, 64, with_exact=False)
    iters, hist = T.solve(1e-10, 1000)
    assert iters == 3 * 4 + 2 and hist[-1] == 0.0 and hist[-2] > 0.0
    got = T.values()
    T2, _, _ = _gpu(3, 2, 5, 64)
    T2.solve(1e-10, 1000)
    assert np.array_equal(got, T2.values())


@pytest.mark.parametrize("prec", [64, 32])
def test_iteration_cap_and_repeated_solves(prec):
    """Iterations are queued in batches of 1, 2, 4, ...: a cap inside and at
    the end of a batch stops at exactly that many sweeps (values and history
    as the oracle's after that many), and solving again starts afresh."""
    from oracle.transport import Transport as OT
    d, p, n = 3, 2, 6
    ue, f, b = smooth(d)
    o = OT(d, p, n, b)
    T, _, xv = _gpu(d, p, n, prec)
    tol = 1e-12 if prec == 64 else 1e-5
    for cap in (1, 2, 3, 5, 7, 8):
        iters, hist = T.solve(1e-10, cap)
        u, oi, oh = o.solve(f, ue, ue, tol=1e-10, max_iters=cap)
        ref = u @ o.Vq.T
        got = T.values()
        err = np.sqrt(np.sum((got - ref) ** 2 * o.Wq)) / np.sqrt(np.sum(ref ** 2 * o.Wq))
        _report("transport cap", prec=prec, cap=cap, iters=iters, rel_l2=err)
        assert iters == oi == cap and len(hist) == cap + 1
        assert err <= tol
        assert np.allclose(hist, oh, rtol=tol, atol=tol * oh[0])
    iters, hist = T.solve(1e-10, 1000)
    assert iters == d * (n - 1) + 2
    first = T.values()
    assert T.solve(1e-10, 1000)[0] == iters
    assert np.array_equal(T.values(), first)
