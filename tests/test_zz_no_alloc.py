"""The allocation-free batched stepping entry point (ewdg_step_batch_static)
called through the C ABI, against ewdg_step_batch on the same requests:
bitwise equal states, times and receiver traces, on two calls in a row, the
second with fewer and smaller requests; and the size limit."""
import ctypes

import numpy as np
import pytest
import torch  # noqa: F401

from workloads.requests import request_stream

pytestmark = pytest.mark.gpu


def _contexts(reqs, precision, rec):
    import paper_1711_01175_amd as P
    out = []
    for r in reqs:
        c = P.Context(r.N, precision)
        c.set_mesh(*r.mesh())
        c.bind_workspace(len(rec), 40)
        c.set_material(*r.material(c.quadrature_points()))
        c.set_source(r.xs, r.direction, 1.0, r.f0, r.t0)
        c.set_receivers(rec)
        out.append(c)
    return out


def _run_pair(reqs, precision, nsteps, rec):
    """States, times and traces after nsteps through ewdg_step_batch (one
    buffer per step) and through ewdg_step_batch_static called from C."""
    import paper_1711_01175_amd as P
    lib = P.load()
    ref = _contexts(reqs, precision, rec)
    dts = [c.cfl_dt(0.5) for c in ref]
    table = torch.empty(P.batch_table_bytes(len(ref)), dtype=torch.uint8, device="cuda")
    P.step_batch(ref, dts, nsteps, table)
    got = _contexts(reqs, precision, rec)
    n = len(got)
    hs = (ctypes.c_void_p * n)(*[c.h for c in got])
    d = (ctypes.c_double * n)(*dts)
    torch.cuda.synchronize()
    rc = lib.ewdg_step_batch_static(hs, n, d, nsteps, ctypes.c_void_p(torch.cuda.current_stream().cuda_stream))
    assert rc == 0, lib.ewdg_last_error(got[0].h)
    torch.cuda.synchronize()
    for a, b in zip(ref, got):
        assert np.array_equal(a.get_state().cpu().numpy(), b.get_state().cpu().numpy())
        assert a.time() == b.time()
        assert np.array_equal(a.receivers(), b.receivers())
    return [c.K for c in got]


@pytest.mark.parametrize("precision", [32, 64])
def test_static_batch_matches_step_batch(precision):
    rec = np.array([[0.1, 0.2, -0.3], [-0.6, 0.05, 0.4]])
    big = request_stream(6, n_range=(4, 6), degrees=(2, 3, 4, 5), nsteps=9, seed0=300)
    sizes1 = _run_pair(big, precision, 9, rec)
    small = request_stream(2, n_range=(3, 3), degrees=(3, 4), nsteps=5, seed0=310)
    sizes2 = _run_pair(small, precision, 5, rec)
    print("first call K", sizes1, "second call K", sizes2, flush=True)
    assert len(sizes2) < len(sizes1) and max(sizes2) < max(sizes1)


def test_static_batch_size_limit():
    import paper_1711_01175_amd as P
    lib = P.load()
    cap = P.ewdg.static_table_max_bytes()
    n = 1
    while P.batch_table_bytes(n) <= cap:
        n += 1
    reqs = request_stream(1, n_range=(3, 3), degrees=(2,), nsteps=1, seed0=5)
    c = _contexts(reqs, 32, np.zeros((0, 3)))[0]
    before = c.get_state().cpu().numpy()
    hs = (ctypes.c_void_p * n)(*([c.h] * n))
    d = (ctypes.c_double * n)(*([c.cfl_dt(0.5)] * n))
    # the size is checked before the contexts (a repeated one is an error too)
    rc = lib.ewdg_step_batch_static(hs, n, d, 1, ctypes.c_void_p(0))
    assert rc == P.ewdg.EWDG_ENOMEM
    assert b"static launch table" in lib.ewdg_last_error(c.h)
    assert np.array_equal(c.get_state().cpu().numpy(), before) and c.time() == 0.0
