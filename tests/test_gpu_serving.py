"""GPU checks of batched stepping and the continuous-batching server.

Each request's result must be the same alone and in any mix: the batched
launch runs exactly the per-request arithmetic of a solo ewdg_step, so the
comparison is bitwise.  Served requests are also compared with the FP64
oracle run of the same request (relative L2 at the quadrature points
<= 1e-12 in FP64, <= 1e-5 in FP32).
"""
import numpy as np
import pytest
import torch  # noqa: F401

from workloads.requests import Request, request_stream

pytestmark = pytest.mark.gpu


def _solo(req, precision, nsteps):
    import paper_1711_01175_amd as P
    c = P.Context(req.N, precision)
    c.set_mesh(*req.mesh())
    c.bind_workspace()
    c.set_material(*req.material(c.quadrature_points()))
    c.set_source(req.xs, req.direction, 1.0, req.f0, req.t0)
    dt = c.cfl_dt(0.5)
    c.step(dt, nsteps)
    return c.get_state().cpu().numpy(), c


@pytest.mark.parametrize("whole", [False, True])
@pytest.mark.parametrize("precision", [32, 64])
def test_step_batch_equals_solo(precision, whole):
    """whole=False: a one-step table (one upload per step, one stream);
    whole=True: room for every step's table (one upload, a stream per
    degree class)."""
    import paper_1711_01175_amd as P
    reqs = request_stream(5, n_range=(3, 5), degrees=(2, 3, 4, 5), nsteps=12, seed0=40)
    solo = [_solo(r, precision, 12)[0] for r in reqs]
    ctxs, dts = [], []
    for r in reqs:
        c = P.Context(r.N, precision)
        c.set_mesh(*r.mesh())
        c.bind_workspace()
        c.set_material(*r.material(c.quadrature_points()))
        c.set_source(r.xs, r.direction, 1.0, r.f0, r.t0)
        ctxs.append(c)
        dts.append(c.cfl_dt(0.5))
    per_step = P.batch_table_bytes(len(ctxs))
    size = (per_step + 255) // 256 * 256 * 7 if whole else per_step
    table = torch.empty(size, dtype=torch.uint8, device="cuda")
    P.step_batch(ctxs, dts, 5, table)
    P.step_batch(ctxs, dts, 7, table)
    torch.cuda.synchronize()
    print("degrees", [r.N for r in reqs], "sizes", [c.K for c in ctxs], flush=True)
    for c, ref in zip(ctxs, solo):
        assert np.array_equal(c.get_state().cpu().numpy(), ref)
    assert all(abs(c.time() - 12 * dt) < 1e-12 for c, dt in zip(ctxs, dts))


def test_server_continuous_batching_alone_vs_mix():
    from paper_1711_01175_amd.serving import Server
    reqs = request_stream(7, n_range=(3, 5), degrees=(2, 3, 4), nsteps=20, seed0=77)
    # all queued at t = 0 with 3 slots and different lengths: queued requests
    # are admitted at chunk boundaries while others are still mid-run
    for i, r in enumerate(reqs):
        r.nsteps = 12 + 8 * (i % 3)
    rec = np.array([[0.1, 0.2, -0.3], [-0.7, 0.0, 0.4]])
    for r in reqs:
        r.receivers = rec
    fps = []
    import paper_1711_01175_amd as P
    for r in reqs:
        c = P.Context(r.N, 32)
        c.set_mesh(*r.mesh())
        fps.append(c.workspace_bytes(len(rec), r.nsteps))
    budget = int(2.5 * max(fps))
    srv = Server(budget_bytes=budget, slots=3, precision=32, chunk_steps=4, keep_state=True)
    stats = srv.run(reqs)
    print(stats.summary(), "max_active", stats.max_active, flush=True)
    assert len(stats.results) == len(reqs) and not stats.rejected
    assert stats.max_used_bytes <= budget and stats.max_active <= 3
    by = {r.rid: r for r in stats.results}
    # some request was admitted while another was still running
    overlap = any(a.admitted < b.finished and a.admitted > b.admitted
                  for a in stats.results for b in stats.results if a.rid != b.rid)
    assert overlap
    for r in reqs:
        alone = Server(budget_bytes=budget, slots=1, precision=32, chunk_steps=7, keep_state=True)
        r2 = Request(r.rid, r.n, r.N, r.nsteps, r.xs, r.phases, r.amps, 0.0, r.direction, r.f0, r.t0, rec)
        res = alone.run([r2]).results[0]
        assert np.array_equal(res.state, by[r.rid].state)
        assert np.array_equal(res.traces, by[r.rid].traces)
        assert res.traces.shape == (r.nsteps, len(rec), 3) and np.abs(res.traces).max() > 0


@pytest.mark.parametrize("precision", [64, 32])
def test_served_requests_match_oracle(precision):
    """Three requests (N = 3, 4 and 5 on cubes of 3^3 and 4^3 hexahedra, each
    with its own medium and source) served together with two slots, so one
    joins while the others run; every result against the oracle."""
    import paper_1711_01175_amd as P
    from helpers import quad_points
    from oracle import timestep
    from oracle.dg import Elastic
    from oracle.reference import stroud_rule
    from paper_1711_01175_amd.serving import Server
    reqs = request_stream(3, n_range=(3, 4), degrees=(3, 4, 5), nsteps=16, seed0=90)
    for r, N in zip(reqs, (3, 4, 5)):
        r.N = N
    reqs[2].nsteps = 10
    tol = 1e-12 if precision == 64 else 1e-5
    budget = 0
    for r in reqs:
        c = P.Context(r.N, precision)
        c.set_mesh(*r.mesh())
        budget += c.workspace_bytes()
        c.close()
    srv = Server(budget_bytes=budget, slots=2, precision=precision, chunk_steps=4, keep_state=True)
    stats = srv.run(reqs)
    assert len(stats.results) == 3 and not stats.rejected
    by = {x.rid: x for x in stats.results}
    for r in reqs:
        EToV, VXYZ = r.mesh()
        xyz = quad_points(VXYZ, stroud_rule(r.N)[0])
        mat = r.material(xyz)
        op = Elastic(r.N, VXYZ, *mat)
        src = timestep.Source(r.xs, r.direction, 1.0, r.f0, r.t0)
        dt = timestep.cfl_dt(op, 0.5)
        cT, _, _ = timestep.run(op, np.zeros((op.K, 9, op.Np)), dt, r.nsteps, source=src)
        ref = op.to_q(cT)
        c = P.Context(r.N, precision)
        c.set_mesh(EToV, VXYZ)
        c.bind_workspace()
        c.set_material(*mat)
        got = c.eval_quadrature(torch.from_numpy(by[r.rid].state).cuda()).cpu().numpy()
        err = op.l2_q(got - ref) / op.l2_q(ref)
        print("served", r.rid, "N", r.N, "K", op.K, "steps", r.nsteps, "rel_l2", f"{err:.3e}", flush=True)
        assert err <= tol


def test_guard_stops_a_poisoned_request():
    """One request's state is set to contain a NaN right after its admission
    (from Python, through the binding).  The server's energy guard stops it
    after its first chunk and frees its slot; the other requests finish, and
    their states and traces equal bitwise those of a run without it."""
    from paper_1711_01175_amd.serving import Server
    rec = np.array([[0.1, 0.2, -0.3]])
    reqs = request_stream(4, n_range=(3, 4), degrees=(2, 3), nsteps=12, seed0=130)
    for r in reqs:
        r.receivers = rec
    bad = reqs[2].rid

    def poison(rid, ctx):
        if rid == bad:
            q = torch.zeros((ctx.K, 9, ctx.Np), dtype=ctx.torch_dtype, device="cuda")
            q[ctx.K // 2, 4, 0] = float("nan")
            ctx.set_state(q, 0.0)

    srv = Server(budget_bytes=1 << 34, slots=4, precision=32, chunk_steps=3, keep_state=True)
    stats = srv.run(reqs, on_admit=poison)
    print(stats.summary(), [(f.rid, f.reason, f.steps_done) for f in stats.failed], flush=True)
    assert [f.rid for f in stats.failed] == [bad]
    assert stats.failed[0].reason == "non-finite energy" and stats.failed[0].steps_done == 3
    assert sorted(r.rid for r in stats.results) == sorted(r.rid for r in reqs if r.rid != bad)
    clean = Server(budget_bytes=1 << 34, slots=4, precision=32, chunk_steps=3, keep_state=True)
    ref = {x.rid: x for x in clean.run([Request(r.rid, r.n, r.N, r.nsteps, r.xs, r.phases, r.amps, 0.0,
                                                r.direction, r.f0, r.t0, rec) for r in reqs if r.rid != bad]).results}
    for x in stats.results:
        assert np.array_equal(x.state, ref[x.rid].state)
        assert np.array_equal(x.traces, ref[x.rid].traces)
        assert np.isfinite(x.energy)
