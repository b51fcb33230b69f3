"""Continuous-batching server for many independent forward solves.

Requests (a mesh, degree, medium, source and step count each) arrive over
time.  A request is admitted as soon as a slot is free and its exact device
footprint (ewdg_workspace_bytes) fits in the remaining HBM budget, in arrival
order, except that a later request may pass a head that does not fit if it
cannot delay that head (backfilling, admit_backfill); its state then stays on
the device until it retires.  All admitted requests advance
together through ewdg_step_batch: each LSRK stage is one ragged launch per
degree class over every active request's elements, so requests that arrive
while others run join the same launches at the next chunk boundary.  Each
request's arithmetic is identical to a solo run, so results do not depend on
the mix.

Host preparation of arrived requests (worker threads) and device setup of
admitted ones (a side stream) overlap the running chunk, and chunks are
queued two deep so the device does not wait for the host between them.

Each request's health is checked after every chunk: its energy (the FP64
reduction of the library, enqueued on the chunk stream without a sync) must
stay finite and must not grow by more than a set factor within one chunk.
A request that fails stops advancing; its slot and memory are released once
the chunks already queued with it have run, and the other requests are not
affected (their arithmetic never reads another request's data).

Only orchestration lives here; every step of the method runs in libewdg.
"""
import math
import time
from collections import deque
from dataclasses import dataclass, field

import numpy as np

from . import ewdg as B


def admit_backfill(waiting, n_active, used_bytes, slots, budget, releases=()):
    """First-in first-out admission with backfilling.

    waiting: sequence of (key, footprint_bytes) in arrival order; releases:
    (steps_left, footprint_bytes) of every running request (all of them
    advance together, so they retire in the order of their steps left).
    Returns (admitted keys, rejected keys).  Requests are admitted in order
    while a slot is free and the footprint fits in the remaining budget.  When
    the head of the queue does not fit, it holds a reservation: the first
    retirement after which the memory and the slot it needs are free.  A
    request behind it is admitted now only if it fits now and what it takes
    still leaves the reservation intact (it is assumed to run past it), so the
    head is never delayed by a request that arrived after it.  Only the head
    holds a reservation: a request further back can start a little later than
    under strict arrival order, while on average requests start earlier.  A
    request larger than the whole budget is rejected.
    """
    admitted, rejected = [], []
    free_slots = slots - n_active
    free_bytes = budget - used_bytes
    spare = None               # (bytes, slots) left over at the head's reservation
    for key, fp in waiting:
        if fp > budget:
            rejected.append(key)
            continue
        if spare is None:
            if free_slots > 0 and fp <= free_bytes:
                admitted.append(key)
                free_slots -= 1
                free_bytes -= fp
                continue
            # the head waits: memory and slots at its reservation
            fb, fs = free_bytes, free_slots
            spare = (0, 0)
            rel = sorted(releases)
            i = 0
            while i < len(rel):
                left = rel[i][0]
                while i < len(rel) and rel[i][0] == left:
                    fb += rel[i][1]
                    fs += 1
                    i += 1
                if fb >= fp and fs >= 1:
                    spare = (fb - fp, fs - 1)
                    break
            continue
        if free_slots > 0 and fp <= free_bytes and fp <= spare[0] and spare[1] >= 1:
            admitted.append(key)
            free_slots -= 1
            free_bytes -= fp
            spare = (spare[0] - fp, spare[1] - 1)
    return admitted, rejected


@dataclass
class _Live:
    req: object
    ctx: object
    footprint: int
    dt: float = 0.0
    done: int = 0        # steps completed on the device
    sched: int = 0       # steps queued (done plus those of chunks in flight)
    t_admit: float = 0.0
    ws: object = None
    material: object = None
    inflight: int = 0    # queued chunks not yet completed
    energy: float = 0.0  # energy after the last checked chunk
    failed: str = None   # why the guard stopped the request


@dataclass
class Result:
    rid: int
    arrival: float
    admitted: float
    finished: float
    latency: float
    K: int
    N: int
    nsteps: int
    energy: float
    traces: np.ndarray
    state: object = None


@dataclass
class Failure:
    rid: int
    arrival: float
    admitted: float
    stopped: float
    reason: str
    K: int
    N: int
    steps_done: int
    energy: float


def energy_check(previous, current, growth_limit):
    """Health of a request after a chunk: None if fine, else the reason.

    The energy must be finite; once it is positive it may not grow by more
    than growth_limit within one chunk (the upwind flux only removes energy;
    the point source adds it smoothly, far below such factors)."""
    if not math.isfinite(current):
        return "non-finite energy"
    if growth_limit is not None and previous > 0.0 and current > growth_limit * previous:
        return f"energy grew {current / previous:.3g}x within one chunk"
    return None


@dataclass
class ServeStats:
    results: list = field(default_factory=list)
    rejected: list = field(default_factory=list)
    failed: list = field(default_factory=list)
    makespan: float = 0.0
    dof_stages: float = 0.0
    max_used_bytes: int = 0
    max_active: int = 0

    def latencies(self):
        return np.array([r.latency for r in self.results])

    def summary(self):
        lat = self.latencies()
        return {
            "requests": len(self.results),
            "rejected": len(self.rejected),
            "failed": len(self.failed),
            "p50_s": float(np.percentile(lat, 50)) if len(lat) else None,
            "p99_s": float(np.percentile(lat, 99)) if len(lat) else None,
            "makespan_s": self.makespan,
            "GDOF_per_s": self.dof_stages / self.makespan / 1e9 if self.makespan > 0 else None,
        }


class Server:
    """Admission by HBM footprint, continuous batching, per-request results.

    Three things overlap the device work of a running chunk: host preparation
    of arrived requests (mesh, quadrature points, sampled media) in worker
    threads, device setup of admitted requests (workspace, FP64 material
    setup) on a side stream, and the bookkeeping of retired requests.  All
    chunks run on one stream of their own; admitted requests join the next
    chunk.
    """

    def __init__(self, budget_bytes, slots=32, precision=32, chunk_steps=10, cfl=0.5,
                 keep_state=False, prep_workers=4, guard=True, growth_limit=1e6):
        import torch
        from concurrent.futures import ThreadPoolExecutor
        self.torch = torch
        self.budget = int(budget_bytes)
        self.slots = int(slots)
        self.precision = int(precision)
        self.chunk = int(chunk_steps)
        self.cfl = float(cfl)
        self.keep_state = keep_state
        self.stream = torch.cuda.Stream()          # chunks
        self.setup_stream = torch.cuda.Stream()    # admissions
        self.retire_stream = torch.cuda.Stream()   # read-back of finished requests
        self.pool = ThreadPoolExecutor(max_workers=int(prep_workers))
        # room for the tables of a whole chunk: one upload per chunk, and each
        # degree class runs on a stream of its own
        per_step = (B.batch_table_bytes(self.slots) + 255) // 256 * 256
        self.table = torch.empty(per_step * self.chunk, dtype=torch.uint8, device="cuda")
        # per-request energies of the (at most two) chunks in flight
        self.guard = bool(guard)
        self.growth_limit = growth_limit
        self.guard_dev = torch.zeros((2, self.slots), dtype=torch.float64, device="cuda")
        self.guard_host = torch.zeros((2, self.slots), dtype=torch.float64).pin_memory()
        self._gbuf = 0

    def close(self):
        self.pool.shutdown(wait=True)

    def _prepare(self, req):
        """Host only (worker thread): context, mesh, footprint, sampled media."""
        ctx = B.Context(req.N, self.precision, stream=self.setup_stream.cuda_stream)
        ctx.set_mesh(*req.mesh())
        nr = len(req.receivers)
        live = _Live(req, ctx, ctx.workspace_bytes(nr, req.nsteps))
        # torch's CPU kernels sample a large medium several times faster than
        # numpy (the media functions accept either)
        fields = req.material(self.torch.from_numpy(ctx.quadrature_points()))
        live.material = tuple(f.numpy() if isinstance(f, self.torch.Tensor) else np.asarray(f) for f in fields)
        return live

    def _start(self, live, now):
        """Device setup on the side stream; returns when it is complete."""
        req, ctx = live.req, live.ctx
        nr = len(req.receivers)
        with self.torch.cuda.stream(self.setup_stream):
            live.ws = ctx.bind_workspace(nr, req.nsteps)
        ctx.set_material(*live.material)
        live.material = None
        ctx.set_source(req.xs, req.direction, 1.0, req.f0, req.t0)
        if nr:
            ctx.set_receivers(req.receivers)
        live.dt = ctx.cfl_dt(self.cfl)
        self.setup_stream.synchronize()
        ctx.set_stream(self.stream.cuda_stream)
        # the workspace was allocated on the setup stream and is used on the
        # chunk and retire streams: its memory is recycled only after the
        # work queued there when it is freed
        live.ws.record_stream(self.stream)
        live.ws.record_stream(self.retire_stream)
        live.t_admit = now

    def _finish(self, live, now, stats):
        req, ctx = live.req, live.ctx
        # the request's last chunk is complete; read back on a stream of its
        # own so the read-back does not wait for the chunk queued after it.
        # The retire stream is torch's current stream here, so the device
        # copy of the state and its transfer to the host are ordered on it.
        ctx.set_stream(self.retire_stream.cuda_stream)
        with self.torch.cuda.stream(self.retire_stream):
            traces = ctx.receivers() if len(req.receivers) else np.zeros((0, 0, 3))
            state = ctx.get_state().cpu().numpy() if self.keep_state else None
            energy = ctx.energy()
        stats.results.append(Result(req.rid, req.arrival, live.t_admit, now, now - req.arrival, ctx.K,
                                    req.N, req.nsteps, energy, traces, state))
        stats.dof_stages += ctx.K * ctx.Np * 9 * 5 * req.nsteps
        ctx.close()
        live.ws = None

    def _release_failed(self, live, now, stats):
        """Free a request the guard stopped (its queued chunks have run)."""
        req, ctx = live.req, live.ctx
        stats.failed.append(Failure(req.rid, req.arrival, live.t_admit, now, live.failed, ctx.K, req.N,
                                    live.done, live.energy))
        ctx.close()
        live.ws = None

    def run(self, requests, clock=time.perf_counter, sleep=time.sleep, progress=None, on_admit=None):
        """Serve requests arriving at req.arrival seconds after the start.

        Chunks are pipelined two deep: the next chunk of every running
        request is queued behind the one on the device before the host
        waits for the older one, so admissions and read-back overlap device
        work and the device does not idle between chunks.

        progress: optional callable(done, total, elapsed_s) called whenever
        requests complete.  on_admit: optional callable(rid, context) called
        once a request's device setup is done, before its first chunk."""
        torch = self.torch
        stats = ServeStats()
        total = len(requests)
        pending = deque(sorted(requests, key=lambda r: (r.arrival, r.rid)))
        waiting, active = deque(), []      # waiting: futures of requests in preparation, arrival order
        inflight = deque()                 # (event, requests, steps, guard buffer) per queued chunk
        used = 0
        t0 = clock()
        while pending or waiting or active or inflight:
            now = clock() - t0
            while pending and pending[0].arrival <= now:
                waiting.append(self.pool.submit(self._prepare, pending.popleft()))
            # queue the next chunk of every request with steps left to queue
            launch = [a for a in active if a.sched < a.req.nsteps]
            if launch and len(inflight) < 2:
                chunk = min(self.chunk, min(a.req.nsteps - a.sched for a in launch))
                B.step_batch([a.ctx for a in launch], [a.dt for a in launch], chunk, self.table,
                             self.stream.cuda_stream)
                gb = None
                if self.guard:
                    gb = self._gbuf
                    self._gbuf ^= 1
                    with torch.cuda.stream(self.stream):
                        for i, a in enumerate(launch):
                            a.ctx.energy_device(self.guard_dev[gb, i:i + 1])
                        self.guard_host[gb, :len(launch)].copy_(self.guard_dev[gb, :len(launch)],
                                                                 non_blocking=True)
                ev = torch.cuda.Event()
                ev.record(self.stream)
                for a in launch:
                    a.sched += chunk
                    a.inflight += 1
                inflight.append((ev, launch, chunk, gb))
            # admission among prepared requests in arrival order, with
            # backfilling behind a head that does not fit (the first request
            # not yet prepared ends the list)
            ready = []
            for f in waiting:
                if not f.done():
                    break
                ready.append(f.result())
            releases = [(a.req.nsteps - a.done, a.footprint) for a in active]
            adm, rej = admit_backfill([(id(w), w.footprint) for w in ready], len(active), used,
                                      self.slots, self.budget, releases)
            adm, rej = set(adm), set(rej)
            admitted = []
            for w in ready:
                if id(w) in rej:
                    stats.rejected.append(w.req.rid)
                    w.ctx.close()
                elif id(w) in adm:
                    self._start(w, clock() - t0)
                    if on_admit is not None:
                        on_admit(w.req.rid, w.ctx)
                    used += w.footprint
                    admitted.append(w)
            if adm or rej:
                taken = adm | rej
                waiting = deque(f for i, f in enumerate(waiting) if i >= len(ready) or id(ready[i]) not in taken)
            for w in admitted:
                if w.req.nsteps <= 0:          # nothing to run: retire at once
                    self._finish(w, clock() - t0, stats)
                    used -= w.footprint
                else:
                    active.append(w)
            stats.max_used_bytes = max(stats.max_used_bytes, used)
            stats.max_active = max(stats.max_active, len(active))
            # wait for the oldest chunk once another is queued behind it (or
            # nothing more can be queued), then retire what it completed
            more = any(a.sched < a.req.nsteps for a in active)
            if inflight and (len(inflight) >= 2 or not more):
                ev, lives, chunk, gb = inflight.popleft()
                ev.synchronize()
                now = clock() - t0
                finished = 0
                for i, a in enumerate(lives):
                    a.inflight -= 1
                    if a.failed is None:
                        a.done += chunk
                        if gb is not None:
                            E = float(self.guard_host[gb, i])
                            a.failed = energy_check(a.energy, E, self.growth_limit)
                            if a.failed is None:
                                a.energy = E
                            else:
                                active.remove(a)      # no further chunks
                        if a.failed is None and a.done >= a.req.nsteps:
                            self._finish(a, now, stats)
                            used -= a.footprint
                            active.remove(a)
                            finished += 1
                    if a.failed is not None and a.inflight == 0 and a.ws is not None:
                        self._release_failed(a, now, stats)
                        used -= a.footprint
                        finished += 1
                if finished and progress is not None:
                    progress(len(stats.results) + len(stats.failed), total, now)
            elif not inflight and not active:
                if waiting:
                    sleep(0.001)
                elif pending:
                    sleep(max(0.0, min(pending[0].arrival - (clock() - t0), 0.01)))
        stats.makespan = clock() - t0
        return stats
