"""Throughput benchmark of the fused DG right-hand side + LSRK(5,4) step.

Workload (default): heterogeneous periodic cube [-1,1]^3 of 32^3 hexahedra x 6
= 196,608 tetrahedra, degree N=4 (35 nodes), 9 fields, smooth rho, lambda,
mu sampled at the quadrature points, Ricker point source (f0=5), time step
at CFL 0.5.  One "step" is one LSRK(5,4) step, i.e. five fused stage
launches over the whole mesh.  Inputs are resident in HBM before timing.

Prints one JSON line.  GDOF/s counts K*Np*9 degrees of freedom per RHS
evaluation (five per step).  The FP32 run is the headline value; the FP64
run and the FP64 CPU oracle (timed on a bounded sample) are reported beside
it.
"""
import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0
TRAFFIC_PROFILE = os.path.join(ROOT, "profiles", "k_stage_cube32_N4.md")
KERNEL_SOURCES = ("kernels.hip", "kcommon.hpp", "dev.hpp", "tiles.hpp")


def kernel_source_digest():
    """sha256 over the stage kernel's sources (kernels.hip, kcommon.hpp, dev.hpp,
    tiles.hpp), to tell whether the committed
    counter profile was taken on the kernel that runs now."""
    import hashlib
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, "paper_1711_01175_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def profiled_traffic(prec):
    """HBM bytes per stage launch from the committed rocprofv3 counter runs
    (FETCH_SIZE and WRITE_SIZE scaled by the copy calibration), or None if
    the profile is missing or was taken on other kernel sources."""
    try:
        with open(TRAFFIC_PROFILE) as fh:
            text = fh.read()
    except OSError:
        return None
    vals = {}
    for line in text.splitlines():
        if line.startswith("traffic-record "):
            k, _, v = line[len("traffic-record "):].partition("=")
            vals[k.strip()] = v.strip()
    if vals.get("kernel_source_sha256") != kernel_source_digest():
        return None
    v = vals.get(f"bytes_per_launch_fp{prec}")
    return int(v) if v else None
METRIC = "DG RHS GDOF/s at N=4, FP32 vs FP64 vs oracle; batched solve p50/p99 latency"


def algorithmic_bytes_per_element(Np, Nq, b):
    """Compulsory HBM bytes per element per stage: q and the LSRK register
    read and written (36 Np b), the density-weighted mass inverse (Np^2 b),
    lambda and mu at the quadrature points (2 Nq b), geometry (26 b) and
    connectivity (48 B)."""
    return 36 * Np * b + Np * Np * b + 2 * Nq * b + 26 * b + 48


def flops_per_element(Np, Nfp, Nq):
    """Flops per element per stage: volume 36 Np^2 (18 reference products),
    stress projection 24 Nq Np + 10 Nq, lift 72 Np Nfp, mass inverse 6 Np^2,
    interface flux about 480 Nfp, LSRK update 36 Np."""
    return 36 * Np * Np + 24 * Nq * Np + 10 * Nq + 72 * Np * Nfp + 6 * Np * Np + 480 * Nfp + 36 * Np


PEAK_HBM_GBS = 8000.0
PEAK_TFLOPS = {32: 157.3, 64: 78.6}   # MI355X dense FP32 / FP64 matrix


def sweep_degrees(steps=10, warmup=2):
    """Stage time per degree on the workload meshes of each degree (N=3, 4:
    32^3 x 6 tets; N=5: 24^3 x 6; N=7: 16^3 x 6), both precisions, with the
    HBM and matrix-core roofline fractions of the algorithmic work."""
    out = {"sweep": "degrees", "steps": steps, "rows": []}
    for N, n in ((3, 32), (4, 32), (5, 24), (7, 16)):
        EToV, VXYZ, _ = build_workload(n, N)
        for prec in (32, 64):
            r = run_gpu(prec, N, n, steps, warmup, EToV, VXYZ)
            K, Np, Nq = r["K"], r["Np"], r["Nq"]
            Nfp = (N + 1) * (N + 2) // 2
            s = r["ms"] * 1e-3 / (5 * steps)
            b = algorithmic_bytes_per_element(Np, Nq, prec // 8) * K
            f = flops_per_element(Np, Nfp, Nq) * K
            out["rows"].append({"N": N, "K": K, "prec": prec, "stage_us": round(s * 1e6, 1),
                                "GDOF_per_s": round(K * Np * 9 / s / 1e9, 2),
                                "hbm_frac": round(b / s / 1e9 / PEAK_HBM_GBS, 3),
                                "mfma_frac": round(f / s / 1e12 / PEAK_TFLOPS[prec], 3)})
            print(json.dumps(out["rows"][-1]), file=sys.stderr, flush=True)
    print(json.dumps(out), flush=True)


def _jacobians(VXYZ):
    X = VXYZ
    return np.abs(np.linalg.det(np.stack([X[:, 1] - X[:, 0], X[:, 2] - X[:, 0], X[:, 3] - X[:, 0]], -1))) / 8.0


def _l2q(fq, J, wq):
    """L2_Q norm of device values [K][9][Nq] with element Jacobians J [K]."""
    import torch
    w = torch.as_tensor(J, device=fq.device)[:, None, None] * torch.as_tensor(wq, device=fq.device)[None, None, :]
    return float(torch.sqrt(torch.sum(w * fq * fq)))


def _context(prec, N, EToV, VXYZ, perturb=False, max_rec=0, max_steps=0):
    import torch

    import paper_1711_01175_amd as P
    from workloads import media
    c = P.Context(N, prec, stream=torch.cuda.current_stream().cuda_stream)
    c.set_mesh(EToV, VXYZ)
    c.bind_workspace(max_rec, max_steps)
    mat = media.smooth(c.quadrature_points())
    if perturb:
        mat = media.perturb_per_element(*mat, 3, frac=0.1)
    c.set_material(*mat)
    c.set_source([0.05, -0.10, 0.15], [0.0, 0.0, 1.0], 1.0, 5.0, 0.2)
    return c


def run_pair(N, n, nsteps, perturb=False, warmup=0):
    """FP64 and FP32 runs of the same workload from a zero state: stage time
    of each (HIP events around nsteps steps after `warmup` steps, on the
    context's stream), energy, and the FP32 state's relative L2_Q distance
    from the FP64 one after warmup + nsteps steps."""
    import torch
    EToV, VXYZ, _ = build_workload(n, N)
    J = _jacobians(VXYZ)
    out, fq = {}, {}
    for prec in (64, 32):
        c = _context(prec, N, EToV, VXYZ, perturb)
        dt = c.cfl_dt(0.5)
        c.step(dt, warmup)
        stream = torch.cuda.current_stream()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        ev0.record(stream)
        c.step(dt, nsteps)
        ev1.record(stream)
        torch.cuda.synchronize()
        out[prec] = dict(stage_us=ev0.elapsed_time(ev1) * 1e3 / (5 * nsteps), energy=c.energy())
        fq[prec] = c.eval_quadrature()
        wq = c.reference_operator(8)
        K, Np, Nq = c.K, c.Np, c.Nq
        c.close()
    rel = _l2q(fq[32] - fq[64], J, wq) / _l2q(fq[64], J, wq)
    del fq
    torch.cuda.empty_cache()
    return dict(K=K, Np=Np, Nq=Nq, steps=warmup + nsteps, fp32=out[32], fp64=out[64], rel_l2_fp32_vs_fp64=rel)


def run_golden():
    """Both precisions on the 8^3 x 6 = 3,072-tet cube for the 1000 steps of
    the stored oracle run (tests/golden/long_run_n8_N4.npz, written by the
    committed script beside it): relative L2_Q error on the stored elements,
    relative energy error and trace error, against the oracle's values."""
    import torch
    g = np.load(os.path.join(ROOT, "tests", "golden", "long_run_n8_N4.npz"))
    N, nsteps = 4, int(g["nsteps"])
    EToV, VXYZ, _ = build_workload(8, N)
    J = _jacobians(VXYZ)[g["elems"]]
    rec = g["receivers"]
    res = {}
    for prec in (64, 32):
        c = _context(prec, N, EToV, VXYZ, max_rec=len(rec), max_steps=nsteps)
        c.set_receivers(rec)
        c.step(c.cfl_dt(0.5), nsteps)
        got = c.eval_quadrature()[torch.as_tensor(g["elems"], device="cuda")]
        ref = torch.as_tensor(g["fq"], device="cuda")
        wq = c.reference_operator(8)
        tr = c.receivers()
        res[f"fp{prec}"] = {"rel_l2": _l2q(got - ref, J, wq) / _l2q(ref, J, wq),
                            "energy_rel": abs(c.energy() - float(g["energy"])) / float(g["energy"]),
                            "trace_err": float(np.abs(tr - g["traces"]).max() / np.abs(g["traces"]).max())}
        c.close()
    res["workload"] = (f"8^3 hexes x 6 = 3072 tets, N=4, same media and source as the headline, {nsteps} steps, "
                       f"against the FP64 oracle's stored run on {len(g['elems'])} elements")
    return res


def build_workload(n, N):
    from workloads import media
    from workloads.mesh import kuhn_periodic_mesh
    EToV, VXYZ = kuhn_periodic_mesh(n)
    return EToV, VXYZ, media


def run_gpu(prec, N, n, steps, warmup, EToV, VXYZ, boundary=None, mass="exact", keep=False):
    import torch

    import paper_1711_01175_amd as P
    from workloads import media
    stream = torch.cuda.current_stream()
    c = P.Context(N, prec, stream=stream.cuda_stream)
    c.set_mesh(EToV, VXYZ, boundary=boundary)
    c.bind_workspace()
    c.set_mass_inverse(mass)
    xyz = c.quadrature_points()
    rho, lam, mu = media.smooth(xyz)
    del xyz
    c.set_material(rho, lam, mu)
    c.set_source([0.05, -0.10, 0.15], [0.0, 0.0, 1.0], 1.0, 5.0, 0.2)
    dt = c.cfl_dt(0.5)
    c.set_state(torch.zeros((c.K, 9, c.Np), dtype=c.torch_dtype, device="cuda"), 0.0)
    c.step(dt, warmup)
    torch.cuda.synchronize()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    c.step(dt, steps)
    ev1.record(stream)
    torch.cuda.synchronize()
    ms = ev0.elapsed_time(ev1)
    energy = c.energy()
    out = dict(K=c.K, Np=c.Np, Nq=c.Nq, dt=dt, ms=ms, energy=energy, t=c.time())
    if keep:
        out["fq"] = c.eval_quadrature()
        out["wq"] = c.reference_operator(8)
    c.close()
    torch.cuda.empty_cache()
    return out


def probe_copy(nbytes=2 << 30, reps=5):
    """Plain device-to-device copy of nbytes (read nbytes + write nbytes):
    the reference for scaling HBM counters and for achievable bandwidth."""
    import torch
    x = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    y.copy_(x)
    torch.cuda.synchronize()
    ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    ev0.record()
    for _ in range(reps):
        y.copy_(x)
    ev1.record()
    torch.cuda.synchronize()
    s = ev0.elapsed_time(ev1) * 1e-3 / reps
    print(json.dumps({"probe": "copy", "bytes_read": nbytes, "bytes_written": nbytes,
                      "seconds": s, "GBs_read_plus_write": 2 * nbytes / s / 1e9}), flush=True)


def probe_bandwidth(nbytes=4 << 30, reps=10):
    """Achievable HBM rates of plain torch kernels on nbytes FP32 tensors:
    elementwise x + 1 (read + write), fill (write), copy (read + write) and
    sum (read)."""
    import torch
    n = nbytes // 4
    x = torch.ones(n, dtype=torch.float32, device="cuda")
    y = torch.empty_like(x)
    out = {"probe": "bandwidth", "bytes": nbytes}
    for name, fn, moved in (("add_read_plus_write", lambda: torch.add(x, 1.0, out=y), 2 * nbytes),
                            ("fill_write", lambda: y.fill_(1.0), nbytes),
                            ("copy_read_plus_write", lambda: y.copy_(x), 2 * nbytes),
                            ("sum_read", lambda: x.sum(), nbytes)):
        fn()
        torch.cuda.synchronize()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        for _ in range(reps):
            fn()
        ev1.record()
        torch.cuda.synchronize()
        out[name + "_GBs"] = round(moved / (ev0.elapsed_time(ev1) * 1e-3 / reps) / 1e9, 1)
    print(json.dumps(out), flush=True)


def run_serving(full=False):
    """Continuous-batching serving of a seeded stream of independent solves.

    Full stream: 256 requests, n ~ U{8..24} hexes per axis, N ~ U{3,4,5},
    500 steps each, FP32, 32 slots, 16 GB HBM budget.  Default (reduced):
    64 requests, n ~ U{6..14}, 100 steps, same slots and budget.  A first
    pass with every request queued at t = 0 measures the saturation rate
    (requests/s); the reported pass uses Poisson arrivals at 0.8 x that rate.
    """
    from paper_1711_01175_amd.serving import Server
    from workloads.requests import request_stream
    if full:
        kw = dict(count=256, n_range=(8, 24), nsteps=500)
    else:
        kw = dict(count=64, n_range=(6, 14), nsteps=100)
    budget, slots = 16 << 30, 32
    calib_count = min(64, kw["count"])

    def progress(tag):
        last = [0.0]

        def cb(done, total, elapsed):
            if elapsed - last[0] >= 20.0 or done == total:
                last[0] = elapsed
                print(f"serving {tag}: {done}/{total} requests done at {elapsed:.1f} s", file=sys.stderr,
                      flush=True)
        return cb

    # saturation: the stream's first calib_count requests, all queued at t = 0
    srv = Server(budget, slots=slots, precision=32)
    calib = srv.run(request_stream(**kw)[:calib_count], progress=progress("calibration"))
    srv.close()
    sat = len(calib.results) / calib.makespan
    rate = 0.8 * sat
    srv = Server(budget, slots=slots, precision=32)
    stats = srv.run(request_stream(rate=rate, **kw), progress=progress("poisson"))
    srv.close()
    out = stats.summary()
    out.update({"workload": f"{kw['count']} requests, n~U{{{kw['n_range'][0]}..{kw['n_range'][1]}}} hexes/axis x 6 tets, "
                            f"N~U{{3,4,5}}, {kw['nsteps']} LSRK steps each, FP32, random media and source per request, "
                            f"Poisson arrivals",
                "full_stream": bool(full), "slots": slots, "budget_bytes": budget,
                "saturation_req_per_s": sat, "saturation_from": f"the first {calib_count} requests queued at t=0",
                "arrival_rate_req_per_s": rate,
                "accuracy": "each served result equals a solo run bitwise (tests/test_gpu_serving.py); "
                            "solo runs are held to the FP64 oracle at 1e-5 (FP32)",
                "max_active": stats.max_active, "max_used_bytes": stats.max_used_bytes})
    return out


def run_adjoint(check_fp64=True):
    """Misfit gradient on the inversion workload: 12^3 x 6 = 10,368 tets,
    N=4, 16 receivers, 800 steps at CFL 0.5, checkpoints every 50 steps,
    data from the Gaussian-mu model.  Times the checkpointed forward and
    the reverse sweep in FP32 and reports the FP32 gradient's distance from
    the FP64 one."""
    import torch

    import paper_1711_01175_amd as P
    from workloads import inversion
    from workloads.mesh import kuhn_periodic_mesh
    nsteps, every, N = 800, 50, 4
    EToV, VXYZ = kuhn_periodic_mesh(12)
    rec = inversion.receiver_grid()
    S = inversion.SOURCE
    res = {}
    data = dt = None
    for prec in ((64, 32) if check_fp64 else (32,)):
        stream = torch.cuda.current_stream()
        c = P.Context(N, prec, stream=stream.cuda_stream)
        c.set_mesh(EToV, VXYZ)
        c.bind_workspace(len(rec), nsteps)
        c.bind_adjoint_workspace(nsteps, every)
        ref, true = inversion.media_pair(c.quadrature_points())
        c.set_source(S["xs"], S["direction"], S["amp"], S["f0"], S["t0"])
        c.set_receivers(rec)
        if data is None:
            c.set_material(*true)
            dt = c.cfl_dt(0.5)
            c.step(dt, nsteps)
            data = c.receivers()
        c.set_material(*ref)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        J = c.forward_misfit(dt, nsteps, data)
        t1 = time.perf_counter()
        g, _ = c.adjoint_gradient()
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        res[prec] = dict(J=J, g=g.cpu().numpy(), fwd=t1 - t0, adj=t2 - t1, K=c.K,
                         ws=c.workspace_bytes(len(rec), nsteps)
                         + c.adjoint_workspace_bytes(nsteps, every, overlapped=True))
        c.close()
        torch.cuda.empty_cache()
    r = res[32]
    out = {"workload": f"12^3 hexes x 6 = {r['K']} tets, N=4, 16 receivers, {nsteps} LSRK steps at CFL 0.5, "
                       f"checkpoints every {every} steps (next segment recomputed on a second stream), "
                       f"data from a Gaussian mu anomaly; FP32",
           "forward_s": round(r["fwd"], 4), "gradient_s": round(r["adj"], 4),
           "gradient_over_forward": round(r["adj"] / r["fwd"], 3), "J": r["J"],
           "device_bytes": int(r["ws"])}
    if 64 in res:
        g64 = res[64]["g"]
        out["fp32_vs_fp64_gradient_rel_l2"] = float(np.linalg.norm(r["g"] - g64) / np.linalg.norm(g64))
        out["fp64_forward_s"] = round(res[64]["fwd"], 4)
        out["fp64_gradient_s"] = round(res[64]["adj"], 4)
    return out


def implicit_bytes_per_element(Np, b):
    """Compulsory HBM bytes per element of one iHDG-II iteration's update
    kernel: the stored local inverse (9 Np)^2 values, the fixed right-hand
    side, the operator output and the state read, the state written."""
    nv = 9 * Np
    return nv * nv * b + 4 * nv * b


def run_implicit(n=16, N=4, cfl=4.0, theta=0.5, nsteps=10):
    """Locally implicit steps (Crank-Nicolson solved by iHDG-II) on the
    heterogeneous cube of n^3 x 6 tets at degree N, both precisions: set-up
    time, iterations per step, time per step and per iteration, the update
    kernel's inverse stream per iteration, the cost of the same simulated time
    with the explicit LSRK(5,4) path at CFL 0.5, and FP32 against FP64.
    The state is first advanced explicitly to t = 0.2 (the source wavelet's
    peak); the stopping tolerance is 1e-6 (FP32) or 1e-10 (FP64) of the
    state's L2 norm."""
    import torch
    EToV, VXYZ, _ = build_workload(n, N)
    J = _jacobians(VXYZ)
    res, fq = {}, {}
    for prec in (64, 32):
        c = _context(prec, N, EToV, VXYZ)
        wq = c.reference_operator(8)
        dte = c.cfl_dt(0.5)
        c.step(dte, int(round(0.2 / dte)))
        # explicit stage time on the same context (20 steps)
        stream = torch.cuda.current_stream()
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record(stream)
        c.step(dte, 20)
        ev1.record(stream)
        torch.cuda.synchronize()
        stage_us = ev0.elapsed_time(ev1) * 1e3 / 100
        c.bind_implicit_workspace()
        dt = c.cfl_dt(cfl)
        t0 = time.perf_counter()
        c.implicit_setup(dt, theta)
        setup_s = time.perf_counter() - t0
        tol = (1e-6 if prec == 32 else 1e-10) * _l2q(c.eval_quadrature(), J, wq)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        iters, change = c.implicit_step(nsteps, tol, 500)
        torch.cuda.synchronize()
        step_s = (time.perf_counter() - t0) / nsteps
        fq[prec] = c.eval_quadrature()
        nit = float(np.mean(iters))
        res[prec] = {"setup_s": round(setup_s, 3), "iterations_per_step": [int(x) for x in iters],
                     "ms_per_step": round(step_s * 1e3, 3), "ms_per_iteration": round(step_s * 1e3 / nit, 4),
                     "inverse_stream_GBs": round(implicit_bytes_per_element(c.Np, prec // 8) * c.K
                                                 / (step_s / nit) / 1e9, 1),
                     "explicit_stage_us": round(stage_us, 2),
                     "explicit_ms_same_time": round(stage_us * 5 * dt / dte / 1e3, 3),
                     "converged": bool(np.all(change < tol))}
        K = c.K
        c.close()
        torch.cuda.empty_cache()
        print(f"implicit leg FP{prec}: {res[prec]}", file=sys.stderr, flush=True)
    rel = _l2q(fq[32] - fq[64], J, wq) / _l2q(fq[64], J, wq)
    return {"workload": f"{n}^3 hexes x 6 = {K} tets, N={N}, smooth media, Ricker source; Crank-Nicolson "
                        f"(theta={theta}) at CFL {cfl} ({cfl / 0.5:g} x the explicit step), {nsteps} steps from the "
                        f"explicit state at t=0.2, solved by iHDG-II",
            "fp32": res[32], "fp64": res[64], "rel_l2_fp32_vs_fp64": rel,
            "update_kernel_bytes_per_iteration": {str(p): implicit_bytes_per_element(Np, p // 8) * K
                                                  for p, Np in ((32, (N + 1) * (N + 2) * (N + 3) // 6),
                                                                (64, (N + 1) * (N + 2) * (N + 3) // 6))}}


def run_transport(d=3, p=4, n=48):
    """Steady transport (Sec. 4.1) by iHDG-II on n^d cubes of degree p, both
    precisions: iterations (Theorem 1 predicts d (n - 1) + 2 with the stopping
    rule of Sec. 6.1), time per iteration, the sweep's flop rate, FP32 against
    FP64, and the counts of the Table 1 configurations."""
    import paper_1711_01175_amd as P
    sys.path.insert(0, os.path.join(ROOT, "tests"))
    from test_oracle_transport import smooth, table1
    ue, f, b = smooth(d)
    res, vals, inputs = {}, {}, None
    for prec in (64, 32):
        T = P.Transport(d, p, n, b, precision=prec)
        T.bind_workspace()
        if inputs is None:
            xv, xf = T.points()
            inputs = (f(xv), ue(xf), ue(xv))
            del xv, xf
        t0 = time.perf_counter()
        T.set_problem(*inputs)
        setup = time.perf_counter() - t0
        t0 = time.perf_counter()
        iters, hist = T.solve(1e-10, 10 * d * n)
        el = time.perf_counter() - t0
        vals[prec] = T.values()
        flops = 2 * d * T.Np * T.Np * T.E
        res[prec] = {"iterations": iters, "setup_s": round(setup, 3), "solve_s": round(el, 4),
                     "ms_per_iteration": round(el / iters * 1e3, 4),
                     "sweep_TFLOPs": round(flops / (el / iters) / 1e12, 2),
                     "error_vs_exact": float(hist[-1])}
        E, Np = T.E, T.Np
        T.close()
        print(f"transport leg FP{prec}: {res[prec]}", file=sys.stderr, flush=True)
    del inputs
    rel = float(np.linalg.norm(vals[32] - vals[64]) / np.linalg.norm(vals[64]))
    counts = []
    for dd, nn, pp, paper in table1():
        ue2, f2, b2 = smooth(dd)
        T = P.Transport(dd, pp, nn, b2, precision=64)
        T.bind_workspace()
        xv, xf = T.points()
        T.set_problem(f2(xv), ue2(xf), ue2(xv))
        counts.append([dd, nn, pp, paper, T.solve(1e-10, 1000)[0]])
        T.close()
    return {"workload": f"beta . grad u = f on the unit cube, beta = {tuple(b)}, smooth exact solution, {n}^{d} = "
                        f"{E} cubes of degree {p} ({Np} modes), iHDG-II from zero, stopping rule with the exact "
                        f"solution at 1e-10",
            "predicted_iterations": d * (n - 1) + 2, "fp32": res[32], "fp64": res[64],
            "rel_l2_fp32_vs_fp64_at_points": rel, "flops_per_iteration": 2 * d * Np * Np * E,
            "table1_d_n_p_paper_ours": counts}


def run_bounded(n=32, N=4, steps=20, warmup=2):
    """The headline workload on the box [-1,1]^3 without the periodic wrap:
    stage time with traction-free and with absorbing boundary faces (12 n^2
    of them), against the periodic stage of the same run."""
    from workloads.mesh import kuhn_box_mesh
    EToV, VXYZ = kuhn_box_mesh(n)
    out = {"workload": f"{n}^3 hexes x 6 = {6 * n ** 3} tets in the box, N={N}, {12 * n * n} boundary faces, "
                       f"smooth media, Ricker source, {steps} steps"}
    for prec in (32, 64):
        row = {}
        for bc in ("free", "absorbing"):
            r = run_gpu(prec, N, n, steps, warmup, EToV, VXYZ, boundary=bc)
            row[bc + "_stage_us"] = round(r["ms"] * 1e3 / (5 * steps), 2)
        out[f"fp{prec}"] = row
    return out


def wadg_bytes_per_element(Np, Nq, b):
    """Compulsory HBM bytes per element of a stage with the weight-adjusted
    mass inverse: q and the LSRK register read and written (36 Np b), 1/rho,
    lambda, mu at the quadrature points (3 Nq b), geometry and connectivity
    (26 b + 48 B), the raw velocity right-hand side written and read (6 Np b)."""
    return 36 * Np * b + 3 * Nq * b + 26 * b + 48 + 6 * Np * b


def run_wadg(steps=40, warmup=2):
    """Stage time with the weight-adjusted mass inverse (no stored W_rho) at
    N = 4 on 32^3 x 6 tets and N = 7 on 16^3 x 6, both precisions, against
    the exact inverse, and the two schemes' relative L2 distance after
    warmup + steps steps (the approximation, not rounding)."""
    out = {}
    for N, n in ((4, 32), (7, 16)):
        EToV, VXYZ, _ = build_workload(n, N)
        J = _jacobians(VXYZ)
        row = {}
        for prec in (32, 64):
            ex = run_gpu(prec, N, n, steps, warmup, EToV, VXYZ, keep=True)
            wa = run_gpu(prec, N, n, steps, warmup, EToV, VXYZ, mass="weight-adjusted", keep=True)
            K, Np, Nq = wa["K"], wa["Np"], wa["Nq"]
            st = wa["ms"] * 1e-3 / (5 * steps)
            bw = wadg_bytes_per_element(Np, Nq, prec // 8) * K
            row[f"fp{prec}"] = {"exact_stage_us": round(ex["ms"] * 1e3 / (5 * steps), 1),
                                "wadg_stage_us": round(st * 1e6, 1),
                                "wadg_GDOF_per_s": round(K * Np * 9 / st / 1e9, 2),
                                "wadg_bytes_per_stage": bw,
                                "wadg_hbm_frac": round(bw / st / 1e9 / PEAK_HBM_GBS, 3),
                                "rel_l2_wadg_vs_exact": _l2q(wa["fq"] - ex["fq"], J, wa["wq"]) / _l2q(ex["fq"], J, wa["wq"])}
            del ex, wa
            print(f"wadg leg N={N} FP{prec}: {row[f'fp{prec}']}", file=sys.stderr, flush=True)
        out[f"N{N}"] = dict(workload=f"{n}^3 hexes x 6 = {6 * n ** 3} tets, N={N}, smooth media, Ricker source, "
                                     f"{warmup} + {steps} steps", **row)
    return out


def cpu_baseline(N, n_sample, seconds):
    """Time the FP64 oracle's RHS on a smaller mesh of the same workload
    (per-element work does not depend on the mesh size)."""
    from threadpoolctl import threadpool_info

    from oracle.dg import Elastic
    from oracle.reference import stroud_rule
    from workloads import media
    from workloads.mesh import kuhn_periodic_mesh
    EToV, VXYZ = kuhn_periodic_mesh(n_sample)
    xq, _ = stroud_rule(N)
    X0 = VXYZ[:, 0]
    A = np.stack([VXYZ[:, 1] - X0, VXYZ[:, 2] - X0, VXYZ[:, 3] - X0], axis=-1) / 2.0
    xyz = np.einsum('qd,kjd->kqj', xq + 1.0, A) + X0[:, None, :]
    op = Elastic(N, VXYZ, *media.smooth(xyz))
    c = np.random.default_rng(0).standard_normal((op.K, 9, op.Np))
    op.rhs(c)
    calls, t0 = 0, time.perf_counter()
    while True:
        op.rhs(c)
        calls += 1
        el = time.perf_counter() - t0
        if el >= seconds:
            break
    threads = max([t.get("num_threads", 1) for t in threadpool_info()] + [1])
    gdofs = op.K * op.Np * 9 * calls / el / 1e9
    return dict(value=gdofs, unit="GDOF/s", cores=int(threads), kind="oracle",
                sample=f"{calls} RHS evaluations of the FP64 oracle on the same workload "
                       f"(N={N}, same media) restricted to a {n_sample}^3 x 6 = {op.K}-element mesh, "
                       f"{el:.1f} s")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=10)
    ap.add_argument("--n", type=int, default=32, help="hexahedra per axis")
    ap.add_argument("--N", type=int, default=4, help="polynomial degree")
    ap.add_argument("--skip-fp64", action="store_true")
    ap.add_argument("--cpu-seconds", type=float, default=15.0)
    ap.add_argument("--cpu-n", type=int, default=8)
    ap.add_argument("--no-serving", action="store_true", help="skip the serving leg")
    ap.add_argument("--no-adjoint", action="store_true", help="skip the adjoint leg")
    ap.add_argument("--serving-reduced", action="store_true",
                    help="serve a reduced 64-request stream instead of the full 256-request one")
    ap.add_argument("--no-accuracy", action="store_true",
                    help="skip the 1000-step FP32/FP64 and oracle comparisons and the N=7 leg")
    ap.add_argument("--no-implicit", action="store_true", help="skip the locally implicit (iHDG-II) leg")
    ap.add_argument("--no-transport", action="store_true", help="skip the steady transport (iHDG-II) leg")
    ap.add_argument("--wadg-only", action="store_true",
                    help="run only the weight-adjusted mass inverse leg and print its JSON (for profiling)")
    ap.add_argument("--serving-only", action="store_true",
                    help="run only the serving leg (full stream unless --serving-reduced) and print its JSON")
    ap.add_argument("--transport-only", action="store_true",
                    help="run only the steady transport leg and print its JSON (for profiling)")
    ap.add_argument("--implicit-only", action="store_true",
                    help="run only the locally implicit leg and print its JSON (for profiling)")
    ap.add_argument("--adjoint-only", action="store_true",
                    help="run only the FP32 adjoint leg and print its JSON (for profiling)")
    ap.add_argument("--probe-copy", action="store_true",
                    help="time a plain device copy of 2 GiB instead (HBM calibration)")
    ap.add_argument("--sweep-degrees", action="store_true",
                    help="time the stage at N=3, 4, 5, 7 in both precisions instead (one JSON line)")
    ap.add_argument("--probe-bandwidth", action="store_true",
                    help="time plain torch kernels on 4 GiB tensors instead (achievable HBM rates)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py runs on exactly one GPU: the library has no multi-GPU path.", file=sys.stderr)
        sys.exit(2)
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    if args.probe_copy:
        probe_copy()
        return
    if args.probe_bandwidth:
        probe_bandwidth()
        return
    if args.sweep_degrees:
        sweep_degrees()
        return
    if args.adjoint_only:
        print(json.dumps({"adjoint": run_adjoint(check_fp64=False)}), flush=True)
        return
    if args.implicit_only:
        print(json.dumps({"implicit": run_implicit()}), flush=True)
        return
    if args.transport_only:
        print(json.dumps({"transport": run_transport()}), flush=True)
        return
    if args.serving_only:
        print(json.dumps({"serving": run_serving(not args.serving_reduced)}), flush=True)
        return
    if args.wadg_only:
        print(json.dumps({"weight_adjusted": run_wadg()}), flush=True)
        return
    EToV, VXYZ, _ = build_workload(args.n, args.N)
    r32 = run_gpu(32, args.N, args.n, args.steps, args.warmup, EToV, VXYZ)
    r64 = None if args.skip_fp64 else run_gpu(64, args.N, args.n, args.steps, args.warmup, EToV, VXYZ)
    K, Np, Nq = r32["K"], r32["Np"], r32["Nq"]
    dof = K * Np * 9
    g32 = dof * 5 * args.steps / (r32["ms"] * 1e-3) / 1e9
    stage_s = r32["ms"] * 1e-3 / (5 * args.steps)
    algo = algorithmic_bytes_per_element(Np, Nq, 4) * K
    achieved = algo / stage_s / 1e9
    line = {
        "metric": METRIC,
        "value": round(g32, 3),
        "unit": "GDOF/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(r32["ms"] / args.steps, 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {"workload": f"heterogeneous periodic cube {args.n}^3 hexes x 6 = {K} tets, N={args.N} "
                               f"({Np} nodes), 9 fields, smooth rho/lambda/mu at quadrature nodes, "
                               f"Ricker f0=5, LSRK(5,4) at CFL 0.5",
                   "K": K, "N": args.N, "Np": Np, "dt": r32["dt"], "dof_per_stage": dof},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(achieved / HBM_PEAK_GBS, 4), "traffic": profiled_traffic(32),
                     "traffic_from": "rocprofv3 FETCH_SIZE + WRITE_SIZE per launch, copy-calibrated, recorded in "
                                     "profiles/k_stage_cube32_N4.md for these kernel sources (null if they differ)",
                     "kernel": "k_stage (fused stage)", "stage_us": round(stage_s * 1e6, 2),
                     "algorithmic_bytes_per_stage": algo},
    }
    if r64 is not None:
        g64 = dof * 5 * args.steps / (r64["ms"] * 1e-3) / 1e9
        st64 = r64["ms"] * 1e-3 / (5 * args.steps)
        a64 = algorithmic_bytes_per_element(Np, Nq, 8) * K / st64 / 1e9
        line["fp64"] = {"value": round(g64, 3), "unit": "GDOF/s", "ms_per_step": round(r64["ms"] / args.steps, 4),
                        "roofline_frac": round(a64 / HBM_PEAK_GBS, 4), "achieved_GBs": round(a64, 1)}
        line["fp32_vs_fp64_speedup"] = round(r64["ms"] / r32["ms"], 3)
        line["energy_fp32_fp64"] = [r32["energy"], r64["energy"]]
    if not args.no_accuracy:
        # the headline workload after 1000 steps: FP32 against FP64 (the FP64
        # stepping path is held to the oracle by the test suite)
        acc = run_pair(args.N, args.n, 1000)
        line["accuracy"] = {"rel_l2_fp32_vs_fp64_1000_steps": acc["rel_l2_fp32_vs_fp64"],
                            "energy_fp32_fp64_1000_steps": [acc["fp32"]["energy"], acc["fp64"]["energy"]],
                            "vs_oracle_3072_tets_1000_steps": run_golden()}
        # high order (16^3 x 6 = 24,576 tets, N=7, +-10 % per-element media):
        # stage time against the FP32 / FP64 matrix peaks, 500 steps, FP32 vs FP64
        ho = run_pair(7, 16, 495, perturb=True, warmup=5)
        Nfp7 = 36
        fl = flops_per_element(ho["Np"], Nfp7, ho["Nq"]) * ho["K"]
        line["high_order"] = {
            "workload": f"16^3 hexes x 6 = {ho['K']} tets, N=7 (120 nodes), smooth media x (1 + 0.1 u) per element, "
                        f"Ricker source, {ho['steps']} steps",
            "bound": "mfma",
            "fp32": {"stage_us": round(ho["fp32"]["stage_us"], 1),
                     "GDOF_per_s": round(ho["K"] * ho["Np"] * 9 / ho["fp32"]["stage_us"] / 1e3, 2),
                     "achieved_TFLOPs": round(fl / ho["fp32"]["stage_us"] / 1e6, 2), "peak_TFLOPs": PEAK_TFLOPS[32],
                     "frac": round(fl / ho["fp32"]["stage_us"] / 1e6 / PEAK_TFLOPS[32], 4)},
            "fp64": {"stage_us": round(ho["fp64"]["stage_us"], 1),
                     "GDOF_per_s": round(ho["K"] * ho["Np"] * 9 / ho["fp64"]["stage_us"] / 1e3, 2),
                     "achieved_TFLOPs": round(fl / ho["fp64"]["stage_us"] / 1e6, 2), "peak_TFLOPs": PEAK_TFLOPS[64],
                     "frac": round(fl / ho["fp64"]["stage_us"] / 1e6 / PEAK_TFLOPS[64], 4)},
            "rel_l2_fp32_vs_fp64": ho["rel_l2_fp32_vs_fp64"],
            "flops_per_stage": fl}
    if not args.no_serving:
        line["serving"] = run_serving(not args.serving_reduced)
    if not args.no_adjoint:
        line["adjoint"] = run_adjoint()
    if not args.no_implicit:
        line["implicit"] = run_implicit()
    if not args.no_transport:
        line["transport"] = run_transport()
    if not args.no_accuracy:
        line["bounded"] = run_bounded()
        line["weight_adjusted"] = run_wadg()
    if args.cpu_seconds > 0:
        line["cpu_baseline"] = cpu_baseline(args.N, args.cpu_n, args.cpu_seconds)
    print(json.dumps(line), flush=True)


if __name__ == "__main__":
    main()
