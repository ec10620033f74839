"""Benchmark of the winding-number voxelization path on one MI355X.

Headline step (one pass of the hot path over one batch of input): the batched workload
-- 64 seeded ellipsoid-union meshes of 500 to 50 000 faces, each with its own 32^3,
64^3 or 128^3 grid -- voxelized in ONE persistent, graph-captured launch (pack the
meshes' strip-order vertex records, evaluate the winding number at every voxel centre
of every grid, reduce, map to hard occupancy), all in the HIP library, inputs resident
in HBM.  ``value`` = point-triangle evaluations per second over the timed steps; the
same meshes launched one per call (the plain kernel) are timed beside it.

Rows measured in the same run (``rows``; a compact ``summary`` closes the line):
  * forward_c2: the 19 000-face non-watertight union at 128^3, one mesh per launch;
  * adjoint: forward + sigmoid-MSE loss + wn_backward on the 5120-face icosphere at 64^3;
  * served: continuous batching of a seeded Poisson trace, p50/p99 latency vs the
    plain one-mesh-per-launch loop at several offered loads;
  * naive (Eq. 4), eval (Section 3's evaluation chain), morph (Section 2.4), flip
    (Algorithm 2).

The CPU baseline is the FP64 oracle timed on the host's cores over a bounded,
deterministic per-mesh subsample of the same batch (and, for context, the other
workloads and a one-thread run).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "point-triangle evals/s (FP32) vs FP32 peak; p50/p99 latency served vs plain"
UNIT = "point-triangle evals/s"
FLOP_FWD = 86    # algorithmic FLOPs per forward (point, face) pair
FLOP_BWD = 182   # algorithmic FLOPs per adjoint pair
PEAK_FP32 = 157.3e12   # MI355X FP32 vector peak (256 CU x 2.4 GHz x 256 FLOP/clk)
PEAK_HBM = 8.0e12


# Sources that define each profiled kernel (its code and everything it inlines).
KERNEL_SOURCES = {"k_wn_fwd": ("wn_internal.hpp", "wn_fwd.hip"),
                  "k_batched_persistent": ("wn_internal.hpp", "wn_batched.hip"),
                  "k_wn_bwd": ("wn_internal.hpp", "wn_bwd.hip"),
                  "k_wn_bwd_pairs": ("wn_internal.hpp", "wn_bwd_pairs.hip")}


def source_hash(kernel: str = "k_wn_fwd") -> str:
    h = hashlib.sha256()
    cdir = os.path.join(ROOT, "paper_2407_11272_amd", "csrc")
    for name in KERNEL_SOURCES[kernel]:
        h.update(open(os.path.join(cdir, name), "rb").read())
    return h.hexdigest()[:16]


def load_counters(kernel: str, workload: str):
    """Figures from committed rocprofv3 counter runs of a kernel on a workload (HBM bytes
    per launch, FP32 FLOPs and VALU instructions per pair), if they were taken on the
    current kernel sources (else {})."""
    p = os.path.join(ROOT, "profiles", "counters.json")
    if not os.path.exists(p):
        return {}
    try:
        e = json.load(open(p))[kernel][workload]
        if e.get("source_hash") != source_hash(kernel):
            return {}
        return e
    except Exception:
        return {}


def roofline(kernel: str, workload: str, pairs: float, launch_s: float, flop_per_pair: int) -> dict:
    """The FP32-ALU roofline of one launch: algorithmic FLOPs (a fixed count per pair) over
    the measured launch time; with committed counters also the hardware fraction
    (counted FP32 FLOPs over the same time) and the HBM bytes per launch."""
    achieved = pairs * flop_per_pair / launch_s
    c = load_counters(kernel, workload)
    out = {"bound": "alu", "kernel": kernel, "achieved": achieved / 1e12, "peak": PEAK_FP32 / 1e12,
           "unit": "TFLOP/s", "frac": achieved / PEAK_FP32,
           "traffic": c.get("bytes_per_launch"), "flop_per_pair": flop_per_pair, "launch_ms": launch_s * 1e3}
    if c.get("hw_flop_per_pair"):
        out["hw_flop_per_pair"] = c["hw_flop_per_pair"]
        out["hw_frac"] = pairs * c["hw_flop_per_pair"] / launch_s / PEAK_FP32
    if c.get("valu_per_pair"):
        out["valu_per_pair"] = c["valu_per_pair"]
    return out


def time_steps(fn, steps, warmup, stream):
    import torch
    for _ in range(warmup):
        fn()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    ev0.record(stream)
    for _ in range(steps):
        fn()
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    return ev0.elapsed_time(ev1) / 1e3, wall


def bench_forward(steps, warmup, autotune=True, compare=True):
    """The plain forward on the 19 000-face non-watertight union at 128^3 (one mesh per
    launch) with the mesh's triangle-strip record stream (built on the host from F
    before timing, like the mesh itself); also the same step with the default three
    records per face."""
    import torch
    import paper_2407_11272_amd as wn
    import wn_inputs as wi
    c = wi.config2_ellipsoid_union()
    V, F = wn.as_mesh(torch.as_tensor(c.V), torch.as_tensor(c.F))
    t0 = time.perf_counter()
    Rh = wn.wn_build_strips(c.F, len(c.V))
    strip_ms = (time.perf_counter() - t0) * 1e3
    R = torch.as_tensor(Rh).cuda()
    grid = wn.Grid.of(c.grid)
    W = torch.empty(tuple(grid.n), dtype=torch.float32, device="cuda")
    occ = torch.empty(tuple(grid.n), dtype=torch.uint8, device="cuda")
    stream = torch.cuda.current_stream()
    tune = None
    if autotune:
        tune = wn.wn_autotune("voxelize", [wn.MeshJob(V, F, grid, "threshold", W=W, occ=occ, strips=R)])

    def step():
        wn.wn_voxelize_strips(V, F, R, grid=grid, W=W, occupancy="threshold", occ=occ)

    def step_plain():
        wn.wn_voxelize(V, F, grid=grid, W=W, occupancy="threshold", occ=occ)

    dev_s, _ = time_steps(step, steps, warmup, stream)
    pairs = grid.size * len(c.F)
    out = {
        "workload": c.name,
        "faces": int(len(c.F)),
        "points": int(grid.size),
        "pairs_per_launch": int(pairs),
        "ms": dev_s / steps * 1e3,
        "pairs_per_s": pairs * steps / dev_s,
        "strip_records_per_face": len(Rh) / len(c.F),
        "strip_build_ms_host": strip_ms,
        "autotune": tune["chosen"] if tune else None,
        "roofline": roofline("k_wn_fwd", "c2", pairs, dev_s / steps, FLOP_FWD),
    }
    if compare:
        n = max(2, steps // 2)
        plain_s, _ = time_steps(step_plain, n, 1, stream)
        out["three_records_per_face_pairs_per_s"] = pairs * n / plain_s
    return c, out


def bench_adjoint(steps, warmup):
    import torch
    import paper_2407_11272_amd as wn
    import wn_inputs as wi
    c = wi.config3_differentiable()
    V, F = wn.as_mesh(torch.as_tensor(c.V), torch.as_tensor(c.F))
    grid = wn.Grid.of(c.grid)
    T = torch.as_tensor(c.target).cuda()
    W = torch.empty(grid.size, dtype=torch.float32, device="cuda")
    loss = torch.empty(1, dtype=torch.float32, device="cuda")
    dLdW = torch.empty_like(W)
    dLdV = torch.empty_like(V)
    stream = torch.cuda.current_stream()

    def fwd():
        wn.wn_voxelize(V, F, grid=grid, W=W)

    pairs = torch.as_tensor(wn.wn_build_face_pairs(c.F, len(c.V))).cuda()

    def step():
        wn.wn_voxelize(V, F, grid=grid, W=W)
        wn.wn_sigmoid_mse(W, T, 0.5, 50.0, loss=loss, dLdW=dLdW)
        wn.wn_backward(V, F, dLdW, grid=grid, dLdV=dLdV, pairs=pairs)

    def adj():
        wn.wn_backward(V, F, dLdW, grid=grid, dLdV=dLdV, pairs=pairs)

    n = max(2, steps)
    f_s, _ = time_steps(fwd, n, 1, stream)
    s_s, _ = time_steps(step, n, max(1, warmup), stream)
    a_s, _ = time_steps(adj, n, 1, stream)
    npairs = grid.size * len(c.F)
    bwd_s = max(s_s - f_s, 1e-12) / n
    out = {
        "workload": "icosphere-s4-5120f-64cube sigmoid(k=50) MSE, forward+loss+adjoint (two faces per lane, sums shared per vertex)",
        "pairs_per_pass": npairs,
        "ms_per_step": s_s / n * 1e3,
        "fwd_ms": f_s / n * 1e3,
        "bwd_ms": bwd_s * 1e3,
        "adjoint_pairs_per_s": npairs / bwd_s,
        "adjoint_frac_fp32_peak": npairs / bwd_s * FLOP_BWD / PEAK_FP32,
        "step_pairs_per_s": 2 * npairs / (s_s / n),
        # the adjoint call alone (pack, the two-faces-per-lane kernel, split reduction, per-vertex gather)
        "adjoint_call_ms": a_s / n * 1e3,
        "adjoint_call_pairs_per_s": npairs / (a_s / n),
        "roofline": roofline("k_wn_bwd_pairs", "c3", npairs, a_s / n, FLOP_BWD),
    }
    return out


def batch_jobs():
    """The 64 meshes of the batched workload on the device, each with its strip order."""
    import torch
    import paper_2407_11272_amd as wn
    import wn_inputs as wi
    ws = wi.config4_batch()
    jobs = []
    for w in ws:
        V, F = wn.as_mesh(torch.as_tensor(w.V), torch.as_tensor(w.F))
        R = torch.as_tensor(wn.wn_build_strips(w.F, len(w.V))).cuda()
        jobs.append(wn.MeshJob(V, F, wn.Grid.of(w.grid), "threshold", strips=R).prepare())
    return ws, jobs


def bench_batched(steps: int, warmup: int, autotune: bool, compare: bool = True):
    """The headline: 64 meshes of uneven size in one persistent, graph-captured launch;
    beside it the same meshes launched one per call (the plain kernel, same strip order)."""
    import torch
    import paper_2407_11272_amd as wn
    ws, jobs = batch_jobs()
    pairs = sum(int(j.grid.size) * int(j.F.shape[0]) for j in jobs)
    report = wn.wn_autotune("batched", jobs) if autotune else None
    stream = torch.cuda.current_stream()
    b_s, wall_s = time_steps(lambda: wn.wn_voxelize_batched(jobs), steps, warmup, stream)
    out = {
        "workload": "ellipsoid-union-batch-64meshes-500-50000f-32-128cube",
        "meshes": len(jobs),
        "faces_total": int(sum(int(j.F.shape[0]) for j in jobs)),
        "points_total": int(sum(int(j.grid.size) for j in jobs)),
        "pairs_per_launch": int(pairs),
        "grids": {str(r): sum(1 for j in jobs if j.grid.n[0] == r) for r in (32, 64, 128)},
        "ms": b_s / steps * 1e3,
        "wall_ms": wall_s / steps * 1e3,
        "pairs_per_s": pairs * steps / b_s,
        "autotune": report["chosen"] if report else None,
        "autotune_identical": report["identical"] if report else None,
    }
    if compare:
        def plain():
            for j in jobs:
                wn.wn_voxelize_strips(j.V, j.F, j.strips, grid=j.grid, W=j.W, occupancy="threshold", occ=j.occ)

        p_s, _ = time_steps(plain, 2, 1, stream)
        out["plain_one_mesh_per_launch_ms"] = p_s / 2 * 1e3
        out["plain_pairs_per_s"] = pairs * 2 / p_s
        out["batched_over_plain"] = out["pairs_per_s"] / out["plain_pairs_per_s"]
    return ws, pairs, b_s, wall_s, out


def bench_served(n_requests: int, loads, fwd_pairs_per_s: float, adj_pairs_per_s: float, warmup_frac: float = 0.0,
                 policy: str = "edf", step_pairs: float | None = None, burst_requests: int | None = None):
    """Poisson trace through the continuous-batching server and through the plain FIFO
    one-mesh-per-launch loop, at each offered load in ``loads``; p50/p99 latency and
    throughput of both.  A load puts the offered GPU time at that fraction of the wall
    clock, with a request's GPU time estimated from the measured batched forward and
    adjoint pair rates.  The same requests (meshes, grids, targets) are replayed at every
    load; only their arrival times scale.  Statistics skip the first ``warmup_frac`` of
    the requests (by arrival) and are also given per grid resolution; ``slowdown`` is a
    request's latency over its own GPU time estimated from the same pair rates.  The
    server's policy is ``policy``; its adjoint cost per pair and deadline rate come from
    the same measured rates."""
    import numpy as np
    import torch
    import wn_inputs as wi
    from paper_2407_11272_amd.serve import (STEP_PAIRS, GpuExecutor, Server, ServeRequest, latency_stats,
                                            run_plain_fifo)
    step_pairs = STEP_PAIRS if step_pairs is None else float(step_pairs)
    base = wi.config5_trace(n_requests, 1.0)  # arrivals at rate 1; rate r divides them by r
    mean_pairs = float(np.mean([r.faces * r.res ** 3 * (2 if r.wants_grad else 1) for r in base]))
    mean_gpu_s = float(np.mean([r.faces * r.res ** 3 * (1.0 / fwd_pairs_per_s
                                                        + (1.0 / adj_pairs_per_s if r.wants_grad else 0.0))
                                for r in base]))
    built = [(r, r.build()) for r in base]
    total_pairs = sum(int(np.prod(w.grid.n)) * len(w.F) * (2 if r.wants_grad else 1) for r, w in built)
    res_of = {r.rid: r.res for r in base}
    alone_s = {r.rid: r.faces * r.res ** 3 * (1.0 / fwd_pairs_per_s + (1.0 / adj_pairs_per_s if r.wants_grad else 0.0))
               for r in base}
    skip = set(sorted(res_of, key=lambda i: base[i].arrival)[:int(warmup_frac * len(base))])
    sweep = []
    last = [time.perf_counter()]

    def progress(label):
        def tick(done, total):  # a line every 30 s, so that long low-load runs show progress
            now = time.perf_counter()
            if now - last[0] >= 30.0:
                last[0] = now
                print(f"# {label}: {done}/{total} requests submitted", file=sys.stderr, flush=True)
        return tick
    for load in loads:
        rate = load / mean_gpu_s
        reqs = [ServeRequest(r.rid, w.V.astype(np.float32), w.F.astype(np.int32), w.grid, r.arrival / rate,
                             w.occ_mode, w.target) for r, w in built]

        def summary(out):
            span = max(o.done for o in out) - min(o.arrival for o in out)
            kept = [o for o in out if o.rid not in skip]
            st = latency_stats(kept)
            st["throughput_pairs_per_s"] = total_pairs / span
            st["makespan_s"] = span
            st["by_resolution"] = {str(res): latency_stats([o for o in kept if res_of[o.rid] == res])
                                   for res in sorted(set(res_of.values()))}
            sd = np.array([o.latency / alone_s[o.rid] for o in kept if np.isfinite(o.done)])
            st["slowdown_p50"] = float(np.percentile(sd, 50)) if len(sd) else None
            st["slowdown_p99"] = float(np.percentile(sd, 99)) if len(sd) else None
            return st

        print(f"# served load {load}: continuous batching ({len(reqs)} requests)", file=sys.stderr, flush=True)

        srv = Server(GpuExecutor(), hbm_budget=int(torch.cuda.get_device_properties(0).total_memory * 0.5),
                     slots=16, quantum_pairs=step_pairs, policy=policy, adjoint_cost=fwd_pairs_per_s / adj_pairs_per_s,
                     rate_pairs=fwd_pairs_per_s)
        served = srv.run_trace(reqs, progress=progress(f"served load {load}"))
        s_stats = summary(served)
        s_stats["steps"] = srv.steps
        s_stats["peak_active"] = srv.peak_active
        del served
        torch.cuda.synchronize()
        print(f"# served load {load}: plain FIFO", file=sys.stderr, flush=True)
        p_stats = summary(run_plain_fifo(reqs, progress=progress(f"plain FIFO load {load}")))
        sweep.append({"load": load, "rate_req_per_s": rate, "served": s_stats, "plain_fifo": p_stats,
                      "p50_speedup": p_stats["p50_ms"] / s_stats["p50_ms"],
                      "p99_speedup": p_stats["p99_ms"] / s_stats["p99_ms"]})
        print(f"# served load {load}: p50 {s_stats['p50_ms']:.0f} / {p_stats['p50_ms']:.0f} ms, "
              f"p99 {s_stats['p99_ms']:.0f} / {p_stats['p99_ms']:.0f} ms (served / plain)", file=sys.stderr,
              flush=True)
    # saturation: every request (the first burst_requests of the trace) at t = 0, so the
    # makespan measures throughput alone
    bb = built[:burst_requests] if burst_requests else built
    reqs = [ServeRequest(r.rid, w.V.astype(np.float32), w.F.astype(np.int32), w.grid, 0.0, w.occ_mode, w.target)
            for r, w in bb]
    fwd_pairs = sum(int(np.prod(w.grid.n)) * len(w.F) for r, w in bb)
    adj_pairs = sum(int(np.prod(w.grid.n)) * len(w.F) for r, w in bb if r.wants_grad)
    flops = fwd_pairs * FLOP_FWD + adj_pairs * FLOP_BWD

    def burst(out):
        span = max(o.done for o in out)
        return {"makespan_s": span, "throughput_pairs_per_s": (fwd_pairs + adj_pairs) / span,
                "frac_fp32_peak": flops / span / PEAK_FP32}

    print("# served burst: continuous batching", file=sys.stderr, flush=True)
    srv = Server(GpuExecutor(), hbm_budget=int(torch.cuda.get_device_properties(0).total_memory * 0.5),
                 slots=16, quantum_pairs=step_pairs, policy=policy, adjoint_cost=fwd_pairs_per_s / adj_pairs_per_s,
                 rate_pairs=fwd_pairs_per_s)
    b_served = burst(srv.run_trace(reqs))
    torch.cuda.synchronize()
    print("# served burst: plain FIFO", file=sys.stderr, flush=True)
    b_plain = burst(run_plain_fifo(reqs))
    print(f"# served burst: {b_served['throughput_pairs_per_s']:.3g} / {b_plain['throughput_pairs_per_s']:.3g} "
          f"pairs/s (served / plain)", file=sys.stderr, flush=True)
    return {
        "burst": {"what": f"the first {len(bb)} requests at t = 0; pairs count forward and adjoint pairs, the "
                          f"fraction weights them by {FLOP_FWD} and {FLOP_BWD} FLOP",
                  "served": b_served, "plain_fifo": b_plain},
        "workload": f"{n_requests} Poisson requests, 1k-100k faces log-uniform, grids 64^3/128^3/256^3, "
                    f"30% with dL/dV (sigmoid-MSE), offered load swept, first {warmup_frac:.0%} not counted",
        "policy": policy,
        "step_pairs": step_pairs,
        "adjoint_cost": fwd_pairs_per_s / adj_pairs_per_s,
        "mean_pairs_per_request": mean_pairs,
        "mean_gpu_ms_per_request": mean_gpu_s * 1e3,
        "sweep": sweep,
    }


def bench_naive(reps: int, autotune: bool = True):
    """Eq. 4 naive flux sum: forward on the 19 000-face union at 128^3, adjoint on the
    5120-face icosphere at 64^3 (both with one centroid sample per face)."""
    import torch
    import paper_2407_11272_amd as wn
    import wn_inputs as wi
    stream = torch.cuda.current_stream()
    c2 = wi.config2_ellipsoid_union()
    V, F = wn.as_mesh(torch.as_tensor(c2.V), torch.as_tensor(c2.F))
    g2 = wn.Grid.of(c2.grid)
    W = torch.empty(tuple(g2.n), dtype=torch.float32, device="cuda")
    tune = wn.wn_autotune("naive", [wn.MeshJob(V, F, g2, "none", W=W)]) if autotune else None
    f_s, _ = time_steps(lambda: wn.wn_voxelize_naive(V, F, grid=g2, W=W), reps, 1, stream)
    pairs_f = g2.size * len(c2.F)
    c3 = wi.config3_differentiable()
    V3, F3 = wn.as_mesh(torch.as_tensor(c3.V), torch.as_tensor(c3.F))
    g3 = wn.Grid.of(c3.grid)
    g = torch.randn(g3.size, device="cuda", generator=torch.Generator("cuda").manual_seed(0))
    dV = torch.empty_like(V3)
    b_s, _ = time_steps(lambda: wn.wn_backward_naive(V3, F3, g, grid=g3, dLdV=dV), reps, 1, stream)
    pairs_b = g3.size * len(c3.F)
    return {
        "forward_workload": "ellipsoid-union-19000f-128cube, one centroid sample per face",
        "autotune": tune["chosen"] if tune else None,
        "forward_ms": f_s / reps * 1e3,
        "forward_pairs_per_s": pairs_f * reps / f_s,
        "adjoint_workload": "icosphere-s4-5120f-64cube, random dL/dW",
        "adjoint_ms": b_s / reps * 1e3,
        "adjoint_pairs_per_s": pairs_b * reps / b_s,
    }


def bench_flip(reps: int):
    """Algorithm 2 on the open 4864-face icosphere (5 % of faces removed), then the exact
    forward of the duplicated 9728-face mesh at 128^3 in strip order."""
    import torch
    import paper_2407_11272_amd as wn
    import wn_inputs as wi
    stream = torch.cuda.current_stream()
    c = wi.config3_differentiable(res=128, open_variant=True)
    V, F = wn.as_mesh(torch.as_tensor(c.V), torch.as_tensor(c.F))
    d_s, _ = time_steps(lambda: wn.wn_flip_duplicate(V, F, 0.01), reps, 1, stream)
    V2, F2 = wn.wn_flip_duplicate(V, F, 0.01)
    R = torch.as_tensor(wn.wn_build_strips(F2.cpu().numpy(), V2.shape[0])).cuda()
    grid = wn.Grid.of(c.grid)
    W = torch.empty(tuple(grid.n), dtype=torch.float32, device="cuda")
    v_s, _ = time_steps(lambda: wn.wn_voxelize_strips(V2, F2, R, grid=grid, W=W), reps, 1, stream)
    pairs = grid.size * F2.shape[0]
    return {
        "workload": "open icosphere s4 (4864 faces) -> flipped duplicate (9728 faces), 128^3",
        "flip_ms": d_s / reps * 1e3,
        "voxelize_ms": v_s / reps * 1e3,
        "voxelize_pairs_per_s": pairs * reps / v_s,
    }


def bench_morph(iters: int):
    """Mesh morphing (Section 2.4) on the 5120-face icosphere towards the ellipsoid target
    at 64^3: one wn_morph_step call enqueues ``iters`` iterations (forward, loss, adjoint,
    Adam), with the naive integral the paper morphs with and with the exact field."""
    import torch
    import paper_2407_11272_amd as wn
    import wn_inputs as wi
    stream = torch.cuda.current_stream()
    c = wi.config3_differentiable()
    out = {"workload": f"icosphere-s4-5120f -> ellipsoid target, 64^3, sigmoid(k=50) MSE, Adam lr 2e-3, "
                       f"{iters} iterations per call"}
    pairs = c.grid.size * len(c.F) * 2
    for integral in ("naive", "gwn"):
        mo = wn.Morpher(c.V, c.F, c.target.reshape(-1), c.grid, integral=integral, tau=c.tau, k=c.k, lr=2e-3)
        losses = []
        dt, _ = time_steps(lambda: losses.append(mo.run(iters)), 1, 1, stream)
        L = losses[-1].cpu().numpy()
        out[integral] = {"iter_ms": dt / iters * 1e3, "iters_per_s": iters / dt,
                         "pairs_per_s": pairs * iters / dt,
                         "loss_first": float(L[0]), "loss_last": float(L[-1])}
    return out


def bench_eval(reps: int, repeats: int = 3):
    """The evaluation chain of Section 3 on the 19 000-face union at 128^3: strip-order
    forward with threshold occupancy, cube surface, 10 smoothing steps (lambda 0.15, the
    enclosed volume kept), 20 000 samples of the result and of the mesh, Chamfer and
    Hausdorff; and marching cubes of W in place of the cube surface.  The metrics are
    the mean and standard deviation over ``repeats`` independent sample streams (the
    paper reports three repeats); stage times are means over ``reps`` passes."""
    import numpy as np
    import torch
    import paper_2407_11272_amd as wn
    import wn_inputs as wi
    c = wi.config2_ellipsoid_union()
    V, F = wn.as_mesh(torch.as_tensor(c.V), torch.as_tensor(c.F))
    R = torch.as_tensor(wn.wn_build_strips(c.F, len(c.V))).cuda()
    grid = wn.Grid.of(c.grid)
    stages = {}

    def timed(name, fn):
        ev0, ev1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        ev0.record()
        out = fn()
        ev1.record()
        torch.cuda.synchronize()
        stages.setdefault(name, []).append(ev0.elapsed_time(ev1))
        return out

    cube, march = [], []
    for it in range(max(reps, repeats) + 1):
        rep = max(0, it - 1) % repeats
        ua, ub = (torch.as_tensor(u).cuda() for u in wi.evaluation_samples(repeat=rep))
        W, occ = timed("voxelize", lambda: wn.wn_voxelize_strips(V, F, R, grid=grid, occupancy="threshold"))
        Vc, Fc = timed("cubify", lambda: wn.wn_cubify(occ, grid))
        Vs = timed("smooth", lambda: wn.wn_laplacian_smooth(Vc, Fc, 0.15, 10))
        Pa, _ = timed("sample", lambda: wn.wn_sample_surface(Vs, Fc, ua))
        Pb, _ = timed("sample_ref", lambda: wn.wn_sample_surface(V, F, ub))
        m = timed("metrics", lambda: wn.wn_chamfer_hausdorff(Pa, Pb))
        # the alternative mesher: marching cubes of W at 0.5 (two passes: counts, then
        # the mesh), then the same smoothing, samples and metrics
        Vm, Fm = timed("marching", lambda: wn.wn_marching_cubes(W, grid, 0.5))
        Vms = timed("smooth_marching", lambda: wn.wn_laplacian_smooth(Vm, Fm, 0.15, 10))
        Pm, _ = timed("sample_marching", lambda: wn.wn_sample_surface(Vms, Fm, ua))
        mm = timed("metrics_marching", lambda: wn.wn_chamfer_hausdorff(Pm, Pb))
        if 1 <= it <= repeats:   # the first pass is a warm-up
            cube.append(m.cpu().numpy())
            march.append(mm.cpu().numpy())
    ms = {k: sum(v[1:]) / (len(v) - 1) for k, v in stages.items()}
    cube, march = np.array(cube), np.array(march)
    stat = lambda a: {"mean": float(a.mean()), "std": float(a.std(ddof=1)) if len(a) > 1 else 0.0}  # noqa: E731
    cube_keys = ("voxelize", "cubify", "smooth", "sample", "sample_ref", "metrics")
    march_keys = ("voxelize", "marching", "smooth_marching", "sample_marching", "sample_ref", "metrics_marching")
    return {"workload": "ellipsoid-union-19000f-128cube: occupancy -> cube surface -> 10 x Laplacian(0.15, volume "
                        "kept) -> 2 x 20000 samples -> Chamfer/Hausdorff; and marching cubes of W in place of the "
                        "cube surface",
            "repeats": repeats, "stage_ms": ms, "total_ms": sum(ms[k] for k in cube_keys),
            "cube_faces": int(Fc.shape[0]), "chamfer": stat(cube[:, 0]), "hausdorff": stat(cube[:, 1]),
            "marching_faces": int(Fm.shape[0]), "marching_total_ms": sum(ms[k] for k in march_keys),
            "chamfer_marching": stat(march[:, 0]), "hausdorff_marching": stat(march[:, 1])}


def copy_calibration(nbytes: int = 1 << 30, reps: int = 3):
    """A streaming kernel of known size (torch's elementwise negation: reads nbytes,
    writes nbytes): its FETCH_SIZE and WRITE_SIZE counter readings calibrate the
    counters' units for the traffic field."""
    import torch
    src = torch.ones(nbytes // 4, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(reps):
        torch.neg(src, out=dst)
    torch.cuda.synchronize()
    return {"copy_bytes_read": nbytes, "copy_bytes_written": nbytes, "reps": reps}


def _cpu_model():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(batch, budget_s: float = 15.0):
    """The FP64 oracle (as it stands) on a bounded, deterministic subsample of the
    headline batch: the same number of seeded voxels of every mesh (pairs counted with
    each mesh's own face count), sized to about ``budget_s`` on all host threads; then a
    smaller sample on one thread, and the other workloads' rates for context (the small
    plain forward and the differentiable mesh in full, the 128^3 union on a stride)."""
    import numpy as np
    import oracle
    import wn_inputs as wi
    threads = oracle.max_threads()

    def run(per_mesh, nthreads):
        rng = np.random.default_rng(17)
        pairs, t = 0, 0.0
        for w in batch:
            Q = oracle.grid_points(w.grid)
            idx = np.sort(rng.choice(len(Q), min(per_mesh, len(Q)), replace=False))
            t0 = time.perf_counter()
            oracle.winding(w.V, w.F, Q[idx], threads=nthreads)
            t += time.perf_counter() - t0
            pairs += len(idx) * len(w.F)
        return pairs, t

    # calibrate on a small sample, then size the sample to the time budget
    p0, t0 = run(64, threads)
    per_mesh = int(max(256, min(65536, 64 * budget_s / max(t0, 1e-3))))
    pairs, dt = run(per_mesh, threads)
    p1, t1 = run(max(32, per_mesh // (4 * max(1, threads))), 1)
    # (the thread count is passed explicitly: the one-thread run set the runtime's default)
    context = {}
    c1 = wi.config1_icosphere()
    tt = time.perf_counter()
    oracle.winding(c1.V, c1.F, oracle.grid_points(c1.grid), threads=threads)
    context["plain_32cube_full"] = c1.pairs / (time.perf_counter() - tt)
    c3 = wi.config3_differentiable()
    tt = time.perf_counter()
    oracle.winding(c3.V, c3.F, oracle.grid_points(c3.grid), threads=threads)
    context["differentiable_64cube_full"] = c3.pairs / (time.perf_counter() - tt)
    c2 = wi.config2_ellipsoid_union()
    Q2 = oracle.grid_points(c2.grid)[::64]
    tt = time.perf_counter()
    oracle.winding(c2.V, c2.F, Q2, threads=threads)
    context["union_128cube_every_64th_voxel"] = len(Q2) * len(c2.F) / (time.perf_counter() - tt)
    return {
        "value": pairs / dt,
        "unit": UNIT,
        "cores": threads,
        "kind": "oracle",
        "sample": f"{per_mesh} seeded voxels of each of the {len(batch)} meshes of the batch ({pairs:.3g} pairs, "
                  f"{dt:.1f} s, FP64, {_cpu_model()})",
        "value_1thread": p1 / t1,
        "sample_1thread": f"{max(32, per_mesh // (4 * max(1, threads)))} voxels per mesh, {t1:.1f} s on one thread",
        "other_workloads_pairs_per_s": context,
    }


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=10)
    ap.add_argument("--warmup", type=int, default=2)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-rows", action="store_true", help="headline step only")
    ap.add_argument("--cpu-budget", type=float, default=15.0)
    ap.add_argument("--no-autotune", action="store_true")
    ap.add_argument("--served-requests", type=int, default=150)
    ap.add_argument("--rows", default="forward,adjoint,served,naive,flip,morph,eval",
                    help="comma list of extra rows (forward, adjoint, served, naive, flip, morph, eval)")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="run a 1 GiB device copy first (counter calibration for profiling runs)")
    ap.add_argument("--served-loads", default="0.5,0.8,0.95",
                    help="comma list of offered loads (fractions of the GPU's measured capacity)")
    ap.add_argument("--served-policy", default="edf", choices=("edf", "fair", "age"),
                    help="scheduler policy of the served row (earliest deadline first, or shares)")
    ap.add_argument("--served-step-pairs", type=float, default=None,
                    help="pairs of work per scheduler step (default: the server's)")
    ap.add_argument("--served-warmup", type=float, default=0.2,
                    help="fraction of the served requests (earliest arrivals) left out of the statistics")
    ap.add_argument("--served-burst-requests", type=int, default=64,
                    help="requests of the saturated (all at t = 0) served run")
    ap.add_argument("--no-compare", action="store_true",
                    help="skip the one-mesh-per-launch and three-records-per-face comparison launches")
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py: runs on one GPU; --gpus {args.gpus} is not supported (the path would shard by voxel "
              "slabs, each GPU writing its own slab of W, with no collective)", file=sys.stderr)
        sys.exit(2)

    import torch
    if not torch.cuda.is_available():
        print("bench.py: no GPU visible", file=sys.stderr)
        sys.exit(1)
    import paper_2407_11272_amd as wn
    wn.wn_version()
    calib = copy_calibration() if args.copy_calibration else None
    print(f"# bench: batched headline, {args.steps} steps after {args.warmup} warm-up", file=sys.stderr, flush=True)
    batch, pairs, dev_s, wall_s, head = bench_batched(args.steps, args.warmup, not args.no_autotune,
                                                      not args.no_compare)
    launch_s = dev_s / args.steps
    out = {
        "metric": METRIC,
        "value": pairs * args.steps / dev_s,
        "unit": UNIT,
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": launch_s * 1e3,
        "wall_ms_per_step": wall_s / args.steps * 1e3,
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f32",
        "data": "synthetic",
        "config": {
            **head,
            "occupancy": "threshold 0.5",
            "face_order": "triangle strips (host-built from F, resident in HBM)",
            "launch": "one persistent, graph-captured launch for all meshes",
        },
        "paper_context": {
            "kind": "context, not a target: other hardware and precision",
            "hardware": "one NVIDIA RTX A6000, FP16, 2000-point batches (Section 3.1)",
            "pairs_per_s_at_128": [1.25e9, 1.78e9],
            "derived_as": "res^3 x faces / time of the paper's own method at 128^3 (appendix table), "
                          "over its meshes",
        },
        "roofline": roofline("k_batched_persistent", "c4", pairs, launch_s, FLOP_FWD),
    }
    want = set() if args.no_rows else {r.strip() for r in args.rows.split(",") if r.strip()}
    rows = {}
    if "forward" in want:
        print("# bench: forward row (one mesh per launch)", file=sys.stderr, flush=True)
        _, rows["forward_c2"] = bench_forward(max(2, args.steps // 2), 1, not args.no_autotune, not args.no_compare)
    if "adjoint" in want or "served" in want:
        print("# bench: adjoint row", file=sys.stderr, flush=True)
        rows["adjoint"] = bench_adjoint(max(2, args.steps // 2), 1)
    if "served" in want and args.served_requests > 0:
        print("# bench: served row", file=sys.stderr, flush=True)
        rows["served"] = bench_served(args.served_requests, [float(x) for x in args.served_loads.split(",")],
                                      head["pairs_per_s"], rows["adjoint"]["adjoint_call_pairs_per_s"], args.served_warmup,
                                      args.served_policy, args.served_step_pairs, args.served_burst_requests)
    if "naive" in want:
        print("# bench: naive row", file=sys.stderr, flush=True)
        rows["naive"] = bench_naive(3, not args.no_autotune)
    if "eval" in want:
        print("# bench: evaluation-chain row", file=sys.stderr, flush=True)
        rows["eval"] = bench_eval(3)
    if "morph" in want:
        print("# bench: morph row", file=sys.stderr, flush=True)
        rows["morph"] = bench_morph(20)
    if "flip" in want:
        print("# bench: flip row", file=sys.stderr, flush=True)
        rows["flip"] = bench_flip(3)
    if rows:
        out["rows"] = rows
    if calib:
        out["copy_calibration"] = calib
    if not args.no_cpu_baseline:
        print("# bench: cpu baseline (oracle)", file=sys.stderr, flush=True)
        out["cpu_baseline"] = cpu_baseline(batch, args.cpu_budget)
    out["summary"] = summary(out)
    print(json.dumps(out), flush=True)


def summary(out) -> dict:
    """The line's key figures in a few hundred bytes (its last field)."""
    r = out.get("rows", {})
    s = {"batched_c4": {"pairs_per_s": out["value"], "frac": round(out["roofline"]["frac"], 4),
                        "ms": round(out["ms_per_step"], 2),
                        "over_plain": round(out["config"].get("batched_over_plain", 0.0), 4)}}
    if "hw_frac" in out["roofline"]:
        s["batched_c4"]["hw_frac"] = round(out["roofline"]["hw_frac"], 4)
    if "forward_c2" in r:
        f = r["forward_c2"]
        s["forward_c2"] = {"pairs_per_s": f["pairs_per_s"], "frac": round(f["roofline"]["frac"], 4),
                           "ms": round(f["ms"], 3)}
        if "hw_frac" in f["roofline"]:
            s["forward_c2"]["hw_frac"] = round(f["roofline"]["hw_frac"], 4)
    if "adjoint" in r:
        a = r["adjoint"]
        # the adjoint call timed on its own (pack, kernel, split sums, vertex gather); the
        # step difference (step minus a separately timed forward) is kept beside it
        s["adjoint_c3"] = {"pairs_per_s": a["adjoint_call_pairs_per_s"],
                           "frac": round(a["roofline"]["frac"], 4), "ms": round(a["adjoint_call_ms"], 3),
                           "step_diff_frac": round(a["adjoint_frac_fp32_peak"], 4)}
        if "hw_frac" in a["roofline"]:
            s["adjoint_c3"]["hw_frac"] = round(a["roofline"]["hw_frac"], 4)
    if "served" in r:
        s["served_c5"] = [{"load": x["load"], "p50_ms": [round(x["served"]["p50_ms"]), round(x["plain_fifo"]["p50_ms"])],
                           "p99_ms": [round(x["served"]["p99_ms"]), round(x["plain_fifo"]["p99_ms"])]}
                          for x in r["served"]["sweep"]]
        b = r["served"]["burst"]
        s["served_c5_burst_frac"] = [round(b["served"]["frac_fp32_peak"], 4), round(b["plain_fifo"]["frac_fp32_peak"], 4)]
    if "cpu_baseline" in out:
        s["cpu_oracle"] = {"pairs_per_s": out["cpu_baseline"]["value"], "threads": out["cpu_baseline"]["cores"],
                           "pairs_per_s_1thread": out["cpu_baseline"]["value_1thread"]}
    return s


if __name__ == "__main__":
    main()
