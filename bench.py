#!/usr/bin/env python3
"""Throughput of the J-CoMM outer iteration on one MI355X.

Workload: dense 256 x 256 x 256 float32 Poisson counts around a planted rank-32
CP model with Gamma(1,1) factors (seed 0), beta = 1 (KL), L = 5 inner sweeps,
the float64 objective at the reference recorded every outer iteration.  One
step = one J-CoMM outer iteration through the C ABI (reference pass that
rebuilds Xhat, forms P~ and contracts it onto all three modes, then the inner
sweeps and the factor update).  Inputs are resident in HBM before the timed
region; the factors evolve across steps exactly as in a 200-iteration run.

Prints ONE JSON line: outer iterations/s, the roofline of the dominant kernel
(the fused pass, timed with HIP events inside the library on the launch
stream), and the FP64 oracle timed on the host cores on a bounded sample.

  python bench.py [--gpus 1] [--steps 200] [--warmup 5]
  python bench.py --workload tucker [--beta 0|1.5]   # 200^3 Tucker, 16^3 core, J-CoMM L = 1
  python bench.py --workload coo                     # 3.3M-nonzero 4-way COO counts, beta = 1
  python bench.py --workload serving                 # Poisson stream of mixed requests, solves/s, p50/p99
  python bench.py --workload cp4 [--beta B]          # order-4 CP 80x70x60x50, R = 10 (the paper's synthetic shape)
  python bench.py --workload tucker4 [--beta B]      # order-4 Tucker 80x70x60x50, core 10x9x8x7
  python bench.py --workload tucker5 [--beta B]      # order-5 Tucker 27x24x7x100x100, core 10x10x5x10x10
  python bench.py --workload coo_beta [--beta B]     # the sparse counts at beta != 1 (default 1/2)
  python bench.py --workload tucker5_coo [--beta B]  # sparse 27x24x7x100x100 counts, Tucker (10,10,5,10,10)
  python bench.py --calibrate-copy   # plain device copy of known size, for counter scaling
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

METRIC = "J-CoMM outer iters/s (CP 256³ R32 β=1) + %roofline; batched solves/s, p99 ms"
PEAK_FP32_MFMA_TFLOPS = 157.3
PEAK_HBM_GBS = 8000.0
# the pass-kernel launches that carry timing events: every 7th, from the
# first (a prime, so that every launch of a step's fixed launch pattern is
# sampled alike); a timed dispatch costs the stream a few microseconds
PROFILE_EVERY = 7
TRAFFIC_FILE = os.path.join(ROOT, "profiles", "cp3_pass_kl_256_r32_traffic.json")
# sources that define the timed pass kernel; the stored counter figures are
# trusted only while these files are unchanged
KERNEL_SRCS = [os.path.join(ROOT, "paper_2602_14683_amd", "csrc", f)
               for f in ("cp3_impl.h", "cp3_bc_kl.hip", "dmath.h", "kernels.h")]


def kernel_source_hash() -> str:
    h = hashlib.sha256()
    for path in KERNEL_SRCS:
        with open(path, "rb") as f:
            h.update(f.read())
    return h.hexdigest()[:16]


def measured_traffic():
    """HBM bytes per launch of the fused pass from the committed counter runs,
    or None when absent or taken on a different kernel source."""
    try:
        with open(TRAFFIC_FILE) as f:
            t = json.load(f)
    except (OSError, ValueError):
        return None
    if t.get("kernel_source_sha") != kernel_source_hash():
        return None
    return t.get("hbm_bytes_per_launch")


def cpu_baseline(X64, init, beta, L, iters):
    """The FP64 oracle, as it stands, on the same tensor: `iters` outer
    iterations with the BLAS threads the host gives it, and a shorter run
    limited to one thread (the paper's own single-thread setting)."""
    from oracle import cp as ocp
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        threadpool_limits = None
        threads = os.cpu_count() or 1

    def run(n):
        cur = [a.copy() for a in init]
        t0 = time.perf_counter()
        for _ in range(n):
            cur, _ = ocp.jcomm_outer(X64, cur, beta, L=L, return_ref_obj=True)
        return time.perf_counter() - t0

    dt = run(iters)
    out = {"value": iters / dt, "unit": "outer it/s", "cores": int(threads), "kind": "oracle",
           "sample": f"{iters} J-CoMM outer iterations (L={L}, beta={beta}, objective included) on the full "
                     f"256x256x256 rank-32 tensor, NumPy float64 einsum, {dt:.1f} s"}
    if threadpool_limits is not None:
        n1 = max(1, iters // 5)
        with threadpool_limits(limits=1):
            d1 = run(n1)
        out["one_thread"] = {"value": n1 / d1, "unit": "outer it/s", "cores": 1,
                             "sample": f"{n1} outer iterations, {d1:.1f} s"}
    return out


def objective_off_rate(ctx, X, init32, steps):
    """The headline iteration with the objective switched off (pure update
    throughput), float32 tiles."""
    import torch
    fac = [torch.from_numpy(a).cuda() for a in init32]
    for _ in range(3):
        ctx.jcomm_outer(X, fac, beta=1.0, L=5)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.jcomm_outer(X, fac, beta=1.0, L=5)
    torch.cuda.synchronize()
    return round(steps / (time.perf_counter() - t0), 2)


def control_512(ctx, steps):
    """The same pass on 512^3 (537 MB of X, beyond the 256 MB last-level
    cache): pass-kernel time from the library's HIP events and the HBM rate
    it implies for X."""
    import numpy as np
    import torch
    import workloads
    d = workloads.cp_dense(0, dims=(512, 512, 512), rank=32)
    X = torch.from_numpy(d.X.astype(np.float32)).cuda()
    fac = [torch.from_numpy(a.astype(np.float32)).cuda() for a in d.init]
    del d
    obj = torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(2):
        ctx.jcomm_outer(X, fac, beta=1.0, L=5, obj_out=obj)
    torch.cuda.synchronize()
    ctx.profile_enable(PROFILE_EVERY)
    t0 = time.perf_counter()
    for _ in range(steps):
        ctx.jcomm_outer(X, fac, beta=1.0, L=5, obj_out=obj)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms, n = ctx.profile_query()
    ctx.profile_enable(False)
    entries = 512 ** 3
    avg = ms / max(n, 1)
    return {"outer_it_s": round(steps / wall, 2), "pass_avg_us": round(avg * 1e3, 2),
            "x_gbs": round(4 * entries / (avg * 1e-3) / 1e9, 1),
            "tflops": round(6.0 * 32 * entries / (avg * 1e-3) / 1e12, 2), "steps": steps}


def comparisons(ctx, X, init32, steps):
    """Config-2 companions on the same tensor and GPU: J-CoMM at beta = 0.5 (P~/Q~
    recomputed, and with the autotune table's choice) and
    the plain block-MM (B-CoMM) sweep at beta = 1 and 0.5, each from the same
    initial factors, in iterations per second (wall clock around `steps`)."""
    import torch

    def rate(fn):
        for _ in range(3):
            fn()
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for _ in range(steps):
            fn()
        torch.cuda.synchronize()
        return round(steps / (time.perf_counter() - t0), 2)

    res = {}
    obj = torch.zeros(1, dtype=torch.float64, device="cuda")
    for beta in (0.5,):
        fac = [torch.from_numpy(a).cuda() for a in init32]
        res[f"jcomm_beta{beta}_L5_obj_it_s"] = rate(
            lambda: ctx.jcomm_outer(X, fac, beta=beta, L=5, obj_out=obj))
        # the autotune table's choice between streaming the cached P~/Q~ and
        # recomputing them, then the rate with that choice
        fac = [torch.from_numpy(a).cuda() for a in init32]
        tuned = ctx.tune_jcomm(X, fac, beta=beta, L=5, reps=3)
        res[f"jcomm_beta{beta}_L5_tune"] = {k: (round(v, 4) if isinstance(v, float) else v)
                                            for k, v in tuned.items()}
        res[f"jcomm_beta{beta}_L5_obj_auto_it_s"] = rate(
            lambda: ctx.jcomm_outer(X, fac, beta=beta, L=5, obj_out=obj, cache_pq="auto"))
    # beta = 0.5 with bf16 tiles: P~/Q~ recomputed, and cached (as bf16)
    for cache in (False, True):
        fac = [torch.from_numpy(a).cuda() for a in init32]
        res[f"jcomm_beta0.5_L5_obj_bf16_{'cache' if cache else 'recompute'}_it_s"] = rate(
            lambda: ctx.jcomm_outer(X, fac, beta=0.5, L=5, obj_out=obj, cache_pq=cache, precision="bf16"))
    # the headline iteration with bf16 matrix-core tiles, and its objective
    # against the float32 path after the same number of iterations
    fac = [torch.from_numpy(a).cuda() for a in init32]
    res["jcomm_beta1_L5_obj_bf16_it_s"] = rate(lambda: ctx.jcomm_outer(X, fac, beta=1.0, L=5, obj_out=obj,
                                                                       precision="bf16"))
    # the bf16 pass time (HIP events on the launch stream) against its HBM
    # floor: X read once, 4 |X| = 67.1 MB at 8 TB/s = 8.39 us
    _, kms, nl, _ = timed_loop(ctx, lambda t: ctx.jcomm_outer(X, fac, beta=1.0, L=5, obj_out=obj, precision="bf16"),
                            2, steps)
    bf_us = kms / max(nl, 1) * 1e3
    floor_us = 4 * 256 ** 3 / (PEAK_HBM_GBS * 1e9) * 1e6
    res["jcomm_beta1_L5_bf16_pass"] = {"pass_avg_us": round(bf_us, 2), "hbm_floor_us": round(floor_us, 2),
                                       "frac_of_hbm_floor": round(floor_us / bf_us, 4),
                                       "hbm_gbs_algorithmic": round(4 * 256 ** 3 / (bf_us * 1e-6) / 1e9, 1)}
    fb = [torch.from_numpy(a).cuda() for a in init32]
    ff = [torch.from_numpy(a).cuda() for a in init32]
    for _ in range(50):
        ctx.jcomm_outer(X, fb, beta=1.0, L=5, precision="bf16")
        ctx.jcomm_outer(X, ff, beta=1.0, L=5)
    ob = ctx.beta_objective(X, fb, beta=1.0).item()
    of = ctx.beta_objective(X, ff, beta=1.0).item()
    res["bf16_objective_rel_diff_after_50_it"] = abs(ob - of) / of
    for beta in (1.0, 0.5):
        fac = [torch.from_numpy(a).cuda() for a in init32]
        res[f"bcomm_beta{beta}_sweep_it_s"] = rate(lambda: ctx.cp_update(X, fac, block=-1, beta=beta))
    res["note"] = ("B-CoMM sweeps rebuild Xhat before each of the 3 blocks and compute no objective; "
                   f"{steps} timed iterations each; bf16 = contraction tiles in bf16, reconstruction in "
                   "split bf16, objective compared with the float32 run after 50 outer iterations")
    return res


def calibrate_copy():
    import torch
    n = 64 * 1024 * 1024  # 256 MiB of float32
    src = torch.ones(n, dtype=torch.float32, device="cuda")
    dst = torch.empty_like(src)
    for _ in range(3):
        dst.copy_(src)
    torch.cuda.synchronize()
    print(json.dumps({"copy_bytes_read": n * 4, "copy_bytes_written": n * 4, "launches": 3}))


def graph_replay(ctx, X, init32, steps):
    """The headline iteration (beta = 1, L = 5, objective on) captured once into a
    HIP graph (torch.cuda.graph around the library call on the capture stream)
    and replayed: the same kernels without per-call launch gaps.  The captured
    call writes its objective to one fixed slot."""
    import torch
    fac = [torch.from_numpy(a).cuda() for a in init32]
    obj = torch.zeros(1, dtype=torch.float64, device="cuda")
    for _ in range(3):  # grows the workspace before the capture
        ctx.jcomm_outer(X, fac, beta=1.0, L=5, obj_out=obj)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        ctx.jcomm_outer(X, fac, beta=1.0, L=5, obj_out=obj)
    for _ in range(3):
        g.replay()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(steps):
        g.replay()
    torch.cuda.synchronize()
    el = time.perf_counter() - t0
    return {"outer_it_s": round(steps / el, 2), "steps": steps, "ms_per_step": round(el / steps * 1e3, 4)}


def rank16(ctx, steps):
    """256^3 at rank 16 (beta = 1, L = 5, objective on): the 16-wide pass tiles
    (the default at rank <= 16) against the 32-wide ones (an autotune table
    entry on a context of its own), J-CoMM rate and pass time each."""
    import numpy as np
    import torch
    import paper_2602_14683_amd as comm
    import workloads

    R = 16
    d = workloads.cp_dense(0, dims=(256, 256, 256), rank=R)
    X = torch.from_numpy(d.X.astype(np.float32)).cuda()
    init = [torch.from_numpy(a.astype(np.float32)).cuda() for a in d.init]
    flops = 6.0 * R * 256 ** 3
    out = {"workload": "jcomm_cp_dense_256x256x256_r16_beta1_L5_obj"}
    for tile in (0, 32):
        c = comm.Context(0)
        try:
            fac = [a.clone() for a in init]
            if tile:
                c.tune_set(X, fac, beta=1.0, L=5, cp_tile=tile)
            trace = torch.zeros(steps + 4, dtype=torch.float64, device="cuda")

            def step(t):
                c.jcomm_outer(X, fac, beta=1.0, L=5, obj_out=trace[t:t + 1])

            elapsed, kernel_ms, launches, seen = timed_loop(c, step, 3, steps)
            avg_us = kernel_ms / max(launches, 1) * 1e3
            tfl = flops / (avg_us * 1e-6) / 1e12
            out["tiles_16" if tile == 0 else "tiles_32"] = {
                "outer_it_s": round(steps / elapsed, 2), "pass_avg_us": round(avg_us, 2),
                "algorithmic_tflops": round(tfl, 2), "frac_fp32_mfma_peak": round(tfl / PEAK_FP32_MFMA_TFLOPS, 4)}
        finally:
            c.close()
    return out


def timed_loop(ctx, step, warmup, steps):
    """Warm up, then time `steps` calls of step(t) between synchronisations;
    meanwhile every PROFILE_EVERY-th pass-kernel launch on the launch stream
    carries HIP events that its dispatch stamps with the kernel's start and
    end.  Returns (elapsed s, summed ms of the timed launches, timed launches,
    all pass launches)."""
    import torch
    stream = torch.cuda.current_stream()
    for t in range(warmup):
        step(t)
    torch.cuda.synchronize()
    ctx.profile_enable(PROFILE_EVERY)
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    ev0.record(stream)
    for t in range(steps):
        step(warmup + t)
    ev1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    kernel_ms, launches, seen = ctx.profile_query_all()
    ctx.profile_enable(False)
    return max(wall, ev0.elapsed_time(ev1) / 1e3), kernel_ms, launches, seen


def monotone(tr):
    import numpy as np
    return bool(np.all(np.diff(tr) <= np.abs(tr[:-1]) * 1e-6))


def base_line(args, elapsed, unit="outer it/s"):
    return {"metric": METRIC, "value": round(args.steps / elapsed, 2), "unit": unit,
            "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
            "ms_per_step": round(elapsed / args.steps * 1e3, 4), "higher_is_better": True,
            "scaling": "weak", "vs_baseline": None, "dtype": "fp32"}


def run_cp(args, ctx):
    import numpy as np
    import torch
    import workloads

    beta, L, R = 1.0, 5, 32
    d = workloads.cp_dense(0, dims=(256, 256, 256), rank=R)
    X32 = d.X.astype(np.float32)
    init32 = [a.astype(np.float32) for a in d.init]
    X = torch.from_numpy(X32).cuda()
    fac = [torch.from_numpy(a).cuda() for a in init32]
    trace = torch.zeros(args.warmup + args.steps + 1, dtype=torch.float64, device="cuda")

    def step(t):
        ctx.jcomm_outer(X, fac, beta=beta, L=L, obj_out=trace[t:t + 1])

    elapsed, kernel_ms, launches, seen = timed_loop(ctx, step, args.warmup, args.steps)
    tr = trace.cpu().numpy()
    steps_tr = tr[args.warmup:args.warmup + args.steps]

    entries = 256 ** 3
    avg_ms = kernel_ms / max(launches, 1)
    flops = 6.0 * R * entries           # rebuild 2R + mode-3 2R + shared modes-1/2 2R per entry
    achieved_tflops = flops / (avg_ms * 1e-3) / 1e12
    roofline = {"bound": "mfma", "achieved": round(achieved_tflops, 2), "peak": PEAK_FP32_MFMA_TFLOPS,
                "unit": "TFLOP/s", "frac": round(achieved_tflops / PEAK_FP32_MFMA_TFLOPS, 4),
                "traffic": measured_traffic(),
                "kernel": "cp3_pass_kernel<KL> (fused rebuild + P~ + 3 numerators + FP64 objective)",
                "kernel_avg_us": round(avg_ms * 1e3, 2), "launches": seen, "launches_timed": launches,
                "algorithmic_flops_per_launch": flops, "algorithmic_bytes_per_launch": 4 * entries,
                "hbm_gbs_algorithmic": round(4 * entries / (avg_ms * 1e-3) / 1e9, 1)}
    out = base_line(args, elapsed)
    out.update({"data": "synthetic (seeded Poisson around a planted Gamma(1,1) rank-32 CP model)",
                "config": {"workload": "jcomm_cp_dense_256x256x256_r32_beta1_L5_obj", "dims": [256, 256, 256],
                           "rank": R, "beta": beta, "inner_sweeps": L, "objective_every_iteration": True,
                           "parallelism": "single GPU"},
                "roofline": roofline,
                "objective": {"first": float(tr[0]), "last": float(steps_tr[-1]), "monotone": monotone(steps_tr)}})
    if not args.no_comparisons:
        out["same_gpu_comparisons"] = comparisons(ctx, X, init32, args.comparison_steps)
        out["same_gpu_comparisons"]["jcomm_beta1_L5_no_objective_it_s"] = objective_off_rate(
            ctx, X, init32, args.comparison_steps)
        out["control_512"] = control_512(ctx, 20)
        out["rank16"] = rank16(ctx, args.comparison_steps)
        out["graph_replay"] = graph_replay(ctx, X, init32, args.comparison_steps)
    if not args.no_cpu_baseline:
        X64 = X32.astype(np.float64)
        init64 = [a.astype(np.float64) for a in init32]
        out["cpu_baseline"] = cpu_baseline(X64, init64, beta, L, args.cpu_iters)
    return out


def run_tucker(args, ctx):
    """Dense 200^3 Tucker, 16^3 core, J-CoMM L = 1 with the objective."""
    import numpy as np
    import torch
    import workloads

    beta = args.beta if args.beta is not None else 0.0
    d = workloads.tucker_dense(0)
    X = torch.from_numpy(d.X.astype(np.float32)).cuda()
    G = torch.from_numpy(d.init_core.astype(np.float32)).cuda()
    F = [torch.from_numpy(a.astype(np.float32)).cuda() for a in d.init_factors]
    G0, F0 = G.clone(), [a.clone() for a in F]
    trace = torch.zeros(args.warmup + args.steps + 1, dtype=torch.float64, device="cuda")

    def step(t):
        ctx.jcomm_outer(X, F, core=G, beta=beta, L=1, obj_out=trace[t:t + 1])

    elapsed, kernel_ms, launches, seen = timed_loop(ctx, step, args.warmup, args.steps)
    tr = trace.cpu().numpy()[args.warmup:args.warmup + args.steps]
    entries = 200 ** 3
    J = 16
    avg_ms = kernel_ms / max(launches, 1)
    bytes_ = 4 * entries                 # X streamed once per pass
    chains = 2 if beta == 1.0 else 3     # rebuild + numerator (+ denominator) per entry
    flops = 2.0 * J * chains * entries
    gbs = bytes_ / (avg_ms * 1e-3) / 1e9
    out = base_line(args, elapsed)
    out.update({"data": "synthetic (Gamma(shape 10) around a planted 16^3-core Tucker model)",
                "config": {"workload": f"jcomm_tucker_dense_200x200x200_core16_beta{beta}_L1_obj",
                           "dims": [200, 200, 200], "core": [16, 16, 16], "beta": beta, "inner_sweeps": 1,
                           "parallelism": "single GPU"},
                "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                             "frac": round(gbs / PEAK_HBM_GBS, 4), "traffic": None,
                             "kernel": "tk_v_kernel / tk_m3_kernel (fused rebuild + P~, Q~ + numerator and denominator contractions)",
                             "kernel_avg_us": round(avg_ms * 1e3, 2), "launches": seen, "launches_timed": launches,
                             "passes_per_outer_iteration": round(seen / max(args.steps, 1), 3),
                             "algorithmic_bytes_per_launch": bytes_, "algorithmic_flops_per_launch": flops,
                             "tflops_algorithmic": round(flops / (avg_ms * 1e-3) / 1e12, 2)},
                "objective": {"first": float(tr[0]), "last": float(tr[-1]), "monotone": monotone(tr)}})
    # the same iteration with bf16 tiles, and its objective against the
    # float32 path after the same number of iterations
    Gb, Fb = G0.clone(), [a.clone() for a in F0]
    Gf, Ff = G0.clone(), [a.clone() for a in F0]

    def bf16_step(t):
        ctx.jcomm_outer(X, Fb, core=Gb, beta=beta, L=1, obj_out=trace[t:t + 1], precision="bf16")

    el_b, _, _, _ = timed_loop(ctx, bf16_step, 2, args.steps)
    Gb.copy_(G0)
    for a, b in zip(Fb, F0):
        a.copy_(b)
    for _ in range(30):
        ctx.jcomm_outer(X, Fb, core=Gb, beta=beta, L=1, precision="bf16")
        ctx.jcomm_outer(X, Ff, core=Gf, beta=beta, L=1)
    ob = ctx.beta_objective(X, Fb, core=Gb, beta=beta).item()
    of = ctx.beta_objective(X, Ff, core=Gf, beta=beta).item()
    out["bf16"] = {"outer_it_s": round(args.steps / el_b, 2), "objective_rel_diff_vs_fp32_after_30_it": abs(ob - of) / of}
    # the autotune table's choice (P~/Q~ cache, mode-3 pair groups) for this
    # problem, then the same iteration with it
    entry = ctx.tune_jcomm(X, [a.clone() for a in F0], core=G0.clone(), beta=beta, L=1, reps=5)
    Gt, Ft = G0.clone(), [a.clone() for a in F0]

    def tuned_step(t):
        ctx.jcomm_outer(X, Ft, core=Gt, beta=beta, L=1, obj_out=trace[t:t + 1], cache_pq="auto")

    el_t, _, _, _ = timed_loop(ctx, tuned_step, 2, args.steps)
    out["tuned"] = {"entry": {k: (round(v, 4) if isinstance(v, float) else v) for k, v in entry.items()},
                    "outer_it_s": round(args.steps / el_t, 2)}
    return out


def oracle_rate(run, iters, sample, one_thread=True):
    """The FP64 oracle, as it stands: run(n) performs n outer iterations;
    timed with the BLAS threads the host gives it and (unless one_thread is
    False) with one thread."""
    try:
        from threadpoolctl import threadpool_info, threadpool_limits
        threads = max([p.get("num_threads", 1) for p in threadpool_info()] or [1])
    except Exception:
        threadpool_limits = None
        threads = os.cpu_count() or 1
    t0 = time.perf_counter()
    run(iters)
    dt = time.perf_counter() - t0
    out = {"value": iters / dt, "unit": "outer it/s", "cores": int(threads), "kind": "oracle",
           "sample": f"{iters} {sample}, {dt:.1f} s"}
    if one_thread and threadpool_limits is not None:
        with threadpool_limits(limits=1):
            t0 = time.perf_counter()
            run(1)
            d1 = time.perf_counter() - t0
        out["one_thread"] = {"value": 1 / d1, "unit": "outer it/s", "cores": 1, "sample": f"1 iteration, {d1:.1f} s"}
    return out


def run_cp4(args, ctx):
    """The paper's synthetic CP shape: order 4, 80 x 70 x 60 x 50, R = 10,
    J-CoMM (L = 1, objective every iteration).  Runs through the 3-way view
    5600 x 60 x 50 with the Khatri-Rao super factor of modes 1-2."""
    import numpy as np
    import torch
    import workloads
    from oracle import cp as ocp

    beta = args.beta if args.beta is not None else 1.0
    dims, R, L = (80, 70, 60, 50), 10, 1
    d = workloads.cp_dense(0, dims=dims, rank=R)
    X32 = d.X.astype(np.float32)
    init32 = [a.astype(np.float32) for a in d.init]
    X = torch.from_numpy(X32).cuda()
    fac = [torch.from_numpy(a).cuda() for a in init32]
    trace = torch.zeros(args.warmup + args.steps + 1, dtype=torch.float64, device="cuda")

    def step(t):
        ctx.jcomm_outer(X, fac, beta=beta, L=L, obj_out=trace[t:t + 1])

    elapsed, kernel_ms, launches, seen = timed_loop(ctx, step, args.warmup, args.steps)
    tr = trace.cpu().numpy()[args.warmup:args.warmup + args.steps]
    entries = int(np.prod(dims))
    avg_ms = kernel_ms / max(launches, 1)
    # per entry and pass: rebuild 2R plus two contraction chains of 2R (at
    # beta = 1 the reference pass's mode-3 chain and the chain shared by view
    # modes 1-2; otherwise one mode's numerator and denominator), counted at
    # the model's R = 10 although the tile pads R to 32
    flops = 6.0 * R * entries
    tfl = flops / (avg_ms * 1e-3) / 1e12
    out = base_line(args, elapsed)
    out.update({"metric": "J-CoMM outer iters/s (CP order 4, 80x70x60x50, R10)",
                "data": "synthetic (seeded Poisson around a planted Gamma(1,1) rank-10 CP model)",
                "config": {"workload": f"jcomm_cp_dense_80x70x60x50_r10_beta{beta}_L{L}_obj", "dims": list(dims),
                           "rank": R, "beta": beta, "inner_sweeps": L, "parallelism": "single GPU"},
                "roofline": {"bound": "mfma", "achieved": round(tfl, 2), "peak": PEAK_FP32_MFMA_TFLOPS,
                             "unit": "TFLOP/s", "frac": round(tfl / PEAK_FP32_MFMA_TFLOPS, 4), "traffic": None,
                             "kernel": "cp3_pass_kernel on the 5600 x 60 x 50 view",
                             "kernel_avg_us": round(avg_ms * 1e3, 2), "launches": seen, "launches_timed": launches,
                             "algorithmic_flops_per_launch": flops, "algorithmic_bytes_per_launch": 4 * entries,
                             "hbm_gbs_algorithmic": round(4 * entries / (avg_ms * 1e-3) / 1e9, 1)},
                "objective": {"first": float(tr[0]), "last": float(tr[-1]), "monotone": monotone(tr)}})
    if not args.no_cpu_baseline:
        X64 = X32.astype(np.float64)

        def run(n):
            cur = [a.astype(np.float64) for a in init32]
            for _ in range(n):
                cur, _ = ocp.jcomm_outer(X64, cur, beta, L=L, return_ref_obj=True)

        out["cpu_baseline"] = oracle_rate(run, 4, f"J-CoMM outer iterations (L={L}, beta={beta}, objective "
                                                  "included) on the full 80x70x60x50 tensor, NumPy float64")
    return out


def run_tucker4(args, ctx):
    """The paper's synthetic Tucker shape: order 4, 80 x 70 x 60 x 50, core
    10 x 9 x 8 x 7, J-CoMM (L = 1, objective every iteration)."""
    return run_tuckern(args, ctx, (80, 70, 60, 50), (10, 9, 8, 7))


def run_tucker5(args, ctx):
    """The shape and ranks of the paper's 5-way count experiment (27 x 24 x 7 x
    100 x 100, core 10 x 10 x 5 x 10 x 10, run there with dense contractions)
    on a synthetic dense tensor, J-CoMM (L = 1, objective every iteration)."""
    return run_tuckern(args, ctx, (27, 24, 7, 100, 100), (10, 10, 5, 10, 10))


def run_tuckern(args, ctx, dims, J):
    import numpy as np
    import torch
    import workloads
    from oracle import tucker as otk

    beta = args.beta if args.beta is not None else 1.0
    L = 1
    d = workloads.tucker_dense(0, dims=dims, core_dims=J)
    X32 = d.X.astype(np.float32)
    X = torch.from_numpy(X32).cuda()
    G = torch.from_numpy(d.init_core.astype(np.float32)).cuda()
    F = [torch.from_numpy(a.astype(np.float32)).cuda() for a in d.init_factors]
    trace = torch.zeros(args.warmup + args.steps + 1, dtype=torch.float64, device="cuda")

    def step(t):
        ctx.jcomm_outer(X, F, core=G, beta=beta, L=L, obj_out=trace[t:t + 1])

    elapsed, kernel_ms, launches, seen = timed_loop(ctx, step, args.warmup, args.steps)
    tr = trace.cpu().numpy()[args.warmup:args.warmup + args.steps]
    entries = int(np.prod(dims))
    avg_ms = kernel_ms / max(launches, 1)
    bytes_ = 4 * entries
    gbs = bytes_ / (avg_ms * 1e-3) / 1e9
    out = base_line(args, elapsed)
    shape = "x".join(map(str, dims))
    core = "x".join(map(str, J))
    rows = int(np.prod(dims[:-1]))
    out.update({"metric": f"J-CoMM outer iters/s (Tucker order {len(dims)}, {shape}, core {core})",
                "data": "synthetic (Gamma(shape 10) around a planted Tucker model, U(0,1) core and factors)",
                "config": {"workload": f"jcomm_tucker_dense_{shape}_core{core}_beta{beta}_L{L}_obj",
                           "dims": list(dims), "core": list(J), "beta": beta, "inner_sweeps": L,
                           "parallelism": "single GPU"},
                "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                             "frac": round(gbs / PEAK_HBM_GBS, 4), "traffic": None,
                             "kernel": f"tk_v_kernel / tk_m3_kernel on the {rows} x {dims[-1]} view",
                             "kernel_avg_us": round(avg_ms * 1e3, 2), "launches": seen, "launches_timed": launches,
                             "algorithmic_bytes_per_launch": bytes_},
                "objective": {"first": float(tr[0]), "last": float(tr[-1]), "monotone": monotone(tr)}})
    if not args.no_cpu_baseline:
        X64 = X32.astype(np.float64)

        def run(n):
            g, f = d.init_core.astype(np.float32).astype(np.float64), [a.astype(np.float32).astype(np.float64)
                                                                       for a in d.init_factors]
            for _ in range(n):
                g, f, _ = otk.jcomm_outer(X64, g, f, beta, L=L, return_ref_obj=True)

        out["cpu_baseline"] = oracle_rate(run, 3, f"J-CoMM outer iterations (L={L}, beta={beta}, objective "
                                                  f"included) on the full {shape} tensor, NumPy float64")
    return out


def run_coo(args, ctx):
    """Sparse 183x24x1140x1717 counts, 3.3M nonzeros, CP rank 32, beta = 1, L = 1."""
    import numpy as np
    import torch
    import workloads

    s = workloads.sparse_counts(0)
    idx = [torch.tensor(s.idx[:, n].astype(np.int32), device="cuda") for n in range(4)]
    val = torch.from_numpy(s.val.astype(np.float32)).cuda()
    fac = [torch.from_numpy(a.astype(np.float32)).cuda() for a in s.init]
    trace = torch.zeros(args.warmup + args.steps + 1, dtype=torch.float64, device="cuda")
    # the sorted copies are built once per tensor, outside the timed region
    torch.cuda.synchronize()
    tp = time.perf_counter()
    plan = ctx.coo_plan(idx, val, s.dims)
    plan_s = time.perf_counter() - tp

    def step(t):
        ctx.cp_jcomm_outer_coo_plan(plan, fac, L=1, obj_out=trace[t:t + 1])

    elapsed, kernel_ms, launches, seen = timed_loop(ctx, step, args.warmup, args.steps)
    tr = trace.cpu().numpy()[args.warmup:args.warmup + args.steps]
    nnz = int(val.numel())
    avg_ms = kernel_ms / max(launches, 1)
    bytes_ = 20 * nnz                    # 4 int32 indices + 1 float value per nonzero
    gbs = bytes_ / (avg_ms * 1e-3) / 1e9
    out = base_line(args, elapsed)
    out.update({"data": "synthetic (Zipf lat/lon, diurnal hour, Poisson(2)+1 counts)",
                "config": {"workload": "jcomm_cp_coo_183x24x1140x1717_nnz3.3M_r32_beta1_L1_obj",
                           "dims": list(s.dims), "nnz": nnz, "rank": 32, "beta": 1.0, "inner_sweeps": 1,
                           "parallelism": "single GPU"},
                "roofline": {"bound": "hbm", "achieved": round(gbs, 1), "peak": PEAK_HBM_GBS, "unit": "GB/s",
                             "frac": round(gbs / PEAK_HBM_GBS, 4), "traffic": None,
                             "kernel": "coo_plan_pass_kernel (two passes over the sorted copies: LDS-staged row offsets, gathers, model value, run sums)",
                             "kernel_avg_us": round(avg_ms * 1e3, 2), "launches": seen, "launches_timed": launches,
                             "algorithmic_bytes_per_launch": bytes_},
                "plan_build_s": round(plan_s, 4),
                "objective": {"first": float(tr[0]), "last": float(tr[-1]), "monotone": monotone(tr)}})
    plan.close()
    return out


def run_coo_beta(args, ctx):
    """Sparse 183x24x1140x1717 counts, 3.3M nonzeros, CP rank 32, beta != 1
    (default 1/2), J-CoMM L = 1 with the objective: numerators over the
    nonzeros, the Q~ denominators and the zero cells' objective from the dense
    pass over all 8.6G cells (the paper notes these are dense at beta != 1)."""
    import numpy as np
    import torch
    import workloads
    from oracle import cp as ocp

    beta = args.beta if args.beta is not None else 0.5
    s = workloads.sparse_counts(0)
    idx = [torch.tensor(s.idx[:, n].astype(np.int32), device="cuda") for n in range(4)]
    val = torch.from_numpy(s.val.astype(np.float32)).cuda()
    fac = [torch.from_numpy(a.astype(np.float32)).cuda() for a in s.init]
    trace = torch.zeros(args.warmup + args.steps + 1, dtype=torch.float64, device="cuda")

    def step(t):
        ctx.cp_jcomm_outer_coo(idx, val, s.dims, fac, L=1, obj_out=trace[t:t + 1], beta=beta)

    elapsed, kernel_ms, launches, seen = timed_loop(ctx, step, args.warmup, args.steps)
    tr = trace.cpu().numpy()[args.warmup:args.warmup + args.steps]
    cells = int(np.prod(s.dims))
    R = 32
    avg_ms = kernel_ms / max(launches, 1)
    # per cell and pass, what the denominators need: rebuild 2R and the Q
    # contraction chain 2R (the pass also runs its P chain on the zeros)
    flops = 4.0 * R * cells
    tfl = flops / (avg_ms * 1e-3) / 1e12
    out = base_line(args, elapsed)
    out.update({"metric": f"J-CoMM outer iters/s (sparse CP 183x24x1140x1717, 3.3M nnz, R32, beta {beta})",
                "data": "synthetic (Zipf lat/lon, diurnal hour, Poisson(2)+1 counts)",
                "config": {"workload": f"jcomm_cp_coo_183x24x1140x1717_nnz3.3M_r32_beta{beta}_L1_obj",
                           "dims": list(s.dims), "nnz": int(val.numel()), "rank": R, "beta": beta,
                           "inner_sweeps": 1, "parallelism": "single GPU"},
                "roofline": {"bound": "mfma", "achieved": round(tfl, 2), "peak": PEAK_FP32_MFMA_TFLOPS,
                             "unit": "TFLOP/s", "frac": round(tfl / PEAK_FP32_MFMA_TFLOPS, 4), "traffic": None,
                             "kernel": "cp3_pass_kernel over the 4392 x 1140 x 1717 view of the zero tensor",
                             "kernel_avg_us": round(avg_ms * 1e3, 2), "launches": seen, "launches_timed": launches,
                             "algorithmic_flops_per_launch": flops},
                "objective": {"first": float(tr[0]), "last": float(tr[-1]), "monotone": monotone(tr)}})
    if not args.no_cpu_baseline:
        # the dense oracle cannot hold this tensor (69 GB in float64): one outer
        # iteration on the sub-tensor of the first 114 latitude and 171
        # longitude indices (1/100 of the cells), scaled by the cell ratio
        keep = (s.idx[:, 2] < 114) & (s.idx[:, 3] < 171)
        sub = (183, 24, 114, 171)
        X = np.zeros(sub)
        X[tuple(s.idx[keep].T)] = s.val[keep]
        init = [a.astype(np.float32).astype(np.float64) for a in s.init]
        init = [init[0], init[1], init[2][:114], init[3][:171]]
        ratio = cells / float(np.prod(sub))

        def run(n):
            cur = init
            for _ in range(n):
                cur, _ = ocp.jcomm_outer(X, cur, beta, L=1, return_ref_obj=True)

        cb = oracle_rate(run, 1, f"J-CoMM outer iteration (L=1, beta={beta}, objective included) of the dense "
                                 f"oracle on the 183x24x114x171 sub-tensor ({int(keep.sum())} nonzeros), rate "
                                 f"divided by the cell ratio {ratio:.1f}", one_thread=False)
        cb["value"] = cb["value"] / ratio
        out["cpu_baseline"] = cb
    return out


def run_tucker5_coo(args, ctx):
    """Sparse counts with the shape, ranks and sparsity of the paper's 5-way
    experiment: 27 x 24 x 7 x 100 x 100, 0.6% nonzeros (Poisson(2) + 1),
    Tucker core 10 x 10 x 5 x 10 x 10, J-CoMM (L = 1, objective every
    iteration), beta = 1 by default (closed-form denominators, no dense pass)."""
    import numpy as np
    import torch
    import workloads
    from oracle import tucker as otk

    beta = args.beta if args.beta is not None else 1.0
    dims, J = (27, 24, 7, 100, 100), (10, 10, 5, 10, 10)
    s = workloads.sparse_small(0, dims=dims, density=0.006, rank=2)
    rng = np.random.default_rng(1)
    core0 = rng.uniform(0.1, 1.0, J).astype(np.float32)
    fac0 = [rng.uniform(0.1, 1.0, (d, j)).astype(np.float32) for d, j in zip(dims, J)]
    idx = [torch.tensor(s.idx[:, n].astype(np.int32), device="cuda") for n in range(5)]
    val = torch.from_numpy(s.val.astype(np.float32)).cuda()
    G = torch.from_numpy(core0).cuda()
    F = [torch.from_numpy(a).cuda() for a in fac0]
    trace = torch.zeros(args.warmup + args.steps + 1, dtype=torch.float64, device="cuda")

    def step(t):
        ctx.tucker_jcomm_outer_coo(idx, val, dims, G, F, beta=beta, L=1, obj_out=trace[t:t + 1])

    elapsed, kernel_ms, launches, seen = timed_loop(ctx, step, args.warmup, args.steps)
    tr = trace.cpu().numpy()[args.warmup:args.warmup + args.steps]
    nnz = int(val.numel())
    out = base_line(args, elapsed)
    out.update({"metric": f"J-CoMM outer iters/s (sparse Tucker 27x24x7x100x100, {nnz} nnz, core 10x10x5x10x10, "
                          f"beta {beta})",
                "data": "synthetic (uniform 0.6% support, Poisson(2)+1 counts)",
                "config": {"workload": f"jcomm_tucker_coo_27x24x7x100x100_nnz{nnz}_core10x10x5x10x10_beta{beta}_L1_obj",
                           "dims": list(dims), "nnz": nnz, "core": list(J), "beta": beta, "inner_sweeps": 1,
                           "parallelism": "single GPU"},
                "roofline": None if launches == 0 else {
                    "bound": "hbm", "kernel": "tk_v_kernel / tk_m3_kernel on the zero tensor (Q~ denominators)",
                    "kernel_avg_us": round(kernel_ms / launches * 1e3, 2), "launches": seen, "launches_timed": launches},
                "objective": {"first": float(tr[0]), "last": float(tr[-1]), "monotone": monotone(tr)}})
    if not args.no_cpu_baseline:
        X = workloads.densify(s)

        def run(n):
            g, f = core0.astype(np.float64), [a.astype(np.float64) for a in fac0]
            for _ in range(n):
                g, f, _ = otk.jcomm_outer(X, g, f, beta, L=1, return_ref_obj=True)

        out["cpu_baseline"] = oracle_rate(run, 2, f"J-CoMM outer iterations (L=1, beta={beta}, objective included) "
                                                  "of the dense oracle on the densified 45M-cell tensor", one_thread=False)
    return out


def _serving_pool(args):
    """The distinct requests a stream draws from: the first serve_pool specs of
    the seeded generator (dims U{16..256}, rank or core size in {4, 8, 16, 32},
    beta in {0, 1/2, 1, 3/2}, CP or Tucker), materialized once on the host, with
    one float32 payload per precision shared by every request that draws it."""
    import workloads
    from paper_2602_14683_amd import serving
    specs = workloads.serving_specs(seed=0, count=args.serve_pool, rate=1.0)
    mats = [workloads.materialize(s) for s in specs]
    payloads = {prec: [serving.from_workload(m, prec) for m in mats] for prec in ("bf16", "fp32")}
    for prec in payloads:
        for k, d in enumerate(payloads[prec]):
            d.tag = k
    return specs, mats, payloads


def _stream(n, rate, pool_size, seed):
    """n arrivals of a Poisson process of the given rate (per second), each
    drawing one of the pool's requests uniformly (seeded)."""
    import numpy as np
    rng = np.random.default_rng(seed)
    t = np.cumsum(rng.exponential(1.0 / rate, size=n)) if rate > 0 else np.zeros(n)
    return [(k, float(t[k]), int(rng.integers(0, pool_size))) for k in range(n)]


def _serve(ctx, stream, payloads, prec, batched, slots, budget, max_iters, grouped=False):
    from paper_2602_14683_amd import serving
    mode = ("grouped" if grouped else "batched") if batched else "per-request"
    print(f"serving: {len(stream)} requests, {prec}, {mode}", file=sys.stderr, flush=True)
    ex = (serving.BatchedExecutor(ctx, slots, graph=True, grouped=grouped) if batched
          else serving.SingleExecutor(ctx, 1))
    reqs = [serving.ServeRequest(rid, t, payloads[prec][k]) for rid, t, k in stream]
    srv = serving.Server(ex, budget, slots if batched else 1, tol=1e-4, max_iters=max_iters)
    done = srv.run(reqs)
    st = serving.summarize(done)
    st.update({"peak_slots": srv.peak_slots, "peak_bytes": srv.peak_bytes, "steps": srv.steps,
               "mem_waits": srv.mem_waits})
    return {k: (round(v, 3) if isinstance(v, float) else v) for k, v in st.items()}, done


def serving_stream(args, ctx):
    """A Poisson stream of CP / Tucker requests drawn from a pool of distinct
    requests (dims U{16..256}, rank or core size in {4, 8, 16, 32}, beta in {0,
    1/2, 1, 3/2}), each run to a relative objective change <= 1e-4 (or
    max_iters), served four ways on the same GPU: continuous batching with
    bf16 tiles, grouped and ungrouped, continuous batching in float32 (all
    replaying a captured graph of the batched step), and the plain per-request
    float32 loop.  Request
    tensors are drawn on the host before the clock starts; copying them to the
    device is part of each request's service.  Each bf16-served request's final
    objective is compared with the same request's float32 per-request result."""
    specs, mats, payloads = _serving_pool(args)
    stream = _stream(args.serve_requests, args.serve_rate, len(specs), 1)
    budget = int(args.serve_hbm_gib * (1 << 30))
    res, finals = {}, {}
    for name, prec, batched, grouped in (("grouped_bf16", "bf16", True, True), ("batched_bf16", "bf16", True, False),
                                         ("batched_fp32", "fp32", True, False), ("per_request_fp32", "fp32", False, False)):
        res[name], done = _serve(ctx, stream, payloads, prec, batched, args.serve_slots, budget, args.serve_max_iters,
                                 grouped)
        finals[name] = {c.rid: c.objective for c in done}
    base = res["per_request_fp32"]["solves_per_s"]
    res["speedup_solves_per_s"] = {k: round(res[k]["solves_per_s"] / base, 3)
                                   for k in ("grouped_bf16", "batched_bf16", "batched_fp32")}
    rel = [abs(finals["batched_bf16"][r] - finals["per_request_fp32"][r]) / abs(finals["per_request_fp32"][r])
           for r in finals["per_request_fp32"]]
    res["bf16_final_objective_rel_diff_vs_fp32"] = {"max": max(rel), "median": float(sorted(rel)[len(rel) // 2])}
    res["stream"] = {"requests": len(stream), "distinct": len(specs), "rate_per_s": args.serve_rate, "tol": 1e-4,
                     "max_iters": args.serve_max_iters, "slots": args.serve_slots,
                     "hbm_budget_gib": args.serve_hbm_gib,
                     "cp": sum(specs[k].model == "cp" for _, _, k in stream),
                     "tucker": sum(specs[k].model == "tucker" for _, _, k in stream)}
    return res


def run_serving(args, ctx):
    """The serving workload: first the per-request float32 loop's capacity
    (solves/s with every request waiting at t = 0), then Poisson streams of
    serve_requests arrivals at 0.5, 1 and 2 times that capacity, each served by
    grouped and ungrouped batches in bf16 and float32 and by the per-request
    float32 loop; the batched paths' own capacity (the same requests all
    waiting at t = 0); then one grouped bf16 stream at twice the per-request
    capacity with serve_budget_slots slots
    under a 1 GiB device-memory budget (a fresh context, so admission sees all
    the memory the library takes), where memory, not slots, holds requests
    back."""
    import paper_2602_14683_amd as comm
    import torch
    specs, mats, payloads = _serving_pool(args)
    budget = int(args.serve_hbm_gib * (1 << 30))
    cap_stream = _stream(args.serve_capacity_requests, 0.0, len(specs), 2)
    cap, _ = _serve(ctx, cap_stream, payloads, "fp32", False, 1, budget, args.serve_max_iters)
    capacity = cap["solves_per_s"]
    batched_capacity = {}
    for name, prec, grouped in (("grouped_bf16", "bf16", True), ("grouped_fp32", "fp32", True),
                                ("batched_bf16", "bf16", False), ("batched_fp32", "fp32", False)):
        st, _ = _serve(ctx, cap_stream, payloads, prec, True, args.serve_slots, budget, args.serve_max_iters, grouped)
        batched_capacity[name] = st["solves_per_s"]
    runs = {}
    for mult in (0.5, 1.0, 2.0):
        stream = _stream(args.serve_requests, mult * capacity, len(specs), 3)
        per = {}
        for name, prec, batched, grouped in (("grouped_bf16", "bf16", True, True),
                                             ("grouped_fp32", "fp32", True, True),
                                             ("batched_bf16", "bf16", True, False),
                                             ("batched_fp32", "fp32", True, False),
                                             ("per_request_fp32", "fp32", False, False)):
            per[name], done = _serve(ctx, stream, payloads, prec, batched, args.serve_slots, budget,
                                     args.serve_max_iters, grouped)
            if name == "grouped_bf16" and mult == 1.0:
                bf16_done = done
        base = per["per_request_fp32"]["solves_per_s"]
        per["speedup_solves_per_s"] = {k: round(per[k]["solves_per_s"] / base, 3)
                                       for k in ("grouped_bf16", "grouped_fp32", "batched_bf16", "batched_fp32")}
        runs[f"{mult:g}x_capacity"] = per
    # the reported bf16 objectives, re-evaluated in float64 by the library at
    # the returned factors (first served occurrence of each distinct request)
    first = {}
    for c in bf16_done:
        if c.status != "rejected" and c.result is not None:
            k = c.result.get("tag")
            if k is not None and k not in first:
                first[k] = c
    gaps = []
    for k, c in first.items():
        d = payloads["bf16"][k]
        X = torch.from_numpy(d.X).cuda()
        F = [torch.from_numpy(a).cuda() for a in c.result["factors"]]
        G = torch.from_numpy(c.result["core"]).cuda() if c.result["core"] is not None else None
        f64 = ctx.beta_objective(X, F, core=G, beta=d.beta).item()
        gaps.append(abs(c.objective - f64) / abs(f64))
    # admission under a 1 GiB budget, fresh context: enough slots and load that
    # memory binds before the slot count does
    small = comm.Context(0)
    try:
        stream = _stream(args.serve_requests, 2.0 * capacity, len(specs), 4)
        tight, _ = _serve(small, stream, payloads, "bf16", True, args.serve_budget_slots, 1 << 30,
                          args.serve_max_iters, grouped=True)
        tight["slots"] = args.serve_budget_slots
        tight["budget_bytes"] = 1 << 30
    finally:
        small.close()
    b = runs["1x_capacity"]["grouped_bf16"]
    out = {"metric": METRIC, "value": b["solves_per_s"], "unit": "solves/s", "n_gpus": 1,
           "steps": b["steps"], "warmup": 0, "ms_per_step": round(b["span_s"] / max(b["steps"], 1) * 1e3, 4),
           "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "bf16",
           "data": "synthetic (planted U(0,1) CP / Tucker models plus Poisson noise, Poisson arrivals)",
           "config": {"workload": f"serving_stream_{args.serve_requests}req_at_capacity_multiples",
                      "distinct_requests": len(specs), "slots": args.serve_slots, "parallelism": "single GPU"},
           "serving": {"per_request_fp32_capacity_solves_per_s": round(capacity, 3), "capacity_run": cap,
                       "batched_capacity_solves_per_s": batched_capacity,
                       "runs": runs, "budget_1gib_grouped_bf16_at_2x_capacity": tight,
                       "bf16_reported_vs_fp64_reevaluated": {"requests": len(gaps), "max": max(gaps) if gaps else None,
                                                             "median": sorted(gaps)[len(gaps) // 2] if gaps else None}}}
    return out


def main() -> int:
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=200)
    ap.add_argument("--warmup", type=int, default=5)
    ap.add_argument("--workload", choices=["cp", "tucker", "coo", "serving", "cp4", "tucker4", "tucker5", "coo_beta", "tucker5_coo"], default="cp",
                    help="cp: the headline 256^3 rank-32 CP workload; tucker / coo: the other pass kernels")
    ap.add_argument("--beta", type=float, default=None,
                    help="beta for --workload tucker (default 0), cp4, tucker4 and tucker5 (default 1), coo_beta (default 1/2)")
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-iters", type=int, default=15)
    ap.add_argument("--calibrate-copy", action="store_true")
    ap.add_argument("--no-comparisons", action="store_true",
                    help="skip the beta = 0.5 and block-MM rates on the same tensor")
    ap.add_argument("--comparison-steps", type=int, default=40)
    ap.add_argument("--no-serving", action="store_true", help="skip the serving stream in the default run")
    ap.add_argument("--serve-requests", type=int, default=None,
                    help="arrivals per stream (default 64 beside the headline run, 2000 for --workload serving)")
    ap.add_argument("--serve-pool", type=int, default=48, help="distinct requests the streams draw from")
    ap.add_argument("--serve-capacity-requests", type=int, default=150,
                    help="requests of the per-request loop's capacity run (--workload serving)")
    ap.add_argument("--serve-rate", type=float, default=400.0, help="arrivals per second")
    ap.add_argument("--serve-slots", type=int, default=16)
    ap.add_argument("--serve-budget-slots", type=int, default=96,
                    help="slots of the 1 GiB budget run (--workload serving)")
    ap.add_argument("--serve-max-iters", type=int, default=500)
    ap.add_argument("--serve-hbm-gib", type=float, default=64.0, help="device memory budget for admission")
    args = ap.parse_args()
    if args.serve_requests is None:
        args.serve_requests = 2000 if args.workload == "serving" else 64

    if args.gpus != 1:
        print(f"bench.py measures one GPU only: this build has no multi-GPU path (asked for --gpus {args.gpus}).",
              file=sys.stderr)
        return 2
    if args.calibrate_copy:
        calibrate_copy()
        return 0

    import paper_2602_14683_amd as comm
    ctx = comm.Context(0)
    out = {"cp": run_cp, "tucker": run_tucker, "coo": run_coo, "serving": run_serving, "cp4": run_cp4,
           "tucker4": run_tucker4, "tucker5": run_tucker5, "coo_beta": run_coo_beta,
           "tucker5_coo": run_tucker5_coo}[args.workload](args, ctx)
    if args.workload == "cp" and not args.no_serving:
        out["serving"] = serving_stream(args, ctx)
    ctx.close()
    print(json.dumps(out), flush=True)
    return 0


if __name__ == "__main__":
    sys.exit(main())
