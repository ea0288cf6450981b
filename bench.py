"""Benchmark of the ABX hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Workload: the within-speaker triphone-like task at full size (100k items,
40 labels, BY prev / next / speaker, lengths 5-25 frames, dim 768, FP32
features resident in HBM).  One step = the whole hot path on it: build the
task (cells), score every cell (normalise -> frame distances -> DTW ->
triplet comparison -> FP64 recheck -> per-cell counts on the host) and
collapse to the ABX error rate.  `value` is triplets per second of the
BF16-MFMA + FP64-recheck form; the plain FP32 form is timed beside it on the
same data.  A short serving stream (jobs of 1k-50k items, dims 256-1280,
within / across, Poisson arrivals) reports p50 / p99 job latency.

Prints one JSON line: the metric and its value, the step time, device time,
the roofline of the dominant kernel and a CPU baseline of the oracle.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

HBM_PEAK_GBS = 8000.0


MFMA_BF16_PEAK_TFLOPS = 2500.0


def log(msg):
    print(f"[bench {time.strftime('%H:%M:%S')}] {msg}", file=sys.stderr, flush=True)


def _stage_means(results):
    keys = ["ms_total", "ms_normalize", "ms_distance", "ms_triplets", "ms_recheck", "ms_host_setup",
            "ms_host_finish", "ms_task_build", "ms_score_call", "ms_collapse"]
    return {k: float(np.mean([r[k] for r in results])) for k in keys}


# Workloads this bench can time.  The default, "c2", is the headline one; the
# others exist to profile the kernels on large BY groups and the pooled mode.
WORKLOADS = {
    "c2": ("within_c2", "dtw", "within-speaker triphone task: 100k items, 40 labels, BY prev/next/speaker, "
           "lengths 5-25 (median 9), dim 768 fp32, DTW, path-normalised angular"),
    "c3": ("across_c3", "dtw", "across-speaker triphone task: 200k items, 40 labels, 100 speakers, BY prev/next "
           "ACROSS speaker, lengths 3-40, dim 1024 fp32, DTW, path-normalised angular"),
    "c4": ("batched_c4", "dtw", "batched uneven groups: 5000 BY groups of Zipf(1.1) sizes 2-2000 items, lengths "
           "1-60, dim 512 bf16, DTW, path-normalised angular"),
    "c4-pooled": ("batched_c4", "pooled", "batched uneven groups (as c4), mean-pooled mode: one vector per item"),
}


# extra score options (a forced fused-kernel configuration, --fused-config)
SCORE_KW = {}


class _NoCyclicGC:
    """Timed loops run with Python's cyclic garbage collector paused (after a
    collection), as timeit does: a full collection over torch's objects takes
    tens of ms and would land inside one step.  The library's objects are freed
    by reference counting either way."""

    def __enter__(self):
        import gc
        gc.collect()
        self.was = gc.isenabled()
        gc.disable()

    def __exit__(self, *exc):
        import gc
        if self.was:
            gc.enable()


def run_pipelined(fx, ds, w, precision, n, sync, mode="dtw", side="launch", side_serial=True, depth=2, **kw):
    """n steps with host and device work overlapped across steps: while the
    device scores step i, the host builds the task of step i + 1 and collapses
    the result of step i - 1.  `side` picks what runs on a second host thread:
    "launch" (default) leaves the main thread only the task builds, the side
    thread enqueueing each step's score (fabx_score_async) and then waiting for
    and collapsing the step before it; "collapse" keeps the launch on the main
    thread; "none" runs everything on the main thread.  The library's thread
    pool runs a region issued while another thread's region is active in place
    on the issuing thread; with side_serial the second thread's host work
    always runs in place there (fabx_set_thread_serial), so that it never takes
    the pool from a build.  With side "launch", `depth` scores stay enqueued on
    the device: the second thread waits for and collapses step i - depth after
    launching step i, and the main thread builds up to `depth` steps ahead, so
    a host stall shorter than a step leaves the device busy.  Every step still
    runs the whole path on its own task."""
    import concurrent.futures as cf

    stats, errs = [], []

    def finish(res):
        st = res.stats           # waits for the score
        return res.collapse(w.levels), st

    def take(out):
        if out is not None:
            errs.append(out[0])
            stats.append(out[1])

    prev = [None]

    import collections
    pending = collections.deque()   # launched, not yet finished (second thread only)

    def launch_then_finish_old(task):
        pending.append(task.score_async(mode=mode, precision=precision, **SCORE_KW, **kw))
        return finish(pending.popleft()) if len(pending) > depth else None

    def finish_rest():
        return [finish(pending.popleft()) for _ in range(len(pending))]

    fut = None
    futs = collections.deque()
    with cf.ThreadPoolExecutor(max_workers=1, initializer=fx.fabx_set_thread_serial,
                               initargs=(side_serial,)) as pool, _NoCyclicGC():
        t0 = time.perf_counter()
        for _ in range(n):
            task = fx.Task(ds, w.on, w.by, w.across)
            if side == "launch":
                futs.append(pool.submit(launch_then_finish_old, task))
                if len(futs) > depth:
                    take(futs.popleft().result())
                continue
            res = task.score_async(mode=mode, precision=precision, **SCORE_KW, **kw)
            if prev[0] is not None:
                if side == "collapse":
                    if fut is not None:
                        take(fut.result())
                    fut = pool.submit(finish, prev[0])
                else:
                    take(finish(prev[0]))
            prev[0] = res
        while futs:
            take(futs.popleft().result())
        for out in pool.submit(finish_rest).result():
            take(out)
        if fut is not None:
            take(fut.result())
        if prev[0] is not None:
            take(finish(prev[0]))
    sync()
    return time.perf_counter() - t0, stats, errs


def run_steps(fx, ds, w, precision, n, sync, mode="dtw"):
    stats, errs = [], []
    with _NoCyclicGC():
        t0 = time.perf_counter()
        for _ in range(n):
            ta = time.perf_counter()
            task = fx.Task(ds, w.on, w.by, w.across)
            tb = time.perf_counter()
            res = task.score(mode=mode, precision=precision, **SCORE_KW)
            tc = time.perf_counter()
            errs.append(res.collapse(w.levels))
            td = time.perf_counter()
            st = res.stats
            st.update(ms_task_build=(tb - ta) * 1e3, ms_score_call=(tc - tb) * 1e3, ms_collapse=(td - tc) * 1e3)
            stats.append(st)
        sync()
    return time.perf_counter() - t0, stats, errs


def serving_stream(fx, ctx, torch, workloads, n_jobs, seed=4):
    """Poisson arrivals at 0.7 x the alone service rate; p50 / p99 of completion - arrival."""
    jobs = []
    for j in range(n_jobs):
        w = workloads.serving_job(j, seed=seed, device="cuda")
        ds = fx.Dataset(ctx, w.features, w.offsets, w.attrs)
        jobs.append((w, ds))
    log(f"serving: {n_jobs} jobs generated")
    # alone service time of each job (also its reference result)
    alone_ms, ref = [], []
    for w, ds in jobs:
        t0 = time.perf_counter()
        r = fx.Task(ds, w.on, w.by, w.across).score()
        alone_ms.append((time.perf_counter() - t0) * 1e3)
        ref.append(r.half_units.copy())
        st = r.stats
        log(f"serving: alone {w.name} n={w.n_items} dim={w.dim} cells={len(r.half_units)} "
            f"{alone_ms[-1]:.1f} ms  gpu {st['ms_total']:.1f} ms (dist {st['ms_distance']:.1f}, "
            f"trip {st['ms_triplets']:.1f}, recheck {st['ms_recheck']:.1f}) nonrobust={st['n_nonrobust_pairs']} "
            f"recheck_pairs={st['n_recheck_pairs']} recount_rows={st['n_recount_rows']} pairs={st['n_pairs']}")
    mean_s = float(np.mean(alone_ms)) / 1e3
    rng = np.random.default_rng(seed)
    gaps = rng.exponential(mean_s / 0.7, size=n_jobs)
    srv = fx.Server(ctx, hbm_budget_bytes=96 << 30, n_streams=4)
    start = time.perf_counter()
    ids = []
    t_next = start
    for (w, ds), g in zip(jobs, gaps):
        t_next += g
        while time.perf_counter() < t_next:
            time.sleep(0.0002)
        ids.append(srv.submit(ds, w.on, w.by, w.across))
    triplets = 0
    same = True
    log("serving: all jobs submitted")
    for jid, rw in zip(ids, ref):
        keys, W, n, s = srv.wait(jid)
        triplets += int(n.sum())
        same = same and np.array_equal(W, rw)
    wall = time.perf_counter() - start
    st = srv.stats
    srv.close()
    return {"jobs": n_jobs, "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"],
            "triplets_per_s": triplets / wall, "hbm_high_water_bytes": st["hbm_high_water"],
            "alone_mean_ms": float(np.mean(alone_ms)), "arrival_rate_per_s": 0.7 / mean_s,
            "results_equal_alone": bool(same)}


def cpu_baseline(oracle, w, target_seconds=20.0):
    """The FP64 oracle on the host cores: whole BY groups of the same workload, in
    group order, about `target_seconds` of oracle work.  The sample is sized by
    the oracle's cost per group (its squared frame count) at the rate measured
    on a small probe."""
    feats = w.features_f32_host()
    cells = oracle.cells(w.attrs, w.on, w.by, w.across)
    groups, seen = [], set()
    for c in cells:
        if c.by_key not in seen:
            seen.add(c.by_key)
            groups.append(c.by_key)
    frames = {}
    lens = np.diff(w.offsets)
    for i, key in enumerate(map(tuple, w.attrs[:, w.by].tolist())):
        frames[key] = frames.get(key, 0) + int(lens[i])
    cost = np.array([float(frames[tuple(g)]) ** 2 for g in groups])
    log(f"cpu baseline: {len(cells)} cells in {len(groups)} groups")

    def run(take):
        t0 = time.perf_counter()
        r = oracle.score(feats, w.offsets, w.attrs, w.on, w.by, w.across, cell_filter=lambda c: c.by_key in take)
        return r, time.perf_counter() - t0

    # grow the sample (by cost) until one run takes a good part of the target
    ccost = np.cumsum(cost)
    budget = 0.005 * ccost[-1]
    while True:
        n_take = min(len(groups), int(np.searchsorted(ccost, budget)) + 1)
        r, dt = run(set(groups[:n_take]))
        log(f"cpu baseline: {n_take} groups took {dt:.1f} s")
        if dt >= 0.5 * target_seconds or n_take == len(groups):
            break
        budget = ccost[n_take - 1] * min(8.0, target_seconds / max(dt, 1e-3))
    n_trip = int(r.n_triplets.sum())
    return {"value": n_trip / dt, "unit": "triplets/s", "cores": oracle.num_threads(), "kind": "oracle",
            "sample": f"{min(n_take, len(groups))} of {len(groups)} BY groups ({len(r.cells)} cells, {n_trip} "
                      f"triplets) of the same workload, FP64 DTW + scoring, {dt:.1f} s"}


def committed_traffic(kernel_file, profile_file, cols, blocks_per_cu):
    """HBM bytes per launch of the dominant kernel in the configuration that ran,
    from the committed rocprofv3 byte-counter summary, used only while the kernel
    source is the one that was measured (its SHA-256 prefix is recorded beside
    the figure)."""
    import hashlib
    root = os.path.dirname(os.path.abspath(__file__))
    try:
        src = open(os.path.join(root, kernel_file), "rb").read()
        lines = open(os.path.join(root, profile_file)).read().splitlines()
    except OSError:
        return None
    want = {"source_sha256": hashlib.sha256(src).hexdigest()[:16],
            "kernel": f"k_fused<{cols},true>", "blocks_per_cu": str(blocks_per_cu)}
    for line in lines:
        f = line.strip().strip("`").split()
        if not f or f[0] != "traffic":
            continue
        kv = dict(x.split("=", 1) for x in f[1:] if "=" in x)
        if all(kv.get(k) == v for k, v in want.items()):
            return float(kv["bytes_per_launch"])
    return None


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps (default: 200 for c2, whose steps take about 2 ms, else 3)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps (default: 10 for c2, else 1)")
    ap.add_argument("--serve-jobs", type=int, default=12)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--serving-only", action="store_true", help="run only the serving stream")
    ap.add_argument("--no-autotune", action="store_true", help="keep the default fused-kernel tiles")
    ap.add_argument("--fused-config", default=None, metavar="COLS,BLOCKS_PER_CU",
                    help="run the fused kernel with this column width and grid (e.g. 128,0) "
                         "instead of autotuning")
    ap.add_argument("--side", choices=("launch", "collapse", "none"), default="launch",
                    help="work of the pipelined steps on a second host thread: score launch and "
                         "collapse (default), collapse only, or none")
    ap.add_argument("--depth", type=int, default=2,
                    help="scores kept enqueued on the device by the pipelined loop (side 'launch')")
    ap.add_argument("--side-pool", action="store_true",
                    help="let the second host thread's work use the shared host thread pool")
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="c2",
                    help="c2 (default) is the headline workload; c3 / c4 / c4-pooled profile large groups")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run 3 plain device copies of this many MiB (to scale HBM byte counters)")
    args = ap.parse_args()
    if args.steps is None:
        args.steps = 200 if args.workload == "c2" else 3
    if args.warmup is None:
        args.warmup = 10 if args.workload == "c2" else 1
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the ABX hot path here is "
              "single-GPU (it would shard by BY groups, each GPU scoring its groups' cells).", file=sys.stderr)
        sys.exit(2)

    import torch
    import workloads
    import paper_2505_02692_amd as fx

    fx.lib()  # fail loudly if the native library is missing
    torch.cuda.set_device(0)
    sync = torch.cuda.synchronize
    if args.serving_only:
        print(json.dumps({"serving": serving_stream(fx, fx.Context(0), torch, workloads, args.serve_jobs)}))
        return
    if args.copy_calibration_mib > 0:
        n = args.copy_calibration_mib << 18   # float32 elements
        src = torch.ones(n, device="cuda")
        dst = torch.empty_like(src)
        for _ in range(3):
            dst.copy_(src)
        sync()
        log(f"copy calibration: 3 copies of {args.copy_calibration_mib} MiB (read + write each)")
        del src, dst
    gen_name, mode, wl_desc = WORKLOADS[args.workload]
    headline = args.workload == "c2"
    w = getattr(workloads, gen_name)(device="cuda")
    ctx = fx.Context(0)
    ds = fx.Dataset(ctx, w.features, w.offsets, w.attrs)
    log(f"workload {args.workload} ready: {w.n_items} items, {w.n_frames} frames, dim {w.dim}")

    side = args.side
    if args.fused_config:
        cols, bpc = (int(v) for v in args.fused_config.split(","))
        SCORE_KW.update(fused_cols=cols, fused_blocks_per_cu=bpc)
    run_pipelined(fx, ds, w, "bf16", args.warmup, sync, mode, side, not args.side_pool, args.depth)
    sync()
    log("warmup done")
    # untimed: pick the fused kernel's tiles / grid for this task shape
    tune = (fx.Task(ds, w.on, w.by, w.across).autotune(mode=mode)
            if not (args.no_autotune or args.fused_config) else None)
    log(f"autotune: {tune}")
    dt, pstats_, errs = run_pipelined(fx, ds, w, "bf16", args.steps, sync, mode, side, not args.side_pool, args.depth)
    ms_step = dt / args.steps * 1e3
    log(f"bf16 form, pipelined: {ms_step:.2f} ms/step")
    # the same steps one after another, for the per-stage breakdown
    sdt, stats, serrs = run_steps(fx, ds, w, "bf16", args.steps, sync, mode)
    ms_step_serial = sdt / args.steps * 1e3
    log(f"bf16 form, serial: {ms_step_serial:.2f} ms/step, stages {_stage_means(stats)}")
    assert errs[-1] == serrs[-1]
    st0 = stats[-1]
    n_trip = st0["n_triplets"]
    value = n_trip / (ms_step / 1e3)
    stages = _stage_means(stats)
    t_build = []
    for _ in range(3):
        t0 = time.perf_counter()
        fx.Task(ds, w.on, w.by, w.across)
        t_build.append((time.perf_counter() - t0) * 1e3)

    plain = euclid = None
    if not args.no_plain and headline:
        run_pipelined(fx, ds, w, "fp32", 1, sync, mode, side, not args.side_pool, args.depth)
        pdt, _, perrs = run_pipelined(fx, ds, w, "fp32", args.steps, sync, mode, side, not args.side_pool, args.depth)
        pms = pdt / args.steps * 1e3
        psdt, pstats, _ = run_steps(fx, ds, w, "fp32", args.steps, sync, mode)
        pst = _stage_means(pstats)
        log(f"fp32 form: {pms:.2f} ms/step pipelined, {psdt / args.steps * 1e3:.2f} serial, stages {pst}")
        plain = {"triplets_per_s": n_trip / (pms / 1e3), "ms_per_step": pms,
                 "ms_per_step_serial": psdt / args.steps * 1e3,
                 "gcups": pstats[-1]["dtw_cells_sym"] / (pms / 1e3) / 1e9,
                 "gpu_ms": pst["ms_total"], "gpu_triplets_per_s": n_trip / (pst["ms_total"] / 1e3),
                 "abx_error": perrs[-1], "stages_ms": pst}
        # the other distance the Score interface names, in the FP32 form
        run_pipelined(fx, ds, w, "fp32", 1, sync, mode, side, not args.side_pool, args.depth, distance="euclidean")
        edt, estats, eerrs = run_pipelined(fx, ds, w, "fp32", args.steps, sync, mode, side,
                                           not args.side_pool, args.depth, distance="euclidean")
        ems = edt / args.steps * 1e3
        egpu = float(np.median([s_["ms_total"] for s_ in estats]))
        log(f"euclidean fp32 form: {ems:.2f} ms/step pipelined, device {egpu:.2f} ms")
        euclid = {"triplets_per_s": n_trip / (ems / 1e3), "ms_per_step": ems, "gpu_ms_pipelined": egpu,
                  "gpu_triplets_per_s": n_trip / (egpu / 1e3), "abx_error": eerrs[-1]}

    # roofline of the dominant kernel, from the live HIP-event stage times
    dim, dim_pad = w.dim, (w.dim + 63) // 64 * 64
    nf = st0["n_frames"]
    in_bytes = w.features.element_size()
    rows = nf if mode == "dtw" else st0["n_items"]
    norm_bytes = (nf * dim * in_bytes) + rows * dim_pad * 2 + rows * 4
    # DTW: the frame pairs of the unordered item pairs the cells need (the DTW
    # distance is symmetric, so each pair's DTW is needed once)
    dist_flops = 2.0 * dim * (st0["dtw_cells_sym"] if mode == "dtw" else st0["n_pairs"])
    # kernel durations of the timed (pipelined) steps, HIP events on the stream
    # the kernels run on; the serial steps (idle GPU between them) run slower
    pk = {k: float(np.mean([s_[k] for s_ in pstats_])) for k in ("ms_normalize", "ms_distance")}
    if pk["ms_normalize"] >= pk["ms_distance"]:
        ach = norm_bytes / (pk["ms_normalize"] / 1e3) / 1e9
        roof = {"kernel": "k_normalize", "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "traffic": None,
                "algorithmic_bytes_per_launch": norm_bytes, "ms_per_launch": pk["ms_normalize"]}
    else:
        ach = dist_flops / (pk["ms_distance"] / 1e3) / 1e12
        traffic = (committed_traffic("paper_2505_02692_amd/csrc/k_fused.hip", "profiles/hbm_bytes_within_c2.md",
                                     st0["fused_cols"], st0["fused_blocks_per_cu"])
                   if (headline and mode == "dtw") else None)
        roof = {"kernel": "k_fused" if mode == "dtw" else "k_gram_angular_bf16", "bound": "mfma",
                "achieved": ach, "peak": MFMA_BF16_PEAK_TFLOPS,
                "unit": "TFLOP/s", "frac": ach / MFMA_BF16_PEAK_TFLOPS, "traffic": traffic,
                "algorithmic_flops_per_launch": dist_flops, "ms_per_launch": pk["ms_distance"]}

    serving = None
    if args.serve_jobs > 0 and headline:
        serving = serving_stream(fx, ctx, torch, workloads, args.serve_jobs)
        log(f"serving: {serving}")

    cpu = None
    if not args.no_cpu_baseline and headline:
        import oracle
        cpu = cpu_baseline(oracle, w)
        log(f"cpu baseline: {cpu}")

    out = {
        "metric": "ABX triplets/s (BF16 MFMA + FP64 recheck form)",
        "value": value,
        "unit": "triplets/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms_step,
        "ms_per_step_serial": ms_step_serial,
        # device time (first kernel to per-cell results, HIP events) of the
        # pipelined steps themselves, median: the part of a step the GPU is busy
        "gpu_ms_pipelined": float(np.median([s_["ms_total"] for s_ in pstats_])) if pstats_ else None,
        "triplets_per_s_serial": n_trip / (ms_step_serial / 1e3),
        "pipelined": ("host work of neighbouring steps overlaps device work (fabx_score_async)"
                      + {"launch": f"; the main thread builds up to {args.depth} steps ahead while a second "
                                   f"host thread launches step i and collapses step i - {args.depth} "
                                   f"({args.depth} scores stay enqueued on the device)",
                         "collapse": "; the collapse of step i - 1 runs on a second host thread beside "
                                     "the build of step i + 1",
                         "none": ""}[side]),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic (seeded Gaussian SSL-like features: label centroid + speaker offset + frame noise)",
        "config": {"workload": wl_desc,
                   "cells": st0["n_cells"], "triplets": n_trip, "dtw_cells": st0["dtw_cells"],
                   "dtw_cells_unordered": st0["dtw_cells_sym"],
                   "parallelism": "single GPU"},
        "gcups": st0["dtw_cells_sym"] / (ms_step / 1e3) / 1e9,
        "gpu_ms": stages["ms_total"],
        "gpu_triplets_per_s": n_trip / (stages["ms_total"] / 1e3),
        "task_build_ms": float(np.median(t_build)),
        "stages_ms": stages,
        "abx_error": errs[-1],
        "recheck_pairs": st0["n_recheck_pairs"], "nonrobust_pairs": st0["n_nonrobust_pairs"],
        "plain_fp32": plain,
        "euclidean_fp32": euclid,
        "autotune": tune,
        "fused_config": {"cols": st0["fused_cols"], "blocks_per_cu": st0["fused_blocks_per_cu"]},
        "roofline": roof,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
