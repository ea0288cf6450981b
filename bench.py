"""Benchmark of the ABX hot path on one MI355X.

    python bench.py [--steps K] [--warmup W] [--gpus 1]

Headline workload: batched uneven cells, the largest configuration that runs
on one GPU: 5,000 BY groups of Zipf(1.1) sizes 2-2000 items (1.05M items,
31M frames), item lengths 1-60 frames, dim 512, features stored as BF16 and
resident in HBM; ON label BY group, DTW with the path-normalised angular
distance.  One step = the whole hot path on it: build the task (cells),
score every cell (normalise -> frame distances on MFMA -> DTW -> triplet
comparison -> FP64 recheck of near ties -> per-cell counts on the host) and
collapse to the ABX error rate.  `value` is triplets per second of the
BF16-MFMA + FP64-recheck form.  Beside it, on the same MI355X: the plain FP32
form on the same data, the mean-pooled mode, the within-speaker triphone
workload (and a harder variant of it whose near ties go to the FP64 recheck),
a serving stream of 400 jobs (1k-50k items, dims 256-1280, within / across,
Poisson arrivals) with p50 / p99 job latency, and the FP64 oracle timed on the
host cores.

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


# Workloads this bench can time as its main leg.  The default, "c4", is the
# headline: the largest configuration that fits one GPU.
WORKLOADS = {
    "c4": ("batched_c4", "dtw", "batched uneven cells in one persistent launch: 5000 BY groups of Zipf(1.1) "
           "sizes 2-2000 items (1.05M items, 31M frames), lengths 1-60, dim 512 stored bf16, ON label BY group, "
           "DTW, path-normalised angular"),
    "c4-pooled": ("batched_c4", "pooled", "batched uneven cells (as c4), mean-pooled mode: one vector per item"),
    "c2": ("within_c2", "dtw", "within-speaker triphone task: 100k items, 40 labels, BY prev/next/speaker, "
           "lengths 5-25 (median 9), dim 768 fp32, DTW, path-normalised angular"),
    "c3": ("across_c3", "dtw", "across-speaker triphone task: 200k items, 40 labels, 100 speakers, BY prev/next "
           "ACROSS speaker, lengths 3-40, dim 1024 fp32, DTW, path-normalised angular"),
    "c2-hard": ("within_c2", "dtw", "within-speaker triphone task (as c2) with label centroids of std 0.1, "
                "so that many comparisons are near ties and go to the FP64 recheck"),
}
# generator arguments of the workloads above that differ from the generators' defaults
WORKLOAD_KW = {"c2-hard": {"centroid_std": 0.1}}


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


def run_steps(fx, ds, w, precision, n, sync, mode="dtw", **kw):
    """n steps one after another (build, score, collapse), for the per-stage breakdown."""
    stats, errs = [], []
    with _NoCyclicGC():
        t0 = time.perf_counter()
        for _ in range(n):
            ta = time.perf_counter()
            task = fx.Task(ds, w.on, w.by, w.across)
            tb = time.perf_counter()
            res = task.score(mode=mode, precision=precision, **SCORE_KW, **kw)
            tc = time.perf_counter()
            errs.append(res.collapse(w.levels))
            td = time.perf_counter()
            st = res.stats
            st.update(ms_task_build=(tb - ta) * 1e3, ms_score_call=(tc - tb) * 1e3, ms_collapse=(td - tc) * 1e3)
            stats.append(st)
        sync()
    return time.perf_counter() - t0, stats, errs


def pipelined_leg(fx, ds, w, precision, steps, warmup, sync, mode, args, **kw):
    """warmup + timed pipelined steps; (ms per step, per-step stats, ABX errors)."""
    if warmup > 0:
        run_pipelined(fx, ds, w, precision, warmup, sync, mode, args.side, not args.side_pool, args.depth, **kw)
    dt, st, errs = run_pipelined(fx, ds, w, precision, steps, sync, mode, args.side, not args.side_pool,
                                 args.depth, **kw)
    return dt / steps * 1e3, st, errs


def cpu_info():
    model = "unknown"
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                model = line.split(":", 1)[1].strip()
                break
    except OSError:
        pass
    try:
        n = len(os.sched_getaffinity(0))
    except AttributeError:
        n = os.cpu_count()
    return model, n


def serving_stream(fx, ctx, torch, workloads, n_jobs, seed=4, load=0.7, n_streams=4, budget=96 << 30):
    """The serving configuration: n_jobs jobs (1k-50k items, dims 256-1280,
    within / across) arriving as a Poisson stream at `load` x the alone service
    rate.  Each job is first scored alone (its service time and reference
    counts); then the stream is served by a fabx server.  A job's features are
    made on the device just before its arrival time (the client's side; only
    the jobs in flight hold features).  Latency = completion - entry into
    submit, measured by the server, with its parts (task build in submit, queue
    wait, run)."""
    alone_ms, ref, n_trip = [], [], []
    t_alone = time.perf_counter()
    for j in range(n_jobs):
        w = workloads.serving_job(j, seed=seed, device="cuda")
        ds = fx.Dataset(ctx, w.features, w.offsets, w.attrs)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        r = fx.Task(ds, w.on, w.by, w.across).score()
        alone_ms.append((time.perf_counter() - t0) * 1e3)
        ref.append(r.half_units.copy())
        n_trip.append(int(r.n_triplets.sum()))
        st = r.stats
        if j < 8 or j % 50 == 0:
            log(f"serving: alone {w.name} n={w.n_items} dim={w.dim} cells={len(r.half_units)} "
                f"{alone_ms[-1]:.1f} ms  gpu {st['ms_total']:.1f} ms (dist {st['ms_distance']:.1f}, "
                f"trip {st['ms_triplets']:.1f}, recheck {st['ms_recheck']:.1f}) nonrobust={st['n_nonrobust_pairs']} "
                f"recheck_pairs={st['n_recheck_pairs']} recount_rows={st['n_recount_rows']}")
        del r, ds, w
    log(f"serving: {n_jobs} jobs scored alone in {time.perf_counter() - t_alone:.1f} s, "
        f"mean {np.mean(alone_ms):.1f} ms, max {np.max(alone_ms):.1f} ms")
    mean_s = float(np.mean(alone_ms)) / 1e3
    rng = np.random.default_rng(seed)
    arrivals = np.cumsum(rng.exponential(mean_s / load, size=n_jobs))
    srv = fx.Server(ctx, hbm_budget_bytes=budget, n_streams=n_streams)
    inflight = {}
    same, done, late = True, 0, 0
    triplets = 0

    def reap(block=False):
        nonlocal same, done, triplets
        for jid in list(inflight):
            out = srv.wait(jid) if block else srv.poll(jid)
            if out is None:
                continue
            j = inflight.pop(jid)
            same = same and np.array_equal(out[1], ref[j])
            triplets += n_trip[j]
            done += 1

    start = time.perf_counter()
    for j in range(n_jobs):
        w = workloads.serving_job(j, seed=seed, device="cuda")
        ds = fx.Dataset(ctx, w.features, w.offsets, w.attrs)
        t_arr = start + arrivals[j]
        if time.perf_counter() > t_arr + 0.002:
            late += 1
        while time.perf_counter() < t_arr:
            reap()
            time.sleep(0.0002)
        inflight[srv.submit(ds, w.on, w.by, w.across)] = j
        del ds, w
        reap()
        if j % 50 == 49:
            log(f"serving: {j + 1} jobs submitted, {done} done")
    while inflight:
        reap(block=True)
    wall = time.perf_counter() - start
    st = srv.stats
    srv.close()
    return {"jobs": n_jobs, "completed": st["completed"], "failed": st["failed"],
            "p50_ms": st["p50_ms"], "p99_ms": st["p99_ms"],
            "p50_queue_ms": st["p50_queue_ms"], "p99_queue_ms": st["p99_queue_ms"],
            "mean_build_ms": st["mean_build_ms"], "mean_queue_ms": st["mean_queue_ms"],
            "mean_run_ms": st["mean_run_ms"],
            "triplets_per_s": triplets / wall, "wall_s": wall, "hbm_high_water_bytes": st["hbm_high_water"],
            "hbm_budget_bytes": budget, "streams": n_streams,
            "alone_mean_ms": float(np.mean(alone_ms)), "alone_p50_ms": float(np.median(alone_ms)),
            "alone_max_ms": float(np.max(alone_ms)), "arrival_rate_per_s": load / mean_s, "load": load,
            "late_arrivals": late, "results_equal_alone": bool(same)}


def cpu_baseline(oracle, fx, w, target_seconds=15.0, seed=0):
    """The FP64 oracle on the host cores, on a bounded sample of whole BY groups
    of the same workload: groups in a seeded random order, taken while the
    estimated oracle time stays within `target_seconds` (groups whose estimate
    alone exceeds half of it are passed over).  A group's oracle time has two
    parts, its frame distances and DTW (squared frame count times dim) and its
    triplet comparisons; a probe on the smallest groups gives the time per unit
    of each, each charged with the whole probe time, and a group's estimate is
    the larger of the two, so big groups are not underestimated.  The triplets
    per group come from a host-only task of the library (no device work).  Only
    the sampled groups' items are handed to the oracle."""
    by = list(w.by)
    keys = [tuple(r) for r in w.attrs[:, by].tolist()] if by else [()] * w.n_items
    lens = np.diff(w.offsets)
    members, frames = {}, {}
    for i, k in enumerate(keys):
        members.setdefault(k, []).append(i)
        frames[k] = frames.get(k, 0) + int(lens[i])
    groups = sorted(members)
    cost = {g: float(frames[g]) ** 2 * w.dim for g in groups}
    host = fx.Task(fx.Dataset(fx.Context(-1), None, w.offsets, w.attrs), w.on, w.by, w.across)
    ckeys, (nt, _) = host.keys, host.sizes
    trip = {g: 0.0 for g in groups}
    for row, n in zip(ckeys[:, 2:2 + len(by)].tolist(), nt.tolist()):
        trip[tuple(row)] += float(n)
    del host

    def run(take):
        items = np.concatenate([np.asarray(members[g], np.int64) for g in take])
        sub = w.subset_items(np.sort(items))
        feats = sub.features_f32_host()
        t0 = time.perf_counter()
        r = oracle.score(feats, sub.offsets, sub.attrs, sub.on, sub.by, sub.across)
        return r, time.perf_counter() - t0

    # the probe: the smallest groups, doubled until a run takes half a second
    # (or until the next doubling is estimated, at the current rates, to take
    # more than a few seconds: the larger groups come last)
    by_cost = sorted(groups, key=lambda g: cost[g])
    n_probe = 64
    while True:
        probe = by_cost[:n_probe]
        r, dt = run(probe)
        rate_d = dt / sum(cost[g] for g in probe)                  # seconds per distance-cost unit
        rate_t = dt / max(sum(trip[g] for g in probe), 1.0)        # seconds per triplet
        if dt >= 0.5 or n_probe >= len(by_cost):
            break
        nxt = by_cost[:2 * n_probe]
        if sum(max(cost[g] * rate_d, trip[g] * rate_t) for g in nxt) > 4.0:
            break
        n_probe *= 2
    est_of = {g: max(cost[g] * rate_d, trip[g] * rate_t) for g in groups}
    log(f"cpu baseline: probe of {len(probe)} small groups took {dt:.2f} s")
    order = [groups[k] for k in np.random.default_rng(seed).permutation(len(groups))]

    def select(scale):
        take, est = [], 0.0
        for g in order:
            e = est_of[g] * scale
            if e > 0.5 * target_seconds:
                continue
            if est + e > target_seconds:
                break
            take.append(g)
            est += e
        return take, est

    take, est = select(1.0)
    r, dt = run(take)
    log(f"cpu baseline: {len(take)} groups took {dt:.1f} s (estimated {est:.1f} s)")
    # the estimates charge each part with the whole probe time, so they run
    # high; when the sample took well under the target, scale them by what it
    # took and draw the sample again (same order; groups passed over as too
    # large may now fit)
    scale = 1.0
    for _ in range(3):
        if est <= 0 or dt >= 0.4 * target_seconds:
            break
        scale *= max(dt / est, 0.05)
        take2, est2 = select(scale)
        if take2 == take:
            break
        take, est = take2, est2
        r, dt = run(take)
        log(f"cpu baseline: rescaled by {scale:.4f}: {len(take)} groups took {dt:.1f} s "
            f"(estimated {est:.1f} s)")
    n_trip = int(r.n_triplets.sum())
    model, ncpu = cpu_info()
    whole_s = sum(est_of.values()) * scale
    return {"value": n_trip / dt, "unit": "triplets/s", "cores": oracle.num_threads(), "kind": "oracle",
            "cpu_model": model, "nproc": ncpu,
            "sample": f"{len(take)} of {len(groups)} BY groups in seeded random order ({len(r.cells)} cells, "
                      f"{n_trip} triplets) of the same workload, FP64 DTW + scoring, {dt:.1f} s; the whole "
                      f"workload would take about {whole_s:.0f} s by the rescaled estimate"}


FUSED_SOURCES = ("paper_2505_02692_amd/csrc/k_fused.hip", "paper_2505_02692_amd/csrc/device_common.h")


def fused_source_hash():
    """SHA-256 prefix of the fused kernel's sources (the kernel file and the
    device helpers it includes), the key of its committed byte counts."""
    import hashlib
    root = os.path.dirname(os.path.abspath(__file__))
    h = hashlib.sha256()
    for f in FUSED_SOURCES:
        with open(os.path.join(root, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def committed_traffic(profile_file, cols, blocks_per_cu):
    """HBM bytes per launch of the dominant kernel in the configuration that ran,
    from the committed rocprofv3 byte-counter summary, used only while the kernel
    sources are the ones that were measured (their SHA-256 prefix is recorded
    beside the figure)."""
    root = os.path.dirname(os.path.abspath(__file__))
    try:
        lines = open(os.path.join(root, profile_file)).read().splitlines()
        want = {"source_sha256": fused_source_hash(),
                "kernel": f"k_fused<{cols},true>", "blocks_per_cu": str(blocks_per_cu)}
    except OSError:
        return None
    for line in lines:
        f = line.strip().strip("`").split()
        if not f or f[0] != "traffic":
            continue
        kv = dict(x.split("=", 1) for x in f[1:] if "=" in x)
        if all(kv.get(k) == v for k, v in want.items()):
            return float(kv["bytes_per_launch"])
    return None


def roofline(w, mode, st0, pstats, profile_file):
    """Roofline of the dominant kernel of the timed steps (HIP-event stage
    times on the stream the kernels run on)."""
    dim, dim_pad = w.dim, (w.dim + 63) // 64 * 64
    nf = st0["n_frames"]
    in_bytes = w.features.element_size()
    rows = nf if mode == "dtw" else st0["n_items"]
    norm_bytes = (nf * dim * in_bytes) + rows * dim_pad * 2 + rows * 4
    # DTW: the frame pairs of the unordered item pairs the cells need (the DTW
    # distance is symmetric, so each pair's DTW is needed once)
    dist_flops = 2.0 * dim * (st0["dtw_cells_sym"] if mode == "dtw" else st0["n_pairs"])
    pk = {k: float(np.mean([s_[k] for s_ in pstats])) for k in ("ms_normalize", "ms_distance", "ms_triplets")}
    if pk["ms_normalize"] >= max(pk["ms_distance"], pk["ms_triplets"]):
        ach = norm_bytes / (pk["ms_normalize"] / 1e3) / 1e9
        return {"kernel": "k_normalize", "bound": "hbm", "achieved": ach, "peak": HBM_PEAK_GBS,
                "unit": "GB/s", "frac": ach / HBM_PEAK_GBS, "traffic": None,
                "algorithmic_bytes_per_launch": norm_bytes, "ms_per_launch": pk["ms_normalize"]}
    if pk["ms_triplets"] > pk["ms_distance"]:
        return {"kernel": "k_triplets_sorted", "bound": "alu", "ms_per_launch": pk["ms_triplets"],
                "achieved": None, "peak": None, "unit": None, "frac": None, "traffic": None}
    ach = dist_flops / (pk["ms_distance"] / 1e3) / 1e12
    traffic = (committed_traffic(profile_file, st0["fused_cols"], st0["fused_blocks_per_cu"])
               if (mode == "dtw" and profile_file) else None)
    return {"kernel": "k_fused" if mode == "dtw" else "k_gram_angular_bf16", "bound": "mfma",
            "achieved": ach, "peak": MFMA_BF16_PEAK_TFLOPS,
            "unit": "TFLOP/s", "frac": ach / MFMA_BF16_PEAK_TFLOPS, "traffic": traffic,
            "algorithmic_flops_per_launch": dist_flops, "ms_per_launch": pk["ms_distance"]}


def within_c2_legs(fx, ctx, workloads, sync, args):
    """Secondary legs on the within-speaker triphone workload (100k items, dim
    768): BF16 form, plain FP32 form, Euclidean FP32 form, and the BF16 form on
    a harder variant (centroid std 0.1, ABX error about 8%) whose near ties go
    to the FP64 recheck.  200 timed steps for the BF16 leg (a step takes about
    1.4 ms), 20 for the others."""
    out = {}
    for name, cstd, steps in (("c2", 1.0, 200), ("c2_hard", 0.1, 20)):
        w = workloads.within_c2(device="cuda", centroid_std=cstd)
        ds = fx.Dataset(ctx, w.features, w.offsets, w.attrs)
        ms, pst, errs = pipelined_leg(fx, ds, w, "bf16", steps, 3, sync, "dtw", args)
        st = pst[-1]
        n_trip = st["n_triplets"]
        leg = {"triplets_per_s": n_trip / (ms / 1e3), "ms_per_step": ms,
               "gpu_ms_pipelined": float(np.median([s_["ms_total"] for s_ in pst])),
               "k_fused_ms": float(np.mean([s_["ms_distance"] for s_ in pst])),
               "gcups": st["dtw_cells_sym"] / (ms / 1e3) / 1e9, "abx_error": errs[-1],
               "recheck_pairs": st["n_recheck_pairs"], "recount_rows": st["n_recount_rows"],
               "nonrobust_pairs": st["n_nonrobust_pairs"], "ms_recheck": float(np.mean([s_["ms_recheck"] for s_ in pst])),
               "cells": st["n_cells"], "triplets": n_trip}
        log(f"{name} bf16: {ms:.3f} ms/step, {leg}")
        if name == "c2" and not args.no_plain:
            pms, pst2, perr = pipelined_leg(fx, ds, w, "fp32", 20, 1, sync, "dtw", args)
            leg["plain_fp32"] = {"triplets_per_s": n_trip / (pms / 1e3), "ms_per_step": pms,
                                 "gpu_ms_pipelined": float(np.median([s_["ms_total"] for s_ in pst2])),
                                 "gcups": st["dtw_cells_sym"] / (pms / 1e3) / 1e9, "abx_error": perr[-1]}
            ems, est, eerr = pipelined_leg(fx, ds, w, "fp32", 20, 1, sync, "dtw", args, distance="euclidean")
            leg["euclidean_fp32"] = {"triplets_per_s": n_trip / (ems / 1e3), "ms_per_step": ems,
                                     "gpu_ms_pipelined": float(np.median([s_["ms_total"] for s_ in est])),
                                     "abx_error": eerr[-1]}
            log(f"c2 plain fp32: {pms:.2f} ms/step; euclidean fp32: {ems:.2f} ms/step")
        out[name] = leg
        del ds, w
    return out


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None,
                    help="timed steps of the main leg (default: 20, or 200 for c2)")
    ap.add_argument("--warmup", type=int, default=None, help="untimed steps (default: 3, or 10 for c2)")
    ap.add_argument("--workload", choices=sorted(WORKLOADS), default="c4",
                    help="main leg: c4 (default) is the headline workload; the others profile one leg alone")
    ap.add_argument("--serve-jobs", type=int, default=400)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--no-plain", action="store_true")
    ap.add_argument("--no-secondary", action="store_true", help="skip the pooled and within-speaker legs")
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
                    help="let the second host thread's work use the shared host thread pool (the default "
                         "for tasks of a million cells or more)")
    ap.add_argument("--copy-calibration-mib", type=int, default=0,
                    help="also run 3 plain device copies of this many MiB (to scale HBM byte counters)")
    ap.add_argument("--stream-probe-mib", type=int, default=0,
                    help="also run the HBM streaming probe (the normalise kernel's access pattern, FP32 -> BF16, "
                         "dim 768) over this many MiB of FP32 rows, three times, and log its bandwidth")
    args = ap.parse_args()
    c2_main = args.workload == "c2"
    if args.steps is None:
        args.steps = 200 if c2_main else 20
    if args.warmup is None:
        args.warmup = 10 if c2_main else 3
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
    ctx = fx.Context(0)
    if args.serving_only:
        print(json.dumps({"serving": serving_stream(fx, ctx, torch, workloads, args.serve_jobs)}))
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
    if args.stream_probe_mib > 0:
        rows = (args.stream_probe_mib << 20) // (768 * 4)
        src = torch.randn(rows, 768, device="cuda")
        dst = torch.empty(rows, 768, device="cuda", dtype=torch.bfloat16)
        ev = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
        ev[0].record()
        for k in range(3):
            fx.fabx_probe_stream(src, dst)
            ev[k + 1].record()
        sync()
        nbytes = rows * 768 * (4 + 2)
        for k in range(3):
            ms = ev[k].elapsed_time(ev[k + 1])
            log(f"stream probe: {rows} rows x 768, {nbytes / 1e9:.2f} GB moved in {ms:.3f} ms = "
                f"{nbytes / ms / 1e6:.0f} GB/s")
        assert torch.equal(dst, src.to(torch.bfloat16))
        del src, dst
    gen_name, mode, wl_desc = WORKLOADS[args.workload]
    headline = args.workload == "c4"
    t_gen = time.perf_counter()
    w = getattr(workloads, gen_name)(device="cuda", **WORKLOAD_KW.get(args.workload, {}))
    ds = fx.Dataset(ctx, w.features, w.offsets, w.attrs)
    sync()
    log(f"workload {args.workload} ready in {time.perf_counter() - t_gen:.1f} s: {w.n_items} items, "
        f"{w.n_frames} frames, dim {w.dim}")

    if args.fused_config:
        cols, bpc = (int(v) for v in args.fused_config.split(","))
        SCORE_KW.update(fused_cols=cols, fused_blocks_per_cu=bpc)
    # untimed: warm-up steps, then pick the fused kernel's tiles / grid for this task shape
    _, wst, _ = run_pipelined(fx, ds, w, "bf16", args.warmup, sync, mode, args.side, not args.side_pool,
                              args.depth)
    sync()
    # the second thread's host work (score set-up, collapse) runs in place,
    # single-threaded, so that it never takes the pool from the next build;
    # a task of a million cells or more has a collapse that needs the pool
    side_serial = not args.side_pool and (not wst or wst[-1]["n_cells"] < 1_000_000)
    log(f"warmup done; second thread's host work {'in place' if side_serial else 'on the pool'}")
    tune = (fx.Task(ds, w.on, w.by, w.across).autotune(mode=mode)
            if not (args.no_autotune or args.fused_config) else None)
    log(f"autotune: {tune}")
    dt, pstats, errs = run_pipelined(fx, ds, w, "bf16", args.steps, sync, mode, args.side, side_serial,
                                     args.depth)
    ms_step = dt / args.steps * 1e3
    log(f"bf16 form, pipelined: {ms_step:.2f} ms/step")
    # a few of the same steps one after another, for the per-stage breakdown
    n_serial = min(args.steps, 200 if c2_main else 3)
    sdt, stats, serrs = run_steps(fx, ds, w, "bf16", n_serial, sync, mode)
    ms_step_serial = sdt / n_serial * 1e3
    stages = _stage_means(stats)
    log(f"bf16 form, serial: {ms_step_serial:.2f} ms/step, stages {stages}")
    assert errs[-1] == serrs[-1]
    st0 = stats[-1]
    log(f"task: {st0['n_items']} items in cells, {st0['n_frames']} frames packed; fused kernel "
        f"k_fused<{st0['fused_cols']},...> blocks_per_cu={st0['fused_blocks_per_cu']}, "
        f"sources sha256 {fused_source_hash()}")
    n_trip = st0["n_triplets"]
    value = n_trip / (ms_step / 1e3)
    t_build = []
    for _ in range(3):
        t0 = time.perf_counter()
        fx.Task(ds, w.on, w.by, w.across)
        t_build.append((time.perf_counter() - t0) * 1e3)
    roof = roofline(w, mode, st0, pstats, "profiles/hbm_bytes_batched_c4.md" if headline else None)

    # the plain FP32 form on the same data (one step on the headline workload,
    # whose plain step takes tens of seconds)
    plain = None
    if not args.no_plain:
        n_plain = 1 if headline else args.steps
        pdt, pstats_p, perrs = run_steps(fx, ds, w, "fp32", n_plain, sync, mode)
        pms = pdt / n_plain * 1e3
        pst = _stage_means(pstats_p)
        plain = {"triplets_per_s": n_trip / (pms / 1e3), "ms_per_step": pms, "steps": n_plain,
                 "gcups": (st0["dtw_cells_sym"] / (pms / 1e3) / 1e9) if mode == "dtw" else None,
                 "gpu_ms": pst["ms_total"], "gpu_triplets_per_s": n_trip / (pst["ms_total"] / 1e3),
                 "abx_error": perrs[-1], "abx_error_minus_bf16": perrs[-1] - errs[-1], "stages_ms": pst}
        log(f"fp32 form: {pms:.1f} ms/step, stages {pst}, error {perrs[-1]} vs bf16 {errs[-1]}")

    pooled = None
    if headline and not args.no_secondary:
        pooled = {}
        for prec in ("bf16", "fp32"):
            ms, pst, perr = pipelined_leg(fx, ds, w, prec, 20, 2, sync, "pooled", args)
            sp = pst[-1]
            pooled[prec] = {"triplets_per_s": sp["n_triplets"] / (ms / 1e3), "ms_per_step": ms,
                            "gpu_ms_pipelined": float(np.median([s_["ms_total"] for s_ in pst])),
                            "ms_distance": float(np.mean([s_["ms_distance"] for s_ in pst])),
                            "ms_triplets": float(np.mean([s_["ms_triplets"] for s_ in pst])),
                            "abx_error": perr[-1], "pairs": sp["n_pairs"]}
            log(f"pooled {prec}: {pooled[prec]}")

    cpu = None
    if not args.no_cpu_baseline:
        import oracle
        cpu = cpu_baseline(oracle, fx, w)
        log(f"cpu baseline: {cpu}")
    wl_cfg = {"workload": wl_desc, "cells": st0["n_cells"], "triplets": n_trip,
              "dtw_cells": st0["dtw_cells"], "dtw_cells_unordered": st0["dtw_cells_sym"],
              "items": w.n_items, "frames": w.n_frames, "items_in_cells": st0["n_items"],
              "frames_packed": st0["n_frames"], "dim": w.dim, "parallelism": "single GPU"}
    del ds, w

    # each further leg runs on a context of its own: a context keeps the device
    # memory its scores used in a pool until it is destroyed
    del ctx
    import gc
    gc.collect()
    torch.cuda.empty_cache()

    secondary = None
    if headline and not args.no_secondary:
        secondary = within_c2_legs(fx, fx.Context(0), workloads, sync, args)
        gc.collect()
        torch.cuda.empty_cache()

    serving = None
    if args.serve_jobs > 0 and headline:
        serving = serving_stream(fx, fx.Context(0), torch, workloads, args.serve_jobs)
        log(f"serving: {serving}")

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
        "gpu_ms_pipelined": float(np.median([s_["ms_total"] for s_ in pstats])) if pstats else None,
        "triplets_per_s_serial": n_trip / (ms_step_serial / 1e3),
        "pipelined": ("host work of neighbouring steps overlaps device work (fabx_score_async)"
                      + {"launch": f"; the main thread builds up to {args.depth} steps ahead while a second "
                                   f"host thread launches step i and collapses step i - {args.depth} "
                                   f"({args.depth} scores stay enqueued on the device)",
                         "collapse": "; the collapse of step i - 1 runs on a second host thread beside "
                                     "the build of step i + 1",
                         "none": ""}[args.side]),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "bf16",
        "data": "synthetic (seeded Gaussian SSL-like features: label centroid + group offset + frame noise)",
        "config": wl_cfg,
        "gcups": (st0["dtw_cells_sym"] / (ms_step / 1e3) / 1e9) if mode == "dtw" else None,
        "gpu_ms": stages["ms_total"],
        "gpu_triplets_per_s": n_trip / (stages["ms_total"] / 1e3),
        "task_build_ms": float(np.median(t_build)),
        "stages_ms": stages,
        "abx_error": errs[-1],
        "recheck_pairs": st0["n_recheck_pairs"], "nonrobust_pairs": st0["n_nonrobust_pairs"],
        "plain_fp32": plain,
        "chosen_vs_plain": (value / plain["triplets_per_s"]) if plain else None,
        "pooled": pooled,
        "within_speaker": secondary,
        "autotune": tune,
        "fused_config": {"cols": st0["fused_cols"], "blocks_per_cu": st0["fused_blocks_per_cu"]},
        "roofline": roof,
        "serving": serving,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
