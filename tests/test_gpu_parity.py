"""GPU parity: the HIP path (through the C ABI) against the FP64 oracle.

Bars:
* BF16 + FP64-recheck form: per-cell half-unit counts W equal the oracle's
  exactly (near ties are re-decided in FP64), hence identical ABX error.
* plain FP32 form: ABX error within 1e-4 absolute of the oracle, per-cell
  mismatches reported (rare near-tie flips are expected).
* per-pair distances: FP32 within 2e-6, BF16 (robust pairs) within the
  stated margin / 3, FP64-rechecked pairs within 1e-12 of the oracle.
"""
import os
import sys
import time

import numpy as np
import pytest
import torch

import oracle
import workloads
import paper_2505_02692_amd as fx
from paper_2505_02692_amd import _lib as L

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[case] {msg}", flush=True)
    sys.stdout.flush()


_CTX = {}


def ctx():
    if "c" not in _CTX:
        _CTX["c"] = fx.Context(0)
    return _CTX["c"]


def gpu_score(w, **kw):
    feats = w.features.to("cuda").contiguous()
    ds = fx.Dataset(ctx(), feats, w.offsets, w.attrs)
    t = fx.Task(ds, w.on, w.by, w.across)
    res = t.score(**kw)
    torch.cuda.synchronize()
    return t, res


def oracle_score(w, mode="dtw", norm="path"):
    return oracle.score(w.features_f32_host(), w.offsets, w.attrs, w.on, w.by, w.across, mode, norm)


def all_oracle_pairs(orc):
    xs, ys, vs = [], [], []
    for items, M in orc.groups.values():
        i, j = np.nonzero(~np.isnan(M))
        xs.append(items[i])
        ys.append(items[j])
        vs.append(M[i, j])
    return np.concatenate(xs), np.concatenate(ys), np.concatenate(vs)


def check(w, mode="dtw", precision="bf16", norm="path", exact=None, pair_tol=None, levels=True, **kw):
    _say(f"{w.name} n_items={w.n_items} dim={w.dim} mode={mode} precision={precision} norm={norm} {kw}")
    t, res = gpu_score(w, mode=mode, precision=precision, norm=norm, keep_pairs=True, **kw)
    orc = oracle_score(w, mode, norm)
    assert np.array_equal(t.keys, orc.keys.astype(np.int32))
    nt, _ = t.sizes
    assert np.array_equal(nt, orc.n_triplets)
    exact = (precision == "bf16") if exact is None else exact
    mism = int(np.count_nonzero(res.half_units != orc.half_units))
    e_gpu, e_orc = res.collapse(), oracle.error_rate(orc)
    xs, ys, want = all_oracle_pairs(orc)
    f32, fl, f64 = res.pairs(xs, ys)
    err = np.abs(f32.astype(np.float64) - want)
    robust = (fl & 1) == 0
    st = res.stats
    print(f"  cells={st['n_cells']} triplets={st['n_triplets']} pairs={len(want)} mism={mism} "
          f"max_pair_err={err[robust].max():.3g} p99={np.quantile(err[robust], 0.99):.3g} "
          f"margin={st['margin']:.3g} delta={st['delta']:.3g} "
          f"nonrobust={st['n_nonrobust_pairs']} recheck={st['n_recheck_pairs']} "
          f"recount={st['n_recount_rows']} err={e_gpu:.6f} oracle_err={e_orc:.6f}", flush=True)
    if exact:
        assert mism == 0, f"{mism} cells differ"
    assert abs(e_gpu - e_orc) <= (1e-12 if exact else 1e-4)
    if levels and w.levels:
        lg, lo = res.collapse(w.levels), oracle.error_rate(orc, w.levels)
        assert abs(lg - lo) <= (1e-12 if exact else 1e-4)
    if pair_tol is None:
        # BF16: the recheck argument needs every robust pair within margin / 2
        pair_tol = 2e-6 if precision == "fp32" else st["margin"] / 2
    assert err[robust].max() <= pair_tol, f"max pair error {err[robust].max()}"
    rechecked = (fl & 2) != 0
    if rechecked.any():
        assert np.abs(f64[rechecked] - want[rechecked]).max() <= 1e-12
    return t, res, orc


# ------------------------------------------------------------------ C1 --

def test_c1_plain_fp32():
    check(workloads.plain_c1(), precision="fp32", exact=True)


def test_c1_bf16():
    check(workloads.plain_c1())


def test_c1_hard_bf16_exact():
    check(workloads.plain_c1(centroid_std=0.15))


def test_c1_hard_fp32():
    check(workloads.plain_c1(centroid_std=0.15), precision="fp32")


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_c1_hard_raw_cost(precision):
    check(workloads.plain_c1(centroid_std=0.15, seed=5), precision=precision, norm="none",
          pair_tol=(2e-5 if precision == "fp32" else 3e-3))


# ------------------------------------------- C2 / C3 / C4 shaped, reduced --

def test_within_c2_shape_bf16():
    check(workloads.within_c2(n_items=4000, centroid_std=0.1))


def test_within_c2_shape_fp32():
    check(workloads.within_c2(n_items=4000, centroid_std=0.1), precision="fp32")


def test_across_c3_shape_bf16():
    check(workloads.across_c3(n_items=4000, centroid_std=0.1))


def test_across_c3_shape_fp32():
    check(workloads.across_c3(n_items=3000, centroid_std=0.1), precision="fp32")


def test_batched_c4_shape_bf16():
    # groups up to 150 items x up to 60 frames: many row / column blocks per group
    check(workloads.batched_c4(n_groups=24, size_hi=150, centroid_std=0.3, seed=11))


def test_batched_c4_shape_fp32():
    check(workloads.batched_c4(n_groups=12, size_hi=90, centroid_std=0.3, seed=12), precision="fp32")


# ---------------------------------------------------------------- pooled --

@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_pooled_within(precision):
    check(workloads.within_c2(n_items=4000, dim=512, centroid_std=0.05), mode="pooled",
          precision=precision)


@pytest.mark.parametrize("precision", ["fp32", "bf16"])
def test_pooled_c4_shape(precision):
    check(workloads.batched_c4(n_groups=30, size_hi=400, centroid_std=0.2, seed=13), mode="pooled",
          precision=precision)


# ------------------------------------------------------------ edge cases --

@pytest.mark.parametrize("dim", [2, 33, 100, 130])
def test_odd_dims(dim):
    check(workloads.plain_c1(dim=dim, centroid_std=0.3, seed=dim))


def test_single_frame_items_and_long_items():
    w = workloads.batched_c4(n_groups=10, size_hi=70, len_lo=1, len_hi=64, dim=64, centroid_std=0.3,
                             seed=21)
    check(w)
    w1 = workloads.batched_c4(n_groups=10, size_hi=70, len_lo=1, len_hi=1, dim=64, centroid_std=0.3,
                              seed=22)
    check(w1)
    check(w1, precision="fp32")


# Items of more than 64 frames (up to FABX_MAX_ITEM_FRAMES): in the BF16 form
# every pair with such an item is computed in FP64 (tiled DTW, rows in chunks
# of 64 handing their last row to the next chunk), so its FP32 copy is the
# FP64 value rounded once; the plain FP32 form runs its DTW in row chunks.
@pytest.mark.parametrize("precision,norm", [("bf16", "path"), ("bf16", "none"), ("fp32", "path"),
                                            ("fp32", "none")])
def test_long_items_match_oracle(precision, norm):
    w = workloads.batched_c4(n_groups=10, size_lo=5, size_hi=16, len_lo=1, len_hi=200, dim=64,
                             centroid_std=0.3, seed=31)
    lens = np.diff(w.offsets)
    assert (lens > 64).sum() >= 10 and (lens <= 64).sum() >= 10 and lens.max() > 128
    tol = {("fp32", "path"): 2e-5, ("fp32", "none"): 2e-3}.get((precision, norm))
    t, res, orc = check(w, precision=precision, norm=norm, pair_tol=tol)
    xs, ys, want = all_oracle_pairs(orc)
    f32, fl, _ = res.pairs(xs, ys)
    long_pair = (lens[xs] > 64) | (lens[ys] > 64)
    assert long_pair.sum() > 100
    if precision == "bf16":
        # FP64 values rounded once to FP32, and never flagged non-robust
        err = np.abs(f32[long_pair].astype(np.float64) - want[long_pair])
        assert err.max() <= 2.0 ** -23 * np.maximum(np.abs(want[long_pair]), 1.0).max()
        assert not (fl[long_pair] & 1).any()


def test_long_items_at_the_limit_and_beyond():
    """An item of exactly FABX_MAX_ITEM_FRAMES frames (16 row chunks) scores like
    the oracle; one frame more is EINVAL."""
    _say("items of FABX_MAX_ITEM_FRAMES frames")
    rng = np.random.default_rng(41)
    lens = np.array([L.FABX_MAX_ITEM_FRAMES, 3, 70, 1, L.FABX_MAX_ITEM_FRAMES - 1, 20], np.int64)
    dim = 16
    cent = rng.standard_normal((2, dim))
    label = np.array([0, 1, 0, 1, 0, 1], np.int32)
    frames = [cent[l] + 0.8 * rng.standard_normal((n, dim)) for l, n in zip(label, lens)]
    feats = torch.tensor(np.concatenate(frames).astype(np.float32))
    off = np.zeros(len(lens) + 1, np.int64)
    off[1:] = np.cumsum(lens)
    attrs = np.stack([label, np.zeros(6, np.int32)], axis=1)
    w = workloads.Workload("long-limit", feats, off, attrs, ["label", "ctx"], 0, [1], [])
    for precision in ("bf16", "fp32"):
        check(w, precision=precision, pair_tol=(2e-5 if precision == "fp32" else None), levels=False)
    lens2 = lens.copy()
    lens2[0] += 1
    frames[0] = np.concatenate([frames[0], frames[0][:1]])
    off2 = np.zeros(len(lens2) + 1, np.int64)
    off2[1:] = np.cumsum(lens2)
    w2 = workloads.Workload("too-long", torch.tensor(np.concatenate(frames).astype(np.float32)), off2, attrs,
                            ["label", "ctx"], 0, [1], [])
    with pytest.raises(fx.FabxError) as e:
        gpu_score(w2)
    assert e.value.code == L.FABX_EINVAL


def test_exact_copies_tie_at_one_half():
    _say("exact copies")
    rng = np.random.default_rng(3)
    a = rng.standard_normal((7, 40)).astype(np.float32)
    xs = [rng.standard_normal((int(rng.integers(2, 9)), 40)).astype(np.float32) for _ in range(4)]
    frames = [a, a.copy()] + xs
    feats = torch.tensor(np.concatenate(frames))
    off = np.zeros(len(frames) + 1, np.int64)
    off[1:] = np.cumsum([len(f) for f in frames])
    attrs = np.array([[0, 0], [1, 0], [0, 1], [0, 1], [0, 1], [0, 1]], np.int32)
    w = workloads.Workload("copies", feats, off, attrs, ["label", "spk"], 0, [], [1])
    for precision in ("fp32", "bf16"):
        t, res = gpu_score(w, precision=precision)
        k = [tuple(r) for r in t.keys].index((0, 1, 0, 1))
        assert res.half_units[k] == res.n_triplets[k] == 4


def test_zero_norm_frame_is_edomain():
    _say("zero-norm frame / mean")
    w = workloads.plain_c1(dim=16)
    feats = w.features.clone()
    feats[int(w.offsets[5]) + 1] = 0.0                       # one zero frame: DTW mode fails
    w.features = feats
    for precision in ("fp32", "bf16"):
        with pytest.raises(fx.FabxError) as e:
            gpu_score(w, mode="dtw", precision=precision)
        assert e.value.code == L.FABX_EDOMAIN
    feats = w.features.clone()
    feats[int(w.offsets[7]):int(w.offsets[8])] = 0.0         # a whole item zero: its mean is zero
    w.features = feats
    with pytest.raises(fx.FabxError) as e:
        gpu_score(w, mode="pooled", precision="bf16")
    assert e.value.code == L.FABX_EDOMAIN


def test_empty_task_scores():
    _say("empty task")
    w = workloads.plain_c1(dim=8)
    w.attrs = np.zeros_like(w.attrs)        # one ON value: no cell
    t, res = gpu_score(w)
    assert len(t) == 0 and res.half_units.size == 0
    with pytest.raises(fx.FabxError):
        res.collapse()


def test_collapse_level_errors():
    _say("collapse levels")
    w = workloads.within_c2(n_items=1500, dim=64, centroid_std=0.1)
    t, res = gpu_score(w, precision="fp32")
    with pytest.raises(fx.FabxError):
        res.collapse([[0]])                  # the ON attribute
    with pytest.raises(fx.FabxError):
        res.collapse([[9]])


def test_repeat_is_bitwise_deterministic():
    _say("determinism")
    w = workloads.within_c2(n_items=3000, dim=256, centroid_std=0.08, seed=31)
    feats = w.features.to("cuda")
    ds = fx.Dataset(ctx(), feats, w.offsets, w.attrs)
    t = fx.Task(ds, w.on, w.by, w.across)
    r1 = t.score(keep_pairs=True)
    r2 = t.score(keep_pairs=True)
    r3 = fx.Task(ds, w.on, w.by, w.across).score(keep_pairs=True)
    assert np.array_equal(r1.half_units, r2.half_units) and np.array_equal(r1.half_units, r3.half_units)
    # pair distances of the first group, bitwise
    keys = t.keys
    g = tuple(keys[0][2:])
    items = np.nonzero(np.all(w.attrs[:, w.by] == np.array(g), axis=1))[0]
    xs, ys = np.repeat(items, len(items)), np.tile(items, len(items))
    a, b, c = r1.pairs(xs, ys), r2.pairs(xs, ys), r3.pairs(xs, ys)
    assert all(np.array_equal(u, v) for u, v in zip(a, b)) and all(np.array_equal(u, v) for u, v in zip(a, c))
    assert r1.stats["ms_total"] > 0


# ---------------------------------------------------------------- server --

def test_server_alone_equals_mix():
    _say("server alone vs mix")
    jobs = [workloads.serving_job(j, n_items=int(n), dim=d, across=a, centroid_std=0.1)
            for j, (n, d, a) in enumerate([(1200, 256, False), (2500, 512, True), (800, 1280, False),
                                           (3000, 768, True), (1500, 1024, False)])]
    dsets = []
    alone = []
    for w in jobs:
        feats = w.features.to("cuda")
        ds = fx.Dataset(ctx(), feats, w.offsets, w.attrs)
        dsets.append((ds, w))
        t = fx.Task(ds, w.on, w.by, w.across)
        r = t.score()
        alone.append((t.keys.copy(), r.half_units.copy()))
    srv = fx.Server(ctx(), hbm_budget_bytes=8 << 30, n_streams=3)
    ids = [srv.submit(ds, w.on, w.by, w.across) for ds, w in dsets]
    for (keys, W), jid in zip(alone, ids):
        k2, w2, n2, s2 = srv.wait(jid)
        assert np.array_equal(keys, k2) and np.array_equal(W, w2)
    st = srv.stats
    assert st["completed"] == len(jobs) and st["failed"] == 0
    assert st["hbm_high_water"] <= 8 << 30
    srv.close()


def test_server_mix_of_bench_jobs():
    """The serving stream's job mix (items capped at 6k): alone twice, then served on
    4 streams; every job's per-cell counts must agree bitwise, and disagreeing
    groups are checked against the oracle."""
    _say("server: bench job mix")
    jobs = []
    for j in range(12):
        w = workloads.serving_job(j, device="cuda", n_hi=6000)
        jobs.append((w, fx.Dataset(ctx(), w.features, w.offsets, w.attrs)))
    runs = []
    for rep in range(2):
        out = []
        for w, ds in jobs:
            r = fx.Task(ds, w.on, w.by, w.across).score()
            st = r.stats
            if rep == 0:
                print(f"  {w.name} n={w.n_items} dim={w.dim} cells={st['n_cells']} gpu={st['ms_total']:.1f}ms "
                      f"nonrobust={st['n_nonrobust_pairs']} recheck={st['n_recheck_pairs']} "
                      f"recount={st['n_recount_rows']}", flush=True)
            out.append(r.half_units.copy())
        runs.append(out)
    srv = fx.Server(ctx(), hbm_budget_bytes=64 << 30, n_streams=4)
    ids = [srv.submit(ds, w.on, w.by, w.across) for w, ds in jobs]
    served = [srv.wait(i)[1] for i in ids]
    srv.close()
    bad = []
    for k, (w, ds) in enumerate(jobs):
        d_rep = int(np.count_nonzero(runs[0][k] != runs[1][k]))
        d_srv = int(np.count_nonzero(runs[0][k] != served[k]))
        if d_rep or d_srv:
            print(f"  MISMATCH {w.name}: alone-vs-alone {d_rep} cells, alone-vs-served {d_srv} cells", flush=True)
            bad.append(k)
    for k in bad[:2]:
        w, ds = jobs[k]
        t = fx.Task(ds, w.on, w.by, w.across)
        keys = t.keys
        diff = np.nonzero((runs[0][k] != served[k]) | (runs[0][k] != runs[1][k]))[0][:5]
        gkeys = {tuple(int(v) for v in keys[c][2:2 + len(w.by)]) for c in diff}
        orc = oracle.score(w.features_f32_host(), w.offsets, w.attrs, w.on, w.by, w.across,
                           cell_filter=lambda c: c.by_key in gkeys)
        okeys = {tuple(int(v) for v in c.key): int(h) for c, h in zip(orc.cells, orc.half_units)}
        for c in diff:
            kk = tuple(int(v) for v in keys[c])
            print(f"  cell {kk}: alone {runs[0][k][c]} {runs[1][k][c]} served {served[k][c]} "
                  f"oracle {okeys.get(kk)}", flush=True)
    assert not bad


def test_server_rejects_oversized_job():
    _say("server admission")
    w = workloads.serving_job(0, n_items=2000, dim=256, across=False)
    ds = fx.Dataset(ctx(), w.features.to("cuda"), w.offsets, w.attrs)
    srv = fx.Server(ctx(), hbm_budget_bytes=1 << 20, n_streams=1)
    with pytest.raises(fx.FabxError) as e:
        srv.submit(ds, w.on, w.by, w.across)
    assert e.value.code == -2
    srv.close()


# ------------------------------------------- large cells: sorted rows --

def _big_cells(seed, centroid_std=0.3, dim=32):
    # groups of 200-800 items, two labels each: |A| x |B| per x well above the
    # brute-force budget, so every cell is counted from sorted rows
    return workloads.batched_c4(n_groups=8, size_lo=200, size_hi=800, len_lo=1, len_hi=8, dim=dim,
                                centroid_std=centroid_std, seed=seed)


@pytest.mark.parametrize("precision", ["bf16", "fp32"])
def test_large_cells_sorted_rows(precision):
    w = _big_cells(71, centroid_std=0.05)            # close labels: many near ties
    t, res, orc = check(w, precision=precision)
    assert min(len(c.A) * len(c.B) for c in orc.cells) >= 8192


def test_large_cells_sorted_rows_pooled():
    check(_big_cells(72, centroid_std=0.05), mode="pooled")


def test_large_cells_many_exact_ties():
    """Every item of a group repeats the first item's frames (cut or extended to
    its own length): pairs of equal length are exact copies, so many
    comparisons are exact ties, which the sorted rows send to the FP64 recount."""
    _say("large cells, many exact ties")
    w = _big_cells(73)
    feats = w.features.clone()
    for g in np.unique(w.attrs[:, 1]):
        items = np.nonzero(w.attrs[:, 1] == g)[0]
        first = items[0]
        L0 = int(w.offsets[first + 1] - w.offsets[first])
        src = feats[int(w.offsets[first]):int(w.offsets[first]) + L0].clone()
        for i in items[1:]:
            Li = int(w.offsets[i + 1] - w.offsets[i])
            idx = torch.clamp(torch.arange(Li), max=L0 - 1)
            feats[int(w.offsets[i]):int(w.offsets[i]) + Li] = src[idx]
    w.features = feats
    t, res = gpu_score(w)
    assert res.stats["n_recount_rows"] > 0
    orc = oracle_score(w)
    assert np.array_equal(res.half_units, orc.half_units)


@pytest.mark.parametrize("margin", [0.05, 1.0])
def test_margin_sends_rows_to_fp64_recount(margin):
    """A wider near-tie margin sends more rows of the brute-force count (rows of
    several x per wave pass and rows walked in passes) to the FP64 recount; at
    1.0 every row with a comparison goes (theta / pi and its path average lie
    in [0, 1]).  The counts stay those of the FP64 definition."""
    _say(f"near-tie margin {margin}")
    w = workloads.batched_c4(n_groups=24, size_hi=150, centroid_std=0.3, seed=11)
    t, res = gpu_score(w, margin=margin)
    st = res.stats
    assert st["margin"] == margin
    orc = oracle_score(w)
    assert np.array_equal(res.half_units, orc.half_units)
    rows_with_work = sum(len(c.X) for c in orc.cells if (len(c.A) - int(c.exclude_self)) * len(c.B) > 0)
    per_x = [len(c.A) * len(c.B) for c in orc.cells]
    assert min(per_x) <= 64 < max(per_x)
    if margin == 1.0:
        assert st["n_recount_rows"] == rows_with_work
    else:
        assert 0 < st["n_recount_rows"] < rows_with_work


# ---------------------------------------------------------- async score --

def test_score_async_equals_sync():
    _say("async score == sync score")
    w = workloads.within_c2(n_items=6000, dim=256, centroid_std=0.08, seed=51, device="cuda")
    ds = fx.Dataset(ctx(), w.features, w.offsets, w.attrs)
    ref = fx.Task(ds, w.on, w.by, w.across).score(keep_pairs=True)
    t = fx.Task(ds, w.on, w.by, w.across)
    r = t.score_async(keep_pairs=True)
    assert len(t) == len(ref.half_units)             # no wait needed for the cell count
    r.wait()
    assert np.array_equal(r.half_units, ref.half_units)
    g = np.array(t.keys[0][2:2 + len(w.by)])        # a BY group of the task
    items = np.nonzero(np.all(w.attrs[:, w.by] == g, axis=1))[0]
    xs, ys = np.repeat(items, len(items)), np.tile(items, len(items))
    assert all(np.array_equal(u, v) for u, v in zip(r.pairs(xs, ys), ref.pairs(xs, ys)))
    assert r.collapse(w.levels) == ref.collapse(w.levels)


def test_async_pipeline_and_rescore_of_a_pending_task():
    """Two tasks in flight while the host builds and collapses; a task scored
    again while its first score is pending (the second waits for the first)."""
    _say("async pipeline")
    ws = [workloads.within_c2(n_items=5000, dim=128, centroid_std=0.08, seed=60 + k, device="cuda")
          for k in range(3)]
    dss = [fx.Dataset(ctx(), w.features, w.offsets, w.attrs) for w in ws]
    want = [fx.Task(ds, w.on, w.by, w.across).score(keep_pairs=True) for w, ds in zip(ws, dss)]
    got, prev = [], None
    for w, ds in zip(ws, dss):
        r = fx.Task(ds, w.on, w.by, w.across).score_async()
        if prev is not None:
            got.append(prev.collapse(ws[len(got)].levels))
        prev = r
    got.append(prev.collapse(ws[-1].levels))
    assert got == [r.collapse(w.levels) for r, w in zip(want, ws)]
    t = fx.Task(dss[0], ws[0].on, ws[0].by, ws[0].across)
    r1 = t.score_async(keep_pairs=True)
    r2 = t.score_async(precision="fp32", keep_pairs=True)
    assert np.array_equal(r1.half_units, want[0].half_units)
    g = np.array(t.keys[0][2:2 + len(ws[0].by)])
    items = np.nonzero(np.all(ws[0].attrs[:, ws[0].by] == g, axis=1))[0]
    xs, ys = np.repeat(items, len(items)), np.tile(items, len(items))
    p1, p0 = r1.pairs(xs, ys), want[0].pairs(xs, ys)
    assert np.array_equal(p1[0], p0[0])              # r1's pairs were saved before r2 ran
    assert abs(r2.collapse() - want[0].collapse()) <= 1e-4
    r3 = t.score_async()
    del r3                                           # freeing a pending result waits for it
    assert np.array_equal(t.score().half_units, want[0].half_units)


def test_async_edomain_reported_on_completion():
    _say("async EDOMAIN")
    w = workloads.plain_c1(dim=16, device="cuda")
    feats = w.features.clone()
    feats[int(w.offsets[5]) + 1] = 0.0
    ds = fx.Dataset(ctx(), feats, w.offsets, w.attrs)
    r = fx.Task(ds, w.on, w.by, w.across).score_async()
    for _ in range(2):                               # reported every time it is asked
        with pytest.raises(fx.FabxError) as e:
            r.wait()
        assert e.value.code == L.FABX_EDOMAIN
    with pytest.raises(fx.FabxError):
        r.collapse()


def test_threaded_pipeline_equals_serial():
    """Build + async score on one thread while another thread waits for and
    collapses the previous results: same per-cell counts as serial scores."""
    from concurrent.futures import ThreadPoolExecutor
    _say("threaded pipeline")
    ws = [workloads.within_c2(n_items=8000, dim=128, centroid_std=0.08, seed=80 + k, device="cuda")
          for k in range(4)]
    dss = [fx.Dataset(ctx(), w.features, w.offsets, w.attrs) for w in ws]
    want = [fx.Task(ds, w.on, w.by, w.across).score().half_units.copy() for w, ds in zip(ws, dss)]
    def finish(r, w):
        return r.half_units.copy(), r.collapse(w.levels)
    with ThreadPoolExecutor(1) as helper:
        futs = []
        for rep in range(3):
            for w, ds in zip(ws, dss):
                r = fx.Task(ds, w.on, w.by, w.across).score_async()
                futs.append(helper.submit(finish, r, w))
        got = [f.result() for f in futs]
    for k, (hu, e) in enumerate(got):
        assert np.array_equal(hu, want[k % len(ws)])


def test_many_tasks_made_before_scoring():
    """A task holds its packed device tables from its creation to its first
    score; once the tasks made ahead hold the context's budget for them, later
    tasks send their tables through the staging buffer on their first score.
    Both give the same counts, also with the scores launched on a second
    thread while the first one makes tasks."""
    from concurrent.futures import ThreadPoolExecutor
    _say("many tasks made before scoring")
    w = workloads.within_c2(n_items=40000, dim=64, centroid_std=0.08, seed=90, device="cuda")
    ds = fx.Dataset(ctx(), w.features, w.offsets, w.attrs)
    want = fx.Task(ds, w.on, w.by, w.across).score().half_units.copy()
    tasks = [fx.Task(ds, w.on, w.by, w.across) for _ in range(48)]
    while tasks:
        t = tasks.pop()
        assert np.array_equal(t.score().half_units, want)
        del t
    with ThreadPoolExecutor(1) as helper:
        futs = [helper.submit(lambda t: t.score_async().half_units.copy(), fx.Task(ds, w.on, w.by, w.across))
                for _ in range(6)]
        for f in futs:
            assert np.array_equal(f.result(), want)


# ------------------------------------------------------------- autotune --

def test_autotune_tiles_give_identical_counts_and_persist(tmp_path, monkeypatch):
    """Every fused-kernel configuration gives the same per-cell counts (checked
    inside fabx_autotune), the chosen one is exact against the oracle, and a new
    context picks it up from the cache file."""
    _say("autotune")
    cache = tmp_path / "tune.txt"
    monkeypatch.setenv("FABX_AUTOTUNE_CACHE", str(cache))
    w = workloads.batched_c4(n_groups=24, size_hi=150, centroid_std=0.3, seed=11)
    feats = w.features.to("cuda")
    c1 = fx.Context(0)
    t = fx.Task(fx.Dataset(c1, feats, w.offsets, w.attrs), w.on, w.by, w.across)
    rep = t.autotune()
    print(f"  tried {rep['tried']} best {rep['best']} key {rep['key']}", flush=True)
    assert len(rep["tried"]) == 4 and rep["best"] is not None
    assert "fused" in cache.read_text()
    r = t.score()
    assert (r.stats["fused_cols"], r.stats["fused_blocks_per_cu"]) == \
        (rep["best"]["cols"], rep["best"]["blocks_per_cu"])
    orc = oracle_score(w)
    assert np.array_equal(r.half_units, orc.half_units)
    c2 = fx.Context(0)                                   # reads the cache file
    r2 = fx.Task(fx.Dataset(c2, feats, w.offsets, w.attrs), w.on, w.by, w.across).score()
    assert r2.stats["fused_cols"] == rep["best"]["cols"]
    assert np.array_equal(r2.half_units, r.half_units)
    assert fx.Task(fx.Dataset(c2, feats, w.offsets, w.attrs), w.on, w.by, w.across).autotune(
        mode="pooled")["tried"] == []                    # nothing to tune outside the fused kernel


@pytest.mark.parametrize("make", [
    lambda: workloads.within_c2(n_items=3000, dim=64, n_labels=8, n_speakers=6, seed=21),
    lambda: workloads.across_c3(n_items=3000, dim=64, n_labels=8, n_speakers=6, seed=22),
])
def test_needed_pair_counts_match_oracle(make):
    """n_pairs, dtw_cells (ordered pairs some cell needs) and dtw_cells_sym
    (unordered pairs needed in either order, the cells of a symmetric
    evaluation) against the pairs the oracle's cells use."""
    w = make()
    _say(f"needed pairs {w.name}")
    _, res = gpu_score(w)
    orc = oracle_score(w)
    lens = np.diff(np.asarray(w.offsets))
    n_pairs = dtw = sym = 0
    for items, M in orc.groups.values():
        i, j = np.nonzero(~np.isnan(M))
        n_pairs += len(i)
        dtw += int(np.sum(lens[items[i]] * lens[items[j]]))
        a, b = np.minimum(i, j), np.maximum(i, j)
        u = np.unique(a * len(items) + b)
        sym += int(np.sum(lens[items[u // len(items)]] * lens[items[u % len(items)]]))
    st = res.stats
    print(f"  pairs {n_pairs} dtw {dtw} sym {sym} computed {st['computed_dtw_cells']}", flush=True)
    assert (st["n_pairs"], st["dtw_cells"], st["dtw_cells_sym"]) == (n_pairs, dtw, sym)
    assert sym <= st["computed_dtw_cells"] <= dtw + sum(int(lens[it].sum()) ** 2 for it, _ in orc.groups.values())


def test_forced_fused_configs_equal_default():
    """Every launch choice forced through the score options (the tile kernel's
    column widths and grids, including persistent grids whose blocks take
    units from the per-XCD counters, down to one block per CU, and the stream
    kernel's segment lengths) gives the per-cell counts of the default, which
    is exact."""
    _say("forced fused-kernel configurations")
    w = workloads.batched_c4(n_groups=24, size_hi=150, centroid_std=0.3, seed=12)
    feats = w.features.to("cuda")
    t = fx.Task(fx.Dataset(fx.Context(0), feats, w.offsets, w.attrs), w.on, w.by, w.across)
    ref = t.score()
    assert np.array_equal(ref.half_units, oracle_score(w).half_units)
    for cols, bpc in ((128, 0), (128, 1), (128, 4), (256, 0), (256, 2), (512, 2), (2048, 0), (1024, 1)):
        r = t.score(fused_cols=cols, fused_blocks_per_cu=bpc)
        print(f"  cols {cols} blocks/CU {bpc}: distance {r.stats['ms_distance']:.3f} ms", flush=True)
        assert (r.stats["fused_cols"], r.stats["fused_blocks_per_cu"]) == (cols, bpc)
        assert np.array_equal(r.half_units, ref.half_units)
    # a fresh task whose first score uses the other width: its tables come from
    # the block packed at task creation, that width's column plan separately
    t2 = fx.Task(fx.Dataset(fx.Context(0), feats, w.offsets, w.attrs), w.on, w.by, w.across)
    r2 = t2.score(fused_cols=256, fused_blocks_per_cu=2)
    assert np.array_equal(r2.half_units, ref.half_units)
    assert np.array_equal(t2.score().half_units, ref.half_units)


# ------------------------------------------------- Euclidean distance --

@pytest.mark.parametrize("mode,norm", [("dtw", "path"), ("dtw", "none"), ("pooled", "path")])
def test_euclidean_fp32(mode, norm):
    """The Euclidean distance in the FP32 form against the FP64 oracle: same
    cells, ABX error within 1e-4 (the FP32 form's bar), every needed pair
    distance within a relative 4 (dim + 64) 2^-24 (sums of non-negative
    squares and costs in FP32), and no cell count off beyond rare near-tie
    flips.  One frame is zero: it has a length, so it is scored."""
    w = workloads.plain_c1(centroid_std=0.15)
    feats = w.features.clone()
    feats[int(w.offsets[5])] = 0.0
    w.features = feats
    _say(f"euclidean fp32 {mode} {norm} n_items={w.n_items}")
    t, res = gpu_score(w, mode=mode, precision="fp32", norm=norm, distance="euclidean", keep_pairs=True)
    orc = oracle.score(w.features_f32_host(), w.offsets, w.attrs, w.on, w.by, w.across, mode, norm,
                       distance="euclidean")
    assert np.array_equal(t.keys, orc.keys.astype(np.int32))
    assert np.array_equal(t.sizes[0], orc.n_triplets)
    xs, ys, want = all_oracle_pairs(orc)
    f32, _, _ = res.pairs(xs, ys)
    rel = np.abs(f32.astype(np.float64) - want) / np.maximum(want, 1e-30)
    tol = 4 * (w.dim + 64) * 2.0 ** -24
    mism = int(np.count_nonzero(res.half_units != orc.half_units))
    e_gpu, e_orc = res.collapse(w.levels), oracle.error_rate(orc, w.levels)
    print(f"  pairs={len(want)} max_rel={rel.max():.2e} tol={tol:.1e} mism={mism}/{len(orc.cells)} "
          f"err={e_gpu:.6f} oracle_err={e_orc:.6f}", flush=True)
    assert rel.max() <= tol
    assert abs(e_gpu - e_orc) <= 1e-4
    assert mism <= max(2, len(orc.cells) // 1000)


def _euclid_case(name):
    if name == "c1-zero-frame":
        w = workloads.plain_c1(centroid_std=0.15)
        feats = w.features.clone()
        feats[int(w.offsets[5])] = 0.0      # a zero frame has a length: it is scored
        w.features = feats
        return w
    if name == "c2-shape-768":
        return workloads.within_c2(n_items=3000, centroid_std=0.1, seed=41)
    if name == "near-copies-1024":
        # half the items with a copy under 1e-4 relative noise: near-parallel,
        # near-equal-length frames, where the cosine form cancels
        w = workloads.batched_c4(n_groups=8, size_lo=6, size_hi=20, len_lo=1, len_hi=12, dim=1024,
                                 centroid_std=0.3, seed=42, dtype=torch.float32)
        return _with_twins(w, 1e-4, seed=7)
    if name == "long-copies-1024":
        # items of 17-64 frames and exact copies: the FP64 recheck takes these
        # pairs (more than 256 frame pairs) in its register-tiled form
        w = workloads.batched_c4(n_groups=6, size_lo=4, size_hi=8, len_lo=17, len_hi=64, dim=1024,
                                 centroid_std=0.3, seed=43, dtype=torch.float32)
        return _with_twins(w, 0.0, seed=8)
    raise ValueError(name)


@pytest.mark.parametrize("mode,norm", [("dtw", "path"), ("dtw", "none"), ("pooled", "path")])
@pytest.mark.parametrize("case", ["c1-zero-frame", "c2-shape-768", "near-copies-1024", "long-copies-1024"])
def test_euclidean_bf16_exact(case, mode, norm):
    """The Euclidean distance in the BF16 + FP64-recheck form: the unit-vector
    cosine from the MFMA Gram tile and each frame's FP32 length give
    |u - v| = sqrt((|u| - |v|)^2 + 2 |u| |v| (1 - cos)); margin and DTW window
    are the angular ones times pi times the largest length S.  Bar: every
    cell's count equals the FP64 oracle's, every robust pair within
    margin / 2, every FP64-rechecked pair within 1e-12 relative."""
    w = _euclid_case(case)
    _say(f"euclidean bf16 {case} {mode} {norm} n_items={w.n_items} dim={w.dim}")
    t, res = gpu_score(w, mode=mode, precision="bf16", norm=norm, distance="euclidean", keep_pairs=True)
    orc = oracle.score(w.features_f32_host(), w.offsets, w.attrs, w.on, w.by, w.across, mode, norm,
                       distance="euclidean")
    assert np.array_equal(t.keys, orc.keys.astype(np.int32))
    assert np.array_equal(t.sizes[0], orc.n_triplets)
    f = w.features_f32_host().astype(np.float64)
    if mode == "dtw":
        S = float(np.sqrt((f * f).sum(axis=1)).max())
    else:
        means = np.stack([f[w.offsets[i]:w.offsets[i + 1]].mean(axis=0) for i in range(w.n_items)])
        S = float(np.sqrt((means * means).sum(axis=1)).max())
    st = res.stats
    margin = st["margin"] * S
    xs, ys, want = all_oracle_pairs(orc)
    f32, fl, f64 = res.pairs(xs, ys)
    err = np.abs(f32.astype(np.float64) - want)
    robust = (fl & 1) == 0
    mism = int(np.count_nonzero(res.half_units != orc.half_units))
    print(f"  S={S:.3f} margin={margin:.3g} max_robust_err={err[robust].max():.3g} "
          f"nonrobust={st['n_nonrobust_pairs']} recheck={st['n_recheck_pairs']} recount={st['n_recount_rows']} "
          f"mism={mism}/{len(orc.cells)} err={res.collapse():.6f} oracle_err={oracle.error_rate(orc):.6f}",
          flush=True)
    assert mism == 0
    assert abs(res.collapse() - oracle.error_rate(orc)) <= 1e-12
    assert err[robust].max() <= margin / 2
    rechecked = (fl & 2) != 0
    if rechecked.any():
        assert (np.abs(f64[rechecked] - want[rechecked]) <= 1e-12 * np.maximum(want[rechecked], 1.0)).all()


# ---------------------------------------------------------- discrete units --

def _unit_workload(seed, n_groups=8, size_hi=40, len_hi=30, vocab=50):
    """Discrete-unit items: per frame, with probability 0.5 one of the label's
    three preferred units, else any unit; ON label BY group."""
    rng = np.random.default_rng(seed)
    sizes = rng.integers(4, size_hi + 1, n_groups)
    label = np.concatenate([rng.integers(0, 4, n) for n in sizes]).astype(np.int32)
    group = np.repeat(np.arange(n_groups), sizes).astype(np.int32)
    lens = rng.integers(1, len_hi + 1, len(label))
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    pref = rng.integers(0, vocab, (4, 3))
    lab_f = np.repeat(label, lens)
    codes = np.where(rng.random(int(off[-1])) < 0.5, pref[lab_f, rng.integers(0, 3, int(off[-1]))],
                     rng.integers(0, vocab, int(off[-1]))).astype(np.int32)
    attrs = np.stack([label, group], axis=1).astype(np.int32)
    return codes, off, attrs


@pytest.mark.parametrize("norm", ["path", "none"])
@pytest.mark.parametrize("case", ["short", "long"])
def test_discrete_units_exact(case, norm):
    """Unit-code datasets (int32 codes, FABX_DISTANCE_UNITS): the frame
    distance is 0 or 1, the DTW costs are exact integers and the
    path-normalised values exact fractions rounded once, so every cell's count
    equals the oracle's, with items of up to 30 frames and of up to 150
    (row chunks)."""
    codes, off, attrs = _unit_workload(80 + (case == "long"), len_hi=30 if case == "short" else 150,
                                       size_hi=40 if case == "short" else 14)
    _say(f"discrete units {case} {norm}: {len(attrs)} items, {len(codes)} frames")
    ds = fx.Dataset(ctx(), torch.tensor(codes, device="cuda"), off, attrs)
    t = fx.Task(ds, 0, [1], [])
    res = t.score(distance="units", norm=norm, keep_pairs=True)
    torch.cuda.synchronize()
    orc = oracle.score(codes.astype(np.float32)[:, None], off, attrs, 0, [1], [], "dtw", norm, distance="units")
    assert np.array_equal(t.keys, orc.keys.astype(np.int32))
    assert np.array_equal(t.sizes[0], orc.n_triplets)
    xs, ys, want = all_oracle_pairs(orc)
    f32, _, _ = res.pairs(xs, ys)
    mism = int(np.count_nonzero(res.half_units != orc.half_units))
    print(f"  cells={len(orc.cells)} pairs={len(want)} max_pair_err={np.abs(f32 - want).max():.3g} mism={mism} "
          f"err={res.collapse():.6f} oracle_err={oracle.error_rate(orc):.6f}", flush=True)
    # each value is the exact fraction rounded once to FP32
    assert np.array_equal(f32, want.astype(np.float32))
    assert mism == 0
    assert 0.0 < oracle.error_rate(orc) < 0.5


# ----------------------------------------------------- item-file front end --

@pytest.mark.parametrize("libri_light", [False, True])
def test_item_file_dataset_scores_like_its_copy(tmp_path, libri_light):
    """Units sliced from whole-utterance features through an item file
    (overlapping windows, no copy) give the per-cell counts of a contiguous
    copy of their frames, and the oracle's on that copy."""
    _say(f"item file front end libri_light={libri_light}")
    rng = np.random.default_rng(91)
    dt, dim = 0.02, 32
    cent = {p: rng.standard_normal(dim).astype(np.float32) for p in "aeioumn"}
    utts, rows = {}, []
    for k in range(12):
        T = int(rng.integers(60, 160))
        name, spk = f"utt{k}", f"s{k % 3}"
        labels = rng.choice(list(cent), (T + 3) // 4)
        frames = np.stack([cent[labels[i // 4]] for i in range(T)]) + \
            0.8 * rng.standard_normal((T, dim)).astype(np.float32)
        utts[name] = torch.tensor(frames)
        t = 0.0
        while True:
            dur = float(rng.uniform(0.05, 0.2))
            if t + dur > T * dt - dt:
                break
            mid = labels[min(int((t + dur / 2) / dt) // 4, len(labels) - 1)]
            rows.append((name, round(t, 4), round(t + dur, 4), mid, spk))
            t += float(rng.uniform(0.03, 0.08))      # steps shorter than units: windows overlap
    path = str(tmp_path / "units.item")
    with open(path, "w") as f:
        f.write("#file onset offset #phone speaker\n")
        for r in rows:
            f.write(" ".join(str(v) for v in r) + "\n")
    ds, names, vocab = fx.Dataset.from_item_file(ctx(), path, {k: v.cuda() for k, v in utts.items()}, dt,
                                                 libri_light)
    on, spk = names.index("phone"), names.index("speaker")
    t = fx.Task(ds, on, [spk], [])
    res = t.score()
    # the same units as a contiguous copy, on the host
    files = [r[0] for r in rows]
    start, length = fx.fabx_slice_frames([r[1] for r in rows], [r[2] for r in rows], dt, libri_light)
    copy = np.concatenate([utts[f].numpy()[s0:s0 + n] for f, s0, n in zip(files, start, length)])
    off = np.concatenate([[0], np.cumsum(length)]).astype(np.int64)
    codes = np.stack([np.unique(np.array([r[3] for r in rows]), return_inverse=True)[1],
                      np.unique(np.array([r[4] for r in rows]), return_inverse=True)[1]], 1).astype(np.int32)
    tc = fx.Task(fx.Dataset(ctx(), torch.tensor(copy).cuda(), off, codes), on, [spk], [])
    rc = tc.score()
    orc = oracle.score(copy, off, codes, on, [spk], [])
    print(f"  units={len(rows)} cells={len(orc.cells)} frames kept={int(length.sum())}", flush=True)
    assert len(orc.cells) > 50
    assert np.array_equal(t.keys, tc.keys)
    assert np.array_equal(res.half_units, rc.half_units)
    assert np.array_equal(res.half_units, orc.half_units)


def _triphone_items(rng, path, n_utts=16, phones="aei", dim=32, dt=0.02):
    """Synthetic utterances of 4-frame phone segments and an item file of
    overlapping triphone-like units over them (phone, prev-phone, next-phone,
    speaker columns); returns the per-utterance features and the rows."""
    cent = {p: 0.3 * rng.standard_normal(dim).astype(np.float32) for p in phones}
    utts, rows = {}, []
    for k in range(n_utts):
        T = int(rng.integers(80, 200))
        name, spk = f"utt{k}", f"s{k % 4}"
        labels = rng.choice(list(phones), (T + 3) // 4)
        utts[name] = torch.tensor(np.stack([cent[labels[i // 4]] for i in range(T)]) +
                                  0.8 * rng.standard_normal((T, dim)).astype(np.float32))
        for j in range(1, len(labels) - 2):
            on, off = 4 * j * dt + float(rng.uniform(-0.01, 0.01)), 4 * (j + 1) * dt + float(rng.uniform(-0.01, 0.01))
            rows.append((name, round(max(on, 0.0), 4), round(off, 4), labels[j], labels[j - 1], labels[j + 1], spk))
    with open(path, "w") as f:
        f.write("#file onset offset #phone prev-phone next-phone speaker\n")
        for r in rows:
            f.write(" ".join(str(v) for v in r) + "\n")
    return utts, rows


@pytest.mark.parametrize("speaker,context", [("within", "within"), ("across", "within"), ("within", "any")])
def test_zerospeech_abx_matches_oracle(tmp_path, speaker, context):
    """zerospeech_abx (item file -> slices -> ON phone, BY context, BY / ACROSS
    speaker -> averages over contexts, then speakers, then phone pairs) equals
    the oracle's error rate on a contiguous copy of the sliced units."""
    _say(f"zerospeech_abx speaker={speaker} context={context}")
    rng = np.random.default_rng(92)
    dt = 0.02
    path = str(tmp_path / "tri.item")
    utts, rows = _triphone_items(rng, path, dt=dt)
    err = fx.zerospeech_abx(ctx(), path, {k: v.cuda() for k, v in utts.items()}, dt, speaker, context)
    start, length = fx.fabx_slice_frames([r[1] for r in rows], [r[2] for r in rows], dt)
    copy = np.concatenate([utts[r[0]].numpy()[s0:s0 + n] for r, s0, n in zip(rows, start, length)])
    off = np.concatenate([[0], np.cumsum(length)]).astype(np.int64)
    codes = np.stack([np.unique(np.array([r[c] for r in rows]), return_inverse=True)[1] for c in (3, 4, 5, 6)],
                     1).astype(np.int32)
    phone, prev, nxt, spk = 0, 1, 2, 3
    ctx_cols = [prev, nxt] if context == "within" else []
    by = ctx_cols + ([spk] if speaker == "within" else [])
    across = [spk] if speaker == "across" else []
    orc = oracle.score(copy, off, codes, phone, by, across)
    levels = ([ctx_cols] if ctx_cols else []) + [[spk]]
    e_orc = oracle.error_rate(orc, levels)
    print(f"  units={len(rows)} cells={len(orc.cells)} err={err:.6f} oracle_err={e_orc:.6f}", flush=True)
    assert len(orc.cells) > 20
    assert abs(err - e_orc) <= 1e-12


def test_zerospeech_command_line(tmp_path):
    """python -m paper_2505_02692_amd ITEM DIR --frame-step: the same error rate
    as zerospeech_abx, from per-utterance .npy files."""
    import json
    import os
    import subprocess
    _say("zerospeech command line")
    rng = np.random.default_rng(93)
    path = str(tmp_path / "tri.item")
    utts, _ = _triphone_items(rng, path, n_utts=8)
    fdir = tmp_path / "feats"
    fdir.mkdir()
    for k, v in utts.items():
        np.save(str(fdir / (k + ".npy")), v.numpy())
    want = fx.zerospeech_abx(ctx(), path, {k: v.cuda() for k, v in utts.items()}, 0.02, "across")
    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    out = subprocess.run([sys.executable, "-m", "paper_2505_02692_amd", path, str(fdir), "--frame-step", "0.02",
                          "--speaker", "across"], capture_output=True, text=True, timeout=240, cwd=root)
    assert out.returncode == 0, out.stderr[-2000:]
    got = json.loads(out.stdout.strip().splitlines()[-1])
    assert got["abx_error"] == want and got["speaker"] == "across"


# ------------------------------------------------------- stream ordering --

def _slow_producer(dst, src):
    """Enqueue on torch's current stream about 0.1 s of matrix products, then the
    copy src -> dst, and return without waiting: whoever reads dst next must be
    ordered after this work on the stream."""
    a = torch.randn(8192, 8192, device="cuda")
    c = torch.empty_like(a)
    for _ in range(12):
        torch.mm(a, a, out=c)
    dst.copy_(src)


def _ordering_case(seed):
    w = workloads.within_c2(n_items=20000, dim=256, centroid_std=0.08, seed=seed, device="cuda")
    ds_ref = fx.Dataset(ctx(), w.features, w.offsets, w.attrs)
    want = fx.Task(ds_ref, w.on, w.by, w.across).score().half_units.copy()
    # valid features of the wrong frames until the producer's copy lands
    buf = torch.roll(w.features, 1, dims=0).contiguous()
    torch.cuda.synchronize()
    return w, want, buf


def test_score_is_ordered_after_producer_on_stream():
    _say("stream order: score")
    w, want, buf = _ordering_case(41)
    _slow_producer(buf, w.features)
    ds = fx.Dataset(ctx(), buf, w.offsets, w.attrs)
    got = fx.Task(ds, w.on, w.by, w.across).score().half_units
    assert np.array_equal(got, want)


def test_server_job_is_ordered_after_producer_on_stream():
    _say("stream order: server")
    w, want, buf = _ordering_case(42)
    srv = fx.Server(ctx(), hbm_budget_bytes=8 << 30, n_streams=2)
    _slow_producer(buf, w.features)
    ds = fx.Dataset(ctx(), buf, w.offsets, w.attrs)
    jid = srv.submit(ds, w.on, w.by, w.across)
    _, got, _, _ = srv.wait(jid)
    srv.close()
    assert np.array_equal(got, want)


# ------------------------------------------ large groups, sampled pairs --

@pytest.mark.parametrize("n_items", [12000, 24000, None])
def test_large_groups_sampled_pairs(n_items):
    """Serving-shaped across job with groups of thousands of items: sampled pair
    distances against the oracle, and no spurious near ties.  n_items=None is the
    serving stream's job 1 as drawn (32,660 items, a 9,616-item group: over 2^32
    work-items if one block per unit were launched)."""
    if n_items is None:
        w = workloads.serving_job(1, device="cuda")
    else:
        w = workloads.serving_job(1, device="cuda", n_items=n_items, dim=1024, across=True)
    _say(f"large groups n_items={n_items}")
    t, res = gpu_score(w, keep_pairs=True)
    st = res.stats
    print(f"  cells={st['n_cells']} pairs={st['n_pairs']} recheck={st['n_recheck_pairs']} "
          f"recount={st['n_recount_rows']} nonrobust={st['n_nonrobust_pairs']} gpu={st['ms_total']:.1f}ms",
          flush=True)
    # sample pairs (x, y) inside the largest BY group, spread over its row / column blocks
    g = np.bincount(w.attrs[:, 1]).argmax()
    items = np.nonzero(w.attrs[:, 1] == g)[0]
    rng = np.random.default_rng(0)
    xs = rng.choice(items, 400)
    ys = rng.choice(items, 400)
    f32, fl, f64 = res.pairs(xs, ys)
    loc = {int(v): k for k, v in enumerate(items)}
    want = oracle.pair_distances(w.features_f32_host(), w.offsets, [items],
                                 [(np.array([loc[int(x)] for x in xs], np.int32),
                                   np.array([loc[int(y)] for y in ys], np.int32))])[0]
    err = np.abs(f32.astype(np.float64) - want)
    worst = np.argsort(err)[-5:]
    for k in worst:
        print(f"  pair ({xs[k]},{ys[k]}) pos ({loc[int(xs[k])]},{loc[int(ys[k])]}) gpu {f32[k]:.6f} "
              f"oracle {want[k]:.6f} flags {fl[k]}", flush=True)
    assert err[(fl & 1) == 0].max() <= st["margin"] / 2
    assert st["n_recheck_pairs"] < 0.01 * st["n_pairs"]


# ----------------------------------------------- full-size bench workload --

def _groups_subset(w, by_values):
    """The items of the given BY groups (tuples of w.by values) as a small
    host dataset: frames (float32), offsets, attrs."""
    mask = np.zeros(w.n_items, bool)
    for v in by_values:
        m = np.ones(w.n_items, bool)
        for col, val in zip(w.by, v):
            m &= w.attrs[:, col] == val
        mask |= m
    items = np.nonzero(mask)[0]
    feats = w.features.float()
    frames = [feats[int(w.offsets[i]):int(w.offsets[i + 1])].cpu().numpy() for i in items]
    off = np.concatenate([[0], np.cumsum([len(f) for f in frames])]).astype(np.int64)
    return np.concatenate(frames), off, np.ascontiguousarray(w.attrs[items])


def test_across_c3_full_size_sampled_groups():
    """The across-speaker workload at full size (200k items, dim 1024, 30.9M
    cells) in the bench's configuration: every cell of 2 sampled BY groups
    equals the oracle's, run on those groups' items (cells never span BY
    groups)."""
    w = workloads.across_c3(device="cuda")
    _say(f"across-c3 full size n_items={w.n_items}")
    t, res = gpu_score(w)
    keys, hu = t.keys, res.half_units
    nb = len(w.by)
    gkeys = [tuple(int(v) for v in k[2:2 + nb]) for k in keys]
    per_group = {}
    for g in gkeys:
        per_group[g] = per_group.get(g, 0) + 1
    mid = sorted(g for g, n in per_group.items() if 2000 <= n <= 15000)   # groups of moderate size
    rng = np.random.default_rng(5)
    chosen = [mid[i] for i in rng.choice(len(mid), 2, replace=False)]
    feats, off, attrs = _groups_subset(w, chosen)
    print(f"  scored {len(keys)} cells on the GPU; oracle on {len(off) - 1} items of groups {chosen}", flush=True)
    orc = oracle.score(feats, off, attrs, w.on, w.by, w.across)
    where = {tuple(int(v) for v in k): c for c, k in enumerate(keys)}
    idx = np.array([where[tuple(int(v) for v in k)] for k in orc.keys])
    in_chosen = np.array([g in set(chosen) for g in gkeys])
    print(f"  cells={len(keys)} sampled groups={chosen} their cells={len(idx)} "
          f"recheck={res.stats['n_recheck_pairs']} recount={res.stats['n_recount_rows']}", flush=True)
    assert len(idx) >= 4000 and int(in_chosen.sum()) == len(idx)
    assert np.array_equal(hu[idx], orc.half_units)
    assert np.array_equal(t.sizes[0][idx], orc.n_triplets)


def test_within_c2_full_size_bf16():
    """The bench workload at full size (100k items, dim 768): every cell exact."""
    w = workloads.within_c2(device="cuda")
    check(w, levels=True)


# ------------------------------------------ plain form in strips / batches --

def test_plain_fp32_in_strips_equals_whole(monkeypatch):
    """The plain form makes a group's frame distance matrix in strips of item
    rows and runs them in batches through one buffer.  With a buffer of 4096
    cells, every group of this task (about 780 frames) is cut into strips of
    a few items and every strip runs alone: the counts and pair distances must
    equal those of the one-batch run bit for bit (the same sums in the same
    order), and the oracle's within the plain form's bar."""
    w = workloads.plain_c1(centroid_std=0.15, seed=3)
    _say("plain fp32: strips vs whole groups")
    feats = w.features.to("cuda").contiguous()
    ds = fx.Dataset(ctx(), feats, w.offsets, w.attrs)
    t = fx.Task(ds, w.on, w.by, w.across)
    whole = t.score(precision="fp32", keep_pairs=True)
    orc = oracle_score(w)
    xs, ys, want = all_oracle_pairs(orc)
    p_whole = whole.pairs(xs, ys)[0]
    monkeypatch.setenv("FABX_PLAIN_DMAT_CELLS", "4096")
    t2 = fx.Task(ds, w.on, w.by, w.across)
    cut = t2.score(precision="fp32", keep_pairs=True)
    p_cut = cut.pairs(xs, ys)[0]
    assert np.array_equal(p_cut, p_whole)
    assert np.array_equal(cut.half_units, whole.half_units)
    assert np.abs(p_cut.astype(np.float64) - want).max() <= 2e-6
    assert abs(cut.collapse() - oracle.error_rate(orc)) <= 1e-4
    # pooled mode and the BF16 form are unaffected by the setting
    _, res_b = gpu_score(w)
    assert np.array_equal(res_b.half_units, orc.half_units)


# ------------------------------------------------- batched workload, full size --

def _groups_by_size(w):
    col = w.attrs[:, w.by[0]]
    ids, counts = np.unique(col, return_counts=True)
    return ids, counts


def _check_sampled_groups(w, t, res, chosen):
    """Every cell of the chosen BY groups (values of the single BY column)
    equals the oracle's, run on those groups' items only."""
    keys, hu = t.keys, res.half_units
    where = {tuple(int(v) for v in k): c for c, k in enumerate(keys)}
    sizes = t.sizes[0]
    n_checked = 0
    # the oracle runs on a few groups at a time (about 8 groups, or one large
    # group), and the progress is printed after each run
    col = w.attrs[:, w.by[0]]
    counts = {int(g): int(np.count_nonzero(col == g)) for g in chosen}
    batches, cur = [], []
    for g in chosen:
        if cur and (len(cur) >= 8 or counts[int(g)] > 200):
            batches.append(cur)
            cur = []
        cur.append(int(g))
    batches.append(cur)
    for b in batches:
        feats, off, attrs = _groups_subset(w, [(g,) for g in b])
        t0 = time.perf_counter()
        orc = oracle.score(feats, off, attrs, w.on, w.by, w.across)
        idx = np.array([where[tuple(int(v) for v in k)] for k in orc.keys])
        bad = np.nonzero(hu[idx] != orc.half_units)[0]
        print(f"  groups {b} ({len(off) - 1} items): {len(idx)} cells, oracle {time.perf_counter() - t0:.1f} s, "
              f"{len(bad)} differ", flush=True)
        for c in bad[:5]:
            print(f"  cell {tuple(orc.keys[c])}: gpu {hu[idx][c]} oracle {orc.half_units[c]}", flush=True)
        assert len(bad) == 0, f"{len(bad)} of {len(idx)} cells differ"
        assert np.array_equal(sizes[idx], orc.n_triplets)
        n_checked += len(idx)
    in_chosen = np.isin(keys[:, 2], np.asarray(chosen, dtype=keys.dtype))
    assert int(in_chosen.sum()) == n_checked
    return n_checked


def test_batched_c4_full_size_sampled_groups():
    """The batched uneven workload at full size (5,000 BY groups of 2-2,000
    items, 1.05M items, lengths 1-60, dim 512 BF16), scored in one persistent
    launch as the bench runs it: every cell of 48 seeded groups of at most 200
    items and 6 groups of 200-600 items equals the oracle's (the oracle takes
    about 15-60 s for each of the latter on 16 cores)."""
    w = workloads.batched_c4(device="cuda")
    _say(f"batched-c4 full size n_items={w.n_items}")
    t, res = gpu_score(w)
    st = res.stats
    print(f"  cells={st['n_cells']} triplets={st['n_triplets']} gpu={st['ms_total']:.0f}ms "
          f"nonrobust={st['n_nonrobust_pairs']} recheck={st['n_recheck_pairs']}", flush=True)
    ids, counts = _groups_by_size(w)
    rng = np.random.default_rng(11)
    small = ids[counts <= 200]
    mid = ids[(counts > 200) & (counts <= 600)]
    chosen = list(rng.choice(small, 48, replace=False)) + list(rng.choice(mid, 6, replace=False))
    n = _check_sampled_groups(w, t, res, chosen)
    print(f"  {n} cells equal the oracle's", flush=True)


@pytest.mark.skipif(not os.environ.get("FABX_SLOW_TESTS"),
                    reason="long oracle run (about 10 min on 16 cores): set FABX_SLOW_TESTS=1")
def test_batched_c4_full_size_all_small_groups_and_largest():
    """As above, on every group of at most 200 items (3,764 groups) and the two
    largest groups (2,000 items each)."""
    w = workloads.batched_c4(device="cuda")
    _say(f"batched-c4 full size, all small groups n_items={w.n_items}")
    t, res = gpu_score(w)
    ids, counts = _groups_by_size(w)
    order = np.argsort(counts)
    chosen = list(ids[counts <= 200]) + list(ids[order[-2:]])
    n = _check_sampled_groups(w, t, res, chosen)
    print(f"  {n} cells equal the oracle's", flush=True)


# ---------------------------------------------- serving jobs vs the oracle --

def _stream_jobs_for_oracle(n_draws=100, max_items=5000, max_cost=2e11):
    """Jobs of the serving stream (its own draws, seed 4) with at most
    max_items items whose oracle cost (sum over BY groups of squared frame
    counts x 2 dim) is at most max_cost; only the host-side draws are made."""
    out = []
    for j in range(n_draws):
        rng = workloads._rng(4 * 100003 + j)
        n = int(np.rint(np.exp(rng.uniform(np.log(1000), np.log(50000)))))
        d = int(rng.choice([256, 512, 768, 1024, 1280]))
        acr = bool(rng.random() < 0.5)
        workloads._zipf_labels(rng, 1.0, 40, n)
        ctxs = workloads._zipf_labels(rng, 1.0, 16, n)
        spk = rng.integers(0, 20, size=n)
        lens = rng.integers(1, 61, size=n)
        key = ctxs if acr else ctxs * 20 + spk
        cost = float((np.bincount(key, weights=lens) ** 2).sum()) * d * 2
        if n <= max_items and cost <= max_cost:
            out.append(j)
    return out


def test_serving_jobs_match_oracle():
    """Jobs of the serving stream as drawn (BF16 features, dims 256-1280,
    within and across speaker, lengths 1-60) with at most 5k items: scored
    alone and then served together on 4 streams, every cell of every job
    equals the oracle's in both."""
    sel = _stream_jobs_for_oracle()
    _say(f"serving jobs vs oracle: {len(sel)} jobs {sel}")
    jobs = []
    for j in sel:
        w = workloads.serving_job(j, device="cuda")
        jobs.append((w, fx.Dataset(ctx(), w.features, w.offsets, w.attrs)))
    assert any(w.across for w, _ in jobs) and any(not w.across for w, _ in jobs)
    alone = [fx.Task(ds, w.on, w.by, w.across).score().half_units.copy() for w, ds in jobs]
    srv = fx.Server(ctx(), hbm_budget_bytes=32 << 30, n_streams=4)
    ids = [srv.submit(ds, w.on, w.by, w.across) for w, ds in jobs]
    served = [srv.wait(i) for i in ids]
    srv.close()
    for (w, ds), a, (keys, W, n, s) in zip(jobs, alone, served):
        orc = oracle.score(w.features_f32_host(), w.offsets, w.attrs, w.on, w.by, w.across)
        assert np.array_equal(keys, orc.keys.astype(np.int32))
        ma, ms_ = int(np.count_nonzero(a != orc.half_units)), int(np.count_nonzero(W != orc.half_units))
        print(f"  {w.name} n={w.n_items} dim={w.dim} cells={len(W)} alone-vs-oracle {ma} "
              f"served-vs-oracle {ms_} err={oracle.error_rate(orc, w.levels):.4f}", flush=True)
        assert ma == 0 and ms_ == 0


def test_server_failing_job_leaves_others_intact():
    """A job whose features hold a zero-norm frame fails with EDOMAIN in the
    middle of a mix; every other job's counts equal its alone result."""
    _say("server: failing job in a mix")
    specs = [(1500, 512, False), (2200, 768, True), (1800, 256, False), (2600, 1024, True), (1200, 1280, False)]
    jobs = []
    for j, (n, d, a) in enumerate(specs):
        w = workloads.serving_job(j, n_items=n, dim=d, across=a, centroid_std=0.1, device="cuda")
        jobs.append((w, fx.Dataset(ctx(), w.features, w.offsets, w.attrs)))
    alone = [fx.Task(ds, w.on, w.by, w.across).score().half_units.copy() for w, ds in jobs]
    bad_w = workloads.serving_job(9, n_items=2000, dim=512, across=False, device="cuda")
    feats = bad_w.features.clone()
    feats[int(bad_w.offsets[700]) + 0].zero_()
    bad_ds = fx.Dataset(ctx(), feats, bad_w.offsets, bad_w.attrs)
    srv = fx.Server(ctx(), hbm_budget_bytes=16 << 30, n_streams=3)
    ids = [srv.submit(ds, w.on, w.by, w.across) for w, ds in jobs[:2]]
    bad_id = srv.submit(bad_ds, bad_w.on, bad_w.by, bad_w.across)
    ids += [srv.submit(ds, w.on, w.by, w.across) for w, ds in jobs[2:]]
    with pytest.raises(fx.FabxError) as e:
        srv.wait(bad_id)
    assert e.value.code == -3
    for jid, a in zip(ids, alone):
        assert np.array_equal(srv.wait(jid)[1], a)
    st = srv.stats
    assert st["failed"] == 1 and st["completed"] == len(jobs)
    # an outcome is handed over once
    with pytest.raises(fx.FabxError) as e2:
        srv.wait(ids[0])
    assert e2.value.code == -7
    srv.close()


def test_server_small_job_passes_a_waiting_large_one():
    """Budget for one large job plus one small one: while a large job runs, a
    second large job waits for memory, and a small job submitted after it is
    admitted at once instead of queueing behind it.  Of the three queue waits
    the median is then near zero (head-of-line admission would make it the
    large job's run time)."""
    _say("server: admission past a waiting job")
    big = [workloads.serving_job(20 + k, n_items=16000, dim=1024, across=True, device="cuda") for k in range(2)]
    small = workloads.serving_job(30, n_items=1000, dim=256, across=False, device="cuda")
    dbig = [fx.Dataset(ctx(), w.features, w.offsets, w.attrs) for w in big]
    dsmall = fx.Dataset(ctx(), small.features, small.offsets, small.attrs)
    t0 = time.perf_counter()
    ref_big = fx.Task(dbig[0], big[0].on, big[0].by, big[0].across).score().half_units.copy()
    t_big = (time.perf_counter() - t0) * 1e3
    ref_small = fx.Task(dsmall, small.on, small.by, small.across).score().half_units.copy()
    # footprints from a first server with room for everything
    probe = fx.Server(ctx(), hbm_budget_bytes=64 << 30, n_streams=1)
    probe.wait(probe.submit(dbig[0], big[0].on, big[0].by, big[0].across))
    fp_big = probe.stats["hbm_high_water"]
    probe.wait(probe.submit(dsmall, small.on, small.by, small.across))
    probe.close()
    srv = fx.Server(ctx(), hbm_budget_bytes=int(fp_big * 1.6), n_streams=3)
    j1 = srv.submit(dbig[0], big[0].on, big[0].by, big[0].across)
    j2 = srv.submit(dbig[1], big[1].on, big[1].by, big[1].across)
    j3 = srv.submit(dsmall, small.on, small.by, small.across)
    assert np.array_equal(srv.wait(j3)[1], ref_small)
    assert np.array_equal(srv.wait(j1)[1], ref_big)
    srv.wait(j2)
    st = srv.stats
    print(f"  big alone {t_big:.1f} ms, footprint {fp_big / 2**30:.2f} GiB; queue p50 {st['p50_queue_ms']:.1f} ms "
          f"p99 {st['p99_queue_ms']:.1f} ms, mean run {st['mean_run_ms']:.1f} ms", flush=True)
    assert st["p50_queue_ms"] < 0.25 * t_big
    assert st["p99_queue_ms"] > 0.25 * t_big   # the second large job did wait
    srv.close()


def test_server_device_memory_steady_over_waves():
    """Finished jobs give their device tables and workspace back to the
    context's pool: a second wave of the same jobs runs in the memory the first
    one left (device free memory unchanged), and nothing stays counted as in
    use once the outcomes are fetched."""
    _say("server: device memory over two waves of jobs")
    ws = [workloads.serving_job(40 + k, n_items=1500 + 300 * k, dim=(256, 512, 768)[k % 3], across=bool(k % 2),
                                device="cuda") for k in range(8)]
    dss = [fx.Dataset(ctx(), w.features, w.offsets, w.attrs) for w in ws]
    srv = fx.Server(ctx(), hbm_budget_bytes=24 << 30, n_streams=1)   # one job at a time: same peak each wave
    free = []
    for wave in range(3):
        ids = [srv.submit(ds, w.on, w.by, w.across) for w, ds in zip(ws, dss)]
        for jid in ids:
            srv.wait(jid)
        torch.cuda.synchronize()
        st = srv.stats
        assert st["hbm_in_use"] == 0 and st["running"] == 0 and st["queued"] == 0
        free.append(torch.cuda.mem_get_info()[0])
        print(f"  wave {wave}: device free {free[-1] / 2**30:.3f} GiB, high water "
              f"{st['hbm_high_water'] / 2**30:.3f} GiB", flush=True)
    assert free[2] == free[1]
    srv.close()


# --------------------------------------------------- column-stream kernel --

_STREAM_CASES = [
    ("c1-hard", lambda: workloads.plain_c1(centroid_std=0.15, seed=31)),
    ("c4-shape", lambda: workloads.batched_c4(n_groups=24, size_hi=150, centroid_std=0.3, seed=32)),
    ("c2-shape", lambda: workloads.within_c2(n_items=4000, centroid_std=0.1, seed=33)),
    ("c3-shape", lambda: workloads.across_c3(n_items=3000, centroid_std=0.1, seed=34)),
    ("len-1-to-64", lambda: workloads.batched_c4(n_groups=10, size_hi=70, len_lo=1, len_hi=64, dim=64,
                                                 centroid_std=0.3, seed=35)),
    ("len-1", lambda: workloads.batched_c4(n_groups=10, size_hi=70, len_lo=1, len_hi=1, dim=64,
                                           centroid_std=0.3, seed=36)),
    ("dim-33", lambda: workloads.plain_c1(dim=33, centroid_std=0.2, seed=37)),
]


@pytest.mark.parametrize("name,make", _STREAM_CASES, ids=[c[0] for c in _STREAM_CASES])
@pytest.mark.parametrize("cols,bpc", [(1024, 2), (512, 0)])
def test_stream_kernel_exact(name, make, cols, bpc):
    """The column-stream kernel (segments of 512 or 1024 frames per wave, a
    persistent grid or a wave per segment): every cell equals the oracle's,
    robust pairs within margin / 2, with both DTW normalisations."""
    w = make()
    check(w, fused_cols=cols, fused_blocks_per_cu=bpc)
    if name in ("c1-hard", "len-1-to-64"):
        check(w, norm="none", fused_cols=cols, fused_blocks_per_cu=bpc)


# ------------------------------------------------- near-parallel frames --

def _with_twins(w, eps, frac=0.5, seed=0):
    """w plus a perturbed copy of a random `frac` of its items: the copy has
    the item's attributes and its frames times (1 + eps N(0, 1)) per value
    (eps = 0: exact copies), so the BY groups hold pairs of nearly parallel
    frames all along their DTW paths."""
    rng = np.random.default_rng(seed)
    src = np.sort(rng.choice(w.n_items, int(frac * w.n_items), replace=False))
    feats = w.features.float().cpu()
    parts, lens = [feats], list(np.diff(w.offsets))
    g = torch.Generator().manual_seed(seed)
    for i in src:
        f = feats[int(w.offsets[i]):int(w.offsets[i + 1])]
        parts.append(f * (1.0 + eps * torch.randn(f.shape, generator=g)))
        lens.append(len(f))
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    attrs = np.concatenate([w.attrs, w.attrs[src]]).astype(np.int32)
    return workloads.Workload(f"{w.name}-twins{eps}", torch.cat(parts).contiguous(), off, attrs,
                              list(w.attr_names), w.on, list(w.by), list(w.across),
                              [list(l) for l in w.levels], w.seed)


@pytest.mark.parametrize("dim", [768, 1024, 1280])
@pytest.mark.parametrize("eps", [0.0, 1e-4, 1e-3])
def test_near_parallel_frames_exact(dim, eps):
    """Items and slightly perturbed copies of them (frames at angles of about
    eps rad, down to exact copies), at the high dims where the margin is
    smallest: acos of a BF16 cosine is off by up to about 1e-4 there, so the
    kernels must flag these pairs for the FP64 recheck; every cell equals the
    oracle's, in DTW and in pooled mode."""
    base = workloads.within_c2(n_items=900, dim=dim, centroid_std=0.1, seed=50 + dim)
    w = _with_twins(base, eps, seed=int(eps * 1e5) + dim)
    _, res, _ = check(w)
    st = res.stats
    print(f"  nonrobust={st['n_nonrobust_pairs']} recheck={st['n_recheck_pairs']}", flush=True)
    assert st["n_nonrobust_pairs"] > 0
    check(w, mode="pooled")


@pytest.mark.parametrize("eps", [0.0, 1e-4])
def test_near_parallel_long_items_exact(eps):
    """Items of 17-64 frames and their (near) copies at dim 1024: the FP64
    recheck takes such pairs (more than 256 frame pairs) as register tiles of
    2 x 2 or 4 x 4 frame pairs, and frame pairs whose cosine is within 2^-20
    of +-1 go to its half-chord pass; every cell equals the oracle's."""
    base = workloads.batched_c4(n_groups=6, size_lo=4, size_hi=8, len_lo=17, len_hi=64, dim=1024,
                                centroid_std=0.1, seed=72, dtype=torch.float32)
    w = _with_twins(base, eps, seed=9)
    _, res, _ = check(w)
    st = res.stats
    print(f"  nonrobust={st['n_nonrobust_pairs']} recheck={st['n_recheck_pairs']}", flush=True)
    assert st["n_recheck_pairs"] > 0


# ---------------------------------------------------------------- subsampler --

@pytest.mark.parametrize("spec", ["within", "across"])
def test_subsampled_tasks_match_oracle(spec):
    """Subsampled tasks (caps on A, B, X per cell; at most 2 ACROSS values of x):
    every kept cell's W equals the oracle's on the same draws, and caps that
    bind nowhere give the full task's counts."""
    if spec == "within":
        w = workloads.within_c2(n_items=3000, dim=128, centroid_std=0.1, seed=61)
        subs = [dict(seed=3, max_a=3, max_b=4), dict(seed=4, max_a=2, max_b=1, max_x=5)]
    else:
        w = workloads.across_c3(n_items=2500, dim=128, centroid_std=0.1, seed=62)
        subs = [dict(seed=5, max_a=3, max_b=3, max_x=2, max_x_across=2), dict(seed=6, max_x=1, max_x_across=1)]
    feats = w.features.to("cuda").contiguous()
    ds = fx.Dataset(ctx(), feats, w.offsets, w.attrs)
    host = w.features_f32_host()
    for sub in subs:
        _say(f"subsampled {spec} {sub}")
        t = fx.Task(ds, w.on, w.by, w.across, subsampler=fx.Subsampler(**sub))
        res = t.score()
        orc = oracle.score(host, w.offsets, w.attrs, w.on, w.by, w.across, subsampler=sub)
        assert np.array_equal(t.keys, orc.keys.astype(np.int32))
        assert np.array_equal(t.sizes[0], orc.n_triplets)
        mism = int(np.count_nonzero(res.half_units != orc.half_units))
        print(f"  cells={len(t)} triplets={int(orc.n_triplets.sum())} mism={mism} "
              f"err={res.collapse(w.levels):.5f} oracle={oracle.error_rate(orc, w.levels):.5f}", flush=True)
        assert mism == 0
        assert abs(res.collapse(w.levels) - oracle.error_rate(orc, w.levels)) <= 1e-12
    big = fx.Subsampler(seed=1, max_a=10 ** 6, max_b=10 ** 6, max_x=10 ** 6, max_x_across=10 ** 6)
    full = fx.Task(ds, w.on, w.by, w.across).score().half_units
    assert np.array_equal(fx.Task(ds, w.on, w.by, w.across, subsampler=big).score().half_units, full)
