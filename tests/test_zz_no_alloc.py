"""fabx_score_noalloc (the score for callers that cannot allocate) against
fabx_score, through the C ABI: the per-cell counts must be identical, on two
calls in a row, the second with a smaller task than the first (the scratch
array keeps the first call's contents), for every form of the score."""
import ctypes

import numpy as np
import pytest
import torch

import workloads
import paper_2505_02692_amd as fx
from paper_2505_02692_amd import _lib as L

pytestmark = pytest.mark.gpu


def _say(msg):
    print(f"[case] {msg}", flush=True)


_CTX = {}


def ctx():
    if "c" not in _CTX:
        _CTX["c"] = fx.Context(0)
    return _CTX["c"]


def _task(w):
    ds = fx.Dataset(ctx(), w.features.to("cuda").contiguous(), w.offsets, w.attrs)
    return ds, fx.Task(ds, w.on, w.by, w.across)


@pytest.mark.parametrize("mode,precision,norm,distance", [
    ("dtw", "bf16", "path", "angular"), ("dtw", "bf16", "none", "angular"), ("dtw", "fp32", "path", "angular"),
    ("pooled", "bf16", "path", "angular"), ("pooled", "fp32", "path", "angular"),
    ("dtw", "bf16", "path", "euclidean"), ("pooled", "bf16", "path", "euclidean")])
def test_noalloc_equals_score_on_two_calls(mode, precision, norm, distance):
    big = workloads.within_c2(n_items=3000, dim=256, centroid_std=0.1, seed=7)
    small = workloads.plain_c1(centroid_std=0.15, seed=2)
    for w in (big, small):
        _say(f"noalloc {mode} {precision} {norm} {distance} {w.name} n_items={w.n_items}")
        ds, t = _task(w)
        ref = t.score(mode=mode, precision=precision, norm=norm, distance=distance)
        opts = fx.make_opts(mode=mode, precision=precision, norm=norm, distance=distance)
        got, st = fx.fabx_score_noalloc(t.h, opts, len(t))
        torch.cuda.synchronize()
        assert np.array_equal(got, ref.half_units)
        assert st["n_cells"] == len(t) and st["n_triplets"] == ref.stats["n_triplets"]
        assert st["n_recheck_pairs"] == ref.stats["n_recheck_pairs"]
        assert 0 < st["workspace_bytes"] <= L.FABX_NOALLOC_SCRATCH_BYTES


@pytest.mark.parametrize("precision", ["bf16", "fp32"])
def test_noalloc_with_items_over_64_frames(precision):
    """Pairs with an item of more than 64 frames take the FP64 kernel (BF16
    form) or row chunks (FP32 form); their slot list lives in the scratch too."""
    w = workloads.batched_c4(n_groups=10, size_lo=5, size_hi=16, len_lo=1, len_hi=200, dim=64,
                             centroid_std=0.3, seed=31)
    small = workloads.plain_c1(centroid_std=0.15, seed=2)
    for wl in (w, small):
        _say(f"noalloc long items {precision} {wl.name} n_items={wl.n_items}")
        ds, t = _task(wl)
        ref = t.score(precision=precision)
        got, st = fx.fabx_score_noalloc(t.h, fx.make_opts(precision=precision), len(t))
        torch.cuda.synchronize()
        assert np.array_equal(got, ref.half_units)


def test_noalloc_discrete_units():
    """Unit-code datasets (the packed codes and the distance tiles of the plain
    kernels) through the scratch array, on two calls in a row."""
    rng = np.random.default_rng(5)
    for n_items in (400, 90):
        _say(f"noalloc discrete units n_items={n_items}")
        lens = rng.integers(1, 40, n_items)
        off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
        label = rng.integers(0, 3, n_items)
        codes = np.where(rng.random(int(off[-1])) < 0.5, np.repeat(label, lens),
                         rng.integers(0, 20, int(off[-1]))).astype(np.int32)
        attrs = np.stack([label, rng.integers(0, 2, n_items)], axis=1).astype(np.int32)
        ds = fx.Dataset(ctx(), torch.tensor(codes, device="cuda"), off, attrs)
        t = fx.Task(ds, 0, [1], [])
        ref = t.score(distance="units")
        got, _ = fx.fabx_score_noalloc(t.h, fx.make_opts(distance="units"), len(t))
        torch.cuda.synchronize()
        assert np.array_equal(got, ref.half_units)


def test_noalloc_rejects_a_task_beyond_the_scratch():
    _say("noalloc: task over the scratch limit")
    w = workloads.within_c2(n_items=30000, dim=768, centroid_std=0.1, seed=8)
    ds, t = _task(w)
    with pytest.raises(fx.FabxError) as e:
        fx.fabx_score_noalloc(t.h, fx.make_opts(precision="fp32"), len(t))
    assert e.value.code == -2
    # the regular entry point has no such limit, and the no-allocation one
    # still works on a small task afterwards
    ref = t.score(precision="fp32")
    assert ref.stats["n_cells"] == len(t)
    w2 = workloads.plain_c1(seed=4)
    ds2, t2 = _task(w2)
    got, _ = fx.fabx_score_noalloc(t2.h, fx.make_opts(), len(t2))
    assert np.array_equal(got, t2.score().half_units)
