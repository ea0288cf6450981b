"""Host-side tests of the C-ABI library (no GPU needed).

* the shared library loads and exports every function include/fastabx.h declares;
* a host-only context (device -1) builds tasks: the cells (keys, |A|, |B|, |X|,
  |C|) equal the oracle's, on random tables and on the workload shapes;
* argument errors return the documented status codes and set the message.
"""
import os
import re

import numpy as np
import pytest

import oracle
import workloads
import paper_2505_02692_amd as fx
from paper_2505_02692_amd import _lib as L

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "fastabx.h")


def _declared_functions():
    src = open(HEADER).read()
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(fabx_\w+)\s*\(", src)))


def test_library_exports_every_declared_symbol():
    lib = fx.lib()
    names = _declared_functions()
    assert len(names) >= 25
    missing = [n for n in names if not hasattr(lib, n)]
    assert missing == []
    assert set(names) == set(L.SIGNATURES)          # the binding declares exactly the ABI
    assert lib.fabx_version().decode().startswith("fastabx-hip")


def _host_task(attrs, on, by, across, lengths=None):
    ctx = fx.Context(-1)
    n = attrs.shape[0]
    lengths = np.ones(n, np.int64) if lengths is None else lengths
    off = np.zeros(n + 1, np.int64)
    off[1:] = np.cumsum(lengths)
    ds = fx.Dataset(ctx, None, off, attrs)
    return fx.Task(ds, on, by, across)


def _compare_cells(attrs, on, by, across):
    t = _host_task(attrs, on, by, across)
    want = oracle.cells(attrs, on, by, across)
    assert len(t) == len(want)
    keys = t.keys
    nt, abx = t.sizes
    for k, c in enumerate(want):
        assert tuple(keys[k]) == tuple(int(v) for v in c.key)
        assert nt[k] == c.n_triplets
        assert tuple(abx[k]) == (len(c.A), len(c.B), len(c.X))


@pytest.mark.parametrize("seed", range(16))
def test_task_cells_match_oracle_random(seed):
    rng = np.random.default_rng(seed)
    n = int(rng.integers(5, 120))
    card = rng.integers(1, 6, size=5)
    attrs = np.stack([rng.integers(-3, -3 + k, size=n) for k in card], axis=1).astype(np.int32)
    specs = [(0, [], []), (0, [1], []), (0, [1, 2], []), (0, [1], [2]), (0, [], [1]),
             (0, [], [1, 2]), (3, [0], [1, 2]), (4, [3, 2, 1], [0])]
    on, by, across = specs[seed % len(specs)]
    _compare_cells(attrs, on, by, across)


def test_task_cells_match_oracle_wide_values():
    rng = np.random.default_rng(99)
    n = 300
    # many distinct values per column: the composite key needs > 64 bits
    attrs = np.stack([rng.integers(0, 3, size=n)] +
                     [rng.integers(-2**30, 2**30, size=n) // (2**27) for _ in range(6)], axis=1).astype(np.int32)
    _compare_cells(attrs, 0, [1, 2, 3], [4])


@pytest.mark.parametrize("make", [
    lambda: workloads.plain_c1(),
    lambda: workloads.within_c2(n_items=3000, dim=8),
    lambda: workloads.across_c3(n_items=3000, dim=8),
    lambda: workloads.batched_c4(n_groups=40, dim=8, size_hi=60),
])
def test_task_cells_match_oracle_workloads(make):
    w = make()
    _compare_cells(w.attrs, w.on, w.by, w.across)


def test_empty_task_is_valid():
    attrs = np.zeros((6, 2), np.int32)
    t = _host_task(attrs, 0, [1], [])
    assert len(t) == 0


@pytest.mark.parametrize("on,by,across", [(0, [0], []), (0, [1], [1]), (0, [7], []), (-1, [], []),
                                          (0, [1, 2], [2])])
def test_task_spec_errors(on, by, across):
    attrs = np.zeros((6, 3), np.int32)
    with pytest.raises(fx.FabxError) as e:
        _host_task(attrs, on, by, across)
    assert e.value.code == L.FABX_EINVAL
    assert fx.lib().fabx_last_error().decode() != ""


def test_dataset_errors():
    ctx = fx.Context(-1)
    attrs = np.zeros((3, 1), np.int32)
    for off in ([0, 1, 1, 2], [1, 2, 3, 4], [0, 2, 1, 3]):       # empty item, bad start, decreasing
        with pytest.raises(fx.FabxError) as e:
            fx.Dataset(ctx, None, np.array(off), attrs)
        assert e.value.code == L.FABX_EINVAL
    with pytest.raises(fx.FabxError):
        fx.fabx_dataset_create(ctx.h, None, L.FABX_DTYPE_F32, 3, 0, np.array([0, 1, 2, 3]), attrs)
    with pytest.raises(fx.FabxError):
        fx.fabx_dataset_create(ctx.h, None, 7, 3, 4, np.array([0, 1, 2, 3]), attrs)


def test_bad_device_and_host_only_score():
    with pytest.raises(fx.FabxError) as e:
        fx.fabx_create(-5, None)
    assert e.value.code == L.FABX_EINVAL
    t = _host_task(np.array([[0], [0], [1]], np.int32), 0, [], [])
    with pytest.raises(fx.FabxError) as e:
        t.score()
    assert e.value.code == L.FABX_EINVAL
    for call in (t.score_async, t.autotune):                 # no device: refused, nothing launched
        with pytest.raises(fx.FabxError) as e:
            call()
        assert e.value.code == L.FABX_EINVAL
    assert fx.lib().fabx_autotune(t.h, None, None) == L.FABX_EINVAL
    assert fx.lib().fabx_result_wait(None) == L.FABX_EINVAL


def test_bad_score_options():
    t = _host_task(np.array([[0], [0], [1]], np.int32), 0, [], [])
    o = fx.make_opts()
    o.mode = 9
    with pytest.raises(fx.FabxError) as e:
        fx.fabx_score(t.h, o)
    assert e.value.code == L.FABX_EINVAL
    o = fx.make_opts()
    o.distance = 3
    with pytest.raises(fx.FabxError):
        fx.fabx_score(t.h, o)
    # the streaming DTW kernel computes the angular distance only
    with pytest.raises(fx.FabxError) as e:
        fx.fabx_score(t.h, fx.make_opts(distance="euclidean", precision="bf16", fused_cols=1024))
    assert e.value.code == L.FABX_EINVAL and "angular distance only" in str(e.value)
    # the Euclidean BF16 form passes the option checks (no device here)
    with pytest.raises(fx.FabxError) as e:
        fx.fabx_score(t.h, fx.make_opts(distance="euclidean", precision="bf16"))
    assert e.value.code == L.FABX_EINVAL and "no device" in str(e.value)
    # a forced fused-kernel configuration must be one the kernel has
    for cols, bpc, msg in ((100, 0, "fused_cols"), (128, -1, "fused_blocks_per_cu"),
                           (256, 65, "fused_blocks_per_cu")):
        with pytest.raises(fx.FabxError) as e:
            fx.fabx_score(t.h, fx.make_opts(fused_cols=cols, fused_blocks_per_cu=bpc))
        assert e.value.code == L.FABX_EINVAL and msg in str(e.value)


def test_score_opts_layout_and_defaults():
    """The ctypes mirror of fabx_score_opts matches the C defaults field by field."""
    o = fx.fabx_score_opts_default()
    assert (o.mode, o.precision, o.dtw_norm, o.keep_pairs) == (L.FABX_MODE_DTW, L.FABX_PREC_BF16_RECHECK,
                                                                L.FABX_NORM_PATH, 0)
    assert (o.margin, o.delta, o.fused_cols, o.fused_blocks_per_cu) == (-1.0, -1.0, 0, 0)
    o2 = fx.make_opts(fused_cols=256, fused_blocks_per_cu=2)
    assert (o2.fused_cols, o2.fused_blocks_per_cu) == (256, 2)


def test_item_length_limits_in_dtw_mode():
    """Items above FABX_MAX_ITEM_FRAMES are rejected in DTW mode; items of
    65..FABX_MAX_ITEM_FRAMES frames pass the option checks except with the
    streaming kernel (fused_cols >= 512), which takes at most 64 frames."""
    attrs = np.array([[0], [0], [1]], np.int32)
    t = _host_task(attrs, 0, [], [], lengths=np.array([3, L.FABX_MAX_ITEM_FRAMES + 1, 2]))
    with pytest.raises(fx.FabxError) as e:
        t.score(mode="dtw")
    assert e.value.code == L.FABX_EINVAL and "FABX_MAX_ITEM_FRAMES" in str(e.value)
    t = _host_task(attrs, 0, [], [], lengths=np.array([3, 65, 2]))
    with pytest.raises(fx.FabxError) as e:
        t.score(mode="dtw", fused_cols=512)
    assert e.value.code == L.FABX_EINVAL and "at most 64 frames" in str(e.value)
    with pytest.raises(fx.FabxError) as e:   # past the option checks: no device here
        t.score(mode="dtw")
    assert e.value.code == L.FABX_EINVAL and "no device" in str(e.value)


def test_null_handles():
    lib = fx.lib()
    assert lib.fabx_task_num_cells(None) == -1
    assert lib.fabx_score(None, None, None) == L.FABX_EINVAL
    assert lib.fabx_collapse(None, None, None, 0, None) == L.FABX_EINVAL
    assert lib.fabx_server_poll(None, 1, None) == L.FABX_EINVAL
    lib.fabx_destroy(None)
    lib.fabx_result_free(None)


def test_concurrent_task_builds_agree():
    """Task builds from several threads at once (the host pool runs a region
    inline when its workers are busy) give the same cells as one build."""
    from concurrent.futures import ThreadPoolExecutor
    import workloads
    w = workloads.within_c2(n_items=20000, dim=8, seed=5)
    ctx = fx.Context(-1)
    ds = fx.Dataset(ctx, None, w.offsets, w.attrs)
    ref = fx.Task(ds, w.on, w.by, w.across)
    ref_keys, ref_sizes = ref.keys, ref.sizes[0]
    def build(_):
        t = fx.Task(ds, w.on, w.by, w.across)
        return t.keys, t.sizes[0]
    with ThreadPoolExecutor(4) as ex:
        for keys, sizes in ex.map(build, range(12)):
            assert np.array_equal(keys, ref_keys) and np.array_equal(sizes, ref_sizes)


def test_thread_serial_switch():
    """fabx_set_thread_serial is per thread and returns the previous setting;
    task builds from a serial thread (beside builds on the pool) give the same
    cells."""
    from concurrent.futures import ThreadPoolExecutor
    import workloads
    w = workloads.within_c2(n_items=20000, dim=8, seed=6)
    ds = fx.Dataset(fx.Context(-1), None, w.offsets, w.attrs)
    ref = fx.Task(ds, w.on, w.by, w.across)
    ref_keys, ref_sizes = ref.keys, ref.sizes[0]
    assert fx.fabx_set_thread_serial(True) is False
    assert fx.fabx_set_thread_serial(True) is True
    t = fx.Task(ds, w.on, w.by, w.across)
    assert np.array_equal(t.keys, ref_keys) and np.array_equal(t.sizes[0], ref_sizes)
    assert fx.fabx_set_thread_serial(False) is True
    def serial_build(_):
        fx.fabx_set_thread_serial(True)
        t = fx.Task(ds, w.on, w.by, w.across)
        return t.keys, t.sizes[0]
    with ThreadPoolExecutor(1) as side:
        futs = [side.submit(serial_build, k) for k in range(3)]
        for _ in range(3):
            t = fx.Task(ds, w.on, w.by, w.across)  # on the pool, beside the serial builds
            assert np.array_equal(t.keys, ref_keys)
        for f in futs:
            keys, sizes = f.result()
            assert np.array_equal(keys, ref_keys) and np.array_equal(sizes, ref_sizes)
    assert fx.fabx_set_thread_serial(False) is False  # this thread's setting is its own


# ------------------------------------------------------------- subsampler --

@pytest.mark.parametrize("seed", range(12))
def test_subsampled_task_cells_match_oracle(seed):
    """The library's Subsampler (host task build) gives the oracle's subsampled
    cells: same kept cells in the same order, same capped |A|, |B|, |X| and
    |C| (the sets themselves are compared through the GPU scores)."""
    rng = np.random.default_rng(100 + seed)
    n = int(rng.integers(40, 400))
    card = rng.integers(2, 7, size=4)
    attrs = np.stack([rng.integers(0, k, size=n) for k in card], axis=1).astype(np.int32)
    specs = [(0, [1], []), (0, [1], [2]), (0, [], [1, 2]), (0, [1, 2], []), (3, [0], [1])]
    on, by, across = specs[seed % len(specs)]
    caps = [dict(max_a=2, max_b=3, max_x=2), dict(max_a=3), dict(max_b=1, max_x_across=2),
            dict(max_a=4, max_b=4, max_x=1, max_x_across=1), dict(max_x=3), dict()][seed % 6]
    sub = dict(seed=seed * 7919 + 1, **caps)
    ctx = fx.Context(-1)
    lengths = np.ones(n, np.int64)
    off = np.zeros(n + 1, np.int64)
    off[1:] = np.cumsum(lengths)
    ds = fx.Dataset(ctx, None, off, attrs)
    t = fx.Task(ds, on, by, across, subsampler=fx.Subsampler(**sub))
    want = oracle.subsample(oracle.cells(attrs, on, by, across), len(across), **sub)
    assert len(t) == len(want)
    keys = t.keys
    nt, abx = t.sizes
    for k, c in enumerate(want):
        assert tuple(keys[k]) == tuple(int(v) for v in c.key)
        assert nt[k] == c.n_triplets
        assert tuple(abx[k]) == (len(c.A), len(c.B), len(c.X))


def test_subsampler_rejects_negative_caps():
    ctx = fx.Context(-1)
    attrs = np.array([[0, 0], [0, 0], [1, 0]], np.int32)
    ds = fx.Dataset(ctx, None, np.arange(4, dtype=np.int64), attrs)
    with pytest.raises(fx.FabxError) as e:
        fx.Task(ds, 0, [1], [], subsampler=fx.Subsampler(max_a=-1))
    assert e.value.code == -1


def test_unit_code_datasets_and_their_distance():
    """Discrete units: int32 codes with dim 1, scored with FABX_DISTANCE_UNITS
    in DTW mode only; the distance and the dtype go together."""
    ctx = fx.Context(-1)
    attrs = np.array([[0], [0], [1]], np.int32)
    off = np.array([0, 2, 5, 6], np.int64)
    with pytest.raises(fx.FabxError) as e:
        fx.fabx_dataset_create(ctx.h, None, L.FABX_DTYPE_UNITS, 12, 2, off * 2, attrs)
    assert e.value.code == L.FABX_EINVAL and "dim 1" in str(e.value)
    h = fx.fabx_dataset_create(ctx.h, None, L.FABX_DTYPE_UNITS, 6, 1, off, attrs)
    t = fx.fabx_task_create(h, 0, [], [])
    for kw, msg in ((dict(distance="angular"), "FABX_DISTANCE_UNITS"),
                    (dict(distance="units", mode="pooled"), "DTW mode only"),
                    (dict(distance="units"), "no device")):
        with pytest.raises(fx.FabxError) as e:
            fx.fabx_score(t, fx.make_opts(**kw))
        assert e.value.code == L.FABX_EINVAL and msg in str(e.value), (kw, str(e.value))
    t2 = _host_task(attrs, 0, [], [])
    with pytest.raises(fx.FabxError) as e:
        t2.score(distance="units")
    assert e.value.code == L.FABX_EINVAL and "FABX_DISTANCE_UNITS" in str(e.value)
