"""Item-file front end ("Slicing features" appendix): frame slicing of aligned
units, item files, and datasets whose items are windows of the features.

* The oracle's slicing is the set definition scanned frame by frame; it is
  pinned to hand-worked units.  The library's closed form (ceil / floor in
  FP64) is checked against it on dyadic units, where every time is exact and
  units start or end exactly on frame times, and on random units.
* A dataset of overlapping windows builds the same cells as a contiguous
  copy of those windows (host-only context), and rejects bad windows.
"""
import os
import sys

import numpy as np
import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

import oracle  # noqa: E402
import paper_2505_02692_amd as fx  # noqa: E402
from paper_2505_02692_amd import _lib as L  # noqa: E402


def test_oracle_slicing_hand_worked():
    """dt = 1/64 s (dyadic, so FP64 is exact), frame times t_i = (2i + 1)/128 s.
    [t_0, t_2] keeps 0..2 (both ends on a frame time); [t_0 + e, t_2 - e]
    keeps 1 only; [0, t_0 / 2] keeps nothing; [t_1, t_4] keeps 1..4 and its
    Libri-Light slicing 1..3; [t_1, t_1] keeps 1 (none with Libri-Light)."""
    dt = 1 / 64
    t = lambda i: (2 * i + 1) / 128
    assert oracle.slice_frames(t(0), t(2), dt) == (0, 3)
    assert oracle.slice_frames(t(0) + 1 / 1024, t(2) - 1 / 1024, dt) == (1, 1)
    assert oracle.slice_frames(0.0, t(0) / 2, dt) == (0, 0)
    assert oracle.slice_frames(t(1), t(4), dt) == (1, 4)
    assert oracle.slice_frames(t(1), t(4), dt, libri_light=True) == (1, 3)
    assert oracle.slice_frames(t(1), t(1), dt) == (1, 1)
    assert oracle.slice_frames(t(1), t(1), dt, libri_light=True)[1] == 0


def _check_against_oracle(onset, offset, dt):
    for ll in (False, True):
        start, length = fx.fabx_slice_frames(onset, offset, dt, ll)
        for k in range(len(onset)):
            s0, n0 = oracle.slice_frames(onset[k], offset[k], dt, ll)
            assert length[k] == n0, (k, onset[k], offset[k], ll)
            if n0:
                assert start[k] == s0, (k, onset[k], offset[k], ll)


def test_slice_frames_dyadic_units_match_definition():
    """Units on a 1/512 s grid with dt = 1/64 s: every frame time is on the grid,
    so many units start or end exactly on one, and FP64 is exact throughout."""
    rng = np.random.default_rng(71)
    a = rng.integers(0, 512, 400)
    b = a + rng.integers(0, 160, 400)
    _check_against_oracle(a / 512, b / 512, 1 / 64)


def test_slice_frames_random_units_match_definition():
    rng = np.random.default_rng(72)
    for dt in (0.01, 0.02, 0.04, 0.08):
        a = rng.uniform(0, 5, 300)
        b = a + rng.uniform(0, 0.5, 300)
        _check_against_oracle(a, b, dt)


@pytest.mark.parametrize("onset,offset,dt", [(0.2, 0.1, 0.02), (-0.1, 0.1, 0.02), (0.0, 0.1, 0.0),
                                             (0.0, float("nan"), 0.02), (0.0, 0.1, float("inf"))])
def test_slice_frames_rejects_bad_units(onset, offset, dt):
    with pytest.raises(fx.FabxError) as e:
        fx.fabx_slice_frames([onset], [offset], dt)
    assert e.value.code == L.FABX_EINVAL


def _write_items(path, rows):
    with open(path, "w") as f:
        f.write("#file onset offset #phone prev-phone next-phone speaker\n")
        for r in rows:
            f.write(" ".join(str(v) for v in r) + "\n")


def test_read_item_file(tmp_path):
    p = str(tmp_path / "a.item")
    _write_items(p, [("u1", 0.01, 0.09, "ah", "b", "k", "s1"), ("u2", 0.0, 0.05, "eh", "#", "t", "s2")])
    names, files, on, off, vals = fx.read_item_file(p)
    assert names == ["phone", "prev-phone", "next-phone", "speaker"]
    assert files == ["u1", "u2"] and list(on) == [0.01, 0.0] and list(off) == [0.09, 0.05]
    assert vals[1] == ["eh", "#", "t", "s2"]
    with open(p, "a") as f:
        f.write("u3 0.1 0.2 ah b\n")
    with pytest.raises(ValueError):
        fx.read_item_file(p)


def test_overlapping_windows_build_the_cells_of_a_copy():
    """Items as overlapping windows of one frame array give the same cells
    (keys, sizes) as a contiguous copy of the windows."""
    import torch
    rng = np.random.default_rng(73)
    n_frames, n_items = 500, 120
    start = rng.integers(0, n_frames - 30, n_items)
    length = rng.integers(1, 30, n_items)
    attrs = np.stack([rng.integers(0, 4, n_items), rng.integers(0, 3, n_items)], 1).astype(np.int32)
    feats = torch.zeros(n_frames, 8)
    ctx = fx.Context(-1)
    dw = fx.Dataset.windows(ctx, feats, start, length, attrs)
    off = np.concatenate([[0], np.cumsum(length)]).astype(np.int64)
    dc = fx.Dataset(ctx, None, off, attrs)
    for on, by in ((0, [1]), (1, [0]), (0, [])):
        tw, tc = fx.Task(dw, on, by, []), fx.Task(dc, on, by, [])
        assert np.array_equal(tw.keys, tc.keys)
        assert np.array_equal(tw.sizes[0], tc.sizes[0]) and np.array_equal(tw.sizes[1], tc.sizes[1])


@pytest.mark.parametrize("start,length", [([0, 5], [3, 0]), ([0, -1], [3, 2]), ([0, 9], [3, 2])])
def test_bad_windows_are_rejected(start, length):
    import torch
    with pytest.raises(fx.FabxError) as e:
        fx.Dataset.windows(fx.Context(-1), torch.zeros(10, 4), np.array(start), np.array(length),
                           np.zeros((2, 1), np.int32))
    assert e.value.code == L.FABX_EINVAL


def test_zerospeech_abx_checks_arguments_and_columns(tmp_path):
    import torch
    p = str(tmp_path / "a.item")
    with open(p, "w") as f:
        f.write("#file onset offset #phone speaker\nu1 0.0 0.1 a s1\n")
    feats = {"u1": torch.zeros(10, 4)}
    ctx = fx.Context(-1)
    with pytest.raises(ValueError, match="speaker"):
        fx.zerospeech_abx(ctx, p, feats, 0.02, speaker="both")
    with pytest.raises(ValueError, match="context"):
        fx.zerospeech_abx(ctx, p, feats, 0.02, context="none")
    with pytest.raises(ValueError, match="prev-phone"):
        fx.zerospeech_abx(ctx, p, feats, 0.02)              # context 'within' needs the context columns
    with pytest.raises(ValueError, match="no features"):
        fx.zerospeech_abx(ctx, p, {}, 0.02, context="any")
