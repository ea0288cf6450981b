"""Pins of the oracle's distance for discrete units (the paper says ABX works
with dense or discrete representations and gives no distance for the
latter; the reading: frames are unit codes and the frame distance is 0 for
equal codes, 1 otherwise, in DTW mode).

* Closed forms: equal codes 0, different codes 1; DTW of a sequence with
  itself 0; DTW of two sequences with no common unit: mean 1 (path-normalised)
  and max(N, M) (raw cost, the fewest cells a monotone path can have).
* A hand-worked cell whose count is fixed by the definition.
* The angular distance between one-hot encodings of the codes is exactly half
  the unit mismatch (theta = pi / 2 or 0), and DTW is linear in the distance,
  so the per-cell counts of the two scorings are equal: checked on random
  tasks with and without ACROSS, both normalisations.
"""
import numpy as np
import pytest

import oracle


def test_unit_frame_distance_closed_forms():
    assert oracle.frame_distance([3.0], [3.0], "units") == 0.0
    assert oracle.frame_distance([3.0], [4.0], "units") == 1.0
    with pytest.raises(ValueError):
        oracle.frame_distance([1.0, 2.0], [1.0, 2.0], "units")   # unit codes have dim 1


def _dtw_units(x, y, norm):
    d = (np.asarray(x, np.float64)[:, None] != np.asarray(y, np.float64)[None, :]).astype(np.float64)
    return oracle.dtw(d, norm)


def test_unit_dtw_closed_forms():
    rng = np.random.default_rng(1)
    for _ in range(20):
        x = rng.integers(0, 5, int(rng.integers(1, 12)))
        assert _dtw_units(x, x, "path")[0] == 0.0 and _dtw_units(x, x, "none")[0] == 0.0
        y = rng.integers(5, 9, int(rng.integers(1, 12)))          # no unit in common with x
        assert _dtw_units(x, y, "path")[0] == 1.0
        assert _dtw_units(x, y, "none")[0] == float(max(len(x), len(y)))


def test_hand_worked_unit_cell():
    """Label 0: x = (1, 1, 2) and a = (1, 2, 2); label 1: b = (3, 3); one
    context.  x and a align at zero cost (1-1, 1-1, 2-2, 2-2), and every frame
    of b differs from every frame of x and a, so d(x, a) = d(a, x) = 0 <
    d(x, b) = d(a, b) = 1.  The cell (0, 1) has A = X = {x, a}, B = {b}: the
    triples (a, b, x) and (x, b, a), each won, W = 2 + 2 = 4 of 2 |C| = 4.
    The cell (1, 0) has a single item in A = X, so no triple."""
    codes = np.array([1, 1, 2, 1, 2, 2, 3, 3], np.float32)[:, None]
    offsets = np.array([0, 3, 6, 8], np.int64)
    attrs = np.array([[0, 0], [0, 0], [1, 0]], np.int32)
    for norm in ("path", "none"):
        r = oracle.score(codes, offsets, attrs, 0, [1], [], "dtw", norm, distance="units")
        assert [tuple(k) for k in r.keys] == [(0, 1, 0)]
        assert list(r.n_triplets) == [2] and list(r.half_units) == [4]


@pytest.mark.parametrize("across", [False, True])
@pytest.mark.parametrize("norm", ["path", "none"])
def test_units_equal_angular_on_one_hot(across, norm):
    rng = np.random.default_rng(7 + across)
    n, vocab = 60, 6
    lens = rng.integers(1, 9, n)
    offsets = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    label = rng.integers(0, 3, n)
    ctx = rng.integers(0, 2, n)
    spk = rng.integers(0, 3, n)
    attrs = np.stack([label, ctx, spk], axis=1).astype(np.int32)
    # codes leaning on a per-label unit, so the error is neither 0 nor 1/2
    codes = np.where(rng.random(int(offsets[-1])) < 0.5, np.repeat(label, lens),
                     rng.integers(0, vocab, int(offsets[-1])))
    onehot = np.eye(vocab, dtype=np.float32)[codes]
    by, acr = ([1], [2]) if across else ([1, 2], [])
    ru = oracle.score(codes.astype(np.float32)[:, None], offsets, attrs, 0, by, acr, "dtw", norm,
                      distance="units")
    ra = oracle.score(onehot, offsets, attrs, 0, by, acr, "dtw", norm, distance="angular")
    assert np.array_equal(ru.keys, ra.keys)
    assert np.array_equal(ru.half_units, ra.half_units)
    assert 0.0 < oracle.error_rate(ru) < 0.5
