"""Pins of the FP64 oracle against facts fixed by the paper and by mathematics.

None of these tests re-types the oracle's formulas: each compares the oracle
with brute force, a closed form, a symmetry, or a value worked by hand (the
fixtures under tests/golden/ carry their derivations and citations).
"""
import itertools
import json
import math
import os

import numpy as np
import pytest

import oracle


# --------------------------------------------------------------- P1: DTW --

def _monotone_paths(N, M):
    """Every path from (0,0) to (N-1,M-1) using steps (1,0), (0,1), (1,1)."""
    out = []

    def rec(i, j, path):
        if i == N - 1 and j == M - 1:
            out.append(list(path))
            return
        for di, dj in ((1, 1), (0, 1), (1, 0)):
            ni, nj = i + di, j + dj
            if ni < N and nj < M:
                path.append((ni, nj))
                rec(ni, nj, path)
                path.pop()

    rec(0, 0, [(0, 0)])
    return out


def _forward_cost(d, path):
    s = d[path[0]]
    for p in path[1:]:
        s = s + d[p]
    return s


def _delannoy(m, n):
    return sum(math.comb(m, k) * math.comb(n, k) * 2 ** k for k in range(min(m, n) + 1))


@pytest.mark.parametrize("N,M", [(1, 1), (1, 4), (3, 1), (2, 2), (3, 5), (5, 4), (5, 5)])
def test_dtw_bruteforce_random(N, M):
    """P1(a): min over all monotone paths of the forward-summed cost equals the
    DTW cost bitwise, and the (unique) optimal path's length equals len."""
    rng = np.random.default_rng(N * 10 + M)
    paths = _monotone_paths(N, M)
    assert len(paths) == _delannoy(N - 1, M - 1)
    for _ in range(20):
        d = rng.random((N, M))
        costs = [_forward_cost(d, p) for p in paths]
        best = min(costs)
        v, L = oracle.dtw(d, norm="none")
        assert v == best
        winners = [p for p, c in zip(paths, costs) if c == best]
        assert len(winners) == 1
        assert L == len(winners[0])
        vp, Lp = oracle.dtw(d, norm="path")
        assert Lp == L and vp == best / L


def _backward_moves(path):
    """Moves into each cell, read from the end: 0 = diagonal, 1 = left (j-1), 2 = up (i-1)."""
    mv = []
    for (i0, j0), (i1, j1) in zip(path[:-1], path[1:]):
        mv.append({(1, 1): 0, (0, 1): 1, (1, 0): 2}[(i1 - i0, j1 - j0)])
    return mv[::-1]


@pytest.mark.parametrize("N,M", [(2, 3), (3, 3), (4, 5), (5, 5), (5, 3)])
def test_dtw_bruteforce_ties(N, M):
    """P1(b): on small-integer matrices (many exact ties) len is the length of the
    optimal path whose backward moves come first under diagonal < left < up."""
    rng = np.random.default_rng(100 + N * 10 + M)
    paths = _monotone_paths(N, M)
    n_tied = 0
    for _ in range(60):
        d = rng.integers(0, 3, size=(N, M)).astype(np.float64)
        costs = [_forward_cost(d, p) for p in paths]
        best = min(costs)
        winners = [p for p, c in zip(paths, costs) if c == best]
        n_tied += len({len(p) for p in winners}) > 1
        first = min(winners, key=_backward_moves)
        v, L = oracle.dtw(d, norm="none")
        assert v == best
        assert L == len(first)
    assert n_tied > 0  # the sample really exercises ties between path lengths


def test_dtw_worked_examples(golden_dir):
    with open(os.path.join(golden_dir, "dtw_worked.json")) as f:
        fx = json.load(f)
    for case in fx["cases"]:
        d = np.array(case["d"])
        v, L = oracle.dtw(d, norm="none")
        assert v == case["cost"] and L == case["len"]
        vp, _ = oracle.dtw(d, norm="path")
        assert vp == pytest.approx(case["path_normalised"], abs=0, rel=1e-15)


@pytest.mark.parametrize("k", [1, 3, 7])
@pytest.mark.parametrize("N,M", [(1, 1), (3, 8), (9, 2), (12, 12)])
def test_dtw_constant_matrix(k, N, M):
    """P3: d = 2^-k everywhere -> raw cost 2^-k max(N, M), normalised cost 2^-k."""
    d = np.full((N, M), 2.0 ** -k)
    v, L = oracle.dtw(d, norm="none")
    assert v == 2.0 ** -k * max(N, M) and L == max(N, M)
    assert oracle.dtw(d, norm="path")[0] == 2.0 ** -k


def test_dtw_single_row_or_column():
    """P4: one row (or column) -> the only path takes every cell: sum / mean."""
    vals = np.array([3, 1, 4, 1, 5, 9, 2, 6]) / 8.0          # dyadic: exact sums
    for d in (vals[None, :], vals[:, None]):
        v, L = oracle.dtw(d, norm="none")
        assert v == 31 / 8 and L == 8
        assert oracle.dtw(d, norm="path")[0] == 31 / 64


def test_dtw_raw_cost_symmetric():
    """P5: the raw cost is symmetric under swapping the two sequences, bitwise."""
    rng = np.random.default_rng(5)
    for _ in range(50):
        N, M = rng.integers(1, 30, size=2)
        d = rng.random((N, M))
        assert oracle.dtw(d, "none")[0] == oracle.dtw(np.ascontiguousarray(d.T), "none")[0]


# -------------------------------------------------------- P6: frame distance --

def test_frame_distance_closed_forms():
    rng = np.random.default_rng(6)
    for D in (2, 7, 64, 768):
        u = rng.standard_normal(D)
        assert oracle.frame_distance(u, u) == 0.0                 # parallel (identical)
        assert oracle.frame_distance(u, 4.0 * u) == 0.0           # parallel, scaled by a power of 2
        assert oracle.frame_distance(u, -u) == 1.0                # antiparallel
        v = np.zeros(D)
        w = np.zeros(D)
        v[: D // 2] = rng.standard_normal(D // 2)
        w[D // 2:] = rng.standard_normal(D - D // 2)
        assert oracle.frame_distance(v, w) == 0.5                 # orthogonal (disjoint supports)
    for phi in np.linspace(0.0, math.pi, 37):
        a = np.array([1.0, 0.0])
        b = np.array([math.cos(phi), math.sin(phi)])
        assert abs(oracle.frame_distance(a, b) - phi / math.pi) < 1e-15


def test_frame_distance_near_parallel_accuracy():
    """The half-chord branch keeps tiny angles accurate (acos alone would lose ~8 digits)."""
    for eps in (1e-3, 1e-6, 1e-9):
        a = np.array([1.0, 0.0, 0.0])
        b = np.array([math.cos(eps), math.sin(eps), 0.0])
        assert abs(oracle.frame_distance(a, b) - eps / math.pi) < 1e-15 * max(1.0, eps / math.pi) + 1e-18


# ---------------------------------------------------- P2 / pooled closed forms --

def _dataset(item_frames):
    feats = np.concatenate([np.asarray(f, np.float32).reshape(len(f), -1) for f in item_frames])
    off = np.zeros(len(item_frames) + 1, np.int64)
    off[1:] = np.cumsum([len(f) for f in item_frames])
    return feats, off


def test_identical_sequences_have_zero_distance():
    """P2: d(u, u) = 0 exactly, hence DTW(x, x) = 0 in both normalisations."""
    rng = np.random.default_rng(2)
    x = rng.standard_normal((7, 33)).astype(np.float32)
    y = rng.standard_normal((4, 33)).astype(np.float32)
    feats, off = _dataset([x, x.copy(), y])
    items = [np.arange(3)]
    pairs = [(np.array([0, 1, 0], np.int32), np.array([1, 0, 2], np.int32))]
    for norm in ("path", "none"):
        d = oracle.pair_distances(feats, off, items, pairs, "dtw", norm)[0]
        assert d[0] == 0.0 and d[1] == 0.0 and d[2] > 0.0
    d = oracle.pair_distances(feats, off, items, pairs, "pooled")[0]
    assert d[0] == 0.0 and d[1] == 0.0


def test_pooled_mean_closed_form():
    """Time pooling: the mean of frames (1,0) and (0,1) is at 45 deg from (1,0) -> 1/4."""
    feats, off = _dataset([[[1.0, 0.0], [0.0, 1.0]], [[3.0, 0.0]], [[0.0, 2.0], [0.0, 1.0], [0.0, 5.0]]])
    items = [np.arange(3)]
    pairs = [(np.array([0, 1, 0], np.int32), np.array([1, 2, 2], np.int32))]
    d = oracle.pair_distances(feats, off, items, pairs, "pooled")[0]
    assert abs(d[0] - 0.25) < 1e-15
    assert d[1] == 0.5
    assert abs(d[2] - 0.25) < 1e-15


# ------------------------------------------------ Euclidean distance (NEXT) --

def test_euclidean_frame_distance_closed_forms():
    """The "euclidean" distance named beside "angular" in the Score interface:
    the length of u - v.  A 3-4-5 triangle placed away from the origin (so
    |u + v| or a missing square root would fail), identity, symmetry,
    translation and power-of-two scale invariance, and a zero vector, which
    has a length but no angle."""
    e = lambda u, v: oracle.frame_distance(u, v, "euclidean")
    assert e([1.0, 1.0], [4.0, 5.0]) == 5.0
    assert e([0.0, 0.0, 0.0], [1.0, 2.0, 2.0]) == 3.0
    assert e([2.0, -1.0, 7.0, 3.0], [2.0, -1.0, 7.0, 3.0]) == 0.0
    rng = np.random.default_rng(61)
    for D in (2, 7, 64, 768):
        u = np.round(rng.standard_normal(D) * 64) / 64       # multiples of 1/64: sums stay exact
        v = np.round(rng.standard_normal(D) * 64) / 64
        t = np.round(rng.standard_normal(D) * 64) / 64
        d = e(u, v)
        assert d == e(v, u)
        assert d == e(u + t, v + t)
        assert e(4.0 * u, 4.0 * v) == 4.0 * d
        assert d == math.sqrt(float(np.sum((u - v) ** 2)))     # exact sums of exact squares here
        assert e(u, u) == 0.0


def test_euclidean_dtw_and_pooled_worked_examples():
    """Worked by hand.  x = [(0,0), (1,0)], y = [(0,0), (0,1), (1,1)]: frame
    distances [[0, 1, r2], [1, r2, 1]] (r2 = sqrt 2), cumulative costs
    [[0, 1, 1 + r2], [1, r2, 2]]; the last cell comes from the diagonal (0, 1),
    so the path is (0,0) (0,1) (1,2): raw cost 2, path length 3, distance 2/3.
    Pooled: the means (1/2, 0) and (1/3, 2/3) are sqrt(1/36 + 4/9) = sqrt(17)/6
    apart.  A zero frame is allowed."""
    x = [[0.0, 0.0], [1.0, 0.0]]
    y = [[0.0, 0.0], [0.0, 1.0], [1.0, 1.0]]
    feats, off = _dataset([x, y])
    items = [np.arange(2)]
    pairs = [(np.array([0, 1], np.int32), np.array([1, 0], np.int32))]
    raw = oracle.pair_distances(feats, off, items, pairs, "dtw", "none", "euclidean")[0]
    assert raw[0] == 2.0 and raw[1] == 2.0
    d = oracle.pair_distances(feats, off, items, pairs, "dtw", "path", "euclidean")[0]
    assert abs(d[0] - 2.0 / 3.0) < 1e-15 and abs(d[1] - 2.0 / 3.0) < 1e-15
    p = oracle.pair_distances(feats, off, items, pairs, "pooled", "path", "euclidean")[0]
    assert abs(p[0] - math.sqrt(17.0) / 6.0) < 1e-15 and p[0] == p[1]


def test_zero_frame_is_rejected():
    feats, off = _dataset([[[1.0, 0.0]], [[0.0, 0.0]]])
    with pytest.raises(ValueError):
        oracle.pair_distances(feats, off, [np.arange(2)], [(np.array([0], np.int32), np.array([1], np.int32))])


# ------------------------------------------------------------ P7: scoring --

def test_swap_a_and_b_complements():
    """P7: with X fixed, swapping A and B turns W into 2|X||A||B| - W exactly."""
    rng = np.random.default_rng(7)
    for _ in range(30):
        X = list(range(0, 4))
        A = list(range(10, 10 + rng.integers(1, 6)))
        B = list(range(20, 20 + rng.integers(1, 6)))
        dist = {}
        for x in X:
            for y in A + B:
                dist[(x, y)] = float(rng.integers(0, 4))           # many exact ties
        w = oracle.cell_half_units(dist, X, A, B, False)
        w_swapped = oracle.cell_half_units(dist, X, B, A, False)
        assert w + w_swapped == 2 * len(X) * len(A) * len(B)


def test_exact_copy_scores_one_half():
    """P7: b an exact copy of a -> every triple is a tie -> D_C = 1/2 exactly."""
    rng = np.random.default_rng(8)
    a = rng.standard_normal((5, 16)).astype(np.float32)
    xs = [rng.standard_normal((int(rng.integers(2, 7)), 16)).astype(np.float32) for _ in range(3)]
    feats, off = _dataset([a, a.copy()] + xs)
    # ON label, ACROSS speaker: a (label 0, spk 0), b (label 1, spk 0), x's (label 0, spk 1)
    attrs = np.array([[0, 0], [1, 0], [0, 1], [0, 1], [0, 1]], np.int32)
    res = oracle.score(feats, off, attrs, on=0, by=[], across=[1])
    keys = [c.key for c in res.cells]
    k = keys.index((0, 1, 0, 1))
    assert res.n_triplets[k] == 3 and res.half_units[k] == 3
    assert res.scores[k] == 0.5


# --------------------------------------------------- P9: tiny end to end --

def test_circle_golden(golden_dir):
    with open(os.path.join(golden_dir, "circle_cells.json")) as f:
        fx = json.load(f)
    feats, off = _dataset([[f] for f in fx["features"]])
    attrs = np.array(fx["labels"], np.int32)[:, None]
    res = oracle.score(feats, off, attrs, on=0, by=[], across=[])
    got = {c.key[:2]: (int(w), int(n)) for c, w, n in zip(res.cells, res.half_units, res.n_triplets)}
    want = {(c["on_ax"], c["on_b"]): (c["half_units"], c["n_triplets"]) for c in fx["cells"]}
    assert got == want
    assert oracle.error_rate(res) == pytest.approx(fx["error_weighted"], abs=1e-15)


# ------------------------------------------------------- P11: aggregation --

def test_collapse_hand_tables():
    """Weighted mean vs averaging level by level, worked by hand.

    Task ON phone BY context, speaker -> key columns (on_ax, on_b, ctx, spk).
    Cells (W, |C|): scores D_C = W / 2|C|.
      (0,1,c0,s0): 2/ (2*1) = 1     (0,1,c1,s0): 0/(2*3) = 0
      (0,1,c0,s1): 3/(2*3) = 1/2    (1,0,c0,s0): 6/(2*4) = 3/4
    levels [ctx], [spk]:
      after ctx: (0,1,s0) = (1+0)/2 = 1/2, (0,1,s1) = 1/2, (1,0,s0) = 3/4
      after spk: (0,1) = 1/2, (1,0) = 3/4; final D = 5/8 -> error 3/8
    weighted: (2+0+3+6) / (2*(1+3+3+4)) = 11/22 = 1/2 -> error 1/2
    """
    keys = np.array([[0, 1, 0, 0], [0, 1, 1, 0], [0, 1, 0, 1], [1, 0, 0, 0]])
    ka = [0, 0, 1, 2]
    W = np.array([2, 0, 3, 6])
    n = np.array([1, 3, 3, 4])
    assert oracle.collapse(keys, ka, W, n) == 0.5
    assert oracle.collapse(keys, ka, W, n, [[1], [2]]) == 3 / 8
    # collapsing both BY attributes at once: (0,1) = (1+0+1/2)/3 = 1/2, (1,0) = 3/4 -> 3/8
    assert oracle.collapse(keys, ka, W, n, [[1, 2]]) == 3 / 8
    # speaker first: (0,1,c0) = (1+1/2)/2 = 3/4, (0,1,c1) = 0, (1,0,c0) = 3/4;
    # then ctx: (0,1) = 3/8, (1,0) = 3/4 -> D = 9/16 -> error 7/16
    assert oracle.collapse(keys, ka, W, n, [[2], [1]]) == 7 / 16
    with pytest.raises(ValueError):
        oracle.collapse(keys, ka, W, n, [[0]])


def test_collapse_equal_scores_any_aggregation():
    """P11: when every D_C is equal, every aggregation returns it."""
    rng = np.random.default_rng(11)
    keys = rng.integers(0, 3, size=(40, 5))
    keys = np.unique(keys, axis=0)
    n = rng.integers(1, 9, size=len(keys))
    W = n.copy()                                  # every D_C = 1/2
    for lv in (None, [[1]], [[1], [2, 3]], [[3], [1], [2]]):
        assert oracle.collapse(keys, [0, 0, 1, 2, 3], W, n, lv) == 0.5


def test_collapse_across_level_hand_table():
    """Z14 / P11: an ACROSS attribute named in a collapse level removes its
    ``_ab`` and ``_x`` key columns together, in one averaging pass (Background:
    averaged over contexts, then speakers, then phonemes; Score.collapse).

    Task ON phone BY context ACROSS speaker -> key columns
    (on_ax, on_b, ctx, spk_ab, spk_x).  Cells (W, |C|) -> D_C = W / 2|C|:
      (0,1,c0,s0,s1) 1/1 -> 1/2     (0,1,c0,s0,s2) 1/3 -> 1/6
      (0,1,c0,s1,s0) 2/3 -> 1/3     (0,1,c1,s0,s1) 1/4 -> 1/8
      (1,0,c0,s1,s0) 2/4 -> 1/4     (0,1,c0,s2,s1) 3/4 -> 3/8
      (1,0,c1,s1,s2) 3/2 -> 3/4
    levels [ctx], [spk]:
      after ctx: (0,1,s0,s1) = (1/2 + 1/8)/2 = 5/16, (0,1,s0,s2) = 1/6,
                 (0,1,s1,s0) = 1/3, (0,1,s2,s1) = 3/8,
                 (1,0,s1,s0) = 1/4, (1,0,s1,s2) = 3/4
      after spk (spk_ab and spk_x together):
                 (0,1) = (5/16 + 1/6 + 1/3 + 3/8)/4 = 19/64, (1,0) = (1/4 + 3/4)/2 = 1/2
      D = (19/64 + 1/2)/2 = 51/128 -> error 77/128
    weighted: sum W / (2 sum |C|) = 13/42 -> error 29/42 (differs from the levels).

    Plausible mistakes give other values on this table, so each fails here:
    dropping only spk_ab -> 101/160, only spk_x -> 245/384; removing spk_ab then
    spk_x in two passes -> 39/64, spk_x then spk_ab -> 341/576; the speaker level
    before the context level -> 81/128; both levels in one pass -> 3/5.
    """
    keys = np.array([[0, 1, 0, 0, 1], [0, 1, 0, 0, 2], [0, 1, 0, 1, 0], [0, 1, 1, 0, 1],
                     [1, 0, 0, 1, 0], [0, 1, 0, 2, 1], [1, 0, 1, 1, 2]])
    ka = [0, 0, 1, 2, 2]
    W = np.array([1, 1, 2, 1, 2, 3, 3])
    n = np.array([1, 3, 3, 4, 4, 4, 2])
    assert oracle.collapse(keys, ka, W, n, [[1], [2]]) == pytest.approx(77 / 128, abs=1e-15)
    assert oracle.collapse(keys, ka, W, n) == pytest.approx(29 / 42, abs=1e-15)
    # the other orders of the same levels, worked the same way
    assert oracle.collapse(keys, ka, W, n, [[2], [1]]) == pytest.approx(81 / 128, abs=1e-15)
    assert oracle.collapse(keys, ka, W, n, [[1, 2]]) == pytest.approx(3 / 5, abs=1e-15)
