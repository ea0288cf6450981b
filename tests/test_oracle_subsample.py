"""Pins of the oracle's Subsampler (Task interface, library overview: caps on
the number of a, b and x per cell, and on the distinct ACROSS values of x).

* The generator: Philox4x32-10 known-answer vectors (tests/golden/philox_kat.json).
* The subsets: each capped set is a subset of the cell's set with exactly
  min(size, cap) items; without ACROSS, X stays the same set as A; caps at
  or above every set size change nothing; the draws are a pure function of
  the seed; over many seeds every item is kept with probability cap / size.
* The ACROSS limit: no family of cells (same on_ax, on_b, by, across_ab)
  keeps more than the limit, families within it are untouched, and the
  cells kept are whole cells of the full task.
* Scores: a subsampled task's W is the definition evaluated on the subsets
  (brute-force triples), and caps that bind nowhere give the full score."""
import json
import os

import numpy as np
import pytest

import oracle

GOLDEN = os.path.join(os.path.dirname(os.path.abspath(__file__)), "golden", "philox_kat.json")


def test_philox_known_answers():
    for v in json.load(open(GOLDEN))["vectors"]:
        ctr = [int(x, 16) for x in v["ctr"]]
        key = [int(x, 16) for x in v["key"]]
        assert oracle.philox4x32_10(ctr, key) == tuple(int(x, 16) for x in v["out"])


def _table(rng, n, n_on=4, n_by=3, n_ac=5):
    return np.stack([rng.integers(0, n_on, n), rng.integers(0, n_by, n), rng.integers(0, n_ac, n)],
                    axis=1).astype(np.int32)


@pytest.mark.parametrize("across", [False, True])
@pytest.mark.parametrize("caps", [(2, 3, 2), (3, 1, 4), (5, 5, 1), (2, 0, 0)])
def test_caps_give_subsets_of_the_right_size(across, caps):
    rng = np.random.default_rng(7)
    attrs = _table(rng, 300)
    by, acr = ([1], [2]) if across else ([1, 2], [])
    full = oracle.cells(attrs, 0, by, acr)
    max_a, max_b, max_x = caps
    sub = oracle.subsample(full, len(acr), seed=11, max_a=max_a, max_b=max_b, max_x=max_x)
    fk = {c.key: c for c in full}

    def cap(v):
        return v if v > 0 else 10 ** 9
    # a within cell needs two a's: a cap of 1 on the shared set leaves none
    assert len(sub) > 0 or (not across and min(cap(max_a), cap(max_x)) < 2)
    for c in sub:
        f = fk[c.key]
        assert set(c.A) <= set(f.A) and set(c.B) <= set(f.B) and set(c.X) <= set(f.X)
        assert list(c.A) == sorted(c.A) and list(c.B) == sorted(c.B)
        assert len(c.B) == min(len(f.B), cap(max_b))
        if across:
            assert len(c.A) == min(len(f.A), cap(max_a)) and len(c.X) == min(len(f.X), cap(max_x))
        else:
            assert c.X is c.A and len(c.A) == min(len(f.A), cap(max_a), cap(max_x))
    # dropped cells are exactly the within cells whose capped A has fewer than 2 items
    dropped = set(fk) - {c.key for c in sub}
    for k in dropped:
        assert not across and min(cap(max_a), cap(max_x)) < 2


def test_no_binding_cap_changes_nothing_and_seed_decides():
    rng = np.random.default_rng(8)
    attrs = _table(rng, 200)
    full = oracle.cells(attrs, 0, [1], [2])
    same = oracle.subsample(full, 1, seed=3, max_a=10 ** 6, max_b=10 ** 6, max_x=10 ** 6, max_x_across=10 ** 6)
    assert [c.key for c in same] == [c.key for c in full]
    assert all(np.array_equal(a.A, b.A) and np.array_equal(a.B, b.B) and np.array_equal(a.X, b.X)
               for a, b in zip(same, full))
    s1 = oracle.subsample(full, 1, seed=5, max_a=2, max_b=2, max_x=2)
    s2 = oracle.subsample(full, 1, seed=5, max_a=2, max_b=2, max_x=2)
    s3 = oracle.subsample(full, 1, seed=6, max_a=2, max_b=2, max_x=2)
    assert all(np.array_equal(a.A, b.A) and np.array_equal(a.X, b.X) for a, b in zip(s1, s2))
    assert any(not np.array_equal(a.A, b.A) or not np.array_equal(a.X, b.X) for a, b in zip(s1, s3))


def test_every_item_kept_with_probability_cap_over_size():
    """A 10-item A capped at 3, over 3000 seeds: each position is kept about
    0.3 of the time (within 5 standard deviations), and A and B are drawn
    independently (their joint inclusion frequency is the product)."""
    attrs = np.array([[0, 0]] * 10 + [[1, 0]] * 10, dtype=np.int32)
    full = oracle.cells(attrs, 0, [1], [])
    cell = full[0]
    n, cap, runs = 10, 3, 3000
    hitA = np.zeros(n)
    joint = 0
    for seed in range(runs):
        c = oracle.subsample(full, 0, seed=seed, max_a=cap, max_b=cap)[0]
        pa = np.searchsorted(cell.A, c.A)
        pb = np.searchsorted(cell.B, c.B)
        hitA[pa] += 1
        joint += (0 in pa) and (0 in pb)
    p = cap / n
    sd = np.sqrt(p * (1 - p) / runs)
    assert np.all(np.abs(hitA / runs - p) < 5 * sd)
    sdj = np.sqrt(p * p * (1 - p * p) / runs)
    assert abs(joint / runs - p * p) < 5 * sdj


@pytest.mark.parametrize("limit", [1, 2, 3])
def test_across_limit_per_family(limit):
    rng = np.random.default_rng(9)
    attrs = _table(rng, 400, n_on=3, n_by=2, n_ac=6)
    full = oracle.cells(attrs, 0, [1], [2])
    sub = oracle.subsample(full, 1, seed=21, max_x_across=limit)
    fam = lambda c: c.key[:-1]
    full_count, sub_count = {}, {}
    for c in full:
        full_count[fam(c)] = full_count.get(fam(c), 0) + 1
    for c in sub:
        sub_count[fam(c)] = sub_count.get(fam(c), 0) + 1
    assert set(sub_count) == set(full_count)
    for f, m in full_count.items():
        assert sub_count[f] == min(m, limit)
    fk = {c.key: c for c in full}
    for c in sub:   # kept cells are whole cells of the full task
        f = fk[c.key]
        assert np.array_equal(c.A, f.A) and np.array_equal(c.B, f.B) and np.array_equal(c.X, f.X)


def _brute_W(M, items, c):
    pos = {int(v): k for k, v in enumerate(items)}
    W = 0
    for x in c.X:
        for a in c.A:
            if c.exclude_self and a == x:
                continue
            for b in c.B:
                da, db = M[pos[int(x)], pos[int(a)]], M[pos[int(x)], pos[int(b)]]
                W += 2 if da < db else (1 if da == db else 0)
    return W


@pytest.mark.parametrize("across", [False, True])
def test_subsampled_score_is_the_definition_on_the_subsets(across):
    rng = np.random.default_rng(12)
    n = 160
    attrs = _table(rng, n, n_on=3, n_by=2, n_ac=4)
    lens = rng.integers(1, 5, n)
    off = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    feats = rng.normal(size=(int(off[-1]), 6)).astype(np.float32)
    by, acr = ([1], [2]) if across else ([1, 2], [])
    sub = dict(seed=4, max_a=3, max_b=2, max_x=2, max_x_across=2)
    res = oracle.score(feats, off, attrs, 0, by, acr, subsampler=sub)
    ref_cells = oracle.subsample(oracle.cells(attrs, 0, by, acr), len(acr), **sub)
    assert [c.key for c in res.cells] == [c.key for c in ref_cells]
    for k, c in enumerate(res.cells):
        items, M = res.groups[c.by_key]
        assert res.half_units[k] == _brute_W(M, items, c)
        assert res.n_triplets[k] == c.n_triplets
    # caps that bind nowhere: the full task's score
    big = dict(seed=4, max_a=n, max_b=n, max_x=n, max_x_across=n)
    a = oracle.score(feats, off, attrs, 0, by, acr, subsampler=big)
    b = oracle.score(feats, off, attrs, 0, by, acr)
    assert np.array_equal(a.half_units, b.half_units)
