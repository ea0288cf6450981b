"""Pins of the oracle's cell enumeration (P8) and the ON / BY / ACROSS semantics.

The triple predicate is the Background section's: ON equal for a and x and
different for b; every BY equal for a, b and x; every ACROSS equal for a and
b and different for x; x is compared to *another* a.
"""
import itertools

import numpy as np
import pytest

import oracle


def _valid(attrs, on, by, across, a, b, x):
    ra, rb, rx = attrs[a], attrs[b], attrs[x]
    if a == x:
        return False
    if not (ra[on] == rx[on] and rb[on] != ra[on]):
        return False
    if any(not (ra[c] == rb[c] == rx[c]) for c in by):
        return False
    if any(not (ra[c] == rb[c] and rx[c] != ra[c]) for c in across):
        return False
    return True


def _cell_triples(c):
    out = []
    for x in c.X:
        for a in c.A:
            if c.exclude_self and a == x:
                continue
            for b in c.B:
                out.append((int(a), int(b), int(x)))
    return out


@pytest.mark.parametrize("seed", range(12))
def test_cells_equal_bruteforce_triples(seed):
    """P8: the union of the cells' triples is exactly the set of valid ordered triples."""
    rng = np.random.default_rng(seed)
    n = int(rng.integers(8, 45))
    n_attr = 4
    card = rng.integers(2, 4, size=n_attr)
    attrs = np.stack([rng.integers(0, k, size=n) for k in card], axis=1).astype(np.int32)
    specs = [(0, [], []), (0, [1], []), (0, [1, 2], []), (0, [1], [2]), (0, [], [1]),
             (0, [], [1, 2]), (3, [0], [1, 2])]
    on, by, across = specs[seed % len(specs)]
    cl = oracle.cells(attrs, on, by, across)
    got = []
    for c in cl:
        t = _cell_triples(c)
        assert len(t) == c.n_triplets > 0
        got.extend(t)
    want = [(a, b, x) for a, b, x in itertools.product(range(n), repeat=3)
            if _valid(attrs, on, by, across, a, b, x)]
    assert len(got) == len(set(got))          # no triple counted twice
    assert sorted(got) == sorted(want)


def test_table1_semantics():
    """Table 1 style cases: fruit / colour / size attributes."""
    # columns: fruit (0 apple, 1 pear, 2 strawberry), colour (0 red, 1 green), size (0 big, 1 small)
    items = {
        "red_apple_big": (0, 0, 0), "green_apple_big": (0, 1, 0), "green_apple_small": (0, 1, 1),
        "green_pear_big": (1, 1, 0), "red_strawberry_big": (2, 0, 0), "red_apple_small": (0, 0, 1),
    }
    names = list(items)
    attrs = np.array([items[k] for k in names], np.int32)
    idx = {k: i for i, k in enumerate(names)}

    def triples(on, by, across):
        return {(names[a], names[b], names[x]) for c in oracle.cells(attrs, on, by, across)
                for a, b, x in _cell_triples(c)}

    # ON fruit BY colour: a and x red apples, b a red strawberry
    t = triples(0, [1], [])
    assert ("red_apple_big", "red_strawberry_big", "red_apple_small") in t
    assert not any(a.startswith("green") != x.startswith("green") for a, _, x in t)
    # ON fruit BY colour ACROSS size: a green apple (big), b green pear (big), x small green apple
    t = triples(0, [1], [2])
    assert ("green_apple_big", "green_pear_big", "green_apple_small") in t
    assert all(items[a][2] == items[b][2] != items[x][2] for a, b, x in t)
    # ON colour (no BY): a and x share colour, b does not
    t = triples(1, [], [])
    assert all(items[a][1] == items[x][1] != items[b][1] for a, b, x in t)
    assert ("red_apple_big", "green_pear_big", "red_strawberry_big") in t


def test_cell_keys_and_order():
    attrs = np.array([[0, 5, 1], [0, 5, 2], [1, 5, 1], [1, 5, 2], [0, 6, 1], [0, 6, 1], [2, 6, 1]], np.int32)
    cl = oracle.cells(attrs, 0, [1], [2])
    # key = (on_ax, on_b, by, across_ab, across_x); by group 5 first
    assert [c.key for c in cl] == [(0, 1, 5, 1, 2), (0, 1, 5, 2, 1), (1, 0, 5, 1, 2), (1, 0, 5, 2, 1)]
    cl = oracle.cells(attrs, 0, [1], [])
    # group 6: label 2 has one item, so only (0, 2) is a cell there (|A| >= 2 without ACROSS)
    assert [c.key for c in cl] == [(0, 1, 5), (1, 0, 5), (0, 2, 6)]
    assert cl[2].n_triplets == 2 * 1 * 1


def test_invalid_task_specs():
    attrs = np.zeros((4, 3), np.int32)
    with pytest.raises(ValueError):
        oracle.cells(attrs, 0, [0], [])
    with pytest.raises(ValueError):
        oracle.cells(attrs, 0, [1], [1])
    with pytest.raises(ValueError):
        oracle.cells(attrs, 0, [5], [])
    assert oracle.cells(attrs, 0, [1], [2]) == []     # a single ON value: no cell
