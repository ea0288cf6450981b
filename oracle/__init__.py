"""FP64 CPU oracle for ABX discriminability -- TEST INFRASTRUCTURE ONLY.

Only ``tests/``, ``__graft_entry__.smoke()`` and the CPU-baseline leg of
``bench.py`` may import this package.  The product library
(``paper_2505_02692_amd``) never imports it, and the two share no code; the
only common input is the seeded generator in ``workloads``.

Every function follows a passage of the paper (Poli, Chemla, Dupoux,
"fastabx: A library for efficient computation of ABX discriminability"):

* ``cells``            -- Background section: the ON / BY / ACROSS conditions
                          (Fig. 1 caption, Table 1) and the cell A x B x X.
* ``frame_distance``   -- the "angular" distance named with the Score class,
                          or the "euclidean" one named beside it, or the
                          0 / 1 mismatch of discrete unit codes.
* ``dtw``              -- the DTW recurrence of "Dynamic Time Warping on GPU".
* ``pair_distances``   -- DTW over frame distances, or time pooling (same
                          section: "pool along the time domain").
* ``cell_half_units``  -- the cell discriminability formula D_C (Background).
* ``collapse``         -- the weighted average of D_C, or averaging across
                          attributes level by level (Score / collapse).
* ``slice_frames``     -- the frames kept for an aligned unit ("Slicing
                          features" appendix), from the set definition.
* ``subsample``        -- the Subsampler of the Task interface (caps on a, b
                          and x per cell; distinct ACROSS values of x), with
                          Philox4x32-10 draws (``philox4x32_10``).

Readings where the paper is silent:
a == x is excluded when A and X are the same set; cells are ordered (o1, o2);
with several ACROSS attributes x differs from a in every one of them; the DTW
boundary is the cumulative first row / column; the path length used for
normalisation is the one of the path that prefers diagonal, then left
(j - 1), then up (i - 1) moves on exact ties; the distance is theta / pi.
"""
from __future__ import annotations

import ctypes
import os
import subprocess
import sysconfig
from dataclasses import dataclass, field
from typing import Dict, List, Optional, Sequence, Tuple

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "abx_oracle.c")
_SO = os.path.join(_HERE, "_abx_oracle.so")

EDOMAIN = -3


def build() -> str:
    """Compile the C part of the oracle (plain gcc, no FMA contraction)."""
    cmd = ["gcc", "-O2", "-std=c11", "-ffp-contract=off", "-fno-fast-math", "-fopenmp",
           "-shared", "-fPIC", "-Wall", "-o", _SO + ".tmp", _SRC, "-lm"]
    subprocess.run(cmd, check=True)
    os.replace(_SO + ".tmp", _SO)
    return _SO


_lib_handle = None


def _lib():
    global _lib_handle
    if _lib_handle is None:
        if not os.path.exists(_SO):
            build()
        lib = ctypes.CDLL(_SO)
        P = ctypes.POINTER
        lib.oracle_frame_distance.argtypes = [P(ctypes.c_double), P(ctypes.c_double), ctypes.c_int,
                                              ctypes.c_int, P(ctypes.c_double)]
        lib.oracle_dtw.argtypes = [P(ctypes.c_double), ctypes.c_int, ctypes.c_int, ctypes.c_int,
                                   P(ctypes.c_double), P(ctypes.c_int64)]
        lib.oracle_pair_distances.argtypes = [
            P(ctypes.c_float), P(ctypes.c_int64), ctypes.c_int, ctypes.c_int64,
            P(ctypes.c_int64), P(ctypes.c_int64), P(ctypes.c_int64), P(ctypes.c_int32),
            P(ctypes.c_int32), ctypes.c_int, ctypes.c_int, ctypes.c_int, P(ctypes.c_double),
            P(ctypes.c_int64)]
        lib.oracle_num_threads.restype = ctypes.c_int
        _lib_handle = lib
    return _lib_handle


def _ptr(a: np.ndarray, ct):
    return a.ctypes.data_as(ctypes.POINTER(ct))


def num_threads() -> int:
    """OpenMP threads the pair-distance stage uses."""
    return int(_lib().oracle_num_threads())


# ---------------------------------------------------------------- distances --

# "units": discrete unit codes (one value per frame, dim 1), distance 0 for
# equal codes and 1 otherwise (DTW mode); the paper says ABX works with
# discrete representations but gives no distance for them.
DISTANCES = {"angular": 0, "euclidean": 1, "units": 2}


def frame_distance(u: Sequence[float], v: Sequence[float], distance: str = "angular") -> float:
    """Distance of two raw vectors in FP64: the angle theta(u, v) / pi
    ("angular"), the length of u - v ("euclidean"), or for one-element
    vectors holding discrete unit codes 0 if the codes are equal, else 1
    ("units")."""
    u = np.ascontiguousarray(u, dtype=np.float64)
    v = np.ascontiguousarray(v, dtype=np.float64)
    out = ctypes.c_double()
    rc = _lib().oracle_frame_distance(_ptr(u, ctypes.c_double), _ptr(v, ctypes.c_double),
                                      int(u.shape[0]), DISTANCES[distance], ctypes.byref(out))
    if rc != 0:
        raise ValueError(f"frame_distance failed ({rc}): zero vector has no angle")
    return out.value


def dtw(d: np.ndarray, norm: str = "path") -> Tuple[float, int]:
    """DTW of a frame-distance matrix (rows = x, cols = y): (distance, path length)."""
    d = np.ascontiguousarray(d, dtype=np.float64)
    N, M = d.shape
    out = ctypes.c_double()
    ln = ctypes.c_int64()
    rc = _lib().oracle_dtw(_ptr(d, ctypes.c_double), N, M, 0 if norm == "path" else 1,
                           ctypes.byref(out), ctypes.byref(ln))
    if rc != 0:
        raise ValueError("dtw: empty matrix")
    return out.value, int(ln.value)


# ------------------------------------------------------------------ slicing --

def slice_frames(onset: float, offset: float, dt: float, libri_light: bool = False) -> Tuple[int, int]:
    """(first frame, frame count) of a unit [onset, offset]: the set
    {i in N : onset <= t_i <= offset} with t_i = dt / 2 + i dt, scanned frame by
    frame in FP64; the Libri-Light slicing drops the last frame of the set."""
    kept = []
    i = 0
    while dt / 2 + i * dt <= offset:
        if onset <= dt / 2 + i * dt:
            kept.append(i)
        i += 1
    if libri_light and kept:
        kept = kept[:-1]
    return (kept[0] if kept else 0), len(kept)


# -------------------------------------------------------------------- cells --

@dataclass
class Cell:
    key: Tuple[int, ...]           # (on_ax, on_b, by..., across_ab..., across_x...)
    by_key: Tuple[int, ...]
    A: np.ndarray                  # item ids
    B: np.ndarray
    X: np.ndarray
    exclude_self: bool             # True when X is A (a == x is not a triple)

    @property
    def n_triplets(self) -> int:
        if self.exclude_self:
            return len(self.A) * (len(self.A) - 1) * len(self.B)
        return len(self.A) * len(self.B) * len(self.X)


def key_attrs(on: int, by: Sequence[int], across: Sequence[int]) -> List[int]:
    """Attribute column behind each cell-key column."""
    return [on, on] + list(by) + list(across) + list(across)


def validate_task(n_attr: int, on: int, by: Sequence[int], across: Sequence[int]) -> None:
    cols = [on] + list(by) + list(across)
    if any(c < 0 or c >= n_attr for c in cols):
        raise ValueError("attribute column out of range")
    if len(set(cols)) != len(cols):
        raise ValueError("ON, BY and ACROSS attributes must be distinct")


def cells(attrs: np.ndarray, on: int, by: Sequence[int], across: Sequence[int]) -> List[Cell]:
    """Every cell of the task, in ascending (by..., on_ax, on_b, across_ab..., across_x...) order.

    A triple (a, b, x) is valid when a and x share the ON value and b does not;
    a, b and x share every BY value; a and b share every ACROSS value while x
    differs from them in every ACROSS attribute.  Without ACROSS, X is A and
    a must differ from x ("another a in A").  Cells without a triple are not
    listed.
    """
    attrs = np.asarray(attrs)
    validate_task(attrs.shape[1], on, by, across)
    by = list(by)
    across = list(across)
    groups: Dict[Tuple[int, ...], Dict[Tuple[int, Tuple[int, ...]], List[int]]] = {}
    for item in range(attrs.shape[0]):
        row = attrs[item]
        g = tuple(int(row[c]) for c in by)
        cls = (int(row[on]), tuple(int(row[c]) for c in across))
        groups.setdefault(g, {}).setdefault(cls, []).append(item)

    out: List[Cell] = []
    for g in sorted(groups):
        classes = groups[g]
        keys = sorted(classes)
        if not across:
            for (o1, _) in keys:
                A = classes[(o1, ())]
                if len(A) < 2:
                    continue
                for (o2, _) in keys:
                    if o2 == o1:
                        continue
                    B = classes[(o2, ())]
                    arrA = np.array(A, dtype=np.int64)
                    out.append(Cell((o1, o2) + g, g, arrA, np.array(B, dtype=np.int64), arrA, True))
        else:
            for (o1, alpha) in keys:
                A = classes[(o1, alpha)]
                for (o2, alpha2) in keys:
                    if o2 == o1 or alpha2 != alpha:
                        continue
                    B = classes[(o2, alpha)]
                    for (o3, beta) in keys:
                        if o3 != o1 or any(bk == ak for bk, ak in zip(beta, alpha)):
                            continue
                        X = classes[(o1, beta)]
                        out.append(Cell((o1, o2) + g + alpha + beta, g,
                                        np.array(A, dtype=np.int64), np.array(B, dtype=np.int64),
                                        np.array(X, dtype=np.int64), False))
    out.sort(key=lambda c: (c.by_key, c.key[:2], c.key[2 + len(by):]))
    return out


# ------------------------------------------------------------------ scoring --

def cell_half_units(dist: Dict[Tuple[int, int], float], X, A, B, exclude_self: bool) -> int:
    """Twice the numerator of D_C: sum over (a, b, x) of 2[d(x,a) < d(x,b)] + [d(x,a) == d(x,b)]."""
    W = 0
    for x in X:
        da = np.array([dist[(int(x), int(a))] for a in A if not (exclude_self and a == x)],
                      dtype=np.float64)
        db = np.array([dist[(int(x), int(b))] for b in B], dtype=np.float64)
        W += 2 * int(np.count_nonzero(da[:, None] < db[None, :]))
        W += int(np.count_nonzero(da[:, None] == db[None, :]))
    return W


def _cell_half_units_dense(M: np.ndarray, X, A, B, exclude_self: bool, chunk: int = 64) -> int:
    """Same count as ``cell_half_units`` on a dense per-group matrix (local indices)."""
    W = 0
    A = np.asarray(A)
    B = np.asarray(B)
    for s in range(0, len(X), chunk):
        xs = np.asarray(X[s:s + chunk])
        da = M[np.ix_(xs, A)]                       # [x, a]
        db = M[np.ix_(xs, B)]                       # [x, b]
        keep = (A[None, :] != xs[:, None]) if exclude_self else np.ones((len(xs), len(A)), bool)
        lt = (da[:, :, None] < db[:, None, :]) & keep[:, :, None]
        eq = (da[:, :, None] == db[:, None, :]) & keep[:, :, None]
        W += 2 * int(np.count_nonzero(lt)) + int(np.count_nonzero(eq))
    return W


@dataclass
class OracleResult:
    cells: List[Cell]
    half_units: np.ndarray          # int64 [n_cells]
    n_triplets: np.ndarray          # int64 [n_cells]
    key_attrs: List[int]
    by: List[int]
    across: List[int]
    on: int
    # per BY group: (item ids sorted, dense FP64 [n, n] matrix, NaN where unused)
    groups: Dict[Tuple[int, ...], Tuple[np.ndarray, np.ndarray]] = field(default_factory=dict)

    @property
    def keys(self) -> np.ndarray:
        k = len(self.key_attrs)
        return np.array([c.key for c in self.cells], dtype=np.int64).reshape(-1, k)

    @property
    def scores(self) -> np.ndarray:
        return self.half_units / (2.0 * self.n_triplets)

    def pair_distance(self, x: int, y: int, attrs: np.ndarray) -> float:
        g = tuple(int(attrs[x][c]) for c in self.by)
        items, M = self.groups[g]
        i = int(np.searchsorted(items, x))
        j = int(np.searchsorted(items, y))
        return float(M[i, j])


def pair_distances(features: np.ndarray, offsets: np.ndarray,
                   group_items: List[np.ndarray], group_pairs: List[Tuple[np.ndarray, np.ndarray]],
                   mode: str = "dtw", norm: str = "path", distance: str = "angular") -> List[np.ndarray]:
    """FP64 distances of the given (x, y) pairs, listed per group as local positions."""
    feats = np.ascontiguousarray(features, dtype=np.float32)
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    D = int(feats.shape[1])
    gptr = np.zeros(len(group_items) + 1, np.int64)
    gptr[1:] = np.cumsum([len(g) for g in group_items])
    gitems = np.ascontiguousarray(np.concatenate(group_items) if group_items else np.zeros(0), np.int64)
    pptr = np.zeros(len(group_pairs) + 1, np.int64)
    pptr[1:] = np.cumsum([len(p[0]) for p in group_pairs])
    px = np.ascontiguousarray(np.concatenate([p[0] for p in group_pairs]) if group_pairs else np.zeros(0), np.int32)
    py = np.ascontiguousarray(np.concatenate([p[1] for p in group_pairs]) if group_pairs else np.zeros(0), np.int32)
    out = np.zeros(int(pptr[-1]), np.float64)
    bad = ctypes.c_int64(-1)
    rc = _lib().oracle_pair_distances(
        _ptr(feats, ctypes.c_float), _ptr(offsets, ctypes.c_int64), D, len(group_items),
        _ptr(gptr, ctypes.c_int64), _ptr(gitems, ctypes.c_int64), _ptr(pptr, ctypes.c_int64),
        _ptr(px, ctypes.c_int32), _ptr(py, ctypes.c_int32),
        0 if mode == "dtw" else 1, 0 if norm == "path" else 1, DISTANCES[distance],
        _ptr(out, ctypes.c_double), ctypes.byref(bad))
    if rc == EDOMAIN:
        raise ValueError(f"zero-norm frame or mean in item {bad.value}: angle undefined")
    if rc != 0:
        raise RuntimeError(f"oracle_pair_distances failed ({rc})")
    return [out[pptr[g]:pptr[g + 1]] for g in range(len(group_items))]


def score(features: np.ndarray, offsets: np.ndarray, attrs: np.ndarray, on: int,
          by: Sequence[int], across: Sequence[int], mode: str = "dtw", norm: str = "path",
          cell_filter=None, distance: str = "angular", subsampler: Optional[dict] = None) -> OracleResult:
    """Per-cell half-unit counts W and triplet counts |C| for the whole task.

    ``cell_filter`` (optional) keeps a subset of the cells, e.g. a sample of
    BY groups for workloads too large to score in full.  ``subsampler``
    (optional): keyword arguments of ``subsample`` (seed, max_a, max_b,
    max_x, max_x_across), applied to the full cell list before the filter.
    """
    cl = cells(attrs, on, by, across)
    if subsampler is not None:
        cl = subsample(cl, len(across), **subsampler)
    if cell_filter is not None:
        cl = [c for c in cl if cell_filter(c)]
    # the (x, y) pairs each BY group needs: X x A without a == x, and X x B
    by_group: Dict[Tuple[int, ...], List[Cell]] = {}
    for c in cl:
        by_group.setdefault(c.by_key, []).append(c)
    gkeys = sorted(by_group)
    group_items, group_pairs, need_mats = [], [], []
    for g in gkeys:
        items = np.unique(np.concatenate([np.concatenate([c.A, c.B, c.X]) for c in by_group[g]]))
        n = len(items)
        need = np.zeros((n, n), dtype=bool)
        for c in by_group[g]:
            xs = np.searchsorted(items, c.X)
            for S in (c.A, c.B):
                need[np.ix_(xs, np.searchsorted(items, S))] = True
        if any(c.exclude_self for c in by_group[g]):
            np.fill_diagonal(need, False)
        xi, yi = np.nonzero(need)
        group_items.append(items)
        group_pairs.append((xi.astype(np.int32), yi.astype(np.int32)))
        need_mats.append(need)
    dists = pair_distances(features, offsets, group_items, group_pairs, mode, norm, distance)
    groups = {}
    for g, items, (xi, yi), dv in zip(gkeys, group_items, group_pairs, dists):
        M = np.full((len(items), len(items)), np.nan)
        M[xi, yi] = dv
        groups[g] = (items, M)
    W = np.zeros(len(cl), np.int64)
    n_trip = np.zeros(len(cl), np.int64)
    for k, c in enumerate(cl):
        items, M = groups[c.by_key]
        W[k] = _cell_half_units_dense(M, np.searchsorted(items, c.X), np.searchsorted(items, c.A),
                                      np.searchsorted(items, c.B), c.exclude_self)
        n_trip[k] = c.n_triplets
    return OracleResult(cl, W, n_trip, key_attrs(on, by, across), list(by), list(across), on, groups)


# ---------------------------------------------------------------- aggregate --

def collapse(keys: np.ndarray, key_attr: Sequence[int], half_units: np.ndarray,
             n_triplets: np.ndarray, levels: Optional[Sequence[Sequence[int]]] = None) -> float:
    """ABX error rate 1 - D.

    Without levels, D is the average of D_C weighted by cell size, i.e.
    sum W / (2 sum |C|).  With levels, for each level in turn the key columns
    of that level's attributes are removed and D_C is averaged (unweighted)
    over the rows that now share a key; the remaining rows are averaged at
    the end.
    """
    half_units = np.asarray(half_units, dtype=np.int64)
    n_triplets = np.asarray(n_triplets, dtype=np.int64)
    if len(half_units) == 0:
        return float("nan")
    if not levels:
        return 1.0 - float(half_units.sum()) / (2.0 * float(n_triplets.sum()))
    key_attr = list(key_attr)
    on = key_attr[0]
    rows = {tuple(int(v) for v in k): float(w) / (2.0 * float(n))
            for k, w, n in zip(np.asarray(keys).tolist(), half_units, n_triplets)}
    cols = list(range(len(key_attr)))
    for level in levels:
        level = set(level)
        if on in level or any(a not in key_attr for a in level):
            raise ValueError("a collapse level may only name BY / ACROSS attributes of the task")
        keep = [c for c in cols if key_attr[c] not in level]
        pos = [cols.index(c) for c in keep]
        acc: Dict[Tuple[int, ...], List[float]] = {}
        for k, s in rows.items():
            acc.setdefault(tuple(k[p] for p in pos), []).append(s)
        rows = {k: sum(v) / len(v) for k, v in acc.items()}
        cols = keep
    return 1.0 - sum(rows.values()) / len(rows)


def error_rate(res: OracleResult, levels=None) -> float:
    return collapse(res.keys, res.key_attrs, res.half_units, res.n_triplets, levels)


# --------------------------------------------------------------- subsampler --
#
# The Subsampler of the Task interface (library overview, "Task" paragraph):
# it caps the number of a, b and x independently in each cell, and, with ACROSS
# conditions, limits the number of distinct values x takes for the ACROSS
# attribute (the text says "for the ON attribute", but x's ON value is fixed
# within a cell; the limit that exists in the Libri-Light evaluation it
# reproduces is on the ACROSS value, e.g. the speaker).  Random choices come
# from the counter-based generator Philox4x32-10 (Salmon, Moraes, Dror, Shaw,
# "Parallel random numbers: as easy as 1, 2, 3", SC'11), so that a subsample
# is a pure function of (seed, cell, set, position) and the GPU library can
# draw the same one without sharing this code.

_PHILOX_M = (0xD2511F53, 0xCD9E8D57)    # round multipliers
_PHILOX_W = (0x9E3779B9, 0xBB67AE85)    # key increments (Weyl sequence)
_U32 = 0xFFFFFFFF


def philox4x32_10(ctr: Sequence[int], key: Sequence[int]) -> Tuple[int, int, int, int]:
    """Philox4x32 with 10 rounds: each round multiplies counter words 0 and 2
    by the two multipliers (64-bit products split into high and low halves),
    mixes the high halves with words 1 and 3 and the key, permutes, and bumps
    the key by the Weyl increments."""
    c0, c1, c2, c3 = (int(v) & _U32 for v in ctr)
    k0, k1 = (int(v) & _U32 for v in key)
    for _ in range(10):
        p0, p1 = _PHILOX_M[0] * c0, _PHILOX_M[1] * c2
        c0, c1, c2, c3 = ((p1 >> 32) ^ c1 ^ k0) & _U32, p1 & _U32, ((p0 >> 32) ^ c3 ^ k1) & _U32, p0 & _U32
        k0 = (k0 + _PHILOX_W[0]) & _U32
        k1 = (k1 + _PHILOX_W[1]) & _U32
    return c0, c1, c2, c3


def _draw(seed: int, a: int, b: int, c: int) -> int:
    """First output word of Philox4x32-10 at counter (a, b, c, 0), key = the seed."""
    return philox4x32_10((a, b, c, 0), (seed & _U32, (seed >> 32) & _U32))[0]


def _pick(items: np.ndarray, cap: int, seed: int, cell: int, which: int) -> np.ndarray:
    """At most `cap` of `items` (ascending item ids): the ones whose draws at
    counter (cell, which, position) are smallest, position breaking ties; all
    of them when cap <= 0 or there are not more than cap."""
    if cap <= 0 or len(items) <= cap:
        return items
    r = [(_draw(seed, cell, which, i), i) for i in range(len(items))]
    keep = sorted(i for _, i in sorted(r)[:cap])
    return items[np.array(keep, dtype=np.int64)]


def subsample(cl: List[Cell], n_across: int, seed: int, max_a: int = 0, max_b: int = 0, max_x: int = 0,
              max_x_across: int = 0) -> List[Cell]:
    """The cells of a subsampled task, from the full list `cl` (as ``cells``
    returns it; position c in it is the cell's index in the draws).

    1. ACROSS tasks with max_x_across > 0: the cells sharing (on_ax, on_b,
       by..., across_ab...) differ only in across_x; of the m cells of such a
       family, those with the max_x_across smallest draws at counter
       (f, 3, j) are kept (f: index of the family's first cell, j: rank of
       the cell in the family).
    2. Each kept cell c caps A, B and X independently: A with the draws at
       (c, 0, position), B at (c, 1, .), X at (c, 2, .).  Without ACROSS, X is
       A itself: the one set is capped by both max_a and max_x, with the A
       draws, and stays the same set.
    3. Cells left without a triple (|A| < 2 without ACROSS) are dropped.
    Caps <= 0 mean no cap."""
    keep = [True] * len(cl)
    if n_across > 0 and max_x_across > 0:
        c = 0
        while c < len(cl):
            fam = cl[c].key[:len(cl[c].key) - n_across]
            e = c + 1
            while e < len(cl) and cl[e].key[:len(cl[e].key) - n_across] == fam:
                e += 1
            if e - c > max_x_across:
                r = sorted((_draw(seed, c, 3, j), j) for j in range(e - c))
                chosen = {j for _, j in r[:max_x_across]}
                for j in range(e - c):
                    keep[c + j] = j in chosen
            c = e
    out: List[Cell] = []
    for c, cell in enumerate(cl):
        if not keep[c]:
            continue
        B = _pick(cell.B, max_b, seed, c, 1)
        if cell.exclude_self:
            caps = [v for v in (max_a, max_x) if v > 0]
            A = _pick(cell.A, min(caps) if caps else 0, seed, c, 0)
            if len(A) < 2:
                continue
            out.append(Cell(cell.key, cell.by_key, A, B, A, True))
        else:
            A = _pick(cell.A, max_a, seed, c, 0)
            X = _pick(cell.X, max_x, seed, c, 2)
            out.append(Cell(cell.key, cell.by_key, A, B, X, False))
    return out
