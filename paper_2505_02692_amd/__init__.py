"""fastabx-hip: ABX discriminability on AMD MI355X (gfx950).

Thin Python binding over the C ABI declared in include/fastabx.h.  The
functions named ``fabx_*`` mirror the C calls one to one (argument
marshalling only: every step runs in the native library's HIP kernels);
``Context`` / ``Dataset`` / ``Task`` / ``Result`` / ``Server`` wrap them with
ownership.  PyTorch is used only for device memory and the current stream.

    ctx = Context(0)
    ds = Dataset(ctx, features, offsets, attrs)       # features: cuda tensor
    task = Task(ds, on=0, by=[1, 2, 3])
    res = task.score(mode="dtw", precision="bf16")
    err = res.collapse(levels=[[1, 2], [3]])
"""
from __future__ import annotations

import ctypes
from typing import Optional, Sequence

import numpy as np

from . import _lib as L
from ._lib import (FABX_DISTANCE_ANGULAR, FABX_DISTANCE_EUCLIDEAN, FABX_DISTANCE_UNITS, FABX_DTYPE_BF16,
                   FABX_DTYPE_F32, FABX_DTYPE_UNITS,
                   FABX_MODE_DTW, FABX_MODE_POOLED, FABX_NORM_NONE,
                   FABX_NORM_PATH, FABX_PREC_BF16_RECHECK, FABX_PREC_FP32, fabx_dataset_desc,
                   fabx_score_opts, fabx_server_stats, fabx_stats)

__all__ = ["FabxError", "Context", "Dataset", "Task", "Result", "Server", "make_opts", "lib",
           "fabx_set_thread_serial", "fabx_slice_frames", "read_item_file", "zerospeech_abx"]


class FabxError(RuntimeError):
    def __init__(self, code: int, msg: str):
        super().__init__(f"{L.STATUS_NAMES.get(code, code)}: {msg}")
        self.code = code


def lib() -> ctypes.CDLL:
    return L.load()


def _check(code: int) -> None:
    if code != 0:
        raise FabxError(code, lib().fabx_last_error().decode())


def _i32p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if a is not None else None


def _i64p(a):
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)) if a is not None else None


# --------------------------------------------------------- same-name calls --

def fabx_set_thread_serial(serial: bool) -> bool:
    """Run the library's host work issued from the calling thread on that
    thread alone (True), instead of on the shared host thread pool; returns
    the previous setting."""
    return bool(lib().fabx_set_thread_serial(1 if serial else 0))


def fabx_create(device: int = 0, stream=None) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(lib().fabx_create(ctypes.byref(h), int(device), stream))
    return h


def fabx_destroy(ctx) -> None:
    lib().fabx_destroy(ctx)


def fabx_dataset_create(ctx, features_ptr: int, dtype: int, n_frames: int, dim: int,
                        offsets: np.ndarray, attrs: np.ndarray) -> ctypes.c_void_p:
    offsets = np.ascontiguousarray(offsets, dtype=np.int64)
    attrs = np.ascontiguousarray(attrs, dtype=np.int32)
    if attrs.ndim == 1:
        attrs = attrs[:, None]
    d = fabx_dataset_desc(features_ptr, dtype, int(n_frames), int(dim), _i64p(offsets),
                          int(attrs.shape[0]), _i32p(attrs), int(attrs.shape[1]))
    h = ctypes.c_void_p()
    _check(lib().fabx_dataset_create(ctx, ctypes.byref(d), ctypes.byref(h)))
    return h


def fabx_dataset_create_windows(ctx, features_ptr: int, dtype: int, n_frames: int, dim: int,
                                item_start: np.ndarray, item_len: np.ndarray,
                                attrs: np.ndarray) -> ctypes.c_void_p:
    item_start = np.ascontiguousarray(item_start, dtype=np.int64)
    item_len = np.ascontiguousarray(item_len, dtype=np.int64)
    attrs = np.ascontiguousarray(attrs, dtype=np.int32)
    if attrs.ndim == 1:
        attrs = attrs[:, None]
    if not (len(item_start) == len(item_len) == attrs.shape[0]):
        raise ValueError("item_start, item_len and attrs must have one entry per item")
    h = ctypes.c_void_p()
    _check(lib().fabx_dataset_create_windows(ctx, features_ptr, dtype, int(n_frames), int(dim), _i64p(item_start),
                                             _i64p(item_len), int(attrs.shape[0]), _i32p(attrs),
                                             int(attrs.shape[1]), ctypes.byref(h)))
    return h


def fabx_dataset_destroy(ds) -> None:
    lib().fabx_dataset_destroy(ds)


def fabx_slice_frames(onset, offset, frame_step: float, libri_light: bool = False):
    """Frames kept for aligned units [onset, offset] (seconds): (start, len) int64 arrays."""
    onset = np.ascontiguousarray(onset, dtype=np.float64)
    offset = np.ascontiguousarray(offset, dtype=np.float64)
    if onset.shape != offset.shape or onset.ndim != 1:
        raise ValueError("onset and offset must be 1-D arrays of one length")
    start = np.zeros(len(onset), np.int64)
    length = np.zeros(len(onset), np.int64)
    _check(lib().fabx_slice_frames(onset.ctypes.data_as(ctypes.POINTER(ctypes.c_double)),
                                   offset.ctypes.data_as(ctypes.POINTER(ctypes.c_double)), len(onset),
                                   float(frame_step), 1 if libri_light else 0, _i64p(start), _i64p(length)))
    return start, length


def read_item_file(path: str):
    """An item file: a header "#file onset offset #<attr> <attr> ..." and one
    line per unit "<file> <onset> <offset> <value> ...".  Returns (attribute
    names, files, onsets, offsets, values [n_units][n_attr] as strings)."""
    with open(path) as f:
        header = f.readline().split()
        if len(header) < 4 or header[0] != "#file" or header[1:3] != ["onset", "offset"]:
            raise ValueError(f"{path}: the header must start with '#file onset offset'")
        names = [h.lstrip("#") for h in header[3:]]
        files, on, off, vals = [], [], [], []
        for ln, line in enumerate(f, start=2):
            parts = line.split()
            if not parts:
                continue
            if len(parts) != 3 + len(names):
                raise ValueError(f"{path}:{ln}: expected {3 + len(names)} columns, got {len(parts)}")
            files.append(parts[0])
            on.append(float(parts[1]))
            off.append(float(parts[2]))
            vals.append(parts[3:])
    return names, files, np.array(on, np.float64), np.array(off, np.float64), vals


def fabx_task_create(ds, on: int, by: Sequence[int], across: Sequence[int]) -> ctypes.c_void_p:
    b = np.ascontiguousarray(list(by), dtype=np.int32)
    a = np.ascontiguousarray(list(across), dtype=np.int32)
    h = ctypes.c_void_p()
    _check(lib().fabx_task_create(ds, int(on), _i32p(b), len(b), _i32p(a), len(a), ctypes.byref(h)))
    return h


def fabx_task_create_subsampled(ds, on: int, by: Sequence[int], across: Sequence[int],
                                sub: "Subsampler") -> ctypes.c_void_p:
    b = np.ascontiguousarray(list(by), dtype=np.int32)
    a = np.ascontiguousarray(list(across), dtype=np.int32)
    s = L.fabx_subsampler(int(sub.seed), int(sub.max_a), int(sub.max_b), int(sub.max_x), int(sub.max_x_across))
    h = ctypes.c_void_p()
    _check(lib().fabx_task_create_subsampled(ds, int(on), _i32p(b), len(b), _i32p(a), len(a), ctypes.byref(s),
                                             ctypes.byref(h)))
    return h


def fabx_task_destroy(t) -> None:
    lib().fabx_task_destroy(t)


def fabx_task_num_cells(t) -> int:
    return int(lib().fabx_task_num_cells(t))


def fabx_task_key_width(t) -> int:
    return int(lib().fabx_task_key_width(t))


def fabx_task_cell_keys(t) -> np.ndarray:
    n, k = fabx_task_num_cells(t), fabx_task_key_width(t)
    out = np.zeros((n, k), np.int32)
    _check(lib().fabx_task_cell_keys(t, _i32p(out)))
    return out


def fabx_task_cell_sizes(t):
    n = fabx_task_num_cells(t)
    nt = np.zeros(n, np.int64)
    abx = np.zeros((n, 3), np.int32)
    _check(lib().fabx_task_cell_sizes(t, _i64p(nt), _i32p(abx)))
    return nt, abx


def fabx_score_opts_default() -> fabx_score_opts:
    o = fabx_score_opts()
    _check(lib().fabx_score_opts_default(ctypes.byref(o)))
    return o


def fabx_score(t, opts: fabx_score_opts) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(lib().fabx_score(t, ctypes.byref(opts), ctypes.byref(h)))
    return h


def fabx_score_async(t, opts: fabx_score_opts) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(lib().fabx_score_async(t, ctypes.byref(opts), ctypes.byref(h)))
    return h


def fabx_score_noalloc(t, opts: fabx_score_opts, n_cells: int):
    """(W per cell as int64 [n_cells], stats dict) from fabx_score_noalloc."""
    w = np.zeros(max(int(n_cells), 1), dtype=np.int64)
    st = fabx_stats()
    _check(lib().fabx_score_noalloc(t, ctypes.byref(opts), w.ctypes.data_as(ctypes.POINTER(ctypes.c_int64)),
                                    ctypes.byref(st)))
    return w[:int(n_cells)], st.as_dict()


def fabx_result_wait(r) -> None:
    _check(lib().fabx_result_wait(r))


def fabx_autotune(t, opts: fabx_score_opts) -> dict:
    rep = L.fabx_tune_report()
    _check(lib().fabx_autotune(t, ctypes.byref(opts), ctypes.byref(rep)))
    return rep.as_dict()


def fabx_result_free(r) -> None:
    lib().fabx_result_free(r)


def fabx_result_num_cells(r) -> int:
    return int(lib().fabx_result_num_cells(r))


def fabx_result_cell_keys(r) -> np.ndarray:
    n, k = fabx_result_num_cells(r), int(lib().fabx_result_key_width(r))
    out = np.zeros((n, k), np.int32)
    _check(lib().fabx_result_cell_keys(r, _i32p(out)))
    return out


def fabx_result_cells(r, n_cells: Optional[int] = None):
    n_cells = fabx_result_num_cells(r) if n_cells is None else n_cells
    w = np.zeros(n_cells, np.int64)
    n = np.zeros(n_cells, np.int64)
    s = np.zeros(n_cells, np.float64)
    _check(lib().fabx_result_cells(r, _i64p(w), _i64p(n), s.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return w, n, s


def fabx_result_pairs(r, xs, ys):
    xs = np.ascontiguousarray(xs, np.int64)
    ys = np.ascontiguousarray(ys, np.int64)
    f32 = np.zeros(len(xs), np.float32)
    fl = np.zeros(len(xs), np.uint8)
    f64 = np.zeros(len(xs), np.float64)
    _check(lib().fabx_result_pairs(r, len(xs), _i64p(xs), _i64p(ys),
                                   f32.ctypes.data_as(ctypes.POINTER(ctypes.c_float)),
                                   fl.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)),
                                   f64.ctypes.data_as(ctypes.POINTER(ctypes.c_double))))
    return f32, fl, f64


def fabx_result_stats(r) -> dict:
    st = fabx_stats()
    _check(lib().fabx_result_stats(r, ctypes.byref(st)))
    return st.as_dict()


def fabx_collapse(r, levels: Optional[Sequence[Sequence[int]]] = None) -> float:
    levels = [list(l) for l in (levels or [])]
    flat = np.ascontiguousarray([a for l in levels for a in l] or [0], np.int32)
    lens = np.ascontiguousarray([len(l) for l in levels] or [0], np.int32)
    out = ctypes.c_double()
    _check(lib().fabx_collapse(r, _i32p(flat), _i32p(lens), len(levels), ctypes.byref(out)))
    return out.value


def fabx_server_create(ctx, hbm_budget_bytes: int, n_streams: int) -> ctypes.c_void_p:
    h = ctypes.c_void_p()
    _check(lib().fabx_server_create(ctx, int(hbm_budget_bytes), int(n_streams), ctypes.byref(h)))
    return h


def fabx_server_destroy(srv) -> None:
    lib().fabx_server_destroy(srv)


def fabx_server_submit(srv, ds, on, by, across, opts: fabx_score_opts) -> int:
    b = np.ascontiguousarray(list(by), dtype=np.int32)
    a = np.ascontiguousarray(list(across), dtype=np.int32)
    jid = ctypes.c_uint64()
    _check(lib().fabx_server_submit(srv, ds, int(on), _i32p(b), len(b), _i32p(a), len(a),
                                    ctypes.byref(opts), ctypes.byref(jid)))
    return int(jid.value)


def fabx_server_poll(srv, job_id: int):
    """(status, result handle or None); status FABX_OK, FABX_EAGAIN or an error code."""
    h = ctypes.c_void_p()
    rc = lib().fabx_server_poll(srv, ctypes.c_uint64(job_id), ctypes.byref(h))
    return rc, (h if rc == 0 else None)


def fabx_server_wait(srv, job_id: int):
    h = ctypes.c_void_p()
    rc = lib().fabx_server_wait(srv, ctypes.c_uint64(job_id), ctypes.byref(h))
    return rc, (h if rc == 0 else None)


def fabx_server_cancel(srv, job_id: int) -> int:
    return int(lib().fabx_server_cancel(srv, ctypes.c_uint64(job_id)))


def fabx_server_stats_get(srv) -> dict:
    st = fabx_server_stats()
    _check(lib().fabx_server_stats_get(srv, ctypes.byref(st)))
    return st.as_dict()


# ----------------------------------------------------------- convenience --

def make_opts(mode: str = "dtw", precision: str = "bf16", norm: str = "path", margin: float = -1.0,
              delta: float = -1.0, keep_pairs: bool = False, fused_cols: int = 0,
              fused_blocks_per_cu: int = 0, distance: str = "angular") -> fabx_score_opts:
    o = fabx_score_opts_default()
    o.distance = {"angular": FABX_DISTANCE_ANGULAR, "euclidean": FABX_DISTANCE_EUCLIDEAN,
                  "units": FABX_DISTANCE_UNITS}[distance]
    o.mode = {"dtw": FABX_MODE_DTW, "pooled": FABX_MODE_POOLED}[mode]
    o.precision = {"fp32": FABX_PREC_FP32, "bf16": FABX_PREC_BF16_RECHECK}[precision]
    o.dtw_norm = {"path": FABX_NORM_PATH, "none": FABX_NORM_NONE}[norm]
    o.margin = float(margin)
    o.delta = float(delta)
    o.keep_pairs = 1 if keep_pairs else 0
    o.fused_cols = int(fused_cols)
    o.fused_blocks_per_cu = int(fused_blocks_per_cu)
    return o


def fabx_probe_stream(src, dst, stream=None) -> None:
    """The HBM streaming probe (measurement only): src float32 [n_rows, dim] and
    dst bfloat16 [n_rows, dim_pad] device tensors, on the given raw stream
    (default: torch's current stream of src's device)."""
    n_rows, dim = int(src.shape[0]), int(src.shape[1])
    if dst.shape[0] != n_rows or dst.shape[1] != (dim + 63) // 64 * 64:
        raise ValueError("dst must be [n_rows, dim rounded up to 64]")
    if stream is None:
        stream = _current_stream_ptr(src.device.index)
    _check(lib().fabx_probe_stream(ctypes.c_void_p(src.data_ptr()), ctypes.c_void_p(dst.data_ptr()), n_rows, dim,
                                   stream))


def _current_stream_ptr(device: int):
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(device).cuda_stream)


class Context:
    """A device (or, with device=-1, a host-only context that can build tasks but not score).

    All device work of the context goes on one HIP stream, in order after what
    was enqueued there before: by default torch's current stream at creation
    (so features made by torch on it need no synchronisation), ``None`` for the
    null stream, or a raw ``hipStream_t`` value."""

    def __init__(self, device: int = 0, stream="torch"):
        self.device = device
        s = None
        if device >= 0 and stream == "torch":
            s = _current_stream_ptr(device)
        elif stream not in (None, "torch"):
            s = ctypes.c_void_p(int(stream))
        self.h = fabx_create(device, s)

    def __del__(self):
        if getattr(self, "h", None) and L is not None and L._lib is not None:
            fabx_destroy(self.h)
            self.h = None


class Dataset:
    """Ragged features (device tensor [n_frames, dim], float32 or bfloat16; or
    int32 unit codes [n_frames] of a discrete representation) + attribute table."""

    def __init__(self, ctx: Context, features, offsets, attrs):
        self.ctx = ctx
        self.features = features  # keep the borrowed tensor alive
        offsets = np.ascontiguousarray(offsets, np.int64)
        attrs = np.ascontiguousarray(attrs, np.int32)
        if features is None:
            ptr, dtype, nf, dim = None, FABX_DTYPE_F32, int(offsets[-1]), 1
        else:
            import torch
            if not features.is_contiguous():
                raise ValueError("features must be contiguous")
            dtype = {torch.float32: FABX_DTYPE_F32, torch.bfloat16: FABX_DTYPE_BF16,
                     torch.int32: FABX_DTYPE_UNITS}[features.dtype]
            nf = int(features.shape[0])
            dim = 1 if features.dim() == 1 else int(features.shape[1])
            ptr = features.data_ptr()
        self.h = fabx_dataset_create(ctx.h, ptr, dtype, nf, dim, offsets, attrs)

    @classmethod
    def windows(cls, ctx: Context, features, item_start, item_len, attrs) -> "Dataset":
        """Items as windows features[item_start[i] : item_start[i] + item_len[i]]
        of one feature tensor; windows may overlap (no copy is made)."""
        import torch
        self = cls.__new__(cls)
        self.ctx = ctx
        self.features = features
        if not features.is_contiguous():
            raise ValueError("features must be contiguous")
        dtype = {torch.float32: FABX_DTYPE_F32, torch.bfloat16: FABX_DTYPE_BF16}[features.dtype]
        self.h = fabx_dataset_create_windows(ctx.h, features.data_ptr(), dtype, int(features.shape[0]),
                                             int(features.shape[1]), item_start, item_len, attrs)
        return self

    @classmethod
    def from_item_file(cls, ctx: Context, item_path: str, features, frame_step: float,
                       libri_light: bool = False):
        """A dataset from an item file and the features of whole files.

        ``features`` maps each file name of the item file to its feature tensor
        [n_frames, dim] on the context's device (frame i at time frame_step / 2
        + i frame_step).  Each unit keeps the frames fabx_slice_frames gives
        (libri_light: the Libri-Light slicing, one frame fewer); a unit with no
        frame, or one past the end of its file's frames, raises ValueError.
        The file tensors are concatenated once on the device and every unit is
        a window of the result.  Attribute columns are label-encoded in sorted
        order of their values.  Returns (dataset, names, vocab): vocab[j][v] is
        the value behind code v of attribute column j (names[j])."""
        import torch
        names, files, onset, offset, vals = read_item_file(item_path)
        if not files:
            raise ValueError(f"{item_path}: no unit")
        order = sorted(set(files))
        missing = [f for f in order if f not in features]
        if missing:
            raise ValueError(f"no features for file {missing[0]!r}")
        base, n = {}, 0
        for f in order:
            base[f] = n
            n += int(features[f].shape[0])
        start, length = fabx_slice_frames(onset, offset, frame_step, libri_light)
        for k, f in enumerate(files):
            if length[k] < 1:
                raise ValueError(f"unit {k} ({f} {onset[k]} {offset[k]}) keeps no frame")
            if start[k] + length[k] > int(features[f].shape[0]):
                raise ValueError(f"unit {k} ({f} {onset[k]} {offset[k]}) ends past the file's "
                                 f"{int(features[f].shape[0])} frames")
        feats = torch.cat([features[f] for f in order]).contiguous()
        item_start = np.array([base[f] for f in files], np.int64) + start
        cols = np.array(vals, dtype=object).reshape(len(files), len(names))
        vocab, codes = [], np.zeros((len(files), len(names)), np.int32)
        for j in range(len(names)):
            v, c = np.unique(cols[:, j].astype(str), return_inverse=True)
            vocab.append(v)
            codes[:, j] = c
        return cls.windows(ctx, feats, item_start, length, codes), names, vocab

    def __del__(self):
        if getattr(self, "h", None) and L is not None and L._lib is not None:
            fabx_dataset_destroy(self.h)
            self.h = None


class Subsampler:
    """The Subsampler of the Task interface (fabx_subsampler): per cell at most
    max_a / max_b / max_x items of A / B / X, and with ACROSS attributes at most
    max_x_across cells per (on_ax, on_b, by, across_ab); 0 means no cap."""

    def __init__(self, seed: int = 0, max_a: int = 0, max_b: int = 0, max_x: int = 0, max_x_across: int = 0):
        self.seed, self.max_a, self.max_b, self.max_x = int(seed), int(max_a), int(max_b), int(max_x)
        self.max_x_across = int(max_x_across)


class Task:
    def __init__(self, ds: Dataset, on: int, by: Sequence[int] = (), across: Sequence[int] = (),
                 subsampler: Optional[Subsampler] = None):
        self.ds = ds
        self.on, self.by, self.across = int(on), list(by), list(across)
        self.subsampler = subsampler
        if subsampler is None:
            self.h = fabx_task_create(ds.h, on, by, across)
        else:
            self.h = fabx_task_create_subsampled(ds.h, on, by, across, subsampler)

    def __len__(self):
        return fabx_task_num_cells(self.h)

    @property
    def keys(self) -> np.ndarray:
        return fabx_task_cell_keys(self.h)

    @property
    def sizes(self):
        return fabx_task_cell_sizes(self.h)

    def score(self, **kw) -> "Result":
        return Result(self, fabx_score(self.h, make_opts(**kw)))

    def autotune(self, **kw) -> dict:
        """Time the fused kernel's launch configurations on this task and keep the
        fastest for its shape class (see fabx_autotune)."""
        return fabx_autotune(self.h, make_opts(**kw))

    def score_async(self, **kw) -> "Result":
        """Enqueue the score and return at once; the result completes on wait()
        or on first use."""
        return Result(self, fabx_score_async(self.h, make_opts(**kw)))

    def __del__(self):
        if getattr(self, "h", None) and L is not None and L._lib is not None:
            fabx_task_destroy(self.h)
            self.h = None


class Result:
    def __init__(self, task: Task, h):
        self.task = task
        self.h = h
        self._cells = None

    def _get_cells(self):
        if self._cells is None:
            self._cells = fabx_result_cells(self.h, len(self.task))
        return self._cells

    @property
    def half_units(self) -> np.ndarray:
        return self._get_cells()[0]

    @property
    def n_triplets(self) -> np.ndarray:
        return self._get_cells()[1]

    @property
    def scores(self) -> np.ndarray:
        return self._get_cells()[2]

    @property
    def stats(self) -> dict:
        return fabx_result_stats(self.h)

    def pairs(self, xs, ys):
        return fabx_result_pairs(self.h, xs, ys)

    def collapse(self, levels=None) -> float:
        return fabx_collapse(self.h, levels)

    def wait(self) -> "Result":
        fabx_result_wait(self.h)
        return self

    def __del__(self):
        if getattr(self, "h", None) and L is not None and L._lib is not None:
            fabx_result_free(self.h)
            self.h = None


class Server:
    def __init__(self, ctx: Context, hbm_budget_bytes: int, n_streams: int = 4):
        self.ctx = ctx
        self.h = fabx_server_create(ctx.h, hbm_budget_bytes, n_streams)
        self._tasks = {}

    def submit(self, ds: Dataset, on, by=(), across=(), **kw) -> int:
        job = fabx_server_submit(self.h, ds.h, on, by, across, make_opts(**kw))
        # the dataset owns (a reference to) the borrowed feature tensor: keep it
        # alive until the job's outcome has been fetched
        self._tasks[job] = ds
        return job

    def wait(self, job_id: int):
        """Block until the job ends; returns (keys, W, |C|, D_C) and frees the native result.
        The server forgets the job once its outcome has been returned (raised)."""
        rc, h = fabx_server_wait(self.h, job_id)
        if rc != -4:   # EAGAIN cannot come from wait; any other outcome ends the job
            self._tasks.pop(job_id, None)
        if rc != 0:
            raise FabxError(rc, lib().fabx_last_error().decode())
        try:
            keys = fabx_result_cell_keys(h)
            w, n, s = fabx_result_cells(h)
        finally:
            fabx_result_free(h)
        return keys, w, n, s

    def poll(self, job_id: int):
        """(keys, W, |C|, D_C) if the job has finished, None while it is queued or
        running; raises the job's error (the server then forgets the job)."""
        rc, h = fabx_server_poll(self.h, job_id)
        if rc == -4:
            return None
        self._tasks.pop(job_id, None)
        if rc != 0:
            raise FabxError(rc, lib().fabx_last_error().decode())
        try:
            keys = fabx_result_cell_keys(h)
            w, n, s = fabx_result_cells(h)
        finally:
            fabx_result_free(h)
        return keys, w, n, s

    @property
    def stats(self) -> dict:
        return fabx_server_stats_get(self.h)

    def close(self):
        if getattr(self, "h", None):
            fabx_server_destroy(self.h)
            self.h = None
            self._tasks.clear()

    def __del__(self):
        self.close()


def zerospeech_abx(ctx: Context, item_path: str, features, frame_step: float, speaker: str = "within",
                   context: str = "within", distance: str = "angular", mode: str = "dtw",
                   precision: Optional[str] = None, libri_light: bool = False) -> float:
    """The phoneme / triphone ABX error rate as the ZeroSpeech challenges
    computed it, from an item file with columns phone, prev-phone, next-phone
    and speaker (and the features of whole utterances, as in
    Dataset.from_item_file).

    ON phone, BY context (prev-phone, next-phone) when ``context`` is
    "within" (none for "any"), and BY speaker ("within") or ACROSS speaker
    ("across"); cell scores are averaged over contexts, then over speakers,
    then over phone pairs (the collapse levels [context], [speaker]).
    ``precision`` defaults to "bf16" for the angular distance and "fp32" for
    the Euclidean one (the only form it has)."""
    if speaker not in ("within", "across"):
        raise ValueError("speaker must be 'within' or 'across'")
    if context not in ("within", "any"):
        raise ValueError("context must be 'within' or 'any'")
    ds, names, _ = Dataset.from_item_file(ctx, item_path, features, frame_step, libri_light)
    need = ["phone", "speaker"] + (["prev-phone", "next-phone"] if context == "within" else [])
    missing = [n for n in need if n not in names]
    if missing:
        raise ValueError(f"{item_path}: no column {missing[0]!r} (columns: {names})")
    on, spk = names.index("phone"), names.index("speaker")
    ctx_cols = [names.index("prev-phone"), names.index("next-phone")] if context == "within" else []
    by = ctx_cols + ([spk] if speaker == "within" else [])
    across = [spk] if speaker == "across" else []
    if precision is None:
        precision = "fp32" if distance == "euclidean" else "bf16"
    res = Task(ds, on, by, across).score(mode=mode, precision=precision, distance=distance)
    levels = ([ctx_cols] if ctx_cols else []) + [[spk]]
    return res.collapse(levels)
