"""ctypes declarations of the fastabx-hip C ABI (include/fastabx.h)."""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libfastabx_hip.so")

FABX_OK = 0
FABX_EINVAL = -1
FABX_ENOMEM = -2
FABX_EDOMAIN = -3
FABX_EAGAIN = -4
FABX_EHIP = -5
FABX_ECANCELED = -6
FABX_ENOTFOUND = -7

FABX_DTYPE_F32 = 0
FABX_DTYPE_BF16 = 1
FABX_DTYPE_UNITS = 2
FABX_DISTANCE_ANGULAR = 0
FABX_DISTANCE_EUCLIDEAN = 1
FABX_DISTANCE_UNITS = 2
FABX_MODE_DTW = 0
FABX_MODE_POOLED = 1
FABX_PREC_FP32 = 0
FABX_PREC_BF16_RECHECK = 1
FABX_NORM_PATH = 0
FABX_NORM_NONE = 1
FABX_MAX_ITEM_FRAMES = 1024
FABX_NOALLOC_SCRATCH_BYTES = 256 * 1024 * 1024

STATUS_NAMES = {0: "FABX_OK", -1: "FABX_EINVAL", -2: "FABX_ENOMEM", -3: "FABX_EDOMAIN",
                -4: "FABX_EAGAIN", -5: "FABX_EHIP", -6: "FABX_ECANCELED", -7: "FABX_ENOTFOUND"}


class fabx_dataset_desc(ctypes.Structure):
    _fields_ = [("features", ctypes.c_void_p), ("dtype", ctypes.c_int32), ("n_frames", ctypes.c_int64),
                ("dim", ctypes.c_int32), ("offsets", ctypes.POINTER(ctypes.c_int64)),
                ("n_items", ctypes.c_int64), ("attrs", ctypes.POINTER(ctypes.c_int32)),
                ("n_attr", ctypes.c_int32)]


class fabx_score_opts(ctypes.Structure):
    _fields_ = [("distance", ctypes.c_int32), ("mode", ctypes.c_int32), ("precision", ctypes.c_int32),
                ("dtw_norm", ctypes.c_int32), ("margin", ctypes.c_double), ("delta", ctypes.c_double),
                ("keep_pairs", ctypes.c_int32), ("fused_cols", ctypes.c_int32),
                ("fused_blocks_per_cu", ctypes.c_int32)]


class fabx_subsampler(ctypes.Structure):
    _fields_ = [("seed", ctypes.c_uint64), ("max_a", ctypes.c_int32), ("max_b", ctypes.c_int32),
                ("max_x", ctypes.c_int32), ("max_x_across", ctypes.c_int32)]


class fabx_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in (
        "n_cells", "n_triplets", "n_items", "n_frames", "n_pairs", "dtw_cells", "computed_dtw_cells",
        "n_nonrobust_pairs", "n_recheck_pairs", "n_recount_rows", "workspace_bytes")] + \
        [(n, ctypes.c_double) for n in ("ms_total", "ms_normalize", "ms_distance", "ms_triplets",
                                         "ms_recheck", "ms_host_setup", "ms_host_finish", "margin", "delta")] + \
        [("fused_cols", ctypes.c_int32), ("fused_blocks_per_cu", ctypes.c_int32),
         ("dtw_cells_sym", ctypes.c_int64)]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


class fabx_tune_entry(ctypes.Structure):
    _fields_ = [("cols", ctypes.c_int32), ("blocks_per_cu", ctypes.c_int32), ("ms_distance", ctypes.c_double)]


class fabx_tune_report(ctypes.Structure):
    _fields_ = [("n_tried", ctypes.c_int32), ("best", ctypes.c_int32), ("key_dim_pad", ctypes.c_int32),
                ("key_max_len", ctypes.c_int32), ("key_frames_log2", ctypes.c_int32),
                ("tried", fabx_tune_entry * 8)]

    def as_dict(self):
        tried = [{"cols": e.cols, "blocks_per_cu": e.blocks_per_cu, "ms_distance": e.ms_distance}
                 for e in self.tried[: self.n_tried]]
        return {"tried": tried, "best": tried[self.best] if self.best >= 0 else None,
                "key": {"dim_pad": self.key_dim_pad, "max_len": self.key_max_len,
                        "frames_log2": self.key_frames_log2}}


class fabx_server_stats(ctypes.Structure):
    _fields_ = [(n, ctypes.c_int64) for n in ("submitted", "completed", "cancelled", "failed", "queued",
                                              "running", "hbm_in_use", "hbm_high_water")] + \
        [(n, ctypes.c_double) for n in ("p50_ms", "p99_ms", "p50_queue_ms", "p99_queue_ms", "mean_build_ms",
                                         "mean_queue_ms", "mean_run_ms")]

    def as_dict(self):
        return {n: getattr(self, n) for n, _ in self._fields_}


_P = ctypes.POINTER
_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64

# name -> (restype, argtypes)
SIGNATURES = {
    "fabx_last_error": (ctypes.c_char_p, []),
    "fabx_version": (ctypes.c_char_p, []),
    "fabx_set_thread_serial": (ctypes.c_int, [ctypes.c_int]),
    "fabx_create": (ctypes.c_int, [_P(_vp), ctypes.c_int, _vp]),
    "fabx_destroy": (None, [_vp]),
    "fabx_dataset_create": (ctypes.c_int, [_vp, _P(fabx_dataset_desc), _P(_vp)]),
    "fabx_dataset_create_windows": (ctypes.c_int, [_vp, _vp, _i32, _i64, _i32, _P(_i64), _P(_i64), _i64,
                                                   _P(_i32), _i32, _P(_vp)]),
    "fabx_dataset_destroy": (None, [_vp]),
    "fabx_slice_frames": (ctypes.c_int, [_P(ctypes.c_double), _P(ctypes.c_double), _i64, ctypes.c_double,
                                         ctypes.c_int, _P(_i64), _P(_i64)]),
    "fabx_task_create": (ctypes.c_int, [_vp, _i32, _P(_i32), _i32, _P(_i32), _i32, _P(_vp)]),
    "fabx_task_create_subsampled": (ctypes.c_int, [_vp, _i32, _P(_i32), _i32, _P(_i32), _i32,
                                                   _P(fabx_subsampler), _P(_vp)]),
    "fabx_task_destroy": (None, [_vp]),
    "fabx_task_num_cells": (_i64, [_vp]),
    "fabx_task_key_width": (_i32, [_vp]),
    "fabx_task_cell_keys": (ctypes.c_int, [_vp, _P(_i32)]),
    "fabx_task_cell_sizes": (ctypes.c_int, [_vp, _P(_i64), _P(_i32)]),
    "fabx_score_opts_default": (ctypes.c_int, [_P(fabx_score_opts)]),
    "fabx_score": (ctypes.c_int, [_vp, _P(fabx_score_opts), _P(_vp)]),
    "fabx_score_async": (ctypes.c_int, [_vp, _P(fabx_score_opts), _P(_vp)]),
    "fabx_score_noalloc": (ctypes.c_int, [_vp, _P(fabx_score_opts), _P(_i64), _P(fabx_stats)]),
    "fabx_result_wait": (ctypes.c_int, [_vp]),
    "fabx_autotune": (ctypes.c_int, [_vp, _P(fabx_score_opts), _P(fabx_tune_report)]),
    "fabx_probe_stream": (ctypes.c_int, [_vp, _vp, _i64, ctypes.c_int32, _vp]),
    "fabx_result_free": (None, [_vp]),
    "fabx_result_num_cells": (_i64, [_vp]),
    "fabx_result_key_width": (_i32, [_vp]),
    "fabx_result_cell_keys": (ctypes.c_int, [_vp, _P(_i32)]),
    "fabx_result_cells": (ctypes.c_int, [_vp, _P(_i64), _P(_i64), _P(ctypes.c_double)]),
    "fabx_result_pairs": (ctypes.c_int, [_vp, _i64, _P(_i64), _P(_i64), _P(ctypes.c_float),
                                         _P(ctypes.c_uint8), _P(ctypes.c_double)]),
    "fabx_result_stats": (ctypes.c_int, [_vp, _P(fabx_stats)]),
    "fabx_collapse": (ctypes.c_int, [_vp, _P(_i32), _P(_i32), _i32, _P(ctypes.c_double)]),
    "fabx_server_create": (ctypes.c_int, [_vp, _i64, _i32, _P(_vp)]),
    "fabx_server_destroy": (None, [_vp]),
    "fabx_server_submit": (ctypes.c_int, [_vp, _vp, _i32, _P(_i32), _i32, _P(_i32), _i32,
                                          _P(fabx_score_opts), _P(ctypes.c_uint64)]),
    "fabx_server_poll": (ctypes.c_int, [_vp, ctypes.c_uint64, _P(_vp)]),
    "fabx_server_wait": (ctypes.c_int, [_vp, ctypes.c_uint64, _P(_vp)]),
    "fabx_server_cancel": (ctypes.c_int, [_vp, ctypes.c_uint64]),
    "fabx_server_stats_get": (ctypes.c_int, [_vp, _P(fabx_server_stats)]),
}

_lib = None


def load() -> ctypes.CDLL:
    """Load the built library; fail loudly when it is missing (no fallback)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(
                f"fastabx-hip native library not found at {LIB_PATH}; build it with "
                "`python -m paper_2505_02692_amd.build` (hipcc, gfx950)")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib
