"""ctypes declarations of libte.so (include/te.h).  Loading fails loudly when the
library has not been built; there is no fallback implementation."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
# TE_LIB_PATH selects another build of the same library (e.g. a tuning variant).
LIB_PATH = os.environ.get("TE_LIB_PATH") or os.path.join(HERE, "libte.so")

TE_OK, TE_ERR_INVALID, TE_ERR_NOMEM, TE_ERR_DEVICE, TE_ERR_BUSY, TE_ERR_TIMEOUT, TE_ERR_CANCELLED = range(7)
STATUS_NAMES = {0: "TE_OK", 1: "TE_ERR_INVALID", 2: "TE_ERR_NOMEM", 3: "TE_ERR_DEVICE", 4: "TE_ERR_BUSY",
                5: "TE_ERR_TIMEOUT", 6: "TE_ERR_CANCELLED"}


class TEError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__("%s: %s" % (STATUS_NAMES.get(status, status), message))
        self.status = status


class Problem(ctypes.Structure):
    _fields_ = [
        ("n_pairs", ctypes.c_int32), ("n_trials", ctypes.c_int32), ("n_samples", ctypes.c_int32),
        ("d_y", ctypes.c_int32), ("d_x", ctypes.c_int32), ("tau", ctypes.c_int32), ("u", ctypes.c_int32),
        ("k", ctypes.c_int32), ("n_points", ctypes.c_int32), ("window", ctypes.c_int32),
        ("window_start", ctypes.POINTER(ctypes.c_int32)), ("window_len", ctypes.POINTER(ctypes.c_int32)),
        ("trials", ctypes.POINTER(ctypes.c_int32)), ("n_surrogates", ctypes.c_int32),
        ("cond_source", ctypes.c_int32), ("seed", ctypes.c_uint64),
    ]


class ServeStats(ctypes.Structure):
    _fields_ = [("p50_s", ctypes.c_double), ("p99_s", ctypes.c_double), ("est_per_s", ctypes.c_double),
                ("completed", ctypes.c_int64), ("failed", ctypes.c_int64), ("cancelled", ctypes.c_int64),
                ("steps", ctypes.c_int64), ("queued", ctypes.c_int64), ("resident", ctypes.c_int64),
                ("peak_slots", ctypes.c_int64), ("peak_bytes", ctypes.c_int64)]


TE_SERVE_DRY_RUN = 1
TE_SERVE_HOLD = 2

_lib = None

_vp = ctypes.c_void_p
_sz = ctypes.c_size_t
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_st = ctypes.c_int
_dp = ctypes.POINTER(ctypes.c_double)
_szp = ctypes.POINTER(ctypes.c_size_t)

SIGNATURES = {
    "te_version": ([], ctypes.c_char_p),
    "te_last_error": ([], ctypes.c_char_p),
    "te_plan_create": ([ctypes.POINTER(Problem), ctypes.POINTER(_vp)], _st),
    "te_plan_destroy": ([_vp], _st),
    "te_plan_workspace_bytes": ([_vp, _szp, _szp, _szp], _st),
    "te_estimate": ([_vp, _vp, _vp, _vp, _sz, _vp, _dp], _st),
    "te_estimate_each": ([_vp, _vp, _vp, _vp, _vp, _sz, _vp, _dp, _dp, _dp], _st),
    "te_surrogates": ([_vp, _vp, _vp, _vp, _vp, _sz, _vp, _i32, _dp, _dp, _dp], _st),
    "te_surrogates_async": ([_vp, _vp, _vp, _vp, _vp, _sz, _vp, _vp], _st),
    "te_knn_counts_workspace_bytes": ([_i32, _i64], _sz),
    "te_profile_enable": ([_i32], _st),
    "te_profile_read": ([_dp, ctypes.POINTER(_i64), _i32], _st),
    "te_profile_work": ([ctypes.POINTER(_i64), ctypes.POINTER(_i64), _i32], _st),
    "te_profile_work_all": ([ctypes.POINTER(_i64), _i32], _st),
    "te_serve_open": ([_vp, _sz, _i32, _i32, _i64, _i32, ctypes.POINTER(_vp)], _st),
    "te_serve_submit": ([_vp, ctypes.POINTER(Problem), _vp, _vp, _vp, ctypes.POINTER(ctypes.c_uint64)], _st),
    "te_serve_wait": ([_vp, ctypes.c_uint64, _i64, _dp, _dp, _dp], _st),
    "te_serve_resume": ([_vp], _st),
    "te_serve_cancel": ([_vp, ctypes.c_uint64], _st),
    "te_serve_stats": ([_vp, ctypes.POINTER(ServeStats)], _st),
    "te_serve_close": ([_vp], _st),
    "te_plan_local_offsets": ([_vp, ctypes.POINTER(_i64)], _st),
    "te_plan_permutations_workspace_bytes": ([_vp], _sz),
    "te_plan_permutations": ([_vp, _vp, _sz, _vp, _vp], _st),
    "te_local": ([_vp, _vp, _vp, _vp, _sz, _vp, _vp, _dp], _st),
    "te_delay_scan_workspace_bytes": ([_vp, _vp, _i32, _szp, _szp], _st),
    "te_delay_scan": ([_vp, _vp, _vp, _vp, _vp, _i32, _vp, _sz, _vp, _dp, _vp, _dp, _dp], _st),
    "te_autotune": ([_i32, _i32, _i32, _i32, _i32, _vp, _sz, _vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                     ctypes.POINTER(_i32), _dp], _st),
    "te_plan_autotune": ([_vp, _vp, _vp, _vp, _vp, _sz, _vp, ctypes.POINTER(_i32), ctypes.POINTER(_i32),
                          ctypes.POINTER(_i32), _dp], _st),
    "te_tune_save": ([ctypes.c_char_p], _st),
    "te_tune_load": ([ctypes.c_char_p], _st),
    "te_tune_clear": ([], _st),
    "te_knn_counts": ([_vp, _i64, ctypes.POINTER(_i64), _i32, _i32, _i32, _i32, _vp, _sz, _vp, _vp, _vp, _dp], _st),
    "te_knn_counts_noalloc": ([_vp, _i64, ctypes.POINTER(_i64), _i32, _i32, _i32, _i32, _vp, _vp, _vp, _dp], _st),
    "te_ragwitz_workspace_bytes": ([_i32, _i32, ctypes.POINTER(_i32), _i32, _szp], _st),
    "te_ragwitz": ([_vp, _i32, _i32, _i32, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32), _i32, _i32, _vp, _sz, _vp,
                    _vp, _dp], _st),
}

# TE_NOALLOC_SCRATCH_BYTES of te.h: the static scratch of te_knn_counts_noalloc, per device
NOALLOC_SCRATCH_BYTES = 32 << 20


def lib():
    """The loaded libte.so.  Raises if it is missing: build it with __graft_entry__.build()."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("libte.so is not built (expected at %s); run `python -c \"import "
                               "__graft_entry__ as g; g.build()\"`" % LIB_PATH)
        L = ctypes.CDLL(LIB_PATH)
        for name, (args, res) in SIGNATURES.items():
            f = getattr(L, name)
            f.argtypes = args
            f.restype = res
        _lib = L
    return _lib


def check(status: int):
    if status != TE_OK:
        raise TEError(status, lib().te_last_error().decode(errors="replace"))
