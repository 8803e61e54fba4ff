"""ctypes view of the C ABI in include/tc_dtw.h (argument marshalling only).

The shared library libtcdtw.so sits next to this file (built by
csrc/build.py).  Loading fails loudly when it is missing: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes as C
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libtcdtw.so")

OK, ERR_INVALID, ERR_WORKSPACE, ERR_UNSUPPORTED, ERR_DEVICE = range(5)
F64 = 1
ABI_VERSION = 7


class TcDtwError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("tc_dtw status %d: %s" % (status, msg))
        self.status = status


class Batch(C.Structure):
    _fields_ = [("data", C.c_void_p), ("offset", C.POINTER(C.c_int64)),
                ("len", C.POINTER(C.c_int32)), ("count", C.c_int32), ("dim", C.c_int32),
                ("uniform_len", C.c_int32), ("dims", C.POINTER(C.c_int32))]


class Tuning(C.Structure):
    _fields_ = [("diag_max_w", C.c_int32), ("waves_per_cu", C.c_int32), ("waves_per_pair", C.c_int32)]


PLAN_MAX_CLASSES = 32


class PlanClass(C.Structure):
    _fields_ = [("rows", C.c_int32), ("wodd", C.c_int32), ("dim", C.c_int32), ("nitems", C.c_int32),
                ("maxm", C.c_int32), ("maxn", C.c_int32), ("maxw", C.c_int32), ("waves_per_pair", C.c_int32),
                ("max_words", C.c_int64), ("desc_off", C.c_int64), ("work", C.c_double),
                ("stream", C.c_int32), ("reserved", C.c_int32)]


class PairsPlan(C.Structure):
    _fields_ = [("buf", C.c_void_p), ("bytes", C.c_size_t), ("npairs", C.c_int32), ("nclasses", C.c_int32),
                ("waves_per_cu", C.c_int32), ("reserved", C.c_int32), ("saved_bytes", C.c_int64),
                ("cls", PlanClass * PLAN_MAX_CLASSES)]


class Window(C.Structure):
    _fields_ = [("window", C.c_int32), ("frac_num", C.c_int32), ("frac_den", C.c_int32)]


MAX_BANKS = 8


class Index(C.Structure):
    _fields_ = [("buf", C.c_void_p), ("bytes", C.c_size_t), ("count", C.c_int32), ("dim", C.c_int32),
                ("uniform_len", C.c_int32), ("max_len", C.c_int32), ("ntiles", C.c_int32),
                ("nbanks", C.c_int32), ("off_series", C.c_int64), ("off_tiles", C.c_int64),
                ("off_gamma", C.c_int64), ("off_meta", C.c_int64), ("off_range", C.c_int64),
                ("total_len", C.c_int64), ("off_dims", C.c_int64), ("reserved", C.c_int64 * 2),
                ("bank_dim", C.c_int32 * MAX_BANKS), ("bank_first", C.c_int32 * MAX_BANKS),
                ("bank_count", C.c_int32 * MAX_BANKS)]


class CandBoxes(C.Structure):
    _fields_ = [("buf", C.c_void_p), ("off_nbox", C.c_int64), ("count", C.c_int32), ("dim", C.c_int32),
                ("query_len", C.c_int32), ("cand_len", C.c_int32), ("weff", C.c_int32), ("groups", C.c_int32),
                ("levels", C.c_int32), ("clusters", C.c_int32), ("group", C.c_int32), ("min_cell", C.c_float)]


class KnnParams(C.Structure):
    _fields_ = [("window", Window), ("bounds", C.c_uint32), ("early_abandon", C.c_int32),
                ("ti_period", C.c_int32), ("ti_top", C.c_int32), ("pc_levels", C.c_int32),
                ("pc_clusters", C.c_int32), ("pc_group", C.c_int32), ("pc_min_cell", C.c_float),
                ("trigger_ti", C.c_float), ("trigger_pc", C.c_float), ("prune_margin", C.c_float),
                ("seed_r", C.c_int32), ("k", C.c_int32), ("independent", C.c_int32),
                ("pc_cand", C.POINTER(CandBoxes)), ("reuse_query_meta", C.c_int32)]


class KnnStats(C.Structure):
    _fields_ = [("pairs", C.c_uint64), ("pruned_mv", C.c_uint64), ("pruned_pc", C.c_uint64),
                ("pruned_ti", C.c_uint64), ("dtw_started", C.c_uint64), ("dtw_abandoned", C.c_uint64),
                ("dtw_completed", C.c_uint64), ("cells", C.c_uint64), ("rescored", C.c_uint64),
                ("stage_ms", C.c_float * 8), ("evaluated_pc", C.c_uint64), ("evaluated_ti", C.c_uint64),
                ("lb_ti_ms", C.c_float)]


LB_MV, LB_PC, LB_TI = 1, 2, 4

_lib = None

# name -> (restype, argtypes)
_SIGS = {
    "tc_dtw_abi_version": (C.c_int, []),
    "tc_dtw_last_error": (C.c_char_p, []),
    "tc_dtw_status_string": (C.c_char_p, [C.c_int]),
    "tc_dtw_sync_status": (C.c_int, [C.c_void_p]),
    "tc_dtw_banded_workspace_bytes": (C.c_size_t, [C.POINTER(Batch), C.POINTER(Batch), Window, C.c_uint32]),
    "tc_dtw_saved_bytes": (C.c_size_t, [C.POINTER(Batch), C.POINTER(Batch), Window]),
    "tc_dtw_banded": (C.c_int, [C.POINTER(Batch), C.POINTER(Batch), Window, C.c_uint32, C.c_void_p,
                                C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "tc_dtw_noalloc_scratch_bytes": (C.c_size_t, []),
    "tc_dtw_banded_noalloc": (C.c_int, [C.POINTER(Batch), C.POINTER(Batch), Window, C.c_uint32, C.c_void_p,
                                        C.c_void_p, C.c_void_p]),
    "tc_dtw_backward_workspace_bytes": (C.c_size_t, [C.POINTER(Batch), C.POINTER(Batch), Window]),
    "tc_dtw_backward": (C.c_int, [C.POINTER(Batch), C.POINTER(Batch), Window, C.c_void_p, C.c_void_p,
                                  C.c_void_p, C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "tc_dtw_pairs_plan_bytes": (C.c_size_t, [C.POINTER(Batch), C.POINTER(Batch), Window, C.POINTER(Tuning)]),
    "tc_dtw_pairs_plan_build": (C.c_int, [C.POINTER(Batch), C.POINTER(Batch), Window, C.POINTER(Tuning),
                                          C.c_void_p, C.c_size_t, C.POINTER(PairsPlan), C.c_void_p]),
    "tc_dtw_banded_run": (C.c_int, [C.POINTER(PairsPlan), C.c_void_p, C.c_void_p, C.c_uint32, C.c_void_p,
                                    C.c_void_p, C.c_void_p]),
    "tc_dtw_backward_run": (C.c_int, [C.POINTER(PairsPlan), C.c_void_p, C.c_void_p, C.c_void_p, C.c_void_p,
                                      C.c_void_p, C.c_void_p, C.c_void_p]),
    "tc_dtw_index_bytes": (C.c_size_t, [C.POINTER(Batch)]),
    "tc_dtw_build_index": (C.c_int, [C.POINTER(Batch), C.c_void_p, C.c_size_t, C.POINTER(Index), C.c_void_p]),
    "tc_dtw_knn_params_default": (None, [C.POINTER(KnnParams)]),
    "tc_dtw_cand_boxes_bytes": (C.c_size_t, [C.POINTER(Index), C.c_int32, C.POINTER(KnnParams)]),
    "tc_dtw_build_cand_boxes": (C.c_int, [C.POINTER(Index), C.c_int32, C.POINTER(KnnParams), C.c_void_p,
                                          C.c_size_t, C.POINTER(CandBoxes), C.c_void_p]),
    "tc_dtw_lower_bounds_workspace_bytes": (C.c_size_t, [C.POINTER(Index), C.POINTER(Batch),
                                                         C.POINTER(KnnParams), C.c_uint32]),
    "tc_dtw_lower_bounds": (C.c_int, [C.POINTER(Index), C.POINTER(Batch), C.POINTER(KnnParams), C.c_uint32,
                                      C.c_void_p, C.c_void_p, C.c_size_t, C.c_void_p]),
    "tc_dtw_knn_workspace_bytes": (C.c_size_t, [C.POINTER(Index), C.POINTER(Batch), C.POINTER(KnnParams)]),
    "tc_dtw_knn": (C.c_int, [C.POINTER(Index), C.POINTER(Batch), C.POINTER(KnnParams), C.c_void_p, C.c_void_p,
                             C.POINTER(KnnStats), C.c_void_p, C.c_size_t, C.c_void_p]),
}


def lib():
    """Load libtcdtw.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError("libtcdtw.so is not built (run __graft_entry__.build() or "
                          "python paper_2101_07731_amd/csrc/build.py): " + LIB_PATH)
    L = C.CDLL(LIB_PATH)
    for name, (res, args) in _SIGS.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    if L.tc_dtw_abi_version() != ABI_VERSION:
        raise ImportError("libtcdtw.so ABI version mismatch")
    _lib = L
    return L


def check(status):
    if status != OK:
        raise TcDtwError(status, lib().tc_dtw_last_error().decode())
