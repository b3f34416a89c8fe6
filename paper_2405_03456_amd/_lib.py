"""ctypes declarations of the C ABI in include/hm.h.

Loading fails loudly when libhm.so has not been built: there is no fallback.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libhm.so")

c_int32, c_int64, c_double, c_void_p, c_uint32 = (ctypes.c_int32, ctypes.c_int64, ctypes.c_double,
                                                  ctypes.c_void_p, ctypes.c_uint32)
P = ctypes.POINTER

HM_OK, HM_EINVAL, HM_ENOMEM, HM_EDEVICE, HM_ELAYOUT, HM_EBUSY, HM_ENOTREADY = 0, -1, -2, -3, -4, -5, -6
HM_FMT_H, HM_FMT_UH, HM_FMT_H2 = 0, 1, 2
HM_F64, HM_F32, HM_BF16, HM_F16, HM_FP8E4M3, HM_VALR_AUTO = 0, 1, 2, 3, 4, 5
HM_FPX24, HM_FPX40, HM_FPX48, HM_FPX56 = 6, 7, 8, 9
HM_AFLP8, HM_AFLP16, HM_AFLP24, HM_AFLP32, HM_AFLP40, HM_AFLP48, HM_AFLP56 = 10, 11, 12, 13, 14, 15, 16
HM_AFLP_AUTO, HM_FPX_AUTO = 17, 18
HM_NDTYPES = 17
HM_ACC_AUTO, HM_ACC_F32, HM_ACC_F64 = 0, 1, 2
HM_CLUSTER_ORDER = 1
HM_ADJOINT = 4


HM_PART_STANDARD, HM_PART_HODLR, HM_PART_BLR = 0, 1, 2


class LayoutOpts(ctypes.Structure):
    _fields_ = [("leaf_size", c_int32), ("eta", c_double), ("partition", c_int32)]


class LayoutView(ctypes.Structure):
    _fields_ = [("n", c_int64), ("nnodes", c_int64), ("nblocks", c_int64), ("depth", c_int32),
                ("perm", P(c_int64)), ("node_begin", P(c_int64)), ("node_end", P(c_int64)),
                ("node_level", P(c_int32)), ("node_parent", P(c_int32)), ("node_son0", P(c_int32)),
                ("node_son1", P(c_int32)), ("blk_tau", P(c_int32)), ("blk_sigma", P(c_int32)),
                ("blk_adm", P(c_int32))]


HM_MAX_LEVELS = 64


class LayoutInfo(ctypes.Structure):
    _fields_ = [("n", c_int64), ("nnodes", c_int64), ("nleaves", c_int64), ("nblocks", c_int64),
                ("ndense", c_int64), ("nlowrank", c_int64), ("ndiag", c_int64), ("depth", c_int32),
                ("min_leaf", c_int32), ("max_leaf", c_int32), ("dense_area", c_double),
                ("lowrank_area", c_double), ("nodes_per_level", c_int64 * HM_MAX_LEVELS),
                ("dense_per_level", c_int64 * HM_MAX_LEVELS), ("lowrank_per_level", c_int64 * HM_MAX_LEVELS),
                ("dense_area_per_level", c_double * HM_MAX_LEVELS),
                ("lowrank_area_per_level", c_double * HM_MAX_LEVELS)]


HM_SCHED_STAGED, HM_SCHED_PERSISTENT = 0, 1


class UploadOpts(ctypes.Structure):
    _fields_ = [("task_bytes", c_int64), ("spread_dense", c_int32), ("dense_grid", c_int32),
                ("fork_after", c_int32), ("valr_promote", c_int32), ("schedule", c_int32),
                ("dense_after", c_int32), ("spin_limit_us", c_int32), ("tickets_per_grab", c_int32),
                ("sync", c_int32), ("adjoint", c_int32), ("h2_levels", c_int32),
                ("chain_task_bytes", c_int64)]


class Values(ctypes.Structure):
    _fields_ = [("dense", c_void_p), ("rank", c_void_p), ("W", c_void_p), ("sigma", c_void_p),
                ("X", c_void_p), ("row_rank", c_void_p), ("col_rank", c_void_p),
                ("row_basis", c_void_p), ("col_basis", c_void_p), ("row_transfer", c_void_p),
                ("col_transfer", c_void_p), ("row_sv", c_void_p), ("col_sv", c_void_p),
                ("coupling", c_void_p)]


class Precision(ctypes.Structure):
    _fields_ = [("eps", c_double), ("dense_dtype", c_int32), ("diag_dtype", c_int32),
                ("factor_dtype", c_int32), ("coupling_dtype", c_int32), ("accum", c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("n", c_int64), ("nblocks", c_int64), ("ndense", c_int64), ("nlowrank", c_int64),
                ("bytes_dense", c_int64), ("bytes_factors", c_int64), ("bytes_coupling", c_int64),
                ("bytes_transfer", c_int64), ("bytes_scales", c_int64), ("bytes_meta", c_int64),
                ("bytes_workspace", c_int64), ("bytes_per_dtype", c_int64 * HM_NDTYPES),
                ("entries_per_dtype", c_int64 * HM_NDTYPES), ("sum_rank", c_int64),
                ("max_rank", c_int32), ("accum", c_int32), ("nlaunch", c_int32),
                ("nowners", c_int64), ("nitems", c_int64), ("ntasks", c_int64),
                ("algorithmic_bytes", c_double), ("method_bytes", c_double)]


class PhaseTiming(ctypes.Structure):
    _fields_ = [("name", ctypes.c_char_p), ("ms_total", c_double), ("launches", c_int64),
                ("algorithmic_bytes", c_double), ("ntasks", c_int32), ("nowners", c_int32),
                ("data_bytes", c_int64), ("data_entries", c_int64), ("nrhs", c_int32),
                ("method_bytes", c_double)]


class TuneResult(ctypes.Structure):
    _fields_ = [("target_bytes", c_int64), ("nrb", c_int32), ("ms", c_double), ("ncandidates", c_int32)]


class TuneMvmResult(ctypes.Structure):
    _fields_ = [("fork_after", c_int32), ("ncandidates", c_int32), ("ms", c_double), ("ms_first", c_double),
                ("schedule", c_int32), ("dense_after", c_int32), ("ms_staged", c_double),
                ("ms_persistent", c_double), ("fork2", c_int32), ("dense_split", c_int32),
                ("dense_grid", c_int32)]


class ServeOpts(ctypes.Structure):
    _fields_ = [("mem_budget", c_int64), ("max_slots", c_int32), ("max_queue", c_int32), ("max_cols", c_int32),
                ("fake", c_int32), ("fake_us", c_int32)]


class ReqStats(ctypes.Structure):
    _fields_ = [("queue_ms", c_double), ("run_ms", c_double), ("latency_ms", c_double), ("group_id", c_int64),
                ("group_requests", c_int32), ("group_cols", c_int32)]


class ServeStats(ctypes.Structure):
    _fields_ = [("submitted", c_int64), ("completed", c_int64), ("groups", c_int64), ("peak_arena_bytes", c_int64),
                ("peak_inflight", c_int32), ("max_group_requests", c_int32)]


HM_TIMING = 2

# name -> (restype, argtypes); every exported symbol of include/hm.h
SIGNATURES = {
    "hm_build_layout": (c_int32, [P(c_double), c_int64, P(LayoutOpts), P(c_void_p)]),
    "hm_layout_export": (c_int32, [c_void_p, P(LayoutView)]),
    "hm_layout_free": (None, [c_void_p]),
    "hm_layout_stats": (c_int32, [c_void_p, P(LayoutInfo)]),
    "hm_upload": (c_int32, [c_void_p, c_int32, P(Values), P(Precision), P(UploadOpts), c_void_p, P(c_void_p)]),
    "hm_matrix_free": (None, [c_void_p]),
    "hm_matrix_stats": (c_int32, [c_void_p, P(Stats)]),
    "hm_plan_stats": (c_int32, [c_void_p, c_int32, P(Values), P(Precision), P(UploadOpts), P(Stats)]),
    "hm_mvm": (c_int32, [c_void_p, c_double, c_void_p, c_void_p, c_uint32, c_void_p]),
    "hm_matrix_check": (c_int32, [c_void_p]),
    "hm_set_schedule": (c_int32, [c_void_p, c_int32, c_int32]),
    "hm_mvm_batch": (c_int32, [P(c_void_p), c_int32, c_double, P(c_void_p), P(c_int64), P(c_int32),
                               P(c_void_p), P(c_int64), c_int32, c_uint32, c_void_p]),
    "hm_mvm_batch_noalloc": (c_int32, [P(c_void_p), c_int32, c_double, P(c_void_p), P(c_int64), P(c_int32),
                                       P(c_void_p), P(c_int64), c_int32, c_uint32, c_void_p]),
    "hm_graph_create": (c_int32, [c_void_p, c_double, c_void_p, c_void_p, c_uint32, c_void_p, P(c_void_p)]),
    "hm_tune_batch": (c_int32, [c_void_p, c_int32, c_int32, c_int32, c_void_p, P(TuneResult)]),
    "hm_tune_mvm": (c_int32, [c_void_p, c_int32, c_void_p, P(TuneMvmResult)]),
    "hm_graph_create_batch": (c_int32, [P(c_void_p), c_int32, c_double, P(c_void_p), P(c_int64), P(c_int32),
                                        P(c_void_p), P(c_int64), c_int32, c_uint32, c_void_p, P(c_void_p)]),
    "hm_graph_launch": (c_int32, [c_void_p, c_void_p]),
    "hm_graph_free": (None, [c_void_p]),
    "hm_timing_read": (c_int32, [c_void_p, P(PhaseTiming), c_int32, P(c_int32)]),
    "hm_serve_create": (c_int32, [P(ServeOpts), P(c_void_p)]),
    "hm_serve_register": (c_int32, [c_void_p, c_void_p, P(c_int32)]),
    "hm_serve_register_shape": (c_int32, [c_void_p, c_int64, P(c_int32)]),
    "hm_serve_submit": (c_int32, [c_void_p, c_int32, c_double, c_void_p, c_int32, c_void_p, P(ctypes.c_uint64)]),
    "hm_serve_poll": (c_int32, [c_void_p, ctypes.c_uint64, P(c_int32), P(ReqStats)]),
    "hm_serve_stats_read": (c_int32, [c_void_p, P(ServeStats)]),
    "hm_serve_destroy": (None, [c_void_p]),
    "hm_round_host": (c_int32, [c_int32, P(c_double), P(c_double), c_int64]),
    "hm_set_dense_split": (c_int32, [c_void_p, c_int32, c_int32]),
    "hm_codec_column": (c_int32, [c_int32, c_double, c_int32, P(c_double), c_int64, P(c_double), P(ctypes.c_uint64),
                                  P(c_int32)]),
    "hm_last_error": (ctypes.c_char_p, []),
    "hm_version": (ctypes.c_char_p, []),
}

_lib = None


class HMError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__(f"hm status {status}: {msg}")
        self.status = status


def lib():
    global _lib
    if _lib is None:
        # PyTorch ships its own HIP runtime under the same soname
        # (libamdhip64.so.7).  Loading torch first makes libhm bind to that
        # copy, so the process has a single HIP runtime and device context.
        try:
            import torch  # noqa: F401
        except ImportError:
            pass
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with paper_2405_03456_amd.build.build() "
                              "(there is no fallback path)")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def check(status):
    if status != HM_OK:
        raise HMError(status, lib().hm_last_error().decode(errors="replace"))
