"""ctypes declarations of libqsw (include/qsw.h).  Argument marshalling only."""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libqsw.so")

QSW_OK = 0
STATUS_NAMES = {0: "QSW_OK", 1: "QSW_ERR_ARG", 2: "QSW_ERR_GRAPH", 3: "QSW_ERR_OOM",
                4: "QSW_ERR_DEVICE", 5: "QSW_ERR_NONFINITE", 6: "QSW_ERR_STATE",
                7: "QSW_ERR_SIZE", 8: "QSW_ERR_SCRATCH"}

QSW_H_LAPLACIAN = 0
QSW_H_ADJACENCY = 1
QSW_R_TRANSITION = 0
QSW_R_COLNORM = 2
QSW_DEPHASING = 4
QSW_PREC_DOUBLE = 0
QSW_PREC_SINGLE = 1
QSW_PREC_FP32 = 2
QSW_PARAMS_KNOWN_NORMS = 16
PREC_NAMES = {0: "double", 1: "single", 2: "fp32"}
NOALLOC_SCRATCH_BYTES = 80 << 20   # QSW_NOALLOC_SCRATCH_BYTES

# Every function the header declares, for the export check.
EXPORTED = ("qsw_superop_build", "qsw_superop_build_ops", "qsw_superop_build_channels",
            "qsw_superop_build_open", "qsw_superop_build_general", "qsw_superop_set_omega",
            "qsw_superop_build_demoralised", "qsw_demoralised_order", "qsw_demoralised_state",
            "qsw_demoralised_populations",
            "qsw_superop_destroy",
            "qsw_superop_info", "qsw_superop_set_precision", "qsw_superop_autotune",
            "qsw_superop_set_pacing",
            "qsw_superop_copy_csr", "qsw_propagate_workspace_bytes",
            "qsw_propagate", "qsw_propagate_noalloc", "qsw_last_stats", "qsw_apply", "qsw_populations", "qsw_theta",
            "qsw_select_params", "qsw_status_str", "qsw_version", "qsw_walk_bytes",
            "qsw_engine_table_bytes", "qsw_engine_create", "qsw_engine_submit", "qsw_engine_run",
            "qsw_engine_poll", "qsw_engine_stats", "qsw_engine_destroy",
            "qsw_batch_workspace_bytes", "qsw_batch_propagate", "qsw_server_create",
            "qsw_server_submit", "qsw_server_step", "qsw_server_poll", "qsw_server_stats",
            "qsw_server_destroy")


class QswError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        super().__init__(f"{what}: {STATUS_NAMES.get(status, status)}")


class Info(ctypes.Structure):
    _fields_ = [("N", ctypes.c_int32), ("n", ctypes.c_int64), ("nnz", ctypes.c_int64),
                ("omega", ctypes.c_double), ("norm1", ctypes.c_double),
                ("d", ctypes.c_double * 10), ("d_index", ctypes.c_int64 * 10),
                ("d_probe", ctypes.c_int32 * 10), ("norm_products", ctypes.c_int32),
                ("build_ms", ctypes.c_double), ("split", ctypes.c_int32),
                ("stream_entries", ctypes.c_int64), ("shared_entries", ctypes.c_int64),
                ("distinct_entries", ctypes.c_int64), ("engine", ctypes.c_int32)]


class Stats(ctypes.Structure):
    _fields_ = [("branch", ctypes.c_int32), ("m", ctypes.c_int32), ("s", ctypes.c_int32),
                ("m0", ctypes.c_int32), ("s0", ctypes.c_int32), ("launched", ctypes.c_int64),
                ("products", ctypes.c_int64), ("nonfinite", ctypes.c_int32),
                ("ms", ctypes.c_double), ("bytes", ctypes.c_double), ("prec", ctypes.c_int32),
                ("trace_dev", ctypes.c_double)]


class Tuning(ctypes.Structure):
    _fields_ = [("staged", ctypes.c_int32), ("grid", ctypes.c_int32),
                ("us_per_product", ctypes.c_double), ("from_cache", ctypes.c_int32)]


class Walk(ctypes.Structure):
    _fields_ = [("op", ctypes.c_void_p), ("n0", ctypes.c_int32), ("rho0", ctypes.c_void_p),
                ("t0", ctypes.c_double), ("dt", ctypes.c_double), ("n_steps", ctypes.c_int32),
                ("out", ctypes.c_void_p), ("pops", ctypes.c_void_p)]


class EngineStats(ctypes.Structure):
    _fields_ = [("cycles", ctypes.c_int64), ("products", ctypes.c_int64),
                ("live", ctypes.c_int32), ("nonfinite", ctypes.c_int32), ("ms", ctypes.c_double),
                ("bytes", ctypes.c_double), ("graphs", ctypes.c_int64),
                ("graph_launches", ctypes.c_int64), ("rounds", ctypes.c_int32),
                ("staged", ctypes.c_int32), ("trace_dev", ctypes.c_double)]


class ServerStats(ctypes.Structure):
    _fields_ = [("submitted", ctypes.c_int64), ("completed", ctypes.c_int64),
                ("cache_hits", ctypes.c_int64), ("cache_misses", ctypes.c_int64),
                ("evictions", ctypes.c_int64), ("cycles", ctypes.c_int64),
                ("products", ctypes.c_int64), ("cache_bytes", ctypes.c_int64),
                ("build_ms", ctypes.c_double)]


_lib = None

_vp = ctypes.c_void_p
_i32 = ctypes.c_int32
_i64 = ctypes.c_int64
_dbl = ctypes.c_double
_u32 = ctypes.c_uint32


def load() -> ctypes.CDLL:
    """Load the in-tree libqsw.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(f"{LIB_PATH} is missing: build it with "
                           "`python -m paper_2003_02450_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    L.qsw_superop_build.restype = _i32
    L.qsw_superop_build.argtypes = [_i32, _vp, _vp, _vp, _dbl, _dbl, _u32, _vp,
                                    ctypes.POINTER(_vp)]
    L.qsw_superop_build_ops.restype = _i32
    L.qsw_superop_build_ops.argtypes = [_i32, _vp, _vp, _vp, _vp, _vp, _vp, _dbl, _u32, _vp,
                                        ctypes.POINTER(_vp)]
    L.qsw_superop_build_channels.restype = _i32
    L.qsw_superop_build_channels.argtypes = [_i32, _vp, _vp, _vp, _dbl, _dbl, _u32, _i32, _vp, _vp,
                                             _i32, _vp, _vp, _vp, ctypes.POINTER(_vp)]
    L.qsw_superop_build_open.restype = _i32
    L.qsw_superop_build_open.argtypes = [_i32, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _vp, _dbl,
                                         _u32, _vp, ctypes.POINTER(_vp)]
    L.qsw_superop_build_general.restype = _i32
    L.qsw_superop_build_general.argtypes = [_i32, _vp, _vp, _vp, _i32, _vp, _vp, _vp, _vp, _vp,
                                            _vp, _dbl, _vp, ctypes.POINTER(_vp)]
    L.qsw_superop_build_demoralised.restype = _i32
    L.qsw_superop_build_demoralised.argtypes = [_i32, _vp, _vp, _vp, _dbl, _dbl, _vp,
                                                ctypes.POINTER(_vp)]
    L.qsw_demoralised_order.restype = _i32
    L.qsw_demoralised_order.argtypes = [_i32, _vp, _vp, _vp]
    L.qsw_demoralised_state.restype = _i32
    L.qsw_demoralised_state.argtypes = [_i32, _vp, _vp, _vp]
    L.qsw_demoralised_populations.restype = _i32
    L.qsw_demoralised_populations.argtypes = [_i32, _vp, _vp, _i32, _vp]
    L.qsw_superop_set_omega.restype = _i32
    L.qsw_superop_set_omega.argtypes = [_vp, _dbl, _vp]
    L.qsw_superop_destroy.restype = None
    L.qsw_superop_destroy.argtypes = [_vp]
    L.qsw_superop_info.restype = _i32
    L.qsw_superop_info.argtypes = [_vp, ctypes.POINTER(Info)]
    L.qsw_superop_set_pacing.restype = _i32
    L.qsw_superop_set_pacing.argtypes = [_vp, _i32]
    L.qsw_superop_set_precision.restype = _i32
    L.qsw_superop_set_precision.argtypes = [_vp, _i32]
    L.qsw_superop_autotune.restype = _i32
    L.qsw_superop_autotune.argtypes = [_vp, _vp, ctypes.POINTER(Tuning)]
    L.qsw_superop_copy_csr.restype = _i32
    L.qsw_superop_copy_csr.argtypes = [_vp, _vp, _vp, _vp]
    L.qsw_propagate_workspace_bytes.restype = ctypes.c_size_t
    L.qsw_propagate_workspace_bytes.argtypes = [_vp, _dbl, _dbl, _i32]
    L.qsw_propagate.restype = _i32
    L.qsw_propagate.argtypes = [_vp, _vp, _dbl, _dbl, _i32, _vp, _vp, ctypes.c_size_t, _vp]
    L.qsw_propagate_noalloc.restype = _i32
    L.qsw_propagate_noalloc.argtypes = [_vp, _vp, _dbl, _dbl, _i32, _vp, _vp]
    L.qsw_last_stats.restype = _i32
    L.qsw_last_stats.argtypes = [_vp, ctypes.POINTER(Stats)]
    L.qsw_apply.restype = _i32
    L.qsw_apply.argtypes = [_vp, _vp, _vp, _vp]
    L.qsw_populations.restype = _i32
    L.qsw_populations.argtypes = [_vp, _vp, _i32, _vp, _vp]
    L.qsw_theta.restype = _dbl
    L.qsw_theta.argtypes = [_i32, _i32]
    L.qsw_select_params.restype = _i32
    L.qsw_select_params.argtypes = [_dbl, _vp, _dbl, _i32, _i32, ctypes.POINTER(_i32),
                                    ctypes.POINTER(_i32)]
    L.qsw_walk_bytes.restype = ctypes.c_size_t
    L.qsw_walk_bytes.argtypes = [ctypes.POINTER(Walk), _i32]
    L.qsw_engine_table_bytes.restype = ctypes.c_size_t
    L.qsw_engine_table_bytes.argtypes = [_i32]
    L.qsw_engine_create.restype = _i32
    L.qsw_engine_create.argtypes = [_i32, _i32, _vp, ctypes.c_size_t, _vp, ctypes.POINTER(_vp)]
    L.qsw_engine_submit.restype = _i32
    L.qsw_engine_submit.argtypes = [_vp, ctypes.POINTER(Walk), ctypes.POINTER(_i64)]
    L.qsw_engine_run.restype = _i32
    L.qsw_engine_run.argtypes = [_vp, _i32, ctypes.POINTER(_i32)]
    L.qsw_engine_poll.restype = _i32
    L.qsw_engine_poll.argtypes = [_vp, _vp, _i32, ctypes.POINTER(_i32)]
    L.qsw_engine_stats.restype = _i32
    L.qsw_engine_stats.argtypes = [_vp, ctypes.POINTER(EngineStats)]
    L.qsw_engine_destroy.restype = None
    L.qsw_engine_destroy.argtypes = [_vp]
    L.qsw_batch_workspace_bytes.restype = ctypes.c_size_t
    L.qsw_batch_workspace_bytes.argtypes = [ctypes.POINTER(Walk), _i32, _i32]
    L.qsw_batch_propagate.restype = _i32
    L.qsw_batch_propagate.argtypes = [ctypes.POINTER(Walk), _i32, _i32, _vp, ctypes.c_size_t, _vp,
                                      ctypes.POINTER(EngineStats)]
    L.qsw_server_create.restype = _i32
    L.qsw_server_create.argtypes = [ctypes.c_size_t, ctypes.c_size_t, _i32, _vp, ctypes.POINTER(_vp)]
    L.qsw_server_submit.restype = _i32
    L.qsw_server_submit.argtypes = [_vp, _i32, _vp, _vp, _vp, _dbl, _dbl, _u32, _vp, _dbl, _dbl,
                                    _i32, _vp, _vp, ctypes.POINTER(_i64)]
    L.qsw_server_step.restype = _i32
    L.qsw_server_step.argtypes = [_vp, _i32, ctypes.POINTER(_i32), ctypes.POINTER(_i32)]
    L.qsw_server_poll.restype = _i32
    L.qsw_server_poll.argtypes = [_vp, _vp, _vp, _i32, ctypes.POINTER(_i32)]
    L.qsw_server_stats.restype = _i32
    L.qsw_server_stats.argtypes = [_vp, ctypes.POINTER(ServerStats)]
    L.qsw_server_destroy.restype = None
    L.qsw_server_destroy.argtypes = [_vp]
    L.qsw_status_str.restype = ctypes.c_char_p
    L.qsw_status_str.argtypes = [_i32]
    L.qsw_version.restype = ctypes.c_char_p
    L.qsw_version.argtypes = []
    _lib = L
    return L


def check(status: int, what: str):
    if status != QSW_OK:
        raise QswError(status, what)
