"""ctypes binding of libmknn.so (argument marshalling only; every step runs in the library)."""
from __future__ import annotations

import ctypes
import os

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libmknn.so")

# status codes of mknn.h
OK, EINVAL, ENOMEM, EDUPLICATE, ENONFINITE, EHIP, ENOTFOUND, EBUSY, EUNSUPPORTED = (
    0, -1, -2, -3, -4, -5, -6, -7, -8)
STATUS_NAMES = {0: "OK", -1: "EINVAL", -2: "ENOMEM", -3: "EDUPLICATE", -4: "ENONFINITE",
                -5: "EHIP", -6: "ENOTFOUND", -7: "EBUSY", -8: "EUNSUPPORTED"}
KMAX = 64

# every symbol the public header declares, with (restype, argtypes)
_P = ctypes.c_void_p
_I32 = ctypes.c_int32
_I64 = ctypes.c_int64
_PP = ctypes.POINTER(ctypes.c_void_p)
SIGNATURES = {
    "mknn_build": (ctypes.c_int, [_P, _I64, _P, _PP]),
    "mknn_build_device": (ctypes.c_int, [_P, _I64, _P, _P, _PP]),
    "mknn_build_device_stats": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_double)]),
    "mknn_size": (_I64, [_P]),
    "mknn_successors": (ctypes.c_int, [_P, _PP, _PP, ctypes.POINTER(_I64)]),
    "mknn_points_by_rank": (ctypes.c_int, [_P, _PP]),
    "mknn_upload": (ctypes.c_int, [_P, _P]),
    "mknn_device_bytes": (_I64, [_P]),
    "mknn_knn": (ctypes.c_int, [_P, _P, _I64, _I32, _I32, _P, _P, _P]),
    "mknn_knn_static": (ctypes.c_int, [_P, _P, _I64, _I32, _I32, _P, _P, _P]),
    "mknn_knn_layout": (ctypes.c_int, [_P, ctypes.c_int32, _P, _I64, _P, _P, _P]),
    "mknn_knn_plane": (ctypes.c_int, [_P, _P, _I64, _I32, _I32, _P, _P, _P, _P]),
    "mknn_knn_var": (ctypes.c_int, [_P, _P, _I64, _P, _P, _P, _I32, _P, _P, _P]),
    "mknn_knn_counts": (ctypes.c_int, [_P, _P, _I64, _I32, _I32, _P, _P, _P, _P]),
    "mknn_timing_enable": (ctypes.c_int, [ctypes.c_int]),
    "mknn_timing_read": (ctypes.c_int, [ctypes.POINTER(ctypes.c_double), ctypes.POINTER(_I64)]),
    "mknn_probe_stream_read": (ctypes.c_int, [_P, _I64, _I32, _P, ctypes.POINTER(ctypes.c_double)]),
    "mknn_probe_gather16": (ctypes.c_int, [_P, _I64, _I64, _I32, _P,
                                           ctypes.POINTER(ctypes.c_double)]),
    "mknn_free": (None, [_P]),
    "mknn_last_error": (ctypes.c_char_p, []),
    "mknn_version": (ctypes.c_char_p, []),
}

class TuneEntry(ctypes.Structure):
    """mknn_tune_entry of mknn.h"""
    _fields_ = [("family", ctypes.c_int32), ("merge_min", ctypes.c_int32),
                ("per_wave", ctypes.c_int32), ("ms", ctypes.c_float)]


class Request(ctypes.Structure):
    """mknn_request of mknn.h"""
    _fields_ = [("cloud", ctypes.c_void_p), ("d_q", ctypes.c_void_p), ("nq", ctypes.c_int64),
                ("k", ctypes.c_int32), ("m", ctypes.c_int32), ("d_idx", ctypes.c_void_p),
                ("d_dist", ctypes.c_void_p)]


SERVER_PLAIN = 1
SERVER_BIND_AT_ADMISSION = 2
SERVER_LAZY_DELETE = 4
BATCH_NO_SORT = 1
BATCH_NO_GRAPH = 2

SIGNATURES.update({
    "mknn_batch_plan_create": (ctypes.c_int, [_I64, _I64, _I32, _I32, _PP]),
    "mknn_batch_plan_run": (ctypes.c_int, [_P, ctypes.POINTER(Request), _I32, _P]),
    "mknn_batch_plan_destroy": (None, [_P]),
    "mknn_batch_knn": (ctypes.c_int, [ctypes.POINTER(Request), _I32, _P]),
    "mknn_delete": (ctypes.c_int, [_P, _P, _I64, _P]),
    "mknn_insert": (ctypes.c_int, [_P, _P, _I64, _P]),
    "mknn_delete_lazy": (ctypes.c_int, [_P, _P, _I64, _P]),
    "mknn_delete_flush": (ctypes.c_int, [_P, _P]),
    "mknn_pending_deletes": (_I64, [_P]),
    "mknn_server_create": (ctypes.c_int, [_I64, _I32, _I32, _I32, _PP]),
    "mknn_server_submit": (ctypes.c_int, [_P, ctypes.POINTER(Request), _P, _P,
                                          ctypes.POINTER(ctypes.c_uint64)]),
    "mknn_server_delete": (ctypes.c_int, [_P, _P, _P, _I64, ctypes.POINTER(ctypes.c_uint64)]),
    "mknn_server_insert": (ctypes.c_int, [_P, _P, _P, _I64, ctypes.POINTER(ctypes.c_uint64)]),
    "mknn_server_poll": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.POINTER(_I32)]),
    "mknn_server_wait": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(_I64)]),
    "mknn_server_stats": (ctypes.c_int, [_P, ctypes.POINTER(_I64), ctypes.POINTER(_I64)]),
    "mknn_server_now": (ctypes.c_double, []),
    "mknn_server_destroy": (None, [_P]),
    "mknn_live_count": (_I64, [_P]),
    "mknn_compact": (ctypes.c_int, [_P, _P]),
    "mknn_autotune": (ctypes.c_int, [_P, _P, _I64, _I32, _I32, _P, ctypes.POINTER(TuneEntry), _I32,
                                     ctypes.POINTER(_I32), ctypes.POINTER(TuneEntry)]),
    "mknn_tune_save": (ctypes.c_int, [ctypes.c_char_p]),
    "mknn_tune_load": (ctypes.c_int, [ctypes.c_char_p]),
    "mknn_tune_reset": (None, []),
    "mknn_batch_plan_tune": (ctypes.c_int, [_P, ctypes.POINTER(Request), _I32, _P,
                                            ctypes.POINTER(_I32)]),
    "mknn_head": (_I32, [_P]),
})

_lib = None


class MknnError(RuntimeError):
    def __init__(self, status: int, message: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {message}")
        self.status = status


def lib():
    """Load libmknn.so; raises if the library has not been built (no fallback exists)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_2605_02224_amd.build`")
        # torch first: the library then binds to the HIP runtime torch has loaded, so one
        # runtime (one device context) serves both
        import torch  # noqa: F401
        h = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(h, name)
            f.restype = res
            f.argtypes = args
        _lib = h
    return _lib


def check(status: int) -> None:
    if status != OK:
        msg = lib().mknn_last_error().decode(errors="replace")
        raise MknnError(status, msg)
