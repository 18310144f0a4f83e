"""ctypes view of ``librqrcp.so`` (the C ABI in include/rqrcp.h).

Argument marshalling only: every step of the factorizations runs in the HIP
library.  Loading fails loudly when the library has not been built.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "librqrcp.so")

c_i64 = ctypes.c_int64
c_p = ctypes.c_void_p

# (name, restype, argtypes) for every exported entry point of include/rqrcp.h
SIGNATURES = {
    "rq_create": (ctypes.c_int32, [ctypes.POINTER(c_p), ctypes.c_int, c_p]),
    "rq_destroy": (ctypes.c_int32, [c_p]),
    "rq_set_stream": (ctypes.c_int32, [c_p, c_p]),
    "rq_sync_status": (ctypes.c_int32, [c_p, ctypes.POINTER(c_i64)]),
    "rq_last_error": (ctypes.c_char_p, [c_p]),
    "rq_workspace_query": (ctypes.c_int32, [c_p, ctypes.c_int32, ctypes.c_int, c_i64, c_i64, c_i64,
                                            c_i64, c_i64, ctypes.POINTER(ctypes.c_size_t)]),
    "rq_workspace_reserve": (ctypes.c_int32, [c_p, ctypes.c_size_t]),
    "rq_workspace_size": (ctypes.c_int32, [c_p, ctypes.POINTER(ctypes.c_size_t)]),
    "rqrcp_factor": (ctypes.c_int32, [c_p, c_i64, c_i64, c_i64, c_i64, c_i64, c_p, c_i64, c_p,
                                      c_i64, c_p, c_p, c_p, c_i64, c_p]),
    "rsrqrcp_factor": (ctypes.c_int32, [c_p, c_i64, c_i64, c_i64, c_i64, c_i64, c_p, c_i64, c_p,
                                        c_i64, c_i64, c_p, c_p, c_p, c_i64]),
    "qrcp_factor": (ctypes.c_int32, [c_p, c_i64, c_i64, c_i64, c_i64, c_p, c_i64, c_p, c_p]),
    "trqrcp_truncate": (ctypes.c_int32, [c_p, ctypes.c_int, c_i64, c_i64, c_i64, c_i64, c_i64,
                                         c_p, c_i64, c_p, c_i64, c_p, c_p, c_i64, c_p, c_i64,
                                         c_p, c_i64]),
    "tuxv_svd": (ctypes.c_int32, [c_p, ctypes.c_int, c_i64, c_i64, c_i64, c_i64, c_i64, c_p,
                                  c_i64, c_p, c_i64, c_p, c_i64, c_p, c_i64, c_p, c_i64, c_p, c_p]),
    "tuxv_svd_iter": (ctypes.c_int32, [c_p, ctypes.c_int, c_i64, c_i64, c_i64, c_i64, c_i64, c_p,
                                       c_i64, c_p, c_i64, c_p, c_i64, c_p, c_i64, c_p, c_i64, c_p,
                                       c_p, c_i64]),
    "rq_singular_values": (ctypes.c_int32, [c_p, c_i64, c_p, c_i64, c_p]),
    "rq_sketch": (ctypes.c_int32, [c_p, ctypes.c_int, c_i64, c_i64, c_i64, c_p, c_i64, c_p,
                                   c_i64, c_p, c_i64]),
    "rq_sample_qrcp": (ctypes.c_int32, [c_p, c_i64, c_i64, c_i64, c_p, c_i64, c_p]),
    "rq_sample_qrcp_noalloc": (ctypes.c_int32, [c_p, c_i64, c_i64, c_i64, c_p, c_i64, c_p]),
    "rq_profile_classes": (ctypes.c_int32, [c_p, ctypes.c_uint32]),
    "rq_profile_start": (ctypes.c_int32, [c_p]),
    "rq_profile_stop": (ctypes.c_int32, [c_p]),
    "rq_profile_count": (ctypes.c_int32, [c_p]),
    "rq_profile_get": (ctypes.c_int32, [c_p, ctypes.c_int32, ctypes.POINTER(ctypes.c_char_p),
                                        ctypes.POINTER(c_i64), ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_double),
                                        ctypes.POINTER(ctypes.c_double)]),
    "rq_serve_start": (ctypes.c_int32, [ctypes.c_int, ctypes.c_size_t, ctypes.c_int32, c_i64, c_i64,
                                        c_i64, c_i64, ctypes.POINTER(c_p)]),
    "rq_serve_submit": (ctypes.c_int32, [c_p, c_p, ctypes.POINTER(ctypes.c_uint64)]),
    "rq_serve_poll": (ctypes.c_int32, [c_p, ctypes.c_uint64, c_p]),
    "rq_serve_wait": (ctypes.c_int32, [c_p, ctypes.c_uint64, c_p]),
    "rq_serve_stats": (ctypes.c_int32, [c_p, ctypes.POINTER(c_i64), ctypes.POINTER(c_i64),
                                        ctypes.POINTER(ctypes.c_int32)]),
    "rq_serve_stop": (ctypes.c_int32, [c_p]),
    "rq_serve_route": (ctypes.c_int32, [ctypes.c_int32, c_i64, c_i64, c_i64, ctypes.c_double]),
}


class Request(ctypes.Structure):
    """Mirror of rq_request (include/rqrcp.h)."""
    _fields_ = [("op", ctypes.c_int32), ("prec", ctypes.c_int32), ("m", c_i64), ("n", c_i64),
                ("k", c_i64), ("b", c_i64), ("p", c_i64), ("A", c_p), ("Omega", c_p),
                ("jpvt", c_p), ("out0", c_p), ("out1", c_p), ("out2", c_p), ("sigma", c_p),
                ("tol", ctypes.c_double)]


class Result(ctypes.Structure):
    """Mirror of rq_result (include/rqrcp.h)."""
    _fields_ = [("state", ctypes.c_int32), ("status", ctypes.c_int32), ("device_error", c_i64),
                ("queue_ms", ctypes.c_double), ("latency_ms", ctypes.c_double),
                ("flops", ctypes.c_double), ("prec_used", ctypes.c_int32),
                ("reserved", ctypes.c_int32)]


RQ_OP_TRQRCP = 0
RQ_OP_TUXV = 1
RQ_OP_RQRCP = 2
RQ_OP_RSRQRCP = 3
RQ_OP_QRCP = 4
RQ_OP_SKETCH = 5
RQ_OP_SAMPLE_QRCP = 6
RQ_REQ_DONE = 2
RQ_REQ_FAILED = 3

RQ_OK = 0
RQ_E_HIP = 1001
RQ_E_NOMEM = 1002
RQ_E_UNSUPPORTED = 1003
RQ_E_DEVICE = 1004
RQ_FP64 = 0
RQ_MIXED_BF16 = 1
RQ_AUTO = 2

_lib = None


def load():
    """Load librqrcp.so and declare every signature; raises if it is missing."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build()")
        lib = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            fn = getattr(lib, name)
            fn.restype = res
            fn.argtypes = args
        _lib = lib
    return _lib


class RQError(RuntimeError):
    def __init__(self, fn, code, detail=""):
        self.code = code
        super().__init__(f"{fn} returned {code}{(': ' + detail) if detail else ''}")
