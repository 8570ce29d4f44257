"""ctypes view of libexsum.so (the C ABI declared in include/exsum.h).

Only argument marshalling lives here.  The shared library must have been built
(``python -m paper_2106_00124_amd.build`` or ``__graft_entry__.build()``);
there is no fallback: a missing library raises at first use.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("EXSUM_LIB", os.path.join(HERE, "libexsum.so"))

MAX_RANK = 8
F32, F64, I32, I64, VALIDX = 0, 1, 2, 3, 4
SUM, MAX, MIN = 0, 1, 2
INCLUDED, EXCLUDED, WEAK = 1, 2, 4
OK, EINVAL, EUNSUPPORTED, ENOMEM, EDEVICE, EAGAIN, ENOTREADY, ENOTFOUND = range(8)

STATUS = {0: "EXS_OK", 1: "EXS_EINVAL", 2: "EXS_EUNSUPPORTED", 3: "EXS_ENOMEM",
          4: "EXS_EDEVICE", 5: "EXS_EAGAIN", 6: "EXS_ENOTREADY", 7: "EXS_ENOTFOUND"}


class ExsJob(ctypes.Structure):
    _fields_ = [
        ("d", ctypes.c_int32),
        ("dtype", ctypes.c_int32),
        ("op", ctypes.c_int32),
        ("mode", ctypes.c_uint32),
        ("dims", ctypes.c_int64 * MAX_RANK),
        ("box", ctypes.c_int64 * MAX_RANK),
        ("in_dev", ctypes.c_void_p),
        ("inc_out_dev", ctypes.c_void_p),
        ("exc_out_dev", ctypes.c_void_p),
    ]


class ExsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS.get(status, status)}: {msg}")
        self.status = status


# every symbol include/exsum.h declares, with its ctypes signature
_P = ctypes.c_void_p
_JP = ctypes.POINTER(ExsJob)
SIGNATURES = {
    "exs_workspace_size": (ctypes.c_int, [_JP, ctypes.POINTER(ctypes.c_size_t)]),
    "exs_run": (ctypes.c_int, [_JP, _P, ctypes.c_size_t, _P]),
    "exs_run_noalloc": (ctypes.c_int, [_JP, _P]),
    "exs_corners_workspace_size": (ctypes.c_int, [_JP, ctypes.POINTER(ctypes.c_size_t)]),
    "exs_run_corners": (ctypes.c_int, [_JP, _P, ctypes.c_size_t, _P]),
    "exs_status_str": (ctypes.c_char_p, [ctypes.c_int]),
    "exs_last_error": (ctypes.c_char_p, []),
    "exs_version": (ctypes.c_char_p, []),
    "exs_fill": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                ctypes.c_uint64, ctypes.c_int64, ctypes.c_int64, _P]),
    "exs_set_op_cost": (ctypes.c_int, [ctypes.c_int32]),
    "exs_op_probe": (ctypes.c_int, [_P, ctypes.c_int64, ctypes.c_int32, _P]),
    "exs_timing_enable": (ctypes.c_int, [ctypes.c_int32]),
    "exs_timing_read": (ctypes.c_int, [ctypes.c_int32, ctypes.c_char_p,
                                       ctypes.POINTER(ctypes.c_int64),
                                       ctypes.POINTER(ctypes.c_double),
                                       ctypes.POINTER(ctypes.c_int32)]),
    "exs_batch_create": (ctypes.c_int, [_JP, ctypes.c_int32, ctypes.c_char_p,
                                        ctypes.POINTER(_P)]),
    "exs_batch_workspace_size": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_size_t)]),
    "exs_batch_launch": (ctypes.c_int, [_P, _P, ctypes.c_size_t, _P]),
    "exs_batch_launch_eager": (ctypes.c_int, [_P, _P, ctypes.c_size_t, _P]),
    "exs_batch_info": (ctypes.c_int, [_P, ctypes.POINTER(ctypes.c_int32),
                                      ctypes.POINTER(ctypes.c_int64)]),
    "exs_batch_destroy": (None, [_P]),
    "exs_server_create": (ctypes.c_int, [ctypes.c_size_t, ctypes.c_int32, ctypes.POINTER(_P)]),
    "exs_server_submit": (ctypes.c_int, [_P, _JP, _P, ctypes.POINTER(ctypes.c_uint64)]),
    "exs_server_submit_generated": (ctypes.c_int, [_P, _JP, ctypes.c_int32, ctypes.c_uint64,
                                                   ctypes.c_int64, ctypes.c_int64,
                                                   ctypes.POINTER(ctypes.c_uint64)]),
    "exs_server_input": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.POINTER(_P)]),
    "exs_server_poll": (ctypes.c_int, [_P, ctypes.c_uint64, ctypes.POINTER(_P),
                                       ctypes.POINTER(_P), ctypes.POINTER(ctypes.c_double)]),
    "exs_server_drain": (ctypes.c_int, [_P]),
    "exs_server_release": (ctypes.c_int, [_P, ctypes.c_uint64, _P]),
    "exs_server_stats": (ctypes.c_int, [_P] + [ctypes.POINTER(ctypes.c_double)] * 4
                         + [ctypes.POINTER(ctypes.c_int64)] * 3),
    "exs_server_destroy": (None, [_P]),
}

_lib = None


def lib():
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"libexsum.so not found at {LIB_PATH}; build it with "
                              "`python -m paper_2106_00124_amd.build`")
        h = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(h, name)
            f.restype = res
            f.argtypes = args
        _lib = h
    return _lib


def check(status: int):
    if status != 0:
        raise ExsError(status, lib().exs_last_error().decode(errors="replace"))


def make_job(d, dtype, op, mode, dims, box, in_ptr, inc_ptr, exc_ptr) -> ExsJob:
    j = ExsJob()
    j.d = d
    j.dtype = dtype
    j.op = op
    j.mode = mode
    for i in range(d):
        j.dims[i] = int(dims[i])
        j.box[i] = int(box[i])
    j.in_dev = in_ptr
    j.inc_out_dev = inc_ptr
    j.exc_out_dev = exc_ptr
    return j
