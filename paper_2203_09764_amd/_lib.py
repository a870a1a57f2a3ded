"""ctypes loader of libvsm.so (the HIP library) and its C signatures.

Loading fails loudly when the library has not been built: there is no other
implementation of the path behind this package.
"""
from __future__ import annotations

import ctypes
import os

import numpy as np

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libvsm.so")

OK = 0
E_DIMS, E_PARAM, E_NULL, E_WORKSPACE, E_BUDGET, E_HIP, E_STATE = -1, -2, -3, -4, -5, -6, -7
FP64, FP32_BULK = 0, 1
JACOBI, ANNEALED = 0, 1
STOUT, MAXRETR = 0, 1
UNDEF = -128

STATS_DTYPE = np.dtype([
    ("plaq", "<f8"), ("action", "<f8"), ("max_unitarity", "<f8"), ("sweep", "<f8"),
    ("flux_mismatch", "<i8"), ("undefined_sector", "<i8"), ("rejected", "<i8"),
    ("nonfinite", "<i8"),
])
STATS_BYTES = STATS_DTYPE.itemsize


class Schedule(ctypes.Structure):
    _fields_ = [("order", ctypes.c_int32), ("update", ctypes.c_int32), ("vp", ctypes.c_int32),
                ("su2_loops", ctypes.c_int32), ("u0", ctypes.c_double), ("alpha", ctypes.c_double)]


class VsmError(RuntimeError):
    def __init__(self, status: int, what: str):
        self.status = status
        msg = lib().vsm_strerror(status).decode()
        if status == E_HIP:
            msg += f" (hipError {lib().vsm_last_hip_error()})"
        super().__init__(f"{what}: {msg} [{status}]")


Dims = ctypes.c_int32 * 4
_P = ctypes.c_void_p
_i32, _i64, _u64, _f64, _sz = ctypes.c_int32, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_size_t

SIGNATURES = {
    "vsm_version": (ctypes.c_char_p, []),
    "vsm_strerror": (ctypes.c_char_p, [ctypes.c_int]),
    "vsm_last_hip_error": (ctypes.c_int, []),
    "vsm_check_dims": (ctypes.c_int, [Dims, _i32, _i32]),
    "vsm_links_bytes": (_sz, [Dims, _i32]),
    "vsm_workspace_bytes": (_sz, [Dims, _i32, _i32]),
    "vsm_set_links": (ctypes.c_int, [Dims, _i32, _P, _P, _P]),
    "vsm_get_links": (ctypes.c_int, [Dims, _i32, _P, _P, _P]),
    "vsm_load_z3": (ctypes.c_int, [Dims, _i32, _P, _P, _P]),
    "vsm_precondition": (ctypes.c_int, [Dims, _i32, _P, _P, _f64, _P, _P, _P]),
    "vsm_gauge_transform": (ctypes.c_int, [Dims, _i32, _P, _P, _P]),
    "vsm_smooth": (ctypes.c_int, [Dims, _i32, _P, _P, _P, _P, _sz, _i32, _f64, _f64,
                                  ctypes.POINTER(Schedule), _i32, _P, _P]),
    "vsm_pass": (ctypes.c_int, [Dims, _i32, _P, _P, _P, _P, _sz, _i32, _i32, _f64, _f64,
                                ctypes.POINTER(Schedule), _P]),
    "vsm_measure": (ctypes.c_int, [Dims, _i32, _P, _P, _P, _sz, _P, _P, _P]),
}

_lib = None


def lib():
    """The loaded library; raises if libvsm.so has not been built."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError(f"{LIB_PATH} is missing: build it with __graft_entry__.build() "
                               "(hipcc, gfx950) before using paper_2203_09764_amd")
        L = ctypes.CDLL(LIB_PATH)
        for name, (res, args) in SIGNATURES.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        for name, (res, args) in EXTRA_SIGNATURES.items():
            if hasattr(L, name):
                f = getattr(L, name)
                f.restype = res
                f.argtypes = args
        _lib = L
    return _lib


EXTRA_SIGNATURES: dict = {}


def dims_arg(dims) -> Dims:
    d = [int(v) for v in dims]
    if len(d) != 4:
        raise ValueError("dims must have four entries")
    return Dims(*d)


def check(status: int, what: str) -> None:
    if status != OK:
        raise VsmError(status, what)
