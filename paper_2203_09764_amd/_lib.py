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
E_DIMS, E_PARAM, E_NULL, E_WORKSPACE, E_BUDGET, E_HIP, E_STATE, E_TIMEOUT = -1, -2, -3, -4, -5, -6, -7, -8
JOB_QUEUED, JOB_RUNNING, JOB_DONE, JOB_FAILED = 0, 1, 2, 3
FP64, FP32_BULK = 0, 1
JACOBI, ANNEALED = 0, 1
STOUT, MAXRETR, APE = 0, 1, 2
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


class ServerConfig(ctypes.Structure):
    _fields_ = [("hbm_budget_bytes", ctypes.c_size_t), ("host_budget_bytes", ctypes.c_size_t),
                ("max_slots", ctypes.c_int32), ("max_inflight", ctypes.c_int32),
                ("device", ctypes.c_int32), ("reserved", ctypes.c_int32)]


class Job(ctypes.Structure):
    _fields_ = [("dims", ctypes.c_int32 * 4), ("precision", ctypes.c_int32), ("n_sweeps", ctypes.c_int32),
                ("rho", ctypes.c_double), ("eps", ctypes.c_double), ("omega", ctypes.c_double),
                ("sched", Schedule), ("measure_every", ctypes.c_int32), ("want_links", ctypes.c_int32),
                ("z3_host", ctypes.c_void_p), ("pair_host", ctypes.c_void_p)]


class JobInfo(ctypes.Structure):
    _fields_ = [("state", ctypes.c_int32), ("status", ctypes.c_int32), ("n_records", ctypes.c_int32),
                ("sweeps_done", ctypes.c_int32), ("t_submit", ctypes.c_double), ("t_admit", ctypes.c_double),
                ("t_done", ctypes.c_double), ("footprint_bytes", ctypes.c_size_t)]


class ServerCounters(ctypes.Structure):
    _fields_ = [("steps", ctypes.c_int64), ("launches", ctypes.c_int64), ("jobs_submitted", ctypes.c_int64),
                ("jobs_done", ctypes.c_int64), ("jobs_failed", ctypes.c_int64),
                ("link_updates", ctypes.c_int64), ("peak_resident_jobs", ctypes.c_int64),
                ("peak_pool_bytes", ctypes.c_size_t), ("busy_seconds", ctypes.c_double)]


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
    "vsm_measure": (ctypes.c_int, [Dims, _i32, _P, _P, _P, _P, _sz, _P, _P, _P]),
    "vsm_noalloc_scratch_bytes": (_sz, []),
    "vsm_smooth_noalloc": (ctypes.c_int, [Dims, _i32, _P, _P, _P, _i32, _f64, _f64, ctypes.POINTER(Schedule),
                                          _i32, _P, _P]),
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
        _lib = L
    return _lib


SIGNATURES.update({
    "vsm_flow_workspace_bytes": (_sz, [Dims, _i32, _i32]),
    "vsm_flow": (ctypes.c_int, [Dims, _i32, _P, _P, _sz, _i32, _f64, _f64, _f64, _i32, _P]),
    "vsm_measure_clover": (ctypes.c_int, [Dims, _i32, _P, _P, _sz, _P, _P, _P, _P]),
    "vsm_correlate": (ctypes.c_int, [_i64, _P, _P, _P, _P]),
    "vsm_server_job_bytes": (_sz, [ctypes.POINTER(Job)]),
    "vsm_server_host_bytes": (_sz, [ctypes.POINTER(Job)]),
    "vsm_server_create": (ctypes.c_int, [ctypes.POINTER(ServerConfig), ctypes.POINTER(ctypes.c_void_p)]),
    "vsm_server_submit": (ctypes.c_int, [_P, ctypes.POINTER(Job), ctypes.POINTER(_u64)]),
    "vsm_server_poll": (ctypes.c_int, [_P, _u64, ctypes.POINTER(JobInfo)]),
    "vsm_server_wait": (ctypes.c_int, [_P, _u64, _f64, ctypes.POINTER(JobInfo)]),
    "vsm_server_fetch": (ctypes.c_int, [_P, _u64, _P, _i32, _P]),
    "vsm_server_clock": (_f64, [_P]),
    "vsm_server_get_counters": (ctypes.c_int, [_P, ctypes.POINTER(ServerCounters)]),
    "vsm_server_destroy": (ctypes.c_int, [_P]),
})


def dims_arg(dims) -> Dims:
    d = [int(v) for v in dims]
    if len(d) != 4:
        raise ValueError("dims must have four entries")
    return Dims(*d)


def check(status: int, what: str) -> None:
    if status != OK:
        raise VsmError(status, what)
