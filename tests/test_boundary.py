"""CPU tests of the C-ABI boundary: the built library exports every function
include/vsm.h declares, and the host-only calls (sizes, validation, errors
returned before anything is enqueued) behave as the header states.  No call
here reaches the GPU."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_2203_09764_amd import _lib
from paper_2203_09764_amd._lib import (E_BUDGET, E_DIMS, E_NULL, E_PARAM, E_WORKSPACE, FP32_BULK, FP64,
                                       ANNEALED, JACOBI, MAXRETR, STOUT, Schedule, dims_arg, lib)

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = set()
    inc = os.path.join(ROOT, "include")
    for fn in os.listdir(inc):
        if not fn.endswith(".h"):
            continue
        text = open(os.path.join(inc, fn)).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^[A-Za-z_][\w\s\*]*?\b(vsm_\w+)\s*\(", text, flags=re.M):
            names.add(m.group(1))
    return names


def test_header_declares_the_path_and_server():
    names = _declared()
    for want in ("vsm_precondition", "vsm_smooth", "vsm_measure", "vsm_pass", "vsm_load_z3",
                 "vsm_server_create", "vsm_server_submit", "vsm_server_fetch", "vsm_server_destroy"):
        assert want in names
    assert len(names) >= 24


def test_library_exports_every_declared_symbol():
    L = ctypes.CDLL(_lib.LIB_PATH)
    missing = [n for n in sorted(_declared()) if not hasattr(L, n)]
    assert not missing, missing
    # the binding knows every one of them too
    assert set(_declared()) <= set(_lib.SIGNATURES)


def test_version_and_errors():
    assert b"gfx950" in lib().vsm_version()
    for code in range(0, -9, -1):
        assert lib().vsm_strerror(code) not in (None, b"unknown status")
    assert lib().vsm_strerror(-99) == b"unknown status"


@pytest.mark.parametrize("prec,entry", [(FP64, 16), (FP32_BULK, 8)])
def test_sizes(prec, entry):
    dims = (8, 12, 16, 4)
    V = 8 * 12 * 16 * 4
    # rows 0 and 1 of 4 links per site, each of the 24 entry arrays followed by
    # a gap of 64 entries
    assert lib().vsm_links_bytes(dims_arg(dims), prec) == 24 * (V + 64) * entry
    ann = lib().vsm_workspace_bytes(dims_arg(dims), prec, ANNEALED)
    jac = lib().vsm_workspace_bytes(dims_arg(dims), prec, JACOBI)
    # counters, measurement partials, the charges in the internal layout
    assert 256 + 4 * V < ann < 256 + 80 * (V // 256 + 1) + 4 * V + 512
    assert jac >= ann + 24 * (V + 64) * entry


@pytest.mark.parametrize("dims", [(8, 8, 8, 6), (2, 8, 8, 8), (8, 8, 8, 0), (8, 8, 8, -4)])
def test_bad_extents(dims):
    assert lib().vsm_check_dims(dims_arg(dims), ANNEALED, FP64) == E_DIMS
    assert lib().vsm_links_bytes(dims_arg(dims), FP64) == 0


def test_volume_limit():
    # 6 (V + 64) * 16 bytes must stay below 2^31
    assert lib().vsm_check_dims(dims_arg((64, 64, 64, 92)), ANNEALED, FP64) == E_DIMS
    assert lib().vsm_check_dims(dims_arg((64, 64, 64, 92)), ANNEALED, FP32_BULK) == 0
    assert lib().vsm_check_dims(dims_arg((8, 8, 8, 8)), ANNEALED, 7) == E_PARAM


def _sched(**kw):
    s = Schedule(ANNEALED, STOUT, 1, 3, 1.0, 1.0)
    for k, v in kw.items():
        setattr(s, k, v)
    return s


def test_smooth_rejects_bad_arguments_before_any_launch():
    d = dims_arg((8, 8, 8, 8))
    fake = ctypes.c_void_p(0x1000)  # never dereferenced: validation fails first
    ws = lib().vsm_workspace_bytes(d, FP64, ANNEALED)
    s = _sched()
    f = lib().vsm_smooth
    assert f(d, FP64, None, fake, None, fake, ws, 1, 0.1, 1.0, ctypes.byref(s), 0, None, None) == E_NULL
    assert f(d, FP64, fake, fake, None, fake, ws - 1, 1, 0.1, 1.0, ctypes.byref(s), 0, None, None) == E_WORKSPACE
    assert f(d, FP64, fake, fake, None, fake, ws, -1, 0.1, 1.0, ctypes.byref(s), 0, None, None) == E_PARAM
    assert f(d, FP64, fake, fake, None, fake, ws, 1, float("nan"), 1.0, ctypes.byref(s), 0, None, None) == E_PARAM
    assert f(d, FP64, fake, None, None, fake, ws, 1, 0.1, 1.0, ctypes.byref(s), 0, None, None) == E_NULL  # vp needs z3
    assert f(d, FP64, fake, fake, None, fake, ws, 1, 0.1, 1.0, ctypes.byref(s), 1, None, None) == E_NULL  # stats
    bad = _sched(u0=0.0)
    assert f(d, FP64, fake, fake, None, fake, ws, 1, 0.1, 1.0, ctypes.byref(bad), 0, None, None) == E_PARAM
    bad = _sched(update=5)
    assert f(d, FP64, fake, fake, None, fake, ws, 1, 0.1, 1.0, ctypes.byref(bad), 0, None, None) == E_PARAM
    assert f(dims_arg((8, 8, 8, 6)), FP64, fake, fake, None, fake, ws, 1, 0.1, 1.0, ctypes.byref(s), 0, None,
             None) == E_DIMS


def test_pass_and_precondition_reject_bad_arguments():
    d = dims_arg((8, 8, 8, 8))
    fake = ctypes.c_void_p(0x1000)
    ws = lib().vsm_workspace_bytes(d, FP64, ANNEALED)
    s = _sched()
    assert lib().vsm_pass(d, FP64, fake, fake, None, fake, ws, 4, 0, 0.1, 1.0, ctypes.byref(s), None) == E_PARAM
    assert lib().vsm_pass(d, FP64, fake, fake, None, fake, ws, 0, 4, 0.1, 1.0, ctypes.byref(s), None) == E_PARAM
    # |omega| < 1/4 keeps every link's sector (Sec. IV.A)
    assert lib().vsm_precondition(d, FP64, fake, fake, 0.25, fake, None, None) == E_PARAM
    assert lib().vsm_precondition(d, FP64, fake, fake, -0.3, fake, None, None) == E_PARAM
    assert lib().vsm_precondition(d, FP64, fake, None, 0.02, fake, None, None) == E_NULL


def _job(dims=(8, 8, 8, 8), **kw):
    V = int(np.prod(dims))
    z = np.zeros(4 * V, np.int8)
    p = np.zeros(4 * V, np.int8)
    j = _lib.Job((ctypes.c_int32 * 4)(*dims), FP32_BULK, 10, 0.06, -0.25, 0.02, _sched(), 0, 0,
                 ctypes.c_void_p(z.ctypes.data), ctypes.c_void_p(p.ctypes.data))
    for k, v in kw.items():
        setattr(j, k, v)
    return j, (z, p)


def test_server_job_footprint():
    j, keep = _job()
    V = 8 ** 4
    base = lib().vsm_server_job_bytes(j)
    # links (FP32 rows 0, 1), charges, pairs, workspace, one record
    assert base >= 24 * (V + 64) * 8 + 4 * V + 4 * V + 256
    j.want_links = 1
    assert lib().vsm_server_job_bytes(j) == base + 4 * V * 9 * 16
    j.want_links = 0
    j.precision = FP64
    assert lib().vsm_server_job_bytes(j) == base + 24 * (V + 64) * 8
    host = lib().vsm_server_host_bytes(j)
    assert host >= 8 * V + 64


def test_server_serves_only_annealed_stout():
    j, keep = _job()
    assert lib().vsm_server_job_bytes(j) > 0
    j.sched.update = MAXRETR
    assert lib().vsm_server_job_bytes(j) == 0
    j.sched.update = STOUT
    j.sched.order = JACOBI
    assert lib().vsm_server_job_bytes(j) == 0
    j.sched.order = ANNEALED
    j.omega = 0.25
    assert lib().vsm_server_job_bytes(j) == 0
    j.omega = 0.02
    j.n_sweeps = -1
    assert lib().vsm_server_job_bytes(j) == 0


def test_server_create_validates_config():
    h = ctypes.c_void_p()
    for cfg in [(0, 1 << 20, 4, 4, 0, 0), (1 << 20, 0, 4, 4, 0, 0), (1 << 20, 1 << 20, 0, 4, 0, 0),
                (1 << 20, 1 << 20, 4, 0, 0, 0), (1 << 20, 1 << 20, 4, 4, -1, 0), (1 << 20, 1 << 20, 300, 4, 0, 0)]:
        c = _lib.ServerConfig(*cfg)
        assert lib().vsm_server_create(ctypes.byref(c), ctypes.byref(h)) == E_PARAM
        assert not h.value
    assert lib().vsm_server_create(None, ctypes.byref(h)) == E_NULL
    assert lib().vsm_server_submit(None, None, None) == E_NULL
    assert E_BUDGET < 0


def test_noalloc_checks_before_any_hip_call():
    """vsm_smooth_noalloc validates and refuses a lattice whose workspace exceeds
    its static scratch (VSM_E_WORKSPACE) before touching the GPU."""
    assert lib().vsm_noalloc_scratch_bytes() == 64 << 20
    sched = Schedule(JACOBI, STOUT, 0, 3, 1.0, 1.0)
    p = ctypes.c_void_p(16)
    # smearing needs a second link buffer: 384 MiB in FP64 at 32^4
    rc = lib().vsm_smooth_noalloc(dims_arg((32, 32, 32, 32)), FP64, p, p, None, 1, 0.1, 1.0, ctypes.byref(sched),
                                  0, None, None)
    assert rc == E_WORKSPACE
    ann = Schedule(ANNEALED, STOUT, 1, 3, 1.0, 1.0)
    # annealed: 4V charge bytes and the reduction slots; 48^3 x 200 (22M sites) is too large in FP32
    rc = lib().vsm_smooth_noalloc(dims_arg((48, 48, 48, 200)), FP32_BULK, p, p, None, 1, 0.1, 1.0,
                                  ctypes.byref(ann), 1, p, None)
    assert rc == E_WORKSPACE
    assert lib().vsm_smooth_noalloc(dims_arg((8, 8, 6, 8)), FP64, p, p, None, 1, 0.1, 1.0, ctypes.byref(ann), 0,
                                    None, None) == E_DIMS
    assert lib().vsm_smooth_noalloc(dims_arg((8, 8, 8, 8)), FP64, p, p, None, 1, 0.1, 1.0, None, 0, None,
                                    None) == E_NULL

