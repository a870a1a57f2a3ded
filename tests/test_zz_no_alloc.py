"""GPU test of vsm_smooth_noalloc, the entry point that allocates nothing (collected
last, so that a failure here hides no other test): it runs
vsm_smooth's kernels on the library's static per-device scratch array instead of
a caller workspace.  Two calls in a row (the second on a smaller lattice, in the
other precision and order) must give links and records bit-identical to
vsm_smooth on the same inputs: the scratch keeps the previous call's contents,
so this also checks that each call re-initialises what it reads."""
import ctypes

import numpy as np
import pytest
import torch

import fieldgen
from paper_2203_09764_amd import api
from paper_2203_09764_amd._lib import E_WORKSPACE, dims_arg, lib

pytestmark = pytest.mark.gpu

CASES = [
    # dims, precision, order, n_sweeps, rho, eps, vp, measure_every, seed
    ((16, 16, 16, 32), "fp64", "annealed", 3, 0.06, -0.25, True, 1, 81),
    ((8, 8, 8, 8), "fp32_bulk", "jacobi", 2, 0.1, 1.0, False, 1, 82),
]


def _field(dims, precision, order, seed):
    n = fieldgen.z3_vortex_charges(dims, 0.1, seed)
    f = api.Field(dims, precision, device=torch.device("cuda:0"), jacobi_workspace=(order == "jacobi"))
    f.set_charges(n)
    api.precondition(f, fieldgen.centrifuge_pairs(dims, seed + 1), 0.02)
    return f


def _noalloc(f, n_sweeps, rho, eps, sched, measure_every, stats):
    stream = ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)
    return lib().vsm_smooth_noalloc(dims_arg(f.dims), f.precision, ctypes.c_void_p(f.links.data_ptr()),
                                    ctypes.c_void_p(f.z3.data_ptr()), None, int(n_sweeps), float(rho), float(eps),
                                    ctypes.byref(sched), int(measure_every), ctypes.c_void_p(stats.data_ptr()),
                                    stream)


def test_noalloc_equals_smooth_on_two_calls_in_a_row():
    assert lib().vsm_noalloc_scratch_bytes() == 64 << 20
    for dims, prec, order, ns, rho, eps, vp, me, seed in CASES:
        print(f"no-alloc case {dims} {prec} {order} {ns} sweeps", flush=True)
        ref = _field(dims, prec, order, seed)
        st_ref = api.smooth(ref, ns, rho, eps, order=order, vp=vp, measure_every=me)
        got = _field(dims, prec, order, seed)
        st_got = api.new_stats(ns // me, got.device)
        st_got.fill_(0xAB)
        sched = api.schedule(order, "stout", vp)
        rc = _noalloc(got, ns, rho, eps, sched, me, st_got)
        assert rc == 0, rc
        torch.cuda.synchronize()
        assert torch.equal(api.get_links(got), api.get_links(ref))
        a = api.stats_to_numpy(st_got, ns // me)
        b = api.stats_to_numpy(st_ref, ns // me)
        assert a.tobytes() == b.tobytes()
        assert np.all(a.flux_mismatch == 0) if vp else True
        if vp:
            assert a.rejected.sum() == b.rejected.sum()


def test_noalloc_refuses_a_lattice_beyond_the_scratch():
    sched = api.schedule("jacobi", "stout", False)
    dims = (32, 32, 32, 32)  # the smearing buffer alone is 384 MiB in FP64
    x = torch.empty(16, dtype=torch.uint8, device="cuda:0")
    p = ctypes.c_void_p(x.data_ptr())
    rc = lib().vsm_smooth_noalloc(dims_arg(dims), 0, p, p, None, 1, 0.1, 1.0, ctypes.byref(sched), 0, None, None)
    assert rc == E_WORKSPACE
