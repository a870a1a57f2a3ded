"""Python binding of the C ABI in include/vsm.h: argument marshalling only.

PyTorch supplies device memory (tensors on the current HIP device) and the
stream (torch.cuda.current_stream()).  Every computation happens in the HIP
kernels of libvsm.so; nothing here touches the link values.
"""
from __future__ import annotations

import ctypes

import numpy as np
import torch

from . import _lib
from ._lib import (ANNEALED, APE, FP32_BULK, FP64, JACOBI, MAXRETR, STATS_BYTES, STATS_DTYPE, STOUT,
                   Schedule, check, dims_arg, lib)

PRECISIONS = {"fp64": FP64, "fp32_bulk": FP32_BULK, "fp32": FP32_BULK, FP64: FP64, FP32_BULK: FP32_BULK}
ORDERS = {"jacobi": JACOBI, "annealed": ANNEALED, JACOBI: JACOBI, ANNEALED: ANNEALED}
UPDATES = {"stout": STOUT, "maxretr": MAXRETR, "cooling": MAXRETR, "ape": APE, STOUT: STOUT, MAXRETR: MAXRETR,
           APE: APE}


def _ptr(t):
    if t is None:
        return None
    if not t.is_cuda:
        raise ValueError("expected a device tensor")
    if not t.is_contiguous():
        raise ValueError("expected a contiguous tensor")
    return ctypes.c_void_p(t.data_ptr())


def _stream(stream=None):
    s = stream if stream is not None else torch.cuda.current_stream()
    return ctypes.c_void_p(s.cuda_stream)


def version() -> str:
    return lib().vsm_version().decode()


def check_dims(dims, order="annealed", precision="fp64") -> int:
    return lib().vsm_check_dims(dims_arg(dims), ORDERS[order], PRECISIONS[precision])


def links_bytes(dims, precision="fp64") -> int:
    return int(lib().vsm_links_bytes(dims_arg(dims), PRECISIONS[precision]))


def workspace_bytes(dims, precision="fp64", order="annealed") -> int:
    return int(lib().vsm_workspace_bytes(dims_arg(dims), PRECISIONS[precision], ORDERS[order]))


class Field:
    """Device buffers of one lattice: the links in the library's internal layout,
    the original Z(3) charges and a workspace large enough for both schedules."""

    def __init__(self, dims, precision="fp64", device=None, jacobi_workspace=True):
        self.dims = tuple(int(v) for v in dims)
        self.precision = PRECISIONS[precision]
        self.device = torch.device(device) if device is not None else torch.device("cuda")
        rc = lib().vsm_check_dims(dims_arg(self.dims), JACOBI, self.precision)
        check(rc, f"dims {self.dims}")
        self.V = self.dims[0] * self.dims[1] * self.dims[2] * self.dims[3]
        nb = links_bytes(self.dims, self.precision)
        self.links = torch.empty(nb, dtype=torch.uint8, device=self.device)
        order = JACOBI if jacobi_workspace else ANNEALED
        ws = int(lib().vsm_workspace_bytes(dims_arg(self.dims), self.precision, order))
        if ws == 0:
            ws = int(lib().vsm_workspace_bytes(dims_arg(self.dims), self.precision, ANNEALED))
        self.workspace = torch.empty(ws, dtype=torch.uint8, device=self.device)
        self.z3 = None

    def set_charges(self, z3):
        z = torch.as_tensor(z3, dtype=torch.int8)
        if tuple(z.shape) != (4, self.V):
            raise ValueError(f"charges must have shape (4, {self.V})")
        self.z3 = z.to(self.device).contiguous()
        return self.z3


def load_z3(field: Field, z3=None, stream=None):
    """Sec. I: links = e^{2 pi i n/3} 1 from the charges (kept as the original charges)."""
    if z3 is not None:
        field.set_charges(z3)
    check(lib().vsm_load_z3(dims_arg(field.dims), field.precision, _ptr(field.z3), _ptr(field.links),
                            _stream(stream)), "vsm_load_z3")


def precondition(field: Field, pairs, omega, z3=None, want_m=False, stream=None):
    """Sec. IV: centrifuge preconditioning; pairs = int8 [4][V] in {0,1,2}."""
    if z3 is not None:
        field.set_charges(z3)
    p = torch.as_tensor(pairs, dtype=torch.int8).to(field.device).contiguous()
    m = torch.empty((4, field.V), dtype=torch.int32, device=field.device) if want_m else None
    check(lib().vsm_precondition(dims_arg(field.dims), field.precision, _ptr(field.z3), _ptr(p),
                                 float(omega), _ptr(field.links), _ptr(m), _stream(stream)),
          "vsm_precondition")
    return m


def gauge_transform(field: Field, gauge, stream=None):
    """Sec. V.C: U_mu(x) -> G(x) U_mu(x) G^dag(x+mu); gauge complex128 [V,3,3] on the device."""
    G = torch.as_tensor(gauge).to(device=field.device, dtype=torch.complex128).contiguous()
    check(lib().vsm_gauge_transform(dims_arg(field.dims), field.precision, _ptr(field.links),
                                    _ptr(G), _stream(stream)), "vsm_gauge_transform")
    return G


def schedule(order="annealed", update="stout", vp=False, u0=1.0, alpha=1.0, su2_loops=3) -> Schedule:
    return Schedule(ORDERS[order], UPDATES[update], int(bool(vp)), int(su2_loops), float(u0),
                    float(alpha))


def new_stats(n: int, device) -> torch.Tensor:
    return torch.zeros((max(n, 1), STATS_BYTES), dtype=torch.uint8, device=device)


def stats_to_numpy(t: torch.Tensor, n: int | None = None) -> np.recarray:
    a = t.detach().cpu().numpy().view(STATS_DTYPE).reshape(-1)
    if n is not None:
        a = a[:n]
    return a.view(np.recarray)


def _check_stats(stats, nrec, device):
    """The library writes nrec records of STATS_BYTES into stats without a bound:
    refuse a tensor that cannot hold them."""
    if (not isinstance(stats, torch.Tensor) or stats.dtype != torch.uint8 or stats.device != torch.device(device)
            or not stats.is_contiguous() or stats.numel() < nrec * STATS_BYTES):
        raise ValueError(f"stats must be a contiguous uint8 tensor on {device} with at least "
                         f"{nrec * STATS_BYTES} bytes ({nrec} records)")


def smooth(field: Field, n_sweeps, rho, eps, *, order="annealed", update="stout", vp=False,
           u0=1.0, alpha=1.0, su2_loops=3, gauge=None, measure_every=0, stats=None, stream=None):
    """n_sweeps sweeps (include/vsm.h, vsm_smooth).  Returns the device stats
    tensor (n_sweeps // measure_every records) when measuring, else None."""
    sch = schedule(order, update, vp, u0, alpha, su2_loops)
    nrec = n_sweeps // measure_every if measure_every > 0 else 0
    if measure_every > 0 and stats is None:
        stats = new_stats(nrec, field.device)
    if measure_every > 0:
        _check_stats(stats, nrec, field.device)
    G = None
    if gauge is not None:
        G = torch.as_tensor(gauge).to(device=field.device, dtype=torch.complex128).contiguous()
    check(lib().vsm_smooth(dims_arg(field.dims), field.precision, _ptr(field.links), _ptr(field.z3),
                           _ptr(G), _ptr(field.workspace), field.workspace.numel(), int(n_sweeps),
                           float(rho), float(eps), ctypes.byref(sch), int(measure_every),
                           _ptr(stats) if measure_every > 0 else None, _stream(stream)),
          "vsm_smooth")
    return stats


def anneal_pass(field: Field, mu, colour, rho, eps, *, update="stout", vp=False, u0=1.0,
                alpha=1.0, su2_loops=3, gauge=None, stream=None):
    """One masked annealing subset (vsm_pass)."""
    sch = schedule("annealed", update, vp, u0, alpha, su2_loops)
    G = None
    if gauge is not None:
        G = torch.as_tensor(gauge).to(device=field.device, dtype=torch.complex128).contiguous()
    check(lib().vsm_pass(dims_arg(field.dims), field.precision, _ptr(field.links), _ptr(field.z3),
                         _ptr(G), _ptr(field.workspace), field.workspace.numel(), int(mu),
                         int(colour), float(rho), float(eps), ctypes.byref(sch), _stream(stream)),
          "vsm_pass")


def measure(field: Field, with_flux=False, gauge=None, stream=None):
    """Sec. I, V.A: one stats record (device tensor) and optionally the flux int8 [6][V];
    with a gauge (complex128 [V,3,3]) the link sectors are taken after undoing it."""
    st = new_stats(1, field.device)
    flux = torch.empty((6, field.V), dtype=torch.int8, device=field.device) if with_flux else None
    G = None
    if gauge is not None:
        G = torch.as_tensor(gauge).to(device=field.device, dtype=torch.complex128).contiguous()
    check(lib().vsm_measure(dims_arg(field.dims), field.precision, _ptr(field.links), _ptr(field.z3), _ptr(G),
                            _ptr(field.workspace), field.workspace.numel(), _ptr(st), _ptr(flux),
                            _stream(stream)), "vsm_measure")
    return (st, flux) if with_flux else st


def get_links(field: Field, stream=None) -> torch.Tensor:
    """Links in the canonical layout: complex128 [4, V, 3, 3] on the device."""
    out = torch.empty((4, field.V, 3, 3), dtype=torch.complex128, device=field.device)
    check(lib().vsm_get_links(dims_arg(field.dims), field.precision, _ptr(field.links), _ptr(out),
                              _stream(stream)), "vsm_get_links")
    return out


def set_links(field: Field, canon, stream=None):
    """Load links from the canonical layout (complex128 [4, V, 3, 3])."""
    c = torch.as_tensor(canon).to(device=field.device, dtype=torch.complex128).contiguous()
    if tuple(c.shape) != (4, field.V, 3, 3):
        raise ValueError(f"links must have shape (4, {field.V}, 3, 3)")
    check(lib().vsm_set_links(dims_arg(field.dims), field.precision, _ptr(c), _ptr(field.links),
                              _stream(stream)), "vsm_set_links")


def measure_clover(field: Field, densities=False, stream=None):
    """Sec. V / V.A: device float64 tensor {<S_R>/beta, Q, <S>/beta, 0}; with
    densities also S(x)/beta and q(x) as device float64 [V] (canonical order)."""
    out = torch.zeros(4, dtype=torch.float64, device=field.device)
    sd = torch.empty(field.V, dtype=torch.float64, device=field.device) if densities else None
    qd = torch.empty(field.V, dtype=torch.float64, device=field.device) if densities else None
    check(lib().vsm_measure_clover(dims_arg(field.dims), field.precision, _ptr(field.links), _ptr(field.workspace),
                                   field.workspace.numel(), _ptr(out), _ptr(sd), _ptr(qd), _stream(stream)),
          "vsm_measure_clover")
    return (out, sd, qd) if densities else out


def correlate(a: torch.Tensor, b: torch.Tensor, stream=None) -> torch.Tensor:
    """Sec. VII: device float64 {<ab>/sqrt(<a^2><b^2>), sum ab, sum a^2, sum b^2}."""
    if a.dtype != torch.float64 or b.dtype != torch.float64 or a.numel() != b.numel():
        raise ValueError("expected two float64 device tensors of the same size")
    out = torch.zeros(4, dtype=torch.float64, device=a.device)
    check(lib().vsm_correlate(a.numel(), _ptr(a.contiguous()), _ptr(b.contiguous()), _ptr(out), _stream(stream)),
          "vsm_correlate")
    return out


def flow(field: Field, n_steps, eps, *, eps_oi=1.0, u0=1.0, integrator="rk3", stream=None):
    """Sec. II.B / V.B: n_steps Wilson-flow steps of size eps, every link at once
    (vsm_flow); integrator "euler" or "rk3".  Allocates its workspace."""
    it = {"euler": 0, "rk3": 1}[integrator]
    nb = int(lib().vsm_flow_workspace_bytes(dims_arg(field.dims), field.precision, it))
    ws = torch.empty(nb, dtype=torch.uint8, device=field.device)
    check(lib().vsm_flow(dims_arg(field.dims), field.precision, _ptr(field.links), _ptr(ws), nb, int(n_steps),
                         float(eps), float(eps_oi), float(u0), it, _stream(stream)), "vsm_flow")
