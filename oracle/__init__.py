"""ctypes binding of the FP64 CPU oracle (oracle.c).

TEST INFRASTRUCTURE: only the test-suite, the smoke check and the CPU-baseline
leg of the benchmark import this package.  The product library never loads it.

Arrays use the canonical interchange layout: links complex128 [4][V][3][3],
charges int8 [4][V], pair choices int8 [4][V], gauge complex128 [V][3][3],
flux int8 [6][V] with planes (01, 02, 03, 12, 13, 23).
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.environ.get("ORACLE_LIB_OVERRIDE") or os.path.join(_HERE, "liboracle.so")
SRC_PATH = os.path.join(_HERE, "oracle.c")

OK, E_DIMS, E_PARAM, E_NULL = 0, -1, -2, -3
UNDEF = -128
JACOBI, ANNEALED = 0, 1
STOUT, MAXRETR, APE = 0, 1, 2

STATS_DTYPE = np.dtype([
    ("plaq", "<f8"), ("action", "<f8"), ("max_unitarity", "<f8"), ("reserved", "<f8"),
    ("flux_mismatch", "<i8"), ("undefined_sector", "<i8"), ("rejected", "<i8"),
    ("nonfinite", "<i8"),
])


def build(force: bool = True) -> str:
    """Compile oracle.c into liboracle.so with gcc (FP64, IEEE, OpenMP)."""
    if force or not os.path.exists(LIB_PATH):
        # written beside the library and renamed over it, so that a process that
        # has the old one loaded keeps a valid mapping
        tmp = LIB_PATH + ".tmp"
        cmd = ["gcc", "-O2", "-fPIC", "-shared", "-fopenmp", "-std=c11", "-Wall",
               SRC_PATH, "-o", tmp, "-lm"]
        subprocess.run(cmd, check=True)
        os.replace(tmp, LIB_PATH)
    return LIB_PATH


_lib = None


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            build()
        L = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        i32, i64, f64 = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        sig = {
            "ora_set_threads": (ctypes.c_int, [ctypes.c_int]),
            "ora_sector": (ctypes.c_int, [f64, f64]),
            "ora_colour": (ctypes.c_int, [P, i32, i64]),
            "ora_z3_field": (ctypes.c_int, [P, P, P]),
            "ora_centrifuge": (ctypes.c_int, [P, P, P, f64, P, P]),
            "ora_gauge_transform": (ctypes.c_int, [P, P, P, P]),
            "ora_staple": (ctypes.c_int, [P, P, i32, i64, f64, f64, P]),
            "ora_generator": (None, [P, P]),
            "ora_expm": (None, [P, P]),
            "ora_maxretr": (None, [P, P, i32, P]),
            "ora_unit_circle_projection": (None, [P, P]),
            "ora_update_link": (ctypes.c_int, [P, P, P, P, i32, i32, f64, f64, f64, f64, i32,
                                               i32, i64, P, P]),
            "ora_update_links": (ctypes.c_int, [P, P, P, P, i32, i32, f64, f64, f64, f64, i32,
                                                i64, P, P, P, P]),
            "ora_clover": (ctypes.c_int, [P, P, P, P, P]),
            "ora_flow": (ctypes.c_int, [P, P, i32, f64, f64, f64, i32]),
            "ora_correlation": (ctypes.c_double, [i64, P, P]),
            "ora_pass": (ctypes.c_int, [P, P, P, P, i32, i32, f64, f64, f64, f64, i32, i32,
                                        i32, P]),
            "ora_smooth": (ctypes.c_int, [P, P, P, P, i32, i32, i32, i32, f64, f64, f64, f64,
                                          i32, i32, P]),
            "ora_measure": (ctypes.c_int, [P, P, P, P, P, P]),
            "ora_sectors": (ctypes.c_int, [P, P, P]),
        }
        for name, (res, args) in sig.items():
            f = getattr(L, name)
            f.restype = res
            f.argtypes = args
        _lib = L
    return _lib


def _p(a):
    return None if a is None else a.ctypes.data_as(ctypes.c_void_p)


def _dims(dims):
    return np.ascontiguousarray(np.asarray(dims, dtype=np.int32))


def _check(rc, what):
    if rc != OK:
        raise ValueError(f"oracle {what} failed with status {rc}")


def _vol(dims):
    d = [int(v) for v in dims]
    return d[0] * d[1] * d[2] * d[3]


def set_threads(n: int) -> int:
    return lib().ora_set_threads(int(n))


def sector(t: complex) -> int:
    return lib().ora_sector(float(t.real), float(t.imag))


def colour(dims, mu, site) -> int:
    return lib().ora_colour(_p(_dims(dims)), int(mu), int(site))


def z3_field(dims, n) -> np.ndarray:
    V = _vol(dims)
    n = np.ascontiguousarray(n, dtype=np.int8)
    out = np.empty((4, V, 3, 3), dtype=np.complex128)
    _check(lib().ora_z3_field(_p(_dims(dims)), _p(n), _p(out)), "z3_field")
    return out


def centrifuge(dims, n, pair, omega, return_m=False):
    V = _vol(dims)
    n = np.ascontiguousarray(n, dtype=np.int8)
    pair = np.ascontiguousarray(pair, dtype=np.int8)
    out = np.empty((4, V, 3, 3), dtype=np.complex128)
    m = np.empty((4, V), dtype=np.int32)
    _check(lib().ora_centrifuge(_p(_dims(dims)), _p(n), _p(pair), float(omega), _p(out), _p(m)),
           "centrifuge")
    return (out, m) if return_m else out


def gauge_transform(dims, links, gauge) -> np.ndarray:
    links = np.ascontiguousarray(links, dtype=np.complex128)
    gauge = np.ascontiguousarray(gauge, dtype=np.complex128)
    out = np.empty_like(links)
    _check(lib().ora_gauge_transform(_p(_dims(dims)), _p(links), _p(gauge), _p(out)),
           "gauge_transform")
    return out


def staple(dims, links, mu, site, eps=1.0, u0=1.0) -> np.ndarray:
    links = np.ascontiguousarray(links, dtype=np.complex128)
    out = np.empty((3, 3), dtype=np.complex128)
    _check(lib().ora_staple(_p(_dims(dims)), _p(links), int(mu), int(site), float(eps), float(u0),
                            _p(out)), "staple")
    return out


def generator(omega) -> np.ndarray:
    om = np.ascontiguousarray(omega, dtype=np.complex128)
    out = np.empty((3, 3), dtype=np.complex128)
    lib().ora_generator(_p(om), _p(out))
    return out


def expm(x) -> np.ndarray:
    xm = np.ascontiguousarray(x, dtype=np.complex128)
    out = np.empty((3, 3), dtype=np.complex128)
    lib().ora_expm(_p(xm), _p(out))
    return out


def maxretr(u, v, loops=3) -> np.ndarray:
    um = np.ascontiguousarray(u, dtype=np.complex128)
    vm = np.ascontiguousarray(v, dtype=np.complex128)
    out = np.empty((3, 3), dtype=np.complex128)
    lib().ora_maxretr(_p(um), _p(vm), int(loops), _p(out))
    return out


def _upd(update):
    return {"stout": STOUT, "maxretr": MAXRETR, "cooling": MAXRETR, "ape": APE}.get(update, update)


def unit_circle_projection(v) -> np.ndarray:
    v = np.ascontiguousarray(v, dtype=np.complex128)
    out = np.empty((3, 3), dtype=np.complex128)
    lib().ora_unit_circle_projection(_p(v), _p(out))
    return out


def update_link(dims, links, n0, mu, site, *, gauge=None, update="stout", vp=False, rho=0.1,
                eps=1.0, u0=1.0, alpha=1.0, su2_loops=3):
    links = np.ascontiguousarray(links, dtype=np.complex128)
    n0 = None if n0 is None else np.ascontiguousarray(n0, dtype=np.int8)
    gauge = None if gauge is None else np.ascontiguousarray(gauge, dtype=np.complex128)
    out = np.empty((3, 3), dtype=np.complex128)
    acc = ctypes.c_int32(0)
    _check(lib().ora_update_link(_p(_dims(dims)), _p(links), _p(n0), _p(gauge), _upd(update),
                                 int(bool(vp)), float(rho), float(eps), float(u0), float(alpha),
                                 int(su2_loops), int(mu), int(site), _p(out), ctypes.byref(acc)),
           "update_link")
    return out, bool(acc.value)


def update_links(dims, links, n0, mus, sites, *, gauge=None, update="stout", vp=False, rho=0.1,
                 eps=1.0, u0=1.0, alpha=1.0, su2_loops=3):
    """update_link for many (mu, site) pairs with one lattice set-up: returns
    (complex128 [count, 3, 3], bool [count])."""
    links = np.ascontiguousarray(links, dtype=np.complex128)
    n0 = None if n0 is None else np.ascontiguousarray(n0, dtype=np.int8)
    gauge = None if gauge is None else np.ascontiguousarray(gauge, dtype=np.complex128)
    mus = np.ascontiguousarray(mus, dtype=np.int32)
    sites = np.ascontiguousarray(sites, dtype=np.int64)
    assert mus.shape == sites.shape and mus.ndim == 1
    out = np.empty((len(mus), 3, 3), dtype=np.complex128)
    acc = np.empty(len(mus), dtype=np.int32)
    _check(lib().ora_update_links(_p(_dims(dims)), _p(links), _p(n0), _p(gauge), _upd(update),
                                  int(bool(vp)), float(rho), float(eps), float(u0), float(alpha),
                                  int(su2_loops), len(mus), _p(mus), _p(sites), _p(out), _p(acc)),
           "update_links")
    return out, acc.astype(bool)


def anneal_pass(dims, links, n0, mu, colour, *, gauge=None, update="stout", vp=False, rho=0.1,
                eps=1.0, u0=1.0, alpha=1.0, su2_loops=3):
    """One masked annealing subset, in place on `links`; returns the rejection count."""
    assert links.dtype == np.complex128 and links.flags.c_contiguous
    n0 = None if n0 is None else np.ascontiguousarray(n0, dtype=np.int8)
    gauge = None if gauge is None else np.ascontiguousarray(gauge, dtype=np.complex128)
    rej = ctypes.c_int64(0)
    _check(lib().ora_pass(_p(_dims(dims)), _p(links), _p(n0), _p(gauge), _upd(update),
                          int(bool(vp)), float(rho), float(eps), float(u0), float(alpha),
                          int(su2_loops), int(mu), int(colour), ctypes.byref(rej)), "pass")
    return int(rej.value)


def smooth(dims, links, n0, n_sweeps, *, order="annealed", update="stout", vp=False, rho=0.1,
           eps=1.0, u0=1.0, alpha=1.0, su2_loops=3, gauge=None, measure_every=1):
    """Run n_sweeps sweeps in place on `links`; returns the per-record stats array."""
    assert links.dtype == np.complex128 and links.flags.c_contiguous
    n0 = None if n0 is None else np.ascontiguousarray(n0, dtype=np.int8)
    gauge = None if gauge is None else np.ascontiguousarray(gauge, dtype=np.complex128)
    o = {"jacobi": JACOBI, "annealed": ANNEALED}.get(order, order)
    nrec = n_sweeps // measure_every if measure_every > 0 else 0
    stats = np.zeros(max(nrec, 1), dtype=STATS_DTYPE)
    _check(lib().ora_smooth(_p(_dims(dims)), _p(links), _p(n0), _p(gauge), int(n_sweeps), o,
                            _upd(update), int(bool(vp)), float(rho), float(eps), float(u0),
                            float(alpha), int(su2_loops), int(measure_every), _p(stats)),
           "smooth")
    return stats[:nrec].view(np.recarray)


def measure(dims, links, n0, with_flux=False, gauge=None):
    """One stats record; with a gauge G (complex128 [V,3,3]) the centre sectors
    of the links are those of G^dag(x) U G(x+mu)."""
    links = np.ascontiguousarray(links, dtype=np.complex128)
    n0 = np.ascontiguousarray(n0, dtype=np.int8)
    gauge = None if gauge is None else np.ascontiguousarray(gauge, dtype=np.complex128)
    st = np.zeros(1, dtype=STATS_DTYPE)
    flux = np.empty((6, _vol(dims)), dtype=np.int8) if with_flux else None
    _check(lib().ora_measure(_p(_dims(dims)), _p(links), _p(n0), _p(gauge), _p(st), _p(flux)), "measure")
    rec = st.view(np.recarray)[0]
    return (rec, flux) if with_flux else rec


def flow(dims, links, n_steps, eps, *, eps_oi=1.0, u0=1.0, integrator="rk3"):
    """Wilson flow in place on `links` (every link at once): Euler or RK3."""
    assert links.dtype == np.complex128 and links.flags.c_contiguous
    it = {"euler": 0, "rk3": 1}[integrator]
    _check(lib().ora_flow(_p(_dims(dims)), _p(links), int(n_steps), float(eps), float(eps_oi), float(u0), it),
           "flow")


def clover(dims, links, densities=False):
    """(<S_R>/beta, Q, <S>/beta) from the 1x1 clover field strength; with
    densities, also S(x)/beta and q(x) as float64 [V] (canonical order)."""
    links = np.ascontiguousarray(links, dtype=np.complex128)
    out = np.zeros(3, dtype=np.float64)
    V = _vol(dims)
    sd = np.empty(V, dtype=np.float64) if densities else None
    qd = np.empty(V, dtype=np.float64) if densities else None
    _check(lib().ora_clover(_p(_dims(dims)), _p(links), _p(out), _p(sd), _p(qd)), "clover")
    sr, q, s = (float(v) for v in out)
    return (sr, q, s, sd, qd) if densities else (sr, q, s)


def correlation(a, b) -> float:
    a = np.ascontiguousarray(a, dtype=np.float64)
    b = np.ascontiguousarray(b, dtype=np.float64)
    assert a.shape == b.shape
    return float(lib().ora_correlation(a.size, _p(a), _p(b)))


def sectors(dims, links) -> np.ndarray:
    links = np.ascontiguousarray(links, dtype=np.complex128)
    out = np.empty((4, _vol(dims)), dtype=np.int8)
    _check(lib().ora_sectors(_p(_dims(dims)), _p(links), _p(out)), "sectors")
    return out
