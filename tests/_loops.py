"""Independent numpy closed-loop products, used to pin the oracle.

Whole-lattice plaquettes and rectangles built with numpy from shifted link
arrays.  The code shares nothing with the oracle's path walker or staples.
"""
import numpy as np

import fieldgen


def shift(dims, arr, mu, step):
    """arr[s] -> arr[s + step*mu] for a per-site array (first axis = site)."""
    return arr[fieldgen.neighbour(dims, mu, step)]


def dag(a):
    return np.conj(np.swapaxes(a, -1, -2))


def plaquettes(dims, U):
    """P_{mu nu}(x) for mu < nu, list of 6 arrays [V,3,3] in plane order 01,02,03,12,13,23."""
    out = []
    for mu in range(4):
        for nu in range(mu + 1, 4):
            a = U[mu]
            b = shift(dims, U[nu], mu, 1)
            c = shift(dims, U[mu], nu, 1)
            d = U[nu]
            out.append(a @ b @ dag(c) @ dag(d))
    return out


def rectangles(dims, U):
    """2x1 rectangles R_{mu nu}(x) (two steps along mu, one along nu) for every
    ordered pair mu != nu: every unoriented 1x2 loop of the lattice exactly once."""
    out = []
    for mu in range(4):
        for nu in range(4):
            if nu == mu:
                continue
            a = U[mu]
            b = shift(dims, U[mu], mu, 1)
            c = shift(dims, shift(dims, U[nu], mu, 1), mu, 1)
            d = shift(dims, shift(dims, U[mu], mu, 1), nu, 1)
            e = shift(dims, U[mu], nu, 1)
            f = U[nu]
            out.append(a @ b @ c @ dag(d) @ dag(e) @ dag(f))
    return out


def improved_action(dims, U, eps, u0=1.0):
    """sum over unoriented plaquettes of c_p Re Tr P plus sum over unoriented
    1x2 rectangles of c_r Re Tr R, with c_p = (5-2eps)/3, c_r = (eps-1)/(12 u0^2)."""
    cp = (5.0 - 2.0 * eps) / 3.0
    cr = (eps - 1.0) / (12.0 * u0 * u0)
    a = cp * sum(np.trace(p, axis1=1, axis2=2).real.sum() for p in plaquettes(dims, U))
    if cr != 0.0:
        a += cr * sum(np.trace(r, axis1=1, axis2=2).real.sum() for r in rectangles(dims, U))
    return a


def gell_mann_generators():
    """T^a = (i/2) lambda_a: traceless anti-Hermitian, Tr T^a T^b = -1/2 delta."""
    lam = np.zeros((8, 3, 3), dtype=np.complex128)
    lam[0][0, 1] = lam[0][1, 0] = 1
    lam[1][0, 1] = -1j
    lam[1][1, 0] = 1j
    lam[2][0, 0] = 1
    lam[2][1, 1] = -1
    lam[3][0, 2] = lam[3][2, 0] = 1
    lam[4][0, 2] = -1j
    lam[4][2, 0] = 1j
    lam[5][1, 2] = lam[5][2, 1] = 1
    lam[6][1, 2] = -1j
    lam[6][2, 1] = 1j
    lam[7] = np.diag([1, 1, -2]) / np.sqrt(3.0)
    return 0.5j * lam
