"""Seeded synthetic inputs shared by the oracle and the HIP path.

This module holds no arithmetic of the smoothing method itself.  It only draws
random numbers and arranges them on the lattice:

* Z(3) vortex charges n_mu(x) in {-1, 0, 1} built from a random gauge part g(x)
  and a sparse random "vortex seed" s_mu(x) (the synthetic stand-in for the
  paper's single Z(3)-projected 20^3 x 40 configuration, which is not available);
* the random pair choice (j, k) of centrifuge preconditioning (Sec. IV draws one
  pair per link at random; the draw is made here and passed to both sides);
* Haar-random SU(3) matrices G(x) for the random-gauge variants (Sec. V.C, VI);
* Poisson arrival streams of smoothing jobs for the serving workload.

Canonical layout (both sides read it): site s = x + Lx*(y + Ly*(z + Lz*t)),
direction mu = 0..3 = (x, y, z, t); charges are int8 [4][V]; pair choices are
int8 [4][V] in {0, 1, 2} meaning (j, k) = (1, 2), (2, 3), (3, 1); gauge matrices
are complex128 [V][3][3].
"""
from __future__ import annotations

import dataclasses

import numpy as np

__all__ = [
    "volume",
    "neighbour",
    "z3_vortex_charges",
    "centrifuge_pairs",
    "haar_su3",
    "JobSpec",
    "poisson_jobs",
    "CONFIGS",
]


def volume(dims) -> int:
    d = [int(v) for v in dims]
    if len(d) != 4 or min(d) < 1:
        raise ValueError(f"dims must be four positive extents, got {dims!r}")
    return d[0] * d[1] * d[2] * d[3]


def neighbour(dims, mu: int, step: int) -> np.ndarray:
    """Index array nb with nb[s] = site s shifted by `step` along direction mu (periodic)."""
    L = [int(v) for v in dims]
    V = volume(L)
    s = np.arange(V, dtype=np.int64)
    coords = []
    r = s
    for d in range(4):
        coords.append(r % L[d])
        r = r // L[d]
    coords[mu] = (coords[mu] + step) % L[mu]
    out = coords[3]
    for d in (2, 1, 0):
        out = out * L[d] + coords[d]
    return out


def z3_vortex_charges(dims, p: float, seed: int, return_parts: bool = False):
    """Z(3) vortex charges n_mu(x) = (g(x+mu) - g(x) + s_mu(x)) mod 3, as int8 [4][V].

    g(x) is uniform in {0, 1, 2}; s_mu(x) is non-zero with probability p, and then
    1 or 2 with equal probability.  The residue 2 is represented by -1, so every
    charge lies in {-1, 0, 1} (the representatives of Eq. (centre_element)).
    With return_parts, (n, g, s) is returned.
    """
    V = volume(dims)
    if not 0.0 <= p <= 1.0:
        raise ValueError("p must lie in [0, 1]")
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 0x5A3]))
    g = rng.integers(0, 3, size=V, dtype=np.int64)
    hit = rng.random((4, V)) < p
    val = 1 + rng.integers(0, 2, size=(4, V), dtype=np.int64)
    s = np.where(hit, val, 0)
    n = np.empty((4, V), dtype=np.int8)
    for mu in range(4):
        r = (g[neighbour(dims, mu, +1)] - g + s[mu]) % 3
        n[mu] = np.where(r == 2, -1, r).astype(np.int8)
    if return_parts:
        return n, g, s
    return n


def centrifuge_pairs(dims, seed: int) -> np.ndarray:
    """Uniform random pair choice per link, int8 [4][V] in {0, 1, 2}."""
    V = volume(dims)
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 0xC3F]))
    return rng.integers(0, 3, size=(4, V), dtype=np.int8)


def haar_su3(count: int, seed: int) -> np.ndarray:
    """`count` Haar-distributed SU(3) matrices, complex128 [count][3][3].

    Drawn as the QR factor of a complex Gaussian matrix with the phases of R's
    diagonal moved into Q (Mezzadri's recipe), then divided by a cube root of
    the determinant so that det = 1.
    """
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 0x6A9]))
    z = (rng.standard_normal((count, 3, 3)) + 1j * rng.standard_normal((count, 3, 3))) / np.sqrt(2.0)
    q, r = np.linalg.qr(z)
    d = np.diagonal(r, axis1=1, axis2=2)
    ph = d / np.abs(d)
    q = q * ph[:, None, :]
    det = np.linalg.det(q)
    q = q / (det ** (1.0 / 3.0))[:, None, None]
    return np.ascontiguousarray(q)


@dataclasses.dataclass(frozen=True)
class JobSpec:
    """One smoothing request of the serving workload."""

    job_id: int
    arrival_s: float
    dims: tuple
    p: float
    field_seed: int
    pair_seed: int
    n_sweeps: int


SERVING_SIZES = ((8, 8, 8, 8), (12, 12, 12, 24), (16, 16, 16, 32), (20, 20, 20, 40))


def poisson_jobs(n_jobs: int, rate_per_s: float, seed: int, sizes=SERVING_SIZES,
                 sweeps_range=(50, 300), p_range=(0.05, 0.15)) -> list:
    """A Poisson stream of smoothing jobs: exponential inter-arrival times with the
    given mean rate; lattice uniform over `sizes`; sweep count uniform integer in
    `sweeps_range` (inclusive); vortex density p uniform in `p_range`."""
    rng = np.random.default_rng(np.random.SeedSequence([int(seed), 0x10B]))
    gaps = rng.exponential(1.0 / rate_per_s, size=n_jobs)
    t = np.cumsum(gaps)
    which = rng.integers(0, len(sizes), size=n_jobs)
    sweeps = rng.integers(sweeps_range[0], sweeps_range[1] + 1, size=n_jobs)
    ps = rng.uniform(p_range[0], p_range[1], size=n_jobs)
    jobs = []
    for j in range(n_jobs):
        jobs.append(JobSpec(job_id=j, arrival_s=float(t[j]), dims=tuple(sizes[int(which[j])]),
                            p=float(ps[j]), field_seed=4000 + j, pair_seed=6000 + j,
                            n_sweeps=int(sweeps[j])))
    return jobs


# The five workloads: lattice, vortex density, seeds and smoothing recipe.
CONFIGS = {
    "c0": dict(dims=(8, 8, 8, 8), p=0.05, field_seed=1000, pair_seed=2000, omega=0.02,
               n_sweeps=10, rho=0.1, eps=1.0, order="jacobi", vp=False),
    "c1": dict(dims=(16, 16, 16, 32), p=0.10, field_seed=1001, pair_seed=2001, omega=0.02,
               n_sweeps=200, rho=0.06, eps=-0.25, order="annealed", vp=True),
    "c2": dict(dims=(32, 32, 32, 64), p=0.10, field_seed=1002, pair_seed=2002, omega=0.02,
               n_sweeps=500, rho=0.06, eps=-0.25, order="annealed", vp=True),
    "c4": dict(dims=(48, 48, 48, 96), p=0.10, field_seed=1004, pair_seed=2004, omega=0.02,
               n_sweeps=300, rho=0.06, eps=-0.25, order="annealed", vp=True),
}
