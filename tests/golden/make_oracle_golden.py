"""Write the long-trajectory fixture of the 16^3 x 32 workload with the FP64 oracle.

Runs only oracle/ (and the seeded input generator): centrifuge preconditioning
(omega = 0.02) of the Z(3) vortex field (p = 0.1, seeds 1001/2001), then 200
annealed over-improved stout sweeps (rho = 0.06, eps = -0.25, u0 = 1) with
vortex preservation.  Records plaquette, action and rejections after every
sweep, and 64 sampled links at each checkpoint sweep.

The same run is repeated from a start perturbed at the rounding level
(U -> (1 + X) U with X anti-Hermitian, entries of size 1e-16, seed 5); the
largest link difference between the two runs at each checkpoint measures how
much the smoothing map itself amplifies a rounding difference by then (the
accept/reject test and the flow near vortex cores are not contractions).  Any
two correct FP64 implementations can differ by that much.
Usage: python tests/golden/make_oracle_golden.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import fieldgen  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "c1_oracle_trajectory.txt")
CHECKPOINTS = (1, 2, 5, 10, 20, 50, 100, 200)
N_SAMPLES = 64


def run(dims, U, n, c):
    """Sweeps up to each checkpoint; per-sweep stats and the field at each checkpoint."""
    stats, snaps, done = [], {}, 0
    for k in CHECKPOINTS:
        st = oracle.smooth(dims, U, n, k - done, order="annealed", rho=c["rho"], eps=c["eps"],
                           vp=True, measure_every=1)
        stats.extend(st)
        snaps[k] = U.copy()
        done = k
    return stats, snaps


def main():
    c = fieldgen.CONFIGS["c1"]
    dims = c["dims"]
    assert CHECKPOINTS[-1] == c["n_sweeps"]
    n = fieldgen.z3_vortex_charges(dims, c["p"], c["field_seed"])
    pairs = fieldgen.centrifuge_pairs(dims, c["pair_seed"])
    U = oracle.centrifuge(dims, n, pairs, c["omega"])
    V = fieldgen.volume(dims)
    rng = np.random.default_rng(5)
    A = rng.normal(size=U.shape) + 1j * rng.normal(size=U.shape)
    X = 0.5 * (A - np.conj(np.swapaxes(A, -1, -2))) * 1e-16
    U2 = np.ascontiguousarray(U + np.einsum("dsij,dsjk->dsik", X, U))
    t = time.time()
    stats, snaps = run(dims, U, n, c)
    dt = time.time() - t
    _, snaps2 = run(dims, U2, n, c)
    rng = np.random.default_rng(777)
    with open(OUT, "w") as f:
        f.write("# FP64 oracle trajectory of the 16^3x32 workload: Z(3) vortex field p=0.1\n")
        f.write("# (seeds 1001/2001), centrifuge omega=0.02, 200 annealed over-improved stout\n")
        f.write("# sweeps rho=0.06 eps=-0.25 u0=1 with vortex preservation (Sec. IV-VI).\n")
        f.write("# Written by tests/golden/make_oracle_golden.py (oracle only); %.0f s per run on %d threads.\n"
                % (dt, oracle.set_threads(0)))
        f.write("# section sweeps: S sweep plaq action rejected flux_mismatch\n")
        for i, r in enumerate(stats):
            f.write("S %d %.17e %.17e %d %d\n" % (i + 1, r.plaq, r.action, r.rejected, r.flux_mismatch))
        f.write("# section sensitivity: C sweep max|U - U'| over all links, U' from the perturbed start\n")
        for k in CHECKPOINTS:
            f.write("C %d %.6e\n" % (k, np.abs(snaps[k] - snaps2[k]).max()))
        f.write("# section links: L sweep mu site then 9 complex entries re im (row-major)\n")
        for k in CHECKPOINTS:
            mus = rng.integers(0, 4, size=N_SAMPLES)
            sites = rng.integers(0, V, size=N_SAMPLES)
            for mu, s in zip(mus, sites):
                vals = " ".join("%.17e %.17e" % (z.real, z.imag) for z in snaps[k][mu, s].reshape(-1))
                f.write("L %d %d %d %s\n" % (k, mu, s, vals))
    print(f"wrote {OUT}: {dt:.0f} s per run")


if __name__ == "__main__":
    main()
