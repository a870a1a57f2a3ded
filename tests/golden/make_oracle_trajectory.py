"""Write the per-sweep fixture of the 32^3 x 64 or 48^3 x 96 workload with the FP64 oracle.

Runs only oracle/ (and the seeded input generator): centrifuge preconditioning
(omega = 0.02) of the workload's Z(3) vortex field (p = 0.1; seeds 1002/2002 for
32^3 x 64, 1004/2004 for 48^3 x 96), then its annealed over-improved stout
sweeps (rho = 0.06, eps = -0.25, u0 = 1) with vortex preservation (all of them,
or the first N with an argument N).  Records plaquette, action and rejections
after every sweep, and 64 sampled links after sweeps 1 and 2 (before the
smoothing map has amplified rounding differences; the 16^3 x 32 fixture
measures that amplification) and after the last sweep.
Usage: python tests/golden/make_oracle_trajectory.py c2|c4 [N]
       (32^3 x 64: about 16 s a sweep on 8 threads; 48^3 x 96: about 5 times that)
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import fieldgen  # noqa: E402
import oracle  # noqa: E402

CFG = sys.argv[1] if len(sys.argv) > 1 else "c2"
N_SWEEPS = int(sys.argv[2]) if len(sys.argv) > 2 else fieldgen.CONFIGS[CFG]["n_sweeps"]
OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), f"{CFG}_oracle_trajectory.txt")
LINK_SWEEPS = (1, 2)
N_SAMPLES = 64
TITLE = {"c2": "32^3x64", "c4": "48^3x96"}


def main():
    c = fieldgen.CONFIGS[CFG]
    dims = c["dims"]
    n = fieldgen.z3_vortex_charges(dims, c["p"], c["field_seed"])
    pairs = fieldgen.centrifuge_pairs(dims, c["pair_seed"])
    U = oracle.centrifuge(dims, n, pairs, c["omega"])
    V = fieldgen.volume(dims)
    rng = np.random.default_rng(778)
    stats, links, done = [], [], 0
    t = time.time()
    for k in sorted(set(LINK_SWEEPS + (N_SWEEPS,))):
        stats.extend(oracle.smooth(dims, U, n, k - done, order="annealed", rho=c["rho"], eps=c["eps"],
                                   vp=True, measure_every=1))
        done = k
        if k in LINK_SWEEPS or k == N_SWEEPS:
            mus = rng.integers(0, 4, size=N_SAMPLES)
            sites = rng.integers(0, V, size=N_SAMPLES)
            links.extend((k, int(mu), int(s), U[mu, s].copy()) for mu, s in zip(mus, sites))
        print(f"sweep {k}: {time.time() - t:.0f} s", flush=True)
    dt = time.time() - t
    with open(OUT, "w") as f:
        f.write("# FP64 oracle, %s workload: Z(3) vortex field p=%g (seeds %d/%d),\n"
                % (TITLE[CFG], c["p"], c["field_seed"], c["pair_seed"]))
        f.write("# centrifuge omega=0.02, the first %d annealed over-improved stout sweeps\n" % N_SWEEPS)
        f.write("# rho=0.06 eps=-0.25 u0=1 with vortex preservation (Sec. IV-VI).\n")
        f.write("# Written by tests/golden/make_oracle_trajectory.py %s (oracle only); %.0f s on %d threads.\n"
                % (CFG, dt, oracle.set_threads(0)))
        f.write("# section sweeps: S sweep plaq action rejected flux_mismatch\n")
        for i, r in enumerate(stats):
            f.write("S %d %.17e %.17e %d %d\n" % (i + 1, r.plaq, r.action, r.rejected, r.flux_mismatch))
        f.write("# section links: L sweep mu site then 9 complex entries re im (row-major)\n")
        for k, mu, s, u in links:
            vals = " ".join("%.17e %.17e" % (z.real, z.imag) for z in u.reshape(-1))
            f.write("L %d %d %d %s\n" % (k, mu, s, vals))
    print(f"wrote {OUT}: {dt:.0f} s")


if __name__ == "__main__":
    main()
