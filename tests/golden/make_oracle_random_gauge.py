"""Write the random-gauge (full SU(3)) fixtures of the 8^4 and 16^3 x 32 workloads
with the FP64 oracle.

Runs only oracle/ (and the seeded input generators).  Each workload's field is
built and preconditioned as usual (Z(3) vortex field, centrifuge omega = 0.02),
then put into a Haar-random gauge G (seed 5000 + workload number, Sec. V.C),
which moves every link off the diagonal subgroup, and smoothed with the
workload's recipe, the vortex-preserving test (where the recipe has it) and the
measurement undoing G (Sec. VI):
  8^4 (p = 0.05, seeds 1000/2000): 10 smearing sweeps of plain stout, rho = 0.1
      (no vortex preservation, as in the workload);
  16^3 x 32 (p = 0.1, seeds 1001/2001): 20 annealed over-improved stout sweeps,
      rho = 0.06, eps = -0.25, with vortex preservation.
Records plaquette, action, rejections and flux mismatches (measured in the
random gauge) after every sweep, and 64 sampled links after sweeps 1, 2 and
the last.
Usage: python tests/golden/make_oracle_random_gauge.py   (about a minute on 8 threads)
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import fieldgen  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "random_gauge_oracle.txt")
RUNS = {"c0": dict(n_sweeps=10, vp=False), "c1": dict(n_sweeps=20, vp=True)}
N_SAMPLES = 64


def main():
    rng = np.random.default_rng(779)
    lines = []
    t0 = time.time()
    for name, run in RUNS.items():
        c = fieldgen.CONFIGS[name]
        dims = c["dims"]
        n = fieldgen.z3_vortex_charges(dims, c["p"], c["field_seed"])
        pairs = fieldgen.centrifuge_pairs(dims, c["pair_seed"])
        V = fieldgen.volume(dims)
        G = fieldgen.haar_su3(V, 5000 + int(name[1:]))
        U = oracle.gauge_transform(dims, oracle.centrifuge(dims, n, pairs, c["omega"]), G)
        ns = run["n_sweeps"]
        stats, done = [], 0
        for k in sorted({1, 2, ns}):
            stats.extend(oracle.smooth(dims, U, n, k - done, order=c["order"], rho=c["rho"], eps=c["eps"],
                                       vp=run["vp"], gauge=G, measure_every=1))
            done = k
            mus = rng.integers(0, 4, size=N_SAMPLES)
            sites = rng.integers(0, V, size=N_SAMPLES)
            for mu, s in zip(mus, sites):
                vals = " ".join("%.17e %.17e" % (z.real, z.imag) for z in U[mu, s].reshape(-1))
                lines.append("L %s %d %d %d %s" % (name, k, mu, s, vals))
        for i, r in enumerate(stats):
            lines.append("S %s %d %.17e %.17e %d %d" % (name, i + 1, r.plaq, r.action, r.rejected, r.flux_mismatch))
        print(f"{name}: {ns} sweeps, {time.time() - t0:.0f} s", flush=True)
    dt = time.time() - t0
    with open(OUT, "w") as f:
        f.write("# FP64 oracle, the 8^4 and 16^3x32 workloads in a Haar-random gauge G (seed 5000 + workload),\n")
        f.write("# measurement and vortex preservation undoing G (Sec. V.C, VI).  8^4: 10 smearing sweeps of plain\n")
        f.write("# stout rho=0.1, no vortex preservation; 16^3x32: with vortex preservation,\n")
        f.write("# 20 annealed over-improved stout sweeps rho=0.06 eps=-0.25.  Fields built as usual\n")
        f.write("# (Z(3) vortex field, centrifuge omega=0.02) and then transformed with G.\n")
        f.write("# Written by tests/golden/make_oracle_random_gauge.py (oracle only); %.0f s on %d threads.\n"
                % (dt, oracle.set_threads(0)))
        f.write("# S workload sweep plaq action rejected flux_mismatch\n")
        f.write("# L workload sweep mu site then 9 complex entries re im (row-major)\n")
        for ln in sorted(lines, key=lambda s: (s[0] != "S", s.split()[1], int(s.split()[2]))):
            f.write(ln + "\n")
    print(f"wrote {OUT}: {dt:.0f} s")


if __name__ == "__main__":
    main()
