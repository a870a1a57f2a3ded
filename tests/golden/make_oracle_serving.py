"""Write the serving-stream fixture with the FP64 oracle.

Runs only oracle/ (and the seeded input generators).  From the serving stream
(Poisson arrivals at 50 jobs/s, arrival seed 3, 200 jobs) the first job of each
lattice size (8^4, 12^3 x 24, 16^3 x 32, 20^3 x 40) is taken with its own vortex
density and seeds; its sweep count is cut so that the oracle finishes in about
two minutes (50, 20, 10 and 6 sweeps).  Each job is the serving recipe:
centrifuge preconditioning (omega = 0.02), then annealed over-improved stout
sweeps (rho = 0.06, eps = -0.25, u0 = 1) with vortex preservation.  Records
plaquette, action, rejections and flux mismatches after every sweep, and 64
sampled links after the last sweep.
Usage: python tests/golden/make_oracle_serving.py
"""
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
sys.path.insert(0, ROOT)

import fieldgen  # noqa: E402
import oracle  # noqa: E402

OUT = os.path.join(os.path.dirname(os.path.abspath(__file__)), "serving_oracle_jobs.txt")
SWEEPS = {(8, 8, 8, 8): 50, (12, 12, 12, 24): 20, (16, 16, 16, 32): 10, (20, 20, 20, 40): 6}
N_SAMPLES = 64


def serving_jobs():
    """(job spec, sweeps) of the first job of each lattice size in the stream."""
    out = {}
    for sp in fieldgen.poisson_jobs(200, 50.0, 3):
        if sp.dims not in out:
            out[sp.dims] = sp
    return [(out[d], SWEEPS[d]) for d in fieldgen.SERVING_SIZES]


def main():
    rng = np.random.default_rng(780)
    lines = []
    t0 = time.time()
    for sp, ns in serving_jobs():
        dims = sp.dims
        n = fieldgen.z3_vortex_charges(dims, sp.p, sp.field_seed)
        pairs = fieldgen.centrifuge_pairs(dims, sp.pair_seed)
        U = oracle.centrifuge(dims, n, pairs, 0.02)
        st = oracle.smooth(dims, U, n, ns, order="annealed", rho=0.06, eps=-0.25, vp=True, measure_every=1)
        tag = "x".join(str(v) for v in dims)
        lines.append("J %s %d %.17e %d %d %d" % (tag, sp.job_id, sp.p, sp.field_seed, sp.pair_seed, ns))
        for i, r in enumerate(st):
            lines.append("S %s %d %.17e %.17e %d %d" % (tag, i + 1, r.plaq, r.action, r.rejected, r.flux_mismatch))
        V = fieldgen.volume(dims)
        for mu, s in zip(rng.integers(0, 4, size=N_SAMPLES), rng.integers(0, V, size=N_SAMPLES)):
            vals = " ".join("%.17e %.17e" % (z.real, z.imag) for z in U[mu, s].reshape(-1))
            lines.append("L %s %d %d %s" % (tag, mu, s, vals))
        print(f"{tag}: {ns} sweeps, {time.time() - t0:.0f} s", flush=True)
    dt = time.time() - t0
    with open(OUT, "w") as f:
        f.write("# FP64 oracle, the first job of each lattice size of the serving stream (Poisson 50 jobs/s,\n")
        f.write("# arrival seed 3): centrifuge omega=0.02, annealed over-improved stout rho=0.06 eps=-0.25\n")
        f.write("# with vortex preservation, sweeps cut to 50 / 20 / 10 / 6 (Sec. IV-VI).\n")
        f.write("# Written by tests/golden/make_oracle_serving.py (oracle only); %.0f s on %d threads.\n"
                % (dt, oracle.set_threads(0)))
        f.write("# J lattice job_id p field_seed pair_seed sweeps\n")
        f.write("# S lattice sweep plaq action rejected flux_mismatch\n")
        f.write("# L lattice mu site then 9 complex entries re im (row-major), after the last sweep\n")
        for ln in lines:
            f.write(ln + "\n")
    print(f"wrote {OUT}: {dt:.0f} s")


if __name__ == "__main__":
    main()
