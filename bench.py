"""Benchmark of the vortex-field smoothing path on one MI355X.

Workload (default c4): a 48^3 x 96 Z(3) vortex field (p = 0.1), centrifuge
preconditioning (omega = 0.02), then annealed over-improved stout sweeps
(rho = 0.06, eps = -0.25, u0 = 1) with vortex preservation and one measurement
record (plaquette, action, vortex-flux check) after every sweep.  One "step" is
one such sweep: 16 subset passes over all 4V links plus the measurement.

Prints ONE JSON line.  value = link updates per second (4V per sweep) of the
whole timed region (inputs resident in HBM, K sweeps, both ends synchronised).
roofline = the dominant kernel (one annealing subset pass) against HBM
bandwidth: algorithmic bytes per launch (every link read once and the updated
one written, counted as full 3x3 complex matrices, plus its charge byte) / the
average launch duration measured with HIP events on the library's stream; the
fraction by the bytes this layout moves (rows 0 and 1 of each link) is given
beside it.  cpu_baseline = the FP64 CPU oracle
timed on a bounded sample (the first subset passes of the same field, ~10 s).
"""
from __future__ import annotations

import argparse
import hashlib
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

HBM_PEAK_GBS = 8000.0  # MI355X HBM3E, published
WORKLOADS = {
    "c4": "48^3x96 Z(3) vortex field p=0.1, centrifuge omega=0.02, annealed over-improved stout "
          "rho=0.06 eps=-0.25 with vortex preservation, measurement every sweep",
    "c2": "32^3x64 Z(3) vortex field p=0.1, centrifuge omega=0.02, annealed over-improved stout "
          "rho=0.06 eps=-0.25 with vortex preservation, measurement every sweep",
    "c1": "16^3x32 Z(3) vortex field p=0.1, centrifuge omega=0.02, annealed over-improved stout "
          "rho=0.06 eps=-0.25 with vortex preservation, measurement every sweep",
}


def pass_bytes_per_lu(precision: str, stored: bool = False) -> int:
    """Algorithmic HBM bytes per link update of one annealing subset pass: the
    pass reads every link of the lattice once (4V links for V/4 updates = 16 per
    update), writes the updated link, and reads its original charge (1 byte).
    A link counts as a full 3x3 complex matrix, 144 B in FP64 and 72 B in FP32
    (2449 and 1225 B per update).  With stored=True the count uses what this
    library's layout moves: rows 0 and 1, 96 B in FP64 and 48 B in FP32 (row 2
    is rebuilt in registers), 1633 and 817 B per update."""
    if stored:
        link = 96 if precision == "fp64" else 48
    else:
        link = 144 if precision == "fp64" else 72
    return 16 * link + link + 1


def _code_only(text: str) -> str:
    """C++ source without its comments and with whitespace runs collapsed, so that
    an edit of a comment leaves the hash of the kernel sources unchanged."""
    out, i, n = [], 0, len(text)
    while i < n:
        c = text[i]
        if c == '"' or c == "'":
            j = i + 1
            while j < n and text[j] != c:
                j += 2 if text[j] == "\\" else 1
            out.append(text[i:j + 1])
            i = j + 1
        elif text.startswith("//", i):
            j = text.find("\n", i)
            i = n if j < 0 else j
        elif text.startswith("/*", i):
            j = text.find("*/", i + 2)
            out.append(" ")
            i = n if j < 0 else j + 2
        else:
            out.append(c)
            i += 1
    return " ".join("".join(out).split())


def kernel_source_hash() -> str:
    """Hash of the code (comments removed) of every file under csrc/."""
    h = hashlib.sha256()
    csrc = os.path.join(ROOT, "paper_2203_09764_amd", "csrc")
    for name in sorted(os.listdir(csrc)):
        with open(os.path.join(csrc, name), encoding="utf-8") as f:
            h.update(name.encode())
            h.update(_code_only(f.read()).encode())
    return h.hexdigest()[:16]


def load_traffic(workload: str, precision: str, launch_lu: int):
    """HBM traffic per launch from the committed rocprofv3 counter summary, or None
    when it is missing or was taken on different kernel sources."""
    p = os.path.join(ROOT, "profiles", f"traffic_{workload}_{precision}.json")
    if not os.path.exists(p):
        return None
    with open(p) as f:
        d = json.load(f)
    if d.get("kernel_source_hash") != kernel_source_hash():
        return None
    return d.get("hbm_bytes_per_launch")


def run_gpu_form(args, precision, dims, n, pairs):
    import torch

    from paper_2203_09764_amd import api

    c = dict(rho=0.06, eps=-0.25)
    f = api.Field(dims, precision, device="cuda:0", jacobi_workspace=False)
    f.set_charges(n)
    api.precondition(f, pairs, 0.02)
    stream = torch.cuda.current_stream()
    # warmup
    if args.warmup > 0:
        api.smooth(f, args.warmup, c["rho"], c["eps"], order="annealed", vp=True, measure_every=1)
    torch.cuda.synchronize()
    stats = api.new_stats(args.steps, f.device)
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    wall0 = time.perf_counter()
    t0.record(stream)
    api.smooth(f, args.steps, c["rho"], c["eps"], order="annealed", vp=True, measure_every=1,
               stats=stats)
    t1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - wall0
    ms = t0.elapsed_time(t1)
    st = api.stats_to_numpy(stats, args.steps)
    V = f.V
    lu = 4 * V * args.steps
    # dominant kernel: one subset pass, timed launch by launch with events
    npass = 16 * args.pass_sweeps
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(npass + 1)]
    k = 0
    evs[0].record(stream)
    for _ in range(args.pass_sweeps):
        for mu in range(4):
            for colour in (0, 2, 1, 3):
                api.anneal_pass(f, mu, colour, c["rho"], c["eps"], vp=True)
                k += 1
                evs[k].record(stream)
    torch.cuda.synchronize()
    durs = [evs[i].elapsed_time(evs[i + 1]) for i in range(npass)]
    avg_pass_ms = sum(durs) / len(durs)
    # field strength of the smoothed field (Sec. V.A smoothness condition), timed
    ce = [torch.cuda.Event(enable_timing=True) for _ in range(4)]
    ce[0].record(stream)
    for i in range(3):
        cl = api.measure_clover(f)
        ce[i + 1].record(stream)
    torch.cuda.synchronize()
    clover_ms = sum(ce[i].elapsed_time(ce[i + 1]) for i in range(3)) / 3
    cl = cl.cpu().numpy()
    launch_lu = V // 4
    algo_bytes = launch_lu * pass_bytes_per_lu(precision)
    achieved = algo_bytes / (avg_pass_ms * 1e-3) / 1e9
    stored_bytes = launch_lu * pass_bytes_per_lu(precision, stored=True)
    return dict(
        precision=precision, ms=ms, wall_s=wall, lu_per_s=lu / (ms * 1e-3),
        ms_per_step=ms / args.steps, avg_pass_ms=avg_pass_ms, pass_launch_lu=launch_lu,
        pass_algo_bytes=algo_bytes, achieved_gbs=achieved, pass_stored_bytes=stored_bytes,
        achieved_stored_gbs=stored_bytes / (avg_pass_ms * 1e-3) / 1e9,
        action=[float(a) for a in st.action], plaq_last=float(st.plaq[-1]),
        flux_mismatch=int(st.flux_mismatch.sum()), nonfinite=int(st.nonfinite.sum()),
        max_unitarity=float(st.max_unitarity.max()), rejected=int(st.rejected.sum()),
        clover={"ms": round(clover_ms, 4), "sr_over_s": float(cl[0] / cl[2]), "Q": float(cl[1])},
    )


def stream_read_gbs(mib: int = 4096, reps: int = 5) -> float:
    """The device's practical HBM read rate: a plain streaming read (a float64
    sum) of `mib` MiB, timed with events."""
    import torch

    a = torch.ones((mib << 20) // 8, dtype=torch.float64, device="cuda:0")
    a.sum()
    stream = torch.cuda.current_stream()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    e0.record(stream)
    for _ in range(reps):
        a.sum()
    e1.record(stream)
    torch.cuda.synchronize()
    gbs = a.numel() * 8 / (e0.elapsed_time(e1) / reps * 1e-3) / 1e9
    del a
    torch.cuda.empty_cache()
    return gbs


def update_form(dims, n, pairs, precision, update="maxretr", sweeps=2, alpha=0.7):
    """Another update on the same preconditioned field, annealed, over-improved
    (eps = -0.25), alpha = 0.7, vortex preservation: MaxReTr (three SU(2)
    loops) or APE with unit circle projection.  Its subset passes are timed with
    events, as for the stout pass."""
    import torch

    from paper_2203_09764_amd import api

    f = api.Field(dims, precision, device="cuda:0", jacobi_workspace=False)
    f.set_charges(n)
    api.precondition(f, pairs, 0.02)
    kw = dict(update=update, alpha=alpha, vp=True)
    for mu in range(4):  # one untimed sweep
        for colour in (0, 2, 1, 3):
            api.anneal_pass(f, mu, colour, 0.0, -0.25, **kw)
    stream = torch.cuda.current_stream()
    evs = [torch.cuda.Event(enable_timing=True) for _ in range(16 * sweeps + 1)]
    k = 0
    evs[0].record(stream)
    for _ in range(sweeps):
        for mu in range(4):
            for colour in (0, 2, 1, 3):
                api.anneal_pass(f, mu, colour, 0.0, -0.25, **kw)
                k += 1
                evs[k].record(stream)
    torch.cuda.synchronize()
    durs = [evs[i].elapsed_time(evs[i + 1]) for i in range(16 * sweeps)]
    avg = sum(durs) / len(durs)
    st = api.stats_to_numpy(api.measure(f), 1)[0]
    lu = f.V // 4
    label = "MaxReTr, 3 SU(2) loops" if update == "maxretr" else "APE, unit circle projection"
    return {"update": "%s, alpha=%g, eps=-0.25, vortex preservation" % (label, alpha),
            "avg_pass_ms": round(avg, 4), "lu_per_s": round(lu / (avg * 1e-3), 1),
            "hbm_frac": round(lu * pass_bytes_per_lu(precision) / (avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "flux_mismatch": int(st.flux_mismatch)}


def flow_form(dims, n, pairs, precision, steps=2, eps=0.02):
    """Third-order Runge-Kutta Wilson flow (every link at once, plain staples)
    on the preconditioned field: the time of one step (3 stages, 12 launches)."""
    import torch

    from paper_2203_09764_amd import api

    f = api.Field(dims, precision, device="cuda:0", jacobi_workspace=False)
    f.set_charges(n)
    api.precondition(f, pairs, 0.02)
    api.flow(f, 1, eps, integrator="rk3")  # untimed, allocates its workspace once
    stream = torch.cuda.current_stream()
    t0 = torch.cuda.Event(enable_timing=True)
    t1 = torch.cuda.Event(enable_timing=True)
    torch.cuda.synchronize()
    t0.record(stream)
    api.flow(f, steps, eps, integrator="rk3")
    t1.record(stream)
    torch.cuda.synchronize()
    ms = t0.elapsed_time(t1) / steps
    return {"update": "Wilson flow, third-order Runge-Kutta, eps=%g, plain staples" % eps,
            "ms_per_step": round(ms, 3), "link_updates_per_s": round(3 * 4 * f.V / (ms * 1e-3), 1)}


def _serve_stream(n_jobs: int, rate: float, slots: int, seed: int) -> dict:
    """One replay of a Poisson stream of `n_jobs` jobs at `rate` jobs/s against a
    fresh server; inputs are generated before the clock starts."""
    import fieldgen
    from paper_2203_09764_amd import serve

    specs = fieldgen.poisson_jobs(n_jobs, rate, seed)
    jobs = []
    for sp in specs:
        n = fieldgen.z3_vortex_charges(sp.dims, sp.p, sp.field_seed)
        pairs = fieldgen.centrifuge_pairs(sp.dims, sp.pair_seed)
        jobs.append((sp.arrival_s, sp.dims, n, pairs, sp.n_sweeps))
    with serve.Server(hbm_budget_bytes=16 << 30, host_budget_bytes=256 << 20, max_slots=slots,
                      max_inflight=4) as srv:
        r = serve.run_stream(srv, jobs, precision="fp32_bulk", measure_every=0, rho=0.06, eps=-0.25,
                             vp=True, omega=0.02, timeout=600)
    r["offered_lu_per_s"] = r["link_updates"] / (specs[-1].arrival_s or 1.0)
    r["lost"] = sum(int(rec.flux_mismatch[-1]) for rec in r["records"])
    return r


def single_field_rates(precision="fp32_bulk", sweeps=8):
    """Link updates per second of vsm_smooth alone on each serving lattice size
    (the serving recipe, no measurement): what the stream would get if every
    job ran by itself on the whole GPU."""
    import torch

    import fieldgen
    from paper_2203_09764_amd import api

    out = {}
    for dims in fieldgen.SERVING_SIZES:
        n = fieldgen.z3_vortex_charges(dims, 0.1, 7)
        f = api.Field(dims, precision, device="cuda:0", jacobi_workspace=False)
        f.set_charges(n)
        api.precondition(f, fieldgen.centrifuge_pairs(dims, 8), 0.02)
        api.smooth(f, 2, 0.06, -0.25, order="annealed", vp=True)
        stream = torch.cuda.current_stream()
        e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
        torch.cuda.synchronize()
        e0.record(stream)
        api.smooth(f, sweeps, 0.06, -0.25, order="annealed", vp=True)
        e1.record(stream)
        torch.cuda.synchronize()
        out["x".join(str(v) for v in dims)] = round(4 * f.V * sweeps / (e0.elapsed_time(e1) * 1e-3), 1)
    return out


def serving_leg(n_jobs: int, rate: float, slots: int = 64, seed: int = 3,
                loads=((0.5, 120), (0.8, 150), (1.0, 150))):
    """The serving stream: Poisson arrivals at `rate` jobs/s of smoothing jobs on
    8^4, 12^3x24, 16^3x32 and 20^3x40 vortex fields (p uniform in [0.05, 0.15],
    50-300 sweeps), FP32-bulk annealed over-improved stout with vortex
    preservation, one final measurement each.  Latency = completion - submission
    on the server's clock.  The configured stream overloads the GPU, so its
    served rate is the capacity; the stream is then replayed at fractions of that
    capacity (other arrival seeds, `loads` = (fraction, jobs)) for the
    latency-versus-load curve."""
    r = _serve_stream(n_jobs, rate, slots, seed)
    c = r["counters"]
    mean_job_lu = r["link_updates"] / r["n_jobs"]
    capacity = r["lu_per_s"] / mean_job_lu
    out = {"workload": "Poisson stream, mean %g jobs/s, %d jobs on 8^4 / 12^3x24 / 16^3x32 / 20^3x40 "
                       "vortex fields, 50-300 sweeps each, FP32-bulk annealed OI stout + VP" % (rate, n_jobs),
           "p50_latency_s": round(r["p50_s"], 4), "p99_latency_s": round(r["p99_s"], 4),
           "mean_queue_s": round(r["mean_queue_s"], 4), "lu_per_s": round(r["lu_per_s"], 1),
           "offered_lu_per_s": round(r["offered_lu_per_s"], 1),
           "span_s": round(r["span_s"], 3), "steps": int(c["steps"]), "launches": int(c["launches"]),
           "peak_resident_jobs": int(c["peak_resident_jobs"]),
           "peak_pool_mib": round(c["peak_pool_bytes"] / 2**20, 1), "flux_mismatch_total": r["lost"],
           "capacity_jobs_per_s": round(capacity, 2)}
    curve = []
    for k, (frac, nj) in enumerate(loads):
        q = _serve_stream(nj, frac * capacity, slots, seed + 10 + k)
        curve.append({"load": frac, "rate_jobs_per_s": round(frac * capacity, 2), "n_jobs": nj,
                      "p50_latency_s": round(q["p50_s"], 4), "p99_latency_s": round(q["p99_s"], 4),
                      "mean_queue_s": round(q["mean_queue_s"], 4), "lu_per_s": round(q["lu_per_s"], 1),
                      "offered_lu_per_s": round(q["offered_lu_per_s"], 1), "flux_mismatch_total": q["lost"]})
    out["latency_vs_load"] = curve
    # the same sizes one at a time through vsm_smooth, and their mix weighted by
    # the stream's link updates (what serving would reach with no batching cost)
    single = single_field_rates()
    out["single_field_lu_per_s"] = single
    specs = fieldgen_mix(n_jobs, rate, seed)
    tot = sum(specs.values())
    out["single_field_mix_lu_per_s"] = round(tot / sum(lu / single[k] for k, lu in specs.items()), 1)
    return out


def fieldgen_mix(n_jobs, rate, seed):
    """Link updates of the stream per lattice size."""
    import fieldgen

    mix = {}
    for sp in fieldgen.poisson_jobs(n_jobs, rate, seed):
        k = "x".join(str(v) for v in sp.dims)
        mix[k] = mix.get(k, 0) + 4 * fieldgen.volume(sp.dims) * sp.n_sweeps
    return mix


def cpu_baseline(dims, n, pairs, threads):
    """The FP64 oracle on the first subset passes (about 10 s) of the same field."""
    import oracle

    used = oracle.set_threads(threads) if threads > 0 else oracle.set_threads(0)
    U = oracle.centrifuge(dims, n, pairs, 0.02)
    V = dims[0] * dims[1] * dims[2] * dims[3]
    done, dt, k = 0, 0.0, 0
    order = [(mu, c) for mu in range(4) for c in (0, 2, 1, 3)]
    while k < len(order) and (dt < 10.0 or k < 1):  # about 10 s of CPU work
        mu, c = order[k]
        t = time.perf_counter()
        oracle.anneal_pass(dims, U, n, mu, c, rho=0.06, eps=-0.25, vp=True)
        dt += time.perf_counter() - t
        done += V // 4
        k += 1
    info = {}
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                key, _, val = line.partition(":")
                key = key.strip()
                if key in ("model name", "cpu MHz", "cpu cores", "siblings", "cache size") and key not in info:
                    info[key] = val.strip()
    except OSError:
        pass
    return dict(value=done / dt, unit="link-updates/s", cores=int(used), kind="oracle",
                sample=f"the first {k} annealing subset passes of the first sweep of the same "
                       f"preconditioned field: {done} link updates in {dt:.1f} s",
                cpu_model=info.get("model name", "unknown"), cpu_mhz=info.get("cpu MHz"),
                cpu_cores_per_socket=info.get("cpu cores"), cpu_siblings=info.get("siblings"),
                cpu_cache=info.get("cache size"), host_cpus=os.cpu_count(),
                threads=int(used), build="gcc -O2 -fopenmp, FP64, OpenMP across the sites of one subset")


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=None, help="timed sweeps (default: the workload's)")
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="c4", choices=sorted(WORKLOADS))
    ap.add_argument("--precision", default="both", choices=["fp64", "fp32_bulk", "both"])
    ap.add_argument("--pass-sweeps", type=int, default=4, help="sweeps timed pass by pass for the roofline")
    ap.add_argument("--cpu-threads", type=int, default=0)
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the MaxReTr, APE and flow legs")
    ap.add_argument("--serving-jobs", type=int, default=200, help="jobs of the serving stream (0: skip)")
    ap.add_argument("--serving-rate", type=float, default=50.0, help="mean arrivals per second")
    ap.add_argument("--serving-slots", type=int, default=64, help="jobs resident at once")
    ap.add_argument("--no-serving-curve", action="store_true", help="skip the latency-versus-load replays")
    ap.add_argument("--copy-calibration", type=int, default=0, metavar="MIB",
                    help="only run 5 plain device copies of MIB mebibytes (counter calibration), then 5 "
                         "reads, and print their rates")
    args = ap.parse_args()
    if args.copy_calibration > 0:
        import torch

        nb = args.copy_calibration << 20
        a = torch.empty(nb, dtype=torch.uint8, device="cuda:0")
        b = torch.empty(nb, dtype=torch.uint8, device="cuda:0")
        a.fill_(1)
        b.copy_(a)  # warm-up: the first copy and the first sum load their kernels
        a.view(torch.float64).sum()
        torch.cuda.synchronize()
        stream = torch.cuda.current_stream()
        e0, e1, e2 = (torch.cuda.Event(enable_timing=True) for _ in range(3))
        e0.record(stream)
        for _ in range(5):
            b.copy_(a)
        e1.record(stream)
        # a plain streaming read of the same bytes, for the practical HBM read rate
        for _ in range(5):
            a.view(torch.float64).sum()
        e2.record(stream)
        torch.cuda.synchronize()
        copy_ms, read_ms = e0.elapsed_time(e1) / 5, e1.elapsed_time(e2) / 5
        print(json.dumps({"copy_calibration_bytes": nb, "copies": 5,
                          "copy_gb_per_s": round(2 * nb / (copy_ms * 1e-3) / 1e9, 1),
                          "read_gb_per_s": round(nb / (read_ms * 1e-3) / 1e9, 1)}))
        return
    if args.gpus != 1:
        print(json.dumps({"error": "this build runs on one GPU only; --gpus must be 1"}))
        sys.exit(2)
    import fieldgen

    cfg = fieldgen.CONFIGS[args.workload]
    if args.steps is None:
        args.steps = cfg["n_sweeps"]
    dims = cfg["dims"]
    n = fieldgen.z3_vortex_charges(dims, cfg["p"], cfg["field_seed"])
    pairs = fieldgen.centrifuge_pairs(dims, cfg["pair_seed"])
    forms = ["fp64", "fp32_bulk"] if args.precision == "both" else [args.precision]
    res = {p: run_gpu_form(args, p, dims, n, pairs) for p in forms}
    head = res["fp64"] if "fp64" in res else res[forms[0]]
    hp = head["precision"]
    traffic = load_traffic(args.workload, hp, head["pass_launch_lu"])
    read_gbs = stream_read_gbs()
    roof = {"bound": "hbm", "achieved": round(head["achieved_gbs"], 1), "peak": HBM_PEAK_GBS,
            "unit": "GB/s", "frac": round(head["achieved_gbs"] / HBM_PEAK_GBS, 4),
            "traffic": traffic,
            "kernel": f"k_update annealed OI stout pass ({hp})",
            "algorithmic_bytes_per_launch": head["pass_algo_bytes"],
            "algorithmic_bytes_per_lu": pass_bytes_per_lu(hp),
            "stored_bytes_per_lu": pass_bytes_per_lu(hp, stored=True),
            "frac_stored_bytes": round(head["achieved_stored_gbs"] / HBM_PEAK_GBS, 4),
            "avg_launch_ms": round(head["avg_pass_ms"], 4),
            "stream_read_gbs": round(read_gbs, 1),
            "frac_of_stream_read": round(head["achieved_gbs"] / read_gbs, 4)}
    out = {
        "metric": "SU(3) link-updates/s per sweep, % HBM roofline; p50/p99 smoothing-job latency",
        "value": round(head["lu_per_s"], 1),
        "unit": "link-updates/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(head["ms_per_step"], 4),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64" if hp == "fp64" else "f32",
        "data": "synthetic",
        "config": {"workload": f"{args.workload}: {WORKLOADS[args.workload]}", "lattice": list(dims),
                   "sweeps": args.steps, "precision": hp},
        "roofline": roof,
    }
    forms_out = {}
    for p, r in res.items():
        forms_out[p] = {"lu_per_s": round(r["lu_per_s"], 1), "ms_per_step": round(r["ms_per_step"], 4),
                        "avg_pass_ms": round(r["avg_pass_ms"], 4),
                        "hbm_frac": round(r["achieved_gbs"] / HBM_PEAK_GBS, 4),
                        "hbm_frac_stored_bytes": round(r["achieved_stored_gbs"] / HBM_PEAK_GBS, 4),
                        "flux_mismatch": r["flux_mismatch"], "nonfinite": r["nonfinite"],
                        "max_unitarity": r["max_unitarity"], "final_action": r["action"][-1],
                        "clover_measure": r["clover"]}
    if "fp64" in res and "fp32_bulk" in res:
        a64, a32 = res["fp64"]["action"], res["fp32_bulk"]["action"]
        forms_out["fp32_bulk"]["speedup_vs_fp64"] = round(res["fp32_bulk"]["lu_per_s"] / res["fp64"]["lu_per_s"], 3)
        forms_out["fp32_bulk"]["max_rel_action_dev_vs_fp64"] = max(abs(x - y) / abs(y) for x, y in zip(a32, a64))
    for p in ([] if args.no_forms else forms):
        for upd in ("maxretr", "ape"):
            forms_out[p + "_" + upd] = update_form(dims, n, pairs, p, upd)
        forms_out[p + "_flow_rk3"] = flow_form(dims, n, pairs, p)
    out["forms"] = forms_out
    if args.serving_jobs > 0:
        out["serving"] = serving_leg(args.serving_jobs, args.serving_rate, args.serving_slots,
                                     loads=() if args.no_serving_curve else ((0.5, 120), (0.8, 150), (1.0, 150)))
    if not args.no_cpu:
        out["cpu_baseline"] = cpu_baseline(dims, n, pairs, args.cpu_threads)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
