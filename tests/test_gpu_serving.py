"""GPU tests of the serving scheduler (continuous batching of smoothing jobs).

Bars: a job's links and records are bit-identical whether it runs alone or in
a mix of other jobs (the same per-link code runs either way and every
reduction is per job, in a fixed order); the served links equal those of the
single-field path (vsm_smooth) bit for bit, and its records within the parity
tolerance of each precision;
admission never exceeds the memory budget, and vortex charges stay preserved.
"""
import numpy as np
import pytest
import torch

import fieldgen
from paper_2203_09764_amd import api, serve
from paper_2203_09764_amd._lib import E_BUDGET, VsmError

pytestmark = pytest.mark.gpu

KW = dict(rho=0.06, eps=-0.25, vp=True, omega=0.02)

# (dims, precision, n_sweeps, field seed); extents all multiples of 4
JOBS = [
    ((8, 8, 8, 8), "fp32_bulk", 6, 11),
    ((12, 12, 12, 24), "fp32_bulk", 4, 12),
    ((8, 8, 8, 16), "fp64", 5, 13),
    ((16, 16, 16, 32), "fp32_bulk", 3, 14),
    ((4, 8, 12, 16), "fp64", 7, 15),
]


def _inputs(dims, seed, p=0.1):
    return fieldgen.z3_vortex_charges(dims, p, seed), fieldgen.centrifuge_pairs(dims, seed + 100)


def _submit(srv, job, measure_every=2):
    dims, prec, ns, seed = job
    n, pairs = _inputs(dims, seed)
    return srv.submit(dims, n, pairs=pairs, n_sweeps=ns, precision=prec, measure_every=measure_every,
                      want_links=True, **KW)


def _run_alone(srv, job, measure_every=2):
    jid = _submit(srv, job, measure_every)
    info = srv.wait(jid, 120)
    assert info["state"] == "done", info
    return srv.fetch(jid)


def _same(a, b):
    ra, la = a
    rb, lb = b
    return ra.tobytes() == rb.tobytes() and la.tobytes() == lb.tobytes()


@pytest.fixture(scope="module")
def server():
    with serve.Server(hbm_budget_bytes=2 << 30, host_budget_bytes=512 << 20, max_slots=32, max_inflight=4) as s:
        yield s


@pytest.fixture(scope="module")
def alone(server):
    return [_run_alone(server, j) for j in JOBS]


def test_alone_results_are_sane(alone):
    for (dims, prec, ns, _), (rec, links) in zip(JOBS, alone):
        assert len(rec) == ns // 2 + (ns % 2)
        assert rec.sweep[-1] == ns
        assert np.all(rec.flux_mismatch == 0) and np.all(rec.nonfinite == 0)
        assert np.all(np.diff(rec.action) < 0)  # over-improved stout lowers the action here
        V = int(np.prod(dims))
        assert links.shape == (4, V, 3, 3)
        uu = np.einsum("dsji,dsjk->dsik", links.conj(), links)
        assert np.abs(uu - np.eye(3)).max() < (1e-13 if prec == "fp64" else 2e-6)


def test_mix_is_bit_identical_to_alone(server, alone):
    """All five jobs submitted together (two precisions, five lattice sizes)."""
    ids = [_submit(server, j) for j in JOBS]
    got = []
    for jid in ids:
        assert server.wait(jid, 120)["state"] == "done"
        got.append(server.fetch(jid))
    for j, a, g in zip(JOBS, alone, got):
        assert _same(a, g), f"job {j} differs between alone and mixed"


def test_staggered_arrivals_are_bit_identical(server, alone):
    """Jobs join while others are mid-run (continuous batching)."""
    import time

    ids = []
    for j in JOBS[::-1]:
        ids.append(_submit(server, j))
        time.sleep(0.003)
    got = {}
    for jid in ids:
        assert server.wait(jid, 120)["state"] == "done"
        got[jid] = server.fetch(jid)
    for k, j in enumerate(JOBS[::-1]):
        assert _same(alone[len(JOBS) - 1 - k], got[ids[k]]), f"job {j} differs when staggered"


def test_more_jobs_than_one_launch_holds():
    """130 resident small jobs: a small-lattice step then spans two launches (at
    most 128 jobs each), and every job still gets the result it gets alone."""
    dims, prec, ns, seed = (8, 8, 8, 8), "fp32_bulk", 40, 21
    n, pairs = _inputs(dims, seed)
    kw = dict(pairs=pairs, n_sweeps=ns, precision=prec, measure_every=4, want_links=True, **KW)
    with serve.Server(hbm_budget_bytes=1 << 30, host_budget_bytes=512 << 20, max_slots=140) as srv:
        ref_id = srv.submit(dims, n, **kw)
        assert srv.wait(ref_id, 120)["state"] == "done"
        ref = srv.fetch(ref_id)
        ids = [srv.submit(dims, n, **kw) for _ in range(130)]
        for jid in ids:
            assert srv.wait(jid, 120)["state"] == "done"
            assert _same(ref, srv.fetch(jid))
        c = srv.counters()
    assert c["peak_resident_jobs"] > 128


def test_small_lattices_run_whole_sweeps_per_launch():
    """Lattices of at most 8192 sites are served by the persistent small-lattice
    path: one workgroup per job runs all 16 passes of several sweeps (8 sweeps
    of an 8^4 lattice per step), so four 8^4 jobs of 40 sweeps take a handful
    of launches instead of one per subset pass (640 steps in pass-by-pass
    batching), with the same links as the single-field path."""
    dims, prec, ns = (8, 8, 8, 8), "fp64", 40
    with serve.Server(hbm_budget_bytes=1 << 30, host_budget_bytes=256 << 20, max_slots=8) as srv:
        ids = []
        for k in range(4):
            n, pairs = _inputs(dims, 31 + k)
            ids.append(srv.submit(dims, n, pairs=pairs, n_sweeps=ns, precision=prec, measure_every=0,
                                  want_links=True, **KW))
        got = []
        for jid in ids:
            assert srv.wait(jid, 120)["state"] == "done"
            got.append(srv.fetch(jid))
        c = srv.counters()
    print(f"4 jobs x {ns} sweeps of 8^4: {c['steps']} steps, {c['launches']} launches")
    # admission (3 launches), final measurement and link read-back (2) per job, plus the steps
    assert c["steps"] <= 2 * ns // 8
    assert c["launches"] <= 4 * 5 + 2 * ns // 8
    for k, (rec, links) in enumerate(got):
        n, pairs = _inputs(dims, 31 + k)
        f = api.Field(dims, prec, device=torch.device("cuda:0"), jacobi_workspace=False)
        f.set_charges(n)
        api.precondition(f, pairs, KW["omega"])
        api.smooth(f, ns, KW["rho"], KW["eps"], order="annealed", vp=True)
        # the same per-link arithmetic, whether the LDS ring or ordinary loads
        # bring the links in: the links agree bit for bit
        assert np.array_equal(api.get_links(f).cpu().numpy(), links)
        assert rec.flux_mismatch[-1] == 0


def test_served_equals_single_field_path(alone):
    """The same job through vsm_precondition + vsm_smooth on a torch stream."""
    for job, (rec, links) in zip(JOBS, alone):
        dims, prec, ns, seed = job
        n, pairs = _inputs(dims, seed)
        f = api.Field(dims, prec, device=torch.device("cuda:0"), jacobi_workspace=False)
        f.set_charges(n)
        api.precondition(f, pairs, KW["omega"])
        st = api.new_stats(ns // 2, f.device)
        api.smooth(f, ns, KW["rho"], KW["eps"], order="annealed", vp=True, measure_every=2, stats=st)
        want = api.stats_to_numpy(st, ns // 2)
        final = api.stats_to_numpy(api.measure(f), 1)[0]
        got_links = api.get_links(f).cpu().numpy()
        torch.cuda.synchronize()
        tol = 1e-12 if prec == "fp64" else 2e-6
        assert np.array_equal(got_links, links)  # the same per-link code: bit for bit
        k = ns // 2
        np.testing.assert_allclose(rec.action[:k], want.action, rtol=tol)
        np.testing.assert_allclose(rec.plaq[-1], final.plaq, rtol=tol)
        if prec == "fp64":
            np.testing.assert_array_equal(rec.rejected[:k], want.rejected)
        np.testing.assert_array_equal(rec.flux_mismatch[:k], want.flux_mismatch)


def test_admission_respects_the_budget(alone):
    """A pool that holds one 16^3x32 job at a time runs three of them one after
    another, each with its alone result."""
    big = JOBS[3]
    probe = serve.Server(hbm_budget_bytes=64 << 20, host_budget_bytes=64 << 20, max_slots=4)
    need = probe.job_bytes(big[0], n_sweeps=big[2], precision=big[1], measure_every=2, want_links=True)
    probe.close()
    with serve.Server(hbm_budget_bytes=need + need // 2, host_budget_bytes=256 << 20, max_slots=4) as s:
        ids = [_submit(s, big) for _ in range(3)]
        infos = [s.wait(jid, 120) for jid in ids]
        for jid in ids:
            assert _same(alone[3], s.fetch(jid))
        for a, b in zip(infos, infos[1:]):
            assert b["t_admit"] >= a["t_done"]  # admitted only once the previous job left
        c = s.counters()
        assert c["peak_resident_jobs"] == 1
        assert c["peak_pool_bytes"] <= need + need // 2
        with pytest.raises(VsmError) as e:
            s.submit((32, 32, 32, 64), np.zeros(4 * 32 ** 3 * 64, np.int8), n_sweeps=1)
        assert e.value.status == E_BUDGET
        with pytest.raises(VsmError) as e:
            s.submit((8, 8, 8, 6), np.zeros(4 * 8 ** 3 * 6, np.int8), n_sweeps=1)
        assert e.value.status != 0


def test_poisson_stream_reports_latency():
    """A short Poisson stream of the serving mix (sweeps cut to 10-30)."""
    specs = fieldgen.poisson_jobs(12, 200.0, seed=7, sweeps_range=(10, 30))
    jobs = []
    for sp in specs:
        n = fieldgen.z3_vortex_charges(sp.dims, sp.p, sp.field_seed)
        pairs = fieldgen.centrifuge_pairs(sp.dims, sp.pair_seed)
        jobs.append((sp.arrival_s, sp.dims, n, pairs, sp.n_sweeps))
    with serve.Server(hbm_budget_bytes=1 << 30, host_budget_bytes=256 << 20, max_slots=16) as s:
        r = serve.run_stream(s, jobs, precision="fp32_bulk", measure_every=0, timeout=120, **KW)
    assert r["n_jobs"] == 12
    assert 0 < r["p50_s"] <= r["p99_s"] < 60
    assert all(int(rec.flux_mismatch[-1]) == 0 for rec in r["records"])
    assert r["lu_per_s"] > 0
    assert r["counters"]["jobs_done"] == 12
