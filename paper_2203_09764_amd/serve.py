"""Serving binding: argument marshalling for the vsm_server_* calls of
include/vsm.h, and a driver that replays a timed stream of jobs against a
server and reports latency percentiles and throughput.

The server owns its device and pinned host pools and its worker thread (all in
libvsm.so); jobs are handed over as host numpy arrays and come back as host
numpy arrays, so this module needs no torch.
"""
from __future__ import annotations

import ctypes
import time

import numpy as np

from ._lib import (ANNEALED, FP32_BULK, FP64, STATS_DTYPE, STOUT,
                   Job, JobInfo, Schedule, ServerConfig, ServerCounters, VsmError, check, lib)

PRECISIONS = {"fp64": FP64, "fp32_bulk": FP32_BULK, "fp32": FP32_BULK, FP64: FP64, FP32_BULK: FP32_BULK}
STATE_NAMES = {0: "queued", 1: "running", 2: "done", 3: "failed"}


def _info_dict(info: JobInfo) -> dict:
    return dict(state=STATE_NAMES.get(info.state, str(info.state)), status=int(info.status),
                n_records=int(info.n_records), sweeps_done=int(info.sweeps_done),
                t_submit=float(info.t_submit), t_admit=float(info.t_admit), t_done=float(info.t_done),
                footprint_bytes=int(info.footprint_bytes))


def _int8_host(a, V: int, what: str) -> np.ndarray:
    a = np.ascontiguousarray(np.asarray(a, dtype=np.int8))
    if a.size != 4 * V:
        raise ValueError(f"{what} must hold 4*V = {4 * V} int8 values, got {a.size}")
    return a


class Server:
    """A smoothing server on one GPU (see vsm_server_create)."""

    def __init__(self, hbm_budget_bytes: int = 8 << 30, host_budget_bytes: int = 1 << 30, max_slots: int = 32,
                 max_inflight: int = 4, device: int = 0):
        self._cfg = ServerConfig(int(hbm_budget_bytes), int(host_budget_bytes), int(max_slots),
                                 int(max_inflight), int(device), 0)
        h = ctypes.c_void_p()
        check(lib().vsm_server_create(ctypes.byref(self._cfg), ctypes.byref(h)), "vsm_server_create")
        self._h = h
        self._meta: dict = {}

    # -- job description
    @staticmethod
    def job_struct(dims, z3, *, pairs=None, omega=0.02, n_sweeps=100, rho=0.06, eps=-0.25,
                   precision="fp32_bulk", vp=True, u0=1.0, measure_every=0, want_links=False):
        """The vsm_job for these arguments, plus the host arrays it points into
        (kept alive by the caller until submit returns)."""
        d = [int(v) for v in dims]
        V = d[0] * d[1] * d[2] * d[3]
        z = _int8_host(z3, V, "z3")
        pr = _int8_host(pairs, V, "pairs") if pairs is not None else None
        sched = Schedule(ANNEALED, STOUT, 1 if vp else 0, 3, float(u0), 1.0)
        j = Job((ctypes.c_int32 * 4)(*d), PRECISIONS[precision], int(n_sweeps), float(rho), float(eps),
                float(omega), sched, int(measure_every), 1 if want_links else 0,
                ctypes.c_void_p(z.ctypes.data), ctypes.c_void_p(pr.ctypes.data) if pr is not None else None)
        return j, (z, pr)

    def job_bytes(self, dims, **kw) -> int:
        d = [int(v) for v in dims]
        V = d[0] * d[1] * d[2] * d[3]
        j, keep = self.job_struct(dims, np.zeros(4 * V, np.int8), **kw)
        return int(lib().vsm_server_job_bytes(ctypes.byref(j)))

    def submit(self, dims, z3, **kw) -> int:
        j, keep = self.job_struct(dims, z3, **kw)
        jid = ctypes.c_uint64()
        check(lib().vsm_server_submit(self._h, ctypes.byref(j), ctypes.byref(jid)), "vsm_server_submit")
        me = int(kw.get("measure_every", 0))
        ns = int(kw.get("n_sweeps", 100))
        nrec = 1 if me <= 0 else ns // me + (1 if ns % me else 0)
        self._meta[jid.value] = (tuple(int(v) for v in dims), nrec, bool(kw.get("want_links", False)))
        return int(jid.value)

    def poll(self, job_id: int) -> dict:
        info = JobInfo()
        check(lib().vsm_server_poll(self._h, ctypes.c_uint64(job_id), ctypes.byref(info)), "vsm_server_poll")
        return _info_dict(info)

    def wait(self, job_id: int, timeout: float | None = None) -> dict:
        """Info of the job once DONE or FAILED; raises VsmError(E_TIMEOUT) on timeout."""
        info = JobInfo()
        st = lib().vsm_server_wait(self._h, ctypes.c_uint64(job_id), -1.0 if timeout is None else float(timeout),
                                   ctypes.byref(info))
        check(st, "vsm_server_wait")
        return _info_dict(info)

    def fetch(self, job_id: int):
        """(records recarray, links complex128 [4][V][3][3] or None) of a DONE job;
        the server forgets the job."""
        dims, nrec, want = self._meta[job_id]
        V = dims[0] * dims[1] * dims[2] * dims[3]
        rec = np.zeros(nrec, dtype=STATS_DTYPE)
        links = np.empty((4, V, 3, 3), dtype=np.complex128) if want else None
        st = lib().vsm_server_fetch(self._h, ctypes.c_uint64(job_id), ctypes.c_void_p(rec.ctypes.data), nrec,
                                    ctypes.c_void_p(links.ctypes.data) if want else None)
        check(st, "vsm_server_fetch")
        del self._meta[job_id]
        return rec.view(np.recarray), links

    def clock(self) -> float:
        return float(lib().vsm_server_clock(self._h))

    def counters(self) -> dict:
        c = ServerCounters()
        check(lib().vsm_server_get_counters(self._h, ctypes.byref(c)), "vsm_server_get_counters")
        return {name: getattr(c, name) for name, _ in ServerCounters._fields_}

    def close(self) -> None:
        if self._h is not None and self._h.value:
            check(lib().vsm_server_destroy(self._h), "vsm_server_destroy")
        self._h = None

    def __enter__(self):
        return self

    def __exit__(self, *exc):
        self.close()

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_stream(server: Server, jobs, *, time_scale: float = 1.0, timeout: float = 600.0, **job_kw) -> dict:
    """Replays `jobs` against `server`: job k is submitted at arrival_s * time_scale
    seconds after the start.  Each element of `jobs` is (arrival_s, dims, z3,
    pairs, n_sweeps); job_kw go to every submit.  Returns per-job latencies
    (t_done - t_submit on the server clock), their p50/p99, the queueing
    delays, and link-updates/s over the span from the first submit to the last
    completion."""
    jobs = sorted(jobs, key=lambda j: j[0])
    ids = []
    lu = 0
    t_start = time.perf_counter()
    for arrival, dims, z3, pairs, n_sweeps in jobs:
        delay = arrival * time_scale - (time.perf_counter() - t_start)
        if delay > 0:
            time.sleep(delay)
        ids.append(server.submit(dims, z3, pairs=pairs, n_sweeps=n_sweeps, **job_kw))
        V = int(np.prod(dims))
        lu += 4 * V * int(n_sweeps)
    infos, records = [], []
    for jid in ids:
        info = server.wait(jid, timeout)
        if info["state"] != "done":
            raise VsmError(info["status"], f"job {jid} {info['state']}")
        rec, _ = server.fetch(jid)
        infos.append(info)
        records.append(rec)
    lat = np.array([i["t_done"] - i["t_submit"] for i in infos])
    queue = np.array([i["t_admit"] - i["t_submit"] for i in infos])
    span = max(i["t_done"] for i in infos) - min(i["t_submit"] for i in infos)
    return dict(n_jobs=len(ids), latency_s=lat, queue_s=queue, p50_s=float(np.percentile(lat, 50)),
                p99_s=float(np.percentile(lat, 99)), mean_queue_s=float(queue.mean()), span_s=float(span),
                link_updates=int(lu), lu_per_s=float(lu / span) if span > 0 else float("nan"),
                records=records, counters=server.counters())
