"""Serving loop over the library's continuous-batching server.

Jobs (one protein family each) arrive on a Poisson clock; each is submitted
when its arrival time passes, admitted by the server when its device
footprint fits the budget, and batched with every other admitted job on each
scheduler step.  Latency is arrival -> last tile delivered.  All computation
is in the HIP library; this module only keeps the clock and the books.
"""
from __future__ import annotations

import ctypes
import time
from typing import Callable, Dict, List, Optional

import numpy as np

from . import binding as B
from . import inputs

# Arrival rate for the c5 serving workload, in jobs per second: 0.7 x the
# saturated job throughput measured on one MI355X (the 200-job c5 mix replayed
# at once: 2.95 s, 67.8 jobs/s).
C5_RATE_PER_S = 47.5


class Server:
    def __init__(self, **opts):
        self.options = B.make_options(**opts)
        h = ctypes.c_void_p()
        B.check(B.lib().famsa_lcs_server_create(ctypes.byref(self.options), ctypes.byref(h)))
        self.handle = h
        self._keep = {}

    def submit(self, codes: np.ndarray, seq_off: np.ndarray) -> int:
        codes = np.ascontiguousarray(codes, np.uint8)
        off = np.ascontiguousarray(seq_off, np.uint64)
        jid = ctypes.c_uint32()
        B.check(B.lib().famsa_lcs_server_submit(
            self.handle, codes.ctypes.data_as(ctypes.POINTER(ctypes.c_uint8)) if codes.size else None,
            off.ctypes.data_as(ctypes.POINTER(ctypes.c_uint64)), off.size - 1, ctypes.byref(jid)))
        return int(jid.value)

    def step(self, fn: Optional[Callable] = None) -> int:
        """One scheduler step; fn(tile) receives delivered host tiles.  Returns jobs not yet done."""
        err = []

        def cb(_u, tp):
            try:
                return int(fn(tp.contents) or 0) if fn else 0
            except BaseException as e:
                err.append(e)
                return 1

        c = B.TILE_FN(cb)
        active = ctypes.c_uint32()
        rc = B.lib().famsa_lcs_server_step(self.handle, c, None, ctypes.byref(active))
        if err:
            raise err[0]
        B.check(rc)
        return int(active.value)

    def job_state(self, jid: int) -> int:
        s = ctypes.c_int()
        B.check(B.lib().famsa_lcs_server_job_state(self.handle, jid, ctypes.byref(s)))
        return int(s.value)

    def memory(self):
        a, p = ctypes.c_uint64(), ctypes.c_uint64()
        B.check(B.lib().famsa_lcs_server_memory(self.handle, ctypes.byref(a), ctypes.byref(p)))
        return int(a.value), int(p.value)

    def close(self):
        if getattr(self, "handle", None):
            B.lib().famsa_lcs_server_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


def run_jobs(jobs: List[inputs.ServeJob], on_tile: Optional[Callable] = None, realtime: bool = True,
             **server_opts) -> Dict:
    """Replay `jobs` against a server; returns latencies and throughput."""
    srv = Server(**server_opts)
    n = len(jobs)
    order = sorted(range(n), key=lambda i: jobs[i].arrival_s)
    ids: Dict[int, int] = {}
    rows_left: Dict[int, int] = {}  # a job's tiles cover its rows; it is done when all have come
    done_t: Dict[int, float] = {}
    submit_t: Dict[int, float] = {}
    step_jobs: List[set] = []  # job ids whose tiles each step call delivered

    def fn(t):
        j = int(t.family)
        step_jobs[-1].add(j)
        if on_tile:
            on_tile(j, t)
        rows_left[j] -= int(t.row_end) - int(t.row_begin)
        if rows_left[j] == 0:
            done_t[j] = time.perf_counter()
        return 0

    t0 = time.perf_counter()
    nxt = 0
    active = 0
    while nxt < n or active:
        now = time.perf_counter() - t0
        submitted = 0
        while nxt < n and (not realtime or jobs[order[nxt]].arrival_s <= now):
            i = order[nxt]
            b = jobs[i].batch
            jid = srv.submit(b.codes, b.seq_off)
            ids[jid] = i
            rows_left[jid] = b.nseq
            submit_t[jid] = t0 + (jobs[i].arrival_s if realtime else 0.0)
            if rows_left[jid] == 0:
                done_t[jid] = time.perf_counter()
            nxt += 1
            submitted += 1
        if nxt < n and active == 0 and not submitted and realtime:
            # nothing to run: wait for the next arrival (a job submitted just
            # now is stepped at once, not after this wait)
            wait = jobs[order[nxt]].arrival_s - (time.perf_counter() - t0)
            if wait > 0:
                time.sleep(min(wait, 0.05))
            continue
        step_jobs.append(set())
        active = srv.step(fn)
    wall = time.perf_counter() - t0
    mem = srv.memory()
    srv.close()
    lat = np.array([1e3 * (done_t[j] - submit_t[j]) for j in sorted(done_t)])
    pairs = sum(jobs[i].batch.pairs() for i in range(n))
    cells = sum(jobs[i].batch.cells() for i in range(n))
    return {"jobs": n, "wall_s": round(wall, 3), "pairs_per_s": round(pairs / wall, 1),
            "gcups": round(cells / wall / 1e9, 1), "p50_ms": round(float(np.percentile(lat, 50)), 2),
            "p99_ms": round(float(np.percentile(lat, 99)), 2), "max_ms": round(float(lat.max()), 2),
            "peak_device_bytes": mem[1], "latencies_ms": lat, "job_ids": ids,
            "max_jobs_per_step": max((len(x) for x in step_jobs), default=0), "step_jobs": step_jobs}


# Serving steps are kept small so that a new job waits for little work ahead of
# it: at most 2^24 values (64 MiB per buffer) and 2^41 cells (about 4 ms of
# device time) per step, and tiles of at most 256 rows and 2^41 cells, which
# hold families of up to ~65,000 sequences.  A job arriving while step s runs
# joins step s + 2 (step s + 1 is already issued), so its wait is about two
# steps.  On the c5 mix (200 jobs at the frozen rate) 2^40-cell steps give a
# median latency of 6.3 ms but a p99 of 511 ms and 10% less capacity; 2^41
# gives 8.9 ms and 386 ms; 2^42 gives 14 ms and 292 ms and 7% more capacity.
SERVE_STEP_VALUES = 1 << 24
SERVE_STEP_CELLS = 1 << 41
SERVE_TILE_ROWS = 256


def alone_ms(jobs: List[inputs.ServeJob], **server_opts) -> np.ndarray:
    """Each job's service time when it has the server to itself: submitted
    to an idle server, stepped until its last tile is delivered (ms)."""
    srv = Server(**server_opts)
    out = np.zeros(len(jobs))
    try:
        for i, job in enumerate(jobs):
            t0 = time.perf_counter()
            srv.submit(job.batch.codes, job.batch.seq_off)
            while srv.step(None):
                pass
            out[i] = 1e3 * (time.perf_counter() - t0)
    finally:
        srv.close()
    return out


def _summary(r: Dict) -> Dict:
    return {k: r[k] for k in ("jobs", "wall_s", "pairs_per_s", "gcups", "p50_ms", "p99_ms", "max_ms",
                              "max_jobs_per_step")}


def run_c5_bench(njobs: int = 200, rate: float = C5_RATE_PER_S, seed: int = 4, loads=(0.5, 0.7, 0.9),
                 workers: int = 16) -> Dict:
    """The serving workload: `njobs` jobs at the frozen arrival rate, the same
    jobs replayed at once (saturated: the capacity in jobs/s), and at each of
    `loads` times that capacity (arrival times rescaled)."""
    import dataclasses
    import os
    try:
        workers = max(1, min(workers, len(os.sched_getaffinity(0))))
    except AttributeError:
        workers = 1
    jobs = inputs.c5(seed=seed, njobs=njobs, rate_per_s=rate, workers=workers)
    opts = dict(step_values=SERVE_STEP_VALUES, step_cells=SERVE_STEP_CELLS, tile_rows=SERVE_TILE_ROWS)
    sat = run_jobs(jobs, realtime=False, **opts)
    capacity = njobs / sat["wall_s"]
    r = run_jobs(jobs, **opts)
    lat = r.pop("latencies_ms")
    ids = r.pop("job_ids")
    r.pop("step_jobs")
    # latency over the job's own service time alone: job cost spans orders of
    # magnitude, so this says how much waiting the mix added to each job
    alone = alone_ms(jobs, **opts)
    slow = np.array([lat[n] / alone[ids[jid]] for n, jid in enumerate(sorted(ids))])
    r["slowdown_p50"] = round(float(np.percentile(slow, 50)), 2)
    r["slowdown_p99"] = round(float(np.percentile(slow, 99)), 2)
    r["alone_ms_sum"] = round(float(alone.sum()), 1)
    r["workload"] = (f"c5: {njobs} jobs, Poisson arrivals at {rate} jobs/s, each a tree-evolved family with k "
                     f"log-uniform [100,20000] and root length log-uniform [50,1500], seed {seed}")
    r["arrival_rate_per_s"] = rate
    r["saturated"] = dict(_summary(sat), capacity_jobs_per_s=round(capacity, 2))
    r["load_sweep"] = {}
    for load in loads:
        lam = load * capacity
        scaled = [dataclasses.replace(j, arrival_s=j.arrival_s * rate / lam) for j in jobs]
        x = run_jobs(scaled, **opts)
        r["load_sweep"][str(load)] = dict(_summary(x), arrival_rate_per_s=round(lam, 2))
    r["frozen_rate_load"] = round(rate / capacity, 3)
    r["step_values"] = SERVE_STEP_VALUES
    r["step_cells"] = SERVE_STEP_CELLS
    r["tile_rows"] = SERVE_TILE_ROWS
    return r
