"""Benchmark of the all-pairs LCS similarity stage on one MI355X.

    python bench.py [--gpus 1] [--steps K] [--warmup W] [--workload c4|c2|c1]
                    [--no-c3] [--no-serve] [--no-cpu] [--no-extra]

One step = one full pass of the stage over the workload: every row tile of
the family computed on the GPU (masks resident in HBM; the plan is built and
tuned before the timed region) and copied to pinned host memory, where the
tile callback receives it.  `value` is GCUPS = sum over pairs of |A||B|
divided by the wall time of a step.  The timed steps run on one compute
stream, so no two launches overlap and each launch's event-timed duration is
the kernel's own.  Also reported, in the same JSON line:

* roofline: the dominant LCS kernel's integer-ALU throughput (3 VALU ops
  per 32 cells: AND, ADD-with-carry, the three-input OR/AND-NOT) against
  gfx950's 256 CUs x 128 lanes x 2.4 GHz, from HIP events around each launch
  on its stream during the timed steps; `traffic` is that kernel's HBM bytes
  per launch from the committed rocprofv3 counter summary when it was taken
  from the current kernel source and this configuration, else null;
* graph_replay: the same pass as the library runs it by default, steps
  replayed as captured hipGraphs on one compute stream;
* two_streams: graph replays with consecutive steps alternating between two
  compute streams, so one step's tail overlaps the next step;
* plain: one pass of the plain baseline kernel over the same workload (one
  pair per lane, one launch per tile), and the batched form's speed-up;
* similarity_tiles: the same pass delivering float32 similarities instead of
  LCS values (the kernels' epilogue computes them);
* gpu_single_linkage: the pass with device tiles feeding the GPU exact
  single-linkage consumer (maximum spanning tree of the similarities), and
  the time to turn its tree into the guide tree's merge list;
* host_slink: the host SLINK consumer's update rate on c2;
* gapped: the gapped sequence representation over the workload's sequences
  (one profile-wide round of gap runs inserted into every sequence, every
  row decoded to host memory);
* cpu_baseline: the CPU oracle (plain DP) on a bounded sample of the same
  workload's pairs, on the host's cores, and its single-thread rate on 10^4
  of those pairs and on every pair of c1;
* c3: batched (persistent, graph-replayed) vs plain (one launch per tile,
  each waiting for the previous tile's delivery) and plain_async (the same
  launches without the waits); median of 5 passes each;
* serve: continuous-batching jobs, pairs/s and p50/p99 latency.
"""
from __future__ import annotations

import argparse
import json
import multiprocessing as mp
import os
import sys
import time

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, HERE)

METRIC = "GCUPS for all-pairs bit-parallel LCS (k=100k), batched vs plain; serve p99 ms"
# int32 VALU lane-ops/s of MI355X: 256 CUs x 128 lanes/clk x 2.4 GHz, the
# fp32-vector lane rate (157.3 TFLOP/s / 2 flops per FMA); the measured VALU
# instruction rate of the LCS kernels exceeds 64 lanes/clk/CU, so 64 is not
# the ceiling.
PEAK_INT_OPS = 256 * 128 * 2.4e9
OPS_PER_CELL = 3.0 / 32.0             # AND + ADDC + BITOP3 per 32-cell dword-step
STEP_VALUES = 1 << 28                 # int32 results per launch step (1 GiB per buffer)
CPU_SHARE = 16                        # host cores a one-GPU machine grants a job
TRAFFIC_SUMMARY = os.path.join(HERE, "profiles", "lcs_fast_c4_hbm_traffic.txt")
# the kernels and the constants that shape them (class bounds, LDS layout)
KERNEL_SOURCES = [os.path.join(HERE, "paper_1603_06958_amd", "csrc", f) for f in ("lcs_kernels.hip", "lcs_common.h")]


def _oracle_worker(args):
    codes, off, ia, ib = args
    import oracle
    t0 = time.perf_counter()
    oracle.lcs_pairs(codes, off, ia, ib)
    return time.perf_counter() - t0


def cpu_baseline(b, seconds_target=12.0, seed=7):
    """The oracle on a seeded sample of the workload's pairs, one process per core."""
    import oracle
    rng = np.random.default_rng(seed)
    L = b.lengths().astype(np.int64)
    k = b.nseq
    # calibrate on a small sample (single core)
    ia = rng.integers(0, k, 200)
    ib = rng.integers(0, k, 200)
    t0 = time.perf_counter()
    oracle.lcs_pairs(b.codes, b.seq_off, ia, ib)
    dt = time.perf_counter() - t0
    rate1 = float((L[ia] * L[ib]).sum()) / max(dt, 1e-9)
    try:
        visible = len(os.sched_getaffinity(0))
    except AttributeError:
        visible = os.cpu_count() or 1
    # the GPU machine's CPU share is 16 cores, whatever the affinity mask shows:
    # one single-threaded worker process per core of that share
    cores = max(1, min(visible, CPU_SHARE))
    per_worker_cells = rate1 * seconds_target
    mean_cells = float((L.mean()) ** 2)
    npw = max(50, int(per_worker_cells / mean_cells))
    jobs = []
    cells = 0
    for _ in range(cores):
        a = rng.integers(0, k, npw)
        c = rng.integers(0, k, npw)
        cells += int((L[a] * L[c]).sum())
        jobs.append((b.codes, b.seq_off, a, c))
    t0 = time.perf_counter()
    with mp.get_context("fork").Pool(cores) as pool:
        pool.map(_oracle_worker, jobs)
    wall = time.perf_counter() - t0
    # one thread: 10^4 seeded pairs of the workload, and every pair of c1
    from paper_1603_06958_amd import inputs
    a = rng.integers(0, k, 10000)
    c = rng.integers(0, k, 10000)
    t0 = time.perf_counter()
    oracle.lcs_pairs(b.codes, b.seq_off, a, c)
    st_sample = float((L[a] * L[c]).sum()) / (time.perf_counter() - t0) / 1e9
    c1 = inputs.c1()
    i1, j1 = np.triu_indices(c1.nseq, 1)
    t0 = time.perf_counter()
    oracle.lcs_pairs(c1.codes, c1.seq_off, i1, j1)
    st_c1 = c1.cells() / (time.perf_counter() - t0) / 1e9
    return {"value": cells / wall / 1e9, "unit": "GCUPS", "cores": cores, "kind": "oracle",
            "affinity_cpus": visible, "cpu_share": CPU_SHARE,
            "sample": f"{cores * npw} random pairs of the workload (seed {seed}), {cells:.3e} cells, "
                      f"{cores} single-threaded processes, {wall:.1f} s wall",
            "single_thread_gcups": {"workload_10k_pairs": round(st_sample, 3), "c1_all_pairs": round(st_c1, 3)}}


def run_main(b, steps, warmup, flags, tile_rows=1024, tune=True):
    from paper_1603_06958_amd import binding as B
    import torch
    p = B.Plan.from_batch(b, tile_rows=tile_rows, flags=flags, step_values=STEP_VALUES)
    if tune:
        t0 = time.perf_counter()
        p.autotune(os.environ.get("FAMSA_LCS_TUNE_CACHE") or None)
        print(f"[bench] autotune {time.perf_counter() - t0:.2f}s -> cols {p.info().cols_per_item} "
              f"waves {list(p.info().waves_per_group)[:3]}", file=sys.stderr, flush=True)
    info = p.info()
    sink = [0]

    def fn(t):
        sink[0] += int(t.count)
        return 0

    for _ in range(warmup):
        p.run(fn)
    torch.cuda.synchronize()
    times, kstats = [], []
    for _ in range(steps):
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        p.run(fn)
        torch.cuda.synchronize()
        times.append(time.perf_counter() - t0)
        kstats.append(p.stats())
    p.close()
    return info, times, kstats, sink[0]


def run_gpu_single_linkage(b, passes=2):
    """Device tiles into the GPU exact single-linkage consumer; best of `passes`."""
    from paper_1603_06958_amd import binding as B
    p = B.Plan.from_batch(b, flags=B.DEVICE_TILES, step_values=STEP_VALUES)
    p.autotune(os.environ.get("FAMSA_LCS_TUNE_CACHE") or None)
    best, edges, rounds, gt_ms = None, 0, 0, None
    for _ in range(passes):
        m = B.Mst(b.lengths())
        t0 = time.perf_counter()
        p.run_native(B.Mst.consume_fn(), m.handle)
        u = m.result()[0]
        dt = time.perf_counter() - t0
        t1 = time.perf_counter()
        left = m.guide_tree()[0]
        gt = 1e3 * (time.perf_counter() - t1)
        edges, rounds = len(u), m.stats()[1]
        assert len(left) == edges
        m.close()
        best = dt if best is None else min(best, dt)
        gt_ms = gt if gt_ms is None else min(gt_ms, gt)
    p.close()
    return {"s": round(best, 4), "gcups": round(b.cells() / best / 1e9, 1), "tree_edges": edges,
            "boruvka_rounds": rounds, "guide_tree_ms": round(gt_ms, 2),
            "delivery": "device tiles, graph replays on one compute stream"}


def run_consumer_alone(b, reps=2):
    """The GPU single-linkage consumer alone: every tile of the workload is
    first computed into one device buffer (the whole matrix, 20 GB for c4),
    then the consumer is timed over the stored tiles; best of `reps`."""
    import ctypes
    import torch
    from paper_1603_06958_amd import binding as B
    k = b.nseq
    buf = torch.empty(k * (k - 1) // 2, dtype=torch.int32, device="cuda")
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpyAsync.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int, ctypes.c_void_p]
    tiles, off = [], [0]

    def keep(t):
        n = int(t.count)
        if n and hip.hipMemcpyAsync(buf.data_ptr() + 4 * off[0], ctypes.cast(t.lcs, ctypes.c_void_p), 4 * n, 3,
                                    t.stream) != 0:
            return 1
        tiles.append((int(t.row_begin), int(t.row_end), off[0], n))
        off[0] += n
        return 0

    with B.Plan.from_batch(b, flags=B.DEVICE_TILES, step_values=STEP_VALUES) as p:
        p.run(keep)
    torch.cuda.synchronize()
    stream = torch.cuda.current_stream().cuda_stream
    best, rounds = None, 0
    for _ in range(reps):
        m = B.Mst(b.lengths())
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        for r0, r1, o, n in tiles:
            t = B.Tile(tile_index=0, family=0, k=k, row_begin=r0, row_end=r1,
                       lcs=ctypes.cast(ctypes.c_void_p(buf.data_ptr() + 4 * o), ctypes.POINTER(ctypes.c_int32)),
                       count=n, stream=stream, values=B.VALUES_LCS)
            B.check(0 if B.lib().famsa_mst_consume(m.handle, ctypes.byref(t)) == 0 else B.EDEVICE)
        edges = len(m.result()[0])
        dt = time.perf_counter() - t0
        rounds = m.stats()[1]
        m.close()
        best = dt if best is None else min(best, dt)
    del buf
    return {"s": round(best, 4), "tiles": len(tiles), "tree_edges": edges, "boruvka_rounds": rounds,
            "ms_per_tile": round(1e3 * best / max(1, len(tiles)), 3)}


def run_host_slink():
    """Host SLINK (exact similarities) over all of c2's tiles: the consumer
    alone (tiles already in host memory, fed last row first), and the whole
    pipeline with the consumer as the plan's tile callback."""
    import ctypes
    from paper_1603_06958_amd import binding as B, inputs
    b = inputs.c2()
    with B.Plan.from_batch(b, flags=B.DESCENDING) as p:
        tiles = p.collect()
        s = B.SLink(b.lengths())
        t0 = time.perf_counter()
        p.run_native(B.SLink.consume_fn(), s.handle)
        pipe = time.perf_counter() - t0
        s.close()
    s = B.SLink(b.lengths())
    order = sorted(tiles, key=lambda key: -key[1])
    t0 = time.perf_counter()
    for idx, (f, r0, r1) in enumerate(order):
        vals = tiles[(f, r0, r1)]
        t = B.Tile()
        t.tile_index, t.family, t.k, t.row_begin, t.row_end, t.count = idx, 0, b.nseq, r0, r1, vals.size
        t.lcs = vals.ctypes.data_as(ctypes.POINTER(ctypes.c_int32)) if vals.size else None
        assert s.feed(t) == 0
    dt = time.perf_counter() - t0
    s.close()
    return {"workload": "c2: one tree-evolved family, k=10000", "consumer_s": round(dt, 3),
            "pair_updates_per_s": round(b.pairs() / dt, 1), "pipeline_s": round(pipe, 3), "threads": 1}


def run_gapped(b, nruns=64, seed=11):
    """Gapped representation over the workload's sequences: one profile-wide
    round of `nruns` gap runs inserted into every sequence, then every row
    decoded to host memory."""
    from paper_1603_06958_amd import binding as B
    rng = np.random.default_rng(seed)
    g = B.Gapped(b.codes, b.seq_off)
    width = int(g.width().min()) + 1
    cols = np.sort(rng.integers(1, width + 1, nruns)).astype(np.uint32)
    lens = rng.integers(1, 4, nruns).astype(np.uint32)
    t0 = time.perf_counter()
    g.insert(cols, lens)
    t_ins = time.perf_counter() - t0
    t0 = time.perf_counter()
    rows = g.decode()
    t_dec = time.perf_counter() - t0
    g.close()
    return {"sequences": b.nseq, "runs": nruns, "insert_ms": round(1e3 * t_ins, 2),
            "run_updates_per_s": round(b.nseq * nruns / t_ins, 1), "decode_ms": round(1e3 * t_dec, 2),
            "decoded_bytes": int(rows.nbytes), "decode_host_gb_s": round(rows.nbytes / t_dec / 1e9, 2)}


def traffic_per_launch(kernel):
    """HBM bytes per launch of `kernel` from the committed counter summary,
    if it was taken from the current kernel source in the bench configuration."""
    import hashlib
    try:
        text = open(TRAFFIC_SUMMARY).read()
        sha = hashlib.sha256(b"".join(open(f, "rb").read() for f in KERNEL_SOURCES)).hexdigest()[:16]
    except OSError:
        return None, "no counter summary"
    if f"sha256[:16] = {sha}" not in text:
        return None, "kernel changed since the counters were taken"
    if f"step_values {STEP_VALUES}, one compute stream" not in text:
        return None, "counters taken in another configuration"
    for line in text.splitlines():
        f = line.split()
        if f and f[0] == kernel and len(f) >= 6:
            return int(round((float(f[4]) + float(f[5])) * 1e6)), "rocprofv3 FETCH_SIZE + WRITE_SIZE, copy-calibrated"
    return None, "kernel not in the counter summary"


def run_peak(variants=(0,), blocks_per_cu=8, iters=20000):
    """The integer-VALU ceiling measured by the library's register-only chains
    of the LCS step's instructions (famsa_valu_peak); best of three each."""
    from paper_1603_06958_amd import binding as B
    names = {0: "recurrence (and, addc chain, bitop3)", 1: "v_and_b32", 2: "v_addc_co_u32 chain", 3: "v_bitop3_b32"}
    out = {}
    for v in variants:
        best = None
        for _ in range(3):
            r = B.valu_peak(v, blocks_per_cu, iters)
            if best is None or r.ops_per_s > best.ops_per_s:
                best = r
        out[names[v]] = {"tops_per_s": round(best.ops_per_s / 1e12, 3), "clock_ghz": round(best.clock_ghz, 3),
                         "lane_ops_per_clk_per_cu": round(best.lane_ops_per_clk_per_cu, 2),
                         "ms": round(best.ms, 3), "cus": int(best.cus)}
    return out


PROFILE_DP_OPS_PER_CELL = 40  # int32 lane-ops of one DP cell: 8 int64 add/sub (2 each), 4 three-way int64 maxima
                              # (2 compares and 2 two-register selects each)


def run_profile_dp(nprob=2048, seed=12, reps=3, cpu_problems=12):
    """Aligning one sequence to a profile (famsa_profile_align) on a synthetic
    progressive-stage level: `nprob` independent problems, profile width
    log-uniform in [50, 500], sequence within 15% of it, 1..200 rows; DP
    cells per second from HIP events around the DP launch, and the oracle's
    rate on a few of the same problems."""
    from oracle import profile as OP
    from paper_1603_06958_amd import binding as B, inputs
    probs = inputs.profile_batch(nprob, seed, m_range=(50, 500), K_range=(1, 200))
    S = inputs.synthetic_subst(20, seed)
    costs = OP.scaled_gap_costs(10000, (9, 2, 12, 3))
    pairs = [(p.seq, p.rows) for p in probs]
    cells = sum((p.seq.size + 1) * (p.rows.shape[1] + 1) for p in probs)
    B.profile_align(pairs, S, costs)  # warm-up
    walls, dps = [], []
    for _ in range(reps):
        t0 = time.perf_counter()
        B.profile_align(pairs, S, costs)
        walls.append(time.perf_counter() - t0)
        dps.append(B.profile_last_dp_ms())
    dp_ms = float(np.median(dps))
    t0 = time.perf_counter()
    cpu_cells = 0
    for p in probs[:cpu_problems]:
        OP.align(p.seq, p.rows, S, costs)
        cpu_cells += (p.seq.size + 1) * (p.rows.shape[1] + 1)
    cpu_s = time.perf_counter() - t0
    achieved = cells / (dp_ms / 1e3) * PROFILE_DP_OPS_PER_CELL
    return {"workload": f"{nprob} sequence-to-profile problems, width log-uniform [50,500], rows log-uniform [1,200], "
                        f"seed {seed}", "cells": int(cells), "dp_kernel_ms": round(dp_ms, 3),
            "dp_gcups": round(cells / (dp_ms / 1e3) / 1e9, 2), "call_ms": round(1e3 * float(np.median(walls)), 2),
            "roofline": {"bound": "alu", "achieved": round(achieved / 1e12, 3), "peak": round(PEAK_INT_OPS / 1e12, 3),
                         "unit": "Tops/s (int32 VALU)", "frac": round(achieved / PEAK_INT_OPS, 4),
                         "ops_per_cell": PROFILE_DP_OPS_PER_CELL, "kernel": "pdp_dp_kernel"},
            "cpu_baseline": {"value": round(cpu_cells / cpu_s / 1e9, 4), "unit": "GCUPS", "cores": 1, "kind": "oracle",
                             "sample": f"the first {cpu_problems} problems through oracle.profile.align"}}


def run_c3(passes=5):
    from paper_1603_06958_amd import binding as B, inputs
    b = inputs.c3()
    out = {"workload": "c3: 64 tree-evolved families, k log-uniform [50,5000], root length log-uniform [30,2000]",
           "pairs": b.pairs(), "cells": b.cells()}
    res = {}
    for name, flags in [("batched", 0), ("plain", B.PLAIN), ("plain_async", B.PLAIN | B.PLAIN_ASYNC)]:
        p = B.Plan.from_batch(b, flags=flags)
        chk = [0]

        def fn(t):
            chk[0] += int(t.count)
            return 0

        p.run(fn)  # warm-up
        times = []
        for _ in range(passes):
            t0 = time.perf_counter()
            p.run(fn)
            times.append(time.perf_counter() - t0)
        med = float(np.median(times))
        res[name] = med
        out[f"{name}_s"] = round(med, 4)
        out[f"{name}_gcups"] = round(b.cells() / med / 1e9, 1)
        p.close()
    out["passes"] = passes
    out["batched_over_plain"] = round(res["plain"] / res["batched"], 2)
    out["batched_over_plain_async"] = round(res["plain_async"] / res["batched"], 2)
    return out


def run_serve():
    from paper_1603_06958_amd import serve
    return serve.run_c5_bench()


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--workload", default="c4", choices=["c1", "c2", "c4"])
    ap.add_argument("--no-c3", action="store_true")
    ap.add_argument("--no-serve", action="store_true")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-extra", action="store_true",
                    help="skip the two-stream, GPU single-linkage and host SLINK measurements")
    ap.add_argument("--copy-calibration", action="store_true",
                    help="only run a plain device copy of 1 GiB (for scaling HBM byte counters)")
    ap.add_argument("--peak", action="store_true",
                    help="only run the integer-VALU ceiling microbenchmark (all four instruction variants)")
    ap.add_argument("--c3-only", action="store_true",
                    help="only run the c3 batching measurement (batched, plain, plain-async)")
    ap.add_argument("--profile-dp", action="store_true",
                    help="only run the sequence-to-profile alignment measurement")
    ap.add_argument("--consumer-alone", action="store_true",
                    help="only time the GPU single-linkage consumer over the workload's tiles kept in HBM")
    a = ap.parse_args()
    if a.copy_calibration:
        import torch
        x = torch.ones(1 << 28, dtype=torch.int32, device="cuda")
        y = torch.empty_like(x)
        torch.cuda.synchronize()
        y.copy_(x)
        torch.cuda.synchronize()
        print(json.dumps({"copy_bytes": x.numel() * 4}))
        return
    if a.peak:
        print(json.dumps({"valu_peak": run_peak(variants=(0, 1, 2, 3))}), flush=True)
        return
    if a.c3_only:
        print(json.dumps({"c3": run_c3()}), flush=True)
        return
    if a.profile_dp:
        print(json.dumps({"profile_dp": run_profile_dp()}), flush=True)
        return
    if a.consumer_alone:
        from paper_1603_06958_amd import inputs
        print(json.dumps({"consumer_alone": run_consumer_alone(getattr(inputs, a.workload)()),
                          "workload": a.workload}), flush=True)
        return
    if a.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py measures one GPU only: the stage runs on a single MI355X here "
              "(sharding across GPUs is a design whose forest merge is tested on one GPU); use --gpus 1",
              file=sys.stderr)
        sys.exit(2)
    from paper_1603_06958_amd import inputs
    import torch
    assert torch.cuda.is_available(), "bench.py needs a GPU"
    t0 = time.time()
    b = inputs.WORKLOADS[a.workload]()
    print(f"[bench] generated {a.workload} in {time.time() - t0:.1f}s: {inputs.stats(b)}", file=sys.stderr,
          flush=True)
    from paper_1603_06958_amd import binding as B
    info, times, kst, count = run_main(b, a.steps, a.warmup, flags=B.ONE_STREAM | B.NO_GRAPH)
    cells = info.cells
    ms = 1e3 * float(np.mean(times))
    value = cells / (ms / 1e3) / 1e9
    # dominant kernel: the fast class with the most cells
    cls = int(np.argmax([kst[-1].cells[c] for c in range(3)]))
    kms = float(np.mean([s.kernel_ms[cls] / max(1, s.launches[cls]) for s in kst]))
    per_launch_cells = kst[-1].cells[cls] / max(1, kst[-1].launches[cls])
    achieved = per_launch_cells * OPS_PER_CELL / (kms / 1e3)
    kname = f"lcs_fast_kernel<{cls},20>"
    peak_meas = run_peak(variants=(0,))["recurrence (and, addc chain, bitop3)"]
    traffic, traffic_src = traffic_per_launch(kname)
    print(f"[bench] steps {[round(t, 3) for t in times]} s; kernel classes ms "
          f"{[round(x, 1) for x in kst[-1].kernel_ms]} launches {list(kst[-1].launches)} "
          f"step_ms {kst[-1].step_ms:.1f}", file=sys.stderr, flush=True)
    res = {
        "metric": METRIC, "value": round(value, 1), "unit": "GCUPS", "n_gpus": 1, "steps": a.steps,
        "warmup": a.warmup, "ms_per_step": round(ms, 2), "higher_is_better": True, "scaling": "weak",
        "vs_baseline": None, "dtype": "u32", "data": "synthetic",
        "config": {"workload": {"c4": "c4: one tree-evolved family, k=100000, root 250, log-normal lengths "
                                      "(median 250, sigma 0.3, clip [40,1500]), seed 3",
                                "c2": "c2: one tree-evolved family, k=10000, root 300, seed 1",
                                "c1": "c1: k=100 i.i.d., lengths U[50,300], seed 0"}[a.workload],
                   "k": b.nseq, "pairs": info.pairs, "cells": cells, "tile_rows": 1024,
                   "step_values": STEP_VALUES, "streams": "one compute stream, one copy stream",
                   "delivery": "host pinned memory, callback per tile"},
        "pairs_per_s": round(info.pairs / (ms / 1e3), 1),
        "whole_job_alu_frac": round(cells * OPS_PER_CELL / (ms / 1e3) / PEAK_INT_OPS, 4),
        "device_gcups": round(cells / (kst[-1].step_ms / 1e3) / 1e9, 1),
        "peak_hbm_bytes": int(info.device_bytes),
        "roofline": {"bound": "alu", "achieved": round(achieved / 1e12, 3), "peak": round(PEAK_INT_OPS / 1e12, 3),
                     "unit": "Tops/s (int32 VALU)", "frac": round(achieved / PEAK_INT_OPS, 4), "traffic": traffic,
                     "traffic_unit": "HBM bytes per launch (read + write)", "traffic_source": traffic_src,
                     "kernel": kname, "avg_launch_ms": round(kms, 3),
                     "cells_per_launch": int(per_launch_cells),
                     "ops_per_cell": "3/32 (AND, ADDC, BITOP3 per 32-cell dword)",
                     "peak_measured": peak_meas["tops_per_s"],
                     "frac_of_measured_peak": round(achieved / 1e12 / peak_meas["tops_per_s"], 4),
                     "peak_measured_source": "famsa_valu_peak: register-only chains of the recurrence's three "
                                             f"instructions on every CU at {peak_meas['clock_ghz']} GHz "
                                             f"({peak_meas['lane_ops_per_clk_per_cu']} lane-ops/clk/CU)"},
        "launch": {"cols_per_item": int(info.cols_per_item), "waves_per_group": list(info.waves_per_group)[:3]},
    }
    if not a.no_extra:
        _, tg, _, _ = run_main(b, 2, 1, flags=0, tune=True)
        res["graph_replay"] = {"value": round(cells / min(tg) / 1e9, 1), "unit": "GCUPS",
                               "ms_per_step": round(1e3 * min(tg), 2),
                               "note": "same pass, steps replayed as hipGraphs on one compute stream (library default)"}
        print(f"[bench] graph_replay {res['graph_replay']}", file=sys.stderr, flush=True)
        _, t2, _, _ = run_main(b, 2, 1, flags=B.TWO_STREAMS, tune=True)
        res["two_streams"] = {"value": round(cells / min(t2) / 1e9, 1), "unit": "GCUPS",
                              "ms_per_step": round(1e3 * min(t2), 2),
                              "note": "same pass, graph replays alternating between two compute streams"}
        print(f"[bench] two_streams {res['two_streams']}", file=sys.stderr, flush=True)
        _, tp, _, _ = run_main(b, 1, 0, flags=B.PLAIN, tune=False)
        res["plain"] = {"value": round(cells / tp[0] / 1e9, 1), "unit": "GCUPS", "ms_per_step": round(1e3 * tp[0], 2),
                        "batched_over_plain": round(tp[0] / (ms / 1e3), 2),
                        "note": "one pass of the plain baseline: one pair per lane, one launch per tile, each "
                                "waiting for the previous tile's delivery"}
        print(f"[bench] plain {res['plain']}", file=sys.stderr, flush=True)
        _, t3, _, _ = run_main(b, 2, 1, flags=B.OUT_SIM, tune=True)
        res["similarity_tiles"] = {"value": round(cells / min(t3) / 1e9, 1), "unit": "GCUPS",
                                   "ms_per_step": round(1e3 * min(t3), 2),
                                   "note": "same pass delivering float32 LCS/indel^2 tiles (FAMSA_LCS_OUT_SIM)"}
        print(f"[bench] similarity_tiles {res['similarity_tiles']}", file=sys.stderr, flush=True)
        if a.workload == "c4":
            res["gpu_single_linkage"] = run_gpu_single_linkage(b)
            print(f"[bench] gpu_single_linkage {res['gpu_single_linkage']}", file=sys.stderr, flush=True)
        res["host_slink"] = run_host_slink()
        print(f"[bench] host_slink {res['host_slink']}", file=sys.stderr, flush=True)
        res["gapped"] = run_gapped(b)
        print(f"[bench] gapped {res['gapped']}", file=sys.stderr, flush=True)
        res["profile_dp"] = run_profile_dp()
        print(f"[bench] profile_dp {res['profile_dp']}", file=sys.stderr, flush=True)
    if not a.no_c3:
        res["c3"] = run_c3()
        print(f"[bench] c3 {res['c3']}", file=sys.stderr, flush=True)
    if not a.no_serve:
        try:
            res["serve"] = run_serve()
        except Exception as e:  # report, do not hide
            res["serve"] = {"error": str(e)}
        print(f"[bench] serve {res['serve']}", file=sys.stderr, flush=True)
    if not a.no_cpu:
        res["cpu_baseline"] = cpu_baseline(b)
    print(json.dumps(res), flush=True)


if __name__ == "__main__":
    main()
