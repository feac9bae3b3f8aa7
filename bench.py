#!/usr/bin/env python3
"""Benchmark of the MI355X BFS hot path.

Default workload (one JSON line on stdout): single-source top-down BFS on an
R-MAT graph of scale 24, edge factor 16 (initiator 0.57/0.19/0.19/0.05,
symmetrised, self-loops and duplicates removed, labels permuted), int32 CSR.
One step = one whole traversal (reset, level loop of Phase 1 expansion and
Phase 2 merge, termination) from one seeded source; K steps use K distinct
seeded sources, run one at a time. `value` is the harmonic mean GTEPS
(edges scanned / traversal time) over the K timed steps.

Other workloads (``--workload``): ``batch`` (1024 sources over 8 R-MAT graphs
as one bitset multi-source launch, queries/s against one-at-a-time BFS),
``serve`` (Poisson stream over a resident pool, p50/p99 latency), ``share29``
(one node's 1/16 share of an R-MAT scale-29 graph with staged butterfly
messages), ``rmat14`` (the small R-MAT scale-14 case).

The oracle is imported only for the cpu_baseline leg.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

import numpy as np

ROOT = os.path.dirname(os.path.abspath(__file__))
if ROOT not in sys.path:
    sys.path.insert(0, ROOT)

import graphgen as gg  # noqa: E402
from paper_2103_13577_amd import metrics  # noqa: E402

HBM_PEAK_GBS = 8000.0

# Seeds of every synthetic input (graph, permutation, sources), fixed per workload.
SEEDS = {
    "rmat24": (0x5EED0024, 0xBEEF0024, 0xC0FFEE24),
    "rmat14": (0x5EED0014, 0xBEEF0014, 0xC0FFEE14),
}


def log(msg):
    print(f"[bench] {msg}", file=sys.stderr, flush=True)


def host_facts():
    cpu = "unknown"
    try:
        with open("/proc/cpuinfo") as f:
            for line in f:
                if line.startswith("model name"):
                    cpu = line.split(":", 1)[1].strip()
                    break
    except OSError:
        pass
    mem_gb = None
    try:
        with open("/proc/meminfo") as f:
            mem_gb = round(int(f.readline().split()[1]) / 2**20, 1)
    except (OSError, ValueError, IndexError):
        pass
    return {"nproc": os.cpu_count(), "cpu": cpu, "mem_gb": mem_gb}


def kernel_source_hash() -> str:
    import hashlib
    h = hashlib.sha256()
    for f in ("bfs_kernels.hip", "bfs_core.hpp", "device.hpp"):
        with open(os.path.join(ROOT, "paper_2103_13577_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def measured_traffic(kernel, per_launch_bytes):
    """HBM bytes per launch of `kernel` from the committed rocprofv3 --pmc
    summary (FETCH_SIZE and WRITE_SIZE, scaled by a plain copy of known size),
    or None when the summary was taken on other kernel sources."""
    path = os.path.join(ROOT, "profiles", "traffic_rmat24.json")
    try:
        with open(path) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    k = rec.get("kernels", {}).get(kernel)
    if not k or rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return {"bytes_per_launch": k["hbm_bytes_per_launch"],
            "vs_algorithmic": round(k["hbm_bytes_per_launch"] / max(per_launch_bytes, 1.0), 3),
            "source": "profiles/traffic_rmat24.json"}


def measured_share_traffic():
    """HBM bytes of the partitioned share's timed top-down traversals from the
    committed rocprofv3 --pmc summary (k_merge per launch, k_expand per
    traversal), or None when it was taken on other kernel sources."""
    try:
        with open(os.path.join(ROOT, "profiles", "traffic_share29.json")) as f:
            rec = json.load(f)
    except (OSError, ValueError):
        return None
    if rec.get("kernel_source_hash") != kernel_source_hash():
        return None
    return rec.get("kernels")


def pinned_core():
    """The first core this process may run on (Linux), or None."""
    try:
        return min(os.sched_getaffinity(0))
    except (AttributeError, OSError, ValueError):
        return None


def cpu_baseline_single(g, sources, budget_s=20.0):
    """Times the CPU oracle (single-threaded FIFO BFS) on a bounded sample of
    the same sources, in order: whole traversals until about budget_s of CPU
    work, with the calling thread pinned to one core for the duration."""
    import oracle
    core = pinned_core()
    saved = None
    if core is not None:
        saved = os.sched_getaffinity(0)
        os.sched_setaffinity(0, {core})
    try:
        edges, secs, used = 0, 0.0, 0
        for s in sources:
            t0 = time.perf_counter()
            d = oracle.bfs(g, int(s))
            dt = time.perf_counter() - t0
            edges += oracle.edges_scanned(g, d)
            secs += dt
            used += 1
            if secs >= budget_s:
                break
    finally:
        if saved is not None:
            os.sched_setaffinity(0, saved)
    return {"value": round(metrics.gteps(edges, secs), 4), "unit": "GTEPS", "cores": 1,
            "kind": "oracle", "pinned_core": core,
            "sample": f"the first {used} of the {len(sources)} timed sources, whole traversals, "
                      f"{secs:.1f} s of single-threaded FIFO BFS on the same graph, thread pinned "
                      f"to core {core}"}


def oracle_check_single(plan, g, source, dist):
    """Runs one timed source again (outside the timed region) and compares its
    whole distance array with the CPU oracle."""
    import oracle
    d, _, _ = plan.run(0, int(source), dist=dist)
    got = d.cpu().numpy()
    ref = oracle.bfs(g, int(source))
    return bool(np.array_equal(got, ref)), int(np.count_nonzero(got != ref))


def headline_sources(g, count):
    """The seeded sources of the scale-24 workload: the first `warmup` warm
    the plan up, the rest are timed."""
    return gg.pick_sources(g, count, seed=SEEDS["rmat24"][2])


# Settings of the scale-24 headline plan (see run_single).
HEADLINE_PLAN = dict(loop_mode=3, small_bin=7, wave_bin=13, chunk_edges=1024, hot_words=20352,
                     sparse_div=-1, relabel=1, autotune=-1)


def run_single(args, name, scale, ef):
    import torch
    import paper_2103_13577_amd as pkg
    gseed, pseed, sseed = SEEDS[name]
    t0 = time.time()
    g = gg.rmat(scale, ef, seed=gseed, perm_seed=pseed)
    log(f"generated {name}: n={g.n} m={g.m} in {time.time() - t0:.1f}s")
    dev = torch.device("cuda:0")
    dg = pkg.DeviceGraph.from_csr(g, dev)
    # The scale-24 line runs the captured level loop: 8 level steps per graph
    # replay (the device decides each level's form and the end of the
    # traversal), one host round trip per replay. Its settings are pinned (a profiler slows every launch and moves the plan
    # autotuner's choices), so profiles of this command time the same kernels.
    # A fully autotuned plan runs first and is reported in the line's detail.
    opts = dict(loop_mode=args.loop_mode, grid_blocks=args.grid_blocks, small_bin=args.small_bin,
                wave_bin=args.wave_bin, chunk_edges=args.chunk_edges, relabel=args.relabel,
                autotune=args.autotune, hot_words=args.hot_words, sparse_div=args.sparse_div,
                direction=args.direction, mark_mode=args.mark_mode)
    headline = args.loop_mode < 0 and name == "rmat24" and not args.direction
    if args.loop_mode < 0:
        opts["loop_mode"] = 0
    if headline:
        for k, v in HEADLINE_PLAN.items():
            if not opts.get(k):
                opts[k] = v
    loop_mode = opts["loop_mode"]
    plan = pkg.Plan([dg], **opts)
    srcs = gg.pick_sources(g, args.warmup + args.steps, seed=sseed)
    dist = torch.empty(g.n, dtype=torch.int32, device=dev)
    auto_line = None
    if headline and args.auto_detail:
        # the autotuner's own choice of level loop over the same sources, run
        # before the timed region (whose launches a profile takes as the last
        # ones of their kernels)
        auto = pkg.Plan([dg], grid_blocks=args.grid_blocks, relabel=args.relabel,
                        autotune=args.autotune, sparse_div=args.sparse_div)
        for s in srcs[:args.warmup]:
            auto.run(0, int(s), dist=dist)
        ast = [auto.run(0, int(s), dist=dist)[2] for s in srcs[args.warmup:]]
        ams = np.array([x.ms for x in ast])
        aedges = np.array([x.edges_scanned for x in ast], dtype=np.float64)
        auto_line = {"plan": auto.tuning(0), "ms_per_step": round(float(np.mean(ams)), 4),
                     "gteps": round(metrics.harmonic_mean(aedges / (ams * 1e-3) / 1e9), 3)}
        auto.close()
    for s in srcs[:args.warmup]:
        plan.run(0, int(s), dist=dist)
    torch.cuda.synchronize()
    stats = []
    t_wall = time.perf_counter()
    for s in srcs[args.warmup:]:
        _, _, st = plan.run(0, int(s), dist=dist)
        stats.append(st)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t_wall
    ms = np.array([s.ms for s in stats])
    loop_ms = np.array([s.loop_ms for s in stats])
    edges = np.array([s.edges_scanned for s in stats], dtype=np.float64)
    reached = np.array([s.reached for s in stats], dtype=np.float64)
    rates = edges / (ms * 1e-3) / 1e9
    hmean = metrics.harmonic_mean(rates)
    tuning = plan.tuning(0)
    exact, mismatches = oracle_check_single(plan, g, srcs[args.warmup], dist)
    log(f"oracle check of source {int(srcs[args.warmup])}: exact={exact}")
    roof_stats, roof_note = stats, None
    if tuning["loop_mode"] == 3 and tuning["direction"] == 0:
        # The captured loop replays its level steps as one graph, inside which
        # no HIP event can bracket a kernel. Its kernels are timed on a second
        # pass over the same timed sources by a plan with the same settings
        # that launches the same level steps directly (BFS_LOOP_ENQUEUE), each
        # launch bracketed by HIP events on the plan's stream.
        rplan = pkg.Plan([dg], **{**opts, "loop_mode": 5})
        for s in srcs[:args.warmup]:
            rplan.run(0, int(s), dist=dist)
        roof_stats = [rplan.run(0, int(s), dist=dist)[2] for s in srcs[args.warmup:]]
        rplan.close()
        roof_note = ("kernel timed with HIP events on a second pass over the same timed sources, "
                     "the same level steps launched directly (loop 5) by a plan with the same "
                     "settings; the value's pass replays them as a captured graph")
    if tuning["direction"] == 1:
        # direction-optimizing: the dominant kernel is the bottom-up step.
        # Per launch it reads two int64 row offsets per unvisited vertex it
        # examines (16 B) and the column index of every adjacency entry it
        # loads (4 B); the device counts both, and the launches are timed with
        # HIP events on the plan's stream.
        kname = "k_bottom_up"
        bu_ms = np.array([s.bottom_up_ms for s in stats])
        launches = np.array([s.bottom_up_levels for s in stats])
        k_bytes = np.array([4.0 * s.bottom_up_edges + 16.0 * s.bottom_up_vertices for s in stats])
        achieved = float(np.sum(k_bytes) / max(np.sum(bu_ms) * 1e-3, 1e-12) / 1e9)
        per_launch_bytes = float(np.sum(k_bytes) / max(np.sum(launches), 1))
        avg_launch_ms = float(np.sum(bu_ms) / max(np.sum(launches), 1))
        n_launches = int(np.sum(launches))
    elif tuning["loop_mode"] in (1, 3, 5):
        # host-driven loop or enqueued level steps: the dominant kernel is the
        # dense expansion (k_expand / k_expand_wide, or the level steps'
        # k_expand_g / k_expand_gw). Per launch it reads the column index of
        # every edge it scans (4 B) and two int64 row offsets per frontier
        # vertex (16 B); the device counts both, and each launch is timed with
        # HIP events on the plan's stream (for the level steps, launches also
        # count the steps of the last round trip that find the traversal
        # finished). Queue-only levels (small frontiers) run another kernel
        # and are not part of this figure.
        if tuning["loop_mode"] in (3, 5):
            kname = "k_expand_gw" if tuning["hot_words"] > 4096 else "k_expand_g"
        else:
            kname = "k_expand+k_expand_wide" if tuning["hot_words"] > 4096 else "k_expand"
        exp_ms = np.array([s.expand_ms for s in roof_stats])
        launches = np.array([s.expand_launches for s in roof_stats])
        k_bytes = np.array([4.0 * s.dense_edges + 16.0 * s.dense_frontier for s in roof_stats])
        achieved = float(np.sum(k_bytes) / (np.sum(exp_ms) * 1e-3) / 1e9)
        per_launch_bytes = float(np.sum(k_bytes) / max(np.sum(launches), 1))
        avg_launch_ms = float(np.sum(exp_ms) / max(np.sum(launches), 1))
        n_launches = int(np.sum(launches))
    else:
        # device-resident loops: one launch per traversal (for the captured
        # graph, the replayed level steps), which also writes each reached
        # vertex's distance (4 B)
        kname = {2: "k_persistent_occ8" if tuning["persist_variant"] == 1 else "k_persistent",
                 4: "k_bfs_cu"}.get(tuning["loop_mode"], "unknown")
        k_bytes = 4 * edges + 16 * reached + 4 * reached
        achieved = float(np.mean(k_bytes) / (np.mean(loop_ms) * 1e-3) / 1e9)
        per_launch_bytes = float(np.mean(k_bytes))
        avg_launch_ms = float(np.mean(loop_ms))
        n_launches = len(stats)
    traffic = measured_traffic(_dense_series(kname), per_launch_bytes)
    whole_bytes = np.array([metrics.bytes_single_source(e, r, g.n) for e, r in zip(edges, reached)])
    out = {
        "metric": "GTEPS (1 MI355X, all edges) + batched queries/sec with p50/p99 latency",
        "value": round(hmean, 3),
        "unit": "GTEPS",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": round(float(np.mean(ms)), 4),
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "int32",
        "data": "synthetic",
        "exact": exact,
        "exact_check": {"source": int(srcs[args.warmup]), "against": "CPU oracle, whole distance array",
                        "mismatched_vertices": mismatches},
        "config": {"workload": f"single-source {'direction-optimizing' if args.direction else 'top-down'} "
                               f"BFS, R-MAT scale {scale} edge factor {ef} "
                               f"(A=.57,B=.19,C=.19), symmetrised, int32 CSR, "
                               f"{args.steps} seeded sources one at a time",
                   "n": g.n, "m_directed": g.m, "sources": args.steps,
                   "plan": plan.tuning(0)},
        "roofline": {"bound": "hbm", "achieved": round(achieved, 1), "peak": HBM_PEAK_GBS,
                     "unit": "GB/s", "frac": round(achieved / HBM_PEAK_GBS, 4),
                     "traffic": traffic["bytes_per_launch"] if traffic else None, "kernel": kname,
                     "bytes_per_launch": int(per_launch_bytes),
                     "avg_launch_ms": round(avg_launch_ms, 4), "launches": n_launches,
                     "traffic_detail": traffic},
        **({"roofline_timing": roof_note} if roof_note else {}),
        "detail": {
            "gteps_trimmed_mean_time": round(metrics.gteps(np.mean(edges), metrics.trimmed_mean(ms) * 1e-3), 3),
            "gteps_whole_graph_convention": round(metrics.harmonic_mean(g.m / (ms * 1e-3) / 1e9), 3),
            "whole_traversal_hbm_frac": round(float(np.mean(whole_bytes) / (np.mean(ms) * 1e-3) / 1e9 / HBM_PEAK_GBS), 4),
            "edges_scanned_mean": int(np.mean(edges)),
            "reached_mean": int(np.mean(reached)),
            "levels": [int(s.levels) for s in stats][:8],
            "wall_s_timed_region": round(wall, 4),
            "host": host_facts(),
        },
    }
    if auto_line is not None:
        out["detail"]["autotuned_loop"] = auto_line
    copy_gbs = measured_copy_gbs()
    out["roofline"]["measured_copy_gbs"] = copy_gbs
    out["roofline"]["frac_of_copy"] = round(achieved / copy_gbs, 4)
    if args.cpu_baseline:
        out["cpu_baseline"] = cpu_baseline_single(g, srcs[args.warmup:], budget_s=args.cpu_budget)
    plan.close()
    return out


# ---------------------------------------------------------------------------
# batched multi-source workload: 1024 sources over 8 R-MAT graphs
# ---------------------------------------------------------------------------

BATCH_SCALES = [16, 17, 18, 19, 20, 21, 22, 22]


def run_batch(args):
    """1024 sources (128 per graph) over R-MAT scales 16..22,22 (edge factor
    16) as one bitset multi-source launch with uint8 outputs, against the same
    1024 (graph, source) pairs run one at a time through bfs_run."""
    import torch
    import paper_2103_13577_amd as pkg
    dev = torch.device("cuda:0")
    t0 = time.time()
    gs = [gg.rmat(s, 16, seed=0x5EED0400 + i, perm_seed=0xBEEF0400 + i)
          for i, s in enumerate(BATCH_SCALES)]
    log(f"generated batch graphs in {time.time() - t0:.1f}s")
    dgs = [pkg.DeviceGraph.from_csr(g, dev) for g in gs]
    plan = pkg.Plan(dgs, batch_lanes=2, grid_blocks=args.grid_blocks)
    single = pkg.Plan(dgs, grid_blocks=args.grid_blocks)
    bt = plan.batch_tuning()
    log(f"batch engine settings {bt}")
    qs = []
    for gi, g in enumerate(gs):
        for s in gg.pick_sources(g, 128, seed=0xC0FFEE00 + gi):
            qs.append((gi, int(s), torch.empty(g.n, dtype=torch.uint8, device=dev)))
    # warm-up
    for _ in range(max(args.warmup, 1)):
        plan.batch_wait(plan.batch_submit(qs, pkg.BATCH_ONE_LAUNCH))
    torch.cuda.synchronize()
    reps = max(1, min(args.steps, 8))
    times = []
    for _ in range(reps):
        t = time.perf_counter()
        tk = plan.batch_submit(qs, pkg.BATCH_ONE_LAUNCH)
        plan.batch_wait(tk)
        times.append(time.perf_counter() - t)
    t_batch = float(np.median(times))
    # one query at a time, same pairs
    dist = torch.empty(max(g.n for g in gs), dtype=torch.int32, device=dev)
    exact = True
    torch.cuda.synchronize()
    t = time.perf_counter()
    for gi, s, _ in qs:
        single.run(gi, s, dist=dist[:gs[gi].n])
    torch.cuda.synchronize()
    t_plain = time.perf_counter() - t
    for gi, s, out in qs:
        d, _, _ = single.run(gi, s)
        ref = torch.where(d < 0, torch.full_like(d, 255), d).to(torch.uint8)
        if not torch.equal(out, ref):
            exact = False
    out = {
        "metric": "batched queries/sec (1024 sources, 8 R-MAT graphs, one launch)",
        "value": round(len(qs) / t_batch, 1), "unit": "queries/s", "n_gpus": 1,
        "steps": reps, "warmup": max(args.warmup, 1), "ms_per_step": round(t_batch * 1e3, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "u8",
        "data": "synthetic",
        "config": {"workload": "batched multi-source BFS, 1024 sources over R-MAT scales "
                               "16,17,18,19,20,21,22,22 (edge factor 16), 128 per graph, "
                               "64 sources per uint64 lane word, uint8 distances",
                   "lanes_per_graph": 2},
        "plain_one_at_a_time": {"value": round(len(qs) / t_plain, 1), "unit": "queries/s",
                                "seconds": round(t_plain, 4)},
        "speedup_vs_plain": round(t_plain / t_batch, 2),
        "latency_ms": {"p50": round(t_batch * 1e3, 3), "p99": round(t_batch * 1e3, 3),
                       "note": "one launch: every query completes with the batch"},
        "exact_vs_plain": exact,
        "plan": {k: bt[k] for k in ("grid_blocks", "small_bin", "wave_bin", "chunk_edges",
                                    "tuned_ms")},
    }
    plan.close()
    single.close()
    return out


# ---------------------------------------------------------------------------
# serving workload: Poisson stream over a resident pool
# ---------------------------------------------------------------------------

def _serve_pool():
    return [
        ("rmat18", lambda: gg.rmat(18, 16, seed=0x5EED0518, perm_seed=0xBEEF0518)),
        ("rmat22", lambda: gg.rmat(22, 16, seed=0x5EED0522, perm_seed=0xBEEF0522)),
        ("rmat26", lambda: gg.rmat(26, 16, seed=0x5EED0526, perm_seed=0xBEEF0526)),
        ("grid4096x4096", lambda: gg.grid(4096, 4096, 0.01, seed=0x5EED0540)),
        ("grid16384x1024", lambda: gg.grid(16384, 1024, 0.01, seed=0x5EED0541)),
    ]


def run_serve(args):
    """Open-loop Poisson stream (mean 20k queries/s, 10k queries) of
    single-source queries over a resident pool; continuous batching in the
    library's serving loop against FIFO one-at-a-time bfs_run."""
    import threading
    import torch
    import paper_2103_13577_amd as pkg
    dev = torch.device("cuda:0")
    nq = args.serve_queries
    t0 = time.time()
    names, gs = [], []
    for name, make in _serve_pool():
        g = make()
        names.append(name)
        gs.append(g)
        log(f"generated {name}: n={g.n} m={g.m} ({time.time() - t0:.0f}s)")
    dgs = [pkg.DeviceGraph.from_csr(g, dev) for g in gs]
    # the serving plan's own single-source settings are not used by the
    # batched path, so it skips the autotuner; the plain baseline is tuned
    # The serving plan's cooperative grid: every level of the batched loop
    # pays two grid barriers whose cost grows with the grid, and the grids'
    # queries run thousands of levels (batched-grid workload: 97-106 us per
    # level at 1024 blocks, 31-47 us at 64-256 for one source); 256 blocks
    # served 24% more queries/s than 1024 on this pool.
    plan = pkg.Plan(dgs, batch_lanes=args.serve_lanes, grid_blocks=args.serve_grid, autotune=-1)
    log("serving plan ready; the baseline plans autotune each graph")
    singles = []
    for gi, dg in enumerate(dgs):
        singles.append(pkg.Plan([dg], grid_blocks=args.grid_blocks))
        log(f"baseline plan for {names[gi]} ready")
    arrivals = gg.poisson_arrivals(nq, 20000.0, seed=0x5EED0550)
    gsel = (gg.draws(0x5EED0551, nq) % np.uint64(len(gs))).astype(np.int64)
    srcs = np.zeros(nq, dtype=np.int64)
    for gi in range(len(gs)):
        idx = np.flatnonzero(gsel == gi)
        srcs[idx] = gg.pick_sources(gs[gi], idx.size, seed=0x5EED0560 + gi)
    # output buffers: a pool per graph bounds the memory held by queries in
    # flight; a query takes a buffer at its arrival, or waits in its graph's
    # queue until one of that graph's buffers is released (that wait counts in
    # its latency; queries of other graphs are not held up)
    per_graph = args.serve_buffers
    pools = [[torch.empty(g.n, dtype=torch.int32, device=dev) for _ in range(per_graph)] for g in gs]
    free = [list(range(per_graph)) for _ in gs]
    waitq = [[] for _ in gs]
    cv = threading.Condition()
    # a seeded sample of the trace whose served answers are kept (a device
    # copy taken as each completes) and compared element by element with
    # bfs_run afterwards, a subset of them also with the CPU oracle
    samp = np.sort(gg.draws(0x5EED0580, min(args.serve_sample, nq)) % np.uint64(nq)).astype(np.int64)
    samp = np.unique(samp)
    samp_set = set(int(q) for q in samp)
    saved = {}
    hstream = torch.cuda.Stream()

    def keep_answer(q, t):
        with torch.cuda.stream(hstream):
            saved[q] = t.clone()
        hstream.synchronize()  # before the buffer is handed to the next query

    done_t = np.zeros(nq)
    tk_info = {}        # ticket -> (query, graph, buffer)
    state = {"completed": 0}
    errors = []

    def submit(q, gi, bi):
        """Submits query q into buffer bi of its graph (called with cv held)."""
        tk = plan.batch_submit([(gi, int(srcs[q]), pools[gi][bi])], pkg.BATCH_STREAMING)
        tk_info[tk] = (q, gi, bi)
        cv.notify_all()

    def consumer():
        while True:
            with cv:
                if state["completed"] == nq:
                    return
            for tk in plan.batch_poll(1024, timeout_us=2000):
                try:
                    r = plan.batch_wait(tk, timeout_us=0)
                    ok = True
                except pkg.BfsError as e:
                    errors.append(str(e))
                    ok = False
                with cv:
                    while tk not in tk_info:  # completed before the submitter recorded it
                        cv.wait()
                    q, gi, bi = tk_info.pop(tk)
                if ok:
                    done_t[q] = r.complete_ns * 1e-9
                    if q in samp_set:
                        keep_answer(q, pools[gi][bi])
                with cv:
                    state["completed"] += 1
                    ncomp = state["completed"]
                    if waitq[gi]:
                        submit(waitq[gi].pop(0), gi, bi)  # the released buffer goes to the next waiting query
                    else:
                        free[gi].append(bi)
                    cv.notify_all()
                if ncomp % 500 == 0:
                    log(f"served {ncomp}/{nq}")

    th = threading.Thread(target=consumer, daemon=True)
    th.start()
    t_start = time.perf_counter()
    t_start_mono = time.monotonic()
    for q in range(nq):
        target = t_start + arrivals[q]
        delay = target - time.perf_counter()
        if delay > 0:
            time.sleep(delay)
        gi = int(gsel[q])
        with cv:
            if free[gi]:
                submit(q, gi, free[gi].pop())
            else:
                waitq[gi].append(q)
    th.join()
    t_end = max(done_t)
    arr_abs = t_start_mono + arrivals  # steady-clock time of each arrival
    lat = done_t - arr_abs
    served_qps = nq / (t_end - arr_abs[0])
    # sequential plain baseline on the seeded sample of the same trace; each
    # plain answer is compared element by element with the served one
    exact = 0
    torch.cuda.synchronize()
    t = time.perf_counter()
    svc = []
    log(f"plain one-at-a-time sample of {samp.size} queries")
    for k, q in enumerate(samp):
        if k % 20 == 0:
            log(f"plain {k}/{samp.size}")
        gi = int(gsel[q])
        ts = time.perf_counter()
        d, _, _ = singles[gi].run(0, int(srcs[q]), dist=pools[gi][0])
        torch.cuda.synchronize()
        svc.append(time.perf_counter() - ts)
        if int(q) in saved and torch.equal(saved[int(q)], d):
            exact += 1
    t_plain = time.perf_counter() - t
    plain_qps = samp.size / t_plain
    # a seeded subset of the sample against the CPU oracle (threads: the
    # oracle releases the interpreter lock)
    import oracle
    from concurrent.futures import ThreadPoolExecutor
    osub = [int(q) for q in samp[:: max(1, samp.size // max(args.serve_oracle, 1))][:args.serve_oracle]]
    log(f"oracle check of {len(osub)} served answers")
    with ThreadPoolExecutor(8) as ex:
        orefs = list(ex.map(lambda q: oracle.bfs(gs[int(gsel[q])], int(srcs[q])), osub))
    oracle_exact = sum(1 for q, r in zip(osub, orefs)
                       if q in saved and np.array_equal(saved[q].cpu().numpy(), r))
    # FIFO one-at-a-time service of the whole trace, with each query's service
    # time drawn from the measured sample of its graph
    by_g = {gi: [s for s, q in zip(svc, samp) if gsel[q] == gi] for gi in range(len(gs))}
    clock, plain_lat = 0.0, []
    for q in range(nq):
        st = by_g[int(gsel[q])]
        service = float(np.mean(st)) if st else float(np.mean(svc))
        clock = max(clock, arrivals[q]) + service
        plain_lat.append(clock - arrivals[q])
    per_graph_lat = {names[gi]: {"p50_ms": round(metrics.percentile(lat[gsel == gi], 50) * 1e3, 2),
                                 "p99_ms": round(metrics.percentile(lat[gsel == gi], 99) * 1e3, 2),
                                 "n": int((gsel == gi).sum())} for gi in range(len(gs))}
    out = {
        "metric": "served queries/sec with p50/p99 latency (Poisson stream, resident pool)",
        "value": round(served_qps, 1), "unit": "queries/s", "n_gpus": 1, "steps": nq,
        "warmup": 0, "ms_per_step": round(1e3 / served_qps, 4), "higher_is_better": True,
        "scaling": "weak", "vs_baseline": None, "dtype": "int32", "data": "synthetic",
        "config": {"workload": "serving: Poisson arrivals, mean 20k queries/s, "
                               f"{nq} queries, uniform over R-MAT 18/22/26 (ef 16) and grids "
                               "4096x4096, 16384x1024 with 1% edge deletions",
                   "lanes_per_graph": args.serve_lanes, "buffers_per_graph": per_graph},
        "latency_ms": {"p50": round(metrics.percentile(lat, 50) * 1e3, 2),
                       "p99": round(metrics.percentile(lat, 99) * 1e3, 2)},
        "per_graph": per_graph_lat,
        "plain_fifo": {"qps": round(plain_qps, 1),
                       "p50_ms": round(metrics.percentile(plain_lat, 50) * 1e3, 2),
                       "p99_ms": round(metrics.percentile(plain_lat, 99) * 1e3, 2),
                       "sample": int(samp.size),
                       "latency_simulated": True,
                       "note": "qps measured on the sample run one at a time; p50/p99 replay the "
                               "whole trace through one FIFO server with each graph's mean "
                               "measured service time"},
        "speedup_qps_vs_plain": round(served_qps / plain_qps, 2),
        "exact": bool(exact == samp.size and oracle_exact == len(osub)),
        "exact_sample": f"{exact}/{samp.size} sampled served answers equal to bfs_run element by "
                        f"element; {oracle_exact}/{len(osub)} of them equal to the CPU oracle",
        "errors": errors[:3],
    }
    plan.close()
    for sp in singles:
        sp.close()
    return out


def run_batch_grid(args):
    """Per-level cost of the batched engine on the serving pool's two
    16M-vertex grids (4096x4096 and 16384x1024, 1% of edges deleted), whose
    thousands of levels dominate the serving latency: one-launch batches of 1
    and 64 sources per grid (uint8 outputs are not enough for these depths:
    int32), against single-source bfs_run (autotuned) on the same sources."""
    import torch
    import paper_2103_13577_amd as pkg
    dev = torch.device("cuda:0")
    pool = [x for x in _serve_pool() if x[0].startswith("grid")]
    gs = [make() for _, make in pool]
    dgs = [pkg.DeviceGraph.from_csr(g, dev) for g in gs]
    plan = pkg.Plan(dgs, batch_lanes=1, autotune=-1, grid_blocks=args.grid_blocks)
    single = pkg.Plan(dgs)
    res = {}
    for gi, (name, _) in enumerate(pool):
        g = gs[gi]
        srcs = [int(s) for s in gg.pick_sources(g, 64, seed=0x5EED0590 + gi)]
        row = {}
        for nsrc in (1, 64):
            outs = [torch.empty(g.n, dtype=torch.int32, device=dev) for _ in range(nsrc)]
            qs = [(gi, s, o) for s, o in zip(srcs[:nsrc], outs)]
            plan.batch_wait(plan.batch_submit(qs, pkg.BATCH_ONE_LAUNCH))  # warm-up
            c0 = plan.batch_counters()
            torch.cuda.synchronize()
            t = time.perf_counter()
            plan.batch_wait(plan.batch_submit(qs, pkg.BATCH_ONE_LAUNCH))
            dt = time.perf_counter() - t
            c1 = plan.batch_counters()
            levels = c1["levels"] - c0["levels"]
            ok = all(torch.equal(o, single.run(gi, s)[0]) for s, o in zip(srcs[:2], outs[:2]))
            row[f"{nsrc}_sources"] = {"ms": round(dt * 1e3, 2), "levels": int(levels),
                                       "us_per_level": round(dt * 1e6 / max(levels, 1), 2),
                                       "launches": int(c1["launches"] - c0["launches"]),
                                       "exact_vs_bfs_run": bool(ok)}
            log(f"{name} {nsrc} sources: {row[f'{nsrc}_sources']}")
        d, _, st = single.run(gi, srcs[0])
        row["bfs_run_one_source"] = {"ms": round(st.ms, 2), "levels": int(st.levels),
                                     "us_per_level": round(st.ms * 1e3 / max(st.levels, 1), 2),
                                     "plan": single.tuning(gi)}
        res[name] = row
    out = {"metric": "batched engine per-level cost on the serving pool's grids",
           "value": res[pool[0][0]]["64_sources"]["us_per_level"], "unit": "us/level",
           "n_gpus": 1, "steps": 1, "warmup": 1, "higher_is_better": False, "scaling": "weak",
           "vs_baseline": None, "dtype": "int32", "data": "synthetic",
           "config": {"workload": "one-launch batches on grids 4096x4096 and 16384x1024 (1% edge "
                                  "deletions), 1 and 64 sources per grid",
                      "batch_tuning": plan.batch_tuning()},
           "grids": res}
    plan.close()
    single.close()
    return out


# ---------------------------------------------------------------------------
# one node's share of R-MAT scale 29 with staged butterfly messages
# ---------------------------------------------------------------------------

def run_share29(args):
    """Partition 0 of a 16-way 1D partition of R-MAT scale 29, edge factor 8:
    only partition 0's rows are resident; the frontier bitmaps span all 2^29
    vertices. Each level runs the local expansion, then merges the 4
    butterfly-stage bitmaps (fanout one, 16 nodes) computed by the oracle from
    the full traversal and staged in device memory."""
    import torch
    import oracle
    import paper_2103_13577_amd as pkg
    dev = torch.device("cuda:0")
    scale, P = args.share_scale, 16
    t0 = time.time()
    g = gg.rmat(scale, 8, seed=0x5EED0029, perm_seed=0xBEEF0029)
    log(f"generated rmat{scale}: n={g.n} m={g.m} in {time.time() - t0:.0f}s")
    b = gg.partition_1d(g.row_ptr, P)
    src = int(gg.pick_sources(g, 1, seed=0xC0FFEE29)[0])
    t0 = time.perf_counter()
    ref = oracle.bfs(g, src)
    t_oracle = time.perf_counter() - t0
    m_all = oracle.edges_scanned(g, ref)
    log(f"oracle full traversal {t_oracle:.1f}s levels={ref.max() + 1}")
    local, inc = oracle.stage(g, ref, b, 0, 2)
    log(f"staged {local.shape[0]} levels x {inc.shape[1]} messages")
    W = (g.n + 63) // 64
    dg = pkg.DeviceGraph.from_csr(g, dev, 0, int(b[1]))
    staged = [[torch.from_numpy(inc[L, j].view(np.int64)).to(dev) for j in range(inc.shape[1])]
              for L in range(local.shape[0])]
    zeros = [torch.zeros(W, dtype=torch.int64, device=dev) for _ in range(inc.shape[1])]
    local_ref = local
    inc_counts = [[int(np.sum(np.bitwise_count(inc[L, j]))) for j in range(inc.shape[1])]
                  for L in range(local.shape[0])]
    del inc
    plan = pkg.Plan([dg])
    dist = torch.empty(g.n, dtype=torch.int32, device=dev)
    e_share = oracle.edges_scanned(g, ref, 0, int(b[1]))

    def one(check):
        ev = []
        t_begin = torch.cuda.Event(enable_timing=True)
        t_begin.record()
        plan.begin(0, src, dist)
        L = 0
        ok = True
        while True:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e2 = torch.cuda.Event(enable_timing=True)
            e0.record()
            addr = plan.expand()
            e1.record()
            if check:
                torch.cuda.synchronize()
                got = torch.empty(W, dtype=torch.int64, device=dev)
                import ctypes
                hip = ctypes.CDLL("libamdhip64.so")
                hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
                hip.hipMemcpy(got.data_ptr(), addr, W * 8, 3)
                exp = local_ref[L] if L < local_ref.shape[0] else np.zeros(W, dtype=np.uint64)
                ok &= bool(np.array_equal(got.cpu().numpy().view(np.uint64), exp))
            msgs = staged[L] if L < len(staged) else zeros
            gnew, _ = plan.merge_frontier(msgs)
            e2.record()
            ev.append((e0, e1, e2))
            if gnew == 0:
                break
            L += 1
        st = plan.finish()
        torch.cuda.synchronize()
        exp_ms = [a.elapsed_time(bb) for a, bb, c in ev]
        mrg_ms = [bb.elapsed_time(c) for a, bb, c in ev]
        total = t_begin.elapsed_time(ev[-1][2])
        return st, exp_ms, mrg_ms, total, ok

    # Vertex-list form of the same messages: a staged message with fewer than
    # n/32 vertices (4 bytes per vertex against n/8 bytes) goes as an ascending
    # list, and the node exports its own global queue as a list when that is
    # the smaller message (what it would send in the first round).
    def to_list(words):
        nz = torch.nonzero(words).flatten()
        ar = torch.arange(64, device=dev, dtype=torch.int64)
        out = []
        for c0 in range(0, nz.numel(), 1 << 21):
            w = nz[c0:c0 + (1 << 21)]
            bits = ((words[w, None] >> ar) & 1).bool()
            out.append((w[:, None] * 64 + ar)[bits])
        return torch.cat(out).to(torch.int32) if out else torch.empty(0, dtype=torch.int32, device=dev)

    forms_all = args.share_forms == "all"
    list_cap = g.n // 32
    lists = []
    for L in range(len(staged)):
        row = []
        for j, m in enumerate(staged[L]):
            row.append(to_list(m) if inc_counts[L][j] < list_cap else m)
        lists.append(row)
    # bytes the node receives per level in each form (each staged message as
    # a bitmap of W words, or in the list form as 4 bytes per vertex when that
    # is smaller)
    bm_bytes = [8 * W * len(row) for row in lists]
    mixed_bytes = [sum(4 * inc_counts[L][j] if m.dtype == torch.int32 else 8 * W
                       for j, m in enumerate(row)) for L, row in enumerate(lists)]
    sendbuf = torch.empty(max(list_cap, 1), dtype=torch.int32, device=dev)
    n_list_msgs = sum(1 for row in lists for m in row if m.dtype == torch.int32)
    log(f"list form: {n_list_msgs} of {sum(len(r) for r in lists)} staged messages go as lists")

    def one_lists(check):
        ev = []
        t_begin = torch.cuda.Event(enable_timing=True)
        t_begin.record()
        plan.begin(0, src, dist)
        L = 0
        ok = True
        sent_lists = 0
        while True:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e2 = torch.cuda.Event(enable_timing=True)
            e0.record()
            plan.expand()
            e1.record()
            try:
                cnt = plan.frontier_list(sendbuf)
                sent_lists += 1
                if check:
                    exp = local_ref[L] if L < local_ref.shape[0] else np.zeros(W, dtype=np.uint64)
                    ok &= int(np.sum(np.bitwise_count(exp))) == cnt
            except pkg.BfsError as err:
                if err.status != 5:
                    raise
            row = lists[L] if L < len(lists) else zeros
            ls = [m for m in row if m.dtype == torch.int32]
            bms = [m for m in row if m.dtype != torch.int32]
            gnew, _ = plan.merge_lists(ls, bitmaps=bms)
            e2.record()
            ev.append((e0, e1, e2))
            if gnew == 0:
                break
            L += 1
        plan.finish()
        torch.cuda.synchronize()
        exp_ms = [a.elapsed_time(bb) for a, bb, c in ev]
        mrg_ms = [bb.elapsed_time(c) for a, bb, c in ev]
        return exp_ms, mrg_ms, t_begin.elapsed_time(ev[-1][2]), ok, sent_lists

    if forms_all:
        _, _, _, ok_l, _ = one_lists(check=True)
        exact_lists = ok_l and np.array_equal(dist.cpu().numpy(), ref)
        log(f"list form exact={exact_lists}")

    # Direction-optimizing: a level whose frontier holds at least n/24
    # vertices runs Phase 1 bottom-up (bfs_expand_bottom_up); its staged
    # messages are then every node's owned vertices of the next level.
    sizes = np.bincount(ref[ref >= 0], minlength=len(staged) + 2)
    bu_levels = sorted(L for L in range(len(staged)) if sizes[L] * 24 >= g.n)
    plan_do = None
    if forms_all:
        bu_local, bu_inc = oracle.stage_bottom_up(g.n, ref, b, 0, 2, levels=set(bu_levels))
        staged_do = [[torch.from_numpy(bu_inc[L, j].view(np.int64)).to(dev) for j in range(bu_inc.shape[1])]
                     if L in bu_levels else staged[L] for L in range(len(staged))]
        del bu_inc
        log(f"direction-optimizing: bottom-up levels {bu_levels}")
        plan_do = pkg.Plan([dg], direction=pkg.DIR_OPTIMIZING)

    def one_do(check):
        ev = []
        t_begin = torch.cuda.Event(enable_timing=True)
        t_begin.record()
        plan_do.begin(0, src, dist)
        L = 0
        ok = True
        while True:
            e0 = torch.cuda.Event(enable_timing=True)
            e1 = torch.cuda.Event(enable_timing=True)
            e2 = torch.cuda.Event(enable_timing=True)
            e0.record()
            up = L in bu_levels
            addr = plan_do.expand_bottom_up() if up else plan_do.expand()
            e1.record()
            if check:
                torch.cuda.synchronize()
                got = torch.empty(W, dtype=torch.int64, device=dev)
                import ctypes
                hip = ctypes.CDLL("libamdhip64.so")
                hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
                hip.hipMemcpy(got.data_ptr(), addr, W * 8, 3)
                src_bm = bu_local if up else local_ref
                exp = src_bm[L] if L < src_bm.shape[0] else np.zeros(W, dtype=np.uint64)
                ok &= bool(np.array_equal(got.cpu().numpy().view(np.uint64), exp))
            msgs = staged_do[L] if L < len(staged_do) else zeros
            gnew, _ = plan_do.merge_frontier(msgs)
            e2.record()
            ev.append((e0, e1, e2))
            if gnew == 0:
                break
            L += 1
        st_do = plan_do.finish()
        torch.cuda.synchronize()
        exp_ms = [a.elapsed_time(bb) for a, bb, c in ev]
        mrg_ms = [bb.elapsed_time(c) for a, bb, c in ev]
        return exp_ms, mrg_ms, t_begin.elapsed_time(ev[-1][2]), ok, st_do

    if forms_all:
        _, _, _, ok_d, _ = one_do(check=True)
        exact_do = ok_d and np.array_equal(dist.cpu().numpy(), ref)
        log(f"direction-optimizing exact={exact_do}")

    st, _, _, _, ok = one(check=True)
    exact = ok and np.array_equal(dist.cpu().numpy(), ref)
    runs = [one(check=False) for _ in range(max(args.steps if args.steps < 64 else 3, 1))]
    if forms_all:
        runs_l = [one_lists(check=False) for _ in range(len(runs))]
        tot_l = np.array([r[2] for r in runs_l])
        runs_d = [one_do(check=False) for _ in range(len(runs))]
        tot_d = np.array([r[2] for r in runs_d])
    tot = np.array([r[3] for r in runs])
    exp_ms = np.mean([r[1] for r in runs], axis=0)
    mrg_ms = np.mean([r[2] for r in runs], axis=0)
    k = 4
    merge_bytes = (k + 3) * W * 8
    mrg_gbs = merge_bytes / (np.mean(mrg_ms) * 1e-3) / 1e9
    # the dense expansion of the share: 4 B per scanned edge and 16 B of row
    # offsets per frontier vertex (counted on the device), over its launches
    exp_bytes = 4.0 * st.dense_edges + 16.0 * st.dense_frontier
    exp_gbs = exp_bytes / (float(np.sum(exp_ms)) * 1e-3) / 1e9
    share_traffic = measured_share_traffic()
    out = {
        "metric": "GTEPS over the share's scanned edges (one node of 16, staged butterfly messages)",
        "value": round(metrics.gteps(e_share, float(np.median(tot)) * 1e-3), 3), "unit": "GTEPS",
        "n_gpus": 1, "steps": len(runs), "warmup": 1, "ms_per_step": round(float(np.median(tot)), 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None, "dtype": "int32",
        "data": "synthetic",
        "config": {"workload": f"partition 0 of 16 of R-MAT scale {scale} edge factor 8, int32 CSR "
                               f"share, 2^{scale}-bit frontier bitmaps, 4 staged butterfly-stage bitmaps "
                               "per level (fanout one)",
                   "n": g.n, "m_directed": g.m, "share_rows": int(b[1]),
                   "share_edges": int(g.row_ptr[b[1]]), "levels": int(st.levels)},
        "per_level_ms": {"expand": [round(x, 3) for x in exp_ms], "merge": [round(x, 3) for x in mrg_ms]},
        "roofline": {"bound": "hbm", "kernel": "k_merge", "achieved": round(mrg_gbs, 1),
                     "peak": HBM_PEAK_GBS, "unit": "GB/s", "frac": round(mrg_gbs / HBM_PEAK_GBS, 4),
                     "traffic": share_traffic["k_merge"]["hbm_bytes_per_launch"] if share_traffic else None,
                     "bytes_per_launch": int(merge_bytes),
                     "launches": len(runs) * len(mrg_ms)},
        "roofline_expansion": {"bound": "hbm", "kernel": "k_expand", "achieved": round(exp_gbs, 1),
                               "peak": HBM_PEAK_GBS, "unit": "GB/s",
                               "frac": round(exp_gbs / HBM_PEAK_GBS, 4),
                               "bytes_per_traversal": int(exp_bytes),
                               "launches_per_traversal": len(exp_ms),
                               "ms_per_traversal": round(float(np.sum(exp_ms)), 3),
                               "traffic_per_traversal": (share_traffic["k_expand"]["hbm_bytes_per_traversal"]
                                                         if share_traffic else None)},
        **({"traffic_source": "profiles/traffic_share29.json"} if share_traffic else {}),
        "exact": bool(exact),
        "cpu_baseline": {"value": round(metrics.gteps(m_all, t_oracle), 4), "unit": "GTEPS",
                         "cores": 1, "kind": "oracle",
                         "sample": f"the oracle's full traversal of the whole scale-{scale} graph "
                                   f"from the same source ({t_oracle:.0f} s)"},
        "edges_scanned_share": int(e_share),
    }
    if forms_all:
        out["list_messages"] = {
            "note": "same traversal with every staged message of fewer than n/32 vertices sent as "
                    "a vertex list (bfs_merge_lists) and the node's own global queue exported as a "
                    "list when it is the smaller message (bfs_frontier_list); merge time includes "
                    "the export",
            "gteps": round(metrics.gteps(e_share, float(np.median(tot_l)) * 1e-3), 3),
            "ms_per_step": round(float(np.median(tot_l)), 3),
            "messages_as_lists": n_list_msgs, "exports_as_lists": int(runs_l[0][4]),
            "received_bytes_per_level": {"bitmaps": bm_bytes, "lists_where_smaller": mixed_bytes},
            "per_level_ms": {"expand": [round(x, 3) for x in np.mean([r[0] for r in runs_l], axis=0)],
                             "merge": [round(x, 3) for x in np.mean([r[1] for r in runs_l], axis=0)]},
            "exact": bool(exact_lists)}
        out["direction_optimizing"] = {
            "note": "same share and source; levels whose frontier holds at least n/24 vertices run "
                    "Phase 1 bottom-up (bfs_expand_bottom_up) with the matching staged messages "
                    "(each node's owned vertices of the next level); GTEPS over the same share "
                    "edges",
            "gteps": round(metrics.gteps(e_share, float(np.median(tot_d)) * 1e-3), 3),
            "ms_per_step": round(float(np.median(tot_d)), 3),
            "bottom_up_levels": bu_levels,
            "adjacency_entries_examined_bottom_up": int(runs_d[0][4].bottom_up_edges),
            "per_level_ms": {"expand": [round(x, 3) for x in np.mean([r[0] for r in runs_d], axis=0)],
                             "merge": [round(x, 3) for x in np.mean([r[1] for r in runs_d], axis=0)]},
            "exact": bool(exact_do)}
    plan.close()
    if plan_do is not None:
        plan_do.close()
    copy_gbs = measured_copy_gbs()
    for key in ("roofline", "roofline_expansion"):
        out[key]["measured_copy_gbs"] = copy_gbs
        out[key]["frac_of_copy"] = round(out[key]["achieved"] / copy_gbs, 4)
    return out


def _bench_line(log_path):
    """The JSON line a bench.py run printed into its log."""
    with open(log_path) as f:
        for line in f:
            if line.startswith('{"metric"'):
                return json.loads(line)
    raise SystemExit(f"no bench JSON line in {log_path}")


def _short(name):
    """Kernel name without namespaces, template arguments and parameters."""
    import re
    n = name.strip('"').replace("(anonymous namespace)", "")
    while True:  # drop innermost template argument lists
        m = re.sub(r"<[^<>]*>", "", n)
        if m == n:
            break
        n = m
    n = n.split("(")[0].strip()
    return n.split("::")[-1].split()[-1] if n else name


def _dense_series(kname):
    """The dense expansion runs as k_expand, or as k_expand_wide on levels with
    a large LDS hub copy: profiles treat both as one series."""
    return "k_expand+k_expand_wide" if kname.split("+")[0] == "k_expand" else kname


def summarize_pmc(args):
    """Writes profiles/traffic_rmat24.json from rocprofv3 --pmc runs: the mean
    FETCH_SIZE and WRITE_SIZE (KiB per dispatch) of each kernel over the timed
    region's launches (the last `launches` dispatches named in the run's bench
    line), scaled by what the same counters read for a plain device copy of
    known size."""
    import csv
    from collections import defaultdict

    fd, wd, cfd, cwd, fetch_log = args.summarize_pmc
    line = _bench_line(fetch_log)
    timed = line["roofline"].get("launches", 0)

    group = _dense_series(line["roofline"]["kernel"])
    members = set(group.split("+"))

    def per_kernel(d, counter, last=0):
        vals = defaultdict(lambda: defaultdict(float))
        with open(os.path.join(d, "run_counter_collection.csv")) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] != counter:
                    continue
                k = _short(r["Kernel_Name"])
                if k in members:
                    k = group  # the roofline's kernel (or kernels) as one series
                vals[k][int(r["Dispatch_Id"])] += float(r["Counter_Value"])
        out, cnt = {}, {}
        for k, per in vals.items():
            ids = sorted(per)
            if last and k in (group, "k_merge", "k_merge_g"):
                ids = ids[-last:]
            out[k] = sum(per[i] for i in ids) / len(ids)
            cnt[k] = len(ids)
        return out, cnt

    fetch, nf = per_kernel(fd, "FETCH_SIZE", timed)
    write, _ = per_kernel(wd, "WRITE_SIZE", timed)
    cf, _ = per_kernel(cfd, "FETCH_SIZE")
    cw, _ = per_kernel(cwd, "WRITE_SIZE")
    copy_kib = args.copy_bytes / 1024.0
    ck = [k for k in cf if "copy" in k.lower()][0]
    fscale, wscale = copy_kib / cf[ck], copy_kib / cw[ck]
    out = {"workload": "R-MAT scale 24 edge factor 16, " + line["config"]["workload"].split(", ")[-1],
           "plan": line["config"].get("plan"),
           "commands": args.pmc_commands,
           "kernel_source_hash": kernel_source_hash(),
           "copy_probe": {"bytes": args.copy_bytes, "fetch_kib": cf[ck], "write_kib": cw[ck],
                          "fetch_scale": fscale, "write_scale": wscale},
           "kernels": {}}
    for k in fetch:
        if k not in (group, "k_merge", "k_merge_g", "k_reset"):
            continue
        fb = fetch[k] * fscale * 1024
        wb = write.get(k, 0.0) * wscale * 1024
        out["kernels"][k] = {"dispatches": nf[k], "fetch_bytes_per_launch": int(fb),
                             "write_bytes_per_launch": int(wb),
                             "hbm_bytes_per_launch": int(fb + wb)}
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", "traffic_rmat24.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


def summarize_trace(args):
    """Writes a short markdown summary of a rocprofv3 --kernel-trace --stats
    run of bench.py: the command, the busiest kernels over the whole run, and
    the dominant kernel's average duration over the timed region (its last
    `launches` dispatches) next to what bench.py measured with HIP events."""
    import csv
    from collections import defaultdict

    d, log, out_name, command = args.summarize_trace
    line = _bench_line(log)
    roof = line.get("roofline")
    rows = list(csv.DictReader(open(os.path.join(d, "run_kernel_stats.csv"))))
    if roof is None:
        # no roofline kernel (e.g. the batched engine's per-level workload):
        # the kernel table and the line's own figures only
        md = [f"# rocprofv3 kernel trace: {line['config']['workload']}", "",
              "Command (from the repository root):", "", "```", command, "```", "",
              f"bench.py line: value {line['value']} {line['unit']}", "",
              "```", json.dumps({k: line[k] for k in line if k not in ('config',)}, indent=1)[:3000], "```",
              "", "| kernel | calls | total ms | average us | share % |", "|---|---|---|---|---|"]
        for r in rows[:12]:
            md.append(f"| `{_short(r['Name'])}` | {r['Calls']} | {int(r['TotalDurationNs']) / 1e6:.2f} | "
                      f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} |")
        os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
        with open(os.path.join(ROOT, "profiles", out_name), "w") as f:
            f.write("\n".join(md) + "\n")
        print("\n".join(md))
        return
    kname, timed = roof["kernel"], roof.get("launches", 0)
    kname = _dense_series(kname)
    members = set(kname.split("+"))
    sel = []
    with open(os.path.join(d, "run_kernel_trace.csv")) as f:
        for r in csv.DictReader(f):
            if _short(r["Kernel_Name"]) in members:
                sel.append((int(r["Dispatch_Id"]), int(r["End_Timestamp"]) - int(r["Start_Timestamp"])))
    sel.sort()
    prev = []
    if timed:
        # a line whose kernel was timed on a second pass: the pass before it
        # (the value's captured-graph replays) launched as many of the kernel
        prev = sel[-2 * timed:-timed] if line.get("roofline_timing") else []
        sel = sel[-timed:]
    avg_ms = sum(x for _, x in sel) / max(len(sel), 1) / 1e6
    md = [f"# rocprofv3 kernel trace: {line['config']['workload']}", "",
          "Command (from the repository root):", "", "```", command, "```", "",
          f"bench.py line: value {line['value']} {line['unit']}, ms_per_step {line['ms_per_step']}, "
          f"plan {json.dumps(line['config'].get('plan'))}", "",
          f"Dominant kernel `{kname}`: {len(sel)} launches in the timed region, "
          f"average {avg_ms:.4f} ms (rocprofv3) vs {roof['avg_launch_ms']} ms (HIP events in "
          f"bench.py); roofline achieved {roof['achieved']} {roof['unit']} "
          f"({roof['frac']} of {roof['peak']}), {roof['bytes_per_launch']} algorithmic bytes "
          f"per launch.", "",
          *([f"The same kernel's {len(prev)} dispatches of the value's pass (level steps replayed "
             f"as a captured graph) average {sum(x for _, x in prev) / len(prev) / 1e6:.4f} ms.", ""]
            if prev else []),
          "Whole run (plan creation and autotuning included):", "",
          "| kernel | calls | total ms | average us | share % |", "|---|---|---|---|---|"]
    for r in rows[:12]:
        md.append(f"| `{_short(r['Name'])}` | {r['Calls']} | {int(r['TotalDurationNs']) / 1e6:.2f} | "
                  f"{float(r['AverageNs']) / 1e3:.1f} | {float(r['Percentage']):.1f} |")
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", out_name), "w") as f:
        f.write("\n".join(md) + "\n")
    print("\n".join(md))


def summarize_share_pmc(args):
    """Writes profiles/traffic_share29.json from two rocprofv3 --pmc runs
    (FETCH_SIZE, then WRITE_SIZE) of `bench.py --workload share29
    --share-forms topdown`: the mean HBM bytes per launch of k_merge and per
    traversal of k_expand over the timed traversals (the last `steps` x
    `levels` dispatches of each), scaled by the copy-probe factors recorded in
    profiles/traffic_rmat24.json."""
    import csv
    from collections import defaultdict

    fd, wd, run_log = args.summarize_share_pmc
    line = _bench_line(run_log)
    steps, levels = int(line["steps"]), int(line["config"]["levels"])
    with open(os.path.join(ROOT, "profiles", "traffic_rmat24.json")) as f:
        probe = json.load(f)["copy_probe"]

    def per_dispatch(d, counter):
        vals = defaultdict(lambda: defaultdict(float))
        with open(os.path.join(d, "run_counter_collection.csv")) as f:
            for r in csv.DictReader(f):
                if r["Counter_Name"] == counter:
                    vals[_short(r["Kernel_Name"])][int(r["Dispatch_Id"])] += float(r["Counter_Value"])
        return {k: [v[i] for i in sorted(v)][-steps * levels:] for k, v in vals.items()}

    fetch = per_dispatch(fd, "FETCH_SIZE")
    write = per_dispatch(wd, "WRITE_SIZE")
    out = {"workload": line["config"]["workload"], "steps": steps, "levels": levels,
           "commands": [f"rocprofv3 --pmc FETCH_SIZE -d {fd} -o run --output-format csv -- python -u bench.py "
                        "--workload share29 --share-forms topdown --steps 1",
                        f"rocprofv3 --pmc WRITE_SIZE -d {wd} -o run --output-format csv -- python -u bench.py "
                        "--workload share29 --share-forms topdown --steps 1"],
           "kernel_source_hash": kernel_source_hash(),
           "copy_probe": probe, "kernels": {}}
    for k in ("k_expand", "k_merge"):
        fb = [x * probe["fetch_scale"] * 1024 for x in fetch.get(k, [])]
        wb = [x * probe["write_scale"] * 1024 for x in write.get(k, [])]
        if not fb or len(fb) != len(wb):
            continue
        rec = {"dispatches": len(fb), "fetch_bytes_per_launch": int(sum(fb) / len(fb)),
               "write_bytes_per_launch": int(sum(wb) / len(wb)),
               "hbm_bytes_per_launch": int((sum(fb) + sum(wb)) / len(fb)),
               "hbm_bytes_per_traversal": int((sum(fb) + sum(wb)) / steps),
               "per_level_mb": [round((a + b) / 1e6, 1) for a, b in zip(fb[-levels:], wb[-levels:])]}
        out["kernels"][k] = rec
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", "traffic_share29.json"), "w") as f:
        json.dump(out, f, indent=1)
    print(json.dumps(out))


def summarize_counters(args):
    """Writes a markdown table of rocprofv3 --pmc counters of a bench.py run:
    for the dominant kernel series the mean per launch over the timed
    region's launches, for every other kernel the mean per dispatch over the
    dispatches from the first timed launch on."""
    import csv
    from collections import defaultdict

    d, log, out_name, command = args.summarize_counters
    line = _bench_line(log)
    group = _dense_series(line["roofline"]["kernel"])
    members = set(group.split("+"))
    timed = line["roofline"].get("launches", 0)
    per = defaultdict(lambda: defaultdict(lambda: defaultdict(float)))
    with open(os.path.join(d, "run_counter_collection.csv")) as f:
        for r in csv.DictReader(f):
            k = _short(r["Kernel_Name"])
            per[k][int(r["Dispatch_Id"])][r["Counter_Name"]] += float(r["Counter_Value"])
    dom = sorted(i for k in members for i in per.get(k, {}))
    dom = dom[-timed:] if timed else dom
    first = dom[0] if dom else 0
    counters = sorted({c for k in per for i in per[k] for c in per[k][i]})
    rows = []
    for k in sorted(per, key=lambda k: (k not in members, k)):
        ids = [i for i in per[k] if (i in dom if k in members else i >= first)]
        if not ids:
            continue
        means = {c: sum(per[k][i].get(c, 0.0) for i in ids) / len(ids) for c in counters}
        rows.append((k, len(ids), means))
    md = [f"# rocprofv3 counters: {line['config']['workload']}", "",
          "Command (from the repository root):", "", "```", command, "```", "",
          f"Means per dispatch over the timed region (the last {timed} launches of "
          f"`{group}`, and every other dispatch from the first of them on).", "",
          "| kernel | dispatches | " + " | ".join(counters) + " |",
          "|---|---|" + "---|" * len(counters)]
    for k, n, means in rows:
        md.append(f"| `{k}` | {n} | " + " | ".join(f"{means[c]:.4g}" for c in counters) + " |")
    os.makedirs(os.path.join(ROOT, "profiles"), exist_ok=True)
    with open(os.path.join(ROOT, "profiles", out_name), "w") as f:
        f.write("\n".join(md) + "\n")
    print("\n".join(md))


def measured_copy_gbs(nbytes=1 << 30, reps=5):
    """HBM rate of a plain device-to-device copy (bytes read + bytes written
    per second), timed with HIP events: the practical ceiling that a
    streaming kernel reaches on this device, reported beside the nominal
    peak."""
    import torch
    x = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda:0")
    y = torch.empty_like(x)
    y.copy_(x)
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record()
    for _ in range(reps):
        y.copy_(x)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / reps
    del x, y
    torch.cuda.empty_cache()
    return round(2.0 * nbytes / (ms * 1e-3) / 1e9, 1)


def copy_probe(nbytes):
    """A plain device copy of known size, for scaling the HBM byte counters."""
    import torch
    x = torch.ones(nbytes // 4, dtype=torch.int32, device="cuda:0")
    y = torch.empty_like(x)
    for _ in range(3):
        y.copy_(x)
    torch.cuda.synchronize()
    print(json.dumps({"copy_probe_bytes": nbytes, "note": "each copy reads and writes this many bytes"}))


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=64)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--workload", default="rmat24",
                    choices=["rmat24", "rmat14", "batch", "batch-grid", "serve", "share29"])
    ap.add_argument("--loop-mode", type=int, default=-1,
                    help="-1: for rmat24 the pinned headline plan (host-driven loop, each "
                         "expansion launch timed), else the tuned loop; 0: tuned; 1..4: BFS_LOOP_*")
    ap.add_argument("--grid-blocks", type=int, default=0)
    ap.add_argument("--small-bin", type=int, default=0)
    ap.add_argument("--wave-bin", type=int, default=0)
    ap.add_argument("--chunk-edges", type=int, default=0)
    ap.add_argument("--relabel", type=int, default=0, help="0 auto, 1 on, -1 off")
    ap.add_argument("--autotune", type=int, default=0, help="0 auto, 1 on, -1 off")
    ap.add_argument("--hot-words", type=int, default=0, help="0 tuned, -1 none")
    ap.add_argument("--sparse-div", type=int, default=0, help="0 tuned, -1 never queue-only")
    ap.add_argument("--direction", type=int, default=0,
                    help="0 top-down (the paper's method), 1 direction-optimizing")
    ap.add_argument("--mark-mode", type=int, default=0,
                    help="0/1: byte marks on dense single-node levels, -1: atomic bitmap ORs")
    ap.add_argument("--auto-detail", type=int, default=1,
                    help="rmat24 headline: also run the fully autotuned plan before the timed "
                         "region and report it in the detail (0 skips it)")
    ap.add_argument("--no-cpu-baseline", dest="cpu_baseline", action="store_false")
    ap.add_argument("--cpu-budget", type=float, default=20.0)
    ap.add_argument("--copy-probe", type=int, default=0)
    ap.add_argument("--serve-queries", type=int, default=10000)
    ap.add_argument("--serve-lanes", type=int, default=1)
    ap.add_argument("--serve-grid", type=int, default=256,
                    help="cooperative grid of the serving plan's batched loop")
    ap.add_argument("--serve-buffers", type=int, default=96)
    ap.add_argument("--serve-sample", type=int, default=200)
    ap.add_argument("--serve-oracle", type=int, default=16,
                    help="sampled served answers also checked against the CPU oracle")
    ap.add_argument("--share-scale", type=int, default=29)
    ap.add_argument("--share-forms", choices=["all", "topdown"], default="all",
                    help="share workload: also the list-message and direction-optimizing forms, "
                         "or the top-down traversals alone (for counter runs)")
    ap.add_argument("--summarize-share-pmc", nargs=3, metavar=("FETCH_DIR", "WRITE_DIR", "RUN_LOG"))
    ap.add_argument("--summarize-pmc", nargs=5, metavar=("FETCH_DIR", "WRITE_DIR", "COPY_FETCH_DIR",
                                                         "COPY_WRITE_DIR", "FETCH_RUN_LOG"))
    ap.add_argument("--summarize-trace", nargs=4, metavar=("TRACE_DIR", "RUN_LOG", "OUT_NAME",
                                                           "COMMAND"))
    ap.add_argument("--summarize-counters", nargs=4, metavar=("PMC_DIR", "RUN_LOG", "OUT_NAME",
                                                              "COMMAND"))
    ap.add_argument("--pmc-commands", nargs="*", default=[],
                    help="the rocprofv3 commands the --summarize-pmc runs came from (recorded)")
    ap.add_argument("--copy-bytes", type=int, default=1 << 30)
    args = ap.parse_args()
    if args.gpus != 1:
        print(f"bench.py runs on one GPU only (got --gpus {args.gpus}): the library has no "
              f"multi-GPU path; the exchange between nodes goes through the caller's "
              f"exchange callback or the step-wise calls, and none is driven here.",
              file=sys.stderr)
        sys.exit(2)
    if args.copy_probe:
        copy_probe(args.copy_probe)
        return
    if args.summarize_pmc:
        summarize_pmc(args)
        return
    if args.summarize_trace:
        summarize_trace(args)
        return
    if args.summarize_counters:
        summarize_counters(args)
        return
    if args.summarize_share_pmc:
        summarize_share_pmc(args)
        return
    if args.workload == "rmat24":
        out = run_single(args, "rmat24", 24, 16)
    elif args.workload == "rmat14":
        out = run_single(args, "rmat14", 14, 8)
    elif args.workload == "batch":
        out = run_batch(args)
    elif args.workload == "batch-grid":
        out = run_batch_grid(args)
    elif args.workload == "serve":
        out = run_serve(args)
    else:
        out = run_share29(args)
    print(json.dumps(out), flush=True)


if __name__ == "__main__":
    main()
