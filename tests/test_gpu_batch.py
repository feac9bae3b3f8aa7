"""GPU parity of the batched multi-source path and of the serving loop.

Every query's distances must equal the oracle's for its (graph, source),
bit for bit (uint8 with 255 = unreached, or int32 with -1), whether the query
ran alone, in a one-launch batch, or joined a running batch.
"""
import time

import numpy as np
import pytest

import graphgen as gg
import oracle
import paper_2103_13577_amd as pkg

pytestmark = pytest.mark.gpu


def _graphs_small():
    return [gg.rmat(s, 8, seed=900 + s, perm_seed=950 + s) for s in (9, 10, 11, 12)] + \
           [gg.grid(40, 30, 0.02, seed=5), gg.path_graph(200), gg.star_graph(300),
            gg.disjoint_union(gg.cycle_graph(50), gg.complete_graph(20))]


def _oracle_out(g, s, dtype):
    d = oracle.bfs(g, int(s))
    if dtype == "u8":
        return np.where(d < 0, 255, d).astype(np.uint8)
    return d


@pytest.mark.parametrize("lw", [1, 2, 4])
def test_one_launch_batch_u8(gpu, lw):
    import torch
    gs = _graphs_small()
    dgs = [pkg.DeviceGraph.from_csr(g, gpu) for g in gs]
    plan = pkg.Plan(dgs, batch_lanes=lw)
    qs, refs = [], []
    for gi, g in enumerate(gs):
        srcs = gg.pick_sources(g, min(64 * lw, 40 + 7 * gi), seed=1000 + gi)
        srcs[:3] = srcs[0]  # duplicate sources share a batch
        for s in srcs:
            out = torch.empty(g.n, dtype=torch.uint8, device=gpu)
            qs.append((gi, int(s), out))
            refs.append(_oracle_out(g, s, "u8"))
    print(f"[gpu] batch lw={lw} queries={len(qs)}", flush=True)
    t = plan.batch_submit(qs, pkg.BATCH_ONE_LAUNCH)
    r = plan.batch_wait(t)
    assert r.status == 0 and r.nq == len(qs)
    for (gi, s, out), ref in zip(qs, refs):
        assert np.array_equal(out.cpu().numpy(), ref), (gi, s)
    plan.close()


def test_more_queries_than_slots_int32(gpu):
    """300 queries on one graph with 64 slots: admission waits for free slots,
    released slots are cleared and reused, every answer is exact."""
    import torch
    g = gg.rmat(11, 8, seed=31, perm_seed=32)
    plan = pkg.Plan([pkg.DeviceGraph.from_csr(g, gpu)], batch_lanes=1)
    srcs = gg.pick_sources(g, 300, seed=33)
    outs = [torch.empty(g.n, dtype=torch.int32, device=gpu) for _ in srcs]
    t = plan.batch_submit([(0, int(s), o) for s, o in zip(srcs, outs)], pkg.BATCH_ONE_LAUNCH)
    plan.batch_wait(t)
    for s, o in zip(srcs, outs):
        assert np.array_equal(o.cpu().numpy(), oracle.bfs(g, int(s))), int(s)
    plan.close()


def test_depth_overflow_u8_and_int32_ok(gpu):
    import torch
    g = gg.path_graph(300)
    plan = pkg.Plan([pkg.DeviceGraph.from_csr(g, gpu)], batch_lanes=1)
    o8 = torch.empty(g.n, dtype=torch.uint8, device=gpu)
    t = plan.batch_submit([(0, 0, o8)])
    with pytest.raises(pkg.BfsError) as e:
        plan.batch_wait(t)
    assert e.value.status == 4
    o32 = torch.empty(g.n, dtype=torch.int32, device=gpu)
    t = plan.batch_submit([(0, 0, o32), (0, 299, torch.empty(g.n, dtype=torch.uint8, device=gpu))])
    with pytest.raises(pkg.BfsError):
        plan.batch_wait(t)  # the uint8 query overflows; the int32 one is exact
    assert np.array_equal(o32.cpu().numpy(), oracle.bfs(g, 0))
    t = plan.batch_submit([(0, 150, o8)])  # depth 150 fits
    plan.batch_wait(t)
    assert np.array_equal(o8.cpu().numpy(), _oracle_out(g, 150, "u8"))
    plan.close()


def test_streaming_alone_equals_in_mix(gpu):
    """Queries submitted while others are running (continuous batching) give
    the same answer as the same query run alone through bfs_run."""
    import torch
    gs = [gg.rmat(13, 8, seed=41, perm_seed=42), gg.grid(64, 64, 0.01, seed=43),
          gg.lollipop_graph(64, 300)]
    dgs = [pkg.DeviceGraph.from_csr(g, gpu) for g in gs]
    plan = pkg.Plan(dgs, batch_lanes=1)
    alone = pkg.Plan(dgs)
    rng = np.random.default_rng(7)
    tickets, items = [], []
    for wave in range(6):
        batch = []
        for _ in range(25):
            gi = int(rng.integers(0, len(gs)))
            s = int(gg.pick_sources(gs[gi], 1, seed=int(rng.integers(1 << 30)))[0])
            out = torch.empty(gs[gi].n, dtype=torch.int32, device=gpu)
            batch.append((gi, s, out))
        tickets.append((plan.batch_submit(batch, pkg.BATCH_STREAMING), len(batch)))
        items += batch
        time.sleep(0.002)
    seen = set()
    while len(seen) < len(tickets):
        seen.update(plan.batch_poll(64, timeout_us=2_000_000))
    assert seen == {t for t, _ in tickets}
    for t, nq in tickets:
        plan.batch_wait(t)
        times = plan.batch_times(t, nq)
        assert np.all(times > 0)
    for gi, s, out in items:
        d, _, _ = alone.run(gi, s)
        assert np.array_equal(out.cpu().numpy(), d.cpu().numpy()), (gi, s)
        assert np.array_equal(out.cpu().numpy(), oracle.bfs(gs[gi], s)), (gi, s)
    c = plan.batch_counters()
    print(f"[gpu] streaming counters {c}", flush=True)
    assert c["admitted"] == len(items)
    # continuous batching: queries joined while others were in flight
    assert c["admitted_midflight"] > 0 and c["max_inflight"] > 1
    assert c["inflight_bytes"] == 0
    plan.close()
    alone.close()


def test_memory_budget_admission(gpu):
    """Streaming queries are admitted by memory (a query's int32 output plus
    its lane share): under a budget of two and a half queries at most two are
    in flight at once, every query still completes exactly, and the budget is
    the only limit (the plan has 64 slots)."""
    import torch
    g = gg.rmat(14, 8, seed=61, perm_seed=62)
    dg = pkg.DeviceGraph.from_csr(g, gpu)
    probe = pkg.Plan([dg], batch_lanes=1, autotune=-1)
    qb = probe.batch_query_bytes(0, pkg.OUT_I32)
    assert qb == 4 * g.n + 24 * g.n // 64
    assert probe.batch_query_bytes(0, pkg.OUT_U8) == g.n + 24 * g.n // 64
    probe.close()
    budget = qb * 5 // 2
    plan = pkg.Plan([dg], batch_lanes=1, autotune=-1, mem_budget_bytes=budget)
    srcs = [int(s) for s in gg.pick_sources(g, 12, seed=63)]
    outs = [torch.empty(g.n, dtype=torch.int32, device=gpu) for _ in srcs]
    t = plan.batch_submit([(0, s, o) for s, o in zip(srcs, outs)], pkg.BATCH_STREAMING)
    plan.batch_wait(t)
    for s, o in zip(srcs, outs):
        assert np.array_equal(o.cpu().numpy(), oracle.bfs(g, s)), s
    c = plan.batch_counters()
    print(f"[gpu] budget counters {c}", flush=True)
    assert c["admitted"] == len(srcs)
    assert c["max_inflight"] == 2 and c["max_inflight_bytes"] <= budget
    assert c["inflight_bytes"] == 0
    plan.close()


def test_memory_budget_refuses_never_admissible(gpu):
    """A query whose own admission cost exceeds the budget can never run: the
    submission is refused with BFS_ERR_CAPACITY (nothing of it is queued), and
    a query that fits is still served."""
    import torch
    g = gg.rmat(13, 8, seed=64, perm_seed=65)
    dg = pkg.DeviceGraph.from_csr(g, gpu)
    budget = 2 * g.n  # fits a uint8 query (n + 24n/64), not an int32 one (4n + 24n/64)
    plan = pkg.Plan([dg], batch_lanes=1, autotune=-1, mem_budget_bytes=budget)
    s = int(gg.pick_sources(g, 1, seed=66)[0])
    o32 = torch.empty(g.n, dtype=torch.int32, device=gpu)
    o8 = torch.empty(g.n, dtype=torch.uint8, device=gpu)
    with pytest.raises(pkg.BfsError) as e:
        plan.batch_submit([(0, s, o8), (0, s, o32)], pkg.BATCH_STREAMING)
    assert e.value.status == 5
    assert plan.batch_counters()["admitted"] == 0
    plan.batch_wait(plan.batch_submit([(0, s, o8)], pkg.BATCH_STREAMING))
    assert np.array_equal(o8.cpu().numpy(), _oracle_out(g, s, "u8"))
    plan.close()


def test_batch_errors(gpu):
    import torch
    g = gg.rmat(9, 8, seed=1, perm_seed=2)
    dg = pkg.DeviceGraph.from_csr(g, gpu)
    plain = pkg.Plan([dg])
    out = torch.empty(g.n, dtype=torch.uint8, device=gpu)
    with pytest.raises(pkg.BfsError) as e:
        plain.batch_submit([(0, 0, out)])
    assert e.value.status == 5
    plain.close()
    plan = pkg.Plan([dg], batch_lanes=1)
    with pytest.raises(pkg.BfsError) as e:
        plan.batch_submit([(0, g.n, out)])
    assert e.value.status == 1
    with pytest.raises(pkg.BfsError) as e:
        plan.batch_submit([(3, 0, out)])
    assert e.value.status == 1
    s = int(gg.pick_sources(g, 1, seed=3)[0])
    t = plan.batch_submit([(0, s, out)])
    plan.batch_wait(t)
    assert np.array_equal(out.cpu().numpy(), _oracle_out(g, s, "u8"))
    plan.close()


def test_full_size_batch_config(gpu):
    """1024 sources over R-MAT scales 16,17,18,19,20,21,22,22 (edge factor 16)
    in one launch, uint8 outputs: every output equals the single-source GPU
    path (bit-exact); every output of the two scale-22 graphs (256 sources)
    and two sources of each other graph equal the CPU oracle."""
    import torch
    scales = [16, 17, 18, 19, 20, 21, 22, 22]
    gs = [gg.rmat(s, 16, seed=0x5EED0400 + i, perm_seed=0xBEEF0400 + i) for i, s in enumerate(scales)]
    dgs = [pkg.DeviceGraph.from_csr(g, gpu) for g in gs]
    plan = pkg.Plan(dgs, batch_lanes=2)
    qs = []
    for gi, g in enumerate(gs):
        for s in gg.pick_sources(g, 128, seed=0xC0FFEE00 + gi):
            qs.append((gi, int(s), torch.empty(g.n, dtype=torch.uint8, device=gpu)))
    bt = plan.batch_tuning()
    print(f"[gpu] full batch submit, batch tuning {bt}", flush=True)
    assert bt["tuned_ms"] > 0 and bt["grid_blocks"] > 0  # above 2^20 edges the tuner runs
    t = plan.batch_submit(qs, pkg.BATCH_ONE_LAUNCH)
    plan.batch_wait(t)
    single = pkg.Plan(dgs)
    for i, (gi, s, out) in enumerate(qs):
        d, _, _ = single.run(gi, s)
        ref = torch.where(d < 0, torch.full_like(d, 255), d).to(torch.uint8)
        assert torch.equal(out, ref), (gi, s)
    single.close()
    # every output of the two largest graphs (scale 22) and two per other graph
    # against the CPU oracle, sixteen oracle traversals at a time
    from concurrent.futures import ThreadPoolExecutor
    picked = [(gi, s, out) for i, (gi, s, out) in enumerate(qs) if scales[gi] == 22 or i % 128 < 2]
    print(f"[gpu] oracle check of {len(picked)} batched outputs", flush=True)
    with ThreadPoolExecutor(16) as ex:
        refs = list(ex.map(lambda q: _oracle_out(gs[q[0]], q[1], "u8"), picked))
    for (gi, s, out), ref in zip(picked, refs):
        assert np.array_equal(out.cpu().numpy(), ref), (gi, s)
    plan.close()


def test_batch_autotuner_leaves_lanes_clean(gpu):
    """The batch autotuner (forced on a small union) times discarded-output
    batches inside plan creation: queries afterwards are exact, an explicit
    option is kept, autotune=-1 leaves it off, and a plan without lanes has no
    batch settings."""
    import torch
    gs = _graphs_small()[:4]
    dgs = [pkg.DeviceGraph.from_csr(g, gpu) for g in gs]
    plan = pkg.Plan(dgs, batch_lanes=1, autotune=1, small_bin=5)
    bt = plan.batch_tuning()
    print(f"[gpu] batch tuning {bt}", flush=True)
    assert bt["tuned_ms"] > 0 and bt["small_bin"] == 5 and bt["grid_blocks"] > 0
    assert bt["chunk_edges"] in (1 << 10, 1 << 11, 1 << 12)
    qs, refs = [], []
    for gi, g in enumerate(gs):
        for s in gg.pick_sources(g, 50, seed=2000 + gi):
            qs.append((gi, int(s), torch.empty(g.n, dtype=torch.int32, device=gpu)))
            refs.append(oracle.bfs(g, int(s)))
    plan.batch_wait(plan.batch_submit(qs, pkg.BATCH_ONE_LAUNCH))
    for (gi, s, out), ref in zip(qs, refs):
        assert np.array_equal(out.cpu().numpy(), ref), (gi, s)
    plan.close()
    off = pkg.Plan(dgs, batch_lanes=1, autotune=-1)
    assert off.batch_tuning()["tuned_ms"] == 0
    off.close()
    plain = pkg.Plan(dgs, autotune=-1)
    with pytest.raises(pkg.BfsError) as e:
        plain.batch_tuning()
    assert e.value.status == 5
    plain.close()
