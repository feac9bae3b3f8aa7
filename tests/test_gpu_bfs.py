"""GPU parity of the single-source path against the CPU oracle (through the C ABI).

Distances are integers: the bar is bit-exact equality with the oracle on
every vertex. Parents are compared with the oracle's canonical parent.
"""
import ctypes

import numpy as np
import pytest

import graphgen as gg
import oracle
import paper_2103_13577_amd as pkg

pytestmark = pytest.mark.gpu


def _run(g, src, gpu, parent=False, **opts):
    import torch
    dg = pkg.DeviceGraph.from_csr(g, gpu)
    plan = pkg.Plan([dg], **opts)
    dist, par, st = plan.run(0, src, parent=parent)
    torch.cuda.synchronize()
    out = dist.cpu().numpy(), (par.cpu().numpy() if par is not None else None), st
    plan.close()
    return out


SMALL_GRAPHS = [
    ("path", lambda: gg.path_graph(300), [0, 150, 299]),
    ("cycle", lambda: gg.cycle_graph(257), [0, 100]),
    ("star", lambda: gg.star_graph(5000), [0, 17]),
    ("complete", lambda: gg.complete_graph(130), [3]),
    ("grid", lambda: gg.grid(97, 61, 0.0, seed=1), [0, 3000]),
    ("grid_del", lambda: gg.grid(128, 128, 0.02, seed=2), [5, 9000]),
    ("hypercube", lambda: gg.hypercube_graph(12), [0, 1234]),
    ("lollipop", lambda: gg.lollipop_graph(64, 300), [0, 363]),
    ("union", lambda: gg.disjoint_union(gg.star_graph(100), gg.path_graph(70)), [0, 120]),
    ("empty", lambda: gg.empty_graph(100), [7]),
    ("single", lambda: gg.empty_graph(1), [0]),
]

MODES = [dict(loop_mode=pkg.LOOP_PERSISTENT), dict(loop_mode=pkg.LOOP_HOST),
         # tiny thresholds push vertices into the wavefront and chunked tiers
         dict(loop_mode=pkg.LOOP_PERSISTENT, small_bin=2, wave_bin=4, chunk_edges=64),
         dict(loop_mode=pkg.LOOP_HOST, small_bin=1, wave_bin=1, chunk_edges=64),
         # the caller's labels, without the degree-sorted copy
         dict(loop_mode=pkg.LOOP_PERSISTENT, relabel=-1),
         dict(loop_mode=pkg.LOOP_HOST, relabel=-1, small_bin=2, wave_bin=4, chunk_edges=64),
         # captured level-step graph, replayed until the traversal ends
         dict(loop_mode=pkg.LOOP_GRAPH),
         # LDS copy of the hubs' visited bits on large levels
         dict(loop_mode=pkg.LOOP_HOST, hot_words=64),
         dict(loop_mode=pkg.LOOP_GRAPH, hot_words=2048, small_bin=9),
         # the 1024-thread expansion that shares a large hub copy per CU
         dict(loop_mode=pkg.LOOP_HOST, hot_words=8192, small_bin=2, wave_bin=4, chunk_edges=64),
         dict(loop_mode=pkg.LOOP_GRAPH, hot_words=16384),
         # one workgroup with the bitmaps in LDS (small whole graphs)
         dict(loop_mode=pkg.LOOP_CU), dict(loop_mode=pkg.LOOP_CU, relabel=-1),
         # every level dense (bitmap merge), and queue-only levels up to a
         # frontier of half the bitmap words
         dict(loop_mode=pkg.LOOP_HOST, sparse_div=-1), dict(loop_mode=pkg.LOOP_HOST, sparse_div=2),
         dict(loop_mode=pkg.LOOP_PERSISTENT, sparse_div=-1),
         # direction-optimizing: large levels bottom-up (next row of the paper's outlook)
         dict(direction=pkg.DIR_OPTIMIZING),
         dict(direction=pkg.DIR_OPTIMIZING, sparse_div=-1, relabel=-1),
         dict(loop_mode=pkg.LOOP_GRAPH, relabel=-1, small_bin=2, wave_bin=4, chunk_edges=64),
         # every level dense (no queue-only level): the expansions set byte
         # marks, hub targets stay in the LDS copy (narrow and wide expansion)
         dict(loop_mode=pkg.LOOP_HOST, sparse_div=-1, hot_words=16384, small_bin=3, wave_bin=6,
              chunk_edges=128),
         dict(loop_mode=pkg.LOOP_HOST, sparse_div=-1, relabel=-1, small_bin=2, wave_bin=4, chunk_edges=64),
         dict(loop_mode=pkg.LOOP_GRAPH, sparse_div=-1, hot_words=16384),
         dict(loop_mode=pkg.LOOP_PERSISTENT, sparse_div=-1, small_bin=2, wave_bin=4, chunk_edges=64),
         # the same all-dense loops with the atomic-OR expansion instead of byte marks
         dict(loop_mode=pkg.LOOP_HOST, sparse_div=-1, hot_words=16384, small_bin=3, wave_bin=6,
              chunk_edges=128, mark_mode=-1),
         # byte marks on dense levels with queue-only levels between them
         # (host-driven and captured loops, wide hub copy)
         dict(loop_mode=pkg.LOOP_HOST, sparse_div=16, hot_words=16384, small_bin=3, wave_bin=6,
              chunk_edges=128),
         dict(loop_mode=pkg.LOOP_GRAPH, sparse_div=16, hot_words=16384),
         # the captured loop's level steps launched directly (queue-only levels
         # and the narrow hub copy; all-dense levels with byte marks and the wide copy)
         dict(loop_mode=pkg.LOOP_ENQUEUE, hot_words=2048),
         dict(loop_mode=pkg.LOOP_ENQUEUE, sparse_div=-1, hot_words=16384, small_bin=3, wave_bin=6,
              chunk_edges=128),
         dict(loop_mode=pkg.LOOP_GRAPH, sparse_div=-1, hot_words=2048, mark_mode=-1),
         dict(loop_mode=pkg.LOOP_PERSISTENT, sparse_div=-1, mark_mode=-1)]


@pytest.mark.parametrize("name,make,sources", SMALL_GRAPHS, ids=[x[0] for x in SMALL_GRAPHS])
@pytest.mark.parametrize("mode", range(len(MODES)))
def test_small_graphs_exact(gpu, name, make, sources, mode):
    g = make()
    for s in sources:
        print(f"[gpu] {name} src={s} mode={MODES[mode]}", flush=True)
        d, p, st = _run(g, s, gpu, parent=True, **MODES[mode])
        ref = oracle.bfs(g, s)
        assert np.array_equal(d, ref)
        assert np.array_equal(p, oracle.parent(g, ref))
        assert st.reached == int((ref >= 0).sum())
        assert st.levels == int(ref.max()) + 1
        assert st.edges_scanned == oracle.edges_scanned(g, ref)


@pytest.mark.parametrize("mode", range(len(MODES)))
def test_rmat_scale14_64_sources(gpu, mode):
    """R-MAT scale 14, edge factor 8: 64 seeded sources, one plan reused."""
    import torch
    g = gg.rmat(14, 8, seed=0x5EED0014, perm_seed=0xBEEF0014)
    srcs = gg.pick_sources(g, 64, seed=0xC0FFEE14)
    dg = pkg.DeviceGraph.from_csr(g, gpu)
    plan = pkg.Plan([dg], **MODES[mode])
    dist = torch.empty(g.n, dtype=torch.int32, device=gpu)
    print(f"[gpu] rmat14 64 sources mode={MODES[mode]}", flush=True)
    for s in srcs:
        plan.run(0, int(s), dist=dist)
        assert np.array_equal(dist.cpu().numpy(), oracle.bfs(g, int(s))), int(s)
    plan.close()


def test_rmat_scale18_ef16_tiers(gpu):
    """Hubs large enough for the chunked workgroup tier with default bins."""
    g = gg.rmat(18, 16, seed=77, perm_seed=78)
    for s in gg.pick_sources(g, 3, seed=79):
        print(f"[gpu] rmat18 src={s}", flush=True)
        d, p, st = _run(g, int(s), gpu, parent=True)
        ref = oracle.bfs(g, int(s))
        assert np.array_equal(d, ref)
        assert np.array_equal(p, oracle.parent(g, ref))


def test_deterministic_repeats(gpu):
    import torch
    g = gg.rmat(16, 16, seed=5, perm_seed=6)
    dg = pkg.DeviceGraph.from_csr(g, gpu)
    plan = pkg.Plan([dg])
    s = int(gg.pick_sources(g, 1, seed=7)[0])
    outs = []
    for _ in range(5):
        d, p, _ = plan.run(0, s, parent=True)
        torch.cuda.synchronize()
        outs.append((d.cpu().numpy().tobytes(), p.cpu().numpy().tobytes()))
    assert all(o == outs[0] for o in outs)
    plan.close()


def test_level_stats(gpu):
    g = gg.rmat(14, 8, seed=3, perm_seed=4)
    s = int(gg.pick_sources(g, 1, seed=5)[0])
    ref = oracle.bfs(g, s)
    deg = g.degrees()
    for mode in (pkg.LOOP_PERSISTENT, pkg.LOOP_HOST, pkg.LOOP_GRAPH, pkg.LOOP_CU, pkg.LOOP_ENQUEUE):
        dg = pkg.DeviceGraph.from_csr(g, gpu)
        plan = pkg.Plan([dg], loop_mode=mode, collect_stats=True)
        plan.run(0, s)
        front, hist = plan.level_stats()
        assert len(front) == ref.max() + 1
        for L in range(len(front)):
            lv = np.flatnonzero(ref == L)
            assert front[L] == lv.size
            bins = np.where(deg[lv] > 0, np.floor(np.log2(np.maximum(deg[lv], 1))).astype(int) + 1, 0)
            assert np.array_equal(hist[L], np.bincount(bins, minlength=pkg.NUM_BINS)), L
        plan.close()


@pytest.mark.parametrize("opts", [dict(), dict(sparse_div=-1), dict(relabel=-1, autotune=-1)])
def test_direction_optimizing_exact(gpu, opts):
    """Bottom-up levels give the oracle's distances and canonical parents, and
    on R-MAT they run on the large levels. Covers the frontier bitmap written by a
    merge (sparse_div=-1: every level dense) and rebuilt from the queues after
    a queue-only level."""
    import torch
    for scale, nsrc in ((14, 24), (17, 6)):
        g = gg.rmat(scale, 16, seed=60 + scale, perm_seed=70 + scale)
        dg = pkg.DeviceGraph.from_csr(g, gpu)
        plan = pkg.Plan([dg], direction=pkg.DIR_OPTIMIZING, **opts)
        assert plan.tuning(0)["direction"] == pkg.DIR_OPTIMIZING
        bu_runs = 0
        for s in gg.pick_sources(g, nsrc, seed=80 + scale):
            print(f"[gpu] DO rmat{scale} src={s} {opts}", flush=True)
            d, p, st = plan.run(0, int(s), parent=True)
            ref = oracle.bfs(g, int(s))
            assert np.array_equal(d.cpu().numpy(), ref)
            assert np.array_equal(p.cpu().numpy(), oracle.parent(g, ref))
            assert st.edges_scanned == oracle.edges_scanned(g, ref)
            assert st.levels == int(ref.max()) + 1
            if st.bottom_up_levels:
                bu_runs += 1
                assert st.bottom_up_edges > 0 and st.bottom_up_vertices > 0
        assert bu_runs >= nsrc // 2, bu_runs
        plan.close()


@pytest.mark.parametrize("opts", [dict(), dict(sparse_div=-1)])
def test_direction_optimizing_returns_top_down(gpu, opts):
    """Top-down levels after bottom-up ones: the merges that finish bottom-up
    levels leave the tier queues unwritten (the step counts the found
    vertices' edges), and the next top-down level (queue-only, or dense with
    sparse_div=-1) fills them from the frontier bitmap. An R-MAT core with a
    40-vertex path hanging off a vertex at the core's largest distance from the
    source: the core's large levels run bottom-up, and top-down levels follow
    on the path."""
    core = gg.rmat(14, 16, seed=91, perm_seed=92)
    src = int(gg.pick_sources(core, 1, seed=93)[0])
    far = int(np.argmax(oracle.bfs(core, src)))
    rows = np.repeat(np.arange(core.n, dtype=np.int64), np.diff(core.row_ptr))
    edges = np.stack([rows, core.col.astype(np.int64)], 1)
    edges = edges[edges[:, 0] < edges[:, 1]]
    path = np.array([(far, core.n)] + [(core.n + i, core.n + i + 1) for i in range(39)], dtype=np.int64)
    g = gg.from_edges(core.n + 40, np.concatenate([edges, path]), "rmat14_path40")
    ref = oracle.bfs(g, src)
    assert ref[core.n + 39] == ref[far] + 40
    dg = pkg.DeviceGraph.from_csr(g, gpu)
    plan = pkg.Plan([dg], direction=pkg.DIR_OPTIMIZING, **opts)
    assert plan.tuning(0)["direction"] == pkg.DIR_OPTIMIZING
    for rep in range(2):  # the second traversal starts from the first one's state
        print(f"[gpu] DO core+path src={src} rep={rep} {opts}", flush=True)
        d, par, st = plan.run(0, src, parent=True)
        assert np.array_equal(d.cpu().numpy(), ref)
        assert np.array_equal(par.cpu().numpy(), oracle.parent(g, ref))
        assert st.edges_scanned == oracle.edges_scanned(g, ref)
        assert st.reached == int((ref >= 0).sum())
        assert st.levels == int(ref.max()) + 1
        # levels 0 and 1 run top-down and the core's large levels bottom-up
        # (the frontier's edges exceed 1/14 of the unvisited edges and n/24);
        # once the frontier is small and not growing the traversal returns to
        # top-down, and a frontier with few edges never enters bottom-up, so
        # every level of the 40-vertex path runs top-down
        assert 0 < st.bottom_up_levels <= 4
        assert st.levels - st.bottom_up_levels >= 42
    plan.close()


def test_dense_work_accounting(gpu):
    """The device's count of the work behind the dense expansions (the bytes
    the benchmark's roofline figure divides by their time): with every level
    dense it is the oracle's edges scanned and reached count; with queue-only
    levels it is the sum over the levels whose frontier reached the threshold."""
    g = gg.rmat(14, 8, seed=11, perm_seed=12)
    s = int(gg.pick_sources(g, 1, seed=13)[0])
    ref = oracle.bfs(g, s)
    deg = g.degrees()
    for mode in (pkg.LOOP_HOST, pkg.LOOP_PERSISTENT):
        _, _, st = _run(g, s, gpu, loop_mode=mode, sparse_div=-1, autotune=-1)
        assert st.dense_edges == oracle.edges_scanned(g, ref)
        assert st.dense_frontier == int((ref >= 0).sum())
    _, _, st = _run(g, s, gpu, loop_mode=pkg.LOOP_HOST, sparse_div=2, autotune=-1)
    words = (g.n + 63) // 64
    dense = [L for L in range(int(ref.max()) + 1) if int((ref == L).sum()) * 2 >= words]
    assert 0 < len(dense) < int(ref.max()) + 1
    assert st.expand_launches == len(dense)
    assert st.dense_frontier == sum(int((ref == L).sum()) for L in dense)
    assert st.dense_edges == sum(int(deg[ref == L].sum()) for L in dense)
    assert st.queue_ms > 0 and st.expand_ms > 0


# ---------------------------------------------------------------------------
# partitioned share: Phase 1 into the global bitmap, Phase 2 with staged
# butterfly messages (one node of a 16-node 1D partition)
# ---------------------------------------------------------------------------

def _words_to_tensor(words, gpu):
    import torch
    return torch.from_numpy(words.view(np.int64).copy()).to(gpu)


@pytest.mark.parametrize("scale,P,radix,node", [(14, 16, 2, 0), (14, 16, 4, 0), (13, 16, 2, 7),
                                                (12, 4, 2, 3)])
def test_partition_share_step_api(gpu, scale, P, radix, node):
    import torch
    g = gg.rmat(scale, 8, seed=100 + scale, perm_seed=200 + scale)
    src = int(gg.pick_sources(g, 1, seed=300 + scale)[0])
    ref = oracle.bfs(g, src)
    b = gg.partition_1d(g.row_ptr, P)
    local, inc = oracle.stage(g, ref, b, node, radix)
    dg = pkg.DeviceGraph.from_csr(g, gpu, int(b[node]), int(b[node + 1]))
    plan = pkg.Plan([dg])
    dist = torch.empty(g.n, dtype=torch.int32, device=gpu)
    plan.begin(0, src, dist)
    W = (g.n + 63) // 64
    L = 0
    while True:
        addr = plan.expand()
        got_next = _read_device_words(addr, W, gpu)
        expect = local[L] if L < local.shape[0] else np.zeros(W, dtype=np.uint64)
        assert np.array_equal(got_next, expect), f"local next at level {L}"
        msgs = [_words_to_tensor(inc[L, j], gpu) for j in range(inc.shape[1])] if L < local.shape[0] \
            else [torch.zeros(W, dtype=torch.int64, device=gpu) for _ in range(inc.shape[1])]
        gnew, onew = plan.merge_frontier(msgs)
        exp_new = int((ref == L + 1).sum())
        assert gnew == exp_new
        own = (ref == L + 1)[b[node]:b[node + 1]].sum()
        assert onew == own
        if gnew == 0:
            break
        L += 1
    st = plan.finish()
    assert st.levels == L + 1 == ref.max() + 1
    assert np.array_equal(dist.cpu().numpy(), ref)
    assert st.edges_scanned == oracle.edges_scanned(g, ref, int(b[node]), int(b[node + 1]))
    plan.close()


@pytest.mark.parametrize("scale,P,radix,node,form", [(14, 16, 2, 0, "list"), (14, 16, 4, 0, "list"),
                                                     (13, 16, 2, 7, "mixed"), (12, 4, 2, 3, "mixed"),
                                                     (14, 16, 4, 5, "mixed")])
def test_partition_share_list_messages(gpu, scale, P, radix, node, form):
    """Phase 2 with vertex-list messages: at every level the exported global
    queue equals the oracle's (ascending, after expansion and after each
    butterfly round), and merging the staged messages as lists -- or as a mix
    of lists (unsorted, with duplicates) and bitmaps -- gives the oracle's
    counts and distances."""
    import torch
    g = gg.rmat(scale, 8, seed=100 + scale, perm_seed=200 + scale)
    src = int(gg.pick_sources(g, 1, seed=300 + scale)[0])
    ref = oracle.bfs(g, src)
    b = gg.partition_1d(g.row_ptr, P)
    local, inc = oracle.stage(g, ref, b, node, radix)
    nlev = local.shape[0]
    dg = pkg.DeviceGraph.from_csr(g, gpu, int(b[node]), int(b[node + 1]))
    plan = pkg.Plan([dg])
    dist = torch.empty(g.n, dtype=torch.int32, device=gpu)
    buf = torch.empty(g.n, dtype=torch.int32, device=gpu)
    W = (g.n + 63) // 64
    zeros = np.zeros(W, dtype=np.uint64)
    per_round = radix - 1
    depth = inc.shape[1] // per_round
    rng = np.random.default_rng(scale * 31 + node)
    plan.begin(0, src, dist)
    L = 0
    while True:
        plan.expand()
        have = (local[L] if L < nlev else zeros).copy()
        cnt = plan.frontier_list(buf)
        assert cnt == plan.frontier_list()
        assert np.array_equal(buf[:cnt].cpu().numpy(), oracle.bitmap_list(have, g.n)), f"level {L}"
        for i in range(depth):
            last = i == depth - 1
            lists, bms = [], []
            for j in range(per_round):
                m = inc[L, i * per_round + j] if L < nlev else zeros
                have |= m
                ids = oracle.bitmap_list(m, g.n)
                as_list = form == "list" or (i + j + L) % 2 == 0
                if as_list:
                    if form == "mixed" and ids.size:
                        ids = np.concatenate([ids, ids[: min(3, ids.size)]])
                        rng.shuffle(ids)
                    lists.append(torch.from_numpy(ids).to(gpu))
                else:
                    bms.append(_words_to_tensor(m, gpu))
            if bms and L % 2:  # the two forms in separate calls of one round
                if lists:
                    plan.merge_lists(lists, keep_next=True)
                gnew, onew = plan.merge_frontier(bms, keep_next=not last)
            else:  # one pass over both forms
                gnew, onew = plan.merge_lists(lists, bitmaps=bms, keep_next=not last)
            if not last:
                cnt = plan.frontier_list(buf)
                assert np.array_equal(buf[:cnt].cpu().numpy(), oracle.bitmap_list(have, g.n)), (L, i)
        assert gnew == int((ref == L + 1).sum())
        assert onew == int((ref == L + 1)[b[node]:b[node + 1]].sum())
        if gnew == 0:
            break
        L += 1
    st = plan.finish()
    assert st.levels == L + 1 == ref.max() + 1
    assert np.array_equal(dist.cpu().numpy(), ref)
    plan.close()


def test_list_message_errors(gpu):
    """Capacity too small, ids out of range, negative counts and wrong call
    order are reported by status; the plan stays usable."""
    import torch
    g = gg.rmat(12, 8, seed=77, perm_seed=78)
    src = int(gg.pick_sources(g, 1, seed=79)[0])
    ref = oracle.bfs(g, src)
    plan = pkg.Plan([pkg.DeviceGraph.from_csr(g, gpu)], autotune=-1)
    dist = torch.empty(g.n, dtype=torch.int32, device=gpu)
    with pytest.raises(pkg.BfsError) as e:
        plan.frontier_list()
    assert e.value.status == 7
    plan.begin(0, src, dist)
    with pytest.raises(pkg.BfsError) as e:
        plan.frontier_list()
    assert e.value.status == 7  # before bfs_expand of the level
    plan.expand()
    level1 = np.flatnonzero(ref == 1).astype(np.int32)
    assert plan.frontier_list() == level1.size > 2
    small = torch.full((2,), -7, dtype=torch.int32, device=gpu)
    with pytest.raises(pkg.BfsError) as e:
        plan.frontier_list(small)
    assert e.value.status == 5
    assert np.array_equal(small.cpu().numpy(), level1[:2])
    h = pkg.lib()
    ptrs = (ctypes.c_void_p * 1)(None)
    cnts = (ctypes.c_int64 * 1)(-1)
    assert h.bfs_merge_lists(plan.h, ptrs, cnts, 1, None, 0, 0, None, None) == 1  # negative count
    cnts[0] = 3
    assert h.bfs_merge_lists(plan.h, ptrs, cnts, 1, None, 0, 0, None, None) == 1  # NULL list
    assert h.bfs_merge_lists(plan.h, None, None, 0, None, 2, 0, None, None) == 1  # NULL bitmaps
    bad = torch.tensor([int(level1[0]), g.n], dtype=torch.int32, device=gpu)
    ptrs[0] = bad.data_ptr()
    cnts[0] = 2
    # keep_next with no counts requested: the bad id is flagged, reported by
    # the call that finishes the level
    assert h.bfs_merge_lists(plan.h, ptrs, cnts, 1, None, 0, 1, None, None) == 0
    with pytest.raises(pkg.BfsError) as e:
        plan.merge_frontier([])
    assert e.value.status == 1
    plan.begin(0, src, dist)
    plan.expand()
    with pytest.raises(pkg.BfsError) as e:
        plan.merge_lists([bad])
    assert e.value.status == 1
    # a fresh traversal with list-form (empty) messages equals the oracle
    plan.begin(0, src, dist)
    while True:
        plan.expand()
        gnew, _ = plan.merge_lists([])
        if gnew == 0:
            break
    plan.finish()
    assert np.array_equal(dist.cpu().numpy(), ref)
    plan.run(0, src, dist=dist)  # the relabelled copy is not exported
    with pytest.raises(pkg.BfsError) as e:
        plan.frontier_list()
    assert e.value.status == 7
    plan.close()


def test_list_export_many_blocks(gpu):
    """2^25 + 1000 vertices (1025 export blocks of 512 bitmap words, a ragged
    last word): a star whose 3000 leaves are spread over the whole id range."""
    import torch
    n = (1 << 25) + 1000
    leaves = np.unique((np.arange(1, 3001, dtype=np.int64) * 11184811 + 977) % (n - 1) + 1)
    leaves = np.union1d(leaves, [n - 1, 64, 63])
    edges = np.stack([np.zeros(leaves.size, dtype=np.int64), leaves], axis=1)
    g = gg.from_edges(n, edges, "spread star")
    plan = pkg.Plan([pkg.DeviceGraph.from_csr(g, gpu)], autotune=-1)
    dist = torch.empty(n, dtype=torch.int32, device=gpu)
    buf = torch.empty(leaves.size + 5, dtype=torch.int32, device=gpu)
    plan.begin(0, 0, dist)
    plan.expand()
    cnt = plan.frontier_list(buf)
    assert cnt == leaves.size
    assert np.array_equal(buf[:cnt].cpu().numpy(), leaves.astype(np.int32))
    gnew, onew = plan.merge_lists([buf[:cnt]])
    assert gnew == onew == leaves.size
    leaf = int(leaves[-1])
    plan.begin(0, leaf, dist)
    plan.expand()
    assert plan.frontier_list(buf) == 1 and int(buf[0]) == 0
    plan.close()


@pytest.mark.parametrize("relabel", [0, -1])
def test_cu_loop_larger_graphs(gpu, relabel):
    """The one-workgroup loop on graphs that fill more of its LDS: R-MAT 16
    (hubs) and a 500 x 400 grid with 2% of edges deleted (hundreds of levels,
    so the two frontier queues alternate many times)."""
    for g in (gg.rmat(16, 8, seed=611, perm_seed=612), gg.grid(500, 400, 0.02, seed=613)):
        plan = pkg.Plan([pkg.DeviceGraph.from_csr(g, gpu)], loop_mode=pkg.LOOP_CU, relabel=relabel,
                        autotune=-1)
        for i, s in enumerate(gg.pick_sources(g, 3, seed=614)):
            print(f"[gpu] cu loop n={g.n} src={s}", flush=True)
            d, p, st = plan.run(0, int(s), parent=(i == 0))
            ref = oracle.bfs(g, int(s))
            assert np.array_equal(d.cpu().numpy(), ref)
            if i == 0:
                assert np.array_equal(p.cpu().numpy(), oracle.parent(g, ref))
            assert st.levels == int(ref.max()) + 1
            assert st.reached == int((ref >= 0).sum())
            assert st.edges_scanned == oracle.edges_scanned(g, ref)
        plan.close()


def _bottom_up_level(pattern, L, frontier, n):
    if pattern == "all":
        return True
    if pattern == "alternate":
        return L % 2 == 1
    return frontier * 24 >= n  # "rule": large frontiers go bottom-up


@pytest.mark.parametrize("scale,P,radix,node,pattern,rounds", [
    (14, 16, 2, 0, "rule", False), (14, 16, 4, 5, "alternate", True), (13, 16, 2, 7, "all", True),
    (12, 4, 2, 3, "alternate", False), (14, 1, 2, 0, "rule", False), (13, 2, 2, 1, "all", False)])
def test_partition_share_bottom_up(gpu, scale, P, radix, node, pattern, rounds):
    """Bottom-up Phase 1 steps on a share behind the staged butterfly
    exchange: after a bottom-up step the node's local bitmap equals its owned
    vertices of the next level (oracle bottom-up staging), after a top-down
    step the oracle's top-down set; merged at once or one round at a time, the
    traversal gives the oracle's counts, distances and owned parents."""
    import torch
    g = gg.rmat(scale, 8, seed=100 + scale, perm_seed=200 + scale)
    src = int(gg.pick_sources(g, 1, seed=300 + scale)[0])
    ref = oracle.bfs(g, src)
    b = gg.partition_1d(g.row_ptr, P)
    lo, hi = int(b[node]), int(b[node + 1])
    td = oracle.stage(g, ref, b, node, radix)
    bu = oracle.stage_bottom_up(g.n, ref, b, node, radix)
    nlev = td[0].shape[0]
    W = (g.n + 63) // 64
    zeros = np.zeros(W, dtype=np.uint64)
    dg = pkg.DeviceGraph.from_csr(g, gpu, lo, hi)
    plan = pkg.Plan([dg], direction=pkg.DIR_OPTIMIZING)
    dist = torch.empty(g.n, dtype=torch.int32, device=gpu)
    parent = torch.empty(g.n, dtype=torch.int32, device=gpu)
    plan.begin(0, src, dist)
    L, n_bu = 0, 0
    frontier = 1
    while True:
        up = _bottom_up_level(pattern, L, frontier, g.n)
        n_bu += int(up)
        local, inc = bu if up else td
        addr = plan.expand_bottom_up() if up else plan.expand()
        exp = local[L] if L < nlev else zeros
        assert np.array_equal(_read_device_words(addr, W, gpu), exp), (L, up)
        msgs = [_words_to_tensor(inc[L, j] if L < nlev else zeros, gpu) for j in range(inc.shape[1])]
        if rounds and len(msgs) > 1:
            per = radix - 1
            for r0 in range(0, len(msgs), per):
                gnew, onew = plan.merge_frontier(msgs[r0:r0 + per], keep_next=r0 + per < len(msgs))
        else:
            gnew, onew = plan.merge_frontier(msgs)
        assert gnew == int((ref == L + 1).sum())
        assert onew == int((ref == L + 1)[lo:hi].sum())
        frontier = gnew
        if gnew == 0:
            break
        L += 1
    st = plan.finish(parent)
    assert st.levels == L + 1 == ref.max() + 1
    assert st.bottom_up_levels == n_bu
    assert np.array_equal(dist.cpu().numpy(), ref)
    assert np.array_equal(parent.cpu().numpy()[lo:hi], oracle.parent(g, ref)[lo:hi])
    plan.close()


def test_bottom_up_step_errors(gpu):
    """A plan without BFS_DIR_OPTIMIZING, a second expansion of one level and
    a bottom-up step before bfs_begin are refused; bfs_run's traversal of the
    relabelled copy is not a step-wise one."""
    import torch
    g = gg.rmat(11, 8, seed=91, perm_seed=92)
    src = int(gg.pick_sources(g, 1, seed=93)[0])
    dist = torch.empty(g.n, dtype=torch.int32, device=gpu)
    plain = pkg.Plan([pkg.DeviceGraph.from_csr(g, gpu)], autotune=-1)
    plain.begin(0, src, dist)
    with pytest.raises(pkg.BfsError) as e:
        plain.expand_bottom_up()
    assert e.value.status == 7
    plain.close()
    plan = pkg.Plan([pkg.DeviceGraph.from_csr(g, gpu)], autotune=-1, direction=pkg.DIR_OPTIMIZING)
    with pytest.raises(pkg.BfsError) as e:
        plan.expand_bottom_up()
    assert e.value.status == 7
    plan.begin(0, src, dist)
    plan.expand_bottom_up()
    with pytest.raises(pkg.BfsError) as e:
        plan.expand_bottom_up()
    assert e.value.status == 7
    with pytest.raises(pkg.BfsError) as e:
        plan.expand()
    assert e.value.status == 7
    plan.merge_frontier([])
    while True:
        plan.expand_bottom_up()
        gnew, _ = plan.merge_frontier([])
        if gnew == 0:
            break
    plan.finish()
    assert np.array_equal(dist.cpu().numpy(), ref := oracle.bfs(g, src))
    d, _, st = plan.run(0, src)
    assert np.array_equal(d.cpu().numpy(), ref)
    with pytest.raises(pkg.BfsError) as e:
        plan.expand_bottom_up()
    assert e.value.status == 7
    plan.close()


def _read_device_words(addr, W, gpu):
    """Copies W uint64 words at a raw device address to the host (hipMemcpy)."""
    import torch
    hip = ctypes.CDLL("libamdhip64.so")
    hip.hipMemcpy.argtypes = [ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_int]
    out = np.empty(W, dtype=np.uint64)
    torch.cuda.synchronize()
    assert hip.hipMemcpy(out.ctypes.data, addr, W * 8, 2) == 0  # DeviceToHost
    return out


def test_partition_share_scale26(gpu):
    """Partition 0 of a 16-way 1D partition of R-MAT scale 26, edge factor 8,
    with the four radix-2 butterfly messages of every level staged from the
    oracle: 2^26-bit (8 MiB) bitmaps, so every merge block strides over
    several steps. The node's global next bitmap after each expansion equals
    the oracle's X_0(L) bit for bit, the level counts match, and the whole
    distance array equals the oracle's."""
    import torch
    print("[gpu] generating rmat26 ef8", flush=True)
    g = gg.rmat(26, 8, seed=0x5EED0026, perm_seed=0xBEEF0026)
    src = int(gg.pick_sources(g, 1, seed=0xC0FFEE26)[0])
    ref = oracle.bfs(g, src)
    b = gg.partition_1d(g.row_ptr, 16)
    local, inc = oracle.stage(g, ref, b, 0, 2)
    print(f"[gpu] share26 staged {local.shape[0]} levels", flush=True)
    dg = pkg.DeviceGraph.from_csr(g, gpu, 0, int(b[1]))
    plan = pkg.Plan([dg])
    dist = torch.empty(g.n, dtype=torch.int32, device=gpu)
    W = (g.n + 63) // 64
    zeros = [torch.zeros(W, dtype=torch.int64, device=gpu) for _ in range(inc.shape[1])]
    plan.begin(0, src, dist)
    L = 0
    while True:
        addr = plan.expand()
        got = _read_device_words(addr, W, gpu)
        exp = local[L] if L < local.shape[0] else np.zeros(W, dtype=np.uint64)
        assert np.array_equal(got, exp), f"local next at level {L}"
        msgs = [_words_to_tensor(inc[L, j], gpu) for j in range(inc.shape[1])] if L < local.shape[0] else zeros
        gnew, onew = plan.merge_frontier(msgs)
        assert gnew == int((ref == L + 1).sum())
        assert onew == int((ref == L + 1)[b[0]:b[1]].sum())
        del msgs
        if gnew == 0:
            break
        L += 1
    st = plan.finish()
    assert st.levels == int(ref.max()) + 1
    assert np.array_equal(dist.cpu().numpy(), ref)
    assert st.edges_scanned == oracle.edges_scanned(g, ref, int(b[0]), int(b[1]))
    plan.close()


@pytest.mark.parametrize("rounds", [False, True])
def test_partition_share_run_with_exchange(gpu, rounds):
    """bfs_run with an exchange callback serving the staged messages; with
    `rounds` the messages are merged one butterfly round at a time."""
    import torch
    g = gg.rmat(15, 8, seed=400, perm_seed=401)
    src = int(gg.pick_sources(g, 1, seed=402)[0])
    ref = oracle.bfs(g, src)
    b = gg.partition_1d(g.row_ptr, 16)
    local, inc = oracle.stage(g, ref, b, 0, 2)
    W = (g.n + 63) // 64
    staged = [[_words_to_tensor(inc[L, j], gpu) for j in range(inc.shape[1])]
              for L in range(local.shape[0])]
    zeros = [torch.zeros(W, dtype=torch.int64, device=gpu) for _ in range(inc.shape[1])]
    seen = []

    def exchange(level, local_next):
        seen.append(level)
        got = _read_device_words(local_next, W, gpu)
        exp = local[level] if level < local.shape[0] else np.zeros(W, dtype=np.uint64)
        if not np.array_equal(got, exp):
            raise AssertionError(level)
        msgs = staged[level] if level < len(staged) else zeros
        return [m.data_ptr() for m in msgs]

    dg = pkg.DeviceGraph.from_csr(g, gpu, 0, int(b[1]))
    if not rounds:
        plan = pkg.Plan([dg], exchange=exchange)
        d, _, st = plan.run(0, src)
        assert np.array_equal(d.cpu().numpy(), ref)
        assert seen == list(range(ref.max() + 1))
        plan.close()
    else:
        plan = pkg.Plan([dg])
        dist = torch.empty(g.n, dtype=torch.int32, device=gpu)
        plan.begin(0, src, dist)
        L = 0
        while True:
            plan.expand()
            msgs = staged[L] if L < len(staged) else zeros
            for j, m in enumerate(msgs):  # one round at a time, level kept open
                plan.merge_frontier([m], keep_next=True)
            gnew, _ = plan.merge_frontier([])
            if gnew == 0:
                break
            L += 1
        plan.finish()
        assert np.array_equal(dist.cpu().numpy(), ref)
        plan.close()


# ---------------------------------------------------------------------------
# merge kernel vs oracle merge on random bitmaps
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,k,vb,ve", [(1000, 0, 0, 1000), (70000, 3, 64, 40000),
                                       (4097, 11, 1024, 4097), (130, 2, 64, 128),
                                       (200000, 8, 0, 200000)])
def test_merge_random_bitmaps(gpu, n, k, vb, ve):
    import torch
    rng = np.random.default_rng(n * 31 + k)
    W = (n + 63) // 64
    valid = np.zeros(W * 64, dtype=bool)
    valid[:n] = True
    vmask = np.packbits(valid, bitorder="little").view(np.uint64)
    inc = [np.packbits(rng.random(W * 64) < 0.03, bitorder="little").view(np.uint64) & vmask
           for _ in range(k)]
    g = gg.empty_graph(n)
    rp = np.zeros(ve - vb + 1, dtype=np.int64)
    dg = pkg.DeviceGraph(n, vb, ve, torch.from_numpy(rp).to(gpu),
                         torch.zeros(0, dtype=torch.int32, device=gpu))
    plan = pkg.Plan([dg])
    dist = torch.empty(n, dtype=torch.int32, device=gpu)
    src = n // 3
    plan.begin(0, src, dist)
    plan.expand()
    gnew, onew = plan.merge_frontier([_words_to_tensor(x, gpu) for x in inc])
    # oracle on the same state: visited = {src}, next = empty
    vis = np.zeros(W, dtype=np.uint64)
    vis[src >> 6] = np.uint64(1) << np.uint64(src & 63)
    odist = np.full(n, -1, dtype=np.int32)
    odist[src] = 0
    tot, q = oracle.merge(n, 0, np.zeros(W, dtype=np.uint64), inc, vis, odist, vb, ve)
    assert gnew == tot and onew == q.size
    assert np.array_equal(dist.cpu().numpy(), odist)
    plan.close()
    del g


# ---------------------------------------------------------------------------
# errors through the C ABI
# ---------------------------------------------------------------------------

def test_error_paths(gpu):
    import torch
    g = gg.rmat(10, 8, seed=1, perm_seed=2)
    dg = pkg.DeviceGraph.from_csr(g, gpu)
    plan = pkg.Plan([dg])
    with pytest.raises(pkg.BfsError) as e:
        plan.run(0, g.n)
    assert e.value.status == 1
    with pytest.raises(pkg.BfsError) as e:
        plan.run(0, -1)
    assert e.value.status == 1
    with pytest.raises(pkg.BfsError) as e:
        plan.run(1, 0)
    assert e.value.status == 1
    s = int(gg.pick_sources(g, 1, seed=3)[0])
    with pytest.raises(pkg.BfsError) as e:  # an LDS hub copy larger than a workgroup's LDS
        pkg.Plan([dg], hot_words=1 << 20)
    assert e.value.status == 1
    with pytest.raises(pkg.BfsError) as e:  # unknown level loop
        pkg.Plan([dg], loop_mode=9)
    assert e.value.status == 1
    big = gg.empty_graph(1 << 20)  # bitmaps of 2^20 bits do not fit one workgroup's LDS
    bplan = pkg.Plan([pkg.DeviceGraph.from_csr(big, gpu)], loop_mode=pkg.LOOP_CU)
    with pytest.raises(pkg.BfsError) as e:
        bplan.run(0, 5)
    assert e.value.status == 1
    bplan.close()
    d, _, _ = plan.run(0, s)  # still usable after errors
    assert np.array_equal(d.cpu().numpy(), oracle.bfs(g, s))
    plan.close()
    # merge before begin
    plan = pkg.Plan([dg])
    with pytest.raises(pkg.BfsError) as e:
        plan.merge_frontier([])
    assert e.value.status == 7
    plan.close()
    # column id out of range is rejected at plan creation
    bad = pkg.DeviceGraph(g.n, 0, g.n, dg.row_ptr, dg.col.clone())
    bad.col[5] = g.n
    with pytest.raises(pkg.BfsError) as e:
        pkg.Plan([bad])
    assert e.value.status == 1
    # workspace too small
    L = pkg.lib()
    arr = (pkg.bfs_graph * 1)(dg.c_struct())
    ws = torch.empty(1 << 12, dtype=torch.uint8, device=gpu)
    h = ctypes.c_void_p(0)
    st = L.bfs_plan_create(arr, 1, None, (ws.data_ptr() + 255) // 256 * 256, 1024, ctypes.byref(h))
    assert st == 2
    # exchange failure is reported and the plan stays usable
    def failing(level, local_next):
        raise RuntimeError("link down")
    plan = pkg.Plan([dg], exchange=failing)
    with pytest.raises(pkg.BfsError) as e:
        plan.run(0, s)
    assert e.value.status == 6
    plan.close()


@pytest.fixture(scope="module")
def rmat24(gpu):
    """The benchmark's graph: R-MAT scale 24, edge factor 16, its seeds, on
    the device, with the oracle's distances cached per source."""
    import bench
    print("[gpu] generating rmat24", flush=True)
    gseed, pseed, _ = bench.SEEDS["rmat24"]
    g = gg.rmat(24, 16, seed=gseed, perm_seed=pseed)
    dg = pkg.DeviceGraph.from_csr(g, gpu)
    refs = {}

    def ref(s):
        if s not in refs:
            refs[s] = oracle.bfs(g, s)
        return refs[s]
    yield g, dg, ref
    del dg


def test_headline_plan_rmat24(gpu, rmat24):
    """Exactly what the benchmark times: its pinned headline plan (captured
    level loop, 8 steps per replay, the 1024-thread expansion with a
    20,352-word LDS hub copy against a 262,144-word bitmap, every level dense,
    byte marks) and the plan that times its kernels (the same settings, level
    steps launched directly), on its graph, from two of its timed sources
    (indices 3 and 4 of its seeded source sequence, timed under the default
    warm-up of 3): whole distance arrays bit-exact against the oracle, and the
    canonical parents of one source."""
    import torch
    import bench
    g, dg, ref = rmat24
    srcs = bench.headline_sources(g, 5)[3:5]
    for loop in (bench.HEADLINE_PLAN["loop_mode"], pkg.LOOP_ENQUEUE):
        plan = pkg.Plan([dg], **{**bench.HEADLINE_PLAN, "loop_mode": loop})
        t = plan.tuning(0)
        assert t["loop_mode"] == loop and t["relabelled"] == 1
        assert 4096 < t["hot_words"] < (g.n + 63) // 64  # wide expansion; copy smaller than the bitmap
        assert t["sparse_div"] == 0 and t["mark_mode"] == 1
        for i, s in enumerate(srcs):
            print(f"[gpu] rmat24 headline plan loop={loop} src={s}", flush=True)
            d, p, st = plan.run(0, int(s), parent=(i == 0))
            torch.cuda.synchronize()
            r = ref(int(s))
            assert np.array_equal(d.cpu().numpy(), r)
            if i == 0:
                assert np.array_equal(p.cpu().numpy(), oracle.parent(g, r))
            assert st.edges_scanned == oracle.edges_scanned(g, r)
            assert st.dense_edges == st.edges_scanned  # every level ran the dense expansion
            if loop == pkg.LOOP_ENQUEUE:
                # all 8 steps of each round trip are timed
                assert st.expand_launches == -(-st.levels // 8) * 8
                a, b, kind = plan.level_times()
                assert len(a) == st.levels and (a > 0).all() and (b > 0).all() and (kind == 0).all()
        plan.close()


FULL_SIZE_PLANS = [dict(loop_mode=pkg.LOOP_HOST, autotune=-1),
                   dict(loop_mode=pkg.LOOP_GRAPH, autotune=-1),
                   dict(loop_mode=pkg.LOOP_PERSISTENT, autotune=-1),
                   dict(loop_mode=pkg.LOOP_GRAPH, autotune=-1, sparse_div=-1, hot_words=16384),
                   dict(loop_mode=pkg.LOOP_HOST, autotune=-1, sparse_div=-1, hot_words=16384,
                        small_bin=8, wave_bin=15, chunk_edges=1024, mark_mode=-1),
                   dict(loop_mode=pkg.LOOP_HOST, autotune=-1, sparse_div=-1, hot_words=20352,
                        small_bin=6, wave_bin=14, chunk_edges=2048)]


@pytest.mark.parametrize("plan_opts", FULL_SIZE_PLANS, ids=[str(i) for i in range(len(FULL_SIZE_PLANS))])
def test_full_size_rmat24_ef16(gpu, rmat24, plan_opts):
    """The benchmark's workload under explicit plans (no autotuning, so the
    kernels covered do not depend on timing): host-driven, captured-graph
    and cooperative loops, all-dense levels with byte marks in the captured
    loop, and the atomic-OR expansion. Whole distance arrays bit-exact
    against the oracle for one of the benchmark's sources."""
    import torch
    import bench
    g, dg, ref = rmat24
    plan = pkg.Plan([dg], **plan_opts)
    s = int(bench.headline_sources(g, 1)[0])
    print(f"[gpu] rmat24 src={s} plan={plan_opts}", flush=True)
    d, _, st = plan.run(0, s)
    torch.cuda.synchronize()
    r = ref(s)
    assert np.array_equal(d.cpu().numpy(), r)
    assert st.edges_scanned == oracle.edges_scanned(g, r)
    plan.close()


@pytest.mark.parametrize("grid", [1, 7, 300, 2048])
def test_persistent_grid_sizes(gpu, grid):
    """The cooperative loop's grid barrier (block 0 collects every block's
    announcement) at one block, at grids that are not multiples of a
    wavefront or of the 256 threads that poll, and at its 2048-block limit:
    R-MAT 14 and a grid graph of ~350 levels (two barriers per level)."""
    import torch
    for g, srcs in ((gg.rmat(14, 8, seed=0x5EED0014, perm_seed=0xBEEF0014), (0, 777)),
                    (gg.grid(200, 150, 0.02, seed=17), (5, 12345))):
        dg = pkg.DeviceGraph.from_csr(g, gpu)
        plan = pkg.Plan([dg], loop_mode=pkg.LOOP_PERSISTENT, grid_blocks=grid, autotune=-1)
        for s in srcs:
            if s >= g.n:
                continue
            print(f"[gpu] persistent grid={grid} n={g.n} src={s}", flush=True)
            try:
                d, _, st = plan.run(0, int(s))
            except pkg.BfsError as err:
                # more blocks than can be co-resident with this kernel's resources
                assert grid == 2048 and "cooperative launch of at most" in str(err)
                break
            torch.cuda.synchronize()
            ref = oracle.bfs(g, int(s))
            assert np.array_equal(d.cpu().numpy(), ref)
            assert st.levels == int(ref.max()) + 1
        plan.close()


def test_graph_replays_match_eager(gpu):
    """The captured level graph is replayed many times per traversal and across
    traversals, with eager launches and synchronisations in between; every
    replayed result equals the eager host-driven result and the oracle."""
    import torch
    g = gg.grid(200, 150, 0.02, seed=17)  # ~350 levels: ~44 replays per traversal
    dg = pkg.DeviceGraph.from_csr(g, gpu)
    pg = pkg.Plan([dg], loop_mode=pkg.LOOP_GRAPH)
    ph = pkg.Plan([dg], loop_mode=pkg.LOOP_HOST)
    for s in gg.pick_sources(g, 4, seed=18):
        dg_, _, st = pg.run(0, int(s))
        torch.cuda.synchronize()
        dh, _, _ = ph.run(0, int(s))
        torch.cuda.synchronize()
        ref = oracle.bfs(g, int(s))
        assert np.array_equal(dg_.cpu().numpy(), ref)
        assert np.array_equal(dh.cpu().numpy(), ref)
        assert st.levels == int(ref.max()) + 1
    pg.close()
    ph.close()


NO_ALLOC_PLANS = [dict(loop_mode=pkg.LOOP_HOST), dict(loop_mode=pkg.LOOP_GRAPH),
                  dict(loop_mode=pkg.LOOP_ENQUEUE, sparse_div=-1, hot_words=8192),
                  dict(loop_mode=pkg.LOOP_GRAPH, sparse_div=-1, hot_words=2048),
                  dict(loop_mode=pkg.LOOP_PERSISTENT), dict(loop_mode=pkg.LOOP_HOST, sparse_div=-1),
                  dict(loop_mode=pkg.LOOP_CU), dict()]


@pytest.mark.parametrize("plan_opts", NO_ALLOC_PLANS, ids=[str(i) for i in range(len(NO_ALLOC_PLANS))])
def test_run_allocates_nothing(gpu, plan_opts):
    """Every buffer is sized at plan creation (Section 3, fixed preallocated
    buffers): device free memory is the same before and after traversals in
    every level loop. The captured level graph is instantiated at plan
    creation, so even the first traversal of that loop allocates nothing;
    other loops get one warm-up traversal first (the HIP runtime may set up a
    kernel's private-memory backing on that kernel's first launch). The
    workspace size depends on the graphs and options only."""
    import torch
    g = gg.rmat(15, 8, seed=91, perm_seed=92)
    dg = pkg.DeviceGraph.from_csr(g, gpu)
    plan = pkg.Plan([dg], **plan_opts)
    plan2 = pkg.Plan([dg], **plan_opts)
    assert plan.workspace_bytes == plan2.workspace_bytes
    plan2.close()
    dist = torch.empty(g.n, dtype=torch.int32, device=gpu)
    srcs = [int(s) for s in gg.pick_sources(g, 5, seed=93)]
    torch.cuda.synchronize()
    if plan.tuning(0)["loop_mode"] != pkg.LOOP_GRAPH:
        plan.run(0, srcs[0], dist=dist)
        torch.cuda.synchronize()
    free0, _ = torch.cuda.mem_get_info()
    for s in srcs[1:]:
        plan.run(0, s, dist=dist)
        torch.cuda.synchronize()
        assert np.array_equal(dist.cpu().numpy(), oracle.bfs(g, s))
    free1, _ = torch.cuda.mem_get_info()
    assert free1 == free0, (free0, free1, plan.tuning(0))
    plan.close()


def test_tune_cache(gpu, tmp_path):
    """A plan with a tuning cache appends its tuned settings; a second plan on
    the same graph, device and options takes them from the cache (no timing
    runs) and traverses exactly; other options make another entry."""
    import time as _time
    g = gg.rmat(15, 16, seed=71, perm_seed=72)
    dg = pkg.DeviceGraph.from_csr(g, gpu)
    path = str(tmp_path / "bfs_tune.txt")
    t0 = _time.perf_counter()
    a = pkg.Plan([dg], autotune=1, tune_cache=path)
    ta = _time.perf_counter() - t0
    lines = open(path).read().splitlines()
    assert len(lines) == 1 and lines[0].startswith("bfs-tune ")
    t0 = _time.perf_counter()
    b = pkg.Plan([dg], autotune=1, tune_cache=path)
    tb = _time.perf_counter() - t0
    assert len(open(path).read().splitlines()) == 1  # read, not re-tuned
    assert a.tuning(0) == b.tuning(0)
    assert tb < ta
    s = int(gg.pick_sources(g, 1, seed=73)[0])
    d, _, _ = b.run(0, s)
    assert np.array_equal(d.cpu().numpy(), oracle.bfs(g, s))
    c = pkg.Plan([dg], autotune=1, tune_cache=path, small_bin=5)
    assert len(open(path).read().splitlines()) == 2
    assert c.tuning(0)["small_bin"] == 5
    a.close()
    b.close()
    c.close()
