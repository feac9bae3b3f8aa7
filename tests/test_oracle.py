"""Pins of the CPU oracle against facts that do not come from the oracle.

Each check is chosen so that a plausible slip in the oracle (a dropped term,
an off-by-one level, a wrong index or owner, a transposed stage) fails one of
them: closed-form distances, a textbook all-pairs algorithm and a library
shortest-path routine on random graphs, BFS invariants, the paper's Figure 1/2
walk-through, and the Algorithm 2 simulation for the butterfly stages.
"""
import os

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.sparse.csgraph import connected_components, shortest_path

import graphgen as gg
import oracle
from oracle import butterfly_sim as bs

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def _adj(g):
    return sp.csr_matrix((np.ones(g.m, dtype=np.int8), g.col, g.row_ptr), shape=(g.n, g.n))


def check_invariants(g, src, dist):
    """Raises AssertionError unless dist is a valid BFS distance array from src
    (root at 0, closed reached set, edges span at most one level, every
    reached vertex has a neighbour one level closer, reached count equals the
    component size from a library connected-components routine)."""
    assert dist[src] == 0
    deg = np.diff(g.row_ptr)
    rows = np.repeat(np.arange(g.n), deg)
    du, dv = dist[rows], dist[g.col]
    assert np.all((du >= 0) == (dv >= 0)), "reached set not closed under adjacency"
    both = (du >= 0) & (dv >= 0)
    assert np.all(np.abs(du[both] - dv[both]) <= 1), "edge spans more than one level"
    has_closer = np.zeros(g.n, dtype=bool)
    np.logical_or.at(has_closer, rows, (dv == du - 1) & (du > 0))
    reached = dist >= 0
    need = reached.copy()
    need[src] = False
    assert np.all(has_closer[need]), "reached vertex without a neighbour one level closer"
    assert np.all(dist[~reached] == -1)
    _, labels = connected_components(_adj(g), directed=False)
    assert reached.sum() == np.sum(labels == labels[src]), "reached count != component size"


# ---------------------------------------------------------------------------
# closed forms
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("n,s", [(1, 0), (2, 1), (17, 0), (300, 123)])
def test_path(n, s):
    g = gg.path_graph(n)
    assert np.array_equal(oracle.bfs(g, s), np.abs(np.arange(n) - s))


@pytest.mark.parametrize("n,s", [(3, 0), (10, 3), (101, 50)])
def test_cycle(n, s):
    g = gg.cycle_graph(n)
    i = np.arange(n)
    assert np.array_equal(oracle.bfs(g, s), np.minimum(np.abs(i - s), n - np.abs(i - s)))


def test_star():
    g = gg.star_graph(50)
    d = oracle.bfs(g, 0)
    assert d[0] == 0 and np.all(d[1:] == 1)
    d = oracle.bfs(g, 7)
    expect = np.full(50, 2)
    expect[0], expect[7] = 1, 0
    assert np.array_equal(d, expect)


def test_complete():
    g = gg.complete_graph(40)
    d = oracle.bfs(g, 5)
    expect = np.ones(40, dtype=np.int32)
    expect[5] = 0
    assert np.array_equal(d, expect)


@pytest.mark.parametrize("W,H,s", [(7, 5, 0), (32, 20, 333), (1, 9, 4)])
def test_grid(W, H, s):
    g = gg.grid(W, H, 0.0, seed=1)
    x, y = np.arange(W * H) % W, np.arange(W * H) // W
    expect = np.abs(x - s % W) + np.abs(y - s // W)
    assert np.array_equal(oracle.bfs(g, s), expect)


@pytest.mark.parametrize("k,s", [(1, 0), (6, 0), (9, 300)])
def test_hypercube(k, s):
    g = gg.hypercube_graph(k)
    expect = np.array([bin(i ^ s).count("1") for i in range(1 << k)])
    assert np.array_equal(oracle.bfs(g, s), expect)


def test_disjoint_union_and_empty():
    g = gg.disjoint_union(gg.path_graph(10), gg.cycle_graph(8))
    d = oracle.bfs(g, 12)
    assert np.all(d[:10] == -1)
    assert np.array_equal(d[10:], [2, 1, 0, 1, 2, 3, 4, 3])
    e = gg.empty_graph(5)
    d = oracle.bfs(e, 3)
    assert np.array_equal(d, [-1, -1, -1, 0, -1])


def test_lollipop_long_tail():
    # K_64 plus a 300-vertex tail: the Webbase-like one-vertex-per-level case.
    g = gg.lollipop_graph(64, 300)
    d = oracle.bfs(g, 0)
    assert np.all(d[1:63] == 1) and d[63] == 1
    assert np.array_equal(d[64:], np.arange(2, 302))
    d = oracle.bfs(g, g.n - 1)
    assert d[63] == 300 and np.all(d[:63] == 301)


def test_bad_source_rejected():
    g = gg.path_graph(4)
    with pytest.raises(ValueError):
        oracle.bfs(g, 4)
    with pytest.raises(ValueError):
        oracle.bfs(g, -1)


# ---------------------------------------------------------------------------
# brute force and library routines
# ---------------------------------------------------------------------------

def floyd_warshall(g):
    """Textbook all-pairs hop distances (integer), -1 for unreachable."""
    INF = 1 << 20
    D = np.full((g.n, g.n), INF, dtype=np.int64)
    np.fill_diagonal(D, 0)
    rows = np.repeat(np.arange(g.n), np.diff(g.row_ptr))
    D[rows, g.col] = 1
    for k in range(g.n):
        D = np.minimum(D, D[:, k:k + 1] + D[k:k + 1, :])
    D[D >= INF] = -1
    return D


@pytest.mark.parametrize("seed", range(100))
def test_floyd_warshall_gnp(seed):
    n = 20 + seed % 40
    g = gg.gnp_graph(n, 0.02 + 0.002 * (seed % 30), seed=1000 + seed)
    D = floyd_warshall(g)
    for s in range(n):
        assert np.array_equal(oracle.bfs(g, s), D[s]), (seed, s)


@pytest.mark.parametrize("seed", range(100))
def test_floyd_warshall_tiny_rmat(seed):
    g = gg.rmat(6 + seed % 3, 4, seed=2000 + seed, perm_seed=3000 + seed)
    D = floyd_warshall(g)
    for s in range(g.n):
        assert np.array_equal(oracle.bfs(g, s), D[s]), (seed, s)


@pytest.mark.parametrize("scale,ef,seed", [(12, 8, 1), (14, 8, 2), (13, 16, 3)])
def test_library_shortest_path_rmat(scale, ef, seed):
    g = gg.rmat(scale, ef, seed=seed, perm_seed=seed + 100)
    srcs = gg.pick_sources(g, 4, seed=seed + 200)
    ref = shortest_path(_adj(g), method="D", unweighted=True, directed=False, indices=srcs)
    for i, s in enumerate(srcs):
        d = oracle.bfs(g, int(s))
        r = np.where(np.isinf(ref[i]), -1, ref[i]).astype(np.int32)
        assert np.array_equal(d, r)
        check_invariants(g, int(s), d)


def test_invariants_grid_with_deletions():
    g = gg.grid(64, 48, 0.05, seed=9)
    for s in [0, 1000, 3071]:
        check_invariants(g, s, oracle.bfs(g, s))


def test_invariant_checker_catches_planted_mistakes():
    """Mistakes planted in a copy of the oracle's output must be caught."""
    g = gg.rmat(10, 8, seed=5, perm_seed=6)
    s = int(gg.pick_sources(g, 1, seed=7)[0])
    d = oracle.bfs(g, s)
    check_invariants(g, s, d)
    far = int(np.argmax(d))
    for mutate in (lambda x: x.__setitem__(far, x[far] + 1),      # level too deep
                   lambda x: x.__setitem__(far, -1),              # dropped vertex
                   lambda x: x.__setitem__(s, 1),                 # root not zero
                   lambda x: x.__setitem__(np.flatnonzero(x == 2)[0], 1)):  # too shallow
        bad = d.copy()
        mutate(bad)
        with pytest.raises(AssertionError):
            check_invariants(g, s, bad)


# ---------------------------------------------------------------------------
# canonical parents
# ---------------------------------------------------------------------------

def test_parent_canonical():
    g = gg.rmat(11, 8, seed=21, perm_seed=22)
    s = int(gg.pick_sources(g, 1, seed=23)[0])
    d = oracle.bfs(g, s)
    p = oracle.parent(g, d)
    assert p[s] == s
    for v in range(g.n):
        if d[v] <= 0:
            if d[v] < 0:
                assert p[v] == -1
            continue
        nb = g.col[g.row_ptr[v]:g.row_ptr[v + 1]]
        cands = nb[d[nb] == d[v] - 1]
        assert p[v] == cands.min()


def test_parent_closed_forms():
    g = gg.path_graph(6)
    assert np.array_equal(oracle.parent(g, oracle.bfs(g, 2)), [1, 2, 2, 2, 3, 4])
    g = gg.complete_graph(5)
    assert np.array_equal(oracle.parent(g, oracle.bfs(g, 3)), [3, 3, 3, 3, 3])
    g = gg.hypercube_graph(3)
    p = oracle.parent(g, oracle.bfs(g, 0))
    for v in range(1, 8):
        hb = 1 << (v.bit_length() - 1)
        assert p[v] == v ^ hb  # clearing the highest set bit gives the smallest neighbour


def test_edges_scanned():
    g = gg.disjoint_union(gg.star_graph(5), gg.path_graph(3))
    d = oracle.bfs(g, 0)
    assert oracle.edges_scanned(g, d) == 8  # star: 4 + 4*1
    assert oracle.edges_scanned(g, d, 1, 3) == 2


# ---------------------------------------------------------------------------
# merge (Algorithm 2 Phase 2 on bitmaps) vs numpy library routines
# ---------------------------------------------------------------------------

def _bits(words, n):
    b = np.unpackbits(words.view(np.uint8), bitorder="little")[:n]
    return b.astype(bool)


@pytest.mark.parametrize("n,k,vb,ve,keep", [(1000, 0, 0, 1000, False), (4097, 3, 64, 2000, False),
                                            (777, 4, 13, 700, True), (64, 1, 0, 64, False),
                                            (130, 2, 129, 130, True)])
def test_merge_vs_numpy(n, k, vb, ve, keep):
    rng = np.random.default_rng(n + k)
    W = (n + 63) // 64
    tail = np.zeros(W * 64, dtype=bool)
    tail[:n] = True
    mask = np.packbits(tail, bitorder="little").view(np.uint64)

    def rnd(p):
        return (np.packbits(rng.random(W * 64) < p, bitorder="little").view(np.uint64) & mask)
    nxt, vis = rnd(0.1), rnd(0.3)
    inc = [rnd(0.05) for _ in range(k)]
    dist = np.where(_bits(vis, n), 3, -1).astype(np.int32)
    nxt0, vis0, dist0 = nxt.copy(), vis.copy(), dist.copy()
    tot, q = oracle.merge(n, 4, nxt, inc, vis, dist, vb, ve, keep_next=keep)
    merged = np.bitwise_or.reduce([nxt0] + inc) if inc else nxt0
    new = merged & ~vis0
    newb = _bits(new, n)
    assert tot == int(newb.sum())
    assert np.array_equal(vis, vis0 | new)
    exp_dist = dist0.copy()
    exp_dist[newb] = 5
    assert np.array_equal(dist, exp_dist)
    idx = np.flatnonzero(newb)
    assert np.array_equal(q, idx[(idx >= vb) & (idx < ve)])
    assert np.array_equal(nxt, merged if keep else np.zeros_like(nxt0))


def test_merge_all_zero_and_all_ones():
    n = 200
    W = 4
    ones = np.array([~np.uint64(0)] * 3 + [np.uint64((1 << 8) - 1)], dtype=np.uint64)
    vis = np.zeros(W, dtype=np.uint64)
    dist = np.full(n, -1, dtype=np.int32)
    tot, q = oracle.merge(n, 0, np.zeros(W, dtype=np.uint64), [ones], vis, dist, 0, n)
    assert tot == n and np.array_equal(q, np.arange(n)) and np.all(dist == 1)
    tot, q = oracle.merge(n, 1, np.zeros(W, dtype=np.uint64), [ones], vis, dist, 0, n)
    assert tot == 0 and q.size == 0


# ---------------------------------------------------------------------------
# butterfly staging: walk-through, Algorithm 2 simulation, union invariant
# ---------------------------------------------------------------------------

def _golden_walkthrough():
    rows, totals = [], []
    with open(os.path.join(GOLDEN, "butterfly_walkthrough.txt")) as f:
        for line in f:
            line = line.split("#")[0].split()
            if not line:
                continue
            if line[0] == "total":
                totals.append(tuple(int(x) for x in line[1:]))
            else:
                r, i, p = int(line[0]), int(line[1]), int(line[2])
                lo, hi = (int(x) for x in line[3].split("-"))
                rows.append((r, i, p, lo, hi))
    return rows, totals


def test_walkthrough_partners_and_blocks():
    rows, totals = _golden_walkthrough()
    for radix, i, partner, lo, hi in rows:
        assert partner in bs.butterfly_direction(0, i, radix)
        # the partner's block at the start of round i: aligned radix^i nodes
        step = radix ** i
        assert (partner // step * step, partner // step * step + step - 1) == (lo, hi)
    for radix in (2, 4):
        got = sorted(p for i in range(2 if radix == 4 else 4) for p in bs.butterfly_direction(0, i, radix))
        exp = sorted(p for r, _, p, _, _ in rows if r == radix)
        assert got == exp
    # message totals as the paper counts them (f messages per node per round,
    # depth log_2 P for fanout one and log_f P otherwise)
    for radix, P, count in totals:
        f = 1 if radix == 2 else radix
        depth = int(round(np.log(P) / np.log(radix)))
        assert P * f * depth == count
    assert bs.message_count(16, 2) == 64 and bs.message_count(16, 4) == 96


def _set(words):
    return set(np.flatnonzero(np.unpackbits(words.view(np.uint8), bitorder="little")).tolist())


@pytest.mark.parametrize("scale,P,radix,node", [(10, 16, 2, 0), (11, 16, 4, 0), (10, 4, 2, 3),
                                                (9, 16, 2, 5), (10, 16, 4, 9)])
def test_stage_matches_algorithm2_simulation(scale, P, radix, node):
    g = gg.rmat(scale, 8, seed=40 + scale, perm_seed=41)
    src = int(gg.pick_sources(g, 1, seed=42)[0])
    d = oracle.bfs(g, src)
    b = gg.partition_1d(g.row_ptr, P)
    dl, rec = bs.simulate(g, src, b, radix, node)
    for c in range(P):  # every node ends with the full distance array
        assert np.array_equal(dl[c], d)
    local, inc = oracle.stage(g, d, b, node, radix)
    assert len(rec) == local.shape[0] == int(d.max())
    for L, r in enumerate(rec):
        assert r["local"] == _set(local[L])
        flat = [s for rnd in r["rounds"] for s in rnd]
        assert len(flat) == inc.shape[1]
        for j, s in enumerate(flat):
            assert s == _set(inc[L, j])


def test_stage_union_is_next_level():
    g = gg.rmat(12, 8, seed=50, perm_seed=51)
    src = int(gg.pick_sources(g, 1, seed=52)[0])
    d = oracle.bfs(g, src)
    b = gg.partition_1d(g.row_ptr, 16)
    local, inc = oracle.stage(g, d, b, 0, 2)
    for L in range(local.shape[0]):
        u = local[L] | np.bitwise_or.reduce(inc[L], axis=0)
        assert _set(u) == set(np.flatnonzero(d == L + 1).tolist())
        # the stages are disjoint only in ownership, not in vertices; but every
        # stage holds only vertices of level L+1
        for j in range(inc.shape[1]):
            assert _set(inc[L, j]) <= set(np.flatnonzero(d == L + 1).tolist())


def test_single_node_stage_is_level_set():
    g = gg.rmat(10, 8, seed=60, perm_seed=61)
    d = oracle.bfs(g, int(gg.pick_sources(g, 1, seed=62)[0]))
    local, inc = oracle.stage(g, d, np.array([0, g.n]), 0, 2)
    assert inc.shape[1] == 0
    for L in range(local.shape[0]):
        assert _set(local[L]) == set(np.flatnonzero(d == L + 1).tolist())


def test_msbfs_u8():
    g = gg.path_graph(300)
    with pytest.raises(OverflowError):
        oracle.msbfs_u8(g, [0])
    g = gg.disjoint_union(gg.path_graph(5), gg.path_graph(3))
    out = oracle.msbfs_u8(g, [0, 6])
    assert np.array_equal(out[0], [0, 1, 2, 3, 4, 255, 255, 255])
    assert np.array_equal(out[1], [255] * 5 + [1, 0, 1])


# ---------------------------------------------------------------------------
# vertex-list messages
# ---------------------------------------------------------------------------

def test_bitmap_list_fixture():
    """Vertex v is bit v & 63 of word v >> 6; the list is ascending and stops
    below n."""
    words = np.array([1 | (1 << 5) | (1 << 63), 1, 1 << 2], dtype=np.uint64)
    assert oracle.bitmap_list(words, 131).tolist() == [0, 5, 63, 64, 130]
    assert oracle.bitmap_list(words, 130).tolist() == [0, 5, 63, 64]
    assert oracle.bitmap_list(np.zeros(4, dtype=np.uint64), 256).size == 0


def test_bitmap_list_round_trip():
    rng = np.random.default_rng(11)
    for n in (1, 63, 64, 65, 1000, 4097):
        W = (n + 63) // 64
        ids = np.unique(rng.integers(0, n, size=max(n // 7, 1)))
        bm = np.zeros(W, dtype=np.uint64)
        for v in ids:
            bm[v >> 6] |= np.uint64(1) << np.uint64(v & 63)
        assert np.array_equal(oracle.bitmap_list(bm, n), ids.astype(np.int32))


@pytest.mark.parametrize("radix", [2, 4])
def test_stage_lists_match_algorithm2_queues(radix):
    """The list form of every staged message equals, in ascending order, the
    global queue the step-by-step simulation of Algorithm 2 copied."""
    g = gg.rmat(10, 8, seed=60, perm_seed=61)
    src = int(gg.pick_sources(g, 1, seed=62)[0])
    d = oracle.bfs(g, src)
    b = gg.partition_1d(g.row_ptr, 16)
    _, rec = bs.simulate(g, src, b, radix, 0)
    local, inc = oracle.stage(g, d, b, 0, radix)
    for L, r in enumerate(rec):
        assert oracle.bitmap_list(local[L], g.n).tolist() == sorted(r["local"])
        flat = [s for rnd in r["rounds"] for s in rnd]
        for j, s in enumerate(flat):
            assert oracle.bitmap_list(inc[L, j], g.n).tolist() == sorted(s)


# ---------------------------------------------------------------------------
# bottom-up Phase 1 behind the butterfly exchange
# ---------------------------------------------------------------------------

@pytest.mark.parametrize("radix,P,node,bu", [(2, 16, 0, "all"), (4, 16, 5, "all"), (2, 8, 3, "mixed"),
                                             (4, 16, 0, "mixed")])
def test_stage_bottom_up_matches_algorithm2_simulation(radix, P, node, bu):
    """Algorithm 2 simulated with bottom-up Phase 1 steps on some levels ends
    with the plain BFS distances on every node, and every level's local set
    and received queues equal the bottom-up staging on bottom-up levels and
    the top-down staging elsewhere."""
    g = gg.rmat(10, 8, seed=70 + P, perm_seed=71)
    src = int(gg.pick_sources(g, 1, seed=72)[0])
    d = oracle.bfs(g, src)
    b = gg.partition_1d(g.row_ptr, P)
    nlev = int(d.max())
    levels = set(range(nlev + 1)) if bu == "all" else {1, 3}
    dl, rec = bs.simulate(g, src, b, radix, node, bottom_up_levels=levels)
    for c in range(P):
        assert np.array_equal(dl[c], d)
    td_local, td_inc = oracle.stage(g, d, b, node, radix)
    bu_local, bu_inc = oracle.stage_bottom_up(g.n, d, b, node, radix)
    assert len(rec) == nlev
    for L, r in enumerate(rec):
        local, inc = (bu_local, bu_inc) if L in levels else (td_local, td_inc)
        assert r["local"] == _set(local[L]), L
        flat = [s for rnd in r["rounds"] for s in rnd]
        for j, s in enumerate(flat):
            assert s == _set(inc[L, j]), (L, j)


def test_stage_bottom_up_closed_form():
    """Bottom-up messages hold only owned vertices of the next level: the
    local set is the node's range of level L+1, and local plus the incoming
    messages covers level L+1 exactly once per owner."""
    g = gg.rmat(11, 8, seed=80, perm_seed=81)
    src = int(gg.pick_sources(g, 1, seed=82)[0])
    d = oracle.bfs(g, src)
    b = gg.partition_1d(g.row_ptr, 16)
    for node in (0, 9):
        local, inc = oracle.stage_bottom_up(g.n, d, b, node, 2)
        lo, hi = int(b[node]), int(b[node + 1])
        for L in range(local.shape[0]):
            lev = set(np.flatnonzero(d == L + 1).tolist())
            assert _set(local[L]) == {v for v in lev if lo <= v < hi}
            parts = [_set(local[L])] + [_set(inc[L, j]) for j in range(inc.shape[1])]
            assert sum(len(x) for x in parts) == len(lev)  # disjoint
            assert set().union(*parts) == lev
