"""Step-by-step simulation of ButterFly BFS (Algorithm 2) on P logical compute
nodes -- TEST INFRASTRUCTURE ONLY (pins :func:`oracle.stage`).

Written from the algorithm's description in Section 3, in its order and
notation: every node g keeps its own distance array d_local[g] over all |V|
vertices, a local queue of owned frontier vertices and a global queue of
everything it found this level. Phase 1 traverses the local queue; Phase 2
runs log_radix(P) exchange rounds in which node g copies the global queue of
each partner given by ButterflyDirection(g, i) and merges it. Slow pure Python,
meant for graphs of a few thousand vertices.

Readings of the paper taken here (listed with the other readings of the
paper): the partner's queue is copied as it stood at the start of the round
(every node copies before any node merges); radix 2 ("fanout one") has a
single partner per round, g XOR 2^i; radix f > 2 has the f-1 partners that
differ from g only in base-f digit i; the loop stops when no node found a
new vertex in the level.
"""
from __future__ import annotations

import numpy as np

INF = -1


def butterfly_direction(g: int, i: int, radix: int) -> list[int]:
    """Partners of node g in round i: g with base-radix digit i replaced by each
    other digit value, in ascending digit order."""
    step = radix ** i
    digit = (g // step) % radix
    base = g - digit * step
    return [base + j * step for j in range(radix) if j != digit]


def message_count(P: int, radix: int) -> int:
    """Messages sent by all nodes over one level: P * (radix-1) * depth."""
    depth = 0
    pw = 1
    while pw < P:
        pw *= radix
        depth += 1
    return P * (radix - 1) * depth


def simulate(g, root: int, bounds, radix: int = 2, record_node: int = 0, bottom_up_levels=()):
    """Run Algorithm 2 with P = len(bounds)-1 nodes. Levels listed in
    ``bottom_up_levels`` run Phase 1 bottom-up: each node checks every vertex
    it owns that it has not reached and takes it when one of its neighbours
    is in the level's frontier (every node holds all distances, so it knows
    the frontier).

    Returns (d_local, records) where d_local is int32[P, n] (-1 = infinity) and
    records[L] = {"local": set X_record_node(L),
                  "rounds": [[set received from each partner] per round]}.
    """
    n = g.n
    P = len(bounds) - 1
    depth = 0
    pw = 1
    while pw < P:
        pw *= radix
        depth += 1
    assert pw == P, "P must be a power of the radix"
    owner = np.searchsorted(np.asarray(bounds), np.arange(n), side="right") - 1
    rp, col = g.row_ptr, g.col

    d_local = np.full((P, n), INF, dtype=np.int32)
    q_local = [[] for _ in range(P)]
    for c in range(P):
        if owner[root] == c:
            q_local[c].append(root)  # only the owner enqueues the root
        d_local[c][root] = 0         # every node sets the root's distance
    level = 0
    records = []
    while True:
        # Phase 1: traversal of each node's local frontier.
        q_global = [[] for _ in range(P)]
        in_global = [set() for _ in range(P)]
        q_next = [[] for _ in range(P)]
        for c in range(P):
            if level in bottom_up_levels:
                for v in range(int(bounds[c]), int(bounds[c + 1])):
                    if d_local[c][v] != INF:
                        continue
                    for e in range(rp[v], rp[v + 1]):
                        if d_local[c][int(col[e])] == level:
                            in_global[c].add(v)
                            q_global[c].append(v)
                            d_local[c][v] = level + 1
                            q_next[c].append(v)
                            break
                continue
            for v in q_local[c]:
                for e in range(rp[v], rp[v + 1]):
                    u = int(col[e])
                    if d_local[c][u] == INF:
                        success = u not in in_global[c]
                        if success:
                            in_global[c].add(u)
                            q_global[c].append(u)
                            d_local[c][u] = level + 1
                            if owner[u] == c:
                                q_next[c].append(u)
        rec = {"local": set(in_global[record_node]), "rounds": []}
        # Phase 2: butterfly rounds; partners' queues copied at round start.
        for i in range(depth):
            snapshot = [list(q) for q in q_global]
            got = []
            for c in range(P):
                for src in butterfly_direction(c, i, radix):
                    temp = snapshot[src]
                    if c == record_node:
                        got.append(set(temp))
                    for v in temp:
                        if d_local[c][v] == INF:
                            q_global[c].append(v)
                            in_global[c].add(v)
                            d_local[c][v] = level + 1
                            if owner[v] == c:
                                q_next[c].append(v)
            rec["rounds"].append(got)
            # Synchronize(): the next round starts after every node merged.
        found_any = any(len(q) > 0 for q in q_global)
        if not found_any:
            break
        records.append(rec)
        q_local = q_next
        level += 1
    return d_local, records
