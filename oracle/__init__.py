"""CPU oracle for the BFS hot path -- TEST INFRASTRUCTURE ONLY.

Only the test suite, the smoke check and the benchmark's CPU-baseline leg may
import this package. The GPU library neither links nor calls it, and this
package imports nothing from the GPU library; the two share only the seeded
input generators in ``graphgen``.

Functions and the passages they follow:

* :func:`bfs` -- hop distances from a root, -1 for unreachable (Section 2,
  Preliminaries; Algorithm 1). Plain FIFO BFS in C (``bfs_oracle.c``).
* :func:`parent` -- canonical parent (smallest-id neighbour one level closer);
  the paper has no parent array, this is our reading.
* :func:`stage` -- per-level butterfly messages received by one compute node
  (Algorithm 2 Phase 1 sets X_c(L), exchanged along Figures 1/2).
* :func:`merge` -- Algorithm 2 Phase 2 on bitmaps.
* :func:`bitmap_list` -- a bitmap message as the ascending list of its
  vertices (Section 3: Phase 2 exchanges lists of active vertices).
* :func:`stage_bottom_up` -- the butterfly messages of a level whose Phase 1
  is a bottom-up step (Section 3 allows bottom-up traversals behind the same
  exchange): each node finds exactly its owned vertices of the next level.
* :func:`msbfs_u8` -- per-source BFS written as uint8 distances (255 means
  unreachable), for the batched multi-source path.
* :mod:`oracle.butterfly_sim` -- a step-by-step simulation of Algorithm 2 with
  P logical compute nodes, used to pin :func:`stage`.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "liboracle.so")
_lib = None


def build(force: bool = True) -> str:
    src = os.path.join(_HERE, "bfs_oracle.c")
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["gcc", "-O2", "-std=c99", "-shared", "-fPIC", src, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int32
    lib.oracle_bfs.restype = i64
    lib.oracle_bfs.argtypes = [i64, vp, vp, i64, vp]
    lib.oracle_parent.restype = None
    lib.oracle_parent.argtypes = [i64, vp, vp, vp, vp]
    lib.oracle_edges_scanned.restype = i64
    lib.oracle_edges_scanned.argtypes = [vp, vp, i64, i64]
    lib.oracle_stage.restype = i32
    lib.oracle_stage.argtypes = [i64, vp, vp, vp, i32, vp, i32, i32, i32, vp, vp]
    lib.oracle_merge.restype = i64
    lib.oracle_merge.argtypes = [i64, i32, vp, vp, i32, vp, vp, i64, i64, i32, vp, vp]
    _lib = lib
    return lib


def _c(a, dtype):
    a = np.ascontiguousarray(a, dtype=dtype)
    return a


def bfs(g, src: int) -> np.ndarray:
    """int32 hop distances from ``src`` (-1 = unreachable)."""
    lib = _load()
    rp, col = _c(g.row_ptr, np.int64), _c(g.col, np.int32)
    dist = np.empty(g.n, dtype=np.int32)
    r = lib.oracle_bfs(g.n, rp.ctypes.data, col.ctypes.data, int(src), dist.ctypes.data)
    if r < 0:
        raise ValueError(f"oracle_bfs: bad source {src} for n={g.n}")
    return dist


def parent(g, dist: np.ndarray) -> np.ndarray:
    lib = _load()
    rp, col = _c(g.row_ptr, np.int64), _c(g.col, np.int32)
    d = _c(dist, np.int32)
    par = np.empty(g.n, dtype=np.int32)
    lib.oracle_parent(g.n, rp.ctypes.data, col.ctypes.data, d.ctypes.data, par.ctypes.data)
    return par


def edges_scanned(g, dist: np.ndarray, v_begin: int = 0, v_end: int | None = None) -> int:
    lib = _load()
    v_end = g.n if v_end is None else v_end
    rp = _c(g.row_ptr, np.int64)
    d = _c(dist, np.int32)
    return int(lib.oracle_edges_scanned(rp.ctypes.data, d.ctypes.data, int(v_begin), int(v_end)))


def stage(g, dist: np.ndarray, bounds: np.ndarray, node: int = 0, radix: int = 2):
    """Butterfly inputs for compute node ``node``.

    Returns ``(local, incoming)`` with ``local`` uint64[nlev, W] = X_node(L) and
    ``incoming`` uint64[nlev, K, W] with K = depth*(radix-1), ordered by round
    then by partner digit (ascending, skipping the node's own digit).
    """
    lib = _load()
    P = len(bounds) - 1
    nlev = int(max(int(dist.max()), 0))
    W = (g.n + 63) // 64
    depth = 0
    pw = 1
    while pw < P:
        pw *= radix
        depth += 1
    if pw != P:
        raise ValueError("P must be a power of the radix")
    K = depth * (radix - 1)
    local = np.zeros((max(nlev, 1), W), dtype=np.uint64)
    inc = np.zeros((max(nlev, 1), max(K, 1), W), dtype=np.uint64)
    rp, col = _c(g.row_ptr, np.int64), _c(g.col, np.int32)
    d = _c(dist, np.int32)
    b = _c(bounds, np.int64)
    r = lib.oracle_stage(g.n, rp.ctypes.data, col.ctypes.data, d.ctypes.data, P, b.ctypes.data,
                         node, radix, nlev, local.ctypes.data, inc.ctypes.data)
    if r < 0:
        raise ValueError("oracle_stage: bad arguments")
    return local[:nlev], inc[:nlev, :K]


def merge(n: int, level: int, next_bm: np.ndarray, incoming, visited: np.ndarray,
          dist: np.ndarray, v_begin: int, v_end: int, keep_next: bool = False):
    """Algorithm 2 Phase 2 on bitmaps; updates next_bm, visited, dist in place.
    Returns (global_new, owned_queue)."""
    lib = _load()
    assert next_bm.dtype == np.uint64 and visited.dtype == np.uint64 and dist.dtype == np.int32
    inc = [np.ascontiguousarray(x, dtype=np.uint64) for x in incoming]
    ptrs = (ctypes.c_void_p * max(len(inc), 1))(*[x.ctypes.data for x in inc])
    q = np.empty(max(v_end - v_begin, 1), dtype=np.int32)
    owned = ctypes.c_int64(0)
    tot = lib.oracle_merge(n, level, next_bm.ctypes.data, ptrs, len(inc), visited.ctypes.data,
                           dist.ctypes.data, v_begin, v_end, int(keep_next), q.ctypes.data,
                           ctypes.byref(owned))
    return int(tot), q[:owned.value].copy()


def bitmap_list(bm: np.ndarray, n: int) -> np.ndarray:
    """Ascending int32 ids v < n whose bit is set (vertex v is bit v & 63 of
    uint64 word v >> 6): the vertex-list form of a butterfly message."""
    words = np.ascontiguousarray(bm, dtype=np.uint64)
    ids = []
    for w in np.flatnonzero(words):
        x = int(words[w])
        b = 0
        while x:
            if x & 1 and 64 * int(w) + b < n:
                ids.append(64 * int(w) + b)
            x >>= 1
            b += 1
    return np.asarray(ids, dtype=np.int32)


def stage_bottom_up(n: int, dist: np.ndarray, bounds: np.ndarray, node: int = 0, radix: int = 2,
                    levels=None):
    """Butterfly inputs for compute node ``node`` when Phase 1 of every level
    is a bottom-up step, in the layout of :func:`stage`.

    A bottom-up step of node c marks every unvisited vertex it owns that has a
    neighbour in the level-L frontier, which is every owned vertex at distance
    L+1, so X_c(L) = {u owned by c : d[u] = L+1}. In round i the partner that
    differs from ``node`` in base-radix digit i sends the union of X_c over its
    aligned block of radix^i nodes (the queues it has merged so far). With
    ``levels`` given, only those levels are filled (the others stay empty).
    """
    P = len(bounds) - 1
    depth, pw = 0, 1
    while pw < P:
        pw *= radix
        depth += 1
    if pw != P:
        raise ValueError("P must be a power of the radix")
    K = depth * (radix - 1)
    nlev = int(max(int(dist.max()), 0))
    W = (n + 63) // 64
    bounds = np.asarray(bounds, dtype=np.int64)

    def bitmap(lev, first_node, count):
        # bit v (v in the nodes' ranges) = lev[v]; bit v is bit v & 63 of word v >> 6
        a, b = int(bounds[first_node]), int(bounds[first_node + count])
        sel = np.zeros(W * 64, dtype=bool)
        sel[a:b] = lev[a:b]
        return np.packbits(sel, bitorder="little").view("<u8").astype(np.uint64)

    local = np.zeros((nlev, W), dtype=np.uint64)
    inc = np.zeros((nlev, K, W), dtype=np.uint64)
    for L in range(nlev):
        if levels is not None and L not in levels:
            continue
        lev = dist == L + 1
        local[L] = bitmap(lev, node, 1)
        k = 0
        for i in range(depth):
            step = radix ** i
            digit = (node // step) % radix
            for j in range(radix):
                if j == digit:
                    continue
                partner = node + (j - digit) * step
                lo = (partner // step) * step  # the partner's block of radix^i nodes
                inc[L, k] = bitmap(lev, lo, step)
                k += 1
    return local, inc


def msbfs_u8(g, sources) -> np.ndarray:
    """uint8 distances [len(sources), n], 255 = unreachable. Raises if a
    reachable vertex is deeper than 254."""
    out = np.empty((len(sources), g.n), dtype=np.uint8)
    for i, s in enumerate(sources):
        d = bfs(g, int(s))
        if d.max() > 254:
            raise OverflowError("depth above 254 does not fit uint8 distances")
        out[i] = np.where(d < 0, 255, d).astype(np.uint8)
    return out
