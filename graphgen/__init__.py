"""Seeded synthetic graph inputs shared by the oracle and the GPU path.

Input preparation only: R-MAT/Kronecker graphs, 2D grids with random edge
deletions, small hand-built graphs, the 1D edge-balanced vertex partition
(Section 4, "Graph Partitioning") and seeded choices of BFS sources and query
arrival times. Nothing here computes a BFS distance, a frontier or a merge.

Every graph is an undirected simple graph stored as symmetric CSR:
``row_ptr`` int64[n+1], ``col`` int32[m], each row sorted ascending, with no
self-loops and no duplicate edges (the paper's undirected conversion,
Section 4 "Inputs").
"""
from __future__ import annotations

import ctypes
import os
import subprocess
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_LIB_PATH = os.path.join(_HERE, "libgraphgen.so")
_lib = None

# Graph500 Kronecker initiator used for every R-MAT input.
RMAT_A, RMAT_B, RMAT_C = 0.57, 0.19, 0.19


def build(force: bool = True) -> str:
    """Compile the generator library in place (g++, OpenMP)."""
    src = os.path.join(_HERE, "gen.cpp")
    if force or not os.path.exists(_LIB_PATH):
        tmp = _LIB_PATH + ".tmp"
        subprocess.check_call(["g++", "-O3", "-march=x86-64-v2", "-fopenmp", "-shared", "-fPIC",
                               "-std=c++17", src, "-o", tmp])
        os.replace(tmp, _LIB_PATH)
    return _LIB_PATH


def _load():
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(_LIB_PATH):
        build(force=False)
    lib = ctypes.CDLL(_LIB_PATH)
    vp, i64, u64, dbl, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_uint64, ctypes.c_double, ctypes.c_int
    lib.gg_rmat.restype = vp
    lib.gg_rmat.argtypes = [i32, i32, dbl, dbl, dbl, u64, u64, i32]
    lib.gg_grid.restype = vp
    lib.gg_grid.argtypes = [i64, i64, dbl, u64, i32]
    lib.gg_from_edges.restype = vp
    lib.gg_from_edges.argtypes = [i64, i64, vp, vp]
    lib.gg_n.restype = i64
    lib.gg_n.argtypes = [vp]
    lib.gg_m.restype = i64
    lib.gg_m.argtypes = [vp]
    lib.gg_copy.restype = None
    lib.gg_copy.argtypes = [vp, vp, vp]
    lib.gg_free.restype = None
    lib.gg_free.argtypes = [vp]
    lib.gg_draws.restype = None
    lib.gg_draws.argtypes = [u64, i64, vp]
    _lib = lib
    return lib


@dataclass
class CSR:
    """Host CSR graph. ``row_ptr[v]..row_ptr[v+1]`` indexes ``col``."""
    n: int
    row_ptr: np.ndarray  # int64[n+1]
    col: np.ndarray      # int32[m]
    name: str = ""

    @property
    def m(self) -> int:
        return int(self.col.shape[0])

    def degrees(self) -> np.ndarray:
        return np.diff(self.row_ptr)


def _take(handle, name: str) -> CSR:
    lib = _load()
    if not handle:
        raise MemoryError(f"graph generation failed for {name}")
    try:
        n, m = lib.gg_n(handle), lib.gg_m(handle)
        row_ptr = np.empty(n + 1, dtype=np.int64)
        col = np.empty(m, dtype=np.int32)
        lib.gg_copy(handle, row_ptr.ctypes.data, col.ctypes.data)
    finally:
        lib.gg_free(handle)
    return CSR(int(n), row_ptr, col, name)


def _threads(nthreads):
    if nthreads:
        return int(nthreads)
    return int(os.environ.get("OMP_NUM_THREADS", "0") or 0) or min(16, os.cpu_count() or 1)


def rmat(scale: int, edge_factor: int, seed: int, perm_seed: int, nthreads: int = 0) -> CSR:
    """R-MAT graph, 2^scale vertices, edge_factor*2^scale undirected samples,
    initiator (0.57, 0.19, 0.19, 0.05), labels permuted from ``perm_seed``."""
    h = _load().gg_rmat(scale, edge_factor, RMAT_A, RMAT_B, RMAT_C, seed & (2**64 - 1),
                        perm_seed & (2**64 - 1), _threads(nthreads))
    return _take(h, f"rmat{scale}_ef{edge_factor}")


def grid(W: int, H: int, p_del: float, seed: int, nthreads: int = 0) -> CSR:
    """W x H 4-neighbour grid (id = y*W + x), each edge deleted with p_del."""
    h = _load().gg_grid(W, H, p_del, seed & (2**64 - 1), _threads(nthreads))
    return _take(h, f"grid{W}x{H}_p{p_del}")


def from_edges(n: int, edges, name: str = "") -> CSR:
    """Symmetric CSR from undirected edges [(u, v), ...]."""
    e = np.asarray(edges, dtype=np.int64).reshape(-1, 2)
    u = np.ascontiguousarray(e[:, 0])
    v = np.ascontiguousarray(e[:, 1])
    h = _load().gg_from_edges(n, e.shape[0], u.ctypes.data, v.ctypes.data)
    if not h:
        raise ValueError("edge endpoint out of range")
    return _take(h, name)


def draws(seed: int, count: int) -> np.ndarray:
    """``count`` seeded uniform uint64 draws (counter-based)."""
    out = np.empty(count, dtype=np.uint64)
    if count:
        _load().gg_draws(seed & (2**64 - 1), count, out.ctypes.data)
    return out


def pick_sources(g: CSR, count: int, seed: int) -> np.ndarray:
    """``count`` seeded sources, uniform over vertices with degree > 0
    (duplicates allowed)."""
    cand = np.flatnonzero(g.degrees() > 0)
    if cand.size == 0:
        return np.zeros(count, dtype=np.int64)
    r = draws(seed, count)
    return cand[(r % np.uint64(cand.size)).astype(np.int64)].astype(np.int64)


def poisson_arrivals(count: int, rate_per_s: float, seed: int) -> np.ndarray:
    """Arrival times (seconds) of an open-loop Poisson stream: exponential gaps
    with mean 1/rate from seeded uniforms."""
    r = draws(seed, count).astype(np.float64)
    u = (r + 0.5) / 18446744073709551616.0
    gaps = -np.log(u) / rate_per_s
    return np.cumsum(gaps) - gaps[0]


# ---------------------------------------------------------------------------
# 1D partitioning (Section 4, "Graph Partitioning"): consecutive vertex ranges
# with near-equal edge counts. Boundary k is the smallest v with
# row_ptr[v] >= ceil(k*m/P), rounded down to a multiple of 64 so every owned
# range starts on a bitmap word; boundary 0 = 0 and boundary P = n.
# ---------------------------------------------------------------------------

def partition_1d(row_ptr: np.ndarray, P: int) -> np.ndarray:
    n = row_ptr.shape[0] - 1
    m = int(row_ptr[-1])
    b = np.zeros(P + 1, dtype=np.int64)
    for k in range(1, P):
        target = -(-k * m // P)
        v = int(np.searchsorted(row_ptr, target, side="left"))
        v = min(v, n)
        b[k] = (v // 64) * 64
    b[P] = n
    b = np.maximum.accumulate(b)
    return b


def slice_csr(g: CSR, v_begin: int, v_end: int):
    """Owned slice of a CSR: (row_ptr rebased to 0, col of global ids)."""
    lo, hi = int(g.row_ptr[v_begin]), int(g.row_ptr[v_end])
    rp = (g.row_ptr[v_begin:v_end + 1] - lo).astype(np.int64)
    return rp, g.col[lo:hi]


# ---------------------------------------------------------------------------
# Small hand-built graphs with known structure (for closed-form tests).
# ---------------------------------------------------------------------------

def path_graph(n: int) -> CSR:
    return from_edges(n, [(i, i + 1) for i in range(n - 1)], f"path{n}")


def cycle_graph(n: int) -> CSR:
    return from_edges(n, [(i, (i + 1) % n) for i in range(n)], f"cycle{n}")


def star_graph(n: int) -> CSR:
    return from_edges(n, [(0, i) for i in range(1, n)], f"star{n}")


def complete_graph(n: int) -> CSR:
    return from_edges(n, [(i, j) for i in range(n) for j in range(i + 1, n)], f"K{n}")


def hypercube_graph(k: int) -> CSR:
    n = 1 << k
    return from_edges(n, [(i, i ^ (1 << b)) for i in range(n) for b in range(k) if i < i ^ (1 << b)],
                      f"Q{k}")


def lollipop_graph(kn: int, tail: int) -> CSR:
    """K_kn with a path of ``tail`` extra vertices hanging off vertex kn-1."""
    e = [(i, j) for i in range(kn) for j in range(i + 1, kn)]
    e += [(kn - 1 + i, kn + i) for i in range(tail)]
    return from_edges(kn + tail, e, f"lollipop{kn}_{tail}")


def empty_graph(n: int) -> CSR:
    return from_edges(n, np.zeros((0, 2), dtype=np.int64), f"empty{n}")


def disjoint_union(a: CSR, b: CSR) -> CSR:
    rp = np.concatenate([a.row_ptr[:-1], b.row_ptr + a.m]).astype(np.int64)
    col = np.concatenate([a.col, b.col + a.n]).astype(np.int32)
    return CSR(a.n + b.n, rp, col, f"{a.name}+{b.name}")


def gnp_graph(n: int, p: float, seed: int) -> CSR:
    """Erdos-Renyi G(n, p) from seeded uniform draws over the n(n-1)/2 pairs."""
    iu, ju = np.triu_indices(n, k=1)
    r = draws(seed, iu.size).astype(np.float64) / 18446744073709551616.0
    keep = r < p
    return from_edges(n, np.stack([iu[keep], ju[keep]], axis=1), f"gnp{n}_{p}")
