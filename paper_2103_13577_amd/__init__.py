"""Python binding of the MI355X BFS hot path (``libbfs.so``).

Argument marshalling only: every step of the traversal runs in the HIP
kernels behind the C ABI declared in ``include/bfs.h``. PyTorch supplies the
device memory (graphs, workspace, outputs) and the stream. If the compiled
library is missing the import of :func:`lib` raises: there is no CPU fallback.
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "libbfs.so")

BFS_OK = 0
STATUS_NAMES = {0: "OK", 1: "ERR_ARG", 2: "ERR_WORKSPACE", 3: "ERR_HIP", 4: "ERR_DEPTH",
                5: "ERR_CAPACITY", 6: "ERR_EXCHANGE", 7: "ERR_STATE", 8: "ERR_TIMEOUT",
                9: "ERR_DEVICE"}
LOOP_AUTO, LOOP_HOST, LOOP_PERSISTENT, LOOP_GRAPH, LOOP_CU, LOOP_ENQUEUE = 0, 1, 2, 3, 4, 5
DIR_TOPDOWN, DIR_OPTIMIZING = 0, 1
OUT_U8, OUT_I32 = 0, 1
BATCH_ONE_LAUNCH, BATCH_STREAMING = 1, 2
NUM_BINS = 34
MAX_LEVEL_STATS = 4096

_u64p = ctypes.POINTER(ctypes.c_uint64)
EXCHANGE_FN = ctypes.CFUNCTYPE(ctypes.c_int32, ctypes.c_void_p, ctypes.c_int32, ctypes.c_void_p,
                               ctypes.POINTER(ctypes.c_void_p), ctypes.POINTER(ctypes.c_int32))


class bfs_graph(ctypes.Structure):
    _fields_ = [("n_global", ctypes.c_int64), ("v_begin", ctypes.c_int64),
                ("v_end", ctypes.c_int64), ("m", ctypes.c_int64),
                ("row_ptr", ctypes.c_void_p), ("col", ctypes.c_void_p)]


class bfs_options(ctypes.Structure):
    _fields_ = [("hip_stream", ctypes.c_void_p), ("loop_mode", ctypes.c_int32),
                ("small_bin", ctypes.c_int32), ("wave_bin", ctypes.c_int32),
                ("chunk_edges", ctypes.c_int32), ("grid_blocks", ctypes.c_int32),
                ("batch_lanes", ctypes.c_int32), ("collect_stats", ctypes.c_int32),
                ("exchange", EXCHANGE_FN), ("exchange_ctx", ctypes.c_void_p),
                ("relabel", ctypes.c_int32), ("autotune", ctypes.c_int32),
                ("hot_words", ctypes.c_int32), ("sparse_div", ctypes.c_int32),
                ("direction", ctypes.c_int32), ("mark_mode", ctypes.c_int32),
                ("mem_budget_bytes", ctypes.c_int64), ("tune_cache", ctypes.c_char_p)]


class bfs_stats(ctypes.Structure):
    _fields_ = [("levels", ctypes.c_int32), ("reached", ctypes.c_int64),
                ("edges_scanned", ctypes.c_int64), ("ms", ctypes.c_float),
                ("loop_ms", ctypes.c_float), ("expand_ms", ctypes.c_float),
                ("merge_ms", ctypes.c_float), ("expand_launches", ctypes.c_int32),
                ("dense_edges", ctypes.c_int64), ("dense_frontier", ctypes.c_int64),
                ("queue_ms", ctypes.c_float), ("bottom_up_levels", ctypes.c_int32),
                ("bottom_up_ms", ctypes.c_float), ("bottom_up_edges", ctypes.c_int64),
                ("bottom_up_vertices", ctypes.c_int64)]


class bfs_tuning(ctypes.Structure):
    _fields_ = [("loop_mode", ctypes.c_int32), ("persist_variant", ctypes.c_int32),
                ("grid_blocks", ctypes.c_int32), ("small_bin", ctypes.c_int32),
                ("wave_bin", ctypes.c_int32), ("chunk_edges", ctypes.c_int32),
                ("relabelled", ctypes.c_int32), ("tuned_ms", ctypes.c_float),
                ("hot_words", ctypes.c_int32), ("sparse_div", ctypes.c_int32),
                ("direction", ctypes.c_int32), ("mark_mode", ctypes.c_int32)]


class bfs_query(ctypes.Structure):
    _fields_ = [("graph", ctypes.c_int32), ("out_type", ctypes.c_int32),
                ("source", ctypes.c_int64), ("out", ctypes.c_void_p)]


class bfs_batch_counters(ctypes.Structure):
    _fields_ = [("launches", ctypes.c_int64), ("levels", ctypes.c_int64),
                ("admitted", ctypes.c_int64), ("admitted_midflight", ctypes.c_int64),
                ("max_inflight", ctypes.c_int64), ("max_inflight_bytes", ctypes.c_int64),
                ("inflight_bytes", ctypes.c_int64)]


class bfs_batch_result(ctypes.Structure):
    _fields_ = [("status", ctypes.c_int32), ("nq", ctypes.c_int32),
                ("submit_ns", ctypes.c_int64), ("complete_ns", ctypes.c_int64)]


_lib = None


def lib():
    """Loads libbfs.so; raises if it has not been built."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise ImportError(f"{LIB_PATH} is missing: build it first (python __graft_entry__.py build)")
    L = ctypes.CDLL(LIB_PATH)
    vp, i32, i64, u32, u64 = (ctypes.c_void_p, ctypes.c_int32, ctypes.c_int64, ctypes.c_uint32,
                              ctypes.c_uint64)
    sig = {
        "bfs_options_default": (None, [ctypes.POINTER(bfs_options)]),
        "bfs_workspace_size": (i32, [ctypes.POINTER(bfs_graph), i32, ctypes.POINTER(bfs_options),
                                     ctypes.POINTER(ctypes.c_size_t)]),
        "bfs_plan_create": (i32, [ctypes.POINTER(bfs_graph), i32, ctypes.POINTER(bfs_options), vp,
                                  ctypes.c_size_t, ctypes.POINTER(vp)]),
        "bfs_plan_destroy": (None, [vp]),
        "bfs_last_error": (ctypes.c_char_p, [vp]),
        "bfs_run": (i32, [vp, i32, i64, vp, vp, ctypes.POINTER(bfs_stats)]),
        "bfs_begin": (i32, [vp, i32, i64, vp]),
        "bfs_expand": (i32, [vp, ctypes.POINTER(vp)]),
        "bfs_merge_frontier": (i32, [vp, ctypes.POINTER(vp), i32, i32, ctypes.POINTER(i64),
                                     ctypes.POINTER(i64)]),
        "bfs_finish": (i32, [vp, vp, ctypes.POINTER(bfs_stats)]),
        "bfs_level_stats": (i32, [vp, vp, vp, i32, ctypes.POINTER(i32)]),
        "bfs_level_times": (i32, [vp, vp, vp, vp, i32, ctypes.POINTER(i32)]),
        "bfs_run_noalloc": (i32, [ctypes.POINTER(bfs_graph), i64, vp, vp, ctypes.POINTER(i32)]),
        "bfs_plan_tuning": (i32, [vp, i32, ctypes.POINTER(bfs_tuning)]),
        "bfs_batch_submit": (i32, [vp, ctypes.POINTER(bfs_query), i32, u32, ctypes.POINTER(u64)]),
        "bfs_batch_wait": (i32, [vp, u64, i64, ctypes.POINTER(bfs_batch_result)]),
        "bfs_batch_times": (i32, [vp, u64, vp, i32]),
        "bfs_batch_poll": (i32, [vp, vp, i32, ctypes.POINTER(i32), i64]),
        "bfs_batch_tuning": (i32, [vp, ctypes.POINTER(bfs_tuning)]),
        "bfs_batch_query_bytes": (i32, [vp, i32, i32, ctypes.POINTER(i64)]),
        "bfs_batch_read_counters": (i32, [vp, ctypes.POINTER(bfs_batch_counters)]),
        "bfs_frontier_list": (i32, [vp, vp, i64, ctypes.POINTER(i64)]),
        "bfs_expand_bottom_up": (i32, [vp, ctypes.POINTER(vp)]),
        "bfs_merge_lists": (i32, [vp, ctypes.POINTER(vp), ctypes.POINTER(i64), i32,
                                  ctypes.POINTER(vp), i32, i32, ctypes.POINTER(i64),
                                  ctypes.POINTER(i64)]),
    }
    for name, (res, args) in sig.items():
        f = getattr(L, name)
        f.restype = res
        f.argtypes = args
    _lib = L
    return L


EXPORTED = ("bfs_options_default", "bfs_workspace_size", "bfs_plan_create", "bfs_plan_destroy",
            "bfs_last_error", "bfs_run", "bfs_begin", "bfs_expand", "bfs_merge_frontier",
            "bfs_finish", "bfs_level_stats", "bfs_level_times", "bfs_plan_tuning", "bfs_batch_submit",
            "bfs_batch_wait", "bfs_batch_times", "bfs_batch_poll", "bfs_batch_tuning",
            "bfs_frontier_list", "bfs_merge_lists", "bfs_expand_bottom_up", "bfs_run_noalloc",
            "bfs_batch_query_bytes", "bfs_batch_read_counters")

NOALLOC_MAX_VERTICES = 1 << 19
NOALLOC_MAX_EDGES = 1 << 25


def run_noalloc(graph: "DeviceGraph", source: int, dist=None, stream=None):
    """bfs_run_noalloc: one traversal of a small whole graph with the
    library's fixed device scratch (no plan, no workspace). Returns
    (dist, levels)."""
    torch = _torch()
    if dist is None:
        dist = torch.empty(graph.n_global, dtype=torch.int32, device=graph.row_ptr.device)
    s = stream if stream is not None else torch.cuda.current_stream()
    g = graph.c_struct()
    lv = ctypes.c_int32(0)
    st = lib().bfs_run_noalloc(ctypes.byref(g), int(source), dist.data_ptr(), s.cuda_stream,
                               ctypes.byref(lv))
    if st != BFS_OK:
        raise BfsError(st, lib().bfs_last_error(None).decode())
    return dist, int(lv.value)


class BfsError(RuntimeError):
    def __init__(self, status: int, msg: str):
        super().__init__(f"{STATUS_NAMES.get(status, status)}: {msg}")
        self.status = status


def _torch():
    import torch
    return torch


@dataclass
class DeviceGraph:
    """A graph (or one node's 1D share of it) resident in device memory."""
    n_global: int
    v_begin: int
    v_end: int
    row_ptr: object  # torch int64 cuda tensor, v_end - v_begin + 1 entries
    col: object      # torch int32 cuda tensor, m entries (global ids)

    @property
    def m(self) -> int:
        return int(self.col.numel())

    @classmethod
    def from_csr(cls, csr, device="cuda", v_begin: int = 0, v_end: int | None = None):
        torch = _torch()
        v_end = csr.n if v_end is None else v_end
        lo, hi = int(csr.row_ptr[v_begin]), int(csr.row_ptr[v_end])
        rp = np.ascontiguousarray(csr.row_ptr[v_begin:v_end + 1] - lo, dtype=np.int64)
        col = np.ascontiguousarray(csr.col[lo:hi], dtype=np.int32)
        return cls(csr.n, v_begin, v_end, torch.from_numpy(rp).to(device),
                   torch.from_numpy(col).to(device))

    def c_struct(self) -> bfs_graph:
        return bfs_graph(self.n_global, self.v_begin, self.v_end, self.m,
                         self.row_ptr.data_ptr(), self.col.data_ptr() if self.m else 0)


@dataclass
class Stats:
    """One traversal's counters and device times (the fields of ``bfs_stats``)."""
    levels: int
    reached: int
    edges_scanned: int
    ms: float
    loop_ms: float
    expand_ms: float = 0.0
    merge_ms: float = 0.0
    expand_launches: int = 0
    dense_edges: int = 0
    dense_frontier: int = 0
    queue_ms: float = 0.0
    bottom_up_levels: int = 0
    bottom_up_ms: float = 0.0
    bottom_up_edges: int = 0
    bottom_up_vertices: int = 0

    @classmethod
    def from_c(cls, st: "bfs_stats") -> "Stats":
        return cls(**{f: getattr(st, f) for f, _ in bfs_stats._fields_})


class Plan:
    """A plan over one or more device graphs (C ABI ``bfs_plan_create``).

    Owns its workspace (a torch uint8 tensor) and keeps the graphs alive.
    """

    def __init__(self, graphs, *, loop_mode=LOOP_AUTO, small_bin=0, wave_bin=0, chunk_edges=0,
                 grid_blocks=0, batch_lanes=0, collect_stats=False, exchange=None, stream=None,
                 relabel=0, autotune=0, hot_words=0, sparse_div=0, direction=0, mark_mode=0,
                 mem_budget_bytes=0, tune_cache=None):
        torch = _torch()
        L = lib()
        if isinstance(graphs, DeviceGraph):
            graphs = [graphs]
        self.graphs = list(graphs)
        self._garr = (bfs_graph * len(self.graphs))(*[g.c_struct() for g in self.graphs])
        self.stream = stream if stream is not None else torch.cuda.current_stream()
        o = bfs_options()
        L.bfs_options_default(ctypes.byref(o))
        o.hip_stream = self.stream.cuda_stream
        o.loop_mode = loop_mode
        o.small_bin, o.wave_bin, o.chunk_edges = small_bin, wave_bin, chunk_edges
        o.grid_blocks, o.batch_lanes, o.collect_stats = grid_blocks, batch_lanes, int(collect_stats)
        o.relabel = int(relabel)
        o.autotune = int(autotune)
        o.hot_words = int(hot_words)
        o.sparse_div = int(sparse_div)
        o.direction = int(direction)
        o.mark_mode = int(mark_mode)
        o.mem_budget_bytes = int(mem_budget_bytes)
        self._tune_cache = tune_cache.encode() if tune_cache else None
        o.tune_cache = self._tune_cache
        self._exchange_py = exchange
        self._exchange_keep = None
        if exchange is not None:
            self._cb = EXCHANGE_FN(self._exchange_trampoline)
            o.exchange = self._cb
        self.opts = o
        nbytes = ctypes.c_size_t(0)
        self._check(L.bfs_workspace_size(self._garr, len(self.graphs), ctypes.byref(o),
                                         ctypes.byref(nbytes)), None)
        self.workspace_bytes = int(nbytes.value)
        self.workspace = torch.empty(max(self.workspace_bytes, 256) + 256, dtype=torch.uint8,
                                     device=self.graphs[0].row_ptr.device)
        base = self.workspace.data_ptr()
        aligned = (base + 255) // 256 * 256
        h = ctypes.c_void_p(0)
        st = L.bfs_plan_create(self._garr, len(self.graphs), ctypes.byref(o), aligned,
                               self.workspace_bytes + 256 - (aligned - base), ctypes.byref(h))
        if st != BFS_OK:
            raise BfsError(st, L.bfs_last_error(None).decode())
        self.h = h

    # -- plumbing -----------------------------------------------------------
    def _check(self, st, h="self"):
        if st != BFS_OK:
            handle = self.h if h == "self" else None
            msg = lib().bfs_last_error(handle)
            raise BfsError(st, msg.decode() if msg else "")

    def _exchange_trampoline(self, ctx, level, local_next, out_ptrs, out_k):
        try:
            ptrs = self._exchange_py(int(level), int(local_next or 0))
        except Exception:  # an exception must not cross the C ABI
            return 1
        arr = (ctypes.c_void_p * max(len(ptrs), 1))(*[int(p) for p in ptrs])
        self._exchange_keep = arr
        out_ptrs[0] = ctypes.cast(arr, ctypes.c_void_p)
        out_k[0] = len(ptrs)
        return 0

    def close(self):
        if getattr(self, "h", None):
            lib().bfs_plan_destroy(self.h)
            self.h = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass

    # -- single source -------------------------------------------------------
    def run(self, graph: int, source: int, dist=None, parent: bool = False):
        """Single-source traversal. Returns (dist, parent or None, Stats)."""
        torch = _torch()
        if not 0 <= graph < len(self.graphs):
            # let the C ABI report the bad index
            self._check(lib().bfs_run(self.h, graph, int(source), None, None, None))
        g = self.graphs[graph]
        dev = g.row_ptr.device
        if dist is None:
            dist = torch.empty(g.n_global, dtype=torch.int32, device=dev)
        par = torch.empty(g.n_global, dtype=torch.int32, device=dev) if parent else None
        st = bfs_stats()
        self._check(lib().bfs_run(self.h, graph, int(source), dist.data_ptr(),
                                  par.data_ptr() if par is not None else None, ctypes.byref(st)))
        return dist, par, Stats.from_c(st)

    def begin(self, graph: int, source: int, dist):
        self._check(lib().bfs_begin(self.h, graph, int(source), dist.data_ptr()))

    def expand(self) -> int:
        """Phase 1 of the current level; returns the device address of the
        node's next-frontier bitmap."""
        p = ctypes.c_void_p(0)
        self._check(lib().bfs_expand(self.h, ctypes.byref(p)))
        return int(p.value or 0)

    def expand_bottom_up(self) -> int:
        """Phase 1 of the current level as a bottom-up step; returns the
        device address of the node's next-frontier bitmap."""
        p = ctypes.c_void_p(0)
        self._check(lib().bfs_expand_bottom_up(self.h, ctypes.byref(p)))
        return int(p.value or 0)

    def merge_frontier(self, incoming=(), keep_next: bool = False):
        """Phase 2 over device bitmaps (torch uint64/int64 tensors or raw
        addresses). Returns (global_new, owned_new) for the level so far."""
        ptrs = [x if isinstance(x, int) else x.data_ptr() for x in incoming]
        arr = (ctypes.c_void_p * max(len(ptrs), 1))(*ptrs)
        gn, on = ctypes.c_int64(0), ctypes.c_int64(0)
        self._check(lib().bfs_merge_frontier(self.h, arr, len(ptrs), int(keep_next),
                                             ctypes.byref(gn), ctypes.byref(on)))
        return int(gn.value), int(on.value)

    def frontier_list(self, out=None) -> int:
        """The node's global queue as ascending int32 ids written into `out`
        (device int32 tensor; None only counts). Returns the vertex count."""
        cnt = ctypes.c_int64(0)
        cap = 0 if out is None else out.numel()
        self._check(lib().bfs_frontier_list(self.h, None if out is None else out.data_ptr(), cap,
                                            ctypes.byref(cnt)))
        return int(cnt.value)

    def merge_lists(self, lists=(), bitmaps=(), keep_next: bool = False):
        """Phase 2 over incoming vertex lists -- (device int32 tensor, count)
        pairs, or tensors whose length is the count -- and bitmaps, in one
        pass. Returns (global_new, owned_new) for the level so far."""
        items = [(x, x.numel()) if not isinstance(x, tuple) else x for x in lists]
        n = max(len(items), 1)
        ptrs = (ctypes.c_void_p * n)(*[t.data_ptr() if c > 0 else None for t, c in items])
        cnts = (ctypes.c_int64 * n)(*[int(c) for _, c in items])
        bps = [x if isinstance(x, int) else x.data_ptr() for x in bitmaps]
        barr = (ctypes.c_void_p * max(len(bps), 1))(*bps)
        gn, on = ctypes.c_int64(0), ctypes.c_int64(0)
        self._check(lib().bfs_merge_lists(self.h, ptrs, cnts, len(items), barr, len(bps),
                                          int(keep_next), ctypes.byref(gn), ctypes.byref(on)))
        return int(gn.value), int(on.value)

    def finish(self, parent=None) -> Stats:
        st = bfs_stats()
        self._check(lib().bfs_finish(self.h, parent.data_ptr() if parent is not None else None,
                                     ctypes.byref(st)))
        return Stats.from_c(st)

    def tuning(self, graph: int = 0) -> dict:
        """Settings the plan uses for one graph (after autotuning)."""
        t = bfs_tuning()
        self._check(lib().bfs_plan_tuning(self.h, graph, ctypes.byref(t)))
        return {f: getattr(t, f) for f, _ in bfs_tuning._fields_}

    def batch_tuning(self) -> dict:
        """Settings of the batched engine (after the batch autotuner)."""
        t = bfs_tuning()
        self._check(lib().bfs_batch_tuning(self.h, ctypes.byref(t)))
        return {f: getattr(t, f) for f, _ in bfs_tuning._fields_}

    def level_stats(self):
        """(frontier sizes per level, degree-bin histogram [levels, 34])."""
        f = np.zeros(MAX_LEVEL_STATS, dtype=np.int64)
        h = np.zeros((MAX_LEVEL_STATS, NUM_BINS), dtype=np.int64)
        nl = ctypes.c_int32(0)
        self._check(lib().bfs_level_stats(self.h, f.ctypes.data, h.ctypes.data, MAX_LEVEL_STATS,
                                          ctypes.byref(nl)))
        return f[:nl.value].copy(), h[:nl.value].copy()

    def level_times(self):
        """(Phase 1 ms, Phase 2 ms, kind) per level of the last host-driven or
        enqueued-step traversal (kind 0 top-down, 1 queue-only, 2 bottom-up)."""
        n = 64
        a = np.zeros(n, dtype=np.float32)
        b = np.zeros(n, dtype=np.float32)
        k = np.zeros(n, dtype=np.int32)
        nl = ctypes.c_int32(0)
        self._check(lib().bfs_level_times(self.h, a.ctypes.data, b.ctypes.data, k.ctypes.data, n,
                                          ctypes.byref(nl)))
        return a[:nl.value].copy(), b[:nl.value].copy(), k[:nl.value].copy()

    # -- batched / serving -----------------------------------------------------
    def batch_submit(self, queries, flags=BATCH_ONE_LAUNCH) -> int:
        """queries: list of (graph, source, out_tensor). Returns a ticket."""
        torch = _torch()
        arr = (bfs_query * max(len(queries), 1))()
        for i, (gi, s, out) in enumerate(queries):
            ot = OUT_U8 if out.dtype == torch.uint8 else OUT_I32
            arr[i] = bfs_query(int(gi), ot, int(s), out.data_ptr())
        t = ctypes.c_uint64(0)
        self._check(lib().bfs_batch_submit(self.h, arr, len(queries), flags, ctypes.byref(t)))
        return int(t.value)

    def batch_wait(self, ticket: int, timeout_us: int = -1) -> bfs_batch_result:
        r = bfs_batch_result()
        self._check(lib().bfs_batch_wait(self.h, ticket, timeout_us, ctypes.byref(r)))
        return r

    def batch_poll(self, max_tickets: int = 1024, timeout_us: int = -1) -> list:
        """Ids of tickets finished since the previous poll (may be empty on
        timeout)."""
        buf = np.zeros(max_tickets, dtype=np.uint64)
        n = ctypes.c_int32(0)
        self._check(lib().bfs_batch_poll(self.h, buf.ctypes.data, max_tickets, ctypes.byref(n),
                                         timeout_us))
        return [int(x) for x in buf[:n.value]]

    def batch_query_bytes(self, graph: int, out_type: int = OUT_I32) -> int:
        """Admission cost of one batched query on `graph` (bytes)."""
        b = ctypes.c_int64(0)
        self._check(lib().bfs_batch_query_bytes(self.h, graph, out_type, ctypes.byref(b)))
        return int(b.value)

    def batch_counters(self) -> dict:
        """Counters of the batched engine over the caller's queries."""
        c = bfs_batch_counters()
        self._check(lib().bfs_batch_read_counters(self.h, ctypes.byref(c)))
        return {f: getattr(c, f) for f, _ in bfs_batch_counters._fields_}

    def batch_times(self, ticket: int, nq: int) -> np.ndarray:
        out = np.zeros(nq, dtype=np.int64)
        self._check(lib().bfs_batch_times(self.h, ticket, out.ctypes.data, nq))
        return out
