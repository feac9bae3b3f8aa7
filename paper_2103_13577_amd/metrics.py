"""Measurement arithmetic for the benchmark (host side, no GPU).

GTEPS follows the paper's convention (traversed edges / time, Table 1) and
its root protocol (Section 4 "Inputs": 100 random roots, the 25 fastest and
25 slowest times dropped, the rest averaged).
"""
from __future__ import annotations

import numpy as np


def gteps(edges: float, seconds: float) -> float:
    return float(edges) / float(seconds) / 1e9


def harmonic_mean(xs) -> float:
    xs = np.asarray(xs, dtype=np.float64)
    return float(xs.size / np.sum(1.0 / xs))


def trimmed_mean(times, drop_frac: float = 0.25) -> float:
    t = np.sort(np.asarray(times, dtype=np.float64))
    k = int(np.floor(t.size * drop_frac))
    return float(np.mean(t[k:t.size - k]))


def bytes_single_source(m_r: int, n_r: int, n: int) -> int:
    """Algorithmic HBM bytes of one top-down traversal: every scanned column
    index once (4 B), two int64 row offsets per frontier vertex (16 B) and the
    int32 distance array written once (4 B per vertex)."""
    return 4 * int(m_r) + 16 * int(n_r) + 4 * int(n)


def percentile(xs, q: float) -> float:
    return float(np.percentile(np.asarray(xs, dtype=np.float64), q))
