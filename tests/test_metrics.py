"""Measurement arithmetic: GTEPS, harmonic mean, the paper's trimmed mean."""
import os

import numpy as np

from paper_2103_13577_amd import metrics

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_gteps_reproduces_table1():
    # Table 1: |E| / DGX-2 time = DGX-2 GTEPS, within the rounding of the
    # printed two-decimal times.
    with open(os.path.join(GOLDEN, "table1_gteps.txt")) as f:
        rows = [line.split() for line in f if line.strip() and not line.startswith("#")]
    assert len(rows) == 9
    for name, e_m, t, g in rows:
        e, t, g = float(e_m) * 1e6, float(t), float(g)
        lo = metrics.gteps(e, t + 0.005)
        hi = metrics.gteps(e, max(t - 0.005, 1e-9))
        assert lo <= g <= hi, name


def test_harmonic_and_trimmed_means():
    assert metrics.harmonic_mean([1.0, 1.0]) == 1.0
    assert abs(metrics.harmonic_mean([1.0, 3.0]) - 1.5) < 1e-12
    # 100 roots: drop the 25 fastest and 25 slowest, average the rest
    t = np.arange(100, dtype=float)
    assert metrics.trimmed_mean(t) == np.mean(np.arange(25, 75))
    t = np.arange(64, dtype=float)
    assert metrics.trimmed_mean(t) == np.mean(np.arange(16, 48))


def test_algorithmic_bytes():
    # 4 B per scanned edge, 16 B per frontier vertex, 4 B per distance
    assert metrics.bytes_single_source(m_r=100, n_r=10, n=50) == 400 + 160 + 200
