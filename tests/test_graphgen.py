"""Properties of the seeded input generators and the 1D partitioner."""
import numpy as np
import pytest

import graphgen as gg


def _check_simple_symmetric(g):
    rp, col = g.row_ptr, g.col
    assert rp[0] == 0 and rp[-1] == g.m and np.all(np.diff(rp) >= 0)
    assert col.dtype == np.int32 and rp.dtype == np.int64
    assert np.all((col >= 0) & (col < g.n))
    rows = np.repeat(np.arange(g.n), np.diff(rp))
    assert not np.any(rows == col), "self-loop"
    key = rows.astype(np.int64) * g.n + col
    assert np.all(np.diff(key) > 0), "rows not sorted or duplicate edges"
    rkey = col.astype(np.int64) * g.n + rows
    assert np.array_equal(np.sort(rkey), key), "not symmetric"


@pytest.mark.parametrize("scale,ef", [(8, 4), (12, 8), (14, 16)])
def test_rmat_properties(scale, ef):
    g = gg.rmat(scale, ef, seed=1, perm_seed=2)
    assert g.n == 1 << scale
    assert g.m <= 2 * ef * g.n
    _check_simple_symmetric(g)
    deg = g.degrees()
    assert deg.max() > 8 * deg.mean(), "R-MAT degrees should be skewed"


def test_rmat_deterministic_and_seeded():
    a = gg.rmat(12, 8, seed=3, perm_seed=4)
    b = gg.rmat(12, 8, seed=3, perm_seed=4, nthreads=3)
    c = gg.rmat(12, 8, seed=5, perm_seed=4)
    assert np.array_equal(a.row_ptr, b.row_ptr) and np.array_equal(a.col, b.col)
    assert not (a.m == c.m and np.array_equal(a.col, c.col))


def test_rmat_permutation_moves_hubs():
    # with the permutation the highest-degree vertex is not pinned at id 0
    hubs = {int(np.argmax(gg.rmat(12, 8, seed=7, perm_seed=p).degrees())) for p in range(5)}
    assert len(hubs) > 1


def test_grid_properties():
    g = gg.grid(50, 40, 0.0, seed=1)
    _check_simple_symmetric(g)
    assert g.m == 2 * (49 * 40 + 50 * 39)
    h = gg.grid(200, 100, 0.01, seed=2)
    _check_simple_symmetric(h)
    full = 2 * (199 * 100 + 200 * 99)
    frac = 1 - h.m / full
    assert 0.005 < frac < 0.015


def test_from_edges_cleans_input():
    g = gg.from_edges(4, [(0, 1), (1, 0), (2, 2), (0, 1), (3, 1)])
    assert np.array_equal(g.row_ptr, [0, 1, 3, 3, 4])
    assert np.array_equal(g.col, [1, 0, 3, 1])
    with pytest.raises(ValueError):
        gg.from_edges(2, [(0, 2)])


@pytest.mark.parametrize("P", [1, 2, 4, 16])
def test_partition_1d(P):
    g = gg.rmat(14, 8, seed=11, perm_seed=12)
    b = gg.partition_1d(g.row_ptr, P)
    assert b[0] == 0 and b[-1] == g.n and np.all(np.diff(b) >= 0)
    assert np.all(b[1:-1] % 64 == 0)
    e = np.diff(g.row_ptr[b])
    # edge-balanced up to one 64-vertex word of rows per boundary
    slack = 2 * 64 * g.degrees().max()
    assert np.all(np.abs(e - g.m / P) <= slack)


def test_slice_csr():
    g = gg.rmat(10, 8, seed=1, perm_seed=2)
    rp, col = gg.slice_csr(g, 128, 512)
    assert rp[0] == 0 and rp[-1] == col.size
    assert np.array_equal(col, g.col[g.row_ptr[128]:g.row_ptr[512]])


def test_sources_and_arrivals():
    g = gg.disjoint_union(gg.star_graph(5), gg.empty_graph(5))
    s = gg.pick_sources(g, 100, seed=1)
    assert np.all(s < 5)
    t = gg.poisson_arrivals(20000, 20000.0, seed=3)
    gaps = np.diff(t)
    assert t[0] == 0 and np.all(gaps > 0)
    assert abs(gaps.mean() - 50e-6) < 2e-6
