"""bfs_run_noalloc (the traversal entry point that allocates nothing, with its
scratch in the library's fixed device array) against bfs_run on the same
inputs, through the C ABI: two calls in a row, the second on a smaller graph,
each equal to bfs_run's output and to the oracle."""
import numpy as np
import pytest

import graphgen as gg
import oracle
import paper_2103_13577_amd as pkg

pytestmark = pytest.mark.gpu


def _plan_run(dg, s, **opts):
    import torch
    plan = pkg.Plan([dg], **opts)
    d, _, st = plan.run(0, s)
    torch.cuda.synchronize()
    out = d.cpu().numpy(), st.levels
    plan.close()
    return out


def test_noalloc_matches_bfs_run(gpu):
    import torch
    big = gg.rmat(17, 16, seed=501, perm_seed=502)  # 131072 vertices
    small = gg.grid(60, 40, 0.02, seed=503)          # 2400 vertices, ~100 levels
    for g, seed in ((big, 504), (small, 505)):
        dg = pkg.DeviceGraph.from_csr(g, gpu)
        s = int(gg.pick_sources(g, 1, seed=seed)[0])
        print(f"[gpu] noalloc n={g.n} m={g.m} src={s}", flush=True)
        d, levels = pkg.run_noalloc(dg, s)
        torch.cuda.synchronize()
        got = d.cpu().numpy()
        ref_run, ref_levels = _plan_run(dg, s)
        ref_cu, _ = _plan_run(dg, s, loop_mode=pkg.LOOP_CU, relabel=-1)
        assert np.array_equal(got, ref_run)
        assert np.array_equal(got, ref_cu)
        assert np.array_equal(got, oracle.bfs(g, s))
        assert levels == ref_levels


def test_noalloc_rejects_large_graphs(gpu):
    import torch
    g = gg.rmat(20, 1, seed=506, perm_seed=507)  # 1,048,576 vertices > the limit
    dg = pkg.DeviceGraph.from_csr(g, gpu)
    with pytest.raises(pkg.BfsError) as e:
        pkg.run_noalloc(dg, 0)
    assert e.value.status == 5
    # a share (not a whole graph) is an argument error
    share = pkg.DeviceGraph(g.n, 0, 64, dg.row_ptr[:65].clone() - 0, dg.col)
    with pytest.raises(pkg.BfsError) as e:
        pkg.run_noalloc(share, 0)
    assert e.value.status in (1, 5)
    torch.cuda.synchronize()
