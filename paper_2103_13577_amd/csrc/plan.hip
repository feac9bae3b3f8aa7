// Plan set-up: input validation on the device, tier thresholds, and the
// stubs that batched execution fills in.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <string>

#include "plan.hpp"
#include "relabel.hpp"

namespace bfsk {

// Flags: 1 = row_ptr[0] != 0, 2 = row_ptr decreasing, 4 = row_ptr[last] != m,
// 8 = column id outside [0, n_global).
__global__ void k_validate(const int64_t *rp, int64_t nrows, const int32_t *col, int64_t m,
                           int64_t n_global, int32_t *flags) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  int32_t f = 0;
  if (tid == 0) {
    if (rp[0] != 0) f |= 1;
    if (rp[nrows] != m) f |= 4;
  }
  for (int64_t i = tid; i < nrows; i += stride)
    if (rp[i + 1] < rp[i]) f |= 2;
  for (int64_t e = tid; e < m; e += stride) {
    const int32_t u = col[e];
    if (u < 0 || (int64_t)u >= n_global) f |= 8;
  }
  if (f) atomicOr(flags, f);
}

bfs_status validate_graphs(Plan *p) {
  int32_t *flag = (int32_t *)((char *)p->ws + p->lay.ctl);  // scratch before any run
  for (size_t i = 0; i < p->graphs.size(); ++i) {
    const bfs_graph &g = p->graphs[i];
    hipError_t e = hipMemsetAsync(flag, 0, sizeof(int32_t), p->stream);
    if (e != hipSuccess) return p->hip_fail(e, "hipMemsetAsync");
    const int grid = p->num_cus * 8;
    hipLaunchKernelGGL(k_validate, dim3(grid), dim3(256), 0, p->stream, g.row_ptr,
                       g.v_end - g.v_begin, g.col, g.m, g.n_global, flag);
    e = hipGetLastError();
    if (e != hipSuccess) return p->hip_fail(e, "validate launch");
    int32_t h = 0;
    e = hipMemcpyAsync(&h, flag, sizeof(int32_t), hipMemcpyDeviceToHost, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return p->hip_fail(e, "validate readback");
    if (h) {
      std::string why;
      if (h & 1) why += " row_ptr[0]!=0";
      if (h & 2) why += " row_ptr decreasing";
      if (h & 4) why += " row_ptr[last]!=m";
      if (h & 8) why += " column id out of range";
      return p->fail(BFS_ERR_ARG, "graph " + std::to_string(i) + " invalid:" + why);
    }
  }
  return BFS_OK;
}

bool relabel_wanted(const bfs_graph &g, const bfs_options *o) {
  const int32_t r = o ? o->relabel : 0;
  if (r < 0) return false;
  // whole graphs only (a share's ids are global and shared with other nodes);
  // the sort helpers take 32-bit item counts
  return g.v_begin == 0 && g.v_end == g.n_global && g.m < (1ll << 31) - 1 && g.n_global > 1;
}

void layout_relabel(const bfs_graph *g, int32_t ng, const bfs_options *o, WsLayout &L, size_t &off) {
  auto take = [&](size_t bytes) {
    size_t r = off;
    off = (off + std::max<size_t>(bytes, 8) + 255) / 256 * 256;
    return r;
  };
  L.rl_rp.assign(ng, 0);
  L.rl_col.assign(ng, 0);
  L.rl_old.assign(ng, 0);
  L.rl_new.assign(ng, 0);
  RelabelSizes mx{};
  bool any = false;
  for (int i = 0; i < ng; ++i) {
    if (!relabel_wanted(g[i], o)) continue;
    any = true;
    L.rl_rp[i] = take(sizeof(int64_t) * (size_t)(g[i].n_global + 1));
    L.rl_col[i] = take(sizeof(int32_t) * (size_t)g[i].m);
    L.rl_old[i] = take(sizeof(int32_t) * (size_t)g[i].n_global);
    L.rl_new[i] = take(sizeof(int32_t) * (size_t)g[i].n_global);
    RelabelSizes s = relabel_sizes(g[i].n_global, g[i].m);
    mx.keys = std::max(mx.keys, s.keys);
    mx.tmp_col = std::max(mx.tmp_col, s.tmp_col);
    mx.temp = std::max(mx.temp, s.temp);
  }
  // scratch distances for the autotuner (whole graphs only, like relabelling)
  int64_t nmax_tune = 0;
  for (int i = 0; i < ng; ++i)
    if (g[i].v_begin == 0 && g[i].v_end == g[i].n_global && !(o && o->autotune < 0))
      nmax_tune = std::max(nmax_tune, g[i].n_global);
  L.tune_dist = nmax_tune > 0 ? take(sizeof(int32_t) * (size_t)nmax_tune) : 0;
  if (!any) return;
  L.rl_keys_a = take(mx.keys);
  L.rl_keys_b = take(mx.keys);
  L.rl_tmp_col = take(mx.tmp_col);
  L.rl_temp = take(mx.temp);
  L.rl_temp_bytes = mx.temp;
}

bfs_status relabel_graphs(Plan *p) {
  char *w = (char *)p->ws;
  for (size_t i = 0; i < p->graphs.size(); ++i) {
    if (!p->lay.rl_rp[i]) continue;
    const bfs_graph &g = p->graphs[i];
    hipError_t e = relabel_build(g.row_ptr, g.col, g.n_global, g.m, (int64_t *)(w + p->lay.rl_rp[i]),
                                 (int32_t *)(w + p->lay.rl_col[i]), (int32_t *)(w + p->lay.rl_old[i]),
                                 (int32_t *)(w + p->lay.rl_new[i]), w + p->lay.rl_keys_a,
                                 w + p->lay.rl_keys_b, w + p->lay.rl_tmp_col, w + p->lay.rl_temp,
                                 p->lay.rl_temp_bytes, p->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
    if (e != hipSuccess) return p->hip_fail(e, "relabel");
    // degrees descend with the new id: the first id without an edge, by
    // bisection over the relabelled row offsets
    const int64_t *rp = (const int64_t *)(w + p->lay.rl_rp[i]);
    int64_t lo = 0, hi = g.n_global;
    while (lo < hi) {
      const int64_t mid = lo + (hi - lo) / 2;
      int64_t r[2] = {0, 0};
      e = hipMemcpy(r, rp + mid, sizeof(r), hipMemcpyDeviceToHost);
      if (e != hipSuccess) return p->hip_fail(e, "relabel");
      if (r[1] > r[0]) lo = mid + 1;
      else hi = mid;
    }
    if (p->rl_live.size() < p->graphs.size()) p->rl_live.assign(p->graphs.size(), 0);
    p->rl_live[i] = lo;
  }
  return BFS_OK;
}

bfs_status choose_tuning(Plan *p) {
  p->tune.assign(p->graphs.size(), Tuning{});
  for (size_t i = 0; i < p->graphs.size(); ++i) {
    Tuning &t = p->tune[i];
    if (p->opt.small_bin > 0) t.small_bin = p->opt.small_bin;
    if (p->opt.wave_bin > 0) t.wave_bin = p->opt.wave_bin;
    if (p->opt.hot_words > 0) t.hot_words = p->opt.hot_words;
    if (p->opt.sparse_div > 0) t.sparse_div = p->opt.sparse_div;
    if (p->opt.sparse_div < 0) t.sparse_div = 0;
    if (p->opt.mark_mode < 0) t.mark = 0;
    // the kernels' static LDS needs under 1 KB next to the hub copy
    if ((int64_t)t.hot_words * 8 + 1024 > p->max_lds)
      return p->fail(BFS_ERR_ARG, "hot_words exceeds the LDS one workgroup may use");
    if (p->opt.chunk_edges > 0) {
      int s = 0;
      while ((1 << s) < p->opt.chunk_edges && s < 30) ++s;
      t.chunk_shift = s;
    }
    if (t.small_bin < 1 || t.small_bin > 24 || t.wave_bin < t.small_bin || t.wave_bin > 25 ||
        t.chunk_shift < 6)
      return p->fail(BFS_ERR_ARG, "bad tier thresholds");
    // untuned default: the cooperative loop with the 64-VGPR budget, one
    // block per 16K edges and vertices of the share (a small grid keeps the
    // grid barriers of small graphs cheap), between 16 blocks and 8 blocks
    // per CU; else launches per phase
    const int64_t m = p->graphs[i].m;
    t.persist_variant = p->bpc[1] > 0 ? 1 : 0;
    const int per_cu = std::min(p->bpc[t.persist_variant], 8);
    const int64_t work_grid = (m + (p->graphs[i].v_end - p->graphs[i].v_begin) + (1 << 14) - 1) >> 14;
    const int64_t max_grid = std::min(per_cu * p->num_cus, kBarrierMaxBlocks);
    t.persist_grid = (int)std::max<int64_t>(1, std::min<int64_t>(max_grid, std::max<int64_t>(work_grid, 16)));
    t.loop_mode = (p->coop && per_cu > 0) ? BFS_LOOP_PERSISTENT : BFS_LOOP_HOST;
    // small whole graphs (up to 2^20 edges): one workgroup with the bitmaps
    // in LDS
    const bfs_graph &gr = p->graphs[i];
    if (cu_fits(gr.n_global, m, gr.v_begin == 0 && gr.v_end == gr.n_global, p->max_lds) &&
        m <= (1ll << 20) && !p->opt.exchange)
      t.loop_mode = BFS_LOOP_CU;
    // an explicit loop is the one every setting is tuned and reported for
    if (p->opt.loop_mode != BFS_LOOP_AUTO) t.loop_mode = p->opt.loop_mode;
    // cstart entries are 32-bit: total chunks must stay below 2^32.
    if ((m >> t.chunk_shift) + (p->graphs[i].v_end - p->graphs[i].v_begin) >= (1ll << 32))
      return p->fail(BFS_ERR_ARG, "chunk_edges too small for this graph");
    // The workgroup-tier queue length shares a 64-bit counter with the chunk
    // total: it must stay below 2^(64-40). Its vertices have degree at least
    // 2^(wave_bin-1), so there are at most m / 2^(wave_bin-1) of them.
    const int64_t heavy_max = std::min<int64_t>(p->graphs[i].v_end - p->graphs[i].v_begin,
                                                (m >> (t.wave_bin - 1)) + 1);
    if (heavy_max >= (1ll << (64 - kHeavyShift)))
      return p->fail(BFS_ERR_ARG, "wave_bin too small for this graph (workgroup-tier queue overflow)");
  }
  return BFS_OK;
}

}  // namespace bfsk
