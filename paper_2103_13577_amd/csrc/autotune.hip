// Plan-time autotuner: times a few whole traversals from four sources per
// candidate setting on the plan's own graph and keeps the fastest. Candidates: the level loop
// (host-driven launches per phase, a captured graph of level steps, the
// cooperative persistent loop with either register budget and several grid
// sizes, or one workgroup for small graphs), the degree-bin thresholds that
// split the frontier into the lane-group, wavefront and chunked tiers, the
// hub chunk size, the LDS hub copy, the queue-only level threshold and, for
// all-dense traversals, byte marks against atomic ORs. Settings given
// explicitly in the options are never changed; a tuning cache file (the
// tune_cache option) records the outcome per graph, device and options.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <vector>

#include "plan.hpp"

namespace bfsk {

namespace {

bool tune_wanted(const Plan *p, size_t gi) {
  const int a = p->opt.autotune;
  if (a < 0 || p->opt.exchange) return false;
  const bfs_graph &g = p->graphs[gi];
  if (g.v_begin != 0 || g.v_end != g.n_global) return false;
  if (a == 0 && g.m < (1ll << 16)) return false;
  return true;
}

// Sources with at least one edge, in caller ids, placed like typical
// sources (a traversal's level profile depends on where it starts). On a
// relabelled graph: the vertices at degree ranks z/8, z/4, z/2 and 3z/4, z the
// number of vertices with an edge (recorded when the graph was relabelled).
// Else up to four vertices with an edge spread over the first 2^16 ids.
bfs_status pick_sources(Plan *p, size_t gi, std::vector<int64_t> &srcs) {
  const bfs_graph &g = p->graphs[gi];
  srcs.clear();
  char *w = (char *)p->ws;
  if (p->lay.rl_old[gi] && p->rl_live.size() > gi) {
    const int32_t *old_id = (const int32_t *)(w + p->lay.rl_old[gi]);
    const int64_t z = std::max<int64_t>(p->rl_live[gi], 1);
    for (int64_t k : {z / 8, z / 4, z / 2, 3 * z / 4}) {
      int32_t v = 0;
      hipError_t e = hipMemcpy(&v, old_id + k, sizeof(int32_t), hipMemcpyDeviceToHost);
      if (e != hipSuccess) return p->hip_fail(e, "autotune sources");
      if (std::find(srcs.begin(), srcs.end(), (int64_t)v) == srcs.end()) srcs.push_back(v);
    }
    return BFS_OK;
  }
  const int64_t cnt = std::min<int64_t>(g.n_global, 1 << 16);
  std::vector<int64_t> rp((size_t)cnt + 1);
  hipError_t e = hipMemcpy(rp.data(), g.row_ptr, sizeof(int64_t) * (cnt + 1), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return p->hip_fail(e, "autotune sources");
  for (int q = 0; q < 4; ++q)
    for (int64_t v = q * cnt / 4; v < cnt; ++v)
      if (rp[v + 1] > rp[v]) {
        if (std::find(srcs.begin(), srcs.end(), v) == srcs.end()) srcs.push_back(v);
        break;
      }
  if (srcs.empty()) srcs.push_back(0);
  return BFS_OK;
}

// Sum over the sources of the median of three timed traversals after one
// warm-up (the first source's second warm-up alone, scaled to all sources,
// when it is already three times slower than the best so far: a kernel's
// first launch in a process carries one-time set-up costs, so the first
// warm-up alone cannot rule a candidate out).
bfs_status time_config(Plan *p, int32_t gi, const std::vector<int64_t> &srcs, float best, float &ms) {
  int32_t *dist = (int32_t *)((char *)p->ws + p->lay.tune_dist);
  bfs_stats st;
  ms = 0.f;
  for (size_t i = 0; i < srcs.size(); ++i) {
    bfs_status s = bfs_run(p, gi, srcs[i], dist, nullptr, &st);
    if (s) return s;
    if (i == 0 && st.ms * (float)srcs.size() > 3.f * best) {
      s = bfs_run(p, gi, srcs[i], dist, nullptr, &st);
      if (s) return s;
      if (st.ms * (float)srcs.size() > 3.f * best) {
        ms = st.ms * (float)srcs.size();
        return BFS_OK;
      }
    }
    float t[3];
    for (float &x : t) {
      s = bfs_run(p, gi, srcs[i], dist, nullptr, &st);
      if (s) return s;
      x = st.ms;
    }
    std::sort(t, t + 3);
    ms += t[1];
  }
  return BFS_OK;
}

// Times the candidates for graph gi and leaves the fastest in p->tune[gi].
bfs_status tune_graph(Plan *p, size_t gi) {
  {
    std::vector<int64_t> src;
    bfs_status s = pick_sources(p, gi, src);
    if (s) return s;
    Tuning &t = p->tune[gi];
    Tuning best = t;
    float best_ms = 1e30f;
    auto trial = [&](const Tuning &c) -> bfs_status {
      const Tuning keep = t;
      t = c;
      float ms = 0.f;
      bfs_status r = time_config(p, (int32_t)gi, src, best_ms, ms);
      if (r == BFS_OK && ms < best_ms) {
        best_ms = ms;
        best = c;
      }
      t = keep;
      return r;
    };
    // 1. level loop, register budget and grid size
    std::vector<Tuning> loops;
    if (p->opt.loop_mode == BFS_LOOP_AUTO) {
      Tuning h = t;
      h.loop_mode = BFS_LOOP_HOST;
      loops.push_back(h);
      h.loop_mode = BFS_LOOP_GRAPH;
      loops.push_back(h);
      // the per-phase loops run the large levels with an LDS hub copy on a
      // relabelled graph, which the cooperative loop does not: compare them
      // with one too, or the loop choice is made without their main advantage
      // the largest hub copy one workgroup's LDS holds (next to 1 KB of static LDS)
      int hw = (int)std::min<int64_t>((p->max_lds - 1024) / 8, kMaxHotWords);
      if (p->lay.rl_rp[gi] && p->opt.hot_words == 0 && (int64_t)hw * 8 + 1024 <= p->max_lds) {
        h.hot_words = hw;
        h.loop_mode = BFS_LOOP_HOST;
        loops.push_back(h);
        h.loop_mode = BFS_LOOP_GRAPH;
        loops.push_back(h);
      }
    }
    if (p->coop && (p->opt.loop_mode == BFS_LOOP_AUTO || p->opt.loop_mode == BFS_LOOP_PERSISTENT)) {
      // grids: all co-resident blocks, half of them, one block per CU, one
      // per four CUs, 32 and 8 blocks (every block pays each grid barrier's
      // release and acquire, so small graphs want few blocks)
      for (int var = 0; var < 2; ++var) {
        const int bpc = p->bpc[var];
        if (bpc <= 0) continue;
        const int cap = std::min(bpc * p->num_cus, kBarrierMaxBlocks);
        int last = -1;
        for (int grid : {cap, (bpc / 2) * p->num_cus, p->num_cus, p->num_cus / 4, 32, 8}) {
          grid = std::min(grid, cap);
          if (p->persist_grid > 0) grid = p->persist_grid;
          if (grid <= 0 || grid == last) continue;
          last = grid;
          Tuning c = t;
          c.loop_mode = BFS_LOOP_PERSISTENT;
          c.persist_variant = var;
          c.persist_grid = grid;
          loops.push_back(c);
          if (p->persist_grid > 0) break;
        }
      }
    }
    if (p->opt.loop_mode == BFS_LOOP_AUTO &&
        cu_fits(p->graphs[gi].n_global, p->graphs[gi].m, true, p->max_lds)) {
      Tuning c = t;
      c.loop_mode = BFS_LOOP_CU;
      loops.push_back(c);
    }
    if (p->direction_optimizing((int32_t)gi)) {  // bfs_run then always drives the levels itself
      loops.clear();
      Tuning h = t;
      h.loop_mode = BFS_LOOP_HOST;
      loops.push_back(h);
    }
    if (loops.empty()) loops.push_back(t);
    for (const Tuning &c : loops)
      if ((s = trial(c))) return s;
    t = best;
    if (best.loop_mode == BFS_LOOP_CU) {  // the tier settings do not apply
      t.tuned_ms = best_ms / (float)src.size();
      return BFS_OK;
    }
    // 2. tier thresholds (degree bins), each kept only if it helps
    if (p->opt.small_bin <= 0)
      for (int sb : {4, 5, 7, 8, 9, 10, 11}) {
        Tuning c = best;
        c.small_bin = sb;
        if (c.wave_bin < sb) continue;
        if ((s = trial(c))) return s;
      }
    t = best;
    if (p->opt.wave_bin <= 0)
      for (int wb : {11, 15}) {
        Tuning c = best;
        c.wave_bin = std::max(wb, c.small_bin);
        const int64_t heavy_max = std::min<int64_t>(p->graphs[gi].n_global,
                                                    (p->graphs[gi].m >> (c.wave_bin - 1)) + 1);
        if (heavy_max >= (1ll << (64 - kHeavyShift))) continue;
        if ((s = trial(c))) return s;
      }
    t = best;
    // LDS copy of the hubs' visited bits (relabelled graphs only)
    if (p->lay.rl_rp[gi] && best.loop_mode != BFS_LOOP_PERSISTENT && p->opt.hot_words == 0)
      for (int hw : {1024, 2048, 4096, 8192, 16384, (int)std::min<int64_t>((p->max_lds - 1024) / 8, kMaxHotWords)}) {
        if ((int64_t)hw * 8 + 1024 > p->max_lds) continue;
        Tuning c = best;
        c.hot_words = hw;
        if ((s = trial(c))) return s;
      }
    t = best;
    if (p->opt.chunk_edges <= 0)
      for (int cs : {10, 12}) {
        Tuning c = best;
        c.chunk_shift = cs;
        if ((s = trial(c))) return s;
      }
    t = best;
    // queue-only levels: never, or below a larger share of the bitmap sweep
    if (p->opt.sparse_div == 0)
      for (int sd : {0, 16, 64}) {
        Tuning c = best;
        c.sparse_div = sd;
        if ((s = trial(c))) return s;
      }
    t = best;
    // dense levels: byte marks against atomic ORs into the bitmap
    if (p->opt.mark_mode == 0) {
      Tuning c = best;
      c.mark = 0;
      if ((s = trial(c))) return s;
    }
    t = best;
    t.tuned_ms = best_ms / (float)src.size();
  }
  return BFS_OK;
}

// Tuning cache. A line per tuned graph:
//   bfs-tune <key> loop= variant= grid= small= wave= chunk= sparse= hot= mark= ms=
// The key hashes (FNV-1a, 64 bits) the device (name, architecture, compute
// units), the graph's sizes and 129 sampled row offsets and column ids, and
// every option the autotuner must respect.
struct Fnv {
  uint64_t h = 1469598103934665603ull;
  void add(const void *d, size_t n) {
    const unsigned char *c = (const unsigned char *)d;
    for (size_t i = 0; i < n; ++i) h = (h ^ c[i]) * 1099511628211ull;
  }
  template <class T>
  void add(const T &x) {
    add(&x, sizeof(T));
  }
};

bfs_status tune_key(Plan *p, size_t gi, uint64_t &key) {
  const bfs_graph &g = p->graphs[gi];
  Fnv f;
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess)
    return p->fail(BFS_ERR_HIP, "tune cache: no device properties");
  f.add(prop.name, strnlen(prop.name, sizeof(prop.name)));
  f.add(prop.gcnArchName, strnlen(prop.gcnArchName, sizeof(prop.gcnArchName)));
  f.add(p->num_cus);
  f.add(g.n_global);
  f.add(g.v_begin);
  f.add(g.v_end);
  f.add(g.m);
  const int64_t nrows = g.v_end - g.v_begin;
  for (int k = 0; k <= 64; ++k) {
    int64_t v = 0;
    hipError_t e = hipMemcpy(&v, g.row_ptr + nrows * k / 64, sizeof(v), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return p->hip_fail(e, "tune cache key");
    f.add(v);
  }
  for (int k = 0; k < 64 && g.m > 0; ++k) {
    int32_t c = 0;
    hipError_t e = hipMemcpy(&c, g.col + g.m * k / 64, sizeof(c), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return p->hip_fail(e, "tune cache key");
    f.add(c);
  }
  const bfs_options &o = p->opt;
  const int32_t opts[] = {o.loop_mode, o.small_bin, o.wave_bin, o.chunk_edges, o.grid_blocks, o.relabel,
                          o.hot_words, o.sparse_div, o.direction, o.mark_mode};
  f.add(opts, sizeof(opts));
  key = f.h;
  return BFS_OK;
}

bool read_cache(const char *path, uint64_t key, Tuning &t) {
  FILE *fp = fopen(path, "r");
  if (!fp) return false;
  char line[512];
  bool found = false;
  Tuning c = t;
  while (fgets(line, sizeof(line), fp)) {
    unsigned long long k = 0;
    int loop, var, grid, sb, wb, cs, sd, hw, mk;
    float ms;
    if (sscanf(line, "bfs-tune %llx loop=%d variant=%d grid=%d small=%d wave=%d chunk=%d sparse=%d hot=%d "
                     "mark=%d ms=%f",
               &k, &loop, &var, &grid, &sb, &wb, &cs, &sd, &hw, &mk, &ms) != 11)
      continue;
    if ((uint64_t)k != key) continue;
    c.loop_mode = loop;
    c.persist_variant = var;
    c.persist_grid = grid;
    c.small_bin = sb;
    c.wave_bin = wb;
    c.chunk_shift = cs;
    c.sparse_div = sd;
    c.hot_words = hw;
    c.mark = mk;
    c.tuned_ms = ms;
    found = true;  // the last matching line wins
  }
  fclose(fp);
  if (found) t = c;
  return found;
}

void append_cache(const char *path, uint64_t key, const Tuning &t) {
  FILE *fp = fopen(path, "a");
  if (!fp) return;  // an unwritable cache only costs the next plan a tuning run
  char line[512];
  const int n = snprintf(line, sizeof(line),
                         "bfs-tune %016llx loop=%d variant=%d grid=%d small=%d wave=%d chunk=%d sparse=%d "
                         "hot=%d mark=%d ms=%.9g\n",
                         (unsigned long long)key, t.loop_mode, t.persist_variant, t.persist_grid, t.small_bin,
                         t.wave_bin, t.chunk_shift, t.sparse_div, t.hot_words, t.mark, t.tuned_ms);
  if (n > 0) (void)fwrite(line, 1, (size_t)n, fp);  // one write per line
  fclose(fp);
}

}  // namespace

bfs_status autotune_graphs(Plan *p) {
  const char *cache = (p->opt.tune_cache && *p->opt.tune_cache) ? p->opt.tune_cache : nullptr;
  for (size_t gi = 0; gi < p->graphs.size(); ++gi) {
    if (!tune_wanted(p, gi) || !p->lay.tune_dist) continue;
    uint64_t key = 0;
    if (cache) {
      bfs_status s = tune_key(p, gi, key);
      if (s) return s;
      if (read_cache(cache, key, p->tune[gi])) continue;
    }
    bfs_status s = tune_graph(p, gi);
    if (s) return s;
    if (cache) append_cache(cache, key, p->tune[gi]);
  }
  return BFS_OK;
}

}  // namespace bfsk
