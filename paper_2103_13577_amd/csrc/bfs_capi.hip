// C ABI of the single-source traversal: plans, workspace layout, the level
// loop (device-resident or host-driven with an exchange callback), the
// step-wise Phase 1 / Phase 2 calls and statistics. Declarations and their
// contracts are in include/bfs.h.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdio>
#include <cstring>
#include <new>
#include <string>
#include <vector>

#include "../../include/bfs.h"
#include "bfs_core.hpp"
#include "plan.hpp"

using namespace bfsk;

namespace {

thread_local std::string g_create_error;

size_t align_up(size_t x, size_t a) { return (x + a - 1) / a * a; }

}  // namespace

namespace bfsk {
void set_create_error(const std::string &msg) { g_create_error = msg; }
}  // namespace bfsk

bfs_status bfs_plan_s::fail(bfs_status st, const std::string &msg) {
  err = msg;
  return st;
}

bfs_status bfs_plan_s::hip_fail(hipError_t e, const char *what) {
  err = std::string(what) + ": " + hipGetErrorString(e);
  return BFS_ERR_HIP;
}

namespace bfsk {

// Workspace regions for single-source runs, sized by the largest graph.
void layout_single(const bfs_graph *g, int32_t ng, WsLayout &L, size_t &off) {
  int64_t nmax = 0, omax = 1;
  for (int i = 0; i < ng; ++i) {
    nmax = std::max(nmax, g[i].n_global);
    omax = std::max(omax, g[i].v_end - g[i].v_begin);
  }
  const int64_t words = (nmax + 63) / 64;
  L.ctl = off; off = align_up(off + sizeof(Ctl), 256);
  L.lvl_frontier = off; off = align_up(off + sizeof(int64_t) * kMaxStatLevels, 256);
  L.lvl_hist = off; off = align_up(off + sizeof(uint32_t) * kMaxStatLevels * kNumBins, 256);
  L.list_blk = off; off = align_up(off + sizeof(uint64_t) * (kListMaxBlocks + 1), 256);
  L.visited = off; off = align_up(off + sizeof(uint64_t) * (size_t)std::max<int64_t>(words, 1), 256);
  L.next = off; off = align_up(off + sizeof(uint64_t) * (size_t)std::max<int64_t>(words, 1), 256);
  L.front = off; off = align_up(off + sizeof(uint64_t) * (size_t)std::max<int64_t>(words, 1), 256);
  // byte marks of dense single-node levels, 64 per bitmap word (whole graphs only)
  int64_t whole_words = 0;
  for (int i = 0; i < ng; ++i)
    if (g[i].v_begin == 0 && g[i].v_end == g[i].n_global)
      whole_words = std::max(whole_words, (g[i].n_global + 63) / 64);
  L.mark = 0;
  if (whole_words > 0) {
    L.mark = off; off = align_up(off + 64 * (size_t)whole_words, 256);
    L.hubnext = off; off = align_up(off + sizeof(uint64_t) * kMaxHotWords, 256);
  }
  for (int t = 0; t < 3; ++t)
    for (int p = 0; p < kRing; ++p) { L.q[t][p] = off; off = align_up(off + sizeof(int32_t) * (size_t)omax, 256); }
  for (int t = 0; t < 2; ++t)
    for (int p = 0; p < kRing; ++p) { L.qr[t][p] = off; off = align_up(off + sizeof(uint64_t) * (size_t)omax, 256); }
  for (int p = 0; p < kRing; ++p) { L.cstart[p] = off; off = align_up(off + sizeof(uint32_t) * (size_t)omax, 256); }
}

}  // namespace bfsk

View bfs_plan_s::view(int32_t gi, int32_t *dist) const {
  View v{};
  const bfs_graph &g = graphs[gi];
  char *b = (char *)ws;
  v.n = g.n_global;
  v.vb = g.v_begin;
  v.ve = g.v_end;
  v.m = g.m;
  v.words = (g.n_global + 63) / 64;
  if (cur_relabel && lay.rl_rp.size() > (size_t)gi && lay.rl_rp[gi]) {
    v.rp = (const int64_t *)(b + lay.rl_rp[gi]);
    v.col = (const int32_t *)(b + lay.rl_col[gi]);
    v.old_id = (const int32_t *)(b + lay.rl_old[gi]);
    v.new_id = (const int32_t *)(b + lay.rl_new[gi]);
    v.live_end = rl_live.size() > (size_t)gi ? rl_live[gi] : g.v_end;
  } else {
    v.rp = g.row_ptr;
    v.col = g.col;
    v.old_id = nullptr;
    v.new_id = nullptr;
    v.live_end = g.v_end;
  }
  v.dist = dist;
  v.visited = (uint64_t *)(b + lay.visited);
  v.next = (uint64_t *)(b + lay.next);
  v.front = cur_front ? (uint64_t *)(b + lay.front) : nullptr;
  for (int p = 0; p < kRing; ++p) {
    v.q0[p] = (int32_t *)(b + lay.q[0][p]);
    v.q1[p] = (int32_t *)(b + lay.q[1][p]);
    v.q2[p] = (int32_t *)(b + lay.q[2][p]);
    v.qr0[p] = (uint64_t *)(b + lay.qr[0][p]);
    v.qr1[p] = (uint64_t *)(b + lay.qr[1][p]);
    v.cstart[p] = (uint32_t *)(b + lay.cstart[p]);
  }
  v.ctl = (Ctl *)(b + lay.ctl);
  v.lvl_frontier = (int64_t *)(b + lay.lvl_frontier);
  v.lvl_hist = (uint32_t *)(b + lay.lvl_hist);
  v.small_bin = tune[gi].small_bin;
  v.wave_bin = tune[gi].wave_bin;
  v.chunk_shift = tune[gi].chunk_shift;
  v.stats = opt.collect_stats ? 1 : 0;
  v.sparse_div = tune[gi].sparse_div;
  v.into_vis = cur_into_vis ? 1 : 0;
  v.mark = cur_mark ? (uint8_t *)(b + lay.mark) : nullptr;
  v.hubnext = cur_mark ? (uint64_t *)(b + lay.hubnext) : nullptr;
  v.hub_words = v.hubnext ? kMaxHotWords : 0;
  return v;
}

int bfs_plan_s::wide_grid() const { return num_cus * std::max(bpc_expand, 1); }

int bfs_plan_s::expand_grid(int hot_words) {
  if (hot_words <= 0) return wide_grid();
  auto it = hot_bpc.find(hot_words);
  if (it == hot_bpc.end()) it = hot_bpc.emplace(hot_words, expand_blocks_per_cu((uint32_t)hot_words)).first;
  return num_cus * std::max(it->second, 1);
}

int bfs_plan_s::merge_grid(int64_t words) const {
  int64_t g = (words + kBlock - 1) / kBlock;
  return (int)std::max<int64_t>(1, std::min<int64_t>(g, (int64_t)num_cus * 8));
}

bfs_status bfs_plan_s::read_ctl(Ctl &c) {
  // The host loop reads the control block after every level: the copy goes
  // to pinned memory, which spares the staging copy of a pageable target.
  hipError_t e = hipMemcpyAsync(hctl, (char *)ws + lay.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync(ctl)");
  e = hipStreamSynchronize(stream);
  if (e != hipSuccess) return hip_fail(e, "hipStreamSynchronize");
  c = *hctl;
  return BFS_OK;
}

// ---------------------------------------------------------------------------
// C ABI
// ---------------------------------------------------------------------------

extern "C" {

void bfs_options_default(bfs_options *o) {
  if (o) memset(o, 0, sizeof(*o));
}

bfs_status bfs_workspace_size(const bfs_graph *graphs, int32_t ngraphs, const bfs_options *o,
                              size_t *bytes) {
  if (!graphs || ngraphs <= 0 || !bytes) return BFS_ERR_ARG;
  bfs_options d;
  bfs_options_default(&d);
  if (!o) o = &d;
  WsLayout L{};
  size_t off = 0;
  layout_single(graphs, ngraphs, L, off);
  layout_relabel(graphs, ngraphs, o, L, off);
  layout_batch(graphs, ngraphs, o, L, off);
  *bytes = off;
  return BFS_OK;
}

bfs_status bfs_plan_create(const bfs_graph *graphs, int32_t ngraphs, const bfs_options *o,
                           void *workspace, size_t ws_bytes, bfs_plan_t *out) {
  g_create_error.clear();
  if (!out) { g_create_error = "out is NULL"; return BFS_ERR_ARG; }
  *out = nullptr;
  if (!graphs || ngraphs <= 0) { g_create_error = "no graphs"; return BFS_ERR_ARG; }
  if (!workspace || ((uintptr_t)workspace & 255)) {
    g_create_error = "workspace must be a non-null 256-byte aligned device pointer";
    return BFS_ERR_ARG;
  }
  bfs_options d;
  bfs_options_default(&d);
  if (!o) o = &d;
  for (int i = 0; i < ngraphs; ++i) {
    const bfs_graph &g = graphs[i];
    if (g.n_global <= 0 || g.n_global >= (1ll << 31) || g.v_begin < 0 || g.v_end < g.v_begin ||
        g.v_end > g.n_global || g.m < 0 || g.m >= (1ll << 40) || !g.row_ptr || (g.m > 0 && !g.col)) {
      g_create_error = "graph " + std::to_string(i) + ": bad sizes or null pointers";
      return BFS_ERR_ARG;
    }
  }
  size_t need = 0;
  bfs_status st = bfs_workspace_size(graphs, ngraphs, o, &need);
  if (st) { g_create_error = "bad arguments"; return st; }
  if (ws_bytes < need) {
    g_create_error = "workspace too small: need " + std::to_string(need) + " bytes";
    return BFS_ERR_WORKSPACE;
  }
  Plan *p = new (std::nothrow) Plan();
  if (!p) { g_create_error = "out of host memory"; return BFS_ERR_ARG; }
  p->graphs.assign(graphs, graphs + ngraphs);
  p->opt = *o;
  p->ws = workspace;
  p->ws_bytes = ws_bytes;
  p->stream = (hipStream_t)o->hip_stream;
  size_t off = 0;
  layout_single(graphs, ngraphs, p->lay, off);
  layout_relabel(graphs, ngraphs, o, p->lay, off);
  layout_batch(graphs, ngraphs, o, p->lay, off);
  int dev = 0;
  hipDeviceProp_t prop;
  if (hipGetDevice(&dev) != hipSuccess || hipGetDeviceProperties(&prop, dev) != hipSuccess) {
    g_create_error = "no HIP device";
    delete p;
    return BFS_ERR_HIP;
  }
  p->num_cus = prop.multiProcessorCount;
  p->coop = prop.cooperativeLaunch;
  p->bpc[0] = persistent_blocks_per_cu(0);
  p->bpc[1] = persistent_blocks_per_cu(1);
  p->bpc_expand = expand_blocks_per_cu(0u);
  p->max_lds = (int)prop.sharedMemPerBlock;
  p->bpc_bu = bottom_up_blocks_per_cu(kBottomUpHot);
  p->persist_grid = o->grid_blocks;  // 0: chosen per graph
  if (o->direction != BFS_DIR_TOPDOWN && o->direction != BFS_DIR_OPTIMIZING) {
    g_create_error = "unknown direction";
    delete p;
    return BFS_ERR_ARG;
  }
  if (o->loop_mode < BFS_LOOP_AUTO || o->loop_mode > BFS_LOOP_ENQUEUE) {
    g_create_error = "unknown loop_mode";
    delete p;
    return BFS_ERR_ARG;
  }
  if (o->grid_blocks > kBarrierMaxBlocks) {
    g_create_error = "grid_blocks above the grid barrier's limit of 2048";
    delete p;
    return BFS_ERR_ARG;
  }
  for (auto &ev : p->ev) {
    if (hipEventCreate(&ev) != hipSuccess) {
      g_create_error = "hipEventCreate failed";
      delete p;
      return BFS_ERR_HIP;
    }
  }
  for (auto &row : p->lev)
    for (auto &ev : row)
      if (hipEventCreate(&ev) != hipSuccess) {
        g_create_error = "hipEventCreate failed";
        delete p;
        return BFS_ERR_HIP;
      }
  if (hipStreamCreateWithFlags(&p->cap_stream, hipStreamNonBlocking) != hipSuccess) {
    g_create_error = "hipStreamCreate failed";
    delete p;
    return BFS_ERR_HIP;
  }
  if (hipHostMalloc((void **)&p->hctl, sizeof(Ctl), hipHostMallocDefault) != hipSuccess) {
    p->hctl = nullptr;
    g_create_error = "hipHostMalloc of the control block's host copy failed";
    delete p;
    return BFS_ERR_HIP;
  }
  p->gexec.assign(ngraphs, nullptr);
  p->gexec_tune.assign(ngraphs, Tuning{});
  st = validate_graphs(p);
  if (st) { g_create_error = p->err; delete p; return st; }
  st = choose_tuning(p);
  if (st) { g_create_error = p->err; delete p; return st; }
  st = relabel_graphs(p);
  if (st) { g_create_error = p->err; delete p; return st; }
  st = autotune_graphs(p);
  if (st) { g_create_error = p->err; delete p; return st; }
  st = prepare_run_loops(p);
  if (st) { g_create_error = p->err; delete p; return st; }
  st = batch_init(p);
  if (st) { g_create_error = p->err; delete p; return st; }
  *out = p;
  return BFS_OK;
}

void bfs_plan_destroy(bfs_plan_t p) {
  if (!p) return;
  batch_shutdown(p);
  // work queued on the plan's streams ends before its graphs and events go
  (void)hipStreamSynchronize(p->stream);
  if (p->cap_stream) (void)hipStreamSynchronize(p->cap_stream);
  delete p;
}

const char *bfs_last_error(bfs_plan_t p) {
  if (!p) return g_create_error.c_str();
  return p->err.c_str();
}

namespace {

// Reset for a traversal. bfs_run may use the relabelled copy of a whole graph
// (its bitmaps never leave the library); the step-wise calls work in caller
// ids because their bitmaps are exchanged with other nodes.
bfs_status begin_impl(bfs_plan_t p, int32_t graph, int64_t source, int32_t *dist, bool relabel) {
  if (graph < 0 || graph >= (int32_t)p->graphs.size())
    return p->fail(BFS_ERR_ARG, "graph index out of range");
  const bfs_graph &g = p->graphs[graph];
  if (source < 0 || source >= g.n_global)
    return p->fail(BFS_ERR_ARG, "source " + std::to_string(source) + " outside [0, n_global)");
  if (!dist) return p->fail(BFS_ERR_ARG, "dist is NULL");
  std::lock_guard<std::mutex> lk(p->run_mu);
  p->cur_graph = graph;
  p->cur_source = source;
  p->cur_dist = dist;
  p->cur_relabel = relabel;
  p->cur_do = relabel && p->direction_optimizing(graph);
  // step-wise traversals of a plan created with BFS_DIR_OPTIMIZING keep the
  // frontier bitmap for bfs_expand_bottom_up (any share)
  p->cur_front = p->cur_do || (!relabel && p->opt.direction == BFS_DIR_OPTIMIZING);
  p->bu_state = false;
  p->cur_into_vis = false;
  p->cur_mark = false;
  p->front_level = -1;
  p->merge_mode = kMergeFull;
  p->queues_stale = false;
  p->edges_after.clear();
  p->bu_levels_run = 0;
  p->level = 0;
  p->expanded_level = -1;
  p->big_level = false;
  p->level_frontier.assign(1, (source >= g.v_begin && source < g.v_end) ? 1 : 0);
  View v = p->view(graph, dist);
  int grid = (int)std::min<int64_t>((g.n_global + kBlock - 1) / kBlock, (int64_t)p->num_cus * 16);
  hipError_t e = launch_reset(v, source, std::max(grid, 1), p->stream);
  if (e != hipSuccess) { p->began = false; return p->hip_fail(e, "reset launch"); }
  p->began = true;
  p->finished = false;
  return BFS_OK;
}

}  // namespace

bfs_status bfs_begin(bfs_plan_t p, int32_t graph, int64_t source, int32_t *dist) {
  if (!p) return BFS_ERR_ARG;
  return begin_impl(p, graph, source, dist, false);
}

namespace {

// Fills the current level's tier queues from the frontier bitmap after a
// merge that left them unwritten.
bfs_status fill_stale_queues(bfs_plan_t p, const View &v) {
  if (!p->queues_stale) return BFS_OK;
  MergeArgs a{};
  a.level = p->level - 1;
  a.mode = kMergeQueuesFromFront;
  hipError_t e = launch_merge(v, a, p->merge_grid(v.words), p->stream);
  if (e != hipSuccess) return p->hip_fail(e, "queue fill launch");
  p->queues_stale = false;
  return BFS_OK;
}

}  // namespace

bfs_status bfs_expand(bfs_plan_t p, const uint64_t **local_next) {
  if (!p) return BFS_ERR_ARG;
  if (!p->began || p->finished) return p->fail(BFS_ERR_STATE, "bfs_expand before bfs_begin");
  View v = p->view(p->cur_graph, p->cur_dist);
  if (p->opt.collect_stats && p->level + 1 < kMaxStatLevels) {
    hipError_t e = launch_clear_stats_row(v, p->level + 1, p->stream);
    if (e != hipSuccess) return p->hip_fail(e, "stats launch");
  }
  if (p->expanded_level == p->level) return p->fail(BFS_ERR_STATE, "level already expanded");
  bfs_status fs = fill_stale_queues(p, v);
  if (fs) return fs;
  const bool timed = p->time_levels && p->level < Plan::kTimedLevels;
  if (timed) {
    p->level_kind[p->level] = 0;
    (void)hipEventRecord(p->lev[p->level][0], p->stream);
  }
  // The LDS copy of the hub bits pays off only on large dense levels.
  const int hot = (p->cur_relabel && p->big_level) ? p->tune[p->cur_graph].hot_words : 0;
  hipError_t e = launch_expand(v, p->level, p->expand_grid(hot), hot, p->stream);
  if (e != hipSuccess) return p->hip_fail(e, "expand launch");
  if (timed) (void)hipEventRecord(p->lev[p->level][1], p->stream);
  p->expanded_level = p->level;
  if (local_next) *local_next = v.next;
  return BFS_OK;
}

bfs_status bfs_expand_bottom_up(bfs_plan_t p, const uint64_t **local_next) {
  if (!p) return BFS_ERR_ARG;
  if (!p->began || p->finished) return p->fail(BFS_ERR_STATE, "bfs_expand_bottom_up before bfs_begin");
  if (p->expanded_level == p->level) return p->fail(BFS_ERR_STATE, "level already expanded");
  if (p->cur_relabel || !p->cur_front)
    return p->fail(BFS_ERR_STATE, "bottom-up steps need a traversal started by bfs_begin on a plan "
                                  "created with direction = BFS_DIR_OPTIMIZING");
  if (p->level > 0 && p->front_level != p->level)
    return p->fail(BFS_ERR_STATE, "the previous level was not finished by a merge");
  View v = p->view(p->cur_graph, p->cur_dist);
  if (p->opt.collect_stats && p->level + 1 < kMaxStatLevels) {
    hipError_t e = launch_clear_stats_row(v, p->level + 1, p->stream);
    if (e != hipSuccess) return p->hip_fail(e, "stats launch");
  }
  const bool timed = p->time_levels && p->level < Plan::kTimedLevels;
  if (timed) {
    p->level_kind[p->level] = 2;
    (void)hipEventRecord(p->lev[p->level][0], p->stream);
  }
  // level 0: the frontier is the root alone, which is what `visited` holds
  const uint64_t *front = p->level == 0 ? v.visited : v.front;
  hipError_t e = launch_bottom_up(v, p->level, p->num_cus * std::max(p->bpc_bu, 1), 0u, front, 0, p->stream);
  if (e != hipSuccess) return p->hip_fail(e, "bottom-up launch");
  if (timed) (void)hipEventRecord(p->lev[p->level][1], p->stream);
  p->expanded_level = p->level;
  p->bu_levels_run += 1;
  if (local_next) *local_next = v.next;
  return BFS_OK;
}

bfs_status bfs_merge_frontier(bfs_plan_t p, const uint64_t *const *incoming, int32_t k,
                              int32_t keep_next, int64_t *global_new, int64_t *owned_new) {
  if (!p) return BFS_ERR_ARG;
  if (!p->began || p->finished) return p->fail(BFS_ERR_STATE, "bfs_merge_frontier before bfs_begin");
  if (p->expanded_level != p->level) return p->fail(BFS_ERR_STATE, "bfs_merge_frontier before bfs_expand of this level");
  if (k < 0 || (k > 0 && !incoming)) return p->fail(BFS_ERR_ARG, "bad incoming list");
  for (int i = 0; i < k; ++i)
    if (!incoming[i]) return p->fail(BFS_ERR_ARG, "incoming bitmap " + std::to_string(i) + " is NULL");
  View v = p->view(p->cur_graph, p->cur_dist);
  int done = 0;
  do {
    MergeArgs a{};
    const int chunk = std::min(k - done, kMaxIncoming);
    for (int i = 0; i < chunk; ++i) a.inc[i] = incoming[done + i];
    a.k = chunk;
    done += chunk;
    a.keep_next = (done < k || keep_next) ? 1 : 0;
    a.level = p->level;
    a.mode = p->merge_mode;
    hipError_t e = launch_merge(v, a, p->merge_grid(v.words), p->stream);
    if (e != hipSuccess) return p->hip_fail(e, "merge launch");
  } while (done < k);
  if (!keep_next && p->time_levels && p->level < Plan::kTimedLevels)
    (void)hipEventRecord(p->lev[p->level][2], p->stream);
  if (global_new || owned_new || !keep_next) {
    Ctl c;
    bfs_status st = p->read_ctl(c);
    if (st) return st;
    if (c.err & kErrListId)
      return p->fail(BFS_ERR_ARG, "an incoming list held a vertex id outside [0, n_global); the "
                                  "traversal must be restarted with bfs_begin");
    if (global_new) *global_new = (int64_t)c.newcnt[p->level % 3];
    if (owned_new) *owned_new = (int64_t)c.ownedcnt[p->level % 3];
    if (!keep_next) {
      // the next level is "big" (worth an LDS copy of the hub bits) when its
      // frontier's edges are at least the vertex count
      p->big_level = (int64_t)c.edges - (p->edges_after.empty() ? 0 : p->edges_after.back()) >= v.n;
      if ((int)p->level_frontier.size() == p->level + 1)
        p->level_frontier.push_back((int64_t)c.ownedcnt[p->level % 3]);
      p->last_level_new = (int64_t)c.newcnt[p->level % 3];
      p->edges_after.push_back((int64_t)c.edges);
      if (v.front) p->front_level = p->level + 1;  // the merge wrote the next frontier bitmap
      p->level += 1;
    }
  }
  return BFS_OK;
}

bfs_status bfs_frontier_list(bfs_plan_t p, int32_t *list, int64_t capacity, int64_t *count) {
  if (!p) return BFS_ERR_ARG;
  if (!p->began || p->finished) return p->fail(BFS_ERR_STATE, "bfs_frontier_list before bfs_begin");
  if (p->expanded_level != p->level)
    return p->fail(BFS_ERR_STATE, "bfs_frontier_list before bfs_expand of this level");
  if (!count) return p->fail(BFS_ERR_ARG, "count is NULL");
  if (capacity < 0 || (capacity > 0 && !list)) return p->fail(BFS_ERR_ARG, "bad list or capacity");
  if (p->cur_relabel) return p->fail(BFS_ERR_STATE, "the traversal runs on the relabelled copy");
  View v = p->view(p->cur_graph, p->cur_dist);
  uint64_t *blk = (uint64_t *)((char *)p->ws + p->lay.list_blk);
  hipError_t e = launch_list_export(v.next, v.words, v.n, blk, list, capacity, p->stream);
  if (e != hipSuccess) return p->hip_fail(e, "list export launch");
  int nblk = 0;
  int64_t per = 0;
  list_geometry(v.words, nblk, per);
  uint64_t total = 0;
  e = hipMemcpyAsync(&total, blk + nblk, sizeof(total), hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return p->hip_fail(e, "list export count");
  *count = (int64_t)total;
  if (capacity > 0 && (int64_t)total > capacity)
    return p->fail(BFS_ERR_CAPACITY, "the global queue holds " + std::to_string(total) +
                                         " vertices, more than the list capacity " + std::to_string(capacity));
  return BFS_OK;
}

bfs_status bfs_merge_lists(bfs_plan_t p, const int32_t *const *lists, const int64_t *counts, int32_t k,
                           const uint64_t *const *bitmaps, int32_t kb, int32_t keep_next,
                           int64_t *global_new, int64_t *owned_new) {
  if (!p) return BFS_ERR_ARG;
  if (!p->began || p->finished) return p->fail(BFS_ERR_STATE, "bfs_merge_lists before bfs_begin");
  if (p->expanded_level != p->level)
    return p->fail(BFS_ERR_STATE, "bfs_merge_lists before bfs_expand of this level");
  if (k < 0 || (k > 0 && (!lists || !counts))) return p->fail(BFS_ERR_ARG, "bad incoming lists");
  if (kb < 0 || (kb > 0 && !bitmaps)) return p->fail(BFS_ERR_ARG, "bad incoming bitmaps");
  for (int i = 0; i < k; ++i) {
    if (counts[i] < 0) return p->fail(BFS_ERR_ARG, "incoming list " + std::to_string(i) + " has a negative count");
    if (counts[i] > 0 && !lists[i]) return p->fail(BFS_ERR_ARG, "incoming list " + std::to_string(i) + " is NULL");
  }
  for (int i = 0; i < kb; ++i)
    if (!bitmaps[i]) return p->fail(BFS_ERR_ARG, "incoming bitmap " + std::to_string(i) + " is NULL");
  if (p->cur_relabel) return p->fail(BFS_ERR_STATE, "the traversal runs on the relabelled copy");
  View v = p->view(p->cur_graph, p->cur_dist);
  for (int i = 0; i < k; ++i) {
    hipError_t e = launch_list_scatter(lists[i], counts[i], v.next, v.n, &v.ctl->err, p->num_cus * 8, p->stream);
    if (e != hipSuccess) return p->hip_fail(e, "list scatter launch");
  }
  // one merge pass over the listed vertices (now in the global queue) and the bitmaps
  return bfs_merge_frontier(p, bitmaps, kb, keep_next, global_new, owned_new);
}

namespace {

// One queue-only level of bfs_run's host-driven loop (single node, small
// frontier): the expansion ORs straight into `visited`, writes distances and
// fills the next level's queues, so the level needs no merge launch.
bfs_status queue_only_level(bfs_plan_t p, int64_t *global_new) {
  View v = p->view(p->cur_graph, p->cur_dist);
  if (p->opt.collect_stats && p->level + 1 < kMaxStatLevels) {
    hipError_t e = launch_clear_stats_row(v, p->level + 1, p->stream);
    if (e != hipSuccess) return p->hip_fail(e, "stats launch");
  }
  bfs_status fs = fill_stale_queues(p, v);
  if (fs) return fs;
  const bool timed = p->time_levels && p->level < Plan::kTimedLevels;
  if (timed) {
    p->level_kind[p->level] = 1;
    (void)hipEventRecord(p->lev[p->level][0], p->stream);
  }
  hipError_t e = launch_expand(v, p->level, p->wide_grid(), kQueueOnly, p->stream);
  if (e != hipSuccess) return p->hip_fail(e, "expand launch");
  if (timed) {
    (void)hipEventRecord(p->lev[p->level][1], p->stream);
    (void)hipEventRecord(p->lev[p->level][2], p->stream);
  }
  p->expanded_level = p->level;
  Ctl c;
  bfs_status st = p->read_ctl(c);
  if (st) return st;
  *global_new = (int64_t)c.newcnt[p->level % 3];
  p->big_level = (int64_t)c.edges - (p->edges_after.empty() ? 0 : p->edges_after.back()) >= v.n;
  p->edges_after.push_back((int64_t)c.edges);
  if ((int)p->level_frontier.size() == p->level + 1)
    p->level_frontier.push_back((int64_t)c.ownedcnt[p->level % 3]);
  p->last_level_new = *global_new;
  p->level += 1;
  return BFS_OK;
}

// One bottom-up level of a direction-optimizing traversal: the frontier
// bitmap (written by the previous merge, else rebuilt from the queues), the
// bottom-up step into `next`, then the ordinary merge.
bfs_status bottom_up_level(bfs_plan_t p, int64_t *global_new) {
  View v = p->view(p->cur_graph, p->cur_dist);
  if (p->opt.collect_stats && p->level + 1 < kMaxStatLevels) {
    hipError_t e = launch_clear_stats_row(v, p->level + 1, p->stream);
    if (e != hipSuccess) return p->hip_fail(e, "stats launch");
  }
  const bool timed = p->time_levels && p->level < Plan::kTimedLevels;
  if (timed) {
    p->level_kind[p->level] = 2;
    (void)hipEventRecord(p->lev[p->level][0], p->stream);
  }
  hipError_t e = hipSuccess;
  if (p->front_level != p->level) e = launch_front_from_queues(v, p->level, p->wide_grid(), p->stream);
  const uint32_t hot = (uint32_t)std::min<int64_t>(kBottomUpHot, v.words);
  // The next level reads the frontier bitmap if it is bottom-up too, so the
  // merge leaves the tier queues unwritten and the step counts the new
  // vertices' edges; a top-down level fills the queues first (with stats on,
  // the merge's degree histogram needs the full merge).
  const bool no_queues = !p->opt.collect_stats;
  if (e == hipSuccess)
    e = launch_bottom_up(v, p->level, p->num_cus * std::max(p->bpc_bu, 1), hot, v.front, no_queues ? 1 : 0,
                         p->stream);
  if (e != hipSuccess) return p->hip_fail(e, "bottom-up launch");
  if (timed) (void)hipEventRecord(p->lev[p->level][1], p->stream);
  p->expanded_level = p->level;
  p->bu_levels_run += 1;
  p->merge_mode = no_queues ? kMergeNoQueues : kMergeFull;
  bfs_status st = bfs_merge_frontier(p, nullptr, 0, 0, global_new, nullptr);
  p->merge_mode = kMergeFull;
  if (st == BFS_OK && no_queues) p->queues_stale = true;
  return st;
}

}  // namespace

bfs_status bfs_finish(bfs_plan_t p, int32_t *parent, bfs_stats *st) {
  if (!p) return BFS_ERR_ARG;
  if (!p->began) return p->fail(BFS_ERR_STATE, "bfs_finish before bfs_begin");
  View v = p->view(p->cur_graph, p->cur_dist);
  if (parent) {
    hipError_t e = launch_parent(v, parent, p->cur_source, p->wide_grid(), p->stream);
    if (e != hipSuccess) return p->hip_fail(e, "parent launch");
  }
  Ctl c;
  bfs_status s = p->read_ctl(c);
  if (s) return s;
  p->finished = true;
  if (st) {
    st->levels = p->persistent_levels > 0 ? p->persistent_levels : p->level;
    st->reached = (int64_t)c.reached;
    st->edges_scanned = (int64_t)c.edges;
    st->ms = p->last_ms;
    st->loop_ms = p->last_loop_ms;
    st->expand_ms = p->last_expand_ms;
    st->merge_ms = p->last_merge_ms;
    st->expand_launches = p->last_expand_launches;
    st->dense_edges = (int64_t)c.xedges;
    st->dense_frontier = (int64_t)c.xfront;
    st->queue_ms = p->last_queue_ms;
    st->bottom_up_levels = p->bu_levels_run;
    st->bottom_up_ms = p->last_bu_ms;
    st->bottom_up_edges = (int64_t)c.buedges;
    st->bottom_up_vertices = (int64_t)c.buverts;
  }
  return BFS_OK;
}

namespace {

bool same_tuning(const Tuning &a, const Tuning &b) {
  return a.small_bin == b.small_bin && a.wave_bin == b.wave_bin && a.chunk_shift == b.chunk_shift &&
         a.sparse_div == b.sparse_div && a.hot_words == b.hot_words && a.mark == b.mark;
}

// The captured graph of kGraphLevels level steps for graph gi (captured on
// first use, and again when the tier settings changed).
bfs_status graph_exec(bfs_plan_t p, int32_t gi, hipGraphExec_t &out) {
  if (p->gexec[gi] && same_tuning(p->gexec_tune[gi], p->tune[gi])) {
    out = p->gexec[gi];
    return BFS_OK;
  }
  if (p->gexec[gi]) {
    (void)hipGraphExecDestroy(p->gexec[gi]);
    p->gexec[gi] = nullptr;
  }
  View v = p->view(gi, nullptr);  // the kernels take the distance array from the control block
  const int max_levels = (int)std::min<int64_t>(p->graphs[gi].n_global + 1, 1ll << 30);
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamBeginCapture(p->cap_stream, hipStreamCaptureModeThreadLocal);
  if (e != hipSuccess) return p->hip_fail(e, "hipStreamBeginCapture");
  const int hot = p->cur_relabel ? p->tune[gi].hot_words : 0;
  hipError_t el = enqueue_graph_levels(v, Plan::kGraphLevels, max_levels, p->expand_grid(hot),
                                       p->merge_grid(v.words), hot, p->cap_stream);
  e = hipStreamEndCapture(p->cap_stream, &g);
  if (el != hipSuccess) e = el;
  if (e != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return p->hip_fail(e, "level graph capture");
  }
  e = hipGraphInstantiate(&p->gexec[gi], g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) {
    p->gexec[gi] = nullptr;
    return p->hip_fail(e, "hipGraphInstantiate");
  }
  p->gexec_tune[gi] = p->tune[gi];
  out = p->gexec[gi];
  return BFS_OK;
}

}  // namespace

namespace {

// A traversal whose levels are all dense and merged without incoming bitmaps
// (single node, no queue-only or bottom-up levels) lets its expansions OR
// straight into `visited` (one bitmap for their random probes instead of two);
// `next` then holds visited as of each level's start, from which the merge
// finds the new vertices. Called after the reset, before the level loop.
// With byte marks (a whole graph whose tuning selects them) the expansions
// leave both bitmaps alone and set one byte per discovered vertex instead;
// the marks must all be zero when the traversal starts. Queue-only levels mix
// with either byte marks (they OR into `visited` themselves and set no mark;
// every dense level's merge clears the marks it read) but not with the OR
// into `visited`, whose snapshot in `next` only dense merges keep.
// The expansion form bfs_run uses for a graph (its flags only; no device
// work): byte marks, an OR into `visited`, or neither (bottom-up levels, an
// exchange, or queue-only levels without byte marks keep the two-bitmap form).
void dense_form(bfs_plan_t p, int32_t graph) {
  p->cur_mark = p->cur_into_vis = false;
  if (p->opt.exchange || p->cur_do) return;
  const bfs_graph &g = p->graphs[graph];
  if (p->tune[graph].mark && p->lay.mark && g.v_begin == 0 && g.v_end == g.n_global)
    p->cur_mark = true;
  else if (p->tune[graph].sparse_div == 0)
    p->cur_into_vis = true;
}

bfs_status into_visited(bfs_plan_t p, int32_t graph, int32_t *dist) {
  dense_form(p, graph);
  if (!p->cur_mark && !p->cur_into_vis) return BFS_OK;
  if (p->cur_mark) {
    if (!p->marks_clean) {
      // the marks and the hub words that follow them
      const size_t bytes = p->lay.hubnext + sizeof(uint64_t) * kMaxHotWords - p->lay.mark;
      hipError_t e = hipMemsetAsync((char *)p->ws + p->lay.mark, 0, bytes, p->stream);
      if (e != hipSuccess) return p->hip_fail(e, "clear marks");
    }
    // set again once the traversal has finished (its merges clear every mark)
    p->marks_clean = false;
    return BFS_OK;
  }
  const View v = p->view(graph, dist);
  hipError_t e = hipMemcpyAsync(v.next, v.visited, sizeof(uint64_t) * (size_t)v.words,
                                hipMemcpyDeviceToDevice, p->stream);
  return e == hipSuccess ? BFS_OK : p->hip_fail(e, "visited snapshot");
}

}  // namespace


bfs_status bfs_run(bfs_plan_t p, int32_t graph, int64_t source, int32_t *dist, int32_t *parent,
                   bfs_stats *st) {
  if (!p) return BFS_ERR_ARG;
  bfs_status s;
  hipError_t e;
  hipEvent_t ev0 = p->ev[0], ev1 = p->ev[1];
  p->persistent_levels = 0;
  p->last_ms = 0.f;
  p->last_loop_ms = 0.f;
  p->last_expand_ms = p->last_merge_ms = p->last_queue_ms = p->last_bu_ms = 0.f;
  p->last_expand_launches = 0;
  e = hipEventRecord(ev0, p->stream);
  if (e != hipSuccess) return p->hip_fail(e, "hipEventRecord");
  s = begin_impl(p, graph, source, dist, p->opt.exchange == nullptr);
  if (s) return s;
  const bfs_graph &g = p->graphs[graph];
  const Tuning &tu = p->tune[graph];
  int mode = p->opt.loop_mode == BFS_LOOP_AUTO ? tu.loop_mode : p->opt.loop_mode;
  if (p->opt.exchange || p->cur_do) mode = BFS_LOOP_HOST;  // the direction test runs on the host
  int grid = 0;
  if (mode == BFS_LOOP_PERSISTENT) {
    grid = p->persist_grid > 0 ? p->persist_grid : tu.persist_grid;
    const int cap = p->bpc[tu.persist_variant] * p->num_cus;
    if (!p->coop || grid <= 0 || grid > cap) {
      if (p->opt.loop_mode == BFS_LOOP_PERSISTENT)
        return p->fail(BFS_ERR_ARG, "persistent loop needs a cooperative launch of at most " +
                                        std::to_string(cap) + " blocks");
      mode = BFS_LOOP_HOST;
    }
  }
  if (mode == BFS_LOOP_CU && !cu_fits(g.n_global, g.m, g.v_begin == 0 && g.v_end == g.n_global,
                                      p->max_lds)) {
    if (p->opt.loop_mode == BFS_LOOP_CU)
      return p->fail(BFS_ERR_ARG, "one-workgroup loop needs a whole graph with m < 2^25 whose "
                                  "two bitmaps fit in one workgroup's LDS");
    mode = BFS_LOOP_HOST;
  }
  const bool host_loop = mode == BFS_LOOP_HOST;
  if (mode == BFS_LOOP_CU) {
    View v = p->view(graph, dist);
    const int max_levels = (int)std::min<int64_t>(g.n_global + 1, 1ll << 30);
    e = hipEventRecord(p->ev[2], p->stream);
    if (e != hipSuccess) return p->hip_fail(e, "hipEventRecord");
    e = launch_bfs_cu(v, source, max_levels, p->stream);
    if (e != hipSuccess) return p->hip_fail(e, "one-workgroup launch");
    e = hipEventRecord(ev1, p->stream);
    if (e != hipSuccess) return p->hip_fail(e, "hipEventRecord");
    Ctl c;
    s = p->read_ctl(c);
    if (s) return s;
    if (c.err) return p->fail(BFS_ERR_DEVICE, "level limit exceeded");
    p->persistent_levels = c.levels;
    p->level = c.levels;
  } else if (mode == BFS_LOOP_GRAPH) {
    s = into_visited(p, graph, dist);  // before the capture, which keeps the setting
    if (s) return s;
    hipGraphExec_t ge = nullptr;
    s = graph_exec(p, graph, ge);
    if (s) return s;
    e = hipEventRecord(p->ev[2], p->stream);
    if (e != hipSuccess) return p->hip_fail(e, "hipEventRecord");
    const int64_t max_launches = g.n_global / Plan::kGraphLevels + 2;
    Ctl c;
    for (int64_t i = 0;; ++i) {
      e = hipGraphLaunch(ge, p->stream);
      if (e != hipSuccess) return p->hip_fail(e, "hipGraphLaunch");
      s = p->read_ctl(c);
      if (s) return s;
      if (c.gdone) break;
      if (i + 1 >= max_launches) return p->fail(BFS_ERR_DEVICE, "level limit exceeded");
    }
    e = hipEventRecord(ev1, p->stream);
    if (e != hipSuccess) return p->hip_fail(e, "hipEventRecord");
    if (c.err) return p->fail(BFS_ERR_DEVICE, "level limit exceeded");
    p->persistent_levels = c.levels;
    p->level = c.levels;
  } else if (mode == BFS_LOOP_ENQUEUE) {
    // the captured loop's steps launched directly: the host enqueues
    // kGraphLevels steps (with the first kTimedLevels steps' events), then
    // reads the control block once
    s = into_visited(p, graph, dist);
    if (s) return s;
    View v = p->view(graph, nullptr);  // the kernels take the distance array from the control block
    const int max_levels = (int)std::min<int64_t>(g.n_global + 1, 1ll << 30);
    const int hot = p->cur_relabel ? tu.hot_words : 0;
    const int egrid = p->expand_grid(hot), mgrid = p->merge_grid(v.words);
    const int64_t max_rounds = g.n_global / Plan::kGraphLevels + 2;
    e = hipEventRecord(p->ev[2], p->stream);
    if (e != hipSuccess) return p->hip_fail(e, "hipEventRecord");
    Ctl c;
    int steps = 0;
    for (int64_t i = 0;; ++i) {
      const bool timed = steps + Plan::kGraphLevels <= Plan::kTimedLevels;
      e = enqueue_graph_levels(v, Plan::kGraphLevels, max_levels, egrid, mgrid, hot, p->stream,
                               timed ? p->lev + steps : nullptr);
      if (e != hipSuccess) return p->hip_fail(e, "level step launch");
      if (timed) steps += Plan::kGraphLevels;
      s = p->read_ctl(c);
      if (s) return s;
      if (c.gdone) break;
      if (i + 1 >= max_rounds) return p->fail(BFS_ERR_DEVICE, "level limit exceeded");
    }
    e = hipEventRecord(ev1, p->stream);
    if (e != hipSuccess) return p->hip_fail(e, "hipEventRecord");
    if (c.err) return p->fail(BFS_ERR_DEVICE, "level limit exceeded");
    p->persistent_levels = c.levels;
    p->level = c.levels;
    p->enqueued_steps = steps;
  } else if (!host_loop) {
    s = into_visited(p, graph, dist);
    if (s) return s;
    View v = p->view(graph, dist);
    const int max_levels = (int)std::min<int64_t>(g.n_global + 1, 1ll << 30);
    e = hipEventRecord(p->ev[2], p->stream);
    if (e != hipSuccess) return p->hip_fail(e, "hipEventRecord");
    e = launch_persistent(v, max_levels, grid, tu.persist_variant, p->stream);
    if (e != hipSuccess) return p->hip_fail(e, "persistent launch");
    e = hipEventRecord(ev1, p->stream);
    if (e != hipSuccess) return p->hip_fail(e, "hipEventRecord");
    Ctl c;
    s = p->read_ctl(c);
    if (s) return s;
    if (c.bar.tripped) return p->fail(BFS_ERR_DEVICE, "grid barrier spin limit exceeded");
    if (c.err) return p->fail(BFS_ERR_DEVICE, "level limit exceeded");
    p->persistent_levels = c.levels;
    p->level = c.levels;
  } else {
    const int64_t words = (g.n_global + 63) / 64;
    s = into_visited(p, graph, dist);
    if (s) return s;
    e = hipEventRecord(p->ev[2], p->stream);
    if (e != hipSuccess) return p->hip_fail(e, "hipEventRecord");
    p->time_levels = true;
    for (;;) {
      if (p->cur_do && p->level >= 2) {
        // edge-count test: frontier edges against the unvisited vertices' edges
        const int L = p->level;
        const int64_t mf = p->edges_after[L - 1] - p->edges_after[L - 2];
        const int64_t mu = g.m - p->edges_after[L - 1];
        const int64_t nf = p->level_frontier[L], nf_prev = p->level_frontier[L - 1];
        if (!p->bu_state) {
          // a frontier with few edges stays top-down even when fewer remain
          // (the end of a long tail): a bottom-up step costs at least a sweep
          // over the unvisited vertices, a top-down one only the frontier's edges
          if (mf * kDirAlpha > mu && mf * kDirBeta >= g.n_global) p->bu_state = true;
        } else if (nf * kDirBeta < g.n_global && nf <= nf_prev) {
          p->bu_state = false;
        }
        if (p->bu_state) {
          int64_t gnew = 0;
          s = bottom_up_level(p, &gnew);
          if (s) { p->time_levels = false; return s; }
          if (gnew == 0) break;
          continue;
        }
      }
      // small frontiers of a single node run queue-only
      const int64_t fr = p->level_frontier.empty() ? 0 : p->level_frontier.back();
      if (!p->opt.exchange && tu.sparse_div > 0 && fr * tu.sparse_div < words) {
        int64_t gnew = 0;
        s = queue_only_level(p, &gnew);
        if (s) { p->time_levels = false; return s; }
        if (gnew == 0) break;
        continue;
      }
      const uint64_t *local_next = nullptr;
      s = bfs_expand(p, &local_next);
      if (s) { p->time_levels = false; return s; }
      const uint64_t *const *inc = nullptr;
      int32_t k = 0;
      if (p->opt.exchange) {
        e = hipStreamSynchronize(p->stream);
        if (e != hipSuccess) return p->hip_fail(e, "hipStreamSynchronize");
        int32_t rc = p->opt.exchange(p->opt.exchange_ctx, p->level, local_next, &inc, &k);
        if (rc != 0) {
        p->time_levels = false;
        return p->fail(BFS_ERR_EXCHANGE, "exchange callback returned " + std::to_string(rc));
      }
        if (k < 0 || (k > 0 && !inc)) {
        p->time_levels = false;
        return p->fail(BFS_ERR_EXCHANGE, "exchange callback gave a bad list");
      }
      }
      int64_t gnew = 0;
      s = bfs_merge_frontier(p, inc, k, 0, &gnew, nullptr);
      if (s) { p->time_levels = false; return s; }
      if (gnew == 0) break;
    }
    p->time_levels = false;
    e = hipEventRecord(ev1, p->stream);
    if (e != hipSuccess) return p->hip_fail(e, "hipEventRecord");
  }
  e = hipEventSynchronize(ev1);
  if (e != hipSuccess) return p->hip_fail(e, "hipEventSynchronize");
  // a traversal that ran to its end left no mark set
  if (p->cur_mark) p->marks_clean = true;
  float ms = 0.f, lms = 0.f;
  if (hipEventElapsedTime(&ms, ev0, ev1) != hipSuccess) ms = -1.f;
  if (hipEventElapsedTime(&lms, p->ev[2], ev1) != hipSuccess) lms = -1.f;
  p->last_ms = ms;
  p->last_loop_ms = lms;
  p->last_expand_ms = p->last_merge_ms = p->last_queue_ms = p->last_bu_ms = 0.f;
  p->last_expand_launches = 0;
  p->timed_levels = 0;
  if (mode == BFS_LOOP_ENQUEUE) {
    // every timed step counts as an expansion launch, also the steps of the
    // last round that found the traversal finished (their kernels return at
    // once), so the totals cover every timed dispatch; per-level times stop
    // at the last level
    for (int L = 0; L < p->enqueued_steps; ++L) {
      float a = 0.f, b = 0.f;
      if (hipEventElapsedTime(&a, p->lev[L][0], p->lev[L][1]) != hipSuccess) a = 0.f;
      if (hipEventElapsedTime(&b, p->lev[L][1], p->lev[L][2]) != hipSuccess) b = 0.f;
      p->last_expand_ms += a;
      p->last_merge_ms += b;
      p->last_expand_launches += 1;
      p->lev_ms[L][0] = a;
      p->lev_ms[L][1] = b;
      p->level_kind[L] = 0;
    }
    p->timed_levels = std::min(p->enqueued_steps, p->level);
  }
  if (host_loop) {
    const int nl = std::min(p->level, Plan::kTimedLevels);
    p->timed_levels = nl;
    for (int L = 0; L < nl; ++L) {
      float a = 0.f, b = 0.f;
      if (hipEventElapsedTime(&a, p->lev[L][0], p->lev[L][1]) != hipSuccess) a = 0.f;
      if (hipEventElapsedTime(&b, p->lev[L][1], p->lev[L][2]) != hipSuccess) b = 0.f;
      p->lev_ms[L][0] = a;
      p->lev_ms[L][1] = p->level_kind[L] == 1 ? 0.f : b;
      b = 0.f;
      if (p->level_kind[L] == 1) {
        p->last_queue_ms += a;
        continue;
      }
      if (p->level_kind[L] == 2) {
        p->last_bu_ms += a;
        if (hipEventElapsedTime(&b, p->lev[L][1], p->lev[L][2]) == hipSuccess) p->last_merge_ms += b;
        continue;
      }
      p->last_expand_ms += a;
      p->last_expand_launches += 1;
      if (hipEventElapsedTime(&b, p->lev[L][1], p->lev[L][2]) == hipSuccess) p->last_merge_ms += b;
    }
  }
  return bfs_finish(p, parent, st);
}

bfs_status bfs_plan_tuning(bfs_plan_t p, int32_t graph, bfs_tuning *out) {
  if (!p) return BFS_ERR_ARG;
  if (graph < 0 || graph >= (int32_t)p->graphs.size() || !out)
    return p->fail(BFS_ERR_ARG, "bad graph index or NULL output");
  const Tuning &t = p->tune[graph];
  // the loop bfs_run drives: an explicit option wins over the tuned choice,
  // and an exchange callback or a direction-optimizing traversal needs the
  // host-driven loop
  out->loop_mode = p->opt.loop_mode != BFS_LOOP_AUTO ? p->opt.loop_mode : t.loop_mode;
  if (p->opt.exchange || p->direction_optimizing(graph)) out->loop_mode = BFS_LOOP_HOST;
  out->persist_variant = t.persist_variant;
  out->grid_blocks = p->persist_grid > 0 ? p->persist_grid : t.persist_grid;
  out->small_bin = t.small_bin;
  out->wave_bin = t.wave_bin;
  out->chunk_edges = 1 << t.chunk_shift;
  out->relabelled = (p->lay.rl_rp.size() > (size_t)graph && p->lay.rl_rp[graph]) ? 1 : 0;
  out->tuned_ms = t.tuned_ms;
  out->hot_words = t.hot_words;
  out->sparse_div = t.sparse_div;
  out->direction = p->direction_optimizing(graph) ? BFS_DIR_OPTIMIZING : BFS_DIR_TOPDOWN;
  out->mark_mode = t.mark ? 1 : -1;
  return BFS_OK;
}

bfs_status bfs_level_times(bfs_plan_t p, float *expand_ms, float *merge_ms, int32_t *kind,
                           int32_t max_levels, int32_t *levels) {
  if (!p) return BFS_ERR_ARG;
  if (!p->began) return p->fail(BFS_ERR_STATE, "no traversal yet");
  if (levels) *levels = p->timed_levels;
  const int cnt = std::min(p->timed_levels, std::max(max_levels, 0));
  for (int L = 0; L < cnt; ++L) {
    if (expand_ms) expand_ms[L] = p->lev_ms[L][0];
    if (merge_ms) merge_ms[L] = p->lev_ms[L][1];
    if (kind) kind[L] = p->level_kind[L];
  }
  return BFS_OK;
}

bfs_status bfs_level_stats(bfs_plan_t p, int64_t *frontier, int64_t *hist, int32_t max_levels,
                           int32_t *levels) {
  if (!p) return BFS_ERR_ARG;
  if (!p->opt.collect_stats) return p->fail(BFS_ERR_STATE, "plan created without collect_stats");
  if (!p->began) return p->fail(BFS_ERR_STATE, "no traversal yet");
  const int nl = std::min(p->level, kMaxStatLevels);
  if (levels) *levels = nl;
  const int cnt = std::min(nl, std::max(max_levels, 0));
  if (cnt <= 0) return BFS_OK;
  std::vector<int64_t> f((size_t)kMaxStatLevels);
  std::vector<uint32_t> h((size_t)kMaxStatLevels * kNumBins);
  hipError_t e = hipMemcpyAsync(f.data(), (char *)p->ws + p->lay.lvl_frontier,
                                sizeof(int64_t) * kMaxStatLevels, hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h.data(), (char *)p->ws + p->lay.lvl_hist,
                       sizeof(uint32_t) * kMaxStatLevels * kNumBins, hipMemcpyDeviceToHost, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) return p->hip_fail(e, "stats copy");
  for (int L = 0; L < cnt; ++L) {
    if (frontier) {
      if (p->persistent_levels > 0 || L == 0) frontier[L] = f[L];
      else frontier[L] = L < (int)p->level_frontier.size() ? p->level_frontier[L] : 0;
    }
    if (hist)
      for (int b = 0; b < kNumBins; ++b) hist[(size_t)L * kNumBins + b] = h[(size_t)L * kNumBins + b];
  }
  return BFS_OK;
}

}  // extern "C"

namespace bfsk {

// Plan creation, after autotuning: everything bfs_run would otherwise set up
// on first use. The captured level-step graph of every graph whose level loop
// is the captured one is instantiated now, with the settings and expansion
// form bfs_run uses, so bfs_run only replays it (no capture, instantiation
// or allocation inside a traversal); the occupancy of the tuned expansion
// kernels is queried here too.
bfs_status prepare_run_loops(Plan *p) {
  for (size_t gi = 0; gi < p->graphs.size(); ++gi) {
    const Tuning &tu = p->tune[gi];
    (void)p->expand_grid(tu.hot_words);
    int mode = p->opt.loop_mode == BFS_LOOP_AUTO ? tu.loop_mode : p->opt.loop_mode;
    if (p->opt.exchange || p->direction_optimizing((int32_t)gi)) mode = BFS_LOOP_HOST;
    if (mode != BFS_LOOP_GRAPH) continue;
    std::lock_guard<std::mutex> lk(p->run_mu);
    p->cur_relabel = true;  // bfs_run's setting without an exchange callback
    p->cur_do = false;
    p->cur_front = false;
    dense_form(p, (int32_t)gi);
    hipGraphExec_t ge = nullptr;
    bfs_status s = graph_exec(p, (int32_t)gi, ge);
    p->cur_mark = p->cur_into_vis = false;
    if (s) return s;
  }
  return BFS_OK;
}

}  // namespace bfsk
