// Host-side plan object behind the opaque bfs_plan_t handle.
#pragma once

#include <hip/hip_runtime.h>

#include <atomic>
#include <condition_variable>
#include <cstdint>
#include <deque>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <thread>
#include <vector>

#include "../../include/bfs.h"
#include "bfs_core.hpp"

namespace bfsk {

// Byte offsets of the workspace regions.
struct WsLayout {
  size_t ctl, lvl_frontier, lvl_hist, visited, next, front;
  size_t list_blk;  // uint64[kListMaxBlocks + 1]: block counts of the list export
  size_t mark = 0;  // uint8[64 * words]: per-vertex marks of dense levels (whole graphs; 0: none)
  size_t hubnext = 0;  // uint64[kMaxHotWords]: hub targets found by a level (follows mark)
  size_t q[3][kRing];
  size_t qr[2][kRing];  // uint64[omax]: packed rows of the tier-0/1 queues
  size_t cstart[kRing];
  // batched multi-source state (see msbfs_core.hpp)
  // relabelled copies (per graph; 0 when the graph is not relabelled) and
  // plan-time scratch for building them
  std::vector<size_t> rl_rp, rl_col, rl_old, rl_new;
  size_t tune_dist = 0;  // int32[n_max] scratch distances for autotuning (0: none)
  size_t rl_keys_a = 0, rl_keys_b = 0, rl_tmp_col = 0, rl_temp = 0, rl_temp_bytes = 0;
  bool ms_on = false;
  int64_t ms_ntot = 0, ms_mtot = 0;
  size_t ms_ctl, ms_graphs, ms_rp, ms_col, ms_F, ms_N, ms_S;
  size_t ms_q[3][2], ms_cstart[2], ms_extra, ms_mark, ms_touched;
  size_t ms_slot_out, ms_slot_type, ms_slot_start, ms_slot_active, ms_newmask, ms_depth_err;
  size_t ms_admit, ms_mask;
};

// Tier thresholds per graph (degree bins; see bfs_core.hpp).
struct Tuning {
  int32_t small_bin = 6;     // degree < 32 -> lane-group tier
  int32_t wave_bin = 13;     // degree < 4096 -> wavefront tier
  int32_t chunk_shift = 11;  // 2048-edge chunks for the hub tier (one wavefront each)
  int32_t sparse_div = 4;    // queue-only level when frontier < words / 4
  int32_t persist_variant = 0;  // 0: default registers, 1: 64-VGPR cap (8 waves/SIMD)
  int32_t persist_grid = 0;     // blocks of the cooperative launch
  int32_t loop_mode = 0;        // chosen level loop (BFS_LOOP_HOST or BFS_LOOP_PERSISTENT)
  float tuned_ms = 0.f;         // best time seen by the autotuner
  int32_t hot_words = 0;        // visited words kept in LDS by each expansion block (0: off)
  int32_t mark = 1;             // single-node dense levels: byte marks (1) or atomic ORs (0)
};

struct BatchState;  // batched / serving state (msbfs.hip)

}  // namespace bfsk

struct bfs_plan_s {
  std::vector<bfs_graph> graphs;
  bfs_options opt{};
  void *ws = nullptr;
  size_t ws_bytes = 0;
  hipStream_t stream = nullptr;
  bfsk::WsLayout lay{};
  std::vector<bfsk::Tuning> tune;
  int num_cus = 0;
  int coop = 0;
  int persist_grid = 0;  // caller's grid_blocks (0: per-graph choice)
  int bpc[2] = {0, 0};   // co-resident blocks per CU of the two persistent variants
  int bpc_expand = 0;    // co-resident blocks per CU of the per-phase expansion
  std::map<int, int> hot_bpc;  // co-resident expansion blocks per CU by LDS hub-copy size
  int max_lds = 65536;          // dynamic LDS bytes one workgroup may use
  int expand_grid(int hot_words);
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  bfsk::Ctl *hctl = nullptr;  // pinned host copy of the control block, read after each level
  std::vector<int64_t> rl_live;  // per relabelled graph: vertices with an edge (ids below it)
  static constexpr int kTimedLevels = 64;
  hipEvent_t lev[kTimedLevels][3] = {};  // per level: before expand, after expand, after merge
  bool time_levels = false;              // set while bfs_run drives the host loop
  float lev_ms[kTimedLevels][2] = {};    // last host-driven traversal: Phase 1 / Phase 2 ms per level
  int32_t timed_levels = 0;              // levels in lev_ms (0: the last traversal was not host-driven)
  int32_t enqueued_steps = 0;            // BFS_LOOP_ENQUEUE: level steps bracketed by lev events
  std::string err;

  // single-source traversal state
  std::mutex run_mu;
  bool began = false, finished = false;
  int32_t cur_graph = 0;
  int64_t cur_source = 0;
  int32_t *cur_dist = nullptr;
  bool cur_relabel = false;  // the current traversal runs on the relabelled copy
  int32_t level = 0;
  int32_t expanded_level = -1;  // last level bfs_expand ran for
  bool big_level = false;       // the current level's frontier is large (host loop)
  int32_t persistent_levels = 0;
  int64_t last_level_new = 0;
  float last_ms = 0.f;
  float last_loop_ms = 0.f;
  float last_expand_ms = 0.f, last_merge_ms = 0.f, last_queue_ms = 0.f;
  int32_t last_expand_launches = 0;
  // host-driven loop: how level L ran (0 dense top-down, 1 queue-only, 2 bottom-up)
  uint8_t level_kind[kTimedLevels] = {};
  float last_bu_ms = 0.f;
  int32_t bu_levels_run = 0;
  // direction-optimizing traversal (bfs_run, whole graph, no exchange)
  bool cur_do = false;                // the running traversal may go bottom-up
  bool cur_front = false;             // merges write the next level's frontier bitmap
  bool cur_into_vis = false;          // dense expansions OR into `visited` (see View::into_vis)
  bool cur_mark = false;              // dense expansions set byte marks (see View::mark)
  bool marks_clean = false;           // every mark byte is 0 (a finished traversal clears its marks)
  bool bu_state = false;              // the current level runs bottom-up
  int front_level = -1;               // level whose frontier the front bitmap holds
  int32_t merge_mode = 0;             // mode of bfs_merge_frontier's merge (bfs_run's bottom-up levels)
  bool queues_stale = false;          // the last merge left the tier queues unwritten
  std::vector<int64_t> edges_after;   // edge counter (sum of reached degrees) after each level
  int bpc_bu = 0;                     // co-resident bottom-up blocks per CU
  bool direction_optimizing(int32_t gi) const {
    return opt.direction == BFS_DIR_OPTIMIZING && !opt.exchange && graphs[gi].v_begin == 0 &&
           graphs[gi].v_end == graphs[gi].n_global;
  }
  std::vector<int64_t> level_frontier;

  // captured level-step graphs, one per graph index, with the settings they
  // were captured with
  static constexpr int kGraphLevels = 8;
  hipStream_t cap_stream = nullptr;
  std::vector<hipGraphExec_t> gexec;
  std::vector<bfsk::Tuning> gexec_tune;

  bfsk::BatchState *batch = nullptr;

  bfs_status fail(bfs_status st, const std::string &msg);
  bfs_status hip_fail(hipError_t e, const char *what);
  bfsk::View view(int32_t gi, int32_t *dist) const;
  int wide_grid() const;
  int merge_grid(int64_t words) const;
  bfs_status read_ctl(bfsk::Ctl &c);

  ~bfs_plan_s() {
    for (auto &e : ev)
      if (e) (void)hipEventDestroy(e);
    for (auto &row : lev)
      for (auto &e : row)
        if (e) (void)hipEventDestroy(e);
    for (auto &g : gexec)
      if (g) (void)hipGraphExecDestroy(g);
    if (cap_stream) (void)hipStreamDestroy(cap_stream);
    if (hctl) (void)hipHostFree(hctl);
  }
};

namespace bfsk {
using Plan = bfs_plan_s;

void layout_single(const bfs_graph *g, int32_t ng, WsLayout &L, size_t &off);
void layout_relabel(const bfs_graph *g, int32_t ng, const bfs_options *o, WsLayout &L, size_t &off);
bool relabel_wanted(const bfs_graph &g, const bfs_options *o);
bfs_status relabel_graphs(Plan *p);
bfs_status autotune_graphs(Plan *p);
bfs_status prepare_run_loops(Plan *p);
// Message that bfs_last_error(NULL) returns on this thread.
void set_create_error(const std::string &msg);
void layout_batch(const bfs_graph *g, int32_t ng, const bfs_options *o, WsLayout &L, size_t &off);
bfs_status validate_graphs(Plan *p);
bfs_status choose_tuning(Plan *p);
bfs_status batch_init(Plan *p);
void batch_shutdown(Plan *p);
}  // namespace bfsk
