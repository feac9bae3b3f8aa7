// Host side of the batched multi-source traversal and of the serving loop.
//
// A plan created with batch_lanes = LW > 0 reserves LW 64-bit lane words per
// vertex of every graph: LW*64 source slots per graph. Submitted queries wait
// in per-graph FIFOs; a scheduler thread admits them into free slots at level
// boundaries (continuous batching: a query joins while others are mid-flight
// and carries its own start level), launches the cooperative level loop over
// all graphs at once, retires slots whose traversal has ended and completes
// tickets. Slot memory is the admission budget: with no free slot a query
// waits until one is released. A streaming launch runs at most 256 levels and
// ends early when a slot of a graph with waiting queries finishes, so long
// traversals (high-diameter graphs) are not cut into many short launches by
// queries of other graphs.

#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cstring>
#include <string>

#include "bfs_core.hpp"
#include "msbfs_core.hpp"
#include "plan.hpp"

namespace bfsk {

namespace {

size_t align256(size_t x) { return (x + 255) / 256 * 256; }

int64_t now_ns() {
  return std::chrono::duration_cast<std::chrono::nanoseconds>(
             std::chrono::steady_clock::now().time_since_epoch())
      .count();
}

}  // namespace

struct MsQuery {
  int32_t graph = 0;
  int32_t type = 0;
  int64_t src = 0;
  void *out = nullptr;
  uint64_t ticket = 0;
  int32_t index_in_ticket = 0;
  int32_t status = BFS_OK;
  int64_t complete_ns = 0;
  int64_t bytes = 0;  // admission cost
};

// Admission cost of a query: its distance output and its share of the three
// lane-word arrays (8 bytes per 64 sources per vertex each).
int64_t query_bytes(int64_t n, int32_t out_type) {
  return n * (out_type == BFS_OUT_U8 ? 1 : 4) + 24 * n / 64;
}

struct MsTicket {
  int32_t nq = 0;
  int32_t done = 0;
  int32_t status = BFS_OK;
  int64_t submit_ns = 0;
  int64_t complete_ns = 0;
  std::vector<int64_t> times;
};

struct BatchState {
  Plan *p = nullptr;
  int lw = 0, ng = 0;
  MsView view{};
  std::vector<MsGraph> ghost;
  int grid = 0;

  std::mutex mu;
  std::condition_variable cv_work, cv_done;
  std::vector<std::deque<MsQuery>> pending;  // per graph
  std::vector<MsQuery> slot_q;               // [ng*lw*64]
  std::vector<uint64_t> active;              // [ng*lw]
  std::vector<uint64_t> dirty;               // [ng*lw] bits to clear before reuse
  std::map<uint64_t, MsTicket> tickets;
  std::deque<uint64_t> completed;  // tickets finished and not yet polled
  uint64_t next_ticket = 1;
  bool stop = false;
  std::string worker_error;
  std::thread worker;

  MsAdmit *h_adm = nullptr;   // pinned staging [ng*lw*64]
  uint64_t *h_mask = nullptr; // pinned staging [4*ng*lw]
  hipStream_t stream = nullptr;

  int64_t launches = 0, levels_total = 0;
  int64_t budget = 0;            // mem_budget_bytes (0: slots only)
  int64_t inflight_bytes = 0;    // admission cost of the queries in slots
  int64_t admitted = 0, admitted_midflight = 0, max_inflight = 0, max_inflight_bytes = 0;
  int32_t last_level = 0;       // global level clock of the engine
  bool streaming_mode = false;  // a streaming ticket was submitted
  float tuned_ms = 0.f;         // batch autotuner: best one-launch batch time (0: not tuned)

  void run();
  bool step(std::unique_lock<std::mutex> &lk);
};

void layout_batch(const bfs_graph *g, int32_t ng, const bfs_options *o, WsLayout &L, size_t &off) {
  L.ms_on = false;
  if (!o || o->batch_lanes <= 0) return;
  const int lw = o->batch_lanes;
  int64_t ntot = 0, mtot = 0;
  for (int i = 0; i < ng; ++i) {
    ntot += g[i].n_global;
    mtot += g[i].m;
  }
  L.ms_on = true;
  L.ms_ntot = ntot;
  L.ms_mtot = mtot;
  const size_t nslot = (size_t)ng * lw * 64, nslotw = (size_t)ng * lw;
  auto take = [&](size_t bytes) {
    size_t r = off;
    off = align256(off + std::max<size_t>(bytes, 8));
    return r;
  };
  L.ms_ctl = take(sizeof(MsCtl));
  L.ms_graphs = take(sizeof(MsGraph) * (size_t)ng);
  L.ms_rp = take(sizeof(int64_t) * (size_t)(ntot + 1));
  L.ms_col = take(sizeof(int32_t) * (size_t)mtot);
  L.ms_F = take(sizeof(uint64_t) * (size_t)ntot * lw);
  L.ms_N = take(sizeof(uint64_t) * (size_t)ntot * lw);
  L.ms_S = take(sizeof(uint64_t) * (size_t)ntot * lw);
  for (int t = 0; t < 3; ++t)
    for (int q = 0; q < 2; ++q) L.ms_q[t][q] = take(sizeof(int32_t) * (size_t)ntot);
  for (int q = 0; q < 2; ++q) L.ms_cstart[q] = take(sizeof(uint32_t) * (size_t)ntot);
  L.ms_extra = take(sizeof(int32_t) * nslot);
  L.ms_mark = take(sizeof(int32_t) * (size_t)ntot);
  L.ms_touched = take(sizeof(int32_t) * (size_t)ntot);
  L.ms_slot_out = take(sizeof(uint64_t) * nslot);
  L.ms_slot_type = take(sizeof(int32_t) * nslot);
  L.ms_slot_start = take(sizeof(int32_t) * nslot);
  L.ms_slot_active = take(sizeof(uint64_t) * nslotw);
  L.ms_newmask = take(sizeof(uint64_t) * 3 * nslotw);
  L.ms_depth_err = take(sizeof(uint64_t) * nslotw);
  L.ms_admit = take(sizeof(MsAdmit) * nslot);
  L.ms_mask = take(sizeof(uint64_t) * nslotw);
}

// Batch autotuner (plan creation, before the scheduler thread starts): times
// one-launch batches of lw*64 sources per graph, outputs discarded, for a few
// settings of the batched kernel -- grid size, then the degree-bin tier
// thresholds, then the hub chunk size -- keeping each change only if it is
// faster. Options given explicitly are not changed. Sources: vertices with an
// edge among the first 2^16 of each graph (R-MAT labels are permuted).
bfs_status batch_autotune(Plan *p, BatchState *b, int bpc) {
  const int a = p->opt.autotune;
  if (a < 0 || (a == 0 && p->lay.ms_mtot < (1ll << 20))) return BFS_OK;
  const int per_graph = b->lw * 64;
  std::vector<std::vector<int64_t>> srcs(b->ng);
  for (int g = 0; g < b->ng; ++g) {
    const bfs_graph &gr = p->graphs[g];
    const int64_t cnt = std::min<int64_t>(gr.n_global, 1 << 16);
    std::vector<int64_t> rp((size_t)cnt + 1);
    hipError_t e = hipMemcpy(rp.data(), gr.row_ptr, sizeof(int64_t) * (cnt + 1), hipMemcpyDeviceToHost);
    if (e != hipSuccess) return p->hip_fail(e, "batch autotune sources");
    for (int64_t v = 0; v < cnt && (int)srcs[g].size() < per_graph; ++v)
      if (rp[v + 1] > rp[v]) srcs[g].push_back(v);
    if (srcs[g].empty()) srcs[g].push_back(0);
  }
  auto run_once = [&](float &ms) -> bfs_status {
    const uint64_t tk = b->next_ticket++;
    MsTicket &t = b->tickets[tk];
    t.nq = b->ng * per_graph;
    t.times.assign((size_t)t.nq, 0);
    t.submit_ns = now_ns();
    int idx = 0;
    for (int g = 0; g < b->ng; ++g)
      for (int k = 0; k < per_graph; ++k) {
        MsQuery q;
        q.graph = g;
        q.type = 2;
        q.src = srcs[g][(size_t)k % srcs[g].size()];
        q.ticket = tk;
        q.index_in_ticket = idx++;
        b->pending[g].push_back(q);
      }
    std::unique_lock<std::mutex> lk(b->mu);
    while (t.done < t.nq && b->step(lk)) {
    }
    const bool ok = t.done == t.nq && t.status == BFS_OK && b->worker_error.empty();
    ms = (float)(t.complete_ns - t.submit_ns) * 1e-6f;
    b->tickets.erase(tk);
    b->completed.clear();
    if (!ok) return p->fail(BFS_ERR_DEVICE, "batch autotune run failed: " + b->worker_error);
    return BFS_OK;
  };
  struct Setting {
    int grid, small_bin, wave_bin, chunk_shift;
  };
  auto apply = [&](const Setting &c) {
    b->grid = c.grid;
    b->view.small_bin = c.small_bin;
    b->view.wave_bin = c.wave_bin;
    b->view.chunk_shift = c.chunk_shift;
  };
  Setting best{b->grid, b->view.small_bin, b->view.wave_bin, b->view.chunk_shift};
  float best_ms = 1e30f;
  auto trial = [&](const Setting &c) -> bfs_status {
    if (c.small_bin < 1 || c.wave_bin < c.small_bin || c.grid <= 0 || c.grid > bpc * p->num_cus ||
        c.grid > kBarrierMaxBlocks)
      return BFS_OK;
    apply(c);
    float warm = 0.f, ms = 0.f;
    bfs_status s = run_once(warm);
    if (s == BFS_OK && warm < 3.f * best_ms) s = run_once(ms);
    else ms = warm;
    if (s) return s;
    if (ms < best_ms) {
      best_ms = ms;
      best = c;
    }
    apply(best);
    return BFS_OK;
  };
  bfs_status s = trial(best);
  const int cus = p->num_cus;
  // grid and tier-0 threshold together: the best grid depends on the
  // threshold (fewer, longer tier-0 batches suit a smaller grid), so tuning
  // them one after the other can stop at the worse pair
  {
    const Setting start = best;
    std::vector<int> grids{start.grid}, sbs{start.small_bin};
    if (p->opt.grid_blocks <= 0) grids = {cus, 2 * cus, std::min(bpc, 8) * cus};
    if (p->opt.small_bin <= 0) sbs = {4, 8};
    for (int g : grids) {
      for (int sb : sbs) {
        Setting c = start;
        c.grid = g;
        c.small_bin = sb;
        if (!s) s = trial(c);
      }
    }
  }
  if (!s && p->opt.wave_bin <= 0)
    for (int wb : {11, 15}) {
      Setting c = best;
      c.wave_bin = std::max(wb, c.small_bin);
      if ((s = trial(c))) break;
    }
  if (!s && p->opt.chunk_edges <= 0)
    for (int cs : {10, 12}) {
      Setting c = best;
      c.chunk_shift = cs;
      if ((s = trial(c))) break;
    }
  apply(best);
  b->tuned_ms = best_ms;
  b->launches = 0;
  b->levels_total = 0;
  return s;
}

bfs_status batch_init(Plan *p) {
  const WsLayout &L = p->lay;
  if (!L.ms_on) return BFS_OK;
  const int lw = p->opt.batch_lanes;
  if (lw != 1 && lw != 2 && lw != 4) return p->fail(BFS_ERR_ARG, "batch_lanes must be 1, 2 or 4");
  const int ng = (int)p->graphs.size();
  if (ng > kMsMaxGraphs) return p->fail(BFS_ERR_ARG, "batched plans take at most 16 graphs");
  if (L.ms_ntot >= (1ll << 31)) return p->fail(BFS_ERR_ARG, "batched graphs exceed 2^31 vertices");
  for (const bfs_graph &g : p->graphs)
    if (g.v_begin != 0 || g.v_end != g.n_global)
      return p->fail(BFS_ERR_ARG, "batched queries need whole graphs, not shares");
  BatchState *b = new (std::nothrow) BatchState();
  if (!b) return p->fail(BFS_ERR_ARG, "out of host memory");
  b->p = p;
  b->lw = lw;
  b->ng = ng;
  b->stream = p->stream;
  char *w = (char *)p->ws;
  MsView &v = b->view;
  v.ng = ng;
  v.lw = lw;
  v.ntot = L.ms_ntot;
  v.rp = (const int64_t *)(w + L.ms_rp);
  v.col = (const int32_t *)(w + L.ms_col);
  v.F = (uint64_t *)(w + L.ms_F);
  v.N = (uint64_t *)(w + L.ms_N);
  v.S = (uint64_t *)(w + L.ms_S);
  for (int q = 0; q < 2; ++q) {
    v.q0[q] = (int32_t *)(w + L.ms_q[0][q]);
    v.q1[q] = (int32_t *)(w + L.ms_q[1][q]);
    v.q2[q] = (int32_t *)(w + L.ms_q[2][q]);
    v.cstart[q] = (uint32_t *)(w + L.ms_cstart[q]);
  }
  v.extra = (int32_t *)(w + L.ms_extra);
  v.mark = (int32_t *)(w + L.ms_mark);
  v.touched = (int32_t *)(w + L.ms_touched);
  v.sparse_shift = 6;
  v.ctl = (MsCtl *)(w + L.ms_ctl);
  v.graphs = (const MsGraph *)(w + L.ms_graphs);
  v.slot_out = (uint64_t *)(w + L.ms_slot_out);
  v.slot_type = (int32_t *)(w + L.ms_slot_type);
  v.slot_start = (int32_t *)(w + L.ms_slot_start);
  v.stop_slots = (uint64_t *)(w + L.ms_slot_active);
  v.newmask = (uint64_t *)(w + L.ms_newmask);
  v.depth_err = (uint64_t *)(w + L.ms_depth_err);
  const Tuning &t = p->tune.empty() ? Tuning{} : p->tune[0];
  v.small_bin = t.small_bin;
  v.wave_bin = t.wave_bin;
  v.chunk_shift = t.chunk_shift;

  // Flat union graph and its table.
  int64_t off = 0, eoff = 0, chunk = 0;
  b->ghost.resize(ng);
  for (int i = 0; i < ng; ++i) {
    const bfs_graph &g = p->graphs[i];
    b->ghost[i] = MsGraph{off, g.n_global, chunk};
    hipError_t e = ms_launch_flatten(g.row_ptr, g.col, g.n_global, g.m, off, eoff,
                                     (int64_t *)v.rp, (int32_t *)v.col, p->stream);
    if (e != hipSuccess) { delete b; return p->hip_fail(e, "flatten launch"); }
    off += g.n_global;
    eoff += g.m;
    chunk += (g.n_global + kMsChunk - 1) / kMsChunk;
  }
  v.nchunks = chunk;
  hipError_t e = hipMemcpyAsync((void *)v.graphs, b->ghost.data(), sizeof(MsGraph) * ng,
                                hipMemcpyHostToDevice, p->stream);
  // Zero every piece of lane state once; afterwards the kernels keep it clean.
  const size_t zero_from = L.ms_ctl;
  if (e == hipSuccess) e = hipMemsetAsync(w + L.ms_F, 0, L.ms_q[0][0] - L.ms_F, p->stream);
  if (e == hipSuccess) e = hipMemsetAsync(w + zero_from, 0, sizeof(MsCtl), p->stream);
  if (e == hipSuccess)
    e = hipMemsetAsync(w + L.ms_slot_active, 0, L.ms_admit - L.ms_slot_active, p->stream);
  if (e == hipSuccess)  // no vertex has been touched at any level yet
    e = hipMemsetAsync(w + L.ms_mark, 0xFF, sizeof(int32_t) * (size_t)L.ms_ntot, p->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(p->stream);
  if (e != hipSuccess) { delete b; return p->hip_fail(e, "batch state init"); }
  const size_t nslot = (size_t)ng * lw * 64;
  if (hipHostMalloc((void **)&b->h_adm, sizeof(MsAdmit) * nslot, hipHostMallocDefault) != hipSuccess ||
      hipHostMalloc((void **)&b->h_mask, sizeof(uint64_t) * 4 * ng * lw, hipHostMallocDefault) != hipSuccess) {
    if (b->h_adm) (void)hipHostFree(b->h_adm);
    delete b;
    return p->fail(BFS_ERR_HIP, "hipHostMalloc of staging buffers failed");
  }
  int bpc = ms_blocks_per_cu(lw);
  b->grid = p->opt.grid_blocks > 0 ? p->opt.grid_blocks : p->num_cus * std::min(std::max(bpc, 1), 4);
  if (b->grid > kBarrierMaxBlocks) {
    (void)hipHostFree(b->h_adm);
    (void)hipHostFree(b->h_mask);
    delete b;
    return p->fail(BFS_ERR_ARG, "grid_blocks exceeds the grid barrier's 2048 blocks");
  }
  if (bpc <= 0 || b->grid > bpc * p->num_cus || !p->coop) {
    (void)hipHostFree(b->h_adm);
    (void)hipHostFree(b->h_mask);
    delete b;
    return p->fail(BFS_ERR_HIP, "cooperative launch of the batched loop is not available");
  }
  b->budget = std::max<int64_t>(p->opt.mem_budget_bytes, 0);
  b->pending.resize(ng);
  b->slot_q.resize(nslot);
  b->active.assign((size_t)ng * lw, 0);
  b->dirty.assign((size_t)ng * lw, 0);
  p->batch = b;
  bfs_status st = batch_autotune(p, b, bpc);
  if (st) {
    p->batch = nullptr;
    (void)hipHostFree(b->h_adm);
    (void)hipHostFree(b->h_mask);
    delete b;
    return st;
  }
  // the counters describe the caller's queries, not the autotuner's batches
  b->launches = b->levels_total = 0;
  b->admitted = b->admitted_midflight = b->max_inflight = b->max_inflight_bytes = 0;
  b->worker = std::thread([b] { b->run(); });
  return BFS_OK;
}

void batch_shutdown(Plan *p) {
  BatchState *b = p->batch;
  if (!b) return;
  {
    std::lock_guard<std::mutex> lk(b->mu);
    b->stop = true;
  }
  b->cv_work.notify_all();
  if (b->worker.joinable()) b->worker.join();
  (void)hipStreamSynchronize(b->stream);
  (void)hipHostFree(b->h_adm);
  (void)hipHostFree(b->h_mask);
  delete b;
  p->batch = nullptr;
}

// One scheduling round: admit, launch, retire. Called with the lock held;
// releases it around device work. Returns false when there is nothing to do.
bool BatchState::step(std::unique_lock<std::mutex> &lk) {
  const int nslotw = ng * lw;
  bool any_active = false, any_pending = false;
  for (int i = 0; i < nslotw; ++i) any_active |= active[i] != 0;
  for (int g = 0; g < ng; ++g) any_pending |= !pending[g].empty();
  if (!any_active && !any_pending) return false;

  // Slots released by finished queries still hold their seen bits; a graph
  // with waiting queries gets those bits cleared before admission (stream
  // order makes the cleared slots usable in this round).
  std::vector<int> clear_graphs;
  for (int g = 0; g < ng; ++g) {
    if (pending[g].empty()) continue;
    bool has_dirty = false;
    for (int l = 0; l < lw; ++l) has_dirty |= dirty[g * lw + l] != 0;
    if (!has_dirty) continue;
    clear_graphs.push_back(g);
    for (int l = 0; l < lw; ++l) {
      h_mask[g * lw + l] = dirty[g * lw + l];
      dirty[g * lw + l] = 0;
    }
  }
  int nadm = 0;
  int64_t maxn = 0;
  const int32_t level = last_level;
  for (int g = 0; g < ng; ++g) {
    auto &q = pending[g];
    while (!q.empty()) {
      int slot = -1;
      for (int l = 0; l < lw && slot < 0; ++l) {
        const uint64_t used = active[g * lw + l] | dirty[g * lw + l];
        if (~used) slot = (g * lw + l) * 64 + __builtin_ctzll(~used);
      }
      if (slot < 0) break;
      if (budget > 0 && inflight_bytes + q.front().bytes > budget) break;
      MsQuery mq = q.front();
      q.pop_front();
      inflight_bytes += mq.bytes;
      admitted += 1;
      if (any_active) admitted_midflight += 1;
      active[slot / 64] |= 1ull << (slot % 64);
      slot_q[slot] = mq;
      h_adm[nadm++] = MsAdmit{ghost[g].off + mq.src, mq.src, ghost[g].n, (uint64_t)mq.out, mq.type,
                              slot};
      maxn = std::max(maxn, ghost[g].n);
    }
  }
  {
    int64_t nact = 0;
    for (int i = 0; i < nslotw; ++i) nact += __builtin_popcountll(active[i]);
    max_inflight = std::max(max_inflight, nact);
    max_inflight_bytes = std::max(max_inflight_bytes, inflight_bytes);
  }
  // A streaming launch stops early only when a slot of a graph with waiting
  // queries finishes (the freed slot can then be refilled); slots of other
  // graphs finish silently and are retired when the launch ends.
  bool still_pending = false;
  for (int g = 0; g < ng; ++g) still_pending |= !pending[g].empty();
  for (int i = 0; i < nslotw; ++i) h_mask[nslotw + i] = pending[i / lw].empty() ? 0ull : active[i];
  const bool streaming = still_pending || streaming_mode;
  lk.unlock();

  // Device work for this round.
  hipError_t e = hipSuccess;
  char *w = (char *)p->ws;
  uint64_t *d_mask = (uint64_t *)(w + p->lay.ms_mask);
  if (!clear_graphs.empty())
    e = hipMemcpyAsync(d_mask, h_mask, sizeof(uint64_t) * nslotw, hipMemcpyHostToDevice, stream);
  for (int g : clear_graphs)
    if (e == hipSuccess)
      e = ms_launch_clear(view, ghost[g].off, ghost[g].off + ghost[g].n, d_mask + g * lw, stream);
  MsAdmit *d_adm = (MsAdmit *)(w + p->lay.ms_admit);
  if (e == hipSuccess && nadm > 0)
    e = hipMemcpyAsync(d_adm, h_adm, sizeof(MsAdmit) * nadm, hipMemcpyHostToDevice, stream);
  if (e == hipSuccess) e = ms_launch_fill(d_adm, nadm, maxn, stream);
  if (e == hipSuccess) e = ms_launch_admit(view, d_adm, nadm, level, stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(view.stop_slots, h_mask + nslotw, sizeof(uint64_t) * nslotw,
                       hipMemcpyHostToDevice, stream);
  MsView v = view;
  v.stream_stop = streaming ? 1 : 0;
  // Streaming launches also end after kStreamLevels levels, which bounds how
  // long a newly submitted query waits for admission.
  const int max_levels = streaming ? kStreamLevels : (1 << 20);
  if (e == hipSuccess) e = ms_launch_persistent(v, max_levels, grid, stream);
  MsCtl ctl{};
  if (e == hipSuccess) e = hipMemcpyAsync(&ctl, view.ctl, sizeof(MsCtl), hipMemcpyDeviceToHost, stream);
  if (e == hipSuccess) e = hipStreamSynchronize(stream);
  const int64_t t_end = now_ns();
  if (e == hipSuccess) {
    const int lastL = ctl.level - 1;
    e = hipMemcpyAsync(h_mask + 2 * nslotw, view.newmask + (size_t)((lastL % 3 + 3) % 3) * nslotw,
                       sizeof(uint64_t) * nslotw, hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess)
      e = hipMemcpyAsync(h_mask + 3 * nslotw, view.depth_err, sizeof(uint64_t) * nslotw,
                         hipMemcpyDeviceToHost, stream);
    if (e == hipSuccess) e = hipStreamSynchronize(stream);
  }

  lk.lock();
  if (e != hipSuccess || ctl.bar.tripped) {
    worker_error = e != hipSuccess ? std::string("batched loop: ") + hipGetErrorString(e)
                                   : std::string("batched loop: grid barrier spin limit exceeded");
    // Fail every admitted query; the engine stops.
    for (int s = 0; s < nslotw * 64; ++s)
      if ((active[s / 64] >> (s % 64)) & 1ull) {
        MsTicket &t = tickets[slot_q[s].ticket];
        t.status = e != hipSuccess ? BFS_ERR_HIP : BFS_ERR_DEVICE;
        t.done += 1;
        t.complete_ns = t_end;
        if (t.done == t.nq) completed.push_back(slot_q[s].ticket);
      }
    std::fill(active.begin(), active.end(), 0);
    inflight_bytes = 0;
    stop = true;
    cv_done.notify_all();
    return false;
  }
  last_level = ctl.level;
  launches += 1;
  levels_total += ctl.levels_run;
  // Retire slots without a new vertex in the last level.
  bool depth_clear = false;
  for (int i = 0; i < nslotw; ++i) {
    uint64_t fin = active[i] & ~h_mask[2 * nslotw + i];
    while (fin) {
      const int b = __builtin_ctzll(fin);
      fin &= fin - 1;
      const int s = i * 64 + b;
      MsQuery &mq = slot_q[s];
      MsTicket &t = tickets[mq.ticket];
      if ((h_mask[3 * nslotw + i] >> b) & 1ull) {
        t.status = BFS_ERR_DEPTH;
        depth_clear = true;
      }
      t.times[mq.index_in_ticket] = t_end;
      t.done += 1;
      if (t.done == t.nq) {
        t.complete_ns = t_end;
        completed.push_back(mq.ticket);
      }
      active[i] &= ~(1ull << b);
      dirty[i] |= 1ull << b;
      inflight_bytes -= mq.bytes;
    }
  }
  if (depth_clear) {
    lk.unlock();
    hipError_t e2 = hipMemsetAsync(view.depth_err, 0, sizeof(uint64_t) * nslotw, stream);
    if (e2 == hipSuccess) e2 = hipStreamSynchronize(stream);
    lk.lock();
  }
  cv_done.notify_all();
  return true;
}

void BatchState::run() {
  std::unique_lock<std::mutex> lk(mu);
  while (true) {
    if (stop) break;
    if (!step(lk)) {
      if (stop) break;
      cv_work.wait(lk, [&] {
        if (stop) return true;
        for (auto &q : pending)
          if (!q.empty()) return true;
        return false;
      });
    }
  }
}

}  // namespace bfsk

using namespace bfsk;

extern "C" {

bfs_status bfs_batch_submit(bfs_plan_t p, const bfs_query *q, int32_t nq, uint32_t flags,
                            uint64_t *ticket) {
  if (!p) return BFS_ERR_ARG;
  BatchState *b = p->batch;
  if (!b) return p->fail(BFS_ERR_CAPACITY, "plan has no lane memory for batched queries (batch_lanes = 0)");
  if (nq < 0 || (nq > 0 && !q) || !ticket) return p->fail(BFS_ERR_ARG, "bad query list");
  if ((flags & (BFS_BATCH_ONE_LAUNCH | BFS_BATCH_STREAMING)) == 0)
    return p->fail(BFS_ERR_ARG, "flags must include BFS_BATCH_ONE_LAUNCH or BFS_BATCH_STREAMING");
  for (int i = 0; i < nq; ++i) {
    if (q[i].graph < 0 || q[i].graph >= b->ng) return p->fail(BFS_ERR_ARG, "query graph out of range");
    if (q[i].source < 0 || q[i].source >= b->ghost[q[i].graph].n)
      return p->fail(BFS_ERR_ARG, "query source out of range");
    if (!q[i].out) return p->fail(BFS_ERR_ARG, "query output is NULL");
    if (q[i].out_type != BFS_OUT_U8 && q[i].out_type != BFS_OUT_I32)
      return p->fail(BFS_ERR_ARG, "query out_type must be BFS_OUT_U8 or BFS_OUT_I32");
    const int64_t qb = query_bytes(b->ghost[q[i].graph].n, q[i].out_type);
    if (b->budget > 0 && qb > b->budget)
      return p->fail(BFS_ERR_CAPACITY, "query " + std::to_string(i) + " needs " + std::to_string(qb) +
                                           " bytes in flight, more than mem_budget_bytes (" +
                                           std::to_string(b->budget) + "): it can never be admitted");
  }
  {
    std::lock_guard<std::mutex> lk(b->mu);
    if (b->stop) return p->fail(BFS_ERR_STATE, "batched engine stopped: " + b->worker_error);
    const uint64_t t = b->next_ticket++;
    MsTicket &tk = b->tickets[t];
    tk.nq = nq;
    tk.submit_ns = now_ns();
    tk.times.assign(nq, 0);
    if (flags & BFS_BATCH_STREAMING) b->streaming_mode = true;
    for (int i = 0; i < nq; ++i) {
      MsQuery mq;
      mq.graph = q[i].graph;
      mq.type = q[i].out_type;
      mq.src = q[i].source;
      mq.out = q[i].out;
      mq.ticket = t;
      mq.index_in_ticket = i;
      mq.bytes = query_bytes(b->ghost[mq.graph].n, mq.type);
      b->pending[mq.graph].push_back(mq);
    }
    if (nq == 0) {
      tk.complete_ns = tk.submit_ns;
      b->completed.push_back(t);
    }
    *ticket = t;
  }
  b->cv_work.notify_all();
  return BFS_OK;
}

bfs_status bfs_batch_wait(bfs_plan_t p, uint64_t ticket, int64_t timeout_us, bfs_batch_result *r) {
  if (!p) return BFS_ERR_ARG;
  BatchState *b = p->batch;
  if (!b) return p->fail(BFS_ERR_CAPACITY, "plan has no lane memory for batched queries");
  std::unique_lock<std::mutex> lk(b->mu);
  auto it = b->tickets.find(ticket);
  if (it == b->tickets.end()) return p->fail(BFS_ERR_ARG, "unknown ticket");
  auto ready = [&] { return it->second.done >= it->second.nq || b->stop; };
  if (timeout_us < 0) {
    b->cv_done.wait(lk, ready);
  } else if (!b->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready)) {
    return p->fail(BFS_ERR_TIMEOUT, "ticket not finished within the timeout");
  }
  const MsTicket &t = it->second;
  if (t.done < t.nq) return p->fail(BFS_ERR_STATE, "batched engine stopped: " + b->worker_error);
  if (r) {
    r->status = t.status;
    r->nq = t.nq;
    r->submit_ns = t.submit_ns;
    r->complete_ns = t.complete_ns;
  }
  if (t.status != BFS_OK) {
    const bfs_status st = t.status;
    return p->fail(st, st == BFS_ERR_DEPTH ? "a uint8 distance exceeded 254" : b->worker_error);
  }
  return BFS_OK;
}

bfs_status bfs_batch_poll(bfs_plan_t p, uint64_t *done, int32_t max, int32_t *n,
                          int64_t timeout_us) {
  if (!p) return BFS_ERR_ARG;
  BatchState *b = p->batch;
  if (!b) return p->fail(BFS_ERR_CAPACITY, "plan has no lane memory for batched queries");
  if (!done || !n || max <= 0) return p->fail(BFS_ERR_ARG, "bad poll buffer");
  std::unique_lock<std::mutex> lk(b->mu);
  auto ready = [&] { return !b->completed.empty() || b->stop; };
  if (timeout_us < 0) b->cv_done.wait(lk, ready);
  else b->cv_done.wait_for(lk, std::chrono::microseconds(timeout_us), ready);
  int32_t k = 0;
  while (k < max && !b->completed.empty()) {
    done[k++] = b->completed.front();
    b->completed.pop_front();
  }
  *n = k;
  return BFS_OK;
}

bfs_status bfs_batch_times(bfs_plan_t p, uint64_t ticket, int64_t *complete_ns, int32_t nq) {
  if (!p) return BFS_ERR_ARG;
  BatchState *b = p->batch;
  if (!b) return p->fail(BFS_ERR_CAPACITY, "plan has no lane memory for batched queries");
  std::lock_guard<std::mutex> lk(b->mu);
  auto it = b->tickets.find(ticket);
  if (it == b->tickets.end()) return p->fail(BFS_ERR_ARG, "unknown ticket");
  const MsTicket &t = it->second;
  if (t.done < t.nq) return p->fail(BFS_ERR_STATE, "ticket not finished");
  for (int i = 0; i < std::min(nq, t.nq); ++i) complete_ns[i] = t.times[i];
  return BFS_OK;
}

bfs_status bfs_batch_query_bytes(bfs_plan_t p, int32_t graph, int32_t out_type, int64_t *bytes) {
  if (!p) return BFS_ERR_ARG;
  BatchState *b = p->batch;
  if (!b) return p->fail(BFS_ERR_CAPACITY, "plan has no lane memory for batched queries");
  if (graph < 0 || graph >= b->ng || !bytes || (out_type != BFS_OUT_U8 && out_type != BFS_OUT_I32))
    return p->fail(BFS_ERR_ARG, "bad graph index, output type or NULL output");
  *bytes = query_bytes(b->ghost[graph].n, out_type);
  return BFS_OK;
}

bfs_status bfs_batch_read_counters(bfs_plan_t p, bfs_batch_counters *out) {
  if (!p) return BFS_ERR_ARG;
  BatchState *b = p->batch;
  if (!b) return p->fail(BFS_ERR_CAPACITY, "plan has no lane memory for batched queries");
  if (!out) return p->fail(BFS_ERR_ARG, "NULL output");
  std::lock_guard<std::mutex> lk(b->mu);
  out->launches = b->launches;
  out->levels = b->levels_total;
  out->admitted = b->admitted;
  out->admitted_midflight = b->admitted_midflight;
  out->max_inflight = b->max_inflight;
  out->max_inflight_bytes = b->max_inflight_bytes;
  out->inflight_bytes = b->inflight_bytes;
  return BFS_OK;
}

bfs_status bfs_batch_tuning(bfs_plan_t p, bfs_tuning *out) {
  if (!p) return BFS_ERR_ARG;
  if (!out) return p->fail(BFS_ERR_ARG, "NULL output");
  BatchState *b = p->batch;
  if (!b) return p->fail(BFS_ERR_CAPACITY, "plan has no lane memory for batched queries");
  std::lock_guard<std::mutex> lk(b->mu);
  *out = bfs_tuning{};
  out->loop_mode = BFS_LOOP_PERSISTENT;
  out->grid_blocks = b->grid;
  out->small_bin = b->view.small_bin;
  out->wave_bin = b->view.wave_bin;
  out->chunk_edges = 1 << b->view.chunk_shift;
  out->tuned_ms = b->tuned_ms;
  out->direction = BFS_DIR_TOPDOWN;
  return BFS_OK;
}

}  // extern "C"
