// Single-source top-down traversal kernels for gfx950.
//
// Phases (Algorithm 2 of the paper; Algorithm 1 is the one-node case):
//   reset   - every distance to infinity, the root to 0 and into the owned
//             frontier if owned (Algorithm 2 set-up).
//   expand  - Phase 1: each owned frontier vertex scans its adjacency; every
//             neighbour not yet visited is marked in the node's next-frontier
//             bitmap with a device-scope atomic OR (the atomic enqueue of
//             Algorithm 2). Work is split by degree tier (logarithmic radix
//             binning, Section 4 "Load Balanced Traversals"):
//               tier 0: small degrees, 64 vertices per wavefront with their
//                       edges spread evenly over the lanes;
//               tier 1: medium degrees, one wavefront per vertex;
//               tier 2: large degrees, fixed-size edge chunks, one wavefront
//                       per chunk (a hub is spread over many CUs).
//   merge   - Phase 2: OR of the local bitmap with k received bitmaps,
//             new = merged & ~visited, distance level+1 for every new vertex,
//             owned new vertices compacted (ballot/popcount) straight into
//             the next level's tier queues.
// The same phase functions run either one launch per phase (host-driven
// loop) or inside one cooperative launch with grid barriers between phases.

#include <hip/hip_runtime.h>

#include "bfs_core.hpp"

namespace bfsk {

// ---------------------------------------------------------------------------
// reset
// ---------------------------------------------------------------------------

// src is a caller id; the traversal works on traversal ids (relabelled graphs).
__global__ void __launch_bounds__(kBlock) k_reset(View v, int64_t src_caller) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = tid; i < v.n; i += stride) v.dist[i] = (i == src_caller) ? 0 : -1;
  const int64_t src = v.new_id ? (int64_t)v.new_id[src_caller] : src_caller;
  const int64_t sw = src >> 6;
  for (int64_t i = tid; i < v.words; i += stride) {
    v.visited[i] = (i == sw) ? (1ull << (src & 63)) : 0ull;
    v.next[i] = 0ull;
  }
  // the grid barrier starts from barrier 0 (every announcement 0)
  if (blockIdx.x == 0)
    for (int i = threadIdx.x; i < kBarrierMaxBlocks; i += blockDim.x) v.ctl->bar.arrive[i] = 0;
  if (tid == 0) {
    Ctl *c = v.ctl;
    c->bar.gen = 0;
    c->bar.tripped = 0;
    for (int r = 0; r < kRing; ++r) {
      c->qn[r][0] = c->qn[r][1] = 0;
      c->heavy[r] = 0;
    }
    for (int k = 0; k < 3; ++k) c->newcnt[k] = c->ownedcnt[k] = 0;
    c->edges = 0;
    c->reached = 1;
    c->levels = 0;
    c->err = 0;
    c->glevel = 0;
    c->gdone = 0;
    c->gdist = v.dist;
    c->xedges = 0;
    c->xfront = 0;
    c->buedges = 0;
    c->buverts = 0;
    const bool owned = src >= v.vb && src < v.ve;
    int64_t deg = 0;
    if (owned) {
      const int64_t li = src - v.vb;
      deg = v.rp[li + 1] - v.rp[li];
      const int b = degree_bin(deg);
      const int t = tier_of_bin(b, v.small_bin, v.wave_bin);
      if (deg > 0) {
        if (t == 0) { v.q0[0][0] = (int32_t)src; v.qr0[0][0] = pack_row(v.rp[li], deg); c->qn[0][0] = 1; }
        else if (t == 1) { v.q1[0][0] = (int32_t)src; v.qr1[0][0] = pack_row(v.rp[li], deg); c->qn[0][1] = 1; }
        else {
          v.q2[0][0] = (int32_t)src;
          v.cstart[0][0] = 0;
          const uint64_t nch = (uint64_t)((deg + (1ll << v.chunk_shift) - 1) >> v.chunk_shift);
          c->heavy[0] = (1ull << kHeavyShift) | nch;
        }
      }
      c->edges = (uint64_t)deg;
    }
    c->gedges[0] = 0;
    c->gedges[1] = c->edges;
    if (v.stats) {
      v.lvl_frontier[0] = owned ? 1 : 0;
      for (int b = 0; b < 2 * kNumBins; ++b) v.lvl_hist[b] = 0;  // rows 0 and 1
      if (owned) v.lvl_hist[degree_bin(deg)] = 1;
    }
  }
}

// ---------------------------------------------------------------------------
// expand (Phase 1)
// ---------------------------------------------------------------------------

// Streams adjacency entries with a non-temporal hint so the bitmaps keep
// their place in L2.
__device__ __forceinline__ int32_t load_col(const int32_t *col, int64_t e) {
  return __builtin_nontemporal_load(col + e);
}

// K independent probes: all visited words are requested before any is
// tested, then all next words, so each lane keeps K random loads in flight.
// The probes read and OR 32-bit halves of the 64-bit bitmap words (bit v is
// bit v & 31 of 32-bit word v >> 5), which halves the registers a probe
// holds. `hot` is a copy of the first `words` 64-bit visited words in LDS
// (the hubs' bits once the graph is relabelled by degree); words == 0
// disables it.
struct HotCache {
  const uint64_t *lds;
  uint32_t words;
};
typedef __attribute__((address_space(3))) uint32_t lds_u32;

// Byte marks (View::mark): `visited` stays read-only during the level, so
// the LDS copy of the hubs' words is exact at the level's start. A hub target
// found unvisited is set in the block's LDS copy (an LDS atomic OR) and
// nowhere else: the block ORs the bits it added into `hubnext` once, at the
// end of the expansion, so hub targets cost no global traffic per edge. Every
// other candidate target takes one plain byte store (repeated stores of the
// same byte are harmless; no global atomic is issued per edge).
template <int K>
__device__ __forceinline__ void mark_targets(const View &v, const int32_t (&u)[K], const uint32_t (&w)[K],
                                             const bool (&need)[K], HotCache hot) {
  lds_u32 *hot32 = (lds_u32 *)(hot.lds);
  const uint32_t hot_w32 = hot.words * 2;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    if (!need[j]) continue;
    if (w[j] < hot_w32)
      (void)__hip_atomic_fetch_or(hot32 + w[j], 1u << (u[j] & 31), __ATOMIC_RELAXED,
                                  __HIP_MEMORY_SCOPE_WORKGROUP);
    else
      v.mark[(uint32_t)u[j]] = 1;
  }
}

template <int K>
__device__ __forceinline__ void probe_batch(const View &v, const int32_t (&u)[K],
                                            const bool (&ok)[K], HotCache hot) {
  const uint32_t *vis32 = reinterpret_cast<const uint32_t *>(v.visited);
  uint32_t *next32 = reinterpret_cast<uint32_t *>(v.next);
  // the copy is read through an LDS-qualified pointer so the reads are LDS
  // instructions rather than generic (flat) loads
  const lds_u32 *hot32 = (const lds_u32 *)(hot.lds);
  const uint32_t hot_w32 = hot.words * 2;
  // LDS and global reads land in separate registers: when both wrote one
  // register the compiler had to wait for each global read before issuing
  // the next LDS read, which serialised the K probes.
  uint32_t w[K], lv[K], gv[K], vis[K], nx[K];
#pragma unroll
  for (int j = 0; j < K; ++j) w[j] = (uint32_t)u[j] >> 5;  // u is 0 where !ok
  if (hot_w32) {
#pragma unroll
    for (int j = 0; j < K; ++j) lv[j] = hot32[min(w[j], hot_w32 - 1)];
  }
#pragma unroll
  for (int j = 0; j < K; ++j) {
    gv[j] = ~0u;
    // mark mode with an LDS copy marks the other targets without reading
    // `visited` (the merge drops those already visited): fewer scattered
    // loads for a few more scattered stores, a net gain on R-MAT levels
    if (ok[j] && w[j] >= hot_w32) gv[j] = (v.mark && hot_w32) ? 0u : vis32[w[j]];
  }
#pragma unroll
  for (int j = 0; j < K; ++j) vis[j] = !ok[j] ? ~0u : (w[j] < hot_w32 ? lv[j] : gv[j]);
  bool need[K];
#pragma unroll
  for (int j = 0; j < K; ++j) need[j] = !((vis[j] >> (u[j] & 31)) & 1u);
  if (v.mark) {
    mark_targets<K>(v, u, w, need, hot);
    return;
  }
  // into_vis: the OR goes into `visited` itself; a target seen unvisited in
  // global memory goes straight to the OR, one seen in the LDS snapshot is
  // read again from global memory first
  uint32_t *tgt32 = v.into_vis ? const_cast<uint32_t *>(vis32) : next32;
#pragma unroll
  for (int j = 0; j < K; ++j) {
    nx[j] = ~0u;
    if (need[j]) nx[j] = (v.into_vis && w[j] >= hot_w32) ? 0u : tgt32[(uint32_t)u[j] >> 5];
  }
#pragma unroll
  for (int j = 0; j < K; ++j)
    if (!((nx[j] >> (u[j] & 31)) & 1u)) atomic_or_noret32(tgt32 + ((uint32_t)u[j] >> 5), 1u << (u[j] & 31));
}

// Per-lane totals of a queue-only level, reduced once per workgroup.
struct SparseAcc {
  uint64_t nnew = 0, owned = 0, edges = 0;
};

// Queue-only level (single node, small frontier): the atomic OR goes straight
// into `visited`; the lane whose OR flipped the bit owns the vertex: it writes
// the distance and appends the vertex to its tier queue for the next level.
// All lanes of the wavefront must call this (the appends use ballots).
template <int K>
__device__ __forceinline__ void probe_batch_sparse(const View &v, const int32_t (&u)[K],
                                                   const bool (&ok)[K], int L, SparseAcc &acc,
                                                   int32_t *dist) {
  const int nxt = (L + 1) % kRing;
  const int lane = lane_id();
  uint64_t vis[K];
#pragma unroll
  for (int j = 0; j < K; ++j) vis[j] = ok[j] ? v.visited[(uint32_t)u[j] >> 6] : ~0ull;
  bool win[K];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const uint64_t bit = 1ull << (u[j] & 63);
    win[j] = false;
    if (!(vis[j] & bit)) win[j] = !(atomic_or64(v.visited + ((uint32_t)u[j] >> 6), bit) & bit);
  }
#pragma unroll
  for (int j = 0; j < K; ++j) {
    int64_t deg = 0, start = 0;
    int t = 0;
    bool own = false;
    if (win[j]) {
      const int64_t x = u[j];
      dist[v.old_id ? (int64_t)v.old_id[x] : x] = L + 1;
      acc.nnew += 1;
      own = x >= v.vb && x < v.ve;
      if (own) {
        const int64_t li = x - v.vb;
        start = v.rp[li];
        deg = v.rp[li + 1] - start;
        const int b = degree_bin(deg);
        t = tier_of_bin(b, v.small_bin, v.wave_bin);
        acc.owned += 1;
        acc.edges += (uint64_t)deg;
        if (v.stats && L + 1 < kMaxStatLevels) atomic_add32(&v.lvl_hist[(L + 1) * kNumBins + b], 1u);
      }
    }
    const uint64_t m0 = ballot(own && t == 0);
    const uint64_t m1 = ballot(own && t == 1);
    if (m0) {
      const int ld = __ffsll((unsigned long long)m0) - 1;
      uint32_t base = 0;
      if (lane == ld) base = atomic_add32(&v.ctl->qn[nxt][0], (uint32_t)__popcll(m0));
      base = __builtin_amdgcn_readlane(base, ld);
      if (own && t == 0) {
        v.q0[nxt][base + rank_below(m0)] = u[j];
        v.qr0[nxt][base + rank_below(m0)] = pack_row(start, deg);
      }
    }
    if (m1) {
      const int ld = __ffsll((unsigned long long)m1) - 1;
      uint32_t base = 0;
      if (lane == ld) base = atomic_add32(&v.ctl->qn[nxt][1], (uint32_t)__popcll(m1));
      base = __builtin_amdgcn_readlane(base, ld);
      if (own && t == 1) {
        v.q1[nxt][base + rank_below(m1)] = u[j];
        v.qr1[nxt][base + rank_below(m1)] = pack_row(start, deg);
      }
    }
    if (own && t == 2) {
      // one packed atomic per hub keeps slot order and chunk starts monotone
      const uint64_t nch = (uint64_t)((deg + (1ll << v.chunk_shift) - 1) >> v.chunk_shift);
      const uint64_t old = atomic_add64(&v.ctl->heavy[nxt], (1ull << kHeavyShift) | nch);
      const uint32_t slot = (uint32_t)(old >> kHeavyShift);
      v.q2[nxt][slot] = u[j];
      v.cstart[nxt][slot] = (uint32_t)(old & kChunkMask);
    }
  }
}

// ---------------------------------------------------------------------------
// Row streams of the dense expansion. A wavefront walks its share of a tier
// as a sequence of rows of up to 64 adjacency entries (one per lane; the
// entry addresses of a row are a wave-uniform base plus the lane). Rows are
// taken K at a time, and the column ids of the next K rows are requested
// before the current K rows are probed, so each wavefront keeps one batch of
// column loads in flight behind its probes.
// ---------------------------------------------------------------------------

template <int K>
struct Rows {
  int64_t base[K];  // wave-uniform
  int32_t cnt[K];   // entries in the row (0: empty)
};

template <int K>
__device__ __forceinline__ void load_rows(const View &v, const Rows<K> &r, int32_t (&u)[K]) {
  const int lane = lane_id();
#pragma unroll
  for (int j = 0; j < K; ++j) {
    u[j] = 0;
    if (lane < r.cnt[j]) u[j] = load_col(v.col, r.base[j] + lane);
  }
}

template <int K, class Src>
__device__ __forceinline__ void stream_rows(const View &v, Src &src, HotCache hot) {
  const int lane = lane_id();
  Rows<K> ra;
  int32_t ua[K];
  if (!src.fill(v, ra)) return;
  load_rows<K>(v, ra, ua);
  for (;;) {
    Rows<K> rb;
    int32_t ub[K];
    const bool more = src.fill(v, rb);
    if (more) load_rows<K>(v, rb, ub);
    bool ok[K];
#pragma unroll
    for (int j = 0; j < K; ++j) ok[j] = lane < ra.cnt[j];
    probe_batch<K>(v, ua, ok, hot);
    if (!more) break;
    ra = rb;
#pragma unroll
    for (int j = 0; j < K; ++j) ua[j] = ub[j];
  }
}

// Tier-1 rows of one wavefront: its vertices are queue entries gwave +
// k * nwaves (k < nmine); their packed rows are read 64 at a time (lane l
// holds vertex wbase + l), the next 64 requested when a window is opened.
struct WaveRows {
  const uint64_t *q;
  uint64_t gwave, nwaves;
  uint32_t nmine, k, wbase;
  uint64_t win, nwin;
  int64_t pos, end;
  uint64_t scanned;

  __device__ __forceinline__ uint64_t window(uint32_t b) const {
    const uint32_t kk = b + (uint32_t)lane_id();
    return kk < nmine ? q[gwave + (uint64_t)kk * nwaves] : 0ull;
  }
  __device__ __forceinline__ void init(const uint64_t *queue, uint64_t gw, uint64_t nw, uint32_t mine) {
    q = queue;
    gwave = gw;
    nwaves = nw;
    nmine = mine;
    k = 0;
    wbase = 0;
    win = window(0);
    nwin = window(kWave);
    pos = end = 0;
    scanned = 0;
  }
  template <int K>
  __device__ __forceinline__ bool fill(const View &, Rows<K> &r) {
    bool any = false;
#pragma unroll
    for (int j = 0; j < K; ++j) {
      while (pos >= end && k < nmine) {
        if (k - wbase == (uint32_t)kWave) {
          win = nwin;
          wbase += kWave;
          nwin = window(wbase + kWave);
        }
        const uint64_t pr = readlane64(win, (int)(k - wbase));
        pos = (int64_t)(pr >> kRowShift);
        end = pos + (int64_t)(pr & ((1ull << kRowShift) - 1));
        scanned += (uint64_t)(end - pos);
        ++k;
      }
      if (pos < end) {
        r.base[j] = pos;
        r.cnt[j] = (int32_t)min<int64_t>(kWave, end - pos);
        pos += kWave;
        any = true;
      } else {
        r.base[j] = 0;
        r.cnt[j] = 0;
      }
    }
    return any;
  }
};

// Tier-2 rows of one wavefront: the chunks [c, c_hi) of the level's chunk
// sequence (hub slot s holds chunks [cstart[s], cstart[s+1]); chunk i of a
// hub covers its entries [i << chunk_shift, (i + 1) << chunk_shift)).
struct HubRows {
  int cur;
  uint32_t n2, s;
  uint64_t nch, c, c_hi;
  int64_t pos, end;
  uint64_t scanned;

  // Opens slot s at chunk c: the entries of chunks [c, min(c_hi, next slot)).
  __device__ __forceinline__ void open(const View &v) {
    const uint64_t cs = v.cstart[cur][s];
    const uint64_t cn = s + 1 < n2 ? (uint64_t)v.cstart[cur][s + 1] : nch;
    const int64_t li = v.q2[cur][s] - v.vb;
    const int64_t rb = v.rp[li], re = v.rp[li + 1];
    const uint64_t stop = min(c_hi, cn);
    pos = uniform64(rb + ((int64_t)(c - cs) << v.chunk_shift));
    end = uniform64(min(re, rb + ((int64_t)(stop - cs) << v.chunk_shift)));
    scanned += (uint64_t)(end - pos);
    c = stop;
  }
  __device__ __forceinline__ void init(const View &v, int cur_, uint32_t n2_, uint64_t nch_, uint64_t c_lo,
                                       uint64_t c_hi_) {
    cur = cur_;
    n2 = n2_;
    nch = nch_;
    c = c_lo;
    c_hi = c_hi_;
    pos = end = 0;
    scanned = 0;
    if (c < c_hi) {
      s = wave_upper_slot(v.cstart[cur], n2, c);
      open(v);
    }
  }
  template <int K>
  __device__ __forceinline__ bool fill(const View &v, Rows<K> &r) {
    bool any = false;
#pragma unroll
    for (int j = 0; j < K; ++j) {
      while (pos >= end && c < c_hi) {
        ++s;
        open(v);
      }
      if (pos < end) {
        r.base[j] = pos;
        r.cnt[j] = (int32_t)min<int64_t>(kWave, end - pos);
        pos += kWave;
        any = true;
      } else {
        r.base[j] = 0;
        r.cnt[j] = 0;
      }
    }
    return any;
  }
};

constexpr int kUnroll = 4;       // edges per lane in flight (wavefront / workgroup tiers)
constexpr int kUnrollSmall = 8;  // edges per lane in flight (lane-group tier)

template <bool SPARSE, int K>
__device__ __forceinline__ void probe_dispatch(const View &v, const int32_t (&u)[K],
                                               const bool (&ok)[K], int L, SparseAcc &acc,
                                               HotCache hot, int32_t *dist) {
  if (SPARSE) probe_batch_sparse<K>(v, u, ok, L, acc, dist);
  else probe_batch<K>(v, u, ok, hot);
}

// One batch of K rows of a tier-0 group's dealt edges, starting at edge e0 of
// the group (edges at or beyond `total` are masked off).
template <bool SPARSE, int K>
__device__ __forceinline__ void deal_rows(const View &v, int32_t incl, int64_t rebase, int32_t e0,
                                          int32_t total, int level, SparseAcc &acc, HotCache hot,
                                          int32_t *dist) {
  const int lane = lane_id();
  int32_t u[K];
  bool ok[K];
#pragma unroll
  for (int j = 0; j < K; ++j) {
    const int32_t e = e0 + j * kWave + lane;
    int k = 0;
#pragma unroll
    for (int step = 32; step >= 1; step >>= 1)
      if (__shfl(incl, k + step - 1) <= e) k += step;
    k = min(k, kWave - 1);
    const int64_t rk = shfl64(rebase, k);
    ok[j] = e < total;
    u[j] = ok[j] ? load_col(v.col, rk + e) : 0;
  }
  probe_dispatch<SPARSE, K>(v, u, ok, level, acc, hot, dist);
}

// Expansion of level `level` by virtual block `vb_id` of `nvb` blocks. Block 0
// first clears the counters of the ring slot two levels ahead (read at level
// L-1, not written before level L+1). Every loop below runs the same number
// of iterations on all lanes of a wavefront (queue-only levels use ballots).
template <bool SPARSE, int BLOCK = kBlock, int KU = kUnroll, int KS = kUnrollSmall>
__device__ __forceinline__ void expand_phase(const View &v, int32_t *dist, int level, uint32_t vb_id,
                                             uint32_t nvb, HotCache hot = HotCache{nullptr, 0}) {
  constexpr int kWaves = BLOCK / kWave;
  __shared__ uint64_t s_acc[3][kWaves];
  const int cur = level % kRing;
  const int lane = lane_id();
  const uint32_t wave = threadIdx.x / kWave;
  const uint64_t gwave = (uint64_t)vb_id * kWaves + wave;
  const uint64_t nwaves = (uint64_t)nvb * kWaves;
  SparseAcc acc;
  uint64_t scanned = 0;  // wave-uniform: edges this wavefront scanned

  if (vb_id == 0 && threadIdx.x == 0) {
    const int r2 = (level + 2) % kRing;
    v.ctl->qn[r2][0] = 0;
    v.ctl->qn[r2][1] = 0;
    v.ctl->heavy[r2] = 0;
    v.ctl->newcnt[(level + 1) % 3] = 0;
    v.ctl->ownedcnt[(level + 1) % 3] = 0;
  }

  // Tier 2: heavy vertices cut into fixed-size edge chunks. A dense level
  // gives each wavefront a contiguous range of chunks and streams its rows
  // (a hub spans the ranges of several wavefronts, and a wavefront's range
  // crosses few hubs); a queue-only level takes one chunk at a time and finds
  // the chunk's vertex with a 64-way search of the chunk starts.
  const uint64_t hv = load_relaxed64(&v.ctl->heavy[cur]);
  const uint32_t n2 = (uint32_t)(hv >> kHeavyShift);
  const uint64_t nch = hv & kChunkMask;
  if (!SPARSE) {
    if (nch) {
      HubRows src;
      src.init(v, cur, n2, nch, gwave * nch / nwaves, (gwave + 1) * nch / nwaves);
      stream_rows<KU>(v, src, hot);
      scanned += src.scanned;
    }
  } else {
    for (uint64_t c = gwave; c < nch; c += nwaves) {
      const uint32_t s = wave_upper_slot(v.cstart[cur], n2, c);
      const int64_t li = v.q2[cur][s] - v.vb;
      const int64_t b = v.rp[li], e = v.rp[li + 1];
      const int64_t lo = b + ((int64_t)(c - v.cstart[cur][s]) << v.chunk_shift);
      const int64_t hi = min(e, lo + (1ll << v.chunk_shift));
      scanned += (uint64_t)(hi - lo);
      for (int64_t e0 = lo; e0 < hi; e0 += kWave * KU) {
        int32_t u[KU];
        bool ok[KU];
#pragma unroll
        for (int j = 0; j < KU; ++j) {
          const int64_t k = e0 + (int64_t)j * kWave + lane;
          ok[j] = k < hi;
          u[j] = ok[j] ? load_col(v.col, k) : 0;
        }
        probe_dispatch<SPARSE, KU>(v, u, ok, level, acc, hot, dist);
      }
    }
  }

  // Tier 1: one wavefront per vertex (vertex i of the queue to wavefront
  // i mod nwaves). A dense level streams the wavefront's vertices as one
  // sequence of 64-entry rows, their packed rows read 64 vertices at a time.
  const uint32_t n1 = load_relaxed32(&v.ctl->qn[cur][1]);
  if (!SPARSE) {
    if (n1 > gwave) {
      WaveRows src;
      src.init(v.qr1[cur], gwave, nwaves, (uint32_t)((n1 - gwave + nwaves - 1) / nwaves));
      stream_rows<KU>(v, src, hot);
      scanned += src.scanned;
    }
  } else {
    for (uint64_t i = gwave; i < n1; i += nwaves) {
      const uint64_t pr = v.qr1[cur][i];
      const int64_t b = (int64_t)(pr >> kRowShift), e = b + (int64_t)(pr & ((1ull << kRowShift) - 1));
      scanned += (uint64_t)(e - b);
      for (int64_t k0 = b; k0 < e; k0 += kWave * KU) {
        int32_t u[KU];
        bool ok[KU];
#pragma unroll
        for (int j = 0; j < KU; ++j) {
          const int64_t k = k0 + (int64_t)j * kWave + lane;
          ok[j] = k < e;
          u[j] = ok[j] ? load_col(v.col, k) : 0;
        }
        probe_dispatch<SPARSE, KU>(v, u, ok, level, acc, hot, dist);
      }
    }
  }

  // Tier 0: 64 vertices per wavefront, their edges dealt evenly to the lanes.
  // Tier-0 degrees are below 2^23 (small_bin <= 24), so the wavefront's edge
  // prefix sums fit in 32 bits and each search step is one 32-bit shuffle.
  // The packed rows of the wavefront's next group are requested before the
  // current group is expanded.
  const uint32_t n0 = load_relaxed32(&v.ctl->qn[cur][0]);
  uint64_t base = gwave * kWave;
  uint64_t pr_cur = base + lane < n0 ? v.qr0[cur][base + lane] : 0ull;
  for (; base < n0; base += nwaves * kWave) {
    const uint64_t nb = base + nwaves * kWave;
    const uint64_t pr_next = nb + lane < n0 ? v.qr0[cur][nb + lane] : 0ull;
    const int64_t start = (int64_t)(pr_cur >> kRowShift);
    const int32_t deg = (int32_t)(pr_cur & ((1ull << kRowShift) - 1));
    pr_cur = pr_next;
    const int32_t incl = wave_incl_scan32(deg);
    const int32_t total = __shfl(incl, kWave - 1);
    // edge e of the batch is edge (e - excl[k]) of lane k's vertex, k the first
    // lane with incl[k] > e: its column index is col[start[k] - excl[k] + e]
    const int64_t rebase = start - (int64_t)(incl - deg);
    scanned += (uint64_t)total;
    // a group whose edges fill at most a quarter (a half) of a batch, the
    // common case on the late levels of power-law graphs, takes a batch of a
    // quarter (a half) the rows: the dealing arithmetic of empty rows is not
    // issued
    if (KS >= 8 && total <= kWave * (KS / 4)) {
      deal_rows<SPARSE, KS / 4>(v, incl, rebase, 0, total, level, acc, hot, dist);
      continue;
    }
    if (KS >= 4 && total <= kWave * (KS / 2)) {
      deal_rows<SPARSE, KS / 2>(v, incl, rebase, 0, total, level, acc, hot, dist);
      continue;
    }
    for (int32_t e0 = 0; e0 < total; e0 += kWave * KS)
      deal_rows<SPARSE, KS>(v, incl, rebase, e0, total, level, acc, hot, dist);
  }

  if (!SPARSE) {
    // Work done by the dense expansion (for the bandwidth accounting): edges
    // scanned, one atomic per workgroup, and the frontier size.
    if (lane == 0) s_acc[0][wave] = scanned;
    __syncthreads();
    if (v.hubnext && hot.words) {
      // hub targets this block found: LDS copy bits not set in `visited`
      // (which no expansion changes in mark mode)
      for (uint32_t i = threadIdx.x; i < hot.words; i += BLOCK) {
        const uint64_t f = hot.lds[i] & ~v.visited[i];
        if (f) atomic_or_noret(v.hubnext + i, f);
      }
    }
    if (threadIdx.x == 0) {
      uint64_t t = 0;
      for (int w = 0; w < kWaves; ++w) t += s_acc[0][w];
      if (t) atomic_add64(&v.ctl->xedges, t);
      if (vb_id == 0) atomic_add64(&v.ctl->xfront, (uint64_t)n0 + n1 + n2);
    }
  }
  if (SPARSE) {
    // Level totals of the queue-only path: one atomic each per workgroup.
    const uint64_t a = (uint64_t)wave_sum((int64_t)acc.nnew);
    const uint64_t b = (uint64_t)wave_sum((int64_t)acc.owned);
    const uint64_t c = (uint64_t)wave_sum((int64_t)acc.edges);
    if (lane == 0) {
      s_acc[0][wave] = a;
      s_acc[1][wave] = b;
      s_acc[2][wave] = c;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      uint64_t ta = 0, tb = 0, tc = 0;
      for (int w = 0; w < kWaves; ++w) {
        ta += s_acc[0][w];
        tb += s_acc[1][w];
        tc += s_acc[2][w];
      }
      if (ta) {
        atomic_add64(&v.ctl->newcnt[level % 3], ta);
        atomic_add64(&v.ctl->reached, ta);
      }
      if (tb) atomic_add64(&v.ctl->ownedcnt[level % 3], tb);
      if (tc) atomic_add64(&v.ctl->edges, tc);
    }
  }
}

// ---------------------------------------------------------------------------
// merge (Phase 2)
// ---------------------------------------------------------------------------

// Bits of word w that fall in the owned range [vb, ve).
__device__ __forceinline__ uint64_t owned_mask(int64_t w, int64_t vb, int64_t ve) {
  const int64_t lo = w * 64, hi = lo + 64;
  if (hi <= vb || lo >= ve) return 0ull;
  uint64_t m = ~0ull;
  if (vb > lo) m &= ~0ull << (vb - lo);
  if (ve < hi) m &= ~0ull >> (hi - ve);
  return m;
}

// Four mark bytes (each 0 or 1) of a little-endian dword -> four bits.
__device__ __forceinline__ uint32_t marks_to_bits(uint32_t x) {
  return (x & 1u) | ((x >> 7) & 2u) | ((x >> 14) & 4u) | ((x >> 21) & 8u);
}

// MODE is a kMerge* constant (the ordinary merge compiles without the other
// modes' branches).
template <int MODE>
__device__ __forceinline__ void merge_phase(const View &v, int32_t *dist, const MergeArgs &a,
                                            uint32_t vb_id, uint32_t nvb) {
  __shared__ uint32_t s_cnt[kWavesPerBlock][3];
  __shared__ uint64_t s_chunks[kWavesPerBlock];
  __shared__ uint32_t s_base[3];
  __shared__ uint64_t s_cbase;
  __shared__ uint32_t s_hist[kNumBins];
  __shared__ uint64_t s_red[2][kWavesPerBlock];

  const int L = a.level;
  const int nxt = (L + 1) % kRing;
  const int lane = lane_id();
  const int wave = threadIdx.x / kWave;
  const int32_t dnew = L + 1;
  const int cs = v.chunk_shift;

  if (v.stats) {
    for (int b = threadIdx.x; b < kNumBins; b += kBlock) s_hist[b] = 0;
    __syncthreads();
  }

  uint64_t my_new = 0, my_edges = 0, my_owned = 0;
  const int64_t group = (int64_t)kBlock;  // words per workgroup step
  for (int64_t g0 = (int64_t)vb_id * group; g0 < v.words; g0 += (int64_t)nvb * group) {
    const int64_t wbase = g0 + wave * kWave;  // first word of this wavefront
    const int64_t w = wbase + lane;
    uint64_t nw = 0, om = 0;
    if (MODE == kMergeQueuesFromFront) {
      if (w < v.words) {
        const uint64_t tail = (w == v.words - 1 && (v.n & 63)) ? ~0ull >> (64 - (v.n & 63)) : ~0ull;
        nw = v.front[w] & tail;
        om = nw & owned_mask(w, v.vb, v.ve);
      }
    } else if (w < v.words && v.mark) {
      // byte marks of the word's 64 vertices (set only for vertices that
      // were unvisited): fold them into a bit mask and clear them
      uint4 *mp = reinterpret_cast<uint4 *>(v.mark + (size_t)w * 64);
      uint4 q[4];
#pragma unroll
      for (int k = 0; k < 4; ++k) q[k] = mp[k];
      uint64_t mk = 0;
#pragma unroll
      for (int k = 0; k < 4; ++k)
        mk |= (uint64_t)(marks_to_bits(q[k].x) | (marks_to_bits(q[k].y) << 4) |
                         (marks_to_bits(q[k].z) << 8) | (marks_to_bits(q[k].w) << 12))
              << (16 * k);
      if (w < v.hub_words) {
        const uint64_t h = v.hubnext[w];
        if (h) {
          v.hubnext[w] = 0ull;
          mk |= h;
        }
      }
      if (mk) {
#pragma unroll
        for (int k = 0; k < 4; ++k)
          if (q[k].x | q[k].y | q[k].z | q[k].w) mp[k] = make_uint4(0u, 0u, 0u, 0u);
        const uint64_t vis = v.visited[w];
        nw = mk & ~vis;
        if (nw) v.visited[w] = vis | nw;
      }
      om = nw & owned_mask(w, v.vb, v.ve);
    } else if (w < v.words && v.into_vis) {
      // the expansion ORed into `visited`; `next` holds visited as it was at
      // the level's start, and becomes the current visited
      const uint64_t vis = v.visited[w], prev = v.next[w];
      nw = vis & ~prev;
      if (nw) v.next[w] = vis;
      om = nw & owned_mask(w, v.vb, v.ve);
    } else if (w < v.words) {
      const uint64_t nx = v.next[w];
      uint64_t m = nx;
      for (int j = 0; j < a.k; ++j) m |= a.inc[j][w];
      const uint64_t vis = v.visited[w];
      nw = m & ~vis;
      if (nw) v.visited[w] = vis | nw;
      if (a.keep_next) {
        if (m != nx) v.next[w] = m;
      } else if (nx) {
        v.next[w] = 0ull;
      }
      const uint64_t tail = (w == v.words - 1 && (v.n & 63)) ? ~0ull >> (64 - (v.n & 63)) : ~0ull;
      nw &= tail;
      // the next level's frontier bitmap: the level's whole global queue
      // (every vertex found in the level, also those merged by earlier
      // keep_next calls of a multi-round exchange)
      if (v.front && !a.keep_next) v.front[w] = m & tail;
      om = nw & owned_mask(w, v.vb, v.ve);
    }
    if (MODE != kMergeQueuesFromFront) my_new += (uint64_t)__popcll(nw);
    // A workgroup step without new vertices (the common case on sparse
    // levels) has no distances, queue entries or counters to write.
    if (!__syncthreads_or(nw != 0ull)) continue;

    // Pass 1: distances of new vertices; degree tier of owned new vertices.
    // Words are taken eight at a time (lanes = the 64 bits of a word) so the
    // row-offset loads of eight words are in flight together.
    uint64_t t1m = 0, t2m = 0;
    uint64_t chunks = 0;  // wave-uniform
    constexpr bool write_dist = MODE != kMergeQueuesFromFront;
    constexpr bool tiers = MODE != kMergeNoQueues;
    uint64_t act = ballot(nw != 0);
    if (ballot(om != 0) == 0ull) {
      // no owned new vertex in this wavefront's words (a node's share covers
      // a fraction of the bitmap): distances only, one word per step
      if (!write_dist) act = 0;
      while (act) {
        const int j = __ffsll((unsigned long long)act) - 1;
        act &= act - 1;
        const uint64_t wj = readlane64(nw, j);
        if ((wj >> lane) & 1ull) {
          const int64_t vtx = (wbase + j) * 64 + lane;
          dist[v.old_id ? (int64_t)v.old_id[vtx] : vtx] = dnew;
        }
      }
    }
    while (act) {
      constexpr int kW = 8;
      int js[kW];
      int cnt = 0;
#pragma unroll
      for (int q = 0; q < kW; ++q) {
        js[q] = act ? __ffsll((unsigned long long)act) - 1 : 0;
        if (act) { act &= act - 1; ++cnt; }
      }
      bool own[kW], isnew[kW];
      int64_t vtx[kW], r0[kW], r1[kW];
#pragma unroll
      for (int q = 0; q < kW; ++q) {
        const uint64_t wj = q < cnt ? readlane64(nw, js[q]) : 0ull;
        const uint64_t oj = q < cnt ? readlane64(om, js[q]) : 0ull;
        vtx[q] = (wbase + js[q]) * 64 + lane;
        isnew[q] = (wj >> lane) & 1ull;
        own[q] = (oj >> lane) & 1ull;
      }
      // Every load of the batch is issued before the first store that
      // depends on one: loads are unconditional, on addresses clamped into
      // the arrays (this loop runs only when some word of the wavefront has
      // an owned new vertex, so the owned range is not empty), so the
      // wavefront waits for memory once per batch rather than once per word.
      int32_t oid[kW];
      if (v.old_id && write_dist) {
#pragma unroll
        for (int q = 0; q < kW; ++q) oid[q] = v.old_id[min(vtx[q], v.n - 1)];
      }
      const int64_t nloc = v.ve - v.vb;
      if (tiers) {
#pragma unroll
        for (int q = 0; q < kW; ++q) {
          const int64_t li = min(max(vtx[q] - v.vb, (int64_t)0), nloc - 1);
          r0[q] = v.rp[li];
          r1[q] = v.rp[li + 1];
        }
      }
      if (write_dist) {
#pragma unroll
        for (int q = 0; q < kW; ++q)
          if (isnew[q]) dist[v.old_id ? (int64_t)oid[q] : vtx[q]] = dnew;
      }
      if (!tiers) continue;
#pragma unroll
      for (int q = 0; q < kW; ++q) {
        if (q >= cnt) break;
        int t = 0;
        const int64_t deg = r1[q] - r0[q];
        if (own[q]) {
          const int b = degree_bin(deg);
          t = tier_of_bin(b, v.small_bin, v.wave_bin);
          if (MODE == kMergeFull) {
            my_edges += (uint64_t)deg;
            if (v.stats) atomicAdd(&s_hist[b], 1u);
          }
        }
        const uint64_t m1 = ballot(own[q] && t == 1);
        const uint64_t m2 = ballot(own[q] && t == 2);
        if (lane == js[q]) { t1m = m1; t2m = m2; }
        if (m2) {
          const uint64_t nc = (own[q] && t == 2) ? (uint64_t)((deg + (1ll << cs) - 1) >> cs) : 0ull;
          chunks += (uint64_t)wave_sum((int64_t)nc);
        }
      }
    }
    if (!tiers) {
      // no queues: the owned new vertices are only counted
      my_owned += (uint64_t)__popcll(om);
      continue;
    }
    const uint32_t c0 = wave_sum_u32((uint32_t)__popcll(om & ~t1m & ~t2m));
    const uint32_t c1 = wave_sum_u32((uint32_t)__popcll(t1m));
    const uint32_t c2 = wave_sum_u32((uint32_t)__popcll(t2m));
    if (MODE == kMergeFull) my_owned += (lane == 0) ? (uint64_t)(c0 + c1 + c2) : 0ull;

    // Workgroup aggregation: one atomic per tier per workgroup step.
    if (lane == 0) {
      s_cnt[wave][0] = c0;
      s_cnt[wave][1] = c1;
      s_cnt[wave][2] = c2;
      s_chunks[wave] = chunks;
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t t0 = 0, t1 = 0, t2 = 0;
      uint64_t ch = 0;
      for (int x = 0; x < kWavesPerBlock; ++x) {
        t0 += s_cnt[x][0];
        t1 += s_cnt[x][1];
        t2 += s_cnt[x][2];
        ch += s_chunks[x];
      }
      s_base[0] = t0 ? atomic_add32(&v.ctl->qn[nxt][0], t0) : 0u;
      s_base[1] = t1 ? atomic_add32(&v.ctl->qn[nxt][1], t1) : 0u;
      if (t2) {
        const uint64_t old =
            atomic_add64(&v.ctl->heavy[nxt], ((uint64_t)t2 << kHeavyShift) | ch);
        s_base[2] = (uint32_t)(old >> kHeavyShift);
        s_cbase = old & kChunkMask;
      } else {
        s_base[2] = 0;
        s_cbase = 0;
      }
    }
    __syncthreads();
    uint32_t b0 = s_base[0], b1 = s_base[1], b2 = s_base[2];
    uint64_t cb = s_cbase;
    for (int x = 0; x < wave; ++x) {
      b0 += s_cnt[x][0];
      b1 += s_cnt[x][1];
      b2 += s_cnt[x][2];
      cb += s_chunks[x];
    }

    // Pass 2: write owned new vertices into the level L+1 tier queues, with
    // the packed rows of tier-0/1 entries. Words are taken eight at a time so
    // their row-offset loads (cache hits after pass 1) are in flight together.
    act = ballot(om != 0);
    while (act) {
      constexpr int kW = 8;
      int js[kW];
      int cnt = 0;
#pragma unroll
      for (int q = 0; q < kW; ++q) {
        js[q] = act ? __ffsll((unsigned long long)act) - 1 : 0;
        if (act) { act &= act - 1; ++cnt; }
      }
      int64_t r0[kW], r1[kW];
#pragma unroll
      for (int q = 0; q < kW; ++q) {
        r0[q] = r1[q] = 0;
        const uint64_t oj = q < cnt ? readlane64(om, js[q]) : 0ull;
        if ((oj >> lane) & 1ull) {
          const int64_t li = (wbase + js[q]) * 64 + lane - v.vb;
          r0[q] = v.rp[li];
          r1[q] = v.rp[li + 1];
        }
      }
#pragma unroll
      for (int q = 0; q < kW; ++q) {
        if (q >= cnt) break;
        const int j = js[q];
        const uint64_t oj = readlane64(om, j);
        const uint64_t m1 = readlane64(t1m, j);
        const uint64_t m2 = readlane64(t2m, j);
        const uint64_t m0 = oj & ~m1 & ~m2;
        const int32_t vtx = (int32_t)((wbase + j) * 64 + lane);
        const int64_t deg = r1[q] - r0[q];
        if ((m0 >> lane) & 1ull) {
          v.q0[nxt][b0 + rank_below(m0)] = vtx;
          v.qr0[nxt][b0 + rank_below(m0)] = pack_row(r0[q], deg);
        } else if ((m1 >> lane) & 1ull) {
          v.q1[nxt][b1 + rank_below(m1)] = vtx;
          v.qr1[nxt][b1 + rank_below(m1)] = pack_row(r0[q], deg);
        }
        b0 += (uint32_t)__popcll(m0);
        b1 += (uint32_t)__popcll(m1);
        if (m2) {
          const bool mine = (m2 >> lane) & 1ull;
          const int64_t nc = mine ? (deg + (1ll << cs) - 1) >> cs : 0;
          const int64_t incl = wave_incl_scan(nc);
          if (mine) {
            const uint32_t slot = b2 + rank_below(m2);
            v.q2[nxt][slot] = vtx;
            v.cstart[nxt][slot] = (uint32_t)(cb + (uint64_t)(incl - nc));
          }
          b2 += (uint32_t)__popcll(m2);
          cb += (uint64_t)shfl64(incl, kWave - 1);
        }
      }
    }
    __syncthreads();  // s_cnt / s_base reuse
  }

  // Level totals: one atomic per workgroup.
  const uint64_t wn = (uint64_t)wave_sum((int64_t)my_new);
  const uint64_t we = (uint64_t)wave_sum((int64_t)my_edges);
  if (lane == 0) {
    s_red[0][wave] = wn;
    s_red[1][wave] = we;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t tn = 0, te = 0;
    for (int x = 0; x < kWavesPerBlock; ++x) { tn += s_red[0][x]; te += s_red[1][x]; }
    if (tn) {
      atomic_add64(&v.ctl->newcnt[L % 3], tn);
      atomic_add64(&v.ctl->reached, tn);
    }
    if (te) atomic_add64(&v.ctl->edges, te);
  }
  const uint64_t wo = (uint64_t)wave_sum((int64_t)my_owned);
  __syncthreads();
  if (lane == 0) s_red[0][wave] = wo;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t to = 0;
    for (int x = 0; x < kWavesPerBlock; ++x) to += s_red[0][x];
    if (to) atomic_add64(&v.ctl->ownedcnt[L % 3], to);
  }
  if (v.stats && L + 1 < kMaxStatLevels) {
    __syncthreads();
    for (int b = threadIdx.x; b < kNumBins; b += kBlock)
      if (s_hist[b]) atomic_add32(&v.lvl_hist[(L + 1) * kNumBins + b], s_hist[b]);
  }
}

// ---------------------------------------------------------------------------
// kernels
// ---------------------------------------------------------------------------

// Loads visited words [0, words) into this block's LDS copy.
template <int BLOCK = kBlock>
__device__ __forceinline__ HotCache load_hot(const View &v, uint64_t *lds, uint32_t words) {
  words = (uint32_t)min<int64_t>(words, v.words);
  for (uint32_t i = threadIdx.x; i < words; i += BLOCK) lds[i] = v.visited[i];
  __syncthreads();
  return HotCache{lds, words};
}

// hot_words > 0: the block keeps the first hot_words visited words in LDS
// (the launch must provide hot_words * 8 bytes of dynamic LDS).
// Queue-only level of the host-driven loop (its own kernel, so the dense
// expansion keeps a small register budget).
__global__ void __launch_bounds__(kBlock) k_expand_q(View v, int level) {
  expand_phase<true>(v, v.dist, level, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(kBlock) k_expand(View v, int level, uint32_t hot_words) {
  extern __shared__ uint64_t s_hot[];
  if (hot_words)
    expand_phase<false>(v, v.dist, level, blockIdx.x, gridDim.x, load_hot(v, s_hot, hot_words));
  else
    expand_phase<false>(v, v.dist, level, blockIdx.x, gridDim.x);
}

// Wide variant for large LDS copies: one 1024-thread workgroup per CU shares
// up to ~144 KB of hub bits (on a degree-relabelled R-MAT graph the first 16K
// words hold the targets of most edges), instead of four 256-thread blocks
// each holding a small copy.
// One block per CU leaves each wavefront up to 128 VGPRs: it keeps twice the
// edges per lane in flight.
__global__ void __launch_bounds__(kWideBlock) k_expand_wide(View v, int level, uint32_t hot_words) {
  extern __shared__ uint64_t s_hot[];
  expand_phase<false, kWideBlock, 2 * kUnroll, 2 * kUnrollSmall>(
      v, v.dist, level, blockIdx.x, gridDim.x, load_hot<kWideBlock>(v, s_hot, hot_words));
}

template <int MODE>
__global__ void __launch_bounds__(kBlock) k_merge(View v, MergeArgs a) {
  merge_phase<MODE>(v, v.dist, a, blockIdx.x, gridDim.x);
}

// ---------------------------------------------------------------------------
// bottom-up step (direction-optimizing traversal, single node, whole graph)
// ---------------------------------------------------------------------------

constexpr int kBuUnroll = 4;  // adjacency entries per lane in flight

// Level L bottom-up: one wavefront per 64-vertex word of `visited` within
// the owned range, one lane per unvisited owned vertex. A lane scans its
// vertex's adjacency kBuUnroll entries at a time until a neighbour is set in
// `front`, the level-L frontier bitmap over all n vertices (on a share it is
// the merged result of the previous level's exchange); the vertices found in
// a word go to `next` with one store (each word belongs to one wavefront),
// and the ordinary merge then finishes the level (distances, visited, queues
// and the next frontier bitmap). The first frontier words are copied to LDS:
// on a relabelled graph every adjacency list starts with the hubs, so the
// first probes of most lanes are LDS reads.
// count_edges: also add the degrees of the vertices found to the traversal's
// edge count (for a merge that leaves the tier queues unwritten).
__global__ void __launch_bounds__(kBlock) k_bottom_up(View v, int level, uint32_t hot_words,
                                                      const uint64_t *front, int count_edges) {
  extern __shared__ uint64_t s_hot[];
  __shared__ uint64_t s_acc[3][kWavesPerBlock];
  const int lane = lane_id();
  const uint32_t wave = threadIdx.x / kWave;
  const uint64_t gwave = (uint64_t)blockIdx.x * kWavesPerBlock + wave;
  const uint64_t nwaves = (uint64_t)gridDim.x * kWavesPerBlock;
  if (blockIdx.x == 0 && threadIdx.x == 0) {  // the ring bookkeeping of an expansion
    const int r2 = (level + 2) % kRing;
    v.ctl->qn[r2][0] = 0;
    v.ctl->qn[r2][1] = 0;
    v.ctl->heavy[r2] = 0;
    v.ctl->newcnt[(level + 1) % 3] = 0;
    v.ctl->ownedcnt[(level + 1) % 3] = 0;
  }
  const uint32_t hw = (uint32_t)min<int64_t>(hot_words, v.words);
  for (uint32_t i = threadIdx.x; i < hw; i += kBlock) s_hot[i] = front[i];
  __syncthreads();
  uint64_t examined = 0, verts = 0, found_edges = 0;
  // vertices without an edge are never found: a relabelled graph keeps them
  // after live_end, and their words are skipped
  const uint64_t wb = (uint64_t)(v.vb >> 6), we = (uint64_t)((min(v.ve, v.live_end) + 63) >> 6);
  for (uint64_t w = wb + gwave; w < we; w += nwaves) {
    const uint64_t vis = v.visited[w];
    if (vis == ~0ull) continue;
    const int64_t x = (int64_t)w * 64 + lane;
    bool todo = x >= v.vb && x < v.ve && !((vis >> lane) & 1ull);
    int64_t k = 0, e = 0;
    if (todo) {
      k = v.rp[x - v.vb];
      e = v.rp[x - v.vb + 1];
      todo = k < e;
    }
    const int64_t k0 = k;
    bool found = false;
    while (ballot(todo && !found && k < e)) {
      if (todo && !found && k < e) {
        int32_t u[kBuUnroll];
#pragma unroll
        for (int j = 0; j < kBuUnroll; ++j) u[j] = (k + j < e) ? v.col[k + j] : -1;
#pragma unroll
        for (int j = 0; j < kBuUnroll; ++j) {
          if (u[j] >= 0) {
            const uint32_t uw = (uint32_t)u[j] >> 6;
            // address-space-qualified reads stay LDS and global instructions
            uint64_t fw;
            if (uw < hw) fw = s_hot[uw];
            else fw = ((const __attribute__((address_space(1))) uint64_t *)front)[uw];
            if ((fw >> (u[j] & 63)) & 1ull) found = true;
          }
        }
        k += kBuUnroll;
      }
    }
    if (todo) {
      examined += (uint64_t)(min(k, e) - k0);
      verts += 1;
      if (found) found_edges += (uint64_t)(e - k0);
    }
    const uint64_t fm = ballot(found);
    if (lane == 0 && fm) v.next[w] = fm;
  }
  const uint64_t te = (uint64_t)wave_sum((int64_t)examined);
  const uint64_t tv = (uint64_t)wave_sum((int64_t)verts);
  const uint64_t tf = (uint64_t)wave_sum((int64_t)found_edges);
  if (lane == 0) {
    s_acc[0][wave] = te;
    s_acc[1][wave] = tv;
    s_acc[2][wave] = tf;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t a = 0, b = 0, f = 0;
    for (int i = 0; i < kWavesPerBlock; ++i) {
      a += s_acc[0][i];
      b += s_acc[1][i];
      f += s_acc[2][i];
    }
    if (a) atomic_add64(&v.ctl->buedges, a);
    if (b) atomic_add64(&v.ctl->buverts, b);
    if (f && count_edges) atomic_add64(&v.ctl->edges, f);
  }
}

// Frontier bitmap of level L from its tier queues (after a queue-only level,
// which leaves the frontier in queues only): clear, then set every entry.
__global__ void __launch_bounds__(kBlock) k_front_zero(View v) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t w = tid; w < v.words; w += (int64_t)gridDim.x * blockDim.x) v.front[w] = 0ull;
}

__global__ void __launch_bounds__(kBlock) k_front_scatter(View v, int level) {
  const int cur = level % kRing;
  const uint64_t n0 = load_relaxed32(&v.ctl->qn[cur][0]);
  const uint64_t n1 = load_relaxed32(&v.ctl->qn[cur][1]);
  const uint64_t n2 = load_relaxed64(&v.ctl->heavy[cur]) >> kHeavyShift;
  const uint64_t tid = (uint64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const uint64_t stride = (uint64_t)gridDim.x * blockDim.x;
  for (uint64_t i = tid; i < n0 + n1 + n2; i += stride) {
    const int32_t x = i < n0 ? v.q0[cur][i] : (i < n0 + n1 ? v.q1[cur][i - n0] : v.q2[cur][i - n0 - n1]);
    atomic_or_noret(v.front + (x >> 6), 1ull << (x & 63));
  }
}

// ---------------------------------------------------------------------------
// graph-launched level loop: the same phases as launches whose level comes
// from the control block, so a fixed sequence can be captured in a hipGraph
// and replayed until the traversal is done
// ---------------------------------------------------------------------------

__device__ __forceinline__ bool level_is_sparse(const View &v, int L) {
  const int cur = L % kRing;
  const uint64_t fsize = (uint64_t)load_relaxed32(&v.ctl->qn[cur][0]) +
                         load_relaxed32(&v.ctl->qn[cur][1]) +
                         (load_relaxed64(&v.ctl->heavy[cur]) >> kHeavyShift);
  return v.sparse_div > 0 && fsize * (uint64_t)v.sparse_div < (uint64_t)v.words;
}

// The caller's distance array of the running traversal comes from the
// control block (the captured launches outlive any one call's pointer).
template <int BLOCK>
__device__ __forceinline__ void expand_g_body(const View &v, uint32_t hot_words) {
  extern __shared__ uint64_t s_hot[];
  if (load_relaxed_i32(&v.ctl->gdone)) return;
  const int L = load_relaxed_i32(&v.ctl->glevel);
  int32_t *dist = v.ctl->gdist;
  if (level_is_sparse(v, L)) {
    expand_phase<true, BLOCK>(v, dist, L, blockIdx.x, gridDim.x);
    return;
  }
  // the LDS copy of the hub bits pays off only when the frontier's edges
  // are at least the vertex count (the host-driven loop's rule)
  const uint64_t fedges = load_relaxed64(&v.ctl->gedges[1]) - load_relaxed64(&v.ctl->gedges[0]);
  // the 1024-thread variant runs one block per CU, which leaves each
  // wavefront the registers for twice the edges per lane in flight
  constexpr int KU = BLOCK == kWideBlock ? 2 * kUnroll : kUnroll;
  constexpr int KS = BLOCK == kWideBlock ? 2 * kUnrollSmall : kUnrollSmall;
  if (hot_words && fedges >= (uint64_t)v.n)
    expand_phase<false, BLOCK, KU, KS>(v, dist, L, blockIdx.x, gridDim.x,
                                       load_hot<BLOCK>(v, s_hot, hot_words));
  else
    expand_phase<false, BLOCK, KU, KS>(v, dist, L, blockIdx.x, gridDim.x);
}

__global__ void __launch_bounds__(kBlock) k_expand_g(View v, uint32_t hot_words) {
  expand_g_body<kBlock>(v, hot_words);
}

__global__ void __launch_bounds__(kWideBlock) k_expand_gw(View v, uint32_t hot_words) {
  expand_g_body<kWideBlock>(v, hot_words);
}

__global__ void __launch_bounds__(kBlock) k_merge_g(View v) {
  if (load_relaxed_i32(&v.ctl->gdone)) return;
  const int L = load_relaxed_i32(&v.ctl->glevel);
  if (level_is_sparse(v, L)) return;  // a queue-only level has nothing to merge
  MergeArgs a;
  a.k = 0;
  a.keep_next = 0;
  a.level = L;
  a.mode = kMergeFull;
  merge_phase<kMergeFull>(v, v.ctl->gdist, a, blockIdx.x, gridDim.x);
}

// One thread: termination test and level advance; clears the histogram row
// written two levels ahead.
__global__ void k_advance_g(View v, int max_levels) {
  if (threadIdx.x != 0 || load_relaxed_i32(&v.ctl->gdone)) return;
  const int L = v.ctl->glevel;
  const uint64_t nn = v.ctl->newcnt[L % 3];
  v.ctl->gedges[0] = v.ctl->gedges[1];
  v.ctl->gedges[1] = v.ctl->edges;
  if (v.stats && L + 1 < kMaxStatLevels) v.lvl_frontier[L + 1] = (int64_t)v.ctl->ownedcnt[L % 3];
  if (v.stats && L + 2 < kMaxStatLevels)
    for (int b = 0; b < kNumBins; ++b) v.lvl_hist[(L + 2) * kNumBins + b] = 0;
  if (nn == 0 || L + 1 >= max_levels) {
    v.ctl->gdone = 1;
    v.ctl->levels = L + 1;
    if (nn != 0) v.ctl->err |= 2;
  } else {
    v.ctl->glevel = L + 1;
  }
}

hipError_t enqueue_graph_levels(const View &v, int levels, int max_levels, int expand_grid,
                                int merge_grid, uint32_t hot_words, hipStream_t s, hipEvent_t (*ev)[3]) {
  for (int i = 0; i < levels; ++i) {
    hipError_t e = ev ? hipEventRecord(ev[i][0], s) : hipSuccess;
    if (e != hipSuccess) return e;
    if (hot_words > kNarrowHotMax)
      hipLaunchKernelGGL(k_expand_gw, dim3(expand_grid), dim3(kWideBlock), hot_words * 8, s, v, hot_words);
    else
      hipLaunchKernelGGL(k_expand_g, dim3(expand_grid), dim3(kBlock), hot_words * 8, s, v, hot_words);
    e = ev ? hipEventRecord(ev[i][1], s) : hipSuccess;
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_merge_g, dim3(merge_grid), dim3(kBlock), 0, s, v);
    e = ev ? hipEventRecord(ev[i][2], s) : hipSuccess;
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL(k_advance_g, dim3(1), dim3(64), 0, s, v, max_levels);
  }
  return hipGetLastError();
}

// Clears the stats row of a level before its merge (host-driven loop).
__global__ void k_clear_stats_row(View v, int level) {
  if (level < kMaxStatLevels)
    for (int b = threadIdx.x; b < kNumBins; b += blockDim.x) v.lvl_hist[level * kNumBins + b] = 0;
}

// Whole traversal in one cooperative launch: expand, barrier, merge, barrier,
// until a level finds no new vertex. Every block runs the same number of
// barriers; the loop also stops if a barrier tripped its spin limit.
__device__ __forceinline__ void persistent_body(const View &v, int max_levels) {
  const uint32_t nb = gridDim.x;
  MergeArgs a;
  a.k = 0;
  a.keep_next = 0;
  a.mode = kMergeFull;
  int L = 0;
  for (;; ++L) {
    // Row L+2 of the histogram is cleared a level ahead: rows L+1 are
    // written during this level (by the merge, or by the queue-only expansion).
    if (v.stats && L + 2 < kMaxStatLevels) {
      if (blockIdx.x == 0)
        for (int b = threadIdx.x; b < kNumBins; b += blockDim.x)
          v.lvl_hist[(L + 2) * kNumBins + b] = 0;
    }
    // Queue-only level when the frontier is small next to the bitmap sweep
    // (every block reads the same final counters).
    const int cur = L % kRing;
    const uint64_t fsize = (uint64_t)load_relaxed32(&v.ctl->qn[cur][0]) +
                           load_relaxed32(&v.ctl->qn[cur][1]) +
                           (load_relaxed64(&v.ctl->heavy[cur]) >> kHeavyShift);
    const bool sparse = v.sparse_div > 0 && fsize * (uint64_t)v.sparse_div < (uint64_t)v.words;
    if (sparse) {
      expand_phase<true>(v, v.dist, L, blockIdx.x, nb);
      grid_barrier(&v.ctl->bar, nb);
    } else {
      expand_phase<false>(v, v.dist, L, blockIdx.x, nb);
      grid_barrier(&v.ctl->bar, nb);
      a.level = L;
      merge_phase<kMergeFull>(v, v.dist, a, blockIdx.x, nb);
      grid_barrier(&v.ctl->bar, nb);
    }
    const uint64_t nn = load_relaxed64(&v.ctl->newcnt[L % 3]);
    if (v.stats && blockIdx.x == 0 && threadIdx.x == 0 && L + 1 < kMaxStatLevels)
      v.lvl_frontier[L + 1] = (int64_t)load_relaxed64(&v.ctl->ownedcnt[L % 3]);
    const int tripped = __hip_atomic_load(&v.ctl->bar.tripped, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
    if (nn == 0 || tripped || L + 1 >= max_levels) break;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    v.ctl->levels = L + 1;
    if (L + 1 >= max_levels) v.ctl->err |= 2;
  }
}

// Two register budgets of the same loop: the default, and one capped at 64
// VGPRs so 8 wavefronts fit per SIMD (more latency hiding in the expansion,
// at the price of a few spills in the merge).
__global__ void __launch_bounds__(kBlock) k_persistent(View v, int max_levels) {
  persistent_body(v, max_levels);
}
__global__ void __launch_bounds__(kBlock) __attribute__((amdgpu_waves_per_eu(8, 8)))
k_persistent_occ8(View v, int max_levels) {
  persistent_body(v, max_levels);
}

// Canonical parents for the owned range: one wavefront per owned vertex takes
// the smallest neighbour one level closer to the root. Non-owned reached
// vertices get -2, unreached -1, the root itself.
// x runs over traversal ids; parents and distances are in caller ids, and the
// minimum is taken over caller ids.
__global__ void __launch_bounds__(kBlock) k_parent(View v, int32_t *parent, int64_t src) {
  const int lane = lane_id();
  const int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / kWave;
  for (int64_t x = gw; x < v.n; x += nw) {
    const int64_t xc = v.old_id ? (int64_t)v.old_id[x] : x;
    const int32_t d = v.dist[xc];
    int32_t out;
    if (d < 0) out = -1;
    else if (xc == src) out = (int32_t)xc;
    else if (x < v.vb || x >= v.ve) out = -2;
    else {
      const int64_t li = x - v.vb;
      int32_t best = 0x7fffffff;
      for (int64_t e = v.rp[li] + lane; e < v.rp[li + 1]; e += kWave) {
        const int32_t u = v.col[e];
        const int32_t uc = v.old_id ? v.old_id[u] : u;
        if (uc < best && v.dist[uc] == d - 1) best = uc;
      }
#pragma unroll
      for (int s = 32; s >= 1; s >>= 1) best = min(best, __shfl_xor(best, s));
      out = best;
    }
    if (lane == 0) parent[xc] = out;
  }
}

}  // namespace bfsk

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------

namespace bfsk {

hipError_t launch_reset(const View &v, int64_t src, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_reset, dim3(grid), dim3(kBlock), 0, s, v, src);
  return hipGetLastError();
}

// hot_words == kQueueOnly runs a queue-only level (no LDS copy).
hipError_t launch_expand(const View &v, int level, int grid, uint32_t hot_words, hipStream_t s) {
  if (hot_words == kQueueOnly)
    hipLaunchKernelGGL(k_expand_q, dim3(grid), dim3(kBlock), 0, s, v, level);
  else if (hot_words > kNarrowHotMax)
    hipLaunchKernelGGL(k_expand_wide, dim3(grid), dim3(kWideBlock), hot_words * 8, s, v, level, hot_words);
  else
    hipLaunchKernelGGL(k_expand, dim3(grid), dim3(kBlock), hot_words * 8, s, v, level, hot_words);
  return hipGetLastError();
}

hipError_t launch_merge(const View &v, const MergeArgs &a, int grid, hipStream_t s) {
  switch (a.mode) {
    case kMergeNoQueues: hipLaunchKernelGGL(k_merge<kMergeNoQueues>, dim3(grid), dim3(kBlock), 0, s, v, a); break;
    case kMergeQueuesFromFront:
      hipLaunchKernelGGL(k_merge<kMergeQueuesFromFront>, dim3(grid), dim3(kBlock), 0, s, v, a);
      break;
    default: hipLaunchKernelGGL(k_merge<kMergeFull>, dim3(grid), dim3(kBlock), 0, s, v, a); break;
  }
  return hipGetLastError();
}

hipError_t launch_clear_stats_row(const View &v, int level, hipStream_t s) {
  hipLaunchKernelGGL(k_clear_stats_row, dim3(1), dim3(64), 0, s, v, level);
  return hipGetLastError();
}

hipError_t launch_parent(const View &v, int32_t *parent, int64_t src, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_parent, dim3(grid), dim3(kBlock), 0, s, v, parent, src);
  return hipGetLastError();
}

hipError_t launch_bottom_up(const View &v, int level, int grid, uint32_t hot_words, const uint64_t *front,
                            int count_edges, hipStream_t s) {
  hipLaunchKernelGGL(k_bottom_up, dim3(grid), dim3(kBlock), (size_t)hot_words * 8, s, v, level, hot_words,
                     front, count_edges);
  return hipGetLastError();
}

hipError_t launch_front_from_queues(const View &v, int level, int grid, hipStream_t s) {
  hipLaunchKernelGGL(k_front_zero, dim3(grid), dim3(kBlock), 0, s, v);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_front_scatter, dim3(grid), dim3(kBlock), 0, s, v, level);
  return hipGetLastError();
}

int bottom_up_blocks_per_cu(uint32_t hot_words) {
  int nb = 0;
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_bottom_up, kBlock, (size_t)hot_words * 8) ==
                 hipSuccess
             ? nb
             : 0;
}

// Co-resident blocks per CU of the per-phase expansion kernel that an LDS
// copy of hot_words visited words selects (the wide kernel above
// kNarrowHotMax words). Raises the wide kernels' dynamic-LDS limit first.
int expand_blocks_per_cu(uint32_t hot_words) {
  const size_t lds = (size_t)hot_words * 8;
  int nb = 0;
  if (hot_words > kNarrowHotMax) {
    (void)hipFuncSetAttribute((const void *)k_expand_wide,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    (void)hipFuncSetAttribute((const void *)k_expand_gw,
                              hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    return hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_expand_wide, kWideBlock, lds) == hipSuccess
               ? nb
               : 0;
  }
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_expand, kBlock, lds) == hipSuccess ? nb : 0;
}

// Co-resident blocks per CU for the persistent kernel (variant 0 or 1).
int persistent_blocks_per_cu(int variant) {
  int nb = 0;
  hipError_t e = variant ? hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persistent_occ8, kBlock, 0)
                         : hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_persistent, kBlock, 0);
  return e == hipSuccess ? nb : 0;
}

hipError_t launch_persistent(const View &v, int max_levels, int grid, int variant, hipStream_t s) {
  View vv = v;
  int ml = max_levels;
  void *args[] = {&vv, &ml};
  const void *fn = variant ? (const void *)k_persistent_occ8 : (const void *)k_persistent;
  return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(kBlock), args, 0, s);
}

}  // namespace bfsk
