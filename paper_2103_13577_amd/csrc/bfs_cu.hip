// Whole traversal of a small graph by one workgroup, its bitmaps in LDS.
//
// For graphs whose visited and next bitmaps fit in one workgroup's LDS (n up
// to about half a million vertices on gfx950), a traversal is bound by
// per-level latency, not by bandwidth: the grid barriers of a cooperative
// launch (each one a device-scope release and acquire on every block) or a
// launch per phase cost more than the level's work. Here one 1024-thread
// workgroup runs the same level-synchronous top-down steps (Algorithm 1;
// Algorithm 2 with a single compute node) with workgroup barriers between
// phases:
//   expand - the frontier queue is dealt 64 entries per wavefront, entry i to
//            wavefront i mod 16 (so the hubs at the front of a degree-sorted
//            queue spread over the wavefronts); each wavefront's 64 adjacency
//            lists are dealt evenly over its lanes (a wavefront prefix sum and
//            a binary search over the shuffled prefix values), and every
//            neighbour whose visited bit is clear is ORed into the LDS next
//            bitmap;
//   merge  - new = next & ~visited per word; the new vertices get distance
//            level+1 and are appended to the next frontier queue (global
//            memory, one LDS counter).
// The control block receives the level count, the reached count and the
// edges scanned, as the other level loops leave them.

#include <hip/hip_runtime.h>

#include "bfs_core.hpp"

namespace bfsk {

namespace {

constexpr int kCuBlock = 1024;
constexpr int kCuWaves = kCuBlock / kWave;
constexpr int kCuUnroll = 4;  // edges per lane in flight
constexpr int kCuMergeWords = 4;  // bitmap words per wavefront step of the merge

__device__ __forceinline__ void lds_or(uint64_t *p, uint64_t bit) {
  (void)__hip_atomic_fetch_or(p, bit, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_WORKGROUP);
}

// Requires a whole graph (owned range [0, n)) with m < 2^25 edges, so one
// wavefront's edge prefix sums fit in 32 bits, 2 * words * 8 bytes of dynamic
// LDS, and two queue buffers of n packed rows (qr0[0], qr0[1]): an entry is
// the vertex's row start << 24 | its degree (the merge has just read both),
// so the expansion goes from the queue straight to the column ids, and each
// round's entries are requested while the previous round is expanded. dist
// was reset by k_reset.
__global__ void __launch_bounds__(kCuBlock) k_bfs_cu(View v, int64_t src_caller, int max_levels) {
  extern __shared__ uint64_t lds[];
  // an error flagged before the launch (an invalid graph) skips the traversal
  if (load_relaxed_i32(&v.ctl->err)) return;
  const int64_t W = v.words;
  uint64_t *vis = lds, *nxt = lds + W;
  __shared__ uint32_t s_qn[2];
  __shared__ unsigned long long s_edges;
  const int tid = threadIdx.x;
  const int lane = lane_id();
  const int wave = tid / kWave;
  const int64_t src = v.new_id ? (int64_t)v.new_id[src_caller] : src_caller;
  for (int64_t w = tid; w < W; w += kCuBlock) {
    vis[w] = (w == (src >> 6)) ? (1ull << (src & 63)) : 0ull;
    nxt[w] = 0ull;
  }
  if (tid == 0) {
    v.qr0[0][0] = pack_row(v.rp[src], v.rp[src + 1] - v.rp[src]);
    s_qn[0] = 1;
    s_edges = 0;
  }
  __syncthreads();
  uint64_t edges = 0;  // lane 0 of each wavefront: degrees of its frontier vertices
  uint64_t reached = 1;
  uint32_t nn = 0;
  int L = 0;
  for (;; ++L) {
    const int cur = L & 1, nx = cur ^ 1;
    const uint64_t *q = v.qr0[cur];
    uint64_t *qn = v.qr0[nx];
    // queue counts are read as wave-uniform values, so the loop's exit test is
    // uniform and the compiler keeps every lane in every iteration
    const int64_t nq = __builtin_amdgcn_readfirstlane(s_qn[cur]);
    // the counter this level's merge fills was last read at the previous
    // level's start; the merge is one barrier away
    if (tid == 0) s_qn[nx] = 0;
    // histogram row L+2 is first written by the merge of level L+1
    if (v.stats && L + 2 < kMaxStatLevels && tid < kNumBins) v.lvl_hist[(L + 2) * kNumBins + tid] = 0;
    // expand: round r covers queue entries [r, r + 1024); lane l of wavefront
    // w takes entry r + w + 16 l
    uint64_t pr_next = 0;
    {
      const int64_t i = wave + (int64_t)kCuWaves * lane;
      if (i < nq) pr_next = q[i];
    }
    for (int64_t r = 0; r < nq; r += kCuBlock) {
      const uint64_t pr = pr_next;
      const int64_t i2 = r + kCuBlock + wave + (int64_t)kCuWaves * lane;
      pr_next = i2 < nq ? q[i2] : 0ull;
      const int64_t start = (int64_t)(pr >> kRowShift);
      const int32_t deg = (int32_t)(pr & ((1ull << kRowShift) - 1));
      const int32_t incl = wave_incl_scan32(deg);
      const int32_t total = __shfl(incl, kWave - 1);
      const int64_t rebase = start - (int64_t)(incl - deg);
      if (lane == 0) edges += (uint64_t)total;
      for (int32_t e0 = 0; e0 < total; e0 += kWave * kCuUnroll) {
        int32_t u[kCuUnroll];
        bool ok[kCuUnroll];
#pragma unroll
        for (int j = 0; j < kCuUnroll; ++j) {
          const int32_t e = e0 + j * kWave + lane;
          int k = 0;
#pragma unroll
          for (int step = 32; step >= 1; step >>= 1)
            if (__shfl(incl, k + step - 1) <= e) k += step;
          k = min(k, kWave - 1);
          const int64_t rk = shfl64(rebase, k);
          ok[j] = e < total;
          u[j] = ok[j] ? __builtin_nontemporal_load(v.col + rk + e) : 0;
        }
#pragma unroll
        for (int j = 0; j < kCuUnroll; ++j) {
          const uint32_t uw = (uint32_t)u[j] >> 6;
          const uint64_t bit = 1ull << (u[j] & 63);
          if (ok[j] && !(vis[uw] & bit) && !(nxt[uw] & bit)) lds_or(nxt + uw, bit);
        }
      }
    }
    __syncthreads();
    // merge: kCuMergeWords words per wavefront step, their row-offset loads
    // in flight together
    for (int64_t w0 = (int64_t)wave * kCuMergeWords; w0 < W; w0 += (int64_t)kCuWaves * kCuMergeWords) {
      uint64_t nw[kCuMergeWords];
      int64_t r0[kCuMergeWords], r1[kCuMergeWords];
#pragma unroll
      for (int q = 0; q < kCuMergeWords; ++q) {
        const int64_t w = w0 + q;
        nw[q] = w < W ? nxt[w] & ~vis[w] : 0ull;
        r0[q] = r1[q] = 0;
        if ((nw[q] >> lane) & 1ull) {
          const int64_t x = w * 64 + lane;
          r0[q] = v.rp[x];
          r1[q] = v.rp[x + 1];
        }
      }
#pragma unroll
      for (int q = 0; q < kCuMergeWords; ++q) {
        const int64_t w = w0 + q;
        if (w >= W) break;
        if (nw[q] != 0ull) {
          uint32_t base = 0;
          if (lane == 0) {
            base = __hip_atomic_fetch_add(&s_qn[nx], (uint32_t)__popcll(nw[q]), __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_WORKGROUP);
            vis[w] |= nw[q];
          }
          base = __shfl(base, 0);
          if ((nw[q] >> lane) & 1ull) {
            const int64_t x = w * 64 + lane;
            v.dist[v.old_id ? (int64_t)v.old_id[x] : x] = L + 1;
            qn[base + rank_below(nw[q])] = pack_row(r0[q], r1[q] - r0[q]);
            if (v.stats && L + 1 < kMaxStatLevels)
              atomic_add32(&v.lvl_hist[(L + 1) * kNumBins + degree_bin(r1[q] - r0[q])], 1u);
          }
        }
        if (lane == 0) nxt[w] = 0ull;
      }
    }
    __syncthreads();
    nn = __builtin_amdgcn_readfirstlane(s_qn[nx]);
    reached += nn;
    if (v.stats && tid == 0 && L + 1 < kMaxStatLevels) v.lvl_frontier[L + 1] = (int64_t)nn;
    if (nn == 0 || L + 1 >= max_levels) break;
  }
  if (lane == 0 && edges)
    (void)__hip_atomic_fetch_add(&s_edges, (unsigned long long)edges, __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_WORKGROUP);
  __syncthreads();
  if (tid == 0) {
    Ctl *c = v.ctl;
    c->levels = L + 1;
    c->reached = reached;
    c->edges = s_edges;
    if (nn != 0) c->err |= 2;
  }
}

}  // namespace

// Dynamic LDS of the one-workgroup traversal of a graph with `words` bitmap words.
size_t cu_lds_bytes(int64_t words) { return (size_t)words * 2 * sizeof(uint64_t); }

// Whether the one-workgroup traversal can run graph g (whole graph, m below
// 2^25, bitmaps within max_lds bytes of LDS next to the static LDS).
bool cu_fits(int64_t n, int64_t m, bool whole, int max_lds) {
  const int64_t words = (n + 63) / 64;
  return whole && n > 0 && m < (1ll << 25) && (int64_t)cu_lds_bytes(words) + 1024 <= max_lds;
}

hipError_t launch_bfs_cu(const View &v, int64_t src, int max_levels, hipStream_t s) {
  const size_t lds = cu_lds_bytes(v.words);
  (void)hipFuncSetAttribute((const void *)k_bfs_cu, hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  hipLaunchKernelGGL(k_bfs_cu, dim3(1), dim3(kCuBlock), lds, s, v, src, max_levels);
  return hipGetLastError();
}

}  // namespace bfsk
