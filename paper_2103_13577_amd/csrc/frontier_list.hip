// Vertex-list form of the butterfly messages (Section 3, Algorithm 2 Phase 2).
//
// A node's global queue is its next-frontier bitmap. For a sparse level the
// message can instead be the list of its set bits, 4 bytes per vertex against
// n/8 bytes for the bitmap, so a list is the smaller message while it holds
// fewer than n/32 vertices (the paper's "lists of active vertices").
//
//   export  - the bitmap's set bits as an ascending int32 list: per-block
//             popcounts over contiguous word ranges, an exclusive scan of the
//             block counts, and a write pass in which each block scans its own
//             words again (workgroup prefix sum of the per-word popcounts) and
//             each lane writes its word's bits in ascending order;
//   receive - every listed vertex is checked against the global queue and
//             added to it when absent (one device-scope OR on its word); the
//             ordinary merge then finds the new vertices, so a list message
//             and the same set sent as a bitmap leave identical state.

#include <hip/hip_runtime.h>

#include <algorithm>

#include "bfs_core.hpp"

namespace bfsk {

namespace {

constexpr int kLB = 256;  // threads per block of the list kernels
constexpr int kLWaves = kLB / kWave;

// Word w of the bitmap with the bits at or above n cleared.
__device__ __forceinline__ uint64_t word_below_n(const uint64_t *bm, int64_t w, int64_t words, int64_t n) {
  uint64_t x = bm[w];
  if (w == words - 1 && (n & 63)) x &= ~0ull >> (64 - (n & 63));
  return x;
}

__global__ void __launch_bounds__(kLB) k_list_count(const uint64_t *bm, int64_t words, int64_t n,
                                                    int64_t per, uint64_t *blk) {
  __shared__ uint64_t s[kLWaves];
  const int64_t lo = (int64_t)blockIdx.x * per;
  const int64_t hi = min(lo + per, words);
  uint64_t c = 0;
  for (int64_t w = lo + threadIdx.x; w < hi; w += kLB) c += (uint64_t)__popcll(word_below_n(bm, w, words, n));
  c = (uint64_t)wave_sum((int64_t)c);
  if (lane_id() == 0) s[threadIdx.x / kWave] = c;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t t = 0;
    for (int i = 0; i < kLWaves; ++i) t += s[i];
    blk[blockIdx.x] = t;
  }
}

// In place: blk[0..nblk) -> exclusive prefix sums, blk[nblk] = total.
// One block of 1024 threads, two counts per thread (nblk <= 2048).
__global__ void __launch_bounds__(1024) k_list_scan(uint64_t *blk, int nblk) {
  __shared__ uint64_t s[1024 / kWave];
  const int t = threadIdx.x;
  const uint64_t a = (2 * t < nblk) ? blk[2 * t] : 0ull;
  const uint64_t b = (2 * t + 1 < nblk) ? blk[2 * t + 1] : 0ull;
  const int64_t loc = (int64_t)(a + b);
  const int64_t incl_w = wave_incl_scan(loc);
  if (lane_id() == kWave - 1) s[t / kWave] = (uint64_t)incl_w;
  __syncthreads();
  uint64_t before = 0;
  for (int i = 0; i < t / kWave; ++i) before += s[i];
  const uint64_t incl = before + (uint64_t)incl_w;
  const uint64_t excl = incl - (uint64_t)loc;
  if (2 * t < nblk) blk[2 * t] = excl;
  if (2 * t + 1 < nblk) blk[2 * t + 1] = excl + a;
  if (t == 1023) blk[nblk] = incl;
}

__global__ void __launch_bounds__(kLB) k_list_write(const uint64_t *bm, int64_t words, int64_t n,
                                                    int64_t per, const uint64_t *blk, int32_t *out,
                                                    int64_t cap) {
  __shared__ uint32_t s[kLWaves];
  const int64_t lo = (int64_t)blockIdx.x * per;
  const int64_t hi = min(lo + per, words);
  const int wave = threadIdx.x / kWave;
  int64_t base = (int64_t)blk[blockIdx.x];
  for (int64_t g0 = lo; g0 < hi; g0 += kLB) {
    const int64_t w = g0 + threadIdx.x;
    uint64_t x = (w < hi) ? word_below_n(bm, w, words, n) : 0ull;
    const int32_t c = __popcll(x);
    const int32_t incl = wave_incl_scan32(c);
    if (lane_id() == kWave - 1) s[wave] = (uint32_t)incl;
    __syncthreads();
    int64_t pos = base + incl - c;
    int64_t tot = 0;
    for (int i = 0; i < kLWaves; ++i) {
      if (i < wave) pos += s[i];
      tot += s[i];
    }
    while (x) {
      const int bit = __ffsll((unsigned long long)x) - 1;
      x &= x - 1;
      if (pos < cap) out[pos] = (int32_t)(w * 64 + bit);
      ++pos;
    }
    base += tot;
    __syncthreads();  // s is rewritten by the next step
  }
}

// Adds every listed vertex to the global queue `next`. Ids outside [0, n)
// are skipped and flagged in err (bit 4).
__global__ void __launch_bounds__(kLB) k_list_scatter(const int32_t *list, int64_t cnt, uint64_t *next,
                                                      int64_t n, int32_t *err) {
  const int64_t stride = (int64_t)gridDim.x * kLB;
  bool bad = false;
  for (int64_t i = (int64_t)blockIdx.x * kLB + threadIdx.x; i < cnt; i += stride) {
    const int32_t u = list[i];
    if (u < 0 || (int64_t)u >= n) {
      bad = true;
      continue;
    }
    const uint64_t bit = 1ull << (u & 63);
    uint64_t *p = next + (u >> 6);
    if (!(*p & bit)) atomic_or_noret(p, bit);
  }
  if (ballot(bad) && lane_id() == 0) atomic_or_noret32((uint32_t *)err, (uint32_t)kErrListId);
}

}  // namespace

void list_geometry(int64_t words, int &nblk, int64_t &per) {
  const int64_t w = words > 0 ? words : 1;
  int64_t nb = (w + kLB - 1) / kLB;
  if (nb > kListMaxBlocks) nb = kListMaxBlocks;
  per = (w + nb - 1) / nb;
  per = (per + kLB - 1) / kLB * kLB;
  nblk = (int)((w + per - 1) / per);
}

hipError_t launch_list_export(const uint64_t *bm, int64_t words, int64_t n, uint64_t *blk, int32_t *out,
                              int64_t cap, hipStream_t s) {
  int nblk = 0;
  int64_t per = 0;
  list_geometry(words, nblk, per);
  hipLaunchKernelGGL(k_list_count, dim3(nblk), dim3(kLB), 0, s, bm, words, n, per, blk);
  hipLaunchKernelGGL(k_list_scan, dim3(1), dim3(1024), 0, s, blk, nblk);
  if (out && cap > 0)
    hipLaunchKernelGGL(k_list_write, dim3(nblk), dim3(kLB), 0, s, bm, words, n, per, blk, out, cap);
  return hipGetLastError();
}

hipError_t launch_list_scatter(const int32_t *list, int64_t cnt, uint64_t *next, int64_t n, int32_t *err,
                               int max_grid, hipStream_t s) {
  if (cnt <= 0) return hipSuccess;
  const int64_t g = std::min<int64_t>((cnt + kLB - 1) / kLB, (int64_t)std::max(max_grid, 1));
  hipLaunchKernelGGL(k_list_scatter, dim3((int)g), dim3(kLB), 0, s, list, cnt, next, n, err);
  return hipGetLastError();
}

}  // namespace bfsk
