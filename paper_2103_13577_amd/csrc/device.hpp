// Device-side building blocks for gfx950 (CDNA4, 64-lane wavefronts):
// wavefront ballot/scan helpers, device-scope atomics and a bounded grid
// barrier for cooperative (co-resident) launches.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace bfsk {

constexpr int kWave = 64;

__device__ __forceinline__ int lane_id() { return __lane_id(); }

// 64-bit ballot of a per-lane predicate.
__device__ __forceinline__ uint64_t ballot(bool p) { return __ballot(p); }

// Number of set bits of `mask` below this lane (exclusive rank).
__device__ __forceinline__ uint32_t rank_below(uint64_t mask) {
  return __builtin_amdgcn_mbcnt_hi((uint32_t)(mask >> 32),
                                   __builtin_amdgcn_mbcnt_lo((uint32_t)mask, 0u));
}

__device__ __forceinline__ uint64_t readlane64(uint64_t x, int l) {
  uint32_t lo = __builtin_amdgcn_readlane((uint32_t)x, l);
  uint32_t hi = __builtin_amdgcn_readlane((uint32_t)(x >> 32), l);
  return ((uint64_t)hi << 32) | lo;
}

// A wave-uniform value held in vector registers, moved to scalar registers
// (so address arithmetic on it is scalar).
__device__ __forceinline__ int64_t uniform64(int64_t x) {
  const uint32_t lo = __builtin_amdgcn_readfirstlane((uint32_t)(uint64_t)x);
  const uint32_t hi = __builtin_amdgcn_readfirstlane((uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}

__device__ __forceinline__ int64_t shfl64(int64_t x, int src) {
  int lo = __shfl((int)(uint32_t)(uint64_t)x, src);
  int hi = __shfl((int)(uint32_t)((uint64_t)x >> 32), src);
  return (int64_t)(((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

// Inclusive prefix sum across the wavefront (Hillis-Steele over 6 steps).
__device__ __forceinline__ int64_t wave_incl_scan(int64_t x) {
  const int l = lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    int64_t y = shfl64(x, l >= d ? l - d : l);
    if (l >= d) x += y;
  }
  return x;
}

__device__ __forceinline__ int32_t wave_incl_scan32(int32_t x) {
  const int l = lane_id();
#pragma unroll
  for (int d = 1; d < kWave; d <<= 1) {
    const int32_t y = __shfl(x, l >= d ? l - d : l);
    if (l >= d) x += y;
  }
  return x;
}

__device__ __forceinline__ int64_t wave_sum(int64_t x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += shfl64(x, lane_id() ^ d);
  return x;
}

__device__ __forceinline__ uint32_t wave_sum_u32(uint32_t x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x += (uint32_t)__shfl_xor((int)x, d);
  return x;
}

// Largest s in [0, n) with a[s] <= key (a strictly ascending, a[0] == 0 <=
// key), found by the whole wavefront: each round samples 64 evenly spaced
// entries of the remaining range and keeps the segment after the last sample
// <= key, so n entries take ceil(log64 n) dependent loads instead of log2 n.
// All lanes must call it; the result is wave-uniform.
__device__ __forceinline__ uint32_t wave_upper_slot(const uint32_t *a, uint32_t n, uint64_t key) {
  const int lane = lane_id();
  uint32_t lo = 0, len = n;  // the answer lies in [lo, lo + len)
  while (len > 1) {
    const uint32_t step = (len + kWave - 1) / kWave;
    const uint32_t idx = lo + (uint32_t)lane * step;
    const bool le = idx < lo + len && (uint64_t)a[idx] <= key;
    const uint32_t cnt = (uint32_t)__popcll(ballot(le));  // >= 1: a[lo] <= key
    const uint32_t nlo = lo + (cnt - 1) * step;
    len = min(step, lo + len - nlo);
    lo = nlo;
  }
  return lo;
}

// Relaxed device-scope atomics (agent scope: every CU of every XCD).
__device__ __forceinline__ void atomic_or_noret(uint64_t *p, uint64_t v) {
  (void)__hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void atomic_or_noret32(uint32_t *p, uint32_t v) {
  (void)__hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t atomic_or64(uint64_t *p, uint64_t v) {
  return __hip_atomic_fetch_or(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t atomic_add32(uint32_t *p, uint32_t v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t atomic_add64(uint64_t *p, uint64_t v) {
  return __hip_atomic_fetch_add(p, v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint32_t load_relaxed32(const uint32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ uint64_t load_relaxed64(const uint64_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ int32_t load_relaxed_i32(const int32_t *p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Grid barrier state. Arrival and release words of each group of blocks and
// the global generation each sit on their own 128-byte cache line, so polling
// is spread over many lines instead of hammering one. Valid from any initial
// generation; every arrival counter must be 0 when no block is inside a
// barrier (the last arriver of each level resets it).
constexpr int kBarrierGroup = 32;      // blocks per group
constexpr int kBarrierMaxGroups = 64;  // up to 2048 blocks
struct GridBarrier {
  uint32_t gen;
  int32_t tripped;  // set when a wait exceeded its spin limit
  uint32_t pad0[30];
  uint32_t top;     // arrivals of group leaders
  uint32_t pad1[31];
  struct {
    uint32_t count;    // arrivals in the group
    uint32_t release;  // generation last released to the group
    uint32_t pad[30];
  } group[kBarrierMaxGroups];
};

// Spin limit per barrier wait: 2^20 polls separated by sleeps is well over
// 0.1 s, orders of magnitude above any legitimate wait for co-resident blocks.
constexpr uint32_t kSpinLimit = 1u << 20;

// Polls with relaxed loads: an acquire load at agent scope invalidates the
// CU's caches on every poll, which with many polling blocks evicts the working
// set of the blocks still computing. The caller issues one acquire fence once
// the word has moved.
__device__ __forceinline__ bool spin_until_changed(const uint32_t *p, uint32_t old, int32_t *tripped) {
  uint32_t spins = 0;
  while (__hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) == old) {
    __builtin_amdgcn_s_sleep(2);
    if (++spins > kSpinLimit) {
      __hip_atomic_store(tripped, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      return false;
    }
  }
  return true;
}

// All blocks of a cooperative launch (at most 2048) must call this the same
// number of times. Arrival is a two-level tree: the last block of each group
// of 32 arrives at the top counter, and the last group leader resets the
// counters and advances the global generation. Release is the same tree in
// reverse: group leaders wait for the global generation and then release
// their group through the group's own word, on which the other members wait.
// Every block reads the word it waits on before it arrives (it cannot move
// until that block has arrived). Release/acquire at agent scope make every
// write before the barrier visible to every read after it. A wait that
// exceeds the spin limit marks `tripped` and lets the block continue, so the
// kernel always terminates; the host reports the trip as an error.
__device__ __forceinline__ void grid_barrier(GridBarrier *b, uint32_t nblocks) {
  __syncthreads();
  if (threadIdx.x == 0) {
    const uint32_t grp = blockIdx.x / kBarrierGroup;
    const uint32_t ngroups = (nblocks + kBarrierGroup - 1) / kBarrierGroup;
    const uint32_t in_grp = min((uint32_t)kBarrierGroup, nblocks - grp * kBarrierGroup);
    const uint32_t r0 =
        __hip_atomic_load(&b->group[grp].release, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    const uint32_t g0 = __hip_atomic_load(&b->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    const uint32_t a1 = __hip_atomic_fetch_add(&b->group[grp].count, 1u, __ATOMIC_ACQ_REL,
                                               __HIP_MEMORY_SCOPE_AGENT) + 1;
    if (a1 == in_grp) {
      // group leader: arrive at the top, wait for the generation, release the group
      __hip_atomic_store(&b->group[grp].count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      const uint32_t a2 =
          __hip_atomic_fetch_add(&b->top, 1u, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) + 1;
      if (a2 == ngroups) {
        __hip_atomic_store(&b->top, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_fetch_add(&b->gen, 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        spin_until_changed(&b->gen, g0, &b->tripped);
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
      __hip_atomic_store(&b->group[grp].release, r0 + 1, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
    } else {
      spin_until_changed(&b->group[grp].release, r0, &b->tripped);
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  }
  __syncthreads();
}

}  // namespace bfsk
