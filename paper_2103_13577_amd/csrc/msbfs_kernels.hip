// Kernels of the batched multi-source traversal (bitset lanes, 64 sources per
// uint64 word per vertex). The level structure is the same top-down
// expansion as the single-source path, carried out on lane words: Phase 1
// ORs each active vertex's frontier words into its neighbours' next words
// (skipping bits a neighbour has already seen), the sweep turns next words
// into new bits, distances and the next active-vertex tier queues.

#include <hip/hip_runtime.h>

#include "bfs_core.hpp"
#include "msbfs_core.hpp"

namespace bfsk {

__device__ __forceinline__ uint64_t wave_or(uint64_t x) {
#pragma unroll
  for (int d = 32; d >= 1; d >>= 1) x |= (uint64_t)shfl64((int64_t)x, lane_id() ^ d);
  return x;
}

__device__ __forceinline__ uint32_t ms_upper_slot(const uint32_t *a, uint32_t n, uint64_t key) {
  uint32_t lo = 0, hi = n - 1;
  while (lo < hi) {
    uint32_t mid = (lo + hi + 1) >> 1;
    if ((uint64_t)a[mid] <= key) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// OR the frontier words f into the next words of u, for bits u has not seen.
template <int LW>
__device__ __forceinline__ void ms_push_edge(const MsView &v, int64_t u, const uint64_t (&f)[LW]) {
#pragma unroll
  for (int l = 0; l < LW; ++l) {
    if (!f[l]) continue;
    const int64_t idx = u * LW + l;
    const uint64_t bits = f[l] & ~v.S[idx];
    if (bits && (bits & ~v.N[idx])) atomic_or_noret(v.N + idx, bits);
  }
}

template <int LW>
__device__ void ms_push_phase(const MsView &v, int L, uint32_t vb_id, uint32_t nvb) {
  __shared__ int64_t s_lo, s_hi;
  __shared__ uint64_t s_f[LW];
  const int cur = L & 1;
  const int lane = lane_id();
  const uint32_t wave = threadIdx.x / kWave;
  const uint64_t gwave = (uint64_t)vb_id * kWavesPerBlock + wave;
  const uint64_t nwaves = (uint64_t)nvb * kWavesPerBlock;

  // Heavy vertices: fixed-size edge chunks, one workgroup each.
  const uint64_t hv = load_relaxed64(&v.ctl->heavy[cur]);
  const uint32_t n2 = (uint32_t)(hv >> kHeavyShift);
  const uint64_t nch = hv & kChunkMask;
  for (uint64_t c = vb_id; c < nch; c += nvb) {
    if (threadIdx.x == 0) {
      const uint32_t s = ms_upper_slot(v.cstart[cur], n2, c);
      const int64_t x = v.q2[cur][s];
      const int64_t b = v.rp[x], e = v.rp[x + 1];
      const int64_t lo = b + ((int64_t)(c - v.cstart[cur][s]) << v.chunk_shift);
      s_lo = lo;
      s_hi = min(e, lo + (1ll << v.chunk_shift));
#pragma unroll
      for (int l = 0; l < LW; ++l) s_f[l] = v.F[x * LW + l];
    }
    __syncthreads();
    uint64_t f[LW];
#pragma unroll
    for (int l = 0; l < LW; ++l) f[l] = s_f[l];
    const int64_t lo = s_lo, hi = s_hi;
    for (int64_t e = lo + threadIdx.x; e < hi; e += kBlock)
      ms_push_edge<LW>(v, __builtin_nontemporal_load(v.col + e), f);
    __syncthreads();
  }

  // Newly admitted sources, then medium vertices: one wavefront per vertex.
  const uint32_t ne = load_relaxed32(&v.ctl->nextra);
  const uint32_t n1 = load_relaxed32(&v.ctl->qn[cur][1]);
  for (uint64_t i = gwave; i < (uint64_t)ne + n1; i += nwaves) {
    const int64_t x = i < ne ? v.extra[i] : v.q1[cur][i - ne];
    uint64_t f[LW];
#pragma unroll
    for (int l = 0; l < LW; ++l) f[l] = v.F[x * LW + l];
    const int64_t b = v.rp[x], e = v.rp[x + 1];
    for (int64_t k = b + lane; k < e; k += kWave)
      ms_push_edge<LW>(v, __builtin_nontemporal_load(v.col + k), f);
  }

  // Small vertices: 64 per wavefront, edges dealt evenly to the lanes.
  const uint32_t n0 = load_relaxed32(&v.ctl->qn[cur][0]);
  for (uint64_t base = gwave * kWave; base < n0; base += nwaves * kWave) {
    const uint64_t i = base + lane;
    int64_t start = 0, deg = 0;
    uint64_t f[LW];
#pragma unroll
    for (int l = 0; l < LW; ++l) f[l] = 0;
    if (i < n0) {
      const int64_t x = v.q0[cur][i];
      start = v.rp[x];
      deg = v.rp[x + 1] - start;
#pragma unroll
      for (int l = 0; l < LW; ++l) f[l] = v.F[x * LW + l];
    }
    const int64_t incl = wave_incl_scan(deg);
    const int64_t total = shfl64(incl, kWave - 1);
    const int64_t excl = incl - deg;
    for (int64_t e0 = 0; e0 < total; e0 += kWave) {
      const int64_t e = e0 + lane;
      int k = 0;
#pragma unroll
      for (int step = 32; step >= 1; step >>= 1) {
        const int64_t val = shfl64(incl, k + step - 1);
        if (val <= e) k += step;
      }
      k = min(k, kWave - 1);
      const int64_t xk = shfl64(excl, k);
      const int64_t sk = shfl64(start, k);
      uint64_t fk[LW];
#pragma unroll
      for (int l = 0; l < LW; ++l) fk[l] = (uint64_t)shfl64((int64_t)f[l], k);
      if (e < total) ms_push_edge<LW>(v, __builtin_nontemporal_load(v.col + sk + (e - xk)), fk);
    }
  }
}

template <int LW>
__device__ void ms_sweep_phase(const MsView &v, int L, uint32_t vb_id, uint32_t nvb) {
  __shared__ uint64_t s_or[kMsMaxGraphs * kMsMaxLW];
  __shared__ uint32_t s_cnt[kWavesPerBlock][3];
  __shared__ uint64_t s_chunks[kWavesPerBlock];
  __shared__ uint32_t s_base[3];
  __shared__ uint64_t s_cbase;
  __shared__ int32_t s_g;
  __shared__ uint64_t s_act[kWavesPerBlock];

  const int cur = L & 1, nxt = cur ^ 1;
  const int lane = lane_id();
  const int wave = threadIdx.x / kWave;
  const int cs = v.chunk_shift;
  const int nslotw = v.ng * LW;

  if (vb_id == 0 && threadIdx.x == 0) {
    v.ctl->qn[cur][0] = 0;
    v.ctl->qn[cur][1] = 0;
    v.ctl->heavy[cur] = 0;
    v.ctl->nextra = 0;
    v.ctl->active[(L + 1) % 3] = 0;
  }
  if (vb_id == 0)
    for (int i = threadIdx.x; i < nslotw; i += kBlock) v.newmask[((L + 1) % 3) * nslotw + i] = 0;
  for (int i = threadIdx.x; i < nslotw; i += kBlock) s_or[i] = 0;
  __syncthreads();

  uint64_t my_active = 0;
  for (int64_t c = vb_id; c < v.nchunks; c += nvb) {
    if (threadIdx.x == 0) {
      int g = 0;
      while (g + 1 < v.ng && v.graphs[g + 1].chunk_begin <= c) ++g;
      s_g = g;
    }
    __syncthreads();
    const int g = s_g;
    const MsGraph gr = v.graphs[g];
    const int64_t xl = (c - gr.chunk_begin) * kMsChunk + threadIdx.x;
    const bool valid = xl < gr.n;
    const int64_t x = gr.off + xl;
    uint64_t nw[LW];
    bool any = false;
#pragma unroll
    for (int l = 0; l < LW; ++l) {
      nw[l] = 0;
      if (valid) {
        const int64_t idx = x * LW + l;
        const uint64_t n = v.N[idx];
        const uint64_t fo = v.F[idx];
        uint64_t w = 0;
        if (n) {
          v.N[idx] = 0;
          const uint64_t s = v.S[idx];
          w = n & ~s;
          if (w) v.S[idx] = s | w;
        }
        if (fo != w) v.F[idx] = w;
        nw[l] = w;
        any |= w != 0;
      }
    }
    // Distances: for every slot with a new bit in this wavefront, the lanes
    // holding the bit write their vertex's entry (coalesced per slot).
#pragma unroll
    for (int l = 0; l < LW; ++l) {
      uint64_t wor = wave_or(nw[l]);
      if (wor && lane == 0) atomicOr((unsigned long long *)&s_or[g * LW + l], (unsigned long long)wor);
      while (wor) {
        const int b = __ffsll((unsigned long long)wor) - 1;
        wor &= wor - 1;
        const int slot = (g * LW + l) * 64 + b;
        if ((nw[l] >> b) & 1ull) {
          const int32_t val = L + 1 - v.slot_start[slot];
          const uint64_t ptr = v.slot_out[slot];
          if (v.slot_type[slot] == 0) {
            if (val > 254) atomic_or64(&v.depth_err[g * LW + l], 1ull << b);
            else ((uint8_t *)ptr)[xl] = (uint8_t)val;
          } else {
            ((int32_t *)ptr)[xl] = val;
          }
        }
      }
    }
    // Active vertices into the next level's tier queues.
    int64_t deg = 0;
    int t = 0;
    if (any) {
      deg = v.rp[x + 1] - v.rp[x];
      t = tier_of_bin(degree_bin(deg), v.small_bin, v.wave_bin);
    }
    const uint64_t m0 = ballot(any && t == 0);
    const uint64_t m1 = ballot(any && t == 1);
    const uint64_t m2 = ballot(any && t == 2);
    const int64_t nc = (any && t == 2) ? ((deg + (1ll << cs) - 1) >> cs) : 0;
    const int64_t ncin = m2 ? wave_incl_scan(nc) : 0;
    const uint64_t wchunks = m2 ? (uint64_t)shfl64(ncin, kWave - 1) : 0ull;
    if (lane == 0) {
      s_cnt[wave][0] = (uint32_t)__popcll(m0);
      s_cnt[wave][1] = (uint32_t)__popcll(m1);
      s_cnt[wave][2] = (uint32_t)__popcll(m2);
      s_chunks[wave] = wchunks;
      my_active += (uint64_t)__popcll(m0 | m1 | m2);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      uint32_t t0 = 0, t1 = 0, t2 = 0;
      uint64_t ch = 0;
      for (int w = 0; w < kWavesPerBlock; ++w) {
        t0 += s_cnt[w][0];
        t1 += s_cnt[w][1];
        t2 += s_cnt[w][2];
        ch += s_chunks[w];
      }
      s_base[0] = t0 ? atomic_add32(&v.ctl->qn[nxt][0], t0) : 0u;
      s_base[1] = t1 ? atomic_add32(&v.ctl->qn[nxt][1], t1) : 0u;
      if (t2) {
        const uint64_t old = atomic_add64(&v.ctl->heavy[nxt], ((uint64_t)t2 << kHeavyShift) | ch);
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
    for (int w = 0; w < wave; ++w) {
      b0 += s_cnt[w][0];
      b1 += s_cnt[w][1];
      b2 += s_cnt[w][2];
      cb += s_chunks[w];
    }
    if ((m0 >> lane) & 1ull) v.q0[nxt][b0 + rank_below(m0)] = (int32_t)x;
    if ((m1 >> lane) & 1ull) v.q1[nxt][b1 + rank_below(m1)] = (int32_t)x;
    if ((m2 >> lane) & 1ull) {
      const uint32_t slot = b2 + rank_below(m2);
      v.q2[nxt][slot] = (int32_t)x;
      v.cstart[nxt][slot] = (uint32_t)(cb + (uint64_t)(ncin - nc));
    }
    __syncthreads();
  }
  // Flush this workgroup's slot masks and active count.
  for (int i = threadIdx.x; i < nslotw; i += kBlock)
    if (s_or[i]) atomic_or64(&v.newmask[(L % 3) * nslotw + i], s_or[i]);
  if (lane == 0) s_act[wave] = my_active;
  __syncthreads();
  if (threadIdx.x == 0) {
    uint64_t a = 0;
    for (int w = 0; w < kWavesPerBlock; ++w) a += s_act[w];
    if (a) atomic_add64(&v.ctl->active[L % 3], a);
  }
}

template <int LW>
__global__ void __launch_bounds__(kBlock) k_ms_persistent(MsView v, int max_levels) {
  const uint32_t nb = gridDim.x;
  int L = load_relaxed_i32(&v.ctl->level);
  int run = 0;
  bool early = false;
  for (;;) {
    ms_push_phase<LW>(v, L, blockIdx.x, nb);
    grid_barrier(&v.ctl->bar, nb);
    ms_sweep_phase<LW>(v, L, blockIdx.x, nb);
    grid_barrier(&v.ctl->bar, nb);
    ++run;
    const uint64_t act = load_relaxed64(&v.ctl->active[L % 3]);
    const int tripped = __hip_atomic_load(&v.ctl->bar.tripped, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
    bool stop = act == 0 || tripped || run >= max_levels;
    if (!stop && v.stream_stop) {
      const int nslotw = v.ng * LW;
      for (int i = 0; i < nslotw; ++i)
        if (v.slot_active[i] & ~load_relaxed64(&v.newmask[(L % 3) * nslotw + i])) {
          stop = true;
          early = true;
          break;
        }
    }
    ++L;
    if (stop) break;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    v.ctl->level = L;
    v.ctl->levels_run = run;
    v.ctl->stopped_early = early ? 1 : 0;
  }
}

// ---------------------------------------------------------------------------
// set-up kernels
// ---------------------------------------------------------------------------

__global__ void k_ms_flatten(const int64_t *rp_g, const int32_t *col_g, int64_t n_g, int64_t m_g,
                             int64_t off, int64_t eoff, int64_t *rp_flat, int32_t *col_flat) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = tid; i <= n_g; i += stride) rp_flat[off + i] = eoff + rp_g[i];
  for (int64_t e = tid; e < m_g; e += stride) col_flat[eoff + e] = (int32_t)(off + col_g[e]);
}

// Output fill: 255 (uint8) or -1 (int32) everywhere; blockIdx.y = admission.
__global__ void k_ms_fill(const MsAdmit *adm) {
  const MsAdmit a = adm[blockIdx.y];
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  if (a.type == 0) {
    uint8_t *o = (uint8_t *)a.out;
    const int64_t n4 = a.n / 4;
    if ((a.out & 3) == 0) {
      for (int64_t i = tid; i < n4; i += stride) ((uint32_t *)o)[i] = 0xFFFFFFFFu;
      for (int64_t i = 4 * n4 + tid; i < a.n; i += stride) o[i] = 0xFF;
    } else {
      for (int64_t i = tid; i < a.n; i += stride) o[i] = 0xFF;
    }
  } else {
    int32_t *o = (int32_t *)a.out;
    for (int64_t i = tid; i < a.n; i += stride) o[i] = -1;
  }
}

// Admission: slot tables, root bits in F and S, root distance 0, and the
// root on the list of vertices expanded at the next level.
template <int LW>
__global__ void k_ms_admit(MsView v, const MsAdmit *adm, int32_t nadm, int32_t level) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= nadm) return;
  const MsAdmit a = adm[i];
  const int slot = a.slot;
  const int l = (slot / 64) % LW;
  const uint64_t bit = 1ull << (slot % 64);
  v.slot_out[slot] = a.out;
  v.slot_type[slot] = a.type;
  v.slot_start[slot] = level;
  atomic_or64(&v.F[a.src_flat * LW + l], bit);
  atomic_or64(&v.S[a.src_flat * LW + l], bit);
  if (a.type == 0) ((uint8_t *)a.out)[a.src_local] = 0;
  else ((int32_t *)a.out)[a.src_local] = 0;
  const uint32_t pos = atomic_add32(&v.ctl->nextra, 1u);
  v.extra[pos] = (int32_t)a.src_flat;
}

// Clears slot bits (mask per lane word of graph g) in [begin, end).
template <int LW>
__global__ void k_ms_clear(MsView v, int64_t begin, int64_t end, const uint64_t *mask) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  uint64_t keep[LW];
#pragma unroll
  for (int l = 0; l < LW; ++l) keep[l] = ~mask[l];
  for (int64_t x = begin + tid; x < end; x += stride) {
#pragma unroll
    for (int l = 0; l < LW; ++l) {
      const int64_t idx = x * LW + l;
      const uint64_t s = v.S[idx];
      if (s & ~keep[l]) v.S[idx] = s & keep[l];
      const uint64_t f = v.F[idx];
      if (f & ~keep[l]) v.F[idx] = f & keep[l];
      const uint64_t n = v.N[idx];
      if (n & ~keep[l]) v.N[idx] = n & keep[l];
    }
  }
}

// ---------------------------------------------------------------------------
// host launchers
// ---------------------------------------------------------------------------

hipError_t ms_launch_flatten(const int64_t *rp_g, const int32_t *col_g, int64_t n_g, int64_t m_g,
                             int64_t off, int64_t eoff, int64_t *rp_flat, int32_t *col_flat,
                             hipStream_t s) {
  const int64_t work = std::max<int64_t>(n_g + 1, m_g);
  const int grid = (int)std::min<int64_t>((work + 255) / 256, 8192);
  hipLaunchKernelGGL(k_ms_flatten, dim3(std::max(grid, 1)), dim3(256), 0, s, rp_g, col_g, n_g, m_g,
                     off, eoff, rp_flat, col_flat);
  return hipGetLastError();
}

hipError_t ms_launch_fill(const MsAdmit *adm, int32_t nadm, int64_t maxn, hipStream_t s) {
  if (nadm <= 0) return hipSuccess;
  const int gx = (int)std::min<int64_t>((maxn + 1023) / 1024, 256);
  hipLaunchKernelGGL(k_ms_fill, dim3(std::max(gx, 1), nadm), dim3(256), 0, s, adm);
  return hipGetLastError();
}

hipError_t ms_launch_admit(const MsView &v, const MsAdmit *adm, int32_t nadm, int32_t level,
                           hipStream_t s) {
  if (nadm <= 0) return hipSuccess;
  const int grid = (nadm + 255) / 256;
  switch (v.lw) {
    case 1: hipLaunchKernelGGL(k_ms_admit<1>, dim3(grid), dim3(256), 0, s, v, adm, nadm, level); break;
    case 2: hipLaunchKernelGGL(k_ms_admit<2>, dim3(grid), dim3(256), 0, s, v, adm, nadm, level); break;
    case 4: hipLaunchKernelGGL(k_ms_admit<4>, dim3(grid), dim3(256), 0, s, v, adm, nadm, level); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

hipError_t ms_launch_clear(const MsView &v, int64_t begin, int64_t end, const uint64_t *mask,
                           hipStream_t s) {
  const int grid = (int)std::min<int64_t>((end - begin + 255) / 256, 8192);
  switch (v.lw) {
    case 1: hipLaunchKernelGGL(k_ms_clear<1>, dim3(std::max(grid, 1)), dim3(256), 0, s, v, begin, end, mask); break;
    case 2: hipLaunchKernelGGL(k_ms_clear<2>, dim3(std::max(grid, 1)), dim3(256), 0, s, v, begin, end, mask); break;
    case 4: hipLaunchKernelGGL(k_ms_clear<4>, dim3(std::max(grid, 1)), dim3(256), 0, s, v, begin, end, mask); break;
    default: return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

int ms_blocks_per_cu(int lw) {
  int nb = 0;
  hipError_t e = hipErrorInvalidValue;
  switch (lw) {
    case 1: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_ms_persistent<1>, kBlock, 0); break;
    case 2: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_ms_persistent<2>, kBlock, 0); break;
    case 4: e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&nb, k_ms_persistent<4>, kBlock, 0); break;
    default: break;
  }
  return e == hipSuccess ? nb : 0;
}

hipError_t ms_launch_persistent(const MsView &v, int32_t max_levels, int32_t grid, hipStream_t s) {
  MsView vv = v;
  int ml = max_levels;
  void *args[] = {&vv, &ml};
  const void *fn = nullptr;
  switch (v.lw) {
    case 1: fn = (const void *)k_ms_persistent<1>; break;
    case 2: fn = (const void *)k_ms_persistent<2>; break;
    case 4: fn = (const void *)k_ms_persistent<4>; break;
    default: return hipErrorInvalidValue;
  }
  return hipLaunchCooperativeKernel(fn, dim3(grid), dim3(kBlock), args, 0, s);
}

}  // namespace bfsk
