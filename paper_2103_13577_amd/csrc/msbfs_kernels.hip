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

// Per-level mode of each graph: dense (sweep every vertex) or sparse (only
// the vertices touched by the expansion are swept).
struct MsModes {
  uint32_t sparse;  // bit g set: graph g runs sparse in this level
};

// Graph of flat vertex x (graphs are laid out in order).
__device__ __forceinline__ int ms_graph_of(const MsView &v, int64_t x, const int64_t *s_off) {
  int g = 0;
  for (int k = 1; k < v.ng; ++k) g += (x >= s_off[k]) ? 1 : 0;
  return g;
}

// Appends u to the touched list with one atomic per wavefront (works in
// divergent code: only lanes with `want` need to be active).
__device__ __forceinline__ void ms_append_touched(const MsView &v, bool want, int64_t u, int L) {
  const uint64_t m = ballot(want);
  if (!m) return;
  const int leader = __ffsll((unsigned long long)m) - 1;
  uint32_t base = 0;
  if (lane_id() == leader) base = atomic_add32(&v.ctl->ntouched[L & 1], (uint32_t)__popcll(m));
  base = __builtin_amdgcn_readlane(base, leader);
  if (want) v.touched[base + rank_below(m)] = (int32_t)u;
}

// OR the frontier words f into the next words of u, for bits u has not seen.
// In a sparse graph the first write into an empty word of u this level
// records u (once, through the level mark) on the touched list.
template <int LW>
__device__ __forceinline__ void ms_push_edge(const MsView &v, int64_t u, const uint64_t (&f)[LW],
                                             bool sparse, int L) {
  bool first = false;
#pragma unroll
  for (int l = 0; l < LW; ++l) {
    if (!f[l]) continue;
    const int64_t idx = u * LW + l;
    const uint64_t bits = f[l] & ~v.S[idx];
    if (!bits || !(bits & ~v.N[idx])) continue;
    if (!sparse) {
      atomic_or_noret(v.N + idx, bits);
    } else if (atomic_or64(v.N + idx, bits) == 0ull) {
      first = true;
    }
  }
  bool want = false;
  if (first) want = __hip_atomic_exchange(v.mark + u, L, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != L;
  if (sparse) ms_append_touched(v, want, u, L);
}

template <int LW>
__device__ void ms_push_phase(const MsView &v, int L, uint32_t vb_id, uint32_t nvb,
                              const int64_t *s_off, uint32_t sparse_mask) {
  const int cur = L & 1;
  const int lane = lane_id();
  const uint32_t wave = threadIdx.x / kWave;
  const uint64_t gwave = (uint64_t)vb_id * kWavesPerBlock + wave;
  const uint64_t nwaves = (uint64_t)nvb * kWavesPerBlock;

  // Heavy vertices: fixed-size edge chunks, one wavefront each (a 64-way
  // search of the chunk starts finds the vertex). Their frontier words are
  // read by several wavefronts and cleared in the sweep.
  const uint64_t hv = load_relaxed64(&v.ctl->heavy[cur]);
  const uint32_t n2 = (uint32_t)(hv >> kHeavyShift);
  const uint64_t nch = hv & kChunkMask;
  for (uint64_t c = gwave; c < nch; c += nwaves) {
    const uint32_t s = wave_upper_slot(v.cstart[cur], n2, c);
    const int64_t x = v.q2[cur][s];
    const int64_t b = v.rp[x], e = v.rp[x + 1];
    const int64_t lo = b + ((int64_t)(c - v.cstart[cur][s]) << v.chunk_shift);
    const int64_t hi = min(e, lo + (1ll << v.chunk_shift));
    uint64_t f[LW];
#pragma unroll
    for (int l = 0; l < LW; ++l) f[l] = v.F[x * LW + l];
    const bool sp = (sparse_mask >> ms_graph_of(v, x, s_off)) & 1u;
    for (int64_t k = lo + lane; k < hi; k += kWave)
      ms_push_edge<LW>(v, __builtin_nontemporal_load(v.col + k), f, sp, L);
  }

  // Newly admitted sources, then medium vertices: one wavefront per vertex.
  // In a sparse graph the wavefront clears the frontier words it has read
  // (a vertex listed twice is pushed in full by whichever copy reads first).
  const uint32_t ne = load_relaxed32(&v.ctl->nextra);
  const uint32_t n1 = load_relaxed32(&v.ctl->qn[cur][1]);
  for (uint64_t i = gwave; i < (uint64_t)ne + n1; i += nwaves) {
    const int64_t x = i < ne ? v.extra[i] : v.q1[cur][i - ne];
    const bool sp = (sparse_mask >> ms_graph_of(v, x, s_off)) & 1u;
    uint64_t f[LW];
#pragma unroll
    for (int l = 0; l < LW; ++l) f[l] = v.F[x * LW + l];
    // The store depends on the loaded value, so it cannot overtake the load.
    if (sp && lane == 0)
#pragma unroll
      for (int l = 0; l < LW; ++l)
        if (f[l]) v.F[x * LW + l] = 0;
    const int64_t b = v.rp[x], e = v.rp[x + 1];
    for (int64_t k = b + lane; k < e; k += kWave)
      ms_push_edge<LW>(v, __builtin_nontemporal_load(v.col + k), f, sp, L);
  }

  // Small vertices: 64 per wavefront, edges dealt evenly to the lanes.
  const uint32_t n0 = load_relaxed32(&v.ctl->qn[cur][0]);
  for (uint64_t base = gwave * kWave; base < n0; base += nwaves * kWave) {
    const uint64_t i = base + lane;
    int64_t start = 0;
    int32_t deg = 0;  // tier-0 degrees are below 2^23 (small_bin <= 24)
    bool sp = false;
    uint64_t f[LW];
#pragma unroll
    for (int l = 0; l < LW; ++l) f[l] = 0;
    if (i < n0) {
      const int64_t x = v.q0[cur][i];
      start = v.rp[x];
      deg = (int32_t)(v.rp[x + 1] - start);
      sp = (sparse_mask >> ms_graph_of(v, x, s_off)) & 1u;
#pragma unroll
      for (int l = 0; l < LW; ++l) f[l] = v.F[x * LW + l];
      if (sp)
#pragma unroll
        for (int l = 0; l < LW; ++l)
          if (f[l]) v.F[x * LW + l] = 0;
    }
    const int32_t incl = wave_incl_scan32(deg);
    const int32_t total = __shfl(incl, kWave - 1);
    // edge e belongs to the first lane k with incl[k] > e; its column index is
    // col[start[k] - excl[k] + e]
    const int64_t rebase = start - (int64_t)(incl - deg);
    const int spi = sp ? 1 : 0;
    for (int32_t e0 = 0; e0 < total; e0 += kWave) {
      const int32_t e = e0 + lane;
      int k = 0;
#pragma unroll
      for (int step = 32; step >= 1; step >>= 1)
        if (__shfl(incl, k + step - 1) <= e) k += step;
      k = min(k, kWave - 1);
      const int64_t rk = shfl64(rebase, k);
      const bool spk = __shfl(spi, k) != 0;
      uint64_t fk[LW];
#pragma unroll
      for (int l = 0; l < LW; ++l) fk[l] = (uint64_t)shfl64((int64_t)f[l], k);
      if (e < total) ms_push_edge<LW>(v, __builtin_nontemporal_load(v.col + rk + e), fk, spk, L);
    }
  }
}

// Sweep state shared by the dense and sparse passes of one workgroup.
struct MsSweepShared {
  uint64_t s_or[kMsMaxGraphs * kMsMaxLW];
  uint64_t s_gact[kMsMaxGraphs];
  uint32_t s_cnt[kWavesPerBlock][3];
  uint64_t s_chunks[kWavesPerBlock];
  uint32_t s_base[3];
  uint64_t s_cbase;
  int32_t s_g;
};

// New bits of flat vertex x (graph g, local id xl): S, F and N updates,
// per-slot distances, and whether x is active in the next level.
template <int LW>
__device__ __forceinline__ bool ms_update_vertex(const MsView &v, int L, bool valid, int64_t x,
                                                 int g, int64_t xl, MsSweepShared &sh,
                                                 bool uniform_graph) {
  const int lane = lane_id();
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
  // Distances: loop over the slot bits present in the wavefront; lanes that
  // hold a bit write their vertex's entry of that slot's output.
#pragma unroll
  for (int l = 0; l < LW; ++l) {
    if (uniform_graph) {
      const uint64_t wor = wave_or(nw[l]);
      if (wor && lane == 0) atomicOr((unsigned long long *)&sh.s_or[g * LW + l], (unsigned long long)wor);
    } else if (nw[l]) {
      atomicOr((unsigned long long *)&sh.s_or[g * LW + l], (unsigned long long)nw[l]);
    }
    uint64_t wor = wave_or(nw[l]);
    if (uniform_graph && wor) {
      // one graph: lane k holds slot k's start level, output and type, and
      // each slot bit reads them from that lane (no memory wait per bit)
      const int sbase = (g * LW + l) * 64;
      const int32_t my_start = v.slot_start[sbase + lane];
      const uint64_t my_out = v.slot_out[sbase + lane];
      const int32_t my_type = v.slot_type[sbase + lane];
      while (wor) {
        const int b = __ffsll((unsigned long long)wor) - 1;
        wor &= wor - 1;
        const int32_t val = L + 1 - __builtin_amdgcn_readlane(my_start, b);
        const uint64_t ptr = readlane64(my_out, b);
        const int32_t type = __builtin_amdgcn_readlane(my_type, b);
        if ((nw[l] >> b) & 1ull) {
          // outputs are device memory: global stores, not generic (flat) ones
          if (type == 0) {
            if (val > 254) atomic_or64(&v.depth_err[g * LW + l], 1ull << b);
            else ((__attribute__((address_space(1))) uint8_t *)ptr)[xl] = (uint8_t)val;
          } else if (type == 1) {
            ((__attribute__((address_space(1))) int32_t *)ptr)[xl] = val;
          }
        }
      }
      continue;
    }
    while (wor) {
      const int b = __ffsll((unsigned long long)wor) - 1;
      wor &= wor - 1;
      if ((nw[l] >> b) & 1ull) {
        const int slot = (g * LW + l) * 64 + b;
        const int32_t val = L + 1 - v.slot_start[slot];
        const uint64_t ptr = v.slot_out[slot];
        // outputs are device memory: global stores, not generic (flat) ones
        const int32_t type = v.slot_type[slot];
        if (type == 0) {
          if (val > 254) atomic_or64(&v.depth_err[g * LW + l], 1ull << b);
          else ((__attribute__((address_space(1))) uint8_t *)ptr)[xl] = (uint8_t)val;
        } else if (type == 1) {
          ((__attribute__((address_space(1))) int32_t *)ptr)[xl] = val;
        }
      }
    }
  }
  return any;
}

// Compacts the active lanes of the workgroup into the next level's tier
// queues (one atomic per tier per workgroup step). All threads must call it.
__device__ __forceinline__ uint64_t ms_compact(const MsView &v, int nxt, bool any, int64_t x,
                                              MsSweepShared &sh) {
  const int lane = lane_id();
  const int wave = threadIdx.x / kWave;
  const int cs = v.chunk_shift;
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
    sh.s_cnt[wave][0] = (uint32_t)__popcll(m0);
    sh.s_cnt[wave][1] = (uint32_t)__popcll(m1);
    sh.s_cnt[wave][2] = (uint32_t)__popcll(m2);
    sh.s_chunks[wave] = wchunks;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    uint32_t t0 = 0, t1 = 0, t2 = 0;
    uint64_t ch = 0;
    for (int w = 0; w < kWavesPerBlock; ++w) {
      t0 += sh.s_cnt[w][0];
      t1 += sh.s_cnt[w][1];
      t2 += sh.s_cnt[w][2];
      ch += sh.s_chunks[w];
    }
    sh.s_base[0] = t0 ? atomic_add32(&v.ctl->qn[nxt][0], t0) : 0u;
    sh.s_base[1] = t1 ? atomic_add32(&v.ctl->qn[nxt][1], t1) : 0u;
    if (t2) {
      const uint64_t old = atomic_add64(&v.ctl->heavy[nxt], ((uint64_t)t2 << kHeavyShift) | ch);
      sh.s_base[2] = (uint32_t)(old >> kHeavyShift);
      sh.s_cbase = old & kChunkMask;
    } else {
      sh.s_base[2] = 0;
      sh.s_cbase = 0;
    }
  }
  __syncthreads();
  uint32_t b0 = sh.s_base[0], b1 = sh.s_base[1], b2 = sh.s_base[2];
  uint64_t cb = sh.s_cbase;
  for (int w = 0; w < wave; ++w) {
    b0 += sh.s_cnt[w][0];
    b1 += sh.s_cnt[w][1];
    b2 += sh.s_cnt[w][2];
    cb += sh.s_chunks[w];
  }
  if ((m0 >> lane) & 1ull) v.q0[nxt][b0 + rank_below(m0)] = (int32_t)x;
  if ((m1 >> lane) & 1ull) v.q1[nxt][b1 + rank_below(m1)] = (int32_t)x;
  if ((m2 >> lane) & 1ull) {
    const uint32_t slot = b2 + rank_below(m2);
    v.q2[nxt][slot] = (int32_t)x;
    v.cstart[nxt][slot] = (uint32_t)(cb + (uint64_t)(ncin - nc));
  }
  __syncthreads();
  return (uint64_t)__popcll(m0 | m1 | m2);
}

template <int LW>
__device__ void ms_sweep_phase(const MsView &v, int L, uint32_t vb_id, uint32_t nvb,
                               const int64_t *s_off, uint32_t sparse_mask) {
  __shared__ MsSweepShared sh;
  const int cur = L & 1, nxt = cur ^ 1;
  const int lane = lane_id();
  const int nslotw = v.ng * LW;

  if (vb_id == 0 && threadIdx.x == 0) {
    v.ctl->qn[cur][0] = 0;
    v.ctl->qn[cur][1] = 0;
    v.ctl->heavy[cur] = 0;
    v.ctl->nextra = 0;
    v.ctl->ntouched[nxt] = 0;
    v.ctl->active[(L + 1) % 3] = 0;
  }
  if (vb_id == 0) {
    for (int i = threadIdx.x; i < nslotw; i += kBlock) v.newmask[((L + 1) % 3) * nslotw + i] = 0;
    for (int i = threadIdx.x; i < kMsMaxGraphs; i += kBlock) v.ctl->gactive[(L + 1) % 3][i] = 0;
  }
  for (int i = threadIdx.x; i < nslotw; i += kBlock) sh.s_or[i] = 0;
  for (int i = threadIdx.x; i < kMsMaxGraphs; i += kBlock) sh.s_gact[i] = 0;
  __syncthreads();

  // Sparse graphs: heavy vertices of this level keep their frontier words
  // only if they were touched again (then the touched pass rewrites them).
  if (sparse_mask) {
    const uint64_t hv = load_relaxed64(&v.ctl->heavy[cur]);
    const uint32_t n2 = (uint32_t)(hv >> kHeavyShift);
    for (uint32_t i = vb_id * kBlock + threadIdx.x; i < n2; i += nvb * kBlock) {
      const int64_t x = v.q2[cur][i];
      if (((sparse_mask >> ms_graph_of(v, x, s_off)) & 1u) && v.mark[x] != L)
#pragma unroll
        for (int l = 0; l < LW; ++l) v.F[x * LW + l] = 0;
    }
  }

  uint64_t my_active = 0;
  // Dense graphs: every vertex, in chunks that never straddle two graphs.
  if (sparse_mask != (1u << v.ng) - 1u) {
    for (int64_t c = vb_id; c < v.nchunks; c += nvb) {
      if (threadIdx.x == 0) {
        int g = 0;
        while (g + 1 < v.ng && v.graphs[g + 1].chunk_begin <= c) ++g;
        sh.s_g = g;
      }
      __syncthreads();
      const int g = sh.s_g;
      if ((sparse_mask >> g) & 1u) {
        __syncthreads();
        continue;
      }
      const MsGraph gr = v.graphs[g];
      const int64_t xl = (c - gr.chunk_begin) * kMsChunk + threadIdx.x;
      const bool valid = xl < gr.n;
      const int64_t x = gr.off + xl;
      const bool any = ms_update_vertex<LW>(v, L, valid, x, g, xl, sh, true);
      const uint64_t a = ms_compact(v, nxt, any, x, sh);
      if (lane == 0 && a) atomicAdd((unsigned long long *)&sh.s_gact[g], (unsigned long long)a);
      my_active += (lane == 0) ? a : 0ull;
    }
  }
  // Sparse graphs: only the vertices the expansion touched.
  if (sparse_mask) {
    const uint32_t nt = load_relaxed32(&v.ctl->ntouched[cur]);
    for (uint32_t base = vb_id * kBlock; base < nt; base += nvb * kBlock) {
      const uint32_t i = base + threadIdx.x;
      const bool valid = i < nt;
      int64_t x = 0, xl = 0;
      int g = 0;
      if (valid) {
        x = v.touched[i];
        g = ms_graph_of(v, x, s_off);
        xl = x - s_off[g];
      }
      const bool any = ms_update_vertex<LW>(v, L, valid, x, g, xl, sh, false);
      if (any) atomicAdd((unsigned long long *)&sh.s_gact[g], 1ull);
      const uint64_t a = ms_compact(v, nxt, any, x, sh);
      my_active += (lane == 0) ? a : 0ull;
    }
  }
  __syncthreads();
  // Flush this workgroup's slot masks and active counts.
  for (int i = threadIdx.x; i < nslotw; i += kBlock)
    if (sh.s_or[i]) atomic_or64(&v.newmask[(L % 3) * nslotw + i], sh.s_or[i]);
  for (int i = threadIdx.x; i < v.ng; i += kBlock)
    if (sh.s_gact[i]) atomic_add64(&v.ctl->gactive[L % 3][i], sh.s_gact[i]);
  const uint64_t wa = (uint64_t)wave_sum((int64_t)my_active);
  if (lane == 0 && wa) atomic_add64(&v.ctl->active[L % 3], wa);
}

template <int LW>
__global__ void __launch_bounds__(kBlock) k_ms_persistent(MsView v, int max_levels) {
  __shared__ int64_t s_off[kMsMaxGraphs];
  __shared__ int64_t s_n[kMsMaxGraphs];
  const uint32_t nb = gridDim.x;
  for (int i = threadIdx.x; i < v.ng; i += kBlock) {
    s_off[i] = v.graphs[i].off;
    s_n[i] = v.graphs[i].n;
  }
  __syncthreads();
  int L = load_relaxed_i32(&v.ctl->level);
  int run = 0, sparse_levels = 0;
  bool early = false;
  for (;;) {
    // Mode of each graph for this level, from its active count (identical in
    // every block: the counts are final after the previous barrier).
    uint32_t sparse_mask = 0;
    for (int g = 0; g < v.ng; ++g) {
      const uint64_t a = load_relaxed64(&v.ctl->gactive[(L + 2) % 3][g]);
      if ((a << v.sparse_shift) < (uint64_t)s_n[g]) sparse_mask |= 1u << g;
    }
    sparse_levels += sparse_mask ? 1 : 0;
    ms_push_phase<LW>(v, L, blockIdx.x, nb, s_off, sparse_mask);
    grid_barrier(&v.ctl->bar, nb);
    ms_sweep_phase<LW>(v, L, blockIdx.x, nb, s_off, sparse_mask);
    grid_barrier(&v.ctl->bar, nb);
    ++run;
    const uint64_t act = load_relaxed64(&v.ctl->active[L % 3]);
    const int tripped = __hip_atomic_load(&v.ctl->bar.tripped, __ATOMIC_RELAXED,
                                          __HIP_MEMORY_SCOPE_AGENT);
    bool stop = act == 0 || tripped || run >= max_levels;
    if (!stop && v.stream_stop) {
      const int nslotw = v.ng * LW;
      for (int i = 0; i < nslotw; ++i)
        if (v.stop_slots[i] & ~load_relaxed64(&v.newmask[(L % 3) * nslotw + i])) {
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
    v.ctl->sparse_levels = sparse_levels;
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
  if (a.type == 2) return;  // output discarded
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
  else if (a.type == 1) ((int32_t *)a.out)[a.src_local] = 0;
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
