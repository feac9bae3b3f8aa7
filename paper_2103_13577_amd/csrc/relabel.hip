// Plan-time relabelling of a whole graph by descending degree.
//
// The paper leaves vertex relabelling to future work (Section 4, "Graph
// Partitioning"). On gfx950 it pays for the top-down probes: most edge
// endpoints of a power-law graph are hubs, and after relabelling the hubs'
// visited bits sit in the first few KB of the bitmap, where they stay in the
// vector L1 of every CU. Each adjacency list is also sorted by new id, so the
// probes of one wavefront fall into few cache lines.
//
// New id i is the i-th vertex in (degree descending, old id ascending)
// order. The traversal runs on the relabelled copy; distances are written
// through old_id[] so the caller always sees original labels.

#include <hip/hip_runtime.h>
#include <hipcub/hipcub.hpp>

#include "relabel.hpp"

namespace bfsk {

namespace {

// key = ((maxdeg - deg) << 32) | old id : ascending key order is the new order.
__global__ void k_rl_keys(const int64_t *rp, int64_t n, uint64_t *keys) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t v = tid; v < n; v += stride) {
    const uint64_t d = (uint64_t)(rp[v + 1] - rp[v]);
    keys[v] = ((0xFFFFFFFFull - d) << 32) | (uint64_t)v;
  }
}

__global__ void k_rl_maps(const uint64_t *sorted, int64_t n, const int64_t *rp, int32_t *old_id,
                          int32_t *new_id, int64_t *new_deg) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = tid; i < n; i += stride) {
    const int32_t v = (int32_t)(uint32_t)sorted[i];
    old_id[i] = v;
    new_id[v] = (int32_t)i;
    new_deg[i] = rp[v + 1] - rp[v];
  }
  if (tid == 0) new_deg[n] = 0;
}

// One wavefront per new vertex copies its row with targets renamed.
__global__ void k_rl_rows(const int64_t *rp, const int32_t *col, int64_t n, const int32_t *old_id,
                          const int32_t *new_id, const int64_t *new_rp, int32_t *tmp_col) {
  const int64_t gw = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) / 64;
  const int64_t nw = ((int64_t)gridDim.x * blockDim.x) / 64;
  const int lane = threadIdx.x & 63;
  for (int64_t i = gw; i < n; i += nw) {
    const int32_t v = old_id[i];
    const int64_t b = rp[v], d = rp[v + 1] - b, o = new_rp[i];
    for (int64_t k = lane; k < d; k += 64) tmp_col[o + k] = new_id[col[b + k]];
  }
}

int grid_for(int64_t work) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((work + 255) / 256, 16384));
}

}  // namespace

RelabelSizes relabel_sizes(int64_t n, int64_t m) {
  RelabelSizes s{};
  size_t t1 = 0, t2 = 0, t3 = 0;
  uint64_t *kn = nullptr;
  int64_t *in = nullptr;
  int32_t *cn = nullptr;
  (void)hipcub::DeviceRadixSort::SortKeys(nullptr, t1, kn, kn, (int)n);
  (void)hipcub::DeviceScan::ExclusiveSum(nullptr, t2, in, in, (int)(n + 1));
  (void)hipcub::DeviceSegmentedRadixSort::SortKeys(nullptr, t3, cn, cn, (int)m, (int)n, in, in + 1);
  s.temp = std::max(t1, std::max(t2, t3));
  s.keys = sizeof(uint64_t) * (size_t)(n + 1);
  s.tmp_col = sizeof(int32_t) * (size_t)std::max<int64_t>(m, 1);
  return s;
}

hipError_t relabel_build(const int64_t *rp, const int32_t *col, int64_t n, int64_t m,
                         int64_t *new_rp, int32_t *new_col, int32_t *old_id, int32_t *new_id,
                         void *keys_a, void *keys_b, void *tmp_col, void *temp, size_t temp_bytes,
                         hipStream_t s) {
  uint64_t *ka = (uint64_t *)keys_a, *kb = (uint64_t *)keys_b;
  hipLaunchKernelGGL(k_rl_keys, dim3(grid_for(n)), dim3(256), 0, s, rp, n, ka);
  hipError_t e = hipGetLastError();
  size_t tb = temp_bytes;
  if (e == hipSuccess) e = hipcub::DeviceRadixSort::SortKeys(temp, tb, ka, kb, (int)n, 0, 64, s);
  // new_deg reuses keys_a (sized for n+1 entries)
  int64_t *new_deg = (int64_t *)keys_a;
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_rl_maps, dim3(grid_for(n)), dim3(256), 0, s, kb, n, rp, old_id, new_id,
                       new_deg);
    e = hipGetLastError();
  }
  tb = temp_bytes;
  if (e == hipSuccess) e = hipcub::DeviceScan::ExclusiveSum(temp, tb, new_deg, new_rp, (int)(n + 1), s);
  if (e == hipSuccess && m > 0) {
    hipLaunchKernelGGL(k_rl_rows, dim3(grid_for(n * 64)), dim3(256), 0, s, rp, col, n, old_id,
                       new_id, new_rp, (int32_t *)tmp_col);
    e = hipGetLastError();
    tb = temp_bytes;
    if (e == hipSuccess)
      e = hipcub::DeviceSegmentedRadixSort::SortKeys(temp, tb, (const int32_t *)tmp_col, new_col,
                                                     (int)m, (int)n, new_rp, new_rp + 1, 0, 32, s);
  }
  return e;
}

}  // namespace bfsk
