// bfs_run_noalloc: a single-source traversal of a small whole graph that
// allocates nothing, for callers that cannot allocate device memory (code
// under HIP graph capture, tight serving loops). It is the one-workgroup
// level loop of bfs_run (BFS_LOOP_CU: both bitmaps in LDS, Algorithm 1 with
// workgroup barriers between Phase 1 and Phase 2) with its device scratch --
// the control block and the two frontier queues -- in a file-scope device
// array of fixed size (8 MiB) instead of a plan's workspace. Every call on a device
// shares that device's array, so calls that overlap on one device race.

#include <hip/hip_runtime.h>

#include <mutex>
#include <string>

#include "../../include/bfs.h"
#include "bfs_core.hpp"
#include "plan.hpp"

namespace bfsk {

namespace {

constexpr int64_t kNaMaxVertices = BFS_NOALLOC_MAX_VERTICES;
constexpr int64_t kNaMaxEdges = BFS_NOALLOC_MAX_EDGES;
constexpr size_t kNaCtlBytes = (sizeof(Ctl) + 255) / 256 * 256;
constexpr size_t kNaQueueBytes = sizeof(uint64_t) * (size_t)kNaMaxVertices;
constexpr size_t kNaBytes = kNaCtlBytes + 2 * kNaQueueBytes;
constexpr int kNaMaxDevices = 64;

// Device scratch: control block, then queue buffers 0 and 1 (n packed rows each).
static __device__ __align__(256) unsigned char scratch[kNaBytes];

static_assert(kNaBytes <= BFS_NOALLOC_SCRATCH_BYTES, "scratch larger than documented");

std::mutex g_na_mu;
void *g_na_ptr[kNaMaxDevices] = {};  // device address of `scratch`, per device
int g_na_lds[kNaMaxDevices] = {};    // LDS bytes one workgroup may use, per device

// Control-block fields the one-workgroup loop reads or reports, cleared, and
// the distances reset (all infinity, the root 0). Also validates the graph:
// a bad row offset or column id sets ctl->err (bit 4), and the traversal
// kernel then does nothing.
__global__ void __launch_bounds__(256) k_na_reset(View v, int64_t src) {
  const int64_t tid = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = tid; i < v.n; i += stride) v.dist[i] = (i == src) ? 0 : -1;
  int32_t bad = 0;
  for (int64_t i = tid; i < v.n; i += stride)
    if (v.rp[i + 1] < v.rp[i]) bad = 1;
  for (int64_t e = tid; e < v.m; e += stride) {
    const int32_t u = v.col[e];
    if (u < 0 || (int64_t)u >= v.n) bad = 1;
  }
  if (tid == 0 && (v.rp[0] != 0 || v.rp[v.n] != v.m)) bad = 1;
  if (bad) atomicOr(&v.ctl->err, 4);
}

__global__ void k_na_clear(Ctl *c) {
  if (threadIdx.x == 0) {
    c->levels = 0;
    c->reached = 0;
    c->edges = 0;
    c->err = 0;
  }
}

// The device address of `scratch` on the current device and that device's
// LDS limit per workgroup (looked up once per device).
bfs_status scratch_ptr(void **out, int *max_lds, std::string &err) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) {
    err = std::string("hipGetDevice: ") + hipGetErrorString(e);
    return BFS_ERR_HIP;
  }
  if (dev < 0 || dev >= kNaMaxDevices) {
    err = "device ordinal out of range";
    return BFS_ERR_HIP;
  }
  std::lock_guard<std::mutex> lk(g_na_mu);
  if (!g_na_ptr[dev]) {
    void *p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || !p) {
      err = std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e);
      return BFS_ERR_HIP;
    }
    int lds = 0;
    e = hipDeviceGetAttribute(&lds, hipDeviceAttributeMaxSharedMemoryPerBlock, dev);
    if (e != hipSuccess) {
      err = std::string("hipDeviceGetAttribute: ") + hipGetErrorString(e);
      return BFS_ERR_HIP;
    }
    g_na_ptr[dev] = p;
    g_na_lds[dev] = lds;
  }
  *out = g_na_ptr[dev];
  *max_lds = g_na_lds[dev];
  return BFS_OK;
}

}  // namespace
}  // namespace bfsk

using namespace bfsk;

extern "C" bfs_status bfs_run_noalloc(const bfs_graph *g, int64_t source, int32_t *dist,
                                      void *hip_stream, int32_t *levels) {
  if (!g || !dist) {
    set_create_error("graph or dist is NULL");
    return BFS_ERR_ARG;
  }
  if (g->n_global <= 0 || g->v_begin != 0 || g->v_end != g->n_global || g->m < 0 || !g->row_ptr ||
      (g->m > 0 && !g->col)) {
    set_create_error("bfs_run_noalloc needs a whole graph (v_begin 0, v_end n_global) with valid pointers");
    return BFS_ERR_ARG;
  }
  if (g->n_global > kNaMaxVertices || g->m >= kNaMaxEdges) {
    set_create_error("bfs_run_noalloc takes graphs of at most " + std::to_string(kNaMaxVertices) +
                     " vertices and fewer than " + std::to_string(kNaMaxEdges) + " edges (got n=" +
                     std::to_string(g->n_global) + ", m=" + std::to_string(g->m) + ")");
    return BFS_ERR_CAPACITY;
  }
  if (source < 0 || source >= g->n_global) {
    set_create_error("source outside [0, n_global)");
    return BFS_ERR_ARG;
  }
  std::string err;
  void *base = nullptr;
  int max_lds = 0;
  bfs_status st = scratch_ptr(&base, &max_lds, err);
  if (st) {
    set_create_error(err);
    return st;
  }
  if (!cu_fits(g->n_global, g->m, true, max_lds)) {
    set_create_error("bfs_run_noalloc: the graph's two bitmaps do not fit one workgroup's LDS");
    return BFS_ERR_CAPACITY;
  }
  hipStream_t s = (hipStream_t)hip_stream;
  View v{};
  v.n = g->n_global;
  v.vb = 0;
  v.ve = g->n_global;
  v.m = g->m;
  v.words = (g->n_global + 63) / 64;
  v.rp = g->row_ptr;
  v.col = g->col;
  v.dist = dist;
  v.live_end = g->n_global;
  char *b = (char *)base;
  v.ctl = (Ctl *)b;
  v.qr0[0] = (uint64_t *)(b + kNaCtlBytes);
  v.qr0[1] = (uint64_t *)(b + kNaCtlBytes + kNaQueueBytes);
  hipLaunchKernelGGL(k_na_clear, dim3(1), dim3(64), 0, s, v.ctl);
  hipError_t e = hipGetLastError();
  const int grid = (int)std::min<int64_t>(std::max<int64_t>((v.n + 255) / 256, 1), 1024);
  if (e == hipSuccess) {
    hipLaunchKernelGGL(k_na_reset, dim3(grid), dim3(256), 0, s, v, source);
    e = hipGetLastError();
  }
  const int max_levels = (int)std::min<int64_t>(g->n_global + 1, 1ll << 30);
  if (e == hipSuccess) e = launch_bfs_cu(v, source, max_levels, s);
  Ctl c{};
  if (e == hipSuccess) e = hipMemcpyAsync(&c, v.ctl, sizeof(Ctl), hipMemcpyDeviceToHost, s);
  if (e == hipSuccess) e = hipStreamSynchronize(s);
  if (e != hipSuccess) {
    set_create_error(std::string("bfs_run_noalloc: ") + hipGetErrorString(e));
    return BFS_ERR_HIP;
  }
  if (c.err & 4) {
    set_create_error("bfs_run_noalloc: invalid graph (row offsets not monotone from 0 to m, or a "
                     "column id outside [0, n_global))");
    return BFS_ERR_ARG;
  }
  if (c.err) {
    set_create_error("bfs_run_noalloc: level limit exceeded");
    return BFS_ERR_DEVICE;
  }
  if (levels) *levels = c.levels;
  return BFS_OK;
}
