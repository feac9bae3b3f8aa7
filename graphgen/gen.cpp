// Seeded synthetic graph inputs: R-MAT (Kronecker initiator) graphs and 2D grids
// with random edge deletions, cleaned into symmetric CSR (undirected conversion
// with self-loops and duplicate edges removed, as in the paper's input
// preparation, Section 4 "Inputs").
//
// This module is input preparation only. It holds none of the BFS arithmetic and
// is the single place where both the oracle and the GPU path get their graphs.
//
// Random numbers come from a counter-based generator (SplitMix64 finaliser,
// Steele/Lea/Flood 2014) so every sample can be produced independently and in
// parallel from (seed, counter).
//
// Build: g++ -O3 -fopenmp -shared -fPIC gen.cpp -o libgraphgen.so

#include <algorithm>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <omp.h>
#include <vector>

namespace {

// One line on stderr per construction phase for very large graphs.
void phase(int64_t n, const char *what) {
  if (n >= (1ll << 26)) {
    fprintf(stderr, "[graphgen] %s\n", what);
    fflush(stderr);
  }
}

inline uint64_t splitmix64(uint64_t x) {
  x += 0x9E3779B97F4A7C15ull;
  x = (x ^ (x >> 30)) * 0xBF58476D1CE4E5B9ull;
  x = (x ^ (x >> 27)) * 0x94D049BB133111EBull;
  return x ^ (x >> 31);
}

// One 64-bit draw for (seed, stream, counter).
inline uint64_t draw(uint64_t seed, uint64_t stream, uint64_t ctr) {
  return splitmix64(seed ^ splitmix64(stream * 0xD1B54A32D192ED03ull + ctr));
}

struct Graph {
  int64_t n = 0;
  int64_t m = 0;
  int64_t *row_ptr = nullptr;  // n+1
  int32_t *col = nullptr;      // m
};

// Random permutation of [0,n) by Fisher-Yates driven by the counter generator.
void make_perm(int64_t n, uint64_t seed, uint32_t *perm) {
  for (int64_t i = 0; i < n; ++i) perm[i] = (uint32_t)i;
  for (int64_t i = n - 1; i > 0; --i) {
    uint64_t r = draw(seed, 7, (uint64_t)i);
    int64_t j = (int64_t)(r % (uint64_t)(i + 1));
    std::swap(perm[i], perm[j]);
  }
}

// Edge sample i of an R-MAT graph: `scale` quadrant choices, two choices per
// 64-bit draw (32 bits each compared against the cumulative initiator).
inline void rmat_sample(uint64_t seed, int scale, uint32_t tA, uint32_t tAB, uint32_t tABC,
                        uint64_t i, uint32_t &u, uint32_t &v) {
  uint32_t uu = 0, vv = 0;
  uint64_t r = 0;
  for (int b = 0; b < scale; ++b) {
    uint32_t x;
    if ((b & 1) == 0) {
      r = draw(seed, 1, i * 32ull + (uint64_t)(b >> 1));
      x = (uint32_t)r;
    } else {
      x = (uint32_t)(r >> 32);
    }
    // Quadrant: [0,A) -> (0,0), [A,A+B) -> (0,1), [A+B,A+B+C) -> (1,0), else (1,1).
    uint32_t ub = x >= tAB;
    uint32_t vb = (uint32_t)(x >= tA) ^ ub ^ (uint32_t)(x >= tABC);
    uu = (uu << 1) | ub;
    vv = (vv << 1) | vb;
  }
  u = uu;
  v = vv;
}

inline uint32_t prob_to_u32(double p) {
  if (p <= 0) return 0;
  if (p >= 1) return 0xFFFFFFFFu;
  return (uint32_t)(p * 4294967296.0);
}

// Build symmetric, sorted, duplicate-free, self-loop-free CSR from an edge
// source. `emit(i, u, v)` returns false for a sample that must be dropped.
// Directed pairs are bucketed by the high bits of their source vertex with
// per-thread counts (no shared counters, so hub vertices cause no contention),
// then each bucket is sorted and deduplicated on its own.
template <class Emit>
Graph *build_csr(int64_t n, int64_t nsamples, Emit emit) {
  Graph *g = new (std::nothrow) Graph();
  if (!g) return nullptr;
  g->n = n;
  int shift = 0;
  while ((n >> shift) > (1 << 15)) ++shift;           // bucket = v >> shift
  int64_t nb = (n >> shift) + 1;
  int nt = omp_get_max_threads();
  std::vector<int64_t> cnt((size_t)nt * (size_t)nb, 0);
  // Pass 1: per-thread bucket counts (both directions).
#pragma omp parallel num_threads(nt)
  {
    int t = omp_get_thread_num();
    int64_t *c = cnt.data() + (size_t)t * (size_t)nb;
    int64_t lo = nsamples * t / nt, hi = nsamples * (t + 1) / nt;
    for (int64_t i = lo; i < hi; ++i) {
      uint32_t u, v;
      if (!emit(i, u, v) || u == v) continue;
      c[u >> shift]++;
      c[v >> shift]++;
    }
  }
  phase(n, "counted");
  std::vector<int64_t> boff((size_t)nb + 1);
  int64_t acc = 0;
  for (int64_t b = 0; b < nb; ++b) {
    boff[b] = acc;
    for (int t = 0; t < nt; ++t) {
      int64_t x = cnt[(size_t)t * nb + b];
      cnt[(size_t)t * nb + b] = acc;
      acc += x;
    }
  }
  boff[nb] = acc;
  uint64_t *pairs = (uint64_t *)malloc(sizeof(uint64_t) * (size_t)std::max<int64_t>(acc, 1));
  if (!pairs) { delete g; return nullptr; }
  // Pass 2: scatter (src << 32 | dst) into bucket regions.
#pragma omp parallel num_threads(nt)
  {
    int t = omp_get_thread_num();
    int64_t *c = cnt.data() + (size_t)t * (size_t)nb;
    int64_t lo = nsamples * t / nt, hi = nsamples * (t + 1) / nt;
    for (int64_t i = lo; i < hi; ++i) {
      uint32_t u, v;
      if (!emit(i, u, v) || u == v) continue;
      pairs[c[u >> shift]++] = ((uint64_t)u << 32) | v;
      pairs[c[v >> shift]++] = ((uint64_t)v << 32) | u;
    }
  }
  phase(n, "scattered");
  // Sort + dedup each bucket; count unique entries per source vertex.
  std::vector<int64_t> deg((size_t)n + 1, 0);
  std::vector<int64_t> bkeep((size_t)nb, 0);
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
  for (int64_t b = 0; b < nb; ++b) {
    uint64_t *s = pairs + boff[b], *e = pairs + boff[b + 1];
    std::sort(s, e);
    uint64_t *k = std::unique(s, e);
    bkeep[b] = k - s;
    for (uint64_t *p = s; p < k; ++p) deg[*p >> 32]++;
  }
  phase(n, "sorted");
  g->row_ptr = (int64_t *)malloc(sizeof(int64_t) * (size_t)(n + 1));
  if (!g->row_ptr) { free(pairs); delete g; return nullptr; }
  acc = 0;
  for (int64_t r = 0; r < n; ++r) { g->row_ptr[r] = acc; acc += deg[r]; }
  g->row_ptr[n] = acc;
  g->m = acc;
  g->col = (int32_t *)malloc(sizeof(int32_t) * (size_t)std::max<int64_t>(acc, 1));
  if (!g->col) { free(pairs); free(g->row_ptr); delete g; return nullptr; }
#pragma omp parallel for schedule(dynamic, 1) num_threads(nt)
  for (int64_t b = 0; b < nb; ++b) {
    const uint64_t *s = pairs + boff[b];
    int64_t k = bkeep[b];
    if (k == 0) continue;
    int32_t *dst = g->col + g->row_ptr[s[0] >> 32];
    for (int64_t j = 0; j < k; ++j) dst[j] = (int32_t)(uint32_t)s[j];
  }
  free(pairs);
  return g;
}

}  // namespace

extern "C" {

// R-MAT graph with 2^scale vertices and edge_factor * 2^scale undirected samples.
// Initiator (a, b, c, 1-a-b-c). Vertex labels are permuted with `perm_seed`.
// Returns an opaque handle or NULL on allocation failure.
void *gg_rmat(int scale, int edge_factor, double a, double b, double c, uint64_t seed,
              uint64_t perm_seed, int nthreads) {
  if (scale < 1 || scale > 31 || edge_factor < 1) return nullptr;
  if (nthreads > 0) omp_set_num_threads(nthreads);
  int64_t n = (int64_t)1 << scale;
  int64_t ns = (int64_t)edge_factor * n;
  std::vector<uint32_t> perm((size_t)n);
  make_perm(n, perm_seed, perm.data());
  uint32_t tA = prob_to_u32(a), tAB = prob_to_u32(a + b), tABC = prob_to_u32(a + b + c);
  const uint32_t *P = perm.data();
  auto emit = [=](int64_t i, uint32_t &u, uint32_t &v) {
    uint32_t x, y;
    rmat_sample(seed, scale, tA, tAB, tABC, (uint64_t)i, x, y);
    u = P[x];
    v = P[y];
    return true;
  };
  return build_csr(n, ns, emit);
}

// W x H 4-neighbour grid, vertex id = y*W + x, each undirected edge deleted
// independently with probability p_del. Edge index: horizontal edges first
// (y*(W-1)+x), then vertical (H*(W-1) + y*W + x).
void *gg_grid(int64_t W, int64_t H, double p_del, uint64_t seed, int nthreads) {
  if (W < 1 || H < 1 || W * H > 0x7fffffffll) return nullptr;
  if (nthreads > 0) omp_set_num_threads(nthreads);
  int64_t nh = H * (W - 1), nv = (H - 1) * W;
  uint64_t thr = (uint64_t)(p_del * 18446744073709551616.0);
  if (p_del >= 1.0) thr = ~0ull;
  auto emit = [=](int64_t i, uint32_t &u, uint32_t &v) {
    if (p_del > 0 && draw(seed, 3, (uint64_t)i) < thr) return false;
    if (i < nh) {
      int64_t y = i / (W - 1), x = i % (W - 1);
      u = (uint32_t)(y * W + x);
      v = (uint32_t)(y * W + x + 1);
    } else {
      int64_t j = i - nh;
      int64_t y = j / W, x = j % W;
      u = (uint32_t)(y * W + x);
      v = (uint32_t)((y + 1) * W + x);
    }
    return true;
  };
  return build_csr(W * H, nh + nv, emit);
}

// Symmetric CSR from an explicit list of undirected edges (u[i], v[i]).
void *gg_from_edges(int64_t n, int64_t ne, const int64_t *u, const int64_t *v) {
  if (n < 0 || n > 0x7fffffffll) return nullptr;
  for (int64_t i = 0; i < ne; ++i)
    if (u[i] < 0 || u[i] >= n || v[i] < 0 || v[i] >= n) return nullptr;
  auto emit = [=](int64_t i, uint32_t &a, uint32_t &b) {
    a = (uint32_t)u[i];
    b = (uint32_t)v[i];
    return true;
  };
  return build_csr(n, ne, emit);
}

int64_t gg_n(void *h) { return h ? ((Graph *)h)->n : -1; }
int64_t gg_m(void *h) { return h ? ((Graph *)h)->m : -1; }

// Copies the CSR into caller buffers (row_ptr: n+1 entries, col: m entries).
void gg_copy(void *h, int64_t *row_ptr, int32_t *col) {
  Graph *g = (Graph *)h;
  memcpy(row_ptr, g->row_ptr, sizeof(int64_t) * (size_t)(g->n + 1));
  memcpy(col, g->col, sizeof(int32_t) * (size_t)g->m);
}

void gg_free(void *h) {
  Graph *g = (Graph *)h;
  if (!g) return;
  free(g->row_ptr);
  free(g->col);
  delete g;
}

// Uniform draws for seeded choices made outside the generator (sources,
// arrival gaps): out[i] = draw(seed, 5, i) for i in [0, cnt).
void gg_draws(uint64_t seed, int64_t cnt, uint64_t *out) {
  for (int64_t i = 0; i < cnt; ++i) out[i] = draw(seed, 5, (uint64_t)i);
}

}  // extern "C"
