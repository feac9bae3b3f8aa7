/*
 * Plain, slow, single-threaded CPU oracle for the BFS hot path.
 *
 * TEST INFRASTRUCTURE ONLY. Nothing on the product path may link, load or call
 * this file; only the test suite, the smoke check and the benchmark's CPU
 * baseline leg use it. It shares no code, header or table with the GPU library.
 *
 * What it computes, and the passage each function follows:
 *   oracle_bfs        - hop distance d[v] from a root r, -1 for "infinity"
 *                       (Section 2, Preliminaries; level-synchronous top-down
 *                       BFS of Algorithm 1 reaches exactly this, so the oracle
 *                       is the textbook FIFO-queue BFS).
 *   oracle_parent     - canonical parent: smallest-id neighbour one level
 *                       closer to the root (the paper defines no parent array;
 *                       this is our stated reading).
 *   oracle_stage      - butterfly frontier-synchronisation inputs for one
 *                       compute node (Section 3, Algorithm 2 Phase 1 sets and
 *                       the Phase 2 exchange schedule of Figures 1 and 2).
 *   oracle_merge      - the Phase 2 merge on bitmaps (Algorithm 2 Phase 2):
 *                       union of the incoming sets, new-vertex detection,
 *                       distance update and the owned next frontier.
 *   oracle_edges_scanned - sum of degrees over reached owned vertices (the
 *                       number of edges a top-down traversal inspects).
 *
 * Conventions: CSR row_ptr int64[n+1], col int32[m]; bitmaps are uint64 words,
 * bit v lives in word v/64 at position v%64.
 */
#include <stdint.h>
#include <stdio.h>
#include <stdlib.h>
#include <string.h>

/* Progress lines on stderr for very large inputs (one per 1/16 of the work),
 * so long runs show that they advance. */
static void progress(const char *what, int64_t done, int64_t total) {
  if (total < ((int64_t)1 << 26)) return;
  const int64_t step = total / 16;
  if (step > 0 && done % step == 0 && done > 0) {
    fprintf(stderr, "[oracle] %s %lld/16\n", what, (long long)(done / step));
    fflush(stderr);
  }
}

/* FIFO BFS. dist must hold n entries. Returns the number of reached vertices,
 * or -1 if src is out of range or memory runs out. */
int64_t oracle_bfs(int64_t n, const int64_t *row_ptr, const int32_t *col, int64_t src,
                   int32_t *dist) {
  if (src < 0 || src >= n) return -1;
  int32_t *queue = (int32_t *)malloc(sizeof(int32_t) * (size_t)n);
  if (!queue) return -1;
  for (int64_t v = 0; v < n; ++v) dist[v] = -1;
  int64_t head = 0, tail = 0;
  dist[src] = 0;
  queue[tail++] = (int32_t)src;
  while (head < tail) {
    progress("bfs", head, n);
    int32_t v = queue[head++];
    for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
      int32_t u = col[e];
      if (dist[u] == -1) {
        dist[u] = dist[v] + 1;
        queue[tail++] = u;
      }
    }
  }
  free(queue);
  return tail;
}

/* parent[v] = min{u in adj(v) : dist[u] == dist[v]-1} for reached v != root,
 * parent[root] = root, -1 for unreached vertices. */
void oracle_parent(int64_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *dist,
                   int32_t *parent) {
  for (int64_t v = 0; v < n; ++v) {
    parent[v] = -1;
    if (dist[v] == 0) {
      parent[v] = (int32_t)v;
    } else if (dist[v] > 0) {
      int32_t best = -1;
      for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
        int32_t u = col[e];
        if (dist[u] == dist[v] - 1 && (best == -1 || u < best)) best = u;
      }
      parent[v] = best;
    }
  }
}

/* Sum of degrees of reached vertices in [v_begin, v_end). */
int64_t oracle_edges_scanned(const int64_t *row_ptr_global, const int32_t *dist, int64_t v_begin,
                             int64_t v_end) {
  int64_t s = 0;
  for (int64_t v = v_begin; v < v_end; ++v)
    if (dist[v] >= 0) s += row_ptr_global[v + 1] - row_ptr_global[v];
  return s;
}

/* Owner of v under consecutive-range partitioning: the c with
 * bounds[c] <= v < bounds[c+1]. */
static int32_t owner_of(int64_t v, int32_t P, const int64_t *bounds) {
  int32_t lo = 0, hi = P - 1;
  while (lo < hi) {
    int32_t mid = (lo + hi + 1) / 2;
    if (bounds[mid] <= v) lo = mid; else hi = mid - 1;
  }
  return lo;
}

/*
 * Butterfly staging for compute node g among P = radix^depth nodes.
 *
 * Phase 1 (Algorithm 2): at level L, node c discovers
 *   X_c(L) = { u : d[u] = L+1 and some v with d[v] = L owned by c has edge (v,u) }.
 * Phase 2: in round i node g receives, from each partner that differs from g
 * only in base-`radix` digit i, that partner's global queue at the start of the
 * round, which is the union of X_c over the partner's aligned block of
 * radix^i nodes (for radix 2, round i's partner is g XOR 2^i; Section 3 walk
 * through of Figure 1: node 0 hears from 1, then 2 holding {2,3}, then 4
 * holding {4..7}, then 8 holding {8..15}).
 *
 * Every node c != g therefore lands in exactly one incoming message: the round
 * i is the most significant base-radix digit where c and g differ, and the
 * partner is the one whose digit i equals c's digit i.
 *
 * Outputs, for levels L = 0..nlev-1 (nlev = max distance, since level nlev has no
 * successors), with W = ceil(n/64) words per bitmap:
 *   local_out[L*W ...]                        = X_g(L)
 *   inc_out[(L*K + i*(radix-1) + j)*W ...]     = message from the j-th partner
 *                                                of round i (partners in
 *                                                ascending digit order, skipping
 *                                                g's own digit), K = depth*(radix-1).
 * Returns nlev, or -1 on bad arguments.
 */
int32_t oracle_stage(int64_t n, const int64_t *row_ptr, const int32_t *col, const int32_t *dist,
                     int32_t P, const int64_t *bounds, int32_t g, int32_t radix, int32_t nlev,
                     uint64_t *local_out, uint64_t *inc_out) {
  if (radix < 2 || P < 1 || g < 0 || g >= P) return -1;
  int32_t depth = 0;
  int64_t pw = 1;
  while (pw < P) { pw *= radix; ++depth; }
  if (pw != P) return -1;
  int64_t W = (n + 63) / 64;
  int32_t K = depth * (radix - 1);
  memset(local_out, 0, sizeof(uint64_t) * (size_t)(W * nlev));
  if (K > 0) memset(inc_out, 0, sizeof(uint64_t) * (size_t)(W * nlev * K));
  for (int64_t v = 0; v < n; ++v) {
    progress("stage", v, n);
    int32_t L = dist[v];
    if (L < 0 || L >= nlev) continue;
    int32_t c = owner_of(v, P, bounds);
    uint64_t *dst;
    if (c == g) {
      dst = local_out + (int64_t)L * W;
    } else {
      /* most significant differing digit i, and c's digit there */
      int32_t i = -1, digit = 0;
      int32_t cc = c, gg = g;
      for (int32_t k = 0; k < depth; ++k) {
        if (cc % radix != gg % radix) { i = k; digit = cc % radix; }
        cc /= radix;
        gg /= radix;
      }
      int32_t gdigit = g;
      for (int32_t k = 0; k < i; ++k) gdigit /= radix;
      gdigit %= radix;
      int32_t j = digit < gdigit ? digit : digit - 1;
      dst = inc_out + ((int64_t)L * K + (int64_t)i * (radix - 1) + j) * W;
    }
    for (int64_t e = row_ptr[v]; e < row_ptr[v + 1]; ++e) {
      int32_t u = col[e];
      if (dist[u] == L + 1) dst[u >> 6] |= (uint64_t)1 << (u & 63);
    }
  }
  return nlev;
}

/*
 * Frontier-synchronisation merge on bitmaps (Algorithm 2 Phase 2, all rounds of
 * one level at once). For every vertex v < n:
 *   v is "received" if its bit is set in next or in any of the k incoming maps;
 *   v is "new" if received and not yet visited;
 *   for every new v: visited gains v, dist[v] = level+1, and if
 *   v_begin <= v < v_end, v is appended to owned_queue (ascending order).
 * next is cleared afterwards unless keep_next is set, in which case next holds
 * the union of next and the incoming maps (the node's global queue).
 * Returns the number of new vertices; *owned_new gets the queue length.
 */
int64_t oracle_merge(int64_t n, int32_t level, uint64_t *next, const uint64_t *const *incoming,
                     int32_t k, uint64_t *visited, int32_t *dist, int64_t v_begin, int64_t v_end,
                     int32_t keep_next, int32_t *owned_queue, int64_t *owned_new) {
  int64_t total = 0, owned = 0;
  for (int64_t v = 0; v < n; ++v) {
    int64_t w = v >> 6;
    uint64_t bit = (uint64_t)1 << (v & 63);
    int received = (next[w] & bit) != 0;
    for (int32_t i = 0; i < k; ++i)
      if (incoming[i][w] & bit) received = 1;
    if (received && !(visited[w] & bit)) {
      visited[w] |= bit;
      dist[v] = level + 1;
      ++total;
      if (v >= v_begin && v < v_end) owned_queue[owned++] = (int32_t)v;
    }
    if (keep_next) {
      if (received) next[w] |= bit;
    }
  }
  if (!keep_next) memset(next, 0, sizeof(uint64_t) * (size_t)((n + 63) / 64));
  *owned_new = owned;
  return total;
}
