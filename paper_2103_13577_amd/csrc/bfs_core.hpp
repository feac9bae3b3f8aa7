// Shared host/device definitions of the single-source traversal: the control
// block and the view of a plan's workspace passed to every kernel.
#pragma once

#include <stdint.h>

#include "device.hpp"

namespace bfsk {

constexpr int kNumBins = 34;   // degree bin 0 (degree 0) .. 33
constexpr int kTiers = 3;      // lane-group, wavefront, chunked workgroup
constexpr int kBlock = 256;    // threads per workgroup for the traversal kernels
constexpr int kWavesPerBlock = kBlock / kWave;
constexpr int kWideBlock = 1024;      // threads per workgroup of the wide expansion
constexpr uint32_t kNarrowHotMax = 4096;  // larger LDS hub copies use the wide expansion
constexpr uint32_t kQueueOnly = 0xFFFFFFFFu;  // k_expand: run a queue-only level
constexpr uint32_t kBottomUpHot = 2048;       // frontier words a bottom-up block keeps in LDS
constexpr int64_t kDirAlpha = 14;  // top-down -> bottom-up when frontier edges * 14 > unvisited edges
constexpr int64_t kDirBeta = 24;   // bottom-up -> top-down when frontier * 24 < n and not growing
constexpr int kMaxStatLevels = 4096;
constexpr int kListMaxBlocks = 2048;  // blocks of the list export (count scratch: 2049 words)
constexpr int32_t kErrListId = 4;     // Ctl::err bit: a received list held an id outside [0, n)
constexpr int kHeavyShift = 40;  // packed heavy-tier counter: count << 40 | chunks
constexpr uint64_t kChunkMask = (1ull << kHeavyShift) - 1;

// Device control block at the start of the workspace.
constexpr int kRing = 3;  // frontier queues rotate over level mod 3

struct Ctl {
  GridBarrier bar;
  uint32_t qn[kRing][2];  // tier-0 and tier-1 queue lengths, by level mod 3
  uint64_t heavy[kRing];  // tier-2 queue: (count << 40) | total chunks, by level mod 3
  uint64_t newcnt[3];     // vertices new in the level (all ranges), by level mod 3
  uint64_t ownedcnt[3];   // owned vertices new in the level, by level mod 3
  uint64_t edges;         // sum of degrees over every enqueued owned vertex
  uint64_t reached;       // vertices with a finite distance
  int32_t levels;         // persistent loop: number of nonempty levels
  int32_t err;            // device-side error flags
  int32_t glevel;         // graph-launched loop: level the next captured step runs
  int32_t gdone;          // graph-launched loop: traversal finished
  int32_t *gdist;         // graph-launched loop: caller's distance array
  uint64_t gedges[2];     // graph-launched loop: `edges` after the merges of the last two
                          // levels ([1] newer; the current frontier's edges are the difference)
  uint64_t xedges;        // edges scanned by dense (bitmap) expansions
  uint64_t xfront;        // frontier vertices of dense expansions
  uint64_t buedges;       // adjacency entries examined by bottom-up steps
  uint64_t buverts;       // unvisited vertices examined by bottom-up steps
};

// Kernel view of a plan's workspace for one graph.
struct View {
  int64_t n;        // n_global
  int64_t vb, ve;   // owned range
  int64_t m;
  int64_t words;    // ceil(n / 64)
  const int64_t *rp;
  const int32_t *col;
  const int32_t *old_id;  // relabelled graph: traversal id -> caller id (NULL: identity)
  const int32_t *new_id;  // caller id -> traversal id (NULL: identity)
  int32_t *dist;          // indexed by caller ids
  uint64_t *visited;
  uint64_t *next;
  uint64_t *front;        // direction-optimizing traversal: frontier bitmap of the
                          // next level (the level's merged global queue), written
                          // by every merge that finishes a level (NULL: off)
  int32_t *q0[kRing];
  int32_t *q1[kRing];
  uint64_t *qr0[kRing];   // tier-0 / tier-1 queue entries' adjacency: (row start << 24) |
  uint64_t *qr1[kRing];   // degree, written with q0 / q1 (tier degrees are below 2^24)
  int32_t *q2[kRing];
  uint32_t *cstart[kRing];
  Ctl *ctl;
  int64_t *lvl_frontier;  // [kMaxStatLevels]
  uint32_t *lvl_hist;     // [kMaxStatLevels * kNumBins]
  int32_t small_bin;      // bins < small_bin -> tier 0
  int32_t wave_bin;       // bins < wave_bin -> tier 1, else tier 2
  int32_t chunk_shift;    // tier-2 work item = 2^chunk_shift edges
  int32_t stats;
  int32_t sparse_div;     // device loop: a level runs queue-only when the
                          // frontier is below words / sparse_div (0 = never)
  int32_t into_vis;       // single-node host loop without queue-only or bottom-up
                          // levels: dense expansions OR straight into `visited`
                          // and `next` holds visited as of the level's start
  int64_t live_end;       // owned vertices at or above it have no edge (a
                          // relabelled graph puts them last); else ve
  uint8_t *mark;          // single-node dense levels: one byte per vertex, set to 1 by a
                          // plain store when the expansion finds the vertex unvisited;
                          // the merge folds each word's 64 bytes into a bit mask and
                          // clears them (NULL: the expansion ORs bits atomically)
  uint64_t *hubnext;      // mark mode: hub targets (those in an expansion block's LDS copy of
                          // the hubs' visited words) found in the level, ORed in per block
                          // at the end of the expansion; the merge folds and clears it
  int32_t hub_words;      // words of hubnext the merge folds in (0: none)
};

constexpr int kMaxIncoming = 8;  // received bitmaps per merge launch
constexpr int kMaxHotWords = 20480;  // largest LDS hub copy (160 KB)

// Packed adjacency of a tier-0/1 queue entry: row start (below 2^40) and
// degree (below 2^24).
constexpr int kRowShift = 24;
__host__ __device__ __forceinline__ uint64_t pack_row(int64_t start, int64_t deg) {
  return ((uint64_t)start << kRowShift) | (uint64_t)deg;
}

// Merge modes: the ordinary merge; a merge that leaves the next level's tier
// queues unwritten (after a bottom-up step, whose successor reads the frontier
// bitmap; the step counts the new vertices' edges itself); and a pass that
// only fills those queues from the frontier bitmap, for a top-down level that
// follows such a merge.
constexpr int32_t kMergeFull = 0, kMergeNoQueues = 1, kMergeQueuesFromFront = 2;

struct MergeArgs {
  const uint64_t *inc[kMaxIncoming];  // received bitmaps (device)
  int32_t k;
  int32_t keep_next;
  int32_t level;
  int32_t mode;  // kMerge*
};

// Degree bin: 0 for degree 0, else 1 + floor(log2(degree)).
__host__ __device__ __forceinline__ int degree_bin(int64_t d) {
#ifdef __HIP_DEVICE_COMPILE__
  return d <= 0 ? 0 : 64 - __clzll((unsigned long long)d);
#else
  return d <= 0 ? 0 : 64 - __builtin_clzll((unsigned long long)d);
#endif
}

__host__ __device__ __forceinline__ int tier_of_bin(int b, int small_bin, int wave_bin) {
  return b < small_bin ? 0 : (b < wave_bin ? 1 : 2);
}

// Host launchers (bfs_kernels.hip).
hipError_t launch_reset(const View &v, int64_t src, int grid, hipStream_t s);
hipError_t launch_expand(const View &v, int level, int grid, uint32_t hot_words, hipStream_t s);
hipError_t launch_merge(const View &v, const MergeArgs &a, int grid, hipStream_t s);
hipError_t launch_clear_stats_row(const View &v, int level, hipStream_t s);
hipError_t launch_parent(const View &v, int32_t *parent, int64_t src, int grid, hipStream_t s);
hipError_t launch_persistent(const View &v, int max_levels, int grid, int variant, hipStream_t s);
// Enqueues `levels` graph-launched level steps (expand, merge, advance) on s;
// used while capturing a hipGraph. ev (NULL: none) holds three events per
// step, recorded before its expansion, after it and after its merge.
hipError_t enqueue_graph_levels(const View &v, int levels, int max_levels, int expand_grid,
                                int merge_grid, uint32_t hot_words, hipStream_t s,
                                hipEvent_t (*ev)[3] = nullptr);
int persistent_blocks_per_cu(int variant);
int expand_blocks_per_cu(uint32_t hot_words);
hipError_t launch_bottom_up(const View &v, int level, int grid, uint32_t hot_words, const uint64_t *front,
                            int count_edges, hipStream_t s);
hipError_t launch_front_from_queues(const View &v, int level, int grid, hipStream_t s);
int bottom_up_blocks_per_cu(uint32_t hot_words);
size_t cu_lds_bytes(int64_t words);
bool cu_fits(int64_t n, int64_t m, bool whole, int max_lds);
hipError_t launch_bfs_cu(const View &v, int64_t src, int max_levels, hipStream_t s);
// Vertex-list messages (frontier_list.hip). The export writes the set bits of
// bm below n, ascending, into out[0..cap) and the total into blk[nblocks]
// (blk: kListMaxBlocks + 1 words of scratch); with out NULL it only counts.
void list_geometry(int64_t words, int &nblk, int64_t &per);
hipError_t launch_list_export(const uint64_t *bm, int64_t words, int64_t n, uint64_t *blk, int32_t *out,
                              int64_t cap, hipStream_t s);
hipError_t launch_list_scatter(const int32_t *list, int64_t cnt, uint64_t *next, int64_t n, int32_t *err,
                               int max_grid, hipStream_t s);

}  // namespace bfsk
