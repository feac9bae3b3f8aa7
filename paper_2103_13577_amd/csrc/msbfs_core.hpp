// Batched multi-source traversal: shared host/device definitions.
//
// All graphs of a plan are laid end to end as one disjoint union ("flat"
// graph, vertex x of graph g is off[g] + x). Each flat vertex owns LW uint64
// lane words in three arrays: F (frontier), N (next) and S (seen); bit b of
// word l of a vertex of graph g belongs to source slot (g, l, b). A level is
// Phase 1 on lane words (every active vertex ORs its frontier words into the
// next words of its neighbours, top-down) followed by a sweep that detects
// new bits (N & ~S), updates S and F, writes distances per slot and compacts
// active vertices into the next level's degree-tier queues.
#pragma once

#include <stdint.h>

#include "device.hpp"

namespace bfsk {

constexpr int kMsMaxGraphs = 16;
constexpr int kMsMaxLW = 4;
constexpr int kMsChunk = 256;  // vertices per sweep work item (one workgroup)
constexpr int kStreamLevels = 256;  // most levels of one streaming launch

struct MsGraph {
  int64_t off;          // first flat vertex
  int64_t n;            // vertices
  int64_t chunk_begin;  // first sweep chunk
};

struct MsCtl {
  GridBarrier bar;
  uint32_t qn[2][2];      // tier-0/1 queue lengths by level parity
  uint64_t heavy[2];      // tier-2: (count << 40) | chunks, by parity
  uint64_t active[3];     // active vertices after the sweep of level L, by L mod 3
  uint64_t gactive[3][kMsMaxGraphs];  // the same per graph
  uint32_t nextra;        // admitted sources to expand at the next level
  uint32_t ntouched[2];   // touched vertices of sparse-mode graphs, by level parity
  int32_t level;          // next level to run (global clock of the batch engine)
  int32_t levels_run;     // levels completed by the last launch
  int32_t stopped_early;  // last launch ended because a slot finished
  int32_t err;
  int32_t sparse_levels;  // levels of the last launch run with a sparse graph
};

struct MsView {
  int32_t ng;
  int32_t lw;
  int64_t ntot;
  int64_t nchunks;
  const int64_t *rp;  // flat row offsets [ntot+1]
  const int32_t *col; // flat column ids
  uint64_t *F, *N, *S;
  int32_t *q0[2], *q1[2], *q2[2];
  uint32_t *cstart[2];
  int32_t *extra;            // admitted sources (flat ids)
  int32_t *mark;             // [ntot] level at which a vertex was last touched
  int32_t *touched;          // [ntot] touched vertices of sparse-mode graphs
  MsCtl *ctl;
  const MsGraph *graphs;     // [ng]
  uint64_t *slot_out;        // [ng*lw*64] device pointers of the outputs
  int32_t *slot_type;        // 0 = uint8, 1 = int32
  int32_t *slot_start;       // level at which the slot's source is expanded
  uint64_t *stop_slots;      // [ng*lw] occupied slots whose finish ends a streaming launch
  uint64_t *newmask;         // [3][ng*lw] slots with a new vertex in level L
  uint64_t *depth_err;       // [ng*lw] uint8 slots whose depth exceeded 254
  int32_t small_bin, wave_bin, chunk_shift;
  int32_t stream_stop;       // stop a launch at the first level a slot of stop_slots finishes
  int32_t sparse_shift;      // a graph runs sparse when active * 2^shift < n
};

// Admission record written by the host for each admitted query.
struct MsAdmit {
  int64_t src_flat;
  int64_t src_local;
  int64_t n;      // vertices of the query's graph (output length)
  uint64_t out;   // device pointer of the output
  int32_t type;   // 0 = uint8, 1 = int32, 2 = discarded (the batch autotuner's timing runs)
  int32_t slot;   // (g*lw + l)*64 + b
};

hipError_t ms_launch_flatten(const int64_t *rp_g, const int32_t *col_g, int64_t n_g, int64_t m_g,
                             int64_t off, int64_t eoff, int64_t *rp_flat, int32_t *col_flat,
                             hipStream_t s);
hipError_t ms_launch_fill(const MsAdmit *adm, int32_t nadm, int64_t maxn, hipStream_t s);
hipError_t ms_launch_admit(const MsView &v, const MsAdmit *adm, int32_t nadm, int32_t level,
                           hipStream_t s);
hipError_t ms_launch_clear(const MsView &v, int64_t begin, int64_t end, const uint64_t *mask_dev,
                           hipStream_t s);
hipError_t ms_launch_persistent(const MsView &v, int32_t max_levels, int32_t grid, hipStream_t s);
int ms_blocks_per_cu(int lw);

}  // namespace bfsk
