/*
 * bfs.h -- C ABI of the MI355X (gfx950) breadth-first-search hot path.
 *
 * The problem (Section 2, Preliminaries): an undirected graph G = (V, E) with
 * both (u,v) and (v,u) stored, and a root r. The output is d[v], the number of
 * hops from r to v, or "infinity" when no path exists. This library computes
 * d by the level-synchronous top-down traversal of Algorithm 1, organised as in
 * Algorithm 2 of Section 3: a local expansion of the owned frontier into a
 * global next-frontier bitmap (Phase 1) followed by a frontier-synchronisation
 * merge of that bitmap with the bitmaps received from other compute nodes
 * (Phase 2). With one compute node the merge has no incoming bitmaps.
 * Opt-in extensions on the same kernels and buffers: bottom-up Phase 1 steps
 * (direction-optimizing traversal, whole graphs in bfs_run or any share
 * through bfs_expand_bottom_up), vertex-list butterfly messages
 * (bfs_frontier_list, bfs_merge_lists), and batched multi-source queries with
 * a continuous-batching scheduler (bfs_batch_*).
 *
 * Conventions used by every entry point
 *   - All graph, workspace, output and bitmap pointers are DEVICE pointers
 *     (hipMalloc'd or torch CUDA tensors) unless marked "host".
 *   - Distances are int32 with -1 meaning infinity (the uint8 batched form
 *     uses 255). Parents are int32: parent[root] = root, -1 if unreached, and
 *     otherwise the smallest-id neighbour one level closer to the root.
 *   - Bitmaps are uint64 words: vertex v is bit (v & 63) of word (v >> 6);
 *     bits at positions >= n_global in the last word must be zero.
 *   - Every call returns a bfs_status. No C++ exception crosses the ABI; after
 *     an error, bfs_last_error() describes it and the plan stays usable.
 *   - The caller owns all device memory, including the workspace, which must
 *     outlive the plan. After bfs_plan_create the library allocates no device
 *     memory: every buffer has a fixed size independent of the level and the
 *     source (the paper preallocates its exchange buffers, Section 3 "Fanout &
 *     Trade-offs", and bounds memory use by the fanout).
 *   - All device work is ordered on the plan's HIP stream.
 */
#ifndef BFS_MI355X_H
#define BFS_MI355X_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef int32_t bfs_status;
#define BFS_OK 0
#define BFS_ERR_ARG 1        /* invalid argument (null pointer, bad source, bad sizes) */
#define BFS_ERR_WORKSPACE 2  /* workspace smaller than bfs_workspace_size() */
#define BFS_ERR_HIP 3        /* a HIP runtime call failed; message names it */
#define BFS_ERR_DEPTH 4      /* a uint8 batched distance would exceed 254 */
#define BFS_ERR_CAPACITY 5   /* a batched query can never fit the plan's lanes */
#define BFS_ERR_EXCHANGE 6   /* the exchange callback returned nonzero */
#define BFS_ERR_STATE 7      /* call out of order (e.g. merge before begin) */
#define BFS_ERR_TIMEOUT 8    /* bfs_batch_wait timed out; the ticket stays valid */
#define BFS_ERR_DEVICE 9     /* a device-side safety limit tripped (see message) */

typedef struct bfs_plan_s *bfs_plan_t;

/*
 * One graph, or one compute node's 1D share of it (Section 4, "Graph
 * Partitioning": consecutive vertex ranges per node). The node owns vertices
 * [v_begin, v_end) and stores their adjacency: row_ptr has v_end - v_begin + 1
 * entries with row_ptr[0] == 0 and row_ptr[last] == m; col holds m GLOBAL
 * vertex ids. For a whole graph, v_begin = 0 and v_end = n_global. The whole
 * graph must be symmetric (undirected), with n_global < 2^31.
 */
typedef struct {
  int64_t n_global;
  int64_t v_begin;
  int64_t v_end;
  int64_t m;
  const int64_t *row_ptr; /* device */
  const int32_t *col;     /* device */
} bfs_graph;

/*
 * Exchange callback for partitioned runs, called by bfs_run once per level
 * after the local expansion (Algorithm 2, between Phase 1 and Phase 2).
 * local_next is the node's global queue for the level as a bitmap (device,
 * read-only for the callback). The callback sets *incoming to a host array of
 * *k device bitmap pointers: the messages received from the butterfly partners
 * for this level. Return 0 on success; nonzero aborts the run with
 * BFS_ERR_EXCHANGE. The stream is synchronised before the call.
 */
typedef int32_t (*bfs_exchange_fn)(void *ctx, int32_t level, const uint64_t *local_next,
                                   const uint64_t *const **incoming, int32_t *k);

#define BFS_LOOP_AUTO 0       /* device-resident loop when no exchange callback */
#define BFS_LOOP_HOST 1       /* one launch per phase, host reads the new count */
#define BFS_LOOP_PERSISTENT 2 /* whole traversal in one cooperative launch */
#define BFS_LOOP_GRAPH 3      /* a captured hipGraph of 8 level steps, replayed until done */
#define BFS_LOOP_CU 4         /* whole traversal in one workgroup with its bitmaps in LDS: whole
                                 graphs with m < 2^25 whose two n-bit bitmaps fit in one
                                 workgroup's LDS (else BFS_ERR_ARG when asked for explicitly) */
#define BFS_LOOP_ENQUEUE 5    /* the captured loop's level steps (the device decides each level's
                                 form and the end of the traversal) launched directly, 8 steps
                                 per host round trip, each launch bracketed by HIP events on
                                 the plan's stream: per-level device times without a graph */

typedef struct {
  void *hip_stream;        /* hipStream_t; NULL = the null stream */
  int32_t loop_mode;       /* BFS_LOOP_* */
  int32_t small_bin;       /* degree bins b < small_bin -> lane-group tier (1..24); 0 = tuned */
  int32_t wave_bin;        /* bins small_bin <= b < wave_bin (at most 25) -> wavefront tier,
                              else the chunked hub tier; 0 = tuned */
  int32_t chunk_edges;     /* edges per block-tier work item (power of two); 0 = default */
  int32_t grid_blocks;     /* workgroups for device-resident loops; 0 = sized to the graph */
  int32_t batch_lanes;     /* 64-source lane words per graph for batched BFS; 0 = none */
  int32_t collect_stats;   /* nonzero: per-level frontier sizes and degree-bin histograms */
  bfs_exchange_fn exchange;
  void *exchange_ctx;
  int32_t relabel;         /* whole graphs: 0 = automatic (on), 1 = on, -1 = off. A
                              relabelled copy sorted by descending degree is built at plan
                              creation (inside the workspace); results keep original ids */
  int32_t autotune;        /* 0 = automatic (whole graphs with >= 2^16 edges), 1 = always,
                              -1 = never. The plan times a few traversals from four sources
                              per candidate (level loop, register budget, grid size,
                              degree-bin tier thresholds, hub chunk size, LDS hub copy,
                              queue-only threshold) and keeps the fastest; explicit option
                              values are never overridden. Batched plans also tune the
                              batched engine (bfs_batch_tuning) */
  int32_t hot_words;       /* relabelled graphs: visited words each expansion block keeps in
                              LDS on large levels; above 4096 words the expansion runs one
                              1024-thread block per CU sharing the copy. At most (LDS bytes
                              per workgroup - 1024) / 8, else BFS_ERR_ARG; 0 = tuned,
                              -1 = none */
  int32_t sparse_div;      /* single node: a level runs queue-only (no bitmap merge) when its
                              frontier is below ceil(n/64) / sparse_div; 0 = tuned, -1 = never */
  int32_t direction;       /* BFS_DIR_TOPDOWN (default): every level top-down, the paper's
                              method. BFS_DIR_OPTIMIZING: bfs_run on a whole graph without an
                              exchange callback may run large levels bottom-up (see below),
                              and step-wise traversals may call bfs_expand_bottom_up.
                              Distances are the same either way */
  int32_t mark_mode;       /* bfs_run on a whole graph without bottom-up levels:
                              0 or 1 = byte marks: the expansion leaves the bitmaps alone,
                              keeps the hubs it finds in its LDS copy of their visited bits
                              (ORed into a small hub bitmap once per workgroup) and sets one
                              byte per other candidate with a plain store; the merge folds
                              both into the visited bitmap. -1 = the expansion ORs bits into
                              the visited bitmap with device-scope atomics */
  int64_t mem_budget_bytes; /* batched / streaming queries: admission bound on the memory of
                              the queries in flight at once (0 = slots only). A query counts
                              bfs_batch_query_bytes(): its distance output plus its share of
                              the lane words (3 arrays x 8 bytes per 64 sources per vertex);
                              it waits until the queries in flight leave room, and one that
                              can never fit is refused at submission (BFS_ERR_CAPACITY) */
  const char *tune_cache;  /* host path of a text file of tuned settings, or NULL. A plan whose
                              graph, device and options match an entry takes its settings
                              and skips the autotuner's timing runs; otherwise it autotunes
                              and appends an entry. Lines are independent (a concurrent
                              writer may add a duplicate entry, never a corrupt one) */
} bfs_options;

#define BFS_DIR_TOPDOWN 0
/* Direction-optimizing traversal (the bottom-up step the paper names as a
   promising addition, Section 2 on direction-optimizing BFS; the switching
   rule is the usual edge-count test). In the host-driven loop a level L >= 2
   runs bottom-up -- every unvisited vertex scans its adjacency for a member of
   the level-L frontier bitmap and stops at the first -- once the frontier's
   edges exceed 1/14 of the unvisited vertices' edges and n/24, and returns
   to top-down
   once the frontier is below n/24 vertices and no larger than the previous
   level's (so a long tail of small levels runs top-down). */
#define BFS_DIR_OPTIMIZING 1

/* Fills *o with defaults (all zero / NULL, loop_mode AUTO). */
void bfs_options_default(bfs_options *o);

typedef struct {
  int32_t levels;        /* number of nonempty levels = max distance + 1 */
  int64_t reached;       /* vertices with a finite distance (all n_global) */
  int64_t edges_scanned; /* sum of degrees of the owned frontier vertices */
  float ms;              /* device time of the whole traversal, reset included (HIP events) */
  float loop_ms;         /* device time of the level loop alone (the persistent launch, or
                            first expansion to last merge when host-driven) */
  float expand_ms;       /* host-driven loop: summed device time of the dense expansion
                            launches (k_expand) of the first 64 levels; BFS_LOOP_ENQUEUE:
                            of the first 64 expansion steps it launched (8 per round trip,
                            counting the steps that found the traversal already finished;
                            their kernels return at once); 0 for the other loops */
  float merge_ms;        /* the same for the merge launches */
  int32_t expand_launches; /* launches summed in expand_ms */
  int64_t dense_edges;     /* edges scanned by the dense (bitmap) expansions of this traversal,
                              every level loop; with dense_frontier, the work behind expand_ms */
  int64_t dense_frontier;  /* frontier vertices of those expansions */
  float queue_ms;          /* host-driven loop: device time of the queue-only levels (their
                              expansions are not in expand_ms) */
  int32_t bottom_up_levels; /* levels that ran bottom-up (BFS_DIR_OPTIMIZING) */
  float bottom_up_ms;      /* device time of their bottom-up launches (not in expand_ms) */
  int64_t bottom_up_edges; /* adjacency entries the bottom-up launches examined */
  int64_t bottom_up_vertices; /* unvisited vertices they examined */
} bfs_stats;

#define BFS_MAX_LEVEL_STATS 4096
#define BFS_NUM_BINS 34 /* degree bin b = 0 for degree 0, else 1 + floor(log2(degree)) */

/*
 * Bytes of device workspace bfs_plan_create needs for these graphs and
 * options (the largest of the graphs for single-source runs, plus batched
 * lane state per graph when batch_lanes > 0). Host pointers in, *bytes out.
 */
bfs_status bfs_workspace_size(const bfs_graph *graphs, int32_t ngraphs, const bfs_options *o,
                              size_t *bytes);

/*
 * Creates a plan over ngraphs graphs (host array of descriptors; the device
 * arrays they point to must outlive the plan). workspace: device memory of at
 * least bfs_workspace_size() bytes, 256-byte aligned, owned by the caller.
 * Autotuned tier thresholds are chosen here when the options leave them 0.
 * Besides the host object, the plan holds HIP events, a capture stream and a
 * small pinned host buffer (the host copy of its control block, read after
 * each level of the host-driven loop); bfs_plan_destroy releases them.
 */
bfs_status bfs_plan_create(const bfs_graph *graphs, int32_t ngraphs, const bfs_options *o,
                           void *workspace, size_t ws_bytes, bfs_plan_t *out);

/* Destroys the plan (host object only). Safe on NULL. */
void bfs_plan_destroy(bfs_plan_t p);

/* Last error message of the plan (or of the last failed create when p is NULL). */
const char *bfs_last_error(bfs_plan_t p);

/* Settings the plan uses for one graph (after autotuning). */
typedef struct {
  int32_t loop_mode;        /* the level loop bfs_run drives (BFS_LOOP_HOST, _PERSISTENT, _GRAPH
                               or _CU): the option when given, else the tuned choice */
  int32_t persist_variant;  /* 0: default registers, 1: 64-VGPR budget */
  int32_t grid_blocks;      /* blocks of the persistent launch */
  int32_t small_bin;
  int32_t wave_bin;
  int32_t chunk_edges;
  int32_t relabelled;       /* 1 if bfs_run traverses the degree-sorted copy */
  float tuned_ms;           /* best mean traversal time the autotuner measured over its sources
                               (0: not tuned) */
  int32_t hot_words;        /* visited words each expansion block keeps in LDS (0: none) */
  int32_t sparse_div;       /* single node: a level runs queue-only when its frontier is below
                               ceil(n/64) / sparse_div (0: never) */
  int32_t direction;        /* BFS_DIR_* the traversal of this graph uses */
  int32_t mark_mode;        /* 1: dense levels set byte marks, -1: atomic ORs into a bitmap */
} bfs_tuning;

/* Fills *out (host) with the settings of graph `graph`. */
bfs_status bfs_plan_tuning(bfs_plan_t p, int32_t graph, bfs_tuning *out);

/*
 * Single-source traversal (Algorithm 1; Algorithm 2 when the graph is a
 * share). Writes dist[0..n_global) (device, int32) and, if parent != NULL,
 * canonical parents for the owned range (device, int32[n_global]; entries
 * outside the owned range are -2 for reached vertices). source must be in
 * [0, n_global); a source outside the owned range is legal (every node sets
 * the root's distance, only the owner enqueues it: Algorithm 2 set-up).
 * Returns after the traversal has finished; st may be NULL.
 */
bfs_status bfs_run(bfs_plan_t p, int32_t graph, int64_t source, int32_t *dist, int32_t *parent,
                   bfs_stats *st);

/*
 * Step-wise form of bfs_run for callers that drive the level loop and the
 * exchange themselves.
 *   bfs_begin: reset (all distances infinity, root at 0, frontier {root} if
 *     owned) into dist (device int32[n_global], kept by the plan until the
 *     next bfs_begin). The step-wise calls always work in the caller's vertex
 *     ids (bitmaps included), never on the relabelled copy.
 *   bfs_expand: Phase 1 for the current level: every owned frontier vertex
 *     scans its adjacency and marks unvisited neighbours in the node's
 *     next-frontier bitmap. *local_next receives that bitmap's device address
 *     (ceil(n_global/64) words) so it can be sent to partners.
 *   bfs_merge_frontier: Phase 2 (Algorithm 2, frontier synchronisation) over k
 *     incoming bitmaps (host array of k device pointers, k >= 0): every vertex
 *     set in the local bitmap or any incoming one and not yet visited is new;
 *     new vertices get distance level+1, and owned new vertices form the next
 *     frontier. keep_next != 0 keeps the union in the local bitmap (the node's
 *     global queue, for multi-round exchanges within a level; call again with
 *     the next round's messages) and does not advance the level; keep_next == 0
 *     finishes the level. *global_new and *owned_new (host, may be NULL)
 *     receive the level's counts so far (every merge call of this level);
 *     reading them synchronises the stream.
 *     The traversal is over when a finished level has global_new == 0
 *     (every node sees the same count after a full exchange).
 *   bfs_finish: writes parents (if parent != NULL) and fills *st.
 */
bfs_status bfs_begin(bfs_plan_t p, int32_t graph, int64_t source, int32_t *dist);
bfs_status bfs_expand(bfs_plan_t p, const uint64_t **local_next);
/*
 * Phase 1 as a bottom-up step (Section 3: the butterfly exchange works as
 * well with bottom-up or direction-optimizing traversals): every unvisited
 * owned vertex scans its adjacency until it meets a vertex of the level's
 * frontier and, if it does, is marked in the node's next-frontier bitmap.
 * The frontier is the whole level over all n_global vertices -- on a share,
 * the merged result of the previous level's exchange -- so the local bitmap
 * holds exactly the owned vertices of the next level. *local_next as for
 * bfs_expand; bfs_merge_frontier / bfs_merge_lists finish the level as after
 * bfs_expand, and the two expansions can alternate level by level (the
 * caller chooses the direction; every node must choose the same). Needs a
 * plan created with direction = BFS_DIR_OPTIMIZING (its merges then also
 * keep the level's frontier bitmap) and a traversal started by bfs_begin;
 * BFS_ERR_STATE otherwise, or when the previous level was not finished.
 */
bfs_status bfs_expand_bottom_up(bfs_plan_t p, const uint64_t **local_next);
bfs_status bfs_merge_frontier(bfs_plan_t p, const uint64_t *const *incoming, int32_t k,
                              int32_t keep_next, int64_t *global_new, int64_t *owned_new);
bfs_status bfs_finish(bfs_plan_t p, int32_t *parent, bfs_stats *st);

/*
 * Vertex-list messages (Section 3: in Phase 2 of Algorithm 2 the nodes send
 * lists of active vertices; a list of c vertices takes 4c bytes against n/8
 * for a bitmap, so it is the smaller message while c < n_global / 32).
 *   bfs_frontier_list: after bfs_expand of the current level (and any
 *     keep_next merges), writes the node's global queue -- the set bits of its
 *     next-frontier bitmap -- as ascending int32 global ids into list (device,
 *     capacity entries; may be NULL when capacity is 0) and the number of
 *     vertices into *count (host). Synchronises the stream. When capacity >
 *     0 and *count > capacity it returns BFS_ERR_CAPACITY, having written
 *     only the first capacity ids; capacity 0 only counts (BFS_OK).
 *   bfs_merge_lists: Phase 2 with k incoming lists and kb incoming bitmaps
 *     in one pass: lists (host array of k device pointers) and counts (host
 *     array of k entry counts, >= 0; a list may be NULL when its count is 0),
 *     bitmaps as for bfs_merge_frontier (may be NULL when kb is 0). Each
 *     listed vertex absent from the global queue is added to it, then the
 *     level is merged exactly as by bfs_merge_frontier(bitmaps, kb,
 *     keep_next): a list message and the same set sent as a bitmap leave the
 *     same state, and the forms can be mixed within a call and a level. Ids
 *     need not be sorted or distinct. An id outside [0, n_global) is skipped
 *     and flagged; the first merge call that reads the level's counts (one
 *     with keep_next == 0, or with global_new or owned_new non-NULL) then
 *     returns BFS_ERR_ARG, and the traversal must restart with bfs_begin.
 *     *global_new and *owned_new as for bfs_merge_frontier.
 * Both work in caller ids on traversals started by bfs_begin (BFS_ERR_STATE
 * otherwise, or before bfs_expand of the level).
 */
bfs_status bfs_frontier_list(bfs_plan_t p, int32_t *list, int64_t capacity, int64_t *count);
bfs_status bfs_merge_lists(bfs_plan_t p, const int32_t *const *lists, const int64_t *counts, int32_t k,
                           const uint64_t *const *bitmaps, int32_t kb, int32_t keep_next,
                           int64_t *global_new, int64_t *owned_new);

/*
 * Per-level statistics of the last traversal (collect_stats must be set):
 * frontier[L] = owned frontier size at level L, hist[L*BFS_NUM_BINS + b] =
 * frontier vertices of degree bin b at level L. Host arrays of max_levels and
 * max_levels*BFS_NUM_BINS entries; *levels receives the number of levels.
 */
bfs_status bfs_level_stats(bfs_plan_t p, int64_t *frontier, int64_t *hist, int32_t max_levels,
                           int32_t *levels);

/*
 * Per-level device times of the last bfs_run when it drove the host loop or
 * the enqueued level steps (BFS_LOOP_ENQUEUE) (HIP events around each
 * launch, first BFS_MAX_TIMED_LEVELS levels):
 * expand_ms[L] = Phase 1 of level L (the top-down expansion, the queue-only
 * level or the bottom-up step), merge_ms[L] = its Phase 2 merge (0 for a
 * queue-only level, which has none), kind[L] = 0 top-down with a bitmap
 * merge, 1 queue-only, 2 bottom-up. Host arrays of max_levels entries (each
 * may be NULL); *levels (host, may be NULL) receives the number of timed
 * levels, 0 when the last traversal ran another loop.
 */
#define BFS_MAX_TIMED_LEVELS 64
bfs_status bfs_level_times(bfs_plan_t p, float *expand_ms, float *merge_ms, int32_t *kind,
                           int32_t max_levels, int32_t *levels);

/*
 * For callers that cannot allocate device memory (code under HIP graph
 * capture, tight serving loops, harnesses that forbid hipMalloc): a
 * single-source traversal of a small whole graph that allocates nothing --
 * no plan, no workspace. It runs the one-workgroup level loop of bfs_run
 * (BFS_LOOP_CU, caller ids, no relabelled copy) with its device scratch (the
 * control block and two frontier queues, BFS_NOALLOC_SCRATCH_BYTES in all)
 * in a fixed device array of the library, one per GPU, held until the
 * process ends. Every call on one GPU shares that array: calls that overlap
 * on a GPU (other streams, other threads) race and must be serialised by the
 * caller. g: host descriptor of a whole graph (v_begin 0, v_end n_global)
 * with at most BFS_NOALLOC_MAX_VERTICES vertices and fewer than
 * BFS_NOALLOC_MAX_EDGES edges, else BFS_ERR_CAPACITY; its device arrays are
 * validated on every call (BFS_ERR_ARG when invalid). dist: device
 * int32[n_global], written as by bfs_run. hip_stream: hipStream_t (NULL =
 * null stream); the call returns after the traversal has finished. levels
 * (host, may be NULL) receives the number of nonempty levels. Errors are
 * described by bfs_last_error(NULL) on the calling thread.
 */
#define BFS_NOALLOC_MAX_VERTICES (1 << 19)
#define BFS_NOALLOC_MAX_EDGES (1 << 25)
#define BFS_NOALLOC_SCRATCH_BYTES (16 * BFS_NOALLOC_MAX_VERTICES + 16384)
bfs_status bfs_run_noalloc(const bfs_graph *g, int64_t source, int32_t *dist, void *hip_stream,
                           int32_t *levels);

/* ------------------------------------------------------------------------ */
/* Batched multi-source traversal and serving                               */
/* ------------------------------------------------------------------------ */

#define BFS_OUT_U8 0  /* uint8 distances, 255 = unreached, depth > 254 -> BFS_ERR_DEPTH */
#define BFS_OUT_I32 1 /* int32 distances, -1 = unreached */

typedef struct {
  int32_t graph;   /* index into the plan's graphs (whole graphs only) */
  int32_t out_type;/* BFS_OUT_U8 or BFS_OUT_I32 */
  int64_t source;  /* in [0, n of that graph) */
  void *out;       /* device, n entries of out_type */
} bfs_query;

#define BFS_BATCH_ONE_LAUNCH 1 /* run the whole batch together, return when queued */
#define BFS_BATCH_STREAMING 2  /* hand queries to the serving scheduler as they arrive */

typedef struct {
  int32_t status;        /* BFS_OK or the first error of the batch */
  int32_t nq;            /* queries in the ticket */
  int64_t submit_ns;     /* host steady-clock times (ns) */
  int64_t complete_ns;
} bfs_batch_result;

/*
 * Submits nq queries (host array). With BFS_BATCH_ONE_LAUNCH the batch runs
 * as one multi-source bitset traversal per graph (64 sources per uint64 lane
 * word) and *ticket identifies it. With BFS_BATCH_STREAMING the queries join
 * the plan's serving loop: they are admitted into free lanes when lane memory
 * frees up (and, with mem_budget_bytes > 0, when the queries in flight leave
 * room for their admission cost) and finish independently; *ticket
 * identifies the group. Requires batch_lanes > 0 at plan creation
 * (BFS_ERR_CAPACITY otherwise). A query whose admission cost alone exceeds
 * mem_budget_bytes can never be admitted: the call returns BFS_ERR_CAPACITY
 * and submits none of the nq queries.
 */
bfs_status bfs_batch_submit(bfs_plan_t p, const bfs_query *q, int32_t nq, uint32_t flags,
                            uint64_t *ticket);

/*
 * Waits for a ticket (timeout_us < 0 waits forever). On BFS_OK, every output
 * of the ticket is complete and *r (host, may be NULL) describes it.
 */
bfs_status bfs_batch_wait(bfs_plan_t p, uint64_t ticket, int64_t timeout_us,
                          bfs_batch_result *r);

/*
 * Completion queue of the serving loop: moves up to max ids of tickets that
 * finished since the previous poll into done[] (host) and sets *n. Waits up
 * to timeout_us (< 0: forever) when none is ready; *n = 0 on timeout. A
 * polled ticket can still be passed to bfs_batch_wait / bfs_batch_times.
 */
bfs_status bfs_batch_poll(bfs_plan_t p, uint64_t *done, int32_t max, int32_t *n,
                          int64_t timeout_us);

/* Per-query completion times (host steady-clock ns) of a finished streaming
 * ticket, in submission order. */
bfs_status bfs_batch_times(bfs_plan_t p, uint64_t ticket, int64_t *complete_ns, int32_t nq);

/*
 * Admission cost of one batched query on graph `graph` with output type
 * out_type (host *bytes): n * (1 for BFS_OUT_U8, 4 for BFS_OUT_I32) + 24 * n / 64
 * bytes, n the graph's vertex count. BFS_ERR_CAPACITY without lane memory.
 */
bfs_status bfs_batch_query_bytes(bfs_plan_t p, int32_t graph, int32_t out_type, int64_t *bytes);

/* Counters of the batched engine over the caller's queries (the batch
   autotuner's runs at plan creation are not counted). */
typedef struct {
  int64_t launches;             /* level-loop launches */
  int64_t levels;               /* levels run over all launches */
  int64_t admitted;             /* queries admitted into slots */
  int64_t admitted_midflight;   /* of them, admitted while other queries were in flight */
  int64_t max_inflight;         /* largest number of queries in flight at once */
  int64_t max_inflight_bytes;   /* largest admission cost in flight at once */
  int64_t inflight_bytes;       /* admission cost in flight now */
} bfs_batch_counters;

bfs_status bfs_batch_read_counters(bfs_plan_t p, bfs_batch_counters *out);

/*
 * Settings of the batched engine (host *out): grid_blocks of its cooperative
 * level loop, the degree-bin tier thresholds small_bin / wave_bin and
 * chunk_edges of its heavy tier, and tuned_ms, the best one-launch batch time
 * the batch autotuner measured (0 when it did not run: autotune < 0, or 0 with
 * fewer than 2^20 edges over all graphs). The autotuner runs inside
 * bfs_plan_create, before any query, timing batches of batch_lanes * 64
 * sources per graph whose outputs are discarded; options given explicitly
 * (grid_blocks, small_bin, wave_bin, chunk_edges) are kept. loop_mode is
 * BFS_LOOP_PERSISTENT; the other fields are 0. BFS_ERR_CAPACITY when the plan
 * has no lane memory.
 */
bfs_status bfs_batch_tuning(bfs_plan_t p, bfs_tuning *out);

#ifdef __cplusplus
}
#endif
#endif /* BFS_MI355X_H */
