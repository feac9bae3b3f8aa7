// Batched multi-source traversal (placeholder until the batch path lands).
#include <hip/hip_runtime.h>

#include "plan.hpp"

namespace bfsk {

struct BatchState {};

void layout_batch(const bfs_graph *, int32_t, const bfs_options *, WsLayout &, size_t &) {}
bfs_status batch_init(Plan *) { return BFS_OK; }
void batch_shutdown(Plan *) {}

}  // namespace bfsk

extern "C" {
bfs_status bfs_batch_submit(bfs_plan_t p, const bfs_query *, int32_t, uint32_t, uint64_t *) {
  if (!p) return BFS_ERR_ARG;
  return p->fail(BFS_ERR_STATE, "batched traversal not built yet");
}
bfs_status bfs_batch_wait(bfs_plan_t p, uint64_t, int64_t, bfs_batch_result *) {
  if (!p) return BFS_ERR_ARG;
  return p->fail(BFS_ERR_STATE, "batched traversal not built yet");
}
bfs_status bfs_batch_times(bfs_plan_t p, uint64_t, int64_t *, int32_t) {
  if (!p) return BFS_ERR_ARG;
  return p->fail(BFS_ERR_STATE, "batched traversal not built yet");
}
}
