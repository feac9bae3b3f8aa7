// Plan-time relabelling of a whole graph by descending degree (relabel.hip).
#pragma once

#include <hip/hip_runtime.h>
#include <stddef.h>
#include <stdint.h>

namespace bfsk {

struct RelabelSizes {
  size_t keys;     // bytes of each of the two key buffers (uint64[n+1])
  size_t tmp_col;  // bytes of the unsorted renamed column array
  size_t temp;     // bytes of sort/scan scratch
};

RelabelSizes relabel_sizes(int64_t n, int64_t m);

// Builds new_rp (int64[n+1]), new_col (int32[m], rows sorted), old_id and
// new_id (int32[n]) on stream s. keys_a/keys_b/tmp_col/temp are scratch.
hipError_t relabel_build(const int64_t *rp, const int32_t *col, int64_t n, int64_t m,
                         int64_t *new_rp, int32_t *new_col, int32_t *old_id, int32_t *new_id,
                         void *keys_a, void *keys_b, void *tmp_col, void *temp, size_t temp_bytes,
                         hipStream_t s);

}  // namespace bfsk
