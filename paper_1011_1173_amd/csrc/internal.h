// internal.h -- library-internal entry points shared between translation
// units of libcholmod_mi355x.so (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include "../../include/cholmod_mi355x.h"

namespace chm {

// Bytes of the batch tables (uploaded at the start of the workspace) and of
// the whole batch workspace; 0 if any descriptor is invalid.
size_t batch_table_bytes(const cholmod_desc* descs, int64_t count);
size_t batch_workspace_bytes(const cholmod_desc* descs, int64_t count);

// Validate, build the tables in the pinned host buffer `stage` (at least
// batch_table_bytes), upload them to `ws` and enqueue the batch on `st`.
// The caller keeps `stage` unchanged until the upload has run.
int enqueue_batch(const cholmod_desc* descs, int64_t count, void* ws, size_t ws_bytes,
                  int64_t* d_info, hipStream_t st, void* stage, size_t stage_bytes);

}  // namespace chm
