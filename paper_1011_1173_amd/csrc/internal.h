// internal.h -- library-internal entry points shared between translation
// units of libcholmod_mi355x.so (not part of the C ABI).
#pragma once
#include <hip/hip_runtime.h>

#include <functional>

#include "../../include/cholmod_mi355x.h"

namespace chm {

// Bytes of the batch tables (uploaded at the start of the workspace) and of
// the whole batch workspace; 0 if any descriptor is invalid.  queued: the
// one-launch form of the batched entry points; otherwise the form with one
// launch per block step (out-of-core, and enqueue_batch with after_step).
size_t batch_table_bytes(const cholmod_desc* descs, int64_t count, bool queued = true);
size_t batch_workspace_bytes(const cholmod_desc* descs, int64_t count, bool queued = true);

// Launches of a factor in a batch: its step s runs in the batch's launch s,
// for s < batch_steps_of(desc); after the launch of its last step the
// factor's L and info word are final.
int64_t batch_steps_of(const cholmod_desc& d);

// Validate, build the tables in the pinned host buffer `stage` (at least
// batch_table_bytes), upload them to `ws` and enqueue the batch on `st`.
// The caller keeps `stage` unchanged until the upload has run.  Without
// after_step the batch is the queued form (one persistent launch); d_done
// (device addresses of `count` int64 words, or null) then receives each
// factor's info word as soon as the factor is finished.  With after_step the
// batch runs one launch per block step and after_step is called after the
// launch of every step s is enqueued (to enqueue more work behind it on
// `st`); a non-zero return stops and is returned.
// plan (or null: the default plan) chooses the schedule of a batch without
// after_step and the queued launch's shape; a batch with d_done must be
// queued.  staged (or null) is recorded on `st` right after the upload of
// the tables from `stage`: once it has completed, `stage` may be rewritten
// while the batch still runs.
int enqueue_batch(const cholmod_desc* descs, int64_t count, void* ws, size_t ws_bytes,
                  int64_t* d_info, hipStream_t st, void* stage, size_t stage_bytes,
                  const std::function<int(int64_t)>* after_step = nullptr,
                  int64_t* d_done = nullptr, const cholmod_plan* plan = nullptr,
                  hipEvent_t staged = nullptr);

// Workspace that fits a batch under either schedule; 0 if invalid.
size_t batch_workspace_bytes_any(const cholmod_desc* descs, int64_t count);

// The launch plan that the plan table gives a batch (descriptors valid).
cholmod_plan select_plan(const cholmod_desc* descs, int64_t count);

}  // namespace chm
