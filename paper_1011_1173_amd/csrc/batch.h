// batch.h -- tables of the batched schedule, shared by the host planner
// (api.hip) and the kernels (sysblk.hip).
#pragma once
#include <stdint.h>

namespace chm {

enum : int32_t { kStoreF64 = 0, kStoreF32 = 1 };

// One factor of a batch, as the kernels see it (device table).
struct BatchFactor {
  void* L;         // caller's factor
  const void* V;   // caller's V (read by the preparation launch only)
  void* W;         // private copy of V in the workspace
  void* T;         // rotation records, n x 16 slots of 32 bytes per 16-column pass
  int64_t* info;   // caller's info word for this factor
  int64_t* stop;   // first failing row
  int32_t* left;   // queued form: the factor's owner items not yet finished
  int64_t* done;   // queued form, or null: where the last item to finish
                   // writes the factor's info word (host-mapped memory)
  void* maps;      // queued form, or null (every block by its rotations): the
                   // block maps, 76 x 64 doubles per block and pass
  int64_t n, k, ldl;
  int32_t sigma, dtype;
};

// One factor's share of one step: block [pc, pc + bbc) of pass m0 (device
// table; a step's entries are contiguous, longest factor first).  Lc and La
// address the rows of block pc and of block pa: element (i, j) of L is at
// Lc + i * ldl + j for i in block pc and at La + i * ldl + j for i in block
// pa (both are the factor's L, except for a factor streamed in row panels,
// whose blocks sit in separate device buffers).
struct BatchEntry {
  void* Lc;
  void* La;
  int64_t pc, pa, m0;
  int32_t f;       // factor index
  int32_t bbc;     // rows of the block
  int32_t kc;      // columns of V in this pass
  int32_t rest0;   // index of the entry's first rest workgroup among the step's
                   // (a rest workgroup applies two 64-column tiles)
};

// One owner item of a queued batch: the columns of block j of factor f,
// every pass (device table, in the order the workgroups take them).
struct QItem {
  int32_t f;
  int32_t j;
};

// Host-side description of one launch.
struct BatchStep {
  int64_t off;     // first entry
  int64_t nent;    // entries (= chain workgroups)
  int64_t nrest;   // rest workgroups
};

}  // namespace chm
