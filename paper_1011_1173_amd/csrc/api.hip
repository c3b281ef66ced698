// api.hip -- the C ABI (include/cholmod_mi355x.h): argument validation on the
// host, workspace layout, schedule selection and the synchronous wrapper.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <condition_variable>
#include <cstdint>
#include <cstring>
#include <functional>
#include <memory>
#include <mutex>
#include <numeric>
#include <thread>
#include <vector>

#include "../../include/cholmod_mi355x.h"
#include "batch.h"
#include "internal.h"
#include "rotations.h"

namespace chm {
hipError_t run_blocked(hipStream_t st, double* L, int64_t n, int64_t ldl, double* W, int64_t k,
                       double sg, Coef* T, int64_t* info, int64_t* stop, bool exact);
hipError_t run_sysblk(hipStream_t st, double* L, int64_t n, int64_t ldl, double* W, int64_t k,
                      double sg, Coef* T, int64_t* info, int64_t* stop, int32_t* tickets,
                      double* maps);
hipError_t run_sysblk_f32(hipStream_t st, float* L, int64_t n, int64_t ldl, float* W, int64_t k,
                          double sg, void* T, int64_t* info, int64_t* stop, int32_t* tickets,
                          double* maps, double* carry);
hipError_t run_sysblk_batch(hipStream_t st, const BatchFactor* d_fac, int64_t count,
                            const BatchEntry* d_ent, const BatchStep* steps, int64_t nsteps);
hipError_t run_sysblk_batch_prepare(hipStream_t st, const BatchFactor* d_fac, int64_t count);
hipError_t run_probe_latency(hipStream_t st, int kc, int blocks, int rounds, double* out4,
                             int* timed_out);
hipError_t run_sysblk_batch_step(hipStream_t st, const BatchFactor* d_fac,
                                 const BatchEntry* d_ent, const BatchStep& S);
hipError_t run_sysblk_qbatch(hipStream_t st, const BatchFactor* d_fac, int64_t count,
                             const QItem* d_items, int64_t nitems, int32_t* d_ticket, int grid,
                             int poll);
int compute_units();

namespace {

constexpr size_t kAlign = 256;
constexpr int64_t kKPass = 64;  // V columns per pass of the blocked schedule

inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Workspace layout (all offsets 256-byte aligned):
//   [0, 768)         control words: the first failing row (int64) at 0
//   W                n*k private copy of V
//   T                n*16*ceil(k/16) rotation records of 32 bytes (16 per row
//                    for each 16-column pass of the fast schedule)
//   F                int32 ticket counters (the first one is the fast
//                    schedule's work counter)
//   M                (with maps) the fast schedule's block maps: 76 x 64
//                    doubles per block and 16-column pass
//   C                (binary32 storage with maps, one factor) V of the odd
//                    pass of each pass pair, n x 16 doubles per pair, that
//                    the even pass leaves for it
struct WsLayout {
  size_t ctrl = 0, w = 0, t = 0, f = 0, m = 0, c = 0, total = 0;
  int64_t nflags = 0, nmaps = 0;
};

constexpr size_t kMapBytes = 76 * 64 * sizeof(double);

bool mul_ok(int64_t a, int64_t b, int64_t lim) { return a == 0 || b <= lim / a; }

bool layout_for(int64_t n, int64_t k, int dtype, WsLayout* out, bool maps = true,
                bool carry = true) {
  if (n < 0 || k < 0) return false;
  if (dtype != CHOLMOD_F64 && dtype != CHOLMOD_F32S) return false;
  const int64_t lim = INT64_MAX / 64;
  if (!mul_ok(n, k, lim)) return false;
  const size_t es = dtype == CHOLMOD_F64 ? 8 : 4;
  WsLayout L;
  L.ctrl = 0;
  L.w = 3 * kAlign;  // control words
  L.t = L.w + align_up((size_t)(n * k) * es);
  // records: 16 per row for every 16-column pass (the fast schedule), which
  // also covers the blocked schedule's min(k, 64) per row
  int64_t kp = (k + 15) / 16 * 16;
  if (kp < 16) kp = 16;
  L.f = L.t + align_up((size_t)(n * kp) * sizeof(Coef));
  L.nflags = (k + 15) / 16;
  L.m = L.f + align_up((size_t)L.nflags * sizeof(int32_t));
  L.nmaps = maps ? L.nflags * ((n + 63) / 64) : 0;
  L.total = L.m + (size_t)L.nmaps * kMapBytes;
  if (carry && dtype == CHOLMOD_F32S && L.nmaps > 0 && L.nflags >= 2) {
    L.c = L.total;
    L.total = L.c + align_up((size_t)(L.nflags / 2) * (size_t)n * 16 * sizeof(double));
  }
  *out = L;
  return true;
}

template <typename ST>
__global__ void k_prepare(const ST* __restrict__ V, ST* __restrict__ W, int64_t count,
                          int64_t* __restrict__ info, int64_t* __restrict__ stop_row,
                          int32_t* __restrict__ flags, int64_t nflags) {
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i0 == 0) {
    *info = INT64_MAX;
    *stop_row = INT64_MAX;
  }
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = i0; i < count; i += stride) W[i] = V[i];
  for (int64_t i = i0; i < nflags; i += stride) flags[i] = 0;
}

int validate(const void* L, const void* V, int64_t n, int64_t k, int64_t ldl, int sigma) {
  if (n < 0 || k < 0) return CHOLMOD_ERR_ARG;
  if (ldl < (n > 1 ? n : 1)) return CHOLMOD_ERR_ARG;
  if (sigma != 1 && sigma != -1) return CHOLMOD_ERR_ARG;
  if (n > 0 && L == nullptr) return CHOLMOD_ERR_ARG;
  if (n > 0 && k > 0 && V == nullptr) return CHOLMOD_ERR_ARG;
  // byte offsets must fit in int64 (L spans n*ldl elements)
  if (!mul_ok(n, ldl, INT64_MAX / 16)) return CHOLMOD_ERR_ARG;
  return CHOLMOD_OK;
}

int enqueue_f64(double* L, const double* V, int64_t n, int64_t k, int64_t ldl, int sigma,
                unsigned flags, void* ws, size_t ws_bytes, int64_t* d_info, hipStream_t st) {
  int v = validate(L, V, n, k, ldl, sigma);
  if (v) return v;
  if (flags & ~(unsigned)(CHOLMOD_FLAG_EXACT | CHOLMOD_FLAG_BLOCKED | CHOLMOD_FLAG_ROTATIONS))
    return CHOLMOD_ERR_ARG;
  if (d_info == nullptr) return CHOLMOD_ERR_ARG;
  if (((uintptr_t)d_info & 7u) != 0) return CHOLMOD_ERR_ARG;
  WsLayout lay;
  if (!layout_for(n, k, CHOLMOD_F64, &lay)) return CHOLMOD_ERR_ARG;
  if (ws == nullptr || ws_bytes < lay.total) return CHOLMOD_ERR_ARG;
  if (((uintptr_t)ws % kAlign) != 0) return CHOLMOD_ERR_ARG;
  char* base = (char*)ws;
  int64_t* stop_row = (int64_t*)(base + lay.ctrl);
  double* W = (double*)(base + lay.w);
  Coef* T = (Coef*)(base + lay.t);
  int32_t* F = (int32_t*)(base + lay.f);
  const bool exact = (flags & CHOLMOD_FLAG_EXACT) != 0;
  const bool blocked = exact || (flags & CHOLMOD_FLAG_BLOCKED) != 0;
  const int64_t count = n * k;  // both schedules work on a private copy of V
  unsigned grid = (unsigned)((count + 255) / 256);
  if (grid < 1) grid = 1;
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(k_prepare<double>, dim3(grid), dim3(256), 0, st, V, W, count, d_info,
                     stop_row, F, lay.nflags);
  if (hipGetLastError() != hipSuccess) return CHOLMOD_ERR_HIP;
  if (n == 0 || k == 0) return CHOLMOD_OK;
  const double sg = (double)sigma;
  hipError_t e;
  if (blocked) {
    e = run_blocked(st, L, n, ldl, W, k, sg, T, d_info, stop_row, exact);
  } else {
    const bool maps = (flags & CHOLMOD_FLAG_ROTATIONS) == 0 && lay.nmaps > 0;
    e = run_sysblk(st, L, n, ldl, W, k, sg, T, d_info, stop_row, F,
                   maps ? (double*)(base + lay.m) : nullptr);
  }
  return e == hipSuccess ? CHOLMOD_OK : CHOLMOD_ERR_HIP;
}

int enqueue_f32s(float* L, const float* V, int64_t n, int64_t k, int64_t ldl, int sigma,
                 unsigned flags, void* ws, size_t ws_bytes, int64_t* d_info, hipStream_t st) {
  int v = validate(L, V, n, k, ldl, sigma);
  if (v) return v;
  if (flags & ~(unsigned)CHOLMOD_FLAG_ROTATIONS) return CHOLMOD_ERR_ARG;
  if (d_info == nullptr) return CHOLMOD_ERR_ARG;
  if (((uintptr_t)d_info & 7u) != 0) return CHOLMOD_ERR_ARG;
  WsLayout lay;
  if (!layout_for(n, k, CHOLMOD_F32S, &lay)) return CHOLMOD_ERR_ARG;
  if (ws == nullptr || ws_bytes < lay.total) return CHOLMOD_ERR_ARG;
  if (((uintptr_t)ws % kAlign) != 0) return CHOLMOD_ERR_ARG;
  char* base = (char*)ws;
  int64_t* stop_row = (int64_t*)(base + lay.ctrl);
  float* W = (float*)(base + lay.w);
  void* T = (void*)(base + lay.t);
  int32_t* F = (int32_t*)(base + lay.f);
  const int64_t count = n * k;
  unsigned grid = (unsigned)((count + 255) / 256);
  if (grid < 1) grid = 1;
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(k_prepare<float>, dim3(grid), dim3(256), 0, st, V, W, count, d_info,
                     stop_row, F, lay.nflags);
  if (hipGetLastError() != hipSuccess) return CHOLMOD_ERR_HIP;
  if (n == 0 || k == 0) return CHOLMOD_OK;
  const bool maps = (flags & CHOLMOD_FLAG_ROTATIONS) == 0 && lay.nmaps > 0;
  hipError_t e = run_sysblk_f32(st, L, n, ldl, W, k, (double)sigma, T, d_info, stop_row, F,
                                maps ? (double*)(base + lay.m) : nullptr,
                                maps && lay.c ? (double*)(base + lay.c) : nullptr);
  return e == hipSuccess ? CHOLMOD_OK : CHOLMOD_ERR_HIP;
}

// Library-owned per-device state: the workspace of the synchronous entry
// points, and the pinned staging buffer of the batched planner with the event
// that marks the end of its last upload.
struct DevWs {
  void* ptr = nullptr;
  size_t bytes = 0;
  int64_t* host_info = nullptr;  // pinned
  void* stage = nullptr;         // pinned
  size_t stage_bytes = 0;
  hipEvent_t stage_done = nullptr;
  bool stage_pending = false;
};
std::mutex g_mu;
std::vector<DevWs> g_ws;

// Synchronous wrapper: library-owned workspace and pinned info word, then
// enqueue, copy the info word back and wait for the stream.
template <typename Enqueue>
int run_sync(int64_t n, int64_t k, int dtype, hipStream_t st, Enqueue enqueue) {
  WsLayout lay;
  if (!layout_for(n, k, dtype, &lay)) return CHOLMOD_ERR_ARG;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return CHOLMOD_ERR_HIP;
  std::lock_guard<std::mutex> lk(g_mu);
  if ((int)g_ws.size() <= dev) g_ws.resize(dev + 1);
  DevWs& d = g_ws[dev];
  const size_t need = lay.total + kAlign;  // + info word
  if (d.bytes < need) {
    if (d.ptr) {
      if (hipDeviceSynchronize() != hipSuccess) return CHOLMOD_ERR_HIP;
      hipFree(d.ptr);
      d.ptr = nullptr;
      d.bytes = 0;
    }
    if (hipMalloc(&d.ptr, need) != hipSuccess) return CHOLMOD_ERR_HIP;
    d.bytes = need;
  }
  if (!d.host_info) {
    if (hipHostMalloc((void**)&d.host_info, sizeof(int64_t), hipHostMallocDefault) != hipSuccess)
      return CHOLMOD_ERR_HIP;
  }
  int64_t* d_info = (int64_t*)((char*)d.ptr + lay.total);
  int rc = enqueue(d.ptr, lay.total, d_info, st);
  if (rc) return rc;
  if (hipMemcpyAsync(d.host_info, d_info, sizeof(int64_t), hipMemcpyDeviceToHost, st) !=
      hipSuccess)
    return CHOLMOD_ERR_HIP;
  if (hipStreamSynchronize(st) != hipSuccess) return CHOLMOD_ERR_HIP;
  return cholmod_decode_info(*d.host_info, k, nullptr, nullptr);
}

// ----------------------------------------------------- allocation-free form
// cholmod_update_noalloc keeps its workspace in this fixed device array
// instead of a caller buffer.  Each device that runs the library holds its
// own copy until the process ends.  In host code `scratch` only names the
// symbol: its device address on the current device comes from
// hipGetSymbolAddress, looked up once per device and kept in g_scratch.
constexpr size_t kScratchBytes = (size_t)32 << 20;
__device__ __align__(256) unsigned char scratch[kScratchBytes];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch[kMaxDevices] = {};

// Device address of the scratch array on device `dev`, or nullptr.
void* scratch_address(int dev) {
  if (dev < 0 || dev >= kMaxDevices) return nullptr;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch[dev] == nullptr) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || p == nullptr) {
      (void)hipGetLastError();
      return nullptr;
    }
    g_scratch[dev] = p;
  }
  return g_scratch[dev];
}

// ------------------------------------------------------------------ batched
constexpr int64_t kBlock = 64, kPass = 16, kMaxBatch = 65535;

// Two forms of a batch.  Queued (the batched entry points): the factors'
// owner items in one table, taken by one persistent launch from a work
// counter; the tables are [factors][items][counter].  Stepped (the
// out-of-core form): one launch per block step; the tables are
// [factors][entries].
struct BatchPlan {
  bool queued = true;
  int grid = 0, poll = 2;  // queued launch: persistent workgroups (0 = one per CU), poll level
  std::vector<BatchFactor> fac;
  std::vector<BatchEntry> ent;
  std::vector<BatchStep> steps;
  std::vector<QItem> items;
  size_t off_ent = 0, off_items = 0, off_ticket = 0, off_left = 0, table_bytes = 0, total = 0;
  std::vector<size_t> off_ctrl, off_w, off_t, off_m;  // off_m: 0 = no maps
};

int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

int validate_desc(const cholmod_desc& d) {
  if (d.dtype != CHOLMOD_F64 && d.dtype != CHOLMOD_F32S) return CHOLMOD_ERR_ARG;
  return validate(d.L, d.V, d.n, d.k, d.ldl, d.sigma);
}

// Sizes and (when ws != nullptr) device pointers of a batch; the schedule
// of each factor is the single-factor one (64-row blocks, 16-column passes,
// the same operations in the same order), so every factor's result is the
// one it gets alone.
int plan_batch(const cholmod_desc* descs, int64_t count, char* ws, BatchPlan* P,
               bool queued = true, int order = CHOLMOD_ORDER_BLOCK, bool maps = true) {
  maps = maps && queued;  // the per-step schedule applies every block by rotations
  if (count < 0 || count > kMaxBatch) return CHOLMOD_ERR_ARG;
  if (count > 0 && descs == nullptr) return CHOLMOD_ERR_ARG;
  P->queued = queued;
  std::vector<int64_t> steps(count), blocks(count);
  int64_t total_ent = 0, total_items = 0, smax = 0, bmax = 0;
  for (int64_t f = 0; f < count; ++f) {
    const int v = validate_desc(descs[f]);
    if (v) return v;
    const cholmod_desc& d = descs[f];
    blocks[f] = (d.n == 0 || d.k == 0) ? 0 : ceil_div(d.n, kBlock);
    steps[f] = blocks[f] * ceil_div(d.k, kPass);
    total_ent += steps[f];
    total_items += blocks[f];
    smax = std::max(smax, steps[f]);
    bmax = std::max(bmax, blocks[f]);
  }
  if (total_items > INT32_MAX) return CHOLMOD_ERR_ARG;
  P->off_ent = P->off_items = align_up((size_t)count * sizeof(BatchFactor));
  if (queued) {
    P->off_ticket = P->off_items + align_up((size_t)total_items * sizeof(QItem));
    P->off_left = P->off_ticket + kAlign;
    P->table_bytes = P->off_left + align_up((size_t)count * sizeof(int32_t));
  } else {
    P->table_bytes = P->off_ent + align_up((size_t)total_ent * sizeof(BatchEntry));
  }
  size_t off = P->table_bytes;
  P->off_ctrl.resize(count);
  P->off_w.resize(count);
  P->off_t.resize(count);
  P->off_m.assign(count, 0);
  for (int64_t f = 0; f < count; ++f) {
    const cholmod_desc& d = descs[f];
    WsLayout lay;
    if (!layout_for(d.n, d.k, d.dtype, &lay, maps, false)) return CHOLMOD_ERR_ARG;
    P->off_ctrl[f] = off + lay.ctrl;
    P->off_w[f] = off + lay.w;
    P->off_t[f] = off + lay.t;
    if (lay.nmaps > 0) P->off_m[f] = off + lay.m;
    off += lay.total;
  }
  P->total = off;
  if (ws == nullptr) return CHOLMOD_OK;
  // factor table
  P->fac.resize(count);
  for (int64_t f = 0; f < count; ++f) {
    const cholmod_desc& d = descs[f];
    BatchFactor& F = P->fac[f];
    F.L = d.L;
    F.V = d.V;
    F.W = ws + P->off_w[f];
    F.T = ws + P->off_t[f];
    F.info = nullptr;  // set by the caller
    F.stop = (int64_t*)(ws + P->off_ctrl[f]);
    F.left = queued ? (int32_t*)(ws + P->off_left) + f : nullptr;
    F.done = nullptr;  // set by a caller that wants per-factor completion
    F.maps = P->off_m[f] ? (void*)(ws + P->off_m[f]) : nullptr;
    F.n = d.n;
    F.k = d.k;
    F.ldl = d.ldl;
    F.sigma = d.sigma;
    F.dtype = d.dtype == CHOLMOD_F64 ? kStoreF64 : kStoreF32;
  }
  // longest factor first; at step s the active factors are a prefix
  std::vector<int64_t> order_of(count);
  std::iota(order_of.begin(), order_of.end(), 0);
  std::stable_sort(order_of.begin(), order_of.end(),
                   [&](int64_t a, int64_t b) { return steps[a] > steps[b]; });
  if (queued) {
    // block-major: by block index, longest factor first within a block
    // index; factor-major: every block of the longest factor, then of the
    // next.  Either way an item waits only for its factor's items of lower
    // blocks, which come earlier.
    P->items.clear();
    P->items.reserve(total_items);
    auto push = [&](int64_t f, int64_t b) {
      QItem it;
      it.f = (int32_t)f;
      it.j = (int32_t)b;
      P->items.push_back(it);
    };
    if (order == CHOLMOD_ORDER_FACTOR) {
      for (int64_t f : order_of) 
        for (int64_t b = 0; b < blocks[f]; ++b) push(f, b);
    } else {
      for (int64_t b = 0; b < bmax; ++b)
        for (int64_t f : order_of)
          if (b < blocks[f]) push(f, b);
    }
    return CHOLMOD_OK;
  }
  P->ent.clear();
  P->ent.reserve(total_ent);
  P->steps.assign(smax, BatchStep{});
  for (int64_t s = 0; s < smax; ++s) {
    BatchStep& S = P->steps[s];
    S.off = (int64_t)P->ent.size();
    int64_t rest = 0;
    for (int64_t f : order_of) {
      if (s >= steps[f]) break;
      const cholmod_desc& d = descs[f];
      const int64_t pass = s / blocks[f], b = s % blocks[f];
      BatchEntry e;
      e.Lc = d.L;
      e.La = d.L;
      e.pc = b * kBlock;
      e.pa = b > 0 ? e.pc - kBlock : -1;
      e.m0 = pass * kPass;
      e.f = (int32_t)f;
      e.bbc = (int32_t)std::min(kBlock, d.n - e.pc);
      e.kc = (int32_t)std::min(kPass, d.k - e.m0);
      e.rest0 = (int32_t)rest;
      // rest workgroups apply two 64-column tiles each
      rest += e.pa >= 0 ? ceil_div(ceil_div(d.n - e.pc - e.bbc, kBlock), 2) : 0;
      P->ent.push_back(e);
    }
    S.nent = (int64_t)P->ent.size() - S.off;
    S.nrest = rest;
  }
  return CHOLMOD_OK;
}

}  // namespace

size_t batch_table_bytes(const cholmod_desc* descs, int64_t count, bool queued) {
  BatchPlan P;
  if (plan_batch(descs, count, nullptr, &P, queued) != CHOLMOD_OK) return 0;
  return P.table_bytes;
}

size_t batch_workspace_bytes(const cholmod_desc* descs, int64_t count, bool queued) {
  BatchPlan P;
  if (plan_batch(descs, count, nullptr, &P, queued) != CHOLMOD_OK) return 0;
  return P.total;
}

// Workspace that fits a batch under either schedule.
size_t batch_workspace_bytes_any(const cholmod_desc* descs, int64_t count) {
  const size_t a = batch_workspace_bytes(descs, count, true);
  const size_t b = batch_workspace_bytes(descs, count, false);
  return (a == 0 || b == 0) ? 0 : std::max(a, b);
}

// The batch tables of plan P (built for workspace ws) in host memory at h.
void write_tables(const BatchPlan& P, char* h) {
  std::memcpy(h, P.fac.data(), P.fac.size() * sizeof(BatchFactor));
  if (P.queued) {
    if (!P.items.empty())
      std::memcpy(h + P.off_items, P.items.data(), P.items.size() * sizeof(QItem));
    std::memset(h + P.off_ticket, 0, kAlign);
  } else if (!P.ent.empty()) {
    std::memcpy(h + P.off_ent, P.ent.data(), P.ent.size() * sizeof(BatchEntry));
  }
}

// The launches of a planned batch on `st` (tables already in ws).
hipError_t run_planned(hipStream_t st, const BatchPlan& P, char* ws, int64_t count) {
  const BatchFactor* d_fac = (const BatchFactor*)ws;
  if (P.queued)
    return run_sysblk_qbatch(st, d_fac, count, (const QItem*)(ws + P.off_items),
                             (int64_t)P.items.size(), (int32_t*)(ws + P.off_ticket), P.grid,
                             P.poll);
  return run_sysblk_batch(st, d_fac, count, (const BatchEntry*)(ws + P.off_ent), P.steps.data(),
                          (int64_t)P.steps.size());
}

int64_t batch_steps_of(const cholmod_desc& d) {
  return (d.n <= 0 || d.k <= 0) ? 0 : ceil_div(d.n, kBlock) * ceil_div(d.k, kPass);
}

// ------------------------------------------------------------ launch plans
// The plan that cholmod_update_batched uses for a batch comes from a table
// indexed by the batch's dominant (storage type, n bucket, k bucket): the
// bucket holding most of the batch's work, n^2 k summed over its factors.
// The table starts with the default plan everywhere; cholmod_set_plan fills
// it, normally from a plan cache that the autotuner wrote.
constexpr int kNBuckets = 5, kKBuckets = 4;
const int64_t kNBucketTop[kNBuckets - 1] = {256, 1024, 4096, 16384};
const int64_t kKBucketTop[kKBuckets - 1] = {16, 32, 64};

cholmod_plan default_plan() {
  cholmod_plan p;
  p.schedule = CHOLMOD_SCHED_QUEUED;
  p.grid = 0;
  p.order = CHOLMOD_ORDER_BLOCK;
  p.poll = 2;
  p.maps = 1;
  return p;
}

struct PlanTable {
  cholmod_plan p[2][kNBuckets][kKBuckets];
  PlanTable() {
    for (auto& a : p)
      for (auto& b : a)
        for (auto& c : b) c = default_plan();
  }
};
std::mutex g_plan_mu;
PlanTable g_plans;

int bucket_of(int64_t v, const int64_t* tops, int n) {
  int b = 0;
  while (b < n - 1 && v > tops[b]) ++b;
  return b;
}

bool plan_ok(const cholmod_plan& p) {
  return (p.schedule == CHOLMOD_SCHED_QUEUED || p.schedule == CHOLMOD_SCHED_STEPPED) &&
         p.grid >= 0 && p.grid <= 65536 &&
         (p.order == CHOLMOD_ORDER_BLOCK || p.order == CHOLMOD_ORDER_FACTOR) && p.poll >= 0 &&
         p.poll <= 2 && (p.maps == 0 || p.maps == 1);
}

// The table's plan for a batch (descriptors already validated).
cholmod_plan select_plan(const cholmod_desc* descs, int64_t count) {
  double work[2][kNBuckets][kKBuckets] = {};
  for (int64_t f = 0; f < count; ++f) {
    const cholmod_desc& d = descs[f];
    const int t = d.dtype == CHOLMOD_F64 ? 0 : 1;
    work[t][bucket_of(d.n, kNBucketTop, kNBuckets)][bucket_of(d.k, kKBucketTop, kKBuckets)] +=
        (double)d.n * (double)d.n * (double)d.k;
  }
  int bt = 0, bn = 0, bk = 0;
  for (int t = 0; t < 2; ++t)
    for (int a = 0; a < kNBuckets; ++a)
      for (int b = 0; b < kKBuckets; ++b)
        if (work[t][a][b] > work[bt][bn][bk]) bt = t, bn = a, bk = b;
  std::lock_guard<std::mutex> lk(g_plan_mu);
  return g_plans.p[bt][bn][bk];
}

int enqueue_batch(const cholmod_desc* descs, int64_t count, void* ws, size_t ws_bytes,
                  int64_t* d_info, hipStream_t st, void* stage, size_t stage_bytes,
                  const std::function<int(int64_t)>* after_step, int64_t* d_done,
                  const cholmod_plan* plan, hipEvent_t staged) {
  BatchPlan P;
  const cholmod_plan lp = plan ? *plan : default_plan();
  if (!plan_ok(lp)) return CHOLMOD_ERR_ARG;
  const bool queued = after_step == nullptr && lp.schedule == CHOLMOD_SCHED_QUEUED;
  int rc = plan_batch(descs, count, nullptr, &P, queued, lp.order, lp.maps != 0);
  if (rc) return rc;
  if (count == 0) return CHOLMOD_OK;
  if (d_info == nullptr || ((uintptr_t)d_info & 7u) != 0) return CHOLMOD_ERR_ARG;
  if (ws == nullptr || ws_bytes < P.total || ((uintptr_t)ws % kAlign) != 0)
    return CHOLMOD_ERR_ARG;
  if (stage == nullptr || stage_bytes < P.table_bytes) return CHOLMOD_ERR_ARG;
  rc = plan_batch(descs, count, (char*)ws, &P, queued, lp.order, lp.maps != 0);
  if (rc) return rc;
  P.grid = lp.grid;
  P.poll = lp.poll;
  for (int64_t f = 0; f < count; ++f) {
    P.fac[f].info = d_info + f;
    if (queued && d_done) P.fac[f].done = d_done + f;
  }
  char* h = (char*)stage;
  write_tables(P, h);
  if (hipMemcpyAsync(ws, h, P.table_bytes, hipMemcpyHostToDevice, st) != hipSuccess)
    return CHOLMOD_ERR_HIP;
  if (staged && hipEventRecord(staged, st) != hipSuccess) return CHOLMOD_ERR_HIP;
  const BatchFactor* d_fac = (const BatchFactor*)ws;
  const BatchEntry* d_ent = (const BatchEntry*)((char*)ws + P.off_ent);
  if (after_step == nullptr) {
    hipError_t e = run_planned(st, P, (char*)ws, count);
    return e == hipSuccess ? CHOLMOD_OK : CHOLMOD_ERR_HIP;
  }
  if (run_sysblk_batch_prepare(st, d_fac, count) != hipSuccess) return CHOLMOD_ERR_HIP;
  for (int64_t s = 0; s < (int64_t)P.steps.size(); ++s) {
    if (run_sysblk_batch_step(st, d_fac, d_ent, P.steps[s]) != hipSuccess) return CHOLMOD_ERR_HIP;
    rc = (*after_step)(s);
    if (rc) return rc;
  }
  return CHOLMOD_OK;
}

// ------------------------------------------------------------ out-of-core
// A factor in host memory streamed through the device in row panels of 64
// rows (block b's rows, columns b*64 .. n-1).  The factor runs the batched
// schedule (one launch per block step); step b touches only the rows of
// blocks b and b-1, so panel b is uploaded before step b and downloaded
// after step b+1 (or after step b for the last block of a pass).  Panel p
// lives in slot p mod kOocSlots; three slots would suffice (the upload of
// panel b never overwrites panels b-1 and b), more let the uploads run
// further ahead of the steps.  A slot holds 64 rows of n elements (row pitch
// n) and keeps the column index of the factor.
//   workspace = [batch workspace of the factor (row pitch n)] [info word]
//               [kOocSlots slots of 64 x n elements]
constexpr int kOocSlots = 6;

struct OocLayout {
  size_t batch = 0, info = 0, slots = 0, slot_bytes = 0, total = 0;
};

// A descriptor for planning only: the planner checks that the pointers are
// set but never dereferences them.
cholmod_desc ooc_desc(void* L_host, const void* V, int64_t n, int64_t k, int sigma, int dtype) {
  cholmod_desc d;
  d.L = L_host;
  d.V = V;
  d.n = n;
  d.k = k;
  d.ldl = n > 1 ? n : 1;  // row pitch of a device slot
  d.sigma = sigma;
  d.dtype = dtype;
  return d;
}

bool ooc_layout(int64_t n, int64_t k, int dtype, OocLayout* out) {
  if (n < 0 || k < 0 || (dtype != CHOLMOD_F64 && dtype != CHOLMOD_F32S)) return false;
  // non-null placeholders: sizing does not look at the pointers
  const cholmod_desc d = ooc_desc((void*)kAlign, (const void*)kAlign, n, k, 1, dtype);
  const size_t batch = batch_workspace_bytes(&d, 1, false);
  if (batch == 0) return false;
  const size_t es = dtype == CHOLMOD_F64 ? 8 : 4;
  if (!mul_ok(kBlock * (int64_t)es, n > 1 ? n : 1, INT64_MAX / 8)) return false;
  OocLayout L;
  L.batch = batch;
  L.info = align_up(batch);
  L.slots = L.info + kAlign;
  L.slot_bytes = align_up((size_t)(kBlock * (n > 1 ? n : 1)) * es);
  L.total = L.slots + kOocSlots * L.slot_bytes;
  *out = L;
  return true;
}

// Host memory the copy engines can reach directly (hipHostMalloc'd, which
// includes torch's pinned tensors).
bool host_pinned(const void* p) {
  hipPointerAttribute_t a;
  if (hipPointerGetAttributes(&a, p) != hipSuccess) {
    (void)hipGetLastError();  // unknown host pointer: not an error here
    return false;
  }
  return a.type == hipMemoryTypeHost;
}

// Copies `rows` rows of `wbytes` bytes between pitched host buffers, split
// over the calling thread and a few helper threads that live as long as the
// object (one out-of-core call).
class RowCopier {
 public:
  explicit RowCopier(int helpers) {
    for (int t = 0; t < helpers; ++t) th_.emplace_back([this, t] { loop(t + 1); });
  }
  ~RowCopier() {
    {
      std::lock_guard<std::mutex> lk(mu_);
      quit_ = true;
    }
    cv_.notify_all();
    for (std::thread& t : th_) t.join();
  }
  void run(char* dst, size_t dpitch, const char* src, size_t spitch, size_t wbytes,
           int64_t rows) {
    const int parts = wbytes * (size_t)rows >= (1u << 20) ? (int)th_.size() + 1 : 1;
    {
      std::lock_guard<std::mutex> lk(mu_);
      dst_ = dst;
      src_ = src;
      dpitch_ = dpitch;
      spitch_ = spitch;
      wbytes_ = wbytes;
      rows_ = rows;
      parts_ = parts;
      pending_ = parts - 1;
      ++gen_;
    }
    if (parts > 1) cv_.notify_all();
    part(0, parts);
    std::unique_lock<std::mutex> lk(mu_);
    done_.wait(lk, [&] { return pending_ == 0; });
  }

 private:
  void part(int t, int parts) {
    const int64_t per = (rows_ + parts - 1) / parts;
    const int64_t a = t * per, b = std::min(rows_, a + per);
    for (int64_t r = a; r < b; ++r)
      std::memcpy(dst_ + r * dpitch_, src_ + r * spitch_, wbytes_);
  }
  void loop(int t) {
    uint64_t seen = 0;
    for (;;) {
      int parts;
      {
        std::unique_lock<std::mutex> lk(mu_);
        cv_.wait(lk, [&] { return quit_ || gen_ != seen; });
        if (quit_) return;
        seen = gen_;
        parts = parts_;
      }
      if (t >= parts) continue;  // a small copy: the caller does it alone
      part(t, parts);
      std::lock_guard<std::mutex> lk(mu_);
      if (--pending_ == 0) done_.notify_all();
    }
  }
  std::vector<std::thread> th_;
  std::mutex mu_;
  std::condition_variable cv_, done_;
  uint64_t gen_ = 0;
  int pending_ = 0, parts_ = 1;
  bool quit_ = false;
  char* dst_ = nullptr;
  const char* src_ = nullptr;
  size_t dpitch_ = 0, spitch_ = 0, wbytes_ = 0;
  int64_t rows_ = 0;
};

int update_ooc(void* L_host, const void* V, int64_t n, int64_t k, int64_t ldl, int sigma,
               int dtype, void* ws, size_t ws_bytes, hipStream_t st, int64_t* info_out) {
  if (info_out) *info_out = CHOLMOD_INFO_NONE;
  if (dtype != CHOLMOD_F64 && dtype != CHOLMOD_F32S) return CHOLMOD_ERR_ARG;
  int v = validate(L_host, V, n, k, ldl, sigma);
  if (v) return v;
  OocLayout lay;
  if (!ooc_layout(n, k, dtype, &lay)) return CHOLMOD_ERR_ARG;
  if (ws != nullptr && (ws_bytes < lay.total || ((uintptr_t)ws % kAlign) != 0))
    return CHOLMOD_ERR_ARG;
  if (n == 0 || k == 0) return CHOLMOD_OK;
  const cholmod_desc d = ooc_desc(L_host, V, n, k, sigma, dtype);
  bool own = false;
  if (ws == nullptr) {
    if (hipMalloc(&ws, lay.total) != hipSuccess) return CHOLMOD_ERR_HIP;
    own = true;
  }
  int rc = CHOLMOD_OK;
  int64_t host_info = CHOLMOD_INFO_NONE;
  do {
    BatchPlan P;
    rc = plan_batch(&d, 1, (char*)ws, &P, false);
    if (rc) break;
    char* base = (char*)ws;
    int64_t* d_info = (int64_t*)(base + lay.info);
    const uintptr_t slots = (uintptr_t)(base + lay.slots);
    const int64_t es = dtype == CHOLMOD_F64 ? 8 : 4;
    // device address of element (b * 64, 0) of a panel: slot base minus the
    // rows before the block, so the kernels index rows and columns as in L
    auto row_base = [&](int64_t b) -> void* {
      const uintptr_t slot = slots + (uintptr_t)(b % kOocSlots) * lay.slot_bytes;
      return (void*)(slot - (uintptr_t)(b * kBlock * n * es));
    };
    P.fac[0].L = nullptr;  // the entries carry the panel addresses
    P.fac[0].info = d_info;
    for (BatchEntry& e : P.ent) {
      const int64_t b = e.pc / kBlock;
      e.Lc = row_base(b);
      e.La = e.pa >= 0 ? row_base(b - 1) : e.Lc;
    }
    std::vector<char> tables(P.table_bytes);
    std::memcpy(tables.data(), P.fac.data(), sizeof(BatchFactor));
    std::memcpy(tables.data() + P.off_ent, P.ent.data(), P.ent.size() * sizeof(BatchEntry));
    if (hipMemcpyAsync(ws, tables.data(), P.table_bytes, hipMemcpyHostToDevice, st) !=
        hipSuccess) {
      rc = CHOLMOD_ERR_HIP;
      break;
    }
    const BatchFactor* d_fac = (const BatchFactor*)ws;
    const BatchEntry* d_ent = (const BatchEntry*)(base + P.off_ent);
    if (run_sysblk_batch_prepare(st, d_fac, 1) != hipSuccess) {
      rc = CHOLMOD_ERR_HIP;
      break;
    }
    const int64_t nb = ceil_div(n, kBlock);
    // Copies in run on `up`, copies out on `down`, steps on `st`: the copy
    // engines move a panel in and another out while a step runs.  Events:
    // in_done[slot] (panel copied in), out_done[slot] (panel copied out),
    // step_done.  A panel is copied into a slot after the slot's previous
    // panel has been copied out, and (in a later pass) after its own copy
    // out of the previous pass: both are ordered on `down` before the
    // latest out_done record of the slot.
    hipStream_t up = nullptr, down = nullptr;
    hipEvent_t in_done[kOocSlots] = {}, out_done[kOocSlots] = {}, step_done = nullptr;
    // Pageable host memory reaches the copy engines only through the
    // runtime's own staging, far below the link rate, so such a factor goes
    // through pinned buffers of this call: host threads pack a panel's rows
    // into one of two in-buffers before its upload, and unpack a downloaded
    // panel from one of two out-buffers two downloads later, before the
    // panel is read again in the next pass, or at the end.  Every host wait
    // is for copies already enqueued.
    const bool staged = !host_pinned(L_host);
    const size_t sbytes = (size_t)(kBlock * n * es);
    char* sin[2] = {nullptr, nullptr};
    char* sout[2] = {nullptr, nullptr};
    hipEvent_t sin_free[2] = {}, sout_full[2] = {};
    bool sin_used[2] = {false, false};
    int64_t pend[2] = {-1, -1};  // panel waiting in sout[i] to be unpacked
    int64_t n_in = 0, n_out = 0;
    std::unique_ptr<RowCopier> copier;
    auto create = [&]() {
      if (hipStreamCreateWithFlags(&up, hipStreamNonBlocking) != hipSuccess) return false;
      if (hipStreamCreateWithFlags(&down, hipStreamNonBlocking) != hipSuccess) return false;
      for (int q = 0; q < kOocSlots; ++q) {
        if (hipEventCreateWithFlags(&in_done[q], hipEventDisableTiming) != hipSuccess) return false;
        if (hipEventCreateWithFlags(&out_done[q], hipEventDisableTiming) != hipSuccess)
          return false;
      }
      if (hipEventCreateWithFlags(&step_done, hipEventDisableTiming) != hipSuccess) return false;
      if (!staged) return true;
      for (int i = 0; i < 2; ++i) {
        if (hipHostMalloc((void**)&sin[i], sbytes, hipHostMallocDefault) != hipSuccess)
          return false;
        if (hipHostMalloc((void**)&sout[i], sbytes, hipHostMallocDefault) != hipSuccess)
          return false;
        if (hipEventCreateWithFlags(&sin_free[i], hipEventDisableTiming) != hipSuccess)
          return false;
        if (hipEventCreateWithFlags(&sout_full[i], hipEventDisableTiming) != hipSuccess)
          return false;
      }
      copier.reset(new RowCopier(3));
      return true;
    };
    // rows [b*64, b*64 + rows) of L, columns b*64 .. n-1: in the device slot
    // (row pitch n), in the host factor (row pitch ldl)
    auto rows_of = [&](int64_t b) { return std::min(kBlock, n - b * kBlock); };
    auto width_of = [&](int64_t b) { return (size_t)((n - b * kBlock) * es); };
    auto dev_panel = [&](int64_t b) {
      return (char*)row_base(b) + (b * kBlock * n + b * kBlock) * es;
    };
    auto host_panel = [&](int64_t b) {
      return (char*)L_host + (b * kBlock * ldl + b * kBlock) * es;
    };
    // the download waiting in sout[i] goes to the host factor
    auto unpack = [&](int i) {
      if (pend[i] < 0) return true;
      if (hipEventSynchronize(sout_full[i]) != hipSuccess) return false;
      const int64_t b = pend[i];
      copier->run(host_panel(b), (size_t)(ldl * es), sout[i], width_of(b), width_of(b),
                  rows_of(b));
      pend[i] = -1;
      return true;
    };
    auto copy_in = [&](int64_t b) {
      const int64_t q = b % kOocSlots;
      const size_t wb = width_of(b);
      if (hipStreamWaitEvent(up, out_done[q], 0) != hipSuccess) return false;
      if (!staged) {
        if (hipMemcpy2DAsync(dev_panel(b), (size_t)(n * es), host_panel(b), (size_t)(ldl * es),
                             wb, (size_t)rows_of(b), hipMemcpyHostToDevice, up) != hipSuccess)
          return false;
      } else {
        const int i = (int)(n_in++ & 1);
        if (sin_used[i] && hipEventSynchronize(sin_free[i]) != hipSuccess) return false;
        for (int j = 0; j < 2; ++j)
          if (pend[j] == b && !unpack(j)) return false;  // the previous pass's result
        copier->run(sin[i], wb, host_panel(b), (size_t)(ldl * es), wb, rows_of(b));
        if (hipMemcpy2DAsync(dev_panel(b), (size_t)(n * es), sin[i], wb, wb, (size_t)rows_of(b),
                             hipMemcpyHostToDevice, up) != hipSuccess ||
            hipEventRecord(sin_free[i], up) != hipSuccess)
          return false;
        sin_used[i] = true;
      }
      return hipEventRecord(in_done[q], up) == hipSuccess;
    };
    auto copy_out = [&](int64_t b) {
      const size_t wb = width_of(b);
      if (hipStreamWaitEvent(down, step_done, 0) != hipSuccess) return false;
      if (!staged) {
        if (hipMemcpy2DAsync(host_panel(b), (size_t)(ldl * es), dev_panel(b), (size_t)(n * es),
                             wb, (size_t)rows_of(b), hipMemcpyDeviceToHost, down) != hipSuccess)
          return false;
      } else {
        const int i = (int)(n_out++ & 1);
        if (!unpack(i)) return false;
        if (hipMemcpy2DAsync(sout[i], wb, dev_panel(b), (size_t)(n * es), wb, (size_t)rows_of(b),
                             hipMemcpyDeviceToHost, down) != hipSuccess ||
            hipEventRecord(sout_full[i], down) != hipSuccess)
          return false;
        pend[i] = b;
      }
      return hipEventRecord(out_done[b % kOocSlots], down) == hipSuccess;
    };
    bool good = create();
    for (int64_t s = 0; good && s < (int64_t)P.steps.size(); ++s) {
      const int64_t b = s % nb, q = b % kOocSlots;
      good = copy_in(b) && hipStreamWaitEvent(st, in_done[q], 0) == hipSuccess &&
             run_sysblk_batch_step(st, d_fac, d_ent, P.steps[s]) == hipSuccess &&
             hipEventRecord(step_done, st) == hipSuccess;
      if (good && b > 0) good = copy_out(b - 1);
      if (good && b == nb - 1) good = copy_out(b);
    }
    // the caller's stream waits for the last copies out
    if (good && nb > 0)
      good = hipStreamWaitEvent(st, out_done[(nb - 1) % kOocSlots], 0) == hipSuccess;
    if (good && nb > 1)
      good = hipStreamWaitEvent(st, out_done[(nb - 2) % kOocSlots], 0) == hipSuccess;
    if (up && hipStreamSynchronize(up) != hipSuccess) good = false;
    if (down && hipStreamSynchronize(down) != hipSuccess) good = false;
    // the older pending download first
    if (good && staged) good = unpack((int)(n_out & 1)) && unpack((int)((n_out + 1) & 1));
    copier.reset();
    for (int i = 0; i < 2; ++i) {
      if (sin[i]) hipHostFree(sin[i]);
      if (sout[i]) hipHostFree(sout[i]);
      if (sin_free[i]) hipEventDestroy(sin_free[i]);
      if (sout_full[i]) hipEventDestroy(sout_full[i]);
    }
    for (int q = 0; q < kOocSlots; ++q) {
      if (in_done[q]) hipEventDestroy(in_done[q]);
      if (out_done[q]) hipEventDestroy(out_done[q]);
    }
    if (step_done) hipEventDestroy(step_done);
    if (up) hipStreamDestroy(up);
    if (down) hipStreamDestroy(down);
    if (!good) rc = CHOLMOD_ERR_HIP;
    if (rc) break;
    if (hipMemcpyAsync(&host_info, d_info, sizeof(int64_t), hipMemcpyDeviceToHost, st) !=
            hipSuccess ||
        hipStreamSynchronize(st) != hipSuccess)
      rc = CHOLMOD_ERR_HIP;
  } while (false);
  if (own) {
    if (hipStreamSynchronize(st) != hipSuccess) rc = CHOLMOD_ERR_HIP;
    hipFree(ws);
  }
  if (rc) return rc;
  if (info_out) *info_out = host_info;
  return cholmod_decode_info(host_info, k, nullptr, nullptr);
}

}  // namespace chm

using namespace chm;

extern "C" {

int cholmod_version(void) { return 100; }

const char* cholmod_status_string(int status) {
  switch (status) {
    case CHOLMOD_OK: return "ok";
    case CHOLMOD_ERR_ARG: return "invalid argument";
    case CHOLMOD_ERR_NOT_PD: return "modified matrix is not positive definite";
    case CHOLMOD_ERR_BAD_DIAG: return "input factor has a diagonal entry that is not > 0";
    case CHOLMOD_ERR_HIP: return "HIP runtime error";
    default: return "unknown status";
  }
}

int cholmod_decode_info(int64_t info, int64_t k, int64_t* row, int64_t* col) {
  if (row) *row = -1;
  if (col) *col = -1;
  if (info == CHOLMOD_INFO_NONE) return CHOLMOD_OK;
  const int64_t code = info & 3, index = info >> 2;
  if (k > 0) {
    if (row) *row = index / k;
    if (col) *col = index % k;
  }
  if (code == kCodeNotPD) return CHOLMOD_ERR_NOT_PD;
  if (code == kCodeBadDiag) return CHOLMOD_ERR_BAD_DIAG;
  return CHOLMOD_ERR_HIP;  // a bounded device-side wait gave up
}

size_t cholmod_workspace_bytes(int64_t n, int64_t k, int dtype) {
  WsLayout lay;
  if (!layout_for(n, k, dtype, &lay)) return 0;
  return lay.total;
}

int cholmod_update_ex(double* L, const double* V, int64_t n, int64_t k, int64_t ldl, int sigma,
                      unsigned flags, void* ws, size_t ws_bytes, int64_t* d_info,
                      cholmod_stream_t stream) {
  return enqueue_f64(L, V, n, k, ldl, sigma, flags, ws, ws_bytes, d_info, (hipStream_t)stream);
}

int cholmod_update_async(double* L, const double* V, int64_t n, int64_t k, int64_t ldl,
                         int sigma, void* ws, size_t ws_bytes, int64_t* d_info,
                         cholmod_stream_t stream) {
  return enqueue_f64(L, V, n, k, ldl, sigma, 0u, ws, ws_bytes, d_info, (hipStream_t)stream);
}

int cholmod_update(double* L, const double* V, int64_t n, int64_t k, int64_t ldl, int sigma,
                   cholmod_stream_t stream) {
  int v = validate(L, V, n, k, ldl, sigma);
  if (v) return v;
  return run_sync(n, k, CHOLMOD_F64, (hipStream_t)stream,
                  [&](void* ws, size_t bytes, int64_t* d_info, hipStream_t st) {
                    return enqueue_f64(L, V, n, k, ldl, sigma, 0u, ws, bytes, d_info, st);
                  });
}

int cholmod_probe_latency(int k, int blocks, int rounds, double* out4, cholmod_stream_t stream) {
  if (k < 1 || k > 16 || blocks < 1 || blocks > 100000 || rounds < 1 || rounds > 1000000 ||
      out4 == nullptr)
    return CHOLMOD_ERR_ARG;
  int timed_out = 0;
  if (run_probe_latency((hipStream_t)stream, k, blocks, rounds, out4, &timed_out) != hipSuccess)
    return CHOLMOD_ERR_HIP;
  return timed_out ? CHOLMOD_ERR_HIP : CHOLMOD_OK;
}

size_t cholmod_noalloc_max_bytes(void) { return kScratchBytes; }

int cholmod_update_noalloc(double* L, const double* V, int64_t n, int64_t k, int64_t ldl,
                           int sigma, int64_t* d_info, cholmod_stream_t stream) {
  // every check before any HIP call
  const int v = validate(L, V, n, k, ldl, sigma);
  if (v) return v;
  if (d_info == nullptr || ((uintptr_t)d_info & 7u) != 0) return CHOLMOD_ERR_ARG;
  WsLayout lay;
  if (!layout_for(n, k, CHOLMOD_F64, &lay) || lay.total > kScratchBytes) return CHOLMOD_ERR_ARG;
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return CHOLMOD_ERR_HIP;
  void* ws = scratch_address(dev);
  if (ws == nullptr) return CHOLMOD_ERR_HIP;
  return enqueue_f64(L, V, n, k, ldl, sigma, 0u, ws, kScratchBytes, d_info, (hipStream_t)stream);
}

int cholmod_update_f32s_async(float* L, const float* V, int64_t n, int64_t k, int64_t ldl,
                              int sigma, void* ws, size_t ws_bytes, int64_t* d_info,
                              cholmod_stream_t stream) {
  return enqueue_f32s(L, V, n, k, ldl, sigma, 0u, ws, ws_bytes, d_info, (hipStream_t)stream);
}

int cholmod_update_f32s_ex(float* L, const float* V, int64_t n, int64_t k, int64_t ldl,
                           int sigma, unsigned flags, void* ws, size_t ws_bytes, int64_t* d_info,
                           cholmod_stream_t stream) {
  return enqueue_f32s(L, V, n, k, ldl, sigma, flags, ws, ws_bytes, d_info, (hipStream_t)stream);
}

int cholmod_update_f32s(float* L, const float* V, int64_t n, int64_t k, int64_t ldl, int sigma,
                        cholmod_stream_t stream) {
  int v = validate(L, V, n, k, ldl, sigma);
  if (v) return v;
  return run_sync(n, k, CHOLMOD_F32S, (hipStream_t)stream,
                  [&](void* ws, size_t bytes, int64_t* d_info, hipStream_t st) {
                    return enqueue_f32s(L, V, n, k, ldl, sigma, 0u, ws, bytes, d_info, st);
                  });
}

size_t cholmod_workspace_bytes_ooc(int64_t n, int64_t k, int dtype) {
  OocLayout lay;
  if (!ooc_layout(n, k, dtype, &lay)) return 0;
  return lay.total;
}

int cholmod_update_ooc(void* L_host, const void* V, int64_t n, int64_t k, int64_t ldl,
                       int sigma, int dtype, void* ws, size_t ws_bytes, int64_t* info,
                       cholmod_stream_t stream) {
  return update_ooc(L_host, V, n, k, ldl, sigma, dtype, ws, ws_bytes, (hipStream_t)stream,
                    info);
}

struct cholmod_batch_graph {
  hipGraphExec_t exec = nullptr;
};

int cholmod_batch_graph_create(const cholmod_desc* descs, int64_t count, void* ws,
                               size_t ws_bytes, int64_t* d_info, cholmod_batch_graph** out) {
  if (out == nullptr) return CHOLMOD_ERR_ARG;
  *out = nullptr;
  if (count < 1) return CHOLMOD_ERR_ARG;
  const size_t need = batch_workspace_bytes_any(descs, count);
  if (need == 0) return CHOLMOD_ERR_ARG;
  if (d_info == nullptr || ((uintptr_t)d_info & 7u) != 0) return CHOLMOD_ERR_ARG;
  if (ws == nullptr || ws_bytes < need || ((uintptr_t)ws % kAlign) != 0) return CHOLMOD_ERR_ARG;
  const cholmod_plan lp = select_plan(descs, count);
  BatchPlan P;
  int rc = plan_batch(descs, count, (char*)ws, &P, lp.schedule == CHOLMOD_SCHED_QUEUED, lp.order,
                      lp.maps != 0);
  if (rc) return rc;
  P.grid = lp.grid;
  P.poll = lp.poll;
  for (int64_t f = 0; f < count; ++f) P.fac[f].info = d_info + f;
  std::vector<char> tables(P.table_bytes);
  write_tables(P, tables.data());
  // the tables stay in the workspace: the graph holds kernel launches only
  if (hipMemcpy(ws, tables.data(), P.table_bytes, hipMemcpyHostToDevice) != hipSuccess)
    return CHOLMOD_ERR_HIP;
  hipStream_t cs = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  rc = CHOLMOD_ERR_HIP;
  if (hipStreamCreateWithFlags(&cs, hipStreamNonBlocking) == hipSuccess) {
    if (hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal) == hipSuccess) {
      const hipError_t e = run_planned(cs, P, (char*)ws, count);
      const hipError_t ee = hipStreamEndCapture(cs, &graph);
      if (e == hipSuccess && ee == hipSuccess && graph != nullptr &&
          hipGraphInstantiate(&exec, graph, nullptr, nullptr, 0) == hipSuccess)
        rc = CHOLMOD_OK;
    }
    hipStreamDestroy(cs);
  }
  if (graph) hipGraphDestroy(graph);
  if (rc) return rc;
  *out = new cholmod_batch_graph;
  (*out)->exec = exec;
  return CHOLMOD_OK;
}

int cholmod_batch_graph_launch(cholmod_batch_graph* g, cholmod_stream_t stream) {
  if (g == nullptr || g->exec == nullptr) return CHOLMOD_ERR_ARG;
  return hipGraphLaunch(g->exec, (hipStream_t)stream) == hipSuccess ? CHOLMOD_OK
                                                                     : CHOLMOD_ERR_HIP;
}

int cholmod_batch_graph_destroy(cholmod_batch_graph* g) {
  if (g == nullptr) return CHOLMOD_OK;
  const hipError_t e = g->exec ? hipGraphExecDestroy(g->exec) : hipSuccess;
  delete g;
  return e == hipSuccess ? CHOLMOD_OK : CHOLMOD_ERR_HIP;
}

size_t cholmod_workspace_bytes_batched(const cholmod_desc* descs, int64_t count) {
  return batch_workspace_bytes_any(descs, count);
}

int cholmod_plan_bucket(int64_t n, int64_t k, int* n_bucket, int* k_bucket) {
  if (n < 0 || k < 0) return CHOLMOD_ERR_ARG;
  if (n_bucket) *n_bucket = bucket_of(n, kNBucketTop, kNBuckets);
  if (k_bucket) *k_bucket = bucket_of(k, kKBucketTop, kKBuckets);
  return CHOLMOD_OK;
}

int cholmod_set_plan(int dtype, int n_bucket, int k_bucket, const cholmod_plan* plan) {
  if (dtype != CHOLMOD_F64 && dtype != CHOLMOD_F32S) return CHOLMOD_ERR_ARG;
  if (n_bucket < 0 || n_bucket >= kNBuckets || k_bucket < 0 || k_bucket >= kKBuckets)
    return CHOLMOD_ERR_ARG;
  if (plan == nullptr || !plan_ok(*plan)) return CHOLMOD_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_plan_mu);
  g_plans.p[dtype == CHOLMOD_F64 ? 0 : 1][n_bucket][k_bucket] = *plan;
  return CHOLMOD_OK;
}

int cholmod_get_plan(int dtype, int n_bucket, int k_bucket, cholmod_plan* plan) {
  if (dtype != CHOLMOD_F64 && dtype != CHOLMOD_F32S) return CHOLMOD_ERR_ARG;
  if (n_bucket < 0 || n_bucket >= kNBuckets || k_bucket < 0 || k_bucket >= kKBuckets)
    return CHOLMOD_ERR_ARG;
  if (plan == nullptr) return CHOLMOD_ERR_ARG;
  std::lock_guard<std::mutex> lk(g_plan_mu);
  *plan = g_plans.p[dtype == CHOLMOD_F64 ? 0 : 1][n_bucket][k_bucket];
  return CHOLMOD_OK;
}

int cholmod_compute_units(void) {
  int n = 0;
  if (hipGetDevice(&n) != hipSuccess) return 0;
  return compute_units();
}

int cholmod_update_batched(const cholmod_desc* descs, int64_t count, void* ws, size_t ws_bytes,
                           int64_t* d_info, cholmod_stream_t stream) {
  return cholmod_update_batched_plan(descs, count, nullptr, ws, ws_bytes, d_info, stream);
}

int cholmod_update_batched_plan(const cholmod_desc* descs, int64_t count,
                                const cholmod_plan* plan, void* ws, size_t ws_bytes,
                                int64_t* d_info, cholmod_stream_t stream) {
  // every argument check happens here, before any HIP call
  if (count < 0) return CHOLMOD_ERR_ARG;
  if (count == 0) return CHOLMOD_OK;
  if (plan != nullptr && !plan_ok(*plan)) return CHOLMOD_ERR_ARG;
  const size_t need = batch_workspace_bytes_any(descs, count);
  if (need == 0) return CHOLMOD_ERR_ARG;
  if (d_info == nullptr || ((uintptr_t)d_info & 7u) != 0) return CHOLMOD_ERR_ARG;
  if (ws == nullptr || ws_bytes < need || ((uintptr_t)ws % kAlign) != 0) return CHOLMOD_ERR_ARG;
  const cholmod_plan lp = plan ? *plan : select_plan(descs, count);
  const size_t tb = batch_table_bytes(descs, count, lp.schedule == CHOLMOD_SCHED_QUEUED);
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return CHOLMOD_ERR_HIP;
  std::lock_guard<std::mutex> lk(g_mu);
  if ((int)g_ws.size() <= dev) g_ws.resize(dev + 1);
  DevWs& d = g_ws[dev];
  // the pinned staging buffer is reused: wait for its previous upload (not
  // for the previous batch, so that this batch's planning overlaps it)
  if (d.stage_pending) {
    if (hipEventSynchronize(d.stage_done) != hipSuccess) return CHOLMOD_ERR_HIP;
    d.stage_pending = false;
  }
  if (!d.stage_done && hipEventCreateWithFlags(&d.stage_done, hipEventDisableTiming) != hipSuccess)
    return CHOLMOD_ERR_HIP;
  if (d.stage_bytes < tb) {
    if (d.stage) hipHostFree(d.stage);
    d.stage = nullptr;
    d.stage_bytes = 0;
    if (hipHostMalloc(&d.stage, tb, hipHostMallocDefault) != hipSuccess) return CHOLMOD_ERR_HIP;
    d.stage_bytes = tb;
  }
  hipStream_t st = (hipStream_t)stream;
  const int rc = enqueue_batch(descs, count, ws, ws_bytes, d_info, st, d.stage, d.stage_bytes,
                               nullptr, nullptr, &lp, d.stage_done);
  // the event may have been recorded even if a later launch failed
  d.stage_pending = true;
  if (rc) return rc;
  return CHOLMOD_OK;
}

}  // extern "C"
