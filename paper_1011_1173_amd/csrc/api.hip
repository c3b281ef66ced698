// api.hip -- the C ABI (include/cholmod_mi355x.h): argument validation on the
// host, workspace layout, schedule selection and the synchronous wrapper.
#include <hip/hip_runtime.h>

#include <climits>
#include <cstdint>
#include <cstring>
#include <mutex>
#include <vector>

#include "../../include/cholmod_mi355x.h"
#include "rotations.h"

namespace chm {
hipError_t run_blocked(hipStream_t st, double* L, int64_t n, int64_t ldl, double* W, int64_t k,
                       double sg, Coef* T, int64_t* info, int64_t* stop, bool exact);
hipError_t run_sysblk(hipStream_t st, double* L, int64_t n, int64_t ldl, double* W, int64_t k,
                      double sg, Coef* T, int64_t* info, int64_t* stop, double* sink);

namespace {

constexpr size_t kAlign = 256;
constexpr int64_t kKPass = 64;  // V columns per pass of the blocked schedule

inline size_t align_up(size_t x) { return (x + kAlign - 1) / kAlign * kAlign; }

// Workspace layout (all offsets 256-byte aligned):
//   [0, 256)         control words: stop row (int64) at 0, a 64-double sink
//                    (absorbs loads and stores of idle lanes) after it
//   W                n*k private copy of V
//   T                n*max(16, min(k, 64)) rotation records {c, s, 1/c, -}
struct WsLayout {
  size_t ctrl = 0, sink = 0, w = 0, t = 0, total = 0;
};

bool mul_ok(int64_t a, int64_t b, int64_t lim) { return a == 0 || b <= lim / a; }

bool layout_for(int64_t n, int64_t k, int dtype, WsLayout* out) {
  if (n < 0 || k < 0) return false;
  if (dtype != CHOLMOD_F64 && dtype != CHOLMOD_F32S) return false;
  const int64_t lim = INT64_MAX / 64;
  if (!mul_ok(n, k, lim)) return false;
  const size_t es = dtype == CHOLMOD_F64 ? 8 : 4;
  WsLayout L;
  L.ctrl = 0;
  L.sink = 64;
  L.w = 2 * kAlign + 256;  // control words + 64-double sink
  L.t = L.w + align_up((size_t)(n * k) * es);
  int64_t kp = k < kKPass ? k : kKPass;
  if (kp < 16) kp = 16;
  L.total = L.t + align_up((size_t)(n * kp) * sizeof(Coef));
  *out = L;
  return true;
}

__global__ void k_prepare(const double* __restrict__ V, double* __restrict__ W, int64_t count,
                          int64_t* __restrict__ info, int64_t* __restrict__ stop_row) {
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i0 == 0) {
    *info = INT64_MAX;
    *stop_row = INT64_MAX;
  }
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = i0; i < count; i += stride) W[i] = V[i];
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
  if (flags & ~(unsigned)(CHOLMOD_FLAG_EXACT | CHOLMOD_FLAG_BLOCKED)) return CHOLMOD_ERR_ARG;
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
  const bool exact = (flags & CHOLMOD_FLAG_EXACT) != 0;
  const bool blocked = exact || (flags & CHOLMOD_FLAG_BLOCKED) != 0;
  const int64_t count = n * k;  // both schedules work on a private copy of V
  unsigned grid = (unsigned)((count + 255) / 256);
  if (grid < 1) grid = 1;
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(k_prepare, dim3(grid), dim3(256), 0, st, V, W, count, d_info, stop_row);
  if (hipGetLastError() != hipSuccess) return CHOLMOD_ERR_HIP;
  if (n == 0 || k == 0) return CHOLMOD_OK;
  const double sg = (double)sigma;
  hipError_t e;
  if (blocked) {
    e = run_blocked(st, L, n, ldl, W, k, sg, T, d_info, stop_row, exact);
  } else {
    e = run_sysblk(st, L, n, ldl, W, k, sg, T, d_info, stop_row, (double*)(base + lay.sink));
  }
  return e == hipSuccess ? CHOLMOD_OK : CHOLMOD_ERR_HIP;
}

// Library-owned workspace for the synchronous entry point (one per device).
struct DevWs {
  void* ptr = nullptr;
  size_t bytes = 0;
  int64_t* host_info = nullptr;  // pinned
};
std::mutex g_mu;
std::vector<DevWs> g_ws;

}  // namespace
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
  WsLayout lay;
  if (!layout_for(n, k, CHOLMOD_F64, &lay)) return CHOLMOD_ERR_ARG;
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
  hipStream_t st = (hipStream_t)stream;
  int rc = enqueue_f64(L, V, n, k, ldl, sigma, 0u, d.ptr, lay.total, d_info, st);
  if (rc) return rc;
  if (hipMemcpyAsync(d.host_info, d_info, sizeof(int64_t), hipMemcpyDeviceToHost, st) !=
      hipSuccess)
    return CHOLMOD_ERR_HIP;
  if (hipStreamSynchronize(st) != hipSuccess) return CHOLMOD_ERR_HIP;
  return cholmod_decode_info(*d.host_info, k, nullptr, nullptr);
}

}  // extern "C"
