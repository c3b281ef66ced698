// blocked.hip -- host-driven blocked schedule of CholeskyModifyB.
//
// Rows are taken in blocks R_p = [p0, p0 + bb).  For each block:
//   * k_block_diag (one workgroup) runs Algorithm 1 restricted to the block:
//     for each row r of the block, the k Compute steps of row r (ascending
//     column order), then the Apply of row r to the columns of the block to
//     the right of r.  It stores the block's rotation table T_p = {c, s, 1/c}.
//   * k_block_trail (one thread per trailing column j >= p0 + bb) applies
//     the rotations of all rows of the block, in row order, to L[r, j] and to
//     the private copy W[j, :] of V (Apply, Algorithm 1; the trailing part of
//     the inner loop of CholeskyModifyB).
// Because row i of L is changed only while row i is processed, this is a
// reordering of the same operations as the serial algorithm.
#include "rotations.h"

namespace chm {

constexpr int kDiagRows = 32;  // block rows handled by k_block_diag
constexpr int kKMax = 64;      // V columns handled per pass

template <bool EXACT>
__global__ __launch_bounds__(64) void k_block_diag(double* __restrict__ L, int64_t ldl,
                                                   double* __restrict__ W, int64_t ldw, int kc,
                                                   int64_t kfull, int64_t m0, double sg, int64_t p0,
                                                   int bb, Coef* __restrict__ T,
                                                   int64_t* __restrict__ info,
                                                   int64_t* __restrict__ stop_row) {
  __shared__ double Wb[kDiagRows][kKMax + 1];
  __shared__ double Lb[kDiagRows][kDiagRows + 1];
  __shared__ Coef Tr[kKMax];
  __shared__ int fail;
  // Rows at or after the first failing row are not processed (a failure
  // found by an earlier column pass still lets later passes finish the rows
  // before it, so the first failure in (row, column) order is the one kept).
  const int64_t lim = __hip_atomic_load(stop_row, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (p0 >= lim) return;
  if (lim - p0 < bb) bb = (int)(lim - p0);
  const int tid = threadIdx.x;
  for (int idx = tid; idx < bb * kc; idx += 64) {
    const int i = idx / kc, m = idx % kc;
    Wb[i][m] = W[(p0 + i) * ldw + m];
  }
  for (int idx = tid; idx < bb * bb; idx += 64) {
    const int i = idx / bb, j = idx % bb;
    if (j >= i) Lb[i][j] = L[(p0 + i) * ldl + p0 + j];
  }
  if (tid == 0) fail = 0;
  __syncthreads();
  int rows_done = 0;
  for (int r = 0; r < bb; ++r) {
    if (tid == 0) {
      int code = 0, m = 0;
      if constexpr (EXACT) {
        double l = Lb[r][r];
        for (m = 0; m < kc; ++m) {
          code = compute_exact(l, Wb[r][m], sg, Tr[m]);
          if (code) break;
        }
        Lb[r][r] = l;
      } else {
        FastDiag d = fast_diag_init(Lb[r][r]);
        for (m = 0; m < kc; ++m) {
          code = compute_fast(d, Wb[r][m], sg, m == 0, Tr[m]);
          if (code) break;
        }
        Lb[r][r] = d.l;
      }
      if (code) {
        atomicMin((unsigned long long*)info,
                  (unsigned long long)info_key((p0 + r) * kfull + m0 + m, code));
        atomicMin((unsigned long long*)stop_row, (unsigned long long)(p0 + r));
        fail = 1;
      } else {
        for (m = 0; m < kc; ++m) T[(p0 + r) * kc + m] = Tr[m];
      }
    }
    __syncthreads();
    if (fail) break;
    if (tid > r && tid < bb) {
      double x = Lb[r][tid];
      for (int m = 0; m < kc; ++m) apply_rot<EXACT>(Tr[m], sg, x, Wb[tid][m]);
      Lb[r][tid] = x;
    }
    rows_done = r + 1;
    __syncthreads();
  }
  for (int idx = tid; idx < rows_done * bb; idx += 64) {
    const int i = idx / bb, j = idx % bb;
    if (j >= i) L[(p0 + i) * ldl + p0 + j] = Lb[i][j];
  }
  for (int idx = tid; idx < bb * kc; idx += 64) {
    const int i = idx / kc, m = idx % kc;
    W[(p0 + i) * ldw + m] = Wb[i][m];
  }
}

template <bool EXACT, int KB>
__global__ __launch_bounds__(64) void k_block_trail(double* __restrict__ L, int64_t ldl,
                                                    double* __restrict__ W, int64_t ldw, int kc,
                                                    int64_t n, double sg, int64_t p0, int bb,
                                                    const Coef* __restrict__ T,
                                                    const int64_t* __restrict__ stop_row) {
  const int64_t j = p0 + bb + (int64_t)blockIdx.x * 64 + threadIdx.x;
  const int64_t lim = __hip_atomic_load(stop_row, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (p0 >= lim) return;
  if (lim - p0 < bb) bb = (int)(lim - p0);
  if (j >= n) return;
  double w[KB];
#pragma unroll
  for (int m = 0; m < KB; ++m) w[m] = (m < kc) ? W[j * ldw + m] : 0.0;
  for (int r = 0; r < bb; ++r) {
    const Coef* tr = T + (p0 + r) * kc;
    double* lp = L + (p0 + r) * ldl + j;
    double x = *lp;
#pragma unroll
    for (int m = 0; m < KB; ++m) {
      if (m < kc) apply_rot<EXACT>(tr[m], sg, x, w[m]);
    }
    *lp = x;
  }
#pragma unroll
  for (int m = 0; m < KB; ++m)
    if (m < kc) W[j * ldw + m] = w[m];
}

template <bool EXACT, int KB>
static void launch_trail(hipStream_t st, double* L, int64_t ldl, double* W, int64_t ldw, int kc,
                         int64_t n, double sg, int64_t p0, int bb, const Coef* T, const int64_t* stop) {
  const int64_t cols = n - p0 - bb;
  const unsigned grid = (unsigned)((cols + 63) / 64);
  hipLaunchKernelGGL((k_block_trail<EXACT, KB>), dim3(grid), dim3(64), 0, st, L, ldl, W, ldw, kc,
                     n, sg, p0, bb, T, stop);
}

template <bool EXACT>
static void launch_trail_k(hipStream_t st, double* L, int64_t ldl, double* W, int64_t ldw, int kc,
                           int64_t n, double sg, int64_t p0, int bb, const Coef* T,
                           const int64_t* stop) {
  if (kc <= 1) launch_trail<EXACT, 1>(st, L, ldl, W, ldw, kc, n, sg, p0, bb, T, stop);
  else if (kc <= 2) launch_trail<EXACT, 2>(st, L, ldl, W, ldw, kc, n, sg, p0, bb, T, stop);
  else if (kc <= 4) launch_trail<EXACT, 4>(st, L, ldl, W, ldw, kc, n, sg, p0, bb, T, stop);
  else if (kc <= 8) launch_trail<EXACT, 8>(st, L, ldl, W, ldw, kc, n, sg, p0, bb, T, stop);
  else if (kc <= 16) launch_trail<EXACT, 16>(st, L, ldl, W, ldw, kc, n, sg, p0, bb, T, stop);
  else if (kc <= 32) launch_trail<EXACT, 32>(st, L, ldl, W, ldw, kc, n, sg, p0, bb, T, stop);
  else launch_trail<EXACT, 64>(st, L, ldl, W, ldw, kc, n, sg, p0, bb, T, stop);
}

// One pass over the rows for V columns [m0, m0 + kc) (kc <= 64).
template <bool EXACT>
static hipError_t run_blocked_pass(hipStream_t st, double* L, int64_t n, int64_t ldl, double* W,
                                   int64_t kfull, int64_t m0, int kc, double sg, Coef* T,
                                   int64_t* info, int64_t* stop) {
  double* Wc = W + m0;
  for (int64_t p0 = 0; p0 < n; p0 += kDiagRows) {
    const int bb = (int)((n - p0) < kDiagRows ? (n - p0) : kDiagRows);
    hipLaunchKernelGGL((k_block_diag<EXACT>), dim3(1), dim3(64), 0, st, L, ldl, Wc, kfull, kc,
                       kfull, m0, sg, p0, bb, T, info, stop);
    if (p0 + bb < n) launch_trail_k<EXACT>(st, L, ldl, Wc, kfull, kc, n, sg, p0, bb, T, stop);
  }
  return hipGetLastError();
}

hipError_t run_blocked(hipStream_t st, double* L, int64_t n, int64_t ldl, double* W, int64_t k,
                       double sg, Coef* T, int64_t* info, int64_t* stop, bool exact) {
  for (int64_t m0 = 0; m0 < k; m0 += kKMax) {
    const int kc = (int)((k - m0) < kKMax ? (k - m0) : kKMax);
    hipError_t e = exact ? run_blocked_pass<true>(st, L, n, ldl, W, k, m0, kc, sg, T, info, stop)
                         : run_blocked_pass<false>(st, L, n, ldl, W, k, m0, kc, sg, T, info, stop);
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace chm
