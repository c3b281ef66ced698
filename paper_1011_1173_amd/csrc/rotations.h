// rotations.h -- the per-element arithmetic of Algorithm 1 (Compute, Apply)
// in the two evaluation modes of the library.  Device code for gfx950.
//
// Notation (Section 2, Algorithm 1): for row i and column m of V,
//   Compute:  w = sqrt(L_ii^2 + sigma V_i^2),  c = w / L_ii,  s = V_i / L_ii,
//             L_ii <- w                            (all from the old L_ii)
//   Apply:    L_ij <- (L_ij + sigma s V_j) / c,   V_j <- c V_j - s L_ij
//             (the second statement uses the new L_ij).
//
// EXACT mode evaluates those statements literally in IEEE binary64 (no FMA
// contraction, correctly rounded sqrt and division).
//
// FAST mode evaluates the same rotation with cheaper operations:
//   * the radicand of column m is carried from column m-1: with
//     t_{m-1} = L_ii^2 as it stood before column m, t_m = t_{m-1} + sigma V^2
//     in one fused multiply-add (for m = 0, t_{-1} = L_ii * L_ii);
//   * y = 1/sqrt(t_m) from the hardware reciprocal square root refined by one
//     third-order step (rsqrt_refined); then w = t y, c = w / L_ii = w * (1/L_ii),
//     s = V / L_ii = V * (1/L_ii), and 1/c = L_ii * y; the next column uses
//     L_ii <- w and 1/L_ii <- y;
//   * Apply multiplies by 1/c and uses fused multiply-adds, keeping the new
//     L_ij in the V update.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace chm {

// One rotation of row i against column m: what Apply needs.
struct alignas(32) Coef {
  double c;   // c = w / L_ii
  double s;   // s = V_i / L_ii
  double ic;  // 1 / c (FAST); unused by EXACT
  double pad;
};

// Info word: min over failures of (index << 2 | code); INT64_MAX = none.
enum : int64_t { kCodeNotPD = 1, kCodeBadDiag = 2, kCodeTimeout = 3 };
__device__ __forceinline__ int64_t info_key(int64_t index, int64_t code) {
  return (index << 2) | code;
}

// ---------------------------------------------------------------- EXACT
// Returns 0 or a failure code.  l is the old diagonal (updated in place).
__device__ __forceinline__ int compute_exact(double& l, double v, double sg, Coef& k) {
#pragma clang fp contract(off)
  if (!(l > 0.0)) return kCodeBadDiag;
  const double t = l * l + sg * (v * v);
  if (!(t > 0.0)) return kCodeNotPD;
  const double w = __builtin_sqrt(t);
  k.c = w / l;
  k.s = v / l;
  k.ic = 0.0;
  l = w;
  return 0;
}
__device__ __forceinline__ void apply_exact(const Coef& k, double sg, double& lij, double& vj) {
#pragma clang fp contract(off)
  const double x = (lij + sg * (k.s * vj)) / k.c;
  lij = x;
  vj = k.c * vj - k.s * x;
}

// ---------------------------------------------------------------- FAST
// 1/sqrt(t): the hardware estimate y0 (relative error about 2^-24) refined by
// one third-order step.  With e = 1 - t y0^2, the exact value is
// y0 (1 - e)^(-1/2) = y0 (1 + e/2 + 3 e^2/8 + O(e^3)); the O(e^3) term is
// below 2^-70, so y = y0 + (y0 e) (1/2 + 3 e/8) is within about one ulp --
// as accurate as two Newton steps, in 5 dependent-light operations instead
// of 8.
__device__ __forceinline__ double rsqrt_refined(double t) {
  const double y0 = __builtin_amdgcn_rsq(t);
  const double r = t * y0;
  const double e = __builtin_fma(-r, y0, 1.0);
  const double h = y0 * e;
  const double p = __builtin_fma(e, 0.375, 0.5);
  return __builtin_fma(h, p, y0);
}

// Per-row running state of FAST Compute.
struct FastDiag {
  double tp;  // radicand of the previous column (L_ii^2)
  double il;  // 1 / L_ii
  double l;   // L_ii
};
__device__ __forceinline__ FastDiag fast_diag_init(double lii) {
  FastDiag d;
  d.l = lii;
  d.il = 1.0 / lii;
  d.tp = lii * lii;
  return d;
}
// Returns 0 or a failure code; first == (m == 0) enables the diagonal check.
__device__ __forceinline__ int compute_fast(FastDiag& d, double v, double sg, bool first, Coef& k) {
  if (first && !(d.l > 0.0)) return kCodeBadDiag;
  const double t = __builtin_fma(sg * v, v, d.tp);
  if (!(t > 0.0)) return kCodeNotPD;
  const double y = rsqrt_refined(t);
  const double w = t * y;
  k.c = w * d.il;
  k.s = v * d.il;
  k.ic = d.l * y;
  d.tp = t;
  d.il = y;
  d.l = w;
  return 0;
}
__device__ __forceinline__ void apply_fast(const Coef& k, double sg, double& lij, double& vj) {
  const double x = __builtin_fma(sg * k.s, vj, lij) * k.ic;
  lij = x;
  vj = __builtin_fma(-k.s, x, k.c * vj);
}

template <bool EXACT>
__device__ __forceinline__ void apply_rot(const Coef& k, double sg, double& lij, double& vj) {
  if constexpr (EXACT) apply_exact(k, sg, lij, vj);
  else apply_fast(k, sg, lij, vj);
}

}  // namespace chm
