// sysblk.hip -- blocked schedule of CholeskyModifyB for the fast evaluation
// mode: per block of 64 rows, one workgroup runs the block's rows from LDS
// (k_block_chain), then a column-parallel kernel applies the block's
// rotations to every column to the right of the block (k_block_apply).
// Up to 16 columns of V per pass.
//
// k_block_chain.  The serial dependence of Algorithm 1 runs through the rows:
// Compute(i, m) needs V_i after the Apply of rows 0..i-1, and L_ii after
// Compute(i, m-1).  Wave 0 is a systolic pipeline over the columns of V:
// lane m runs Compute(i, m) at step t = i + m and passes L_ii^2 and 1/L_ii to
// lane m+1 (DPP row shift).  A block column j (relative index) needs the
// rotations of every earlier block row before it becomes the diagonal:
//   * rows r < j - 2 are applied by two helper waves, one thread per column,
//     in diagonal order: at step t the helper applies (r, m) with
//     r + m = t - 1, whose coefficients wave 0 wrote to LDS at step t - 1;
//     wave 1 takes columns m < 8 of V and wave 2 columns m >= 8, the partly
//     rotated L_rj moving from wave 1 to wave 2 through LDS;
//   * when row j - 3 is done for column m, the helper leaves V_j[m] in LDS
//     and wave 0 applies rows j - 2 and j - 1 itself (lane m at step
//     j - 1 + m, the partly rotated L_rj moving from lane m to lane m+1), so
//     V_j is ready for Compute(j, m) at the next step.
// The step loop touches only LDS; the block is loaded before and written
// after it.
//
// k_block_apply.  One column per group of KS lanes; lane g of a group applies
// columns [g*RPL, (g+1)*RPL) of V's rotations to the column, taking row
// r at sub-step r + g, so the partly rotated L_rj moves to the next lane
// with a DPP row shift.  The block's rotation records sit in LDS.
//
// Each Compute and Apply is the fast-mode arithmetic of rotations.h, applied
// to every element in the same order as the serial algorithm, so the result
// is bit-identical to the other fast schedule.
#include "rotations.h"

namespace chm {

constexpr int kBR = 64;   // block rows
constexpr int kKP = 16;   // V columns per pass

__device__ __forceinline__ double sb_shr1(double x, double fill) {
  const uint64_t b = __builtin_bit_cast(uint64_t, x);
  const uint64_t f = __builtin_bit_cast(uint64_t, fill);
  int lo = __builtin_amdgcn_update_dpp((int)(uint32_t)f, (int)(uint32_t)b, 0x111, 0xF, 0xF, false);
  int hi = __builtin_amdgcn_update_dpp((int)(uint32_t)(f >> 32), (int)(uint32_t)(b >> 32), 0x111,
                                       0xF, 0xF, false);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

struct ChainBlockLds {
  double Lb[kBR][kBR + 1];      // the block's upper triangle (original, then final)
  Coef ring[kBR][kKP];          // rotation records of the block's rows
  double hand[kBR][kKP + 1];    // V_j after rows < j - 2 (helper -> wave 0)
  double xfer[2][kBR];          // L_rj after rotation 7 (wave 1 -> wave 2)
  int stop;                     // first failing row of the block (relative)
};

// One step of the chain (wave 0).
struct ChainRegs {
  double tp_in, il_in;  // L_ii^2 and 1/L_ii from lane m-1
  double vnext;         // V_i for the next Compute
  double v0;            // V of the block's first row
  double Lf[2];         // L_rj from lane m-1 (lane 0: original)
  Coef prev;            // this lane's record of the previous step's row
};

template <int U>
__device__ __forceinline__ void chain_wave_step(ChainBlockLds& sh, ChainRegs& cr, int t, int m,
                                                int kc, int bb, double sg, int64_t p0,
                                                int64_t kfull, int64_t m0, int64_t* info,
                                                int64_t* stop_row) {
  const int stop = sh.stop;
  const int i = t - m;
  const bool cval = (m < kc) && (i >= 0) && (i < bb) && (i < stop);
  Coef cur;
  cur.c = 1.0; cur.s = 0.0; cur.ic = 1.0; cur.pad = 0.0;
  double tpi = cr.tp_in, ili = cr.il_in, lin;
  if (m == 0) {
    const double l0 = cval ? sh.Lb[i][i] : 1.0;
    lin = l0;
    tpi = l0 * l0;
    ili = 1.0 / l0;
  } else {
    lin = tpi * ili;
  }
  double t_out = tpi, y_out = ili;
  const double v = (i == 0) ? cr.v0 : cr.vnext;
  int code = 0;
  if (cval) {
    if (m == 0 && !(lin > 0.0)) code = kCodeBadDiag;
    const double tt = __builtin_fma(sg * v, v, tpi);
    if (!code && !(tt > 0.0)) code = kCodeNotPD;
    if (!code) {
      const double y = rsqrt_refined(tt);
      const double ww = tt * y;
      cur.c = ww * ili;
      cur.s = v * ili;
      cur.ic = lin * y;
      t_out = tt;
      y_out = y;
      if (m == kc - 1) sh.Lb[i][i] = ww;
    }
  }
  if (code) {
    atomicMin((unsigned long long*)info,
              (unsigned long long)info_key((p0 + i) * kfull + m0 + m, code));
    atomicMin((unsigned long long*)stop_row, (unsigned long long)(p0 + i));
    atomicMin(&sh.stop, i);
  }
  if (cval) sh.ring[i][m] = cur;

  // rows i - 1 and i applied to column jj = i + 1
  const int jj = i + 1;
  const bool jval = (m < kc) && (jj >= 1) && (jj < bb);
  double Wc = jval ? sh.hand[jj][m] : 0.0;
  double Lo[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int r = i - 1 + q;
    const bool rv = jval && r >= 0 && r < stop;
    const Coef cf = (q == 1) ? cur : cr.prev;
    Lo[q] = cr.Lf[q];
    if (rv) {
      const double x = __builtin_fma(sg * cf.s, Wc, cr.Lf[q]) * cf.ic;
      Wc = __builtin_fma(-cf.s, x, cf.c * Wc);
      Lo[q] = x;
      if (m == kc - 1) sh.Lb[r][jj] = x;
    }
  }
  cr.vnext = Wc;
  cr.prev = cur;
  // lane 0 starts the next step with the original L of column i + 2, rows i, i + 1
  // (t + 1 - 0 = i + 1 + m for lane 0, i.e. rows t and t + 1 of column t + 2)
  double fill[2];
#pragma unroll
  for (int q = 0; q < 2; ++q) {
    const int r = t + q, c = t + 2;
    fill[q] = (r < bb && c < bb) ? sh.Lb[r][c] : 0.0;
  }
  cr.Lf[0] = sb_shr1(Lo[0], fill[0]);
  cr.Lf[1] = sb_shr1(Lo[1], fill[1]);
  cr.tp_in = sb_shr1(t_out, 0.0);
  cr.il_in = sb_shr1(y_out, 0.0);
}

// One step of a helper wave: half 0 takes V columns [0, 8), half 1 [8, 16).
template <int HALF, int U>
__device__ __forceinline__ void helper_wave_step(ChainBlockLds& sh, double (&W)[8], double (&Lr)[8],
                                                 int t, int jj, int kc, int bb, double sg) {
  const int stop = sh.stop;
  const int mlo = HALF * 8;
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    const int m = mlo + u;
    if (m >= kc) break;
    const int r = t - 1 - m;
    // ring slot of row r: r mod 8 = (t - 1 - u) mod 8, static once t mod 8 is
    constexpr int dummy = 0;
    (void)dummy;
    const int slot = ((U - 1 - u) % 8 + 8) % 8;
    const bool act = (jj < bb) && (r >= 0) && (r < jj - 2) && (r < stop);
    if (act) {
      double lin;
      if (u == 0) lin = (HALF == 0) ? sh.Lb[r][jj] : sh.xfer[(t - 1) & 1][jj];
      else lin = Lr[slot];
      const Coef cf = sh.ring[r][m];
      const double x = __builtin_fma(sg * cf.s, W[u], lin) * cf.ic;
      W[u] = __builtin_fma(-cf.s, x, cf.c * W[u]);
      Lr[slot] = x;
      if (HALF == 0 && u == 7 && kc > 8) sh.xfer[t & 1][jj] = x;
      if (m == kc - 1) sh.Lb[r][jj] = x;
      if (r == jj - 3) sh.hand[jj][m] = W[u];
    }
  }
}

__global__ __launch_bounds__(256) void k_block_chain(double* __restrict__ L, int64_t ldl,
                                                     const double* __restrict__ W, int64_t ldw,
                                                     int kc, int64_t kfull, int64_t m0, double sg,
                                                     int64_t p0, int bb, Coef* __restrict__ Tout,
                                                     int64_t* __restrict__ info,
                                                     int64_t* __restrict__ stop_row) {
  __shared__ ChainBlockLds sh;
  const int64_t lim = __hip_atomic_load(stop_row, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (p0 >= lim) return;
  if (lim - p0 < bb) bb = (int)(lim - p0);
  const int tid = threadIdx.x;
  const int w = tid >> 6, lane = tid & 63;
  for (int idx = tid; idx < bb * bb; idx += 256) {
    const int i = idx / bb, j = idx % bb;
    if (j >= i) sh.Lb[i][j] = L[(p0 + i) * ldl + p0 + j];
  }
  if (tid == 0) sh.stop = bb;
  // helper state: column jj = lane, V columns [8*half, 8*half + 8)
  double Wh[8], Lr[8];
#pragma unroll
  for (int u = 0; u < 8; ++u) {
    Lr[u] = 0.0;
    const int m = (w - 1) * 8 + u;
    Wh[u] = (w >= 1 && w <= 2 && lane < bb && m < kc) ? W[(p0 + lane) * ldw + m] : 0.0;
  }
  // columns 0..2 have no helper rows: their hand-off value is V as loaded
  if ((w == 1 || w == 2) && lane < bb && lane <= 2) {
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int m = (w - 1) * 8 + u;
      if (m < kc) sh.hand[lane][m] = Wh[u];
    }
  }
  ChainRegs cr;
  cr.tp_in = 1.0;
  cr.il_in = 1.0;
  cr.vnext = 0.0;
  cr.v0 = (w == 0 && lane < kc) ? W[p0 * ldw + lane] : 0.0;
  cr.prev.c = 1.0; cr.prev.s = 0.0; cr.prev.ic = 1.0; cr.prev.pad = 0.0;
  __syncthreads();
  // lane 0 of wave 0 starts with the originals of column 1, rows -1 and 0
  cr.Lf[0] = 0.0;
  cr.Lf[1] = (w == 0 && lane == 0 && bb > 1) ? sh.Lb[0][1] : 0.0;
  const int T = bb + kc - 1;
  for (int t0 = 0; t0 < T; t0 += 8) {
#define SB_STEP(U)                                                                          \
  {                                                                                       \
    const int t = t0 + U;                                                                 \
    if (t < T) {                                                                          \
      if (w == 0) chain_wave_step<U>(sh, cr, t, lane, kc, bb, sg, p0, kfull, m0, info,    \
                                     stop_row);                                           \
      else if (w == 1) helper_wave_step<0, U>(sh, Wh, Lr, t, lane, kc, bb, sg);          \
      else if (w == 2) helper_wave_step<1, U>(sh, Wh, Lr, t, lane, kc, bb, sg);          \
    }                                                                                     \
    __syncthreads();                                                                      \
  }
    SB_STEP(0) SB_STEP(1) SB_STEP(2) SB_STEP(3) SB_STEP(4) SB_STEP(5) SB_STEP(6) SB_STEP(7)
#undef SB_STEP
  }
  // write back the block's triangle and its rotation records
  const int rows = sh.stop < bb ? sh.stop + 1 : bb;
  for (int idx = tid; idx < rows * bb; idx += 256) {
    const int i = idx / bb, j = idx % bb;
    if (j >= i) L[(p0 + i) * ldl + p0 + j] = sh.Lb[i][j];
  }
  for (int idx = tid; idx < bb * kc; idx += 256) {
    const int i = idx / kc, m = idx % kc;
    Tout[(p0 + i) * kKP + m] = sh.ring[i][m];
  }
}

// ------------------------------------------------------------------ apply
constexpr int kApre = 8;  // prefetch distance of L rows (sub-steps)

template <int KS, int RPL>
__global__ __launch_bounds__(256) void k_block_apply(double* __restrict__ L, int64_t ldl,
                                                     double* __restrict__ W, int64_t ldw, int kc,
                                                     int64_t n, double sg, int64_t p0, int bb,
                                                     int64_t c0, const Coef* __restrict__ Tin,
                                                     const int64_t* __restrict__ stop_row,
                                                     double* __restrict__ sink) {
  __shared__ Coef Tb[kBR][kKP];
  const int64_t lim = __hip_atomic_load(stop_row, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  if (p0 >= lim) return;
  if (lim - p0 < bb) bb = (int)(lim - p0);
  const int tid = threadIdx.x;
  for (int idx = tid; idx < bb * kc; idx += 256) {
    const int i = idx / kc, m = idx % kc;
    Tb[i][m] = Tin[(p0 + i) * kKP + m];
  }
  __syncthreads();
  constexpr int CPW = 64 / KS;  // columns per wave
  const int w = tid >> 6, lane = tid & 63;
  const int g = lane % KS;
  const int64_t j = c0 + ((int64_t)blockIdx.x * 4 + w) * CPW + lane / KS;
  const bool jv = j < n;
  double Wr[RPL];
#pragma unroll
  for (int u = 0; u < RPL; ++u) {
    const int m = g * RPL + u;
    Wr[u] = (jv && m < kc) ? W[j * ldw + m] : 0.0;
  }
  double* const sk = sink + lane;
  // lane g = 0 feeds row s of column j at sub-step s; ring slot s mod kApre
  double pre[kApre];
#pragma unroll
  for (int s = 0; s < kApre; ++s) pre[s] = *((g == 0 && jv && s < bb) ? L + (p0 + s) * ldl + j : sk);
  double lcur = 0.0;
  const int S = bb + KS - 1;
  for (int s0 = 0; s0 < S; s0 += kApre) {
#pragma unroll
    for (int u8 = 0; u8 < kApre; ++u8) {
      const int s = s0 + u8;
      if (s < S) {
        const int r = s - g;  // row taken by this lane
        const bool rv = jv && r >= 0 && r < bb;
        double x = (g == 0) ? pre[u8] : lcur;
        {
          const int sn = s + kApre;
          pre[u8] = *((g == 0 && jv && sn < bb) ? L + (p0 + sn) * ldl + j : sk);
        }
        if (rv) {
#pragma unroll
          for (int u = 0; u < RPL; ++u) {
            const int m = g * RPL + u;
            if (m < kc) {
              const Coef cf = Tb[r][m];
              x = __builtin_fma(sg * cf.s, Wr[u], x) * cf.ic;
              Wr[u] = __builtin_fma(-cf.s, x, cf.c * Wr[u]);
            }
          }
        }
        // the last lane of a group holds the final value of row r
        *((g == KS - 1 && rv) ? L + (p0 + r) * ldl + j : sk) = x;
        lcur = sb_shr1(x, 0.0);
      }
    }
  }
#pragma unroll
  for (int u = 0; u < RPL; ++u) {
    const int m = g * RPL + u;
    if (jv && m < kc) W[j * ldw + m] = Wr[u];
  }
}

template <int KS, int RPL>
static void launch_apply(hipStream_t st, double* L, int64_t ldl, double* W, int64_t ldw, int kc,
                         int64_t n, double sg, int64_t p0, int bb, int64_t c0, const Coef* T,
                         const int64_t* stop, double* sink) {
  constexpr int CPB = 4 * (64 / KS);  // columns per block
  const int64_t cols = n - c0;
  const unsigned grid = (unsigned)((cols + CPB - 1) / CPB);
  hipLaunchKernelGGL((k_block_apply<KS, RPL>), dim3(grid), dim3(256), 0, st, L, ldl, W, ldw, kc,
                     n, sg, p0, bb, c0, T, stop, sink);
}

// Fast blocked schedule: V columns in passes of 16, rows in blocks of 64.
// W is the private copy of V (row stride k); T holds n x 16 records.
hipError_t run_sysblk(hipStream_t st, double* L, int64_t n, int64_t ldl, double* W, int64_t k,
                      double sg, Coef* T, int64_t* info, int64_t* stop, double* sink) {
  for (int64_t m0 = 0; m0 < k; m0 += kKP) {
    const int kc = (int)((k - m0) < kKP ? (k - m0) : kKP);
    double* Wc = W + m0;
    for (int64_t p0 = 0; p0 < n; p0 += kBR) {
      const int bb = (int)((n - p0) < kBR ? (n - p0) : kBR);
      hipLaunchKernelGGL(k_block_chain, dim3(1), dim3(256), 0, st, L, ldl, (const double*)Wc, k,
                         kc, k, m0, sg, p0, bb, T, info, stop);
      const int64_t c0 = p0 + bb;
      if (c0 < n) {
        if (kc <= 1) launch_apply<1, 1>(st, L, ldl, Wc, k, kc, n, sg, p0, bb, c0, T, stop, sink);
        else if (kc <= 2) launch_apply<1, 2>(st, L, ldl, Wc, k, kc, n, sg, p0, bb, c0, T, stop, sink);
        else if (kc <= 4) launch_apply<1, 4>(st, L, ldl, Wc, k, kc, n, sg, p0, bb, c0, T, stop, sink);
        else if (kc <= 8) launch_apply<2, 4>(st, L, ldl, Wc, k, kc, n, sg, p0, bb, c0, T, stop, sink);
        else launch_apply<4, 4>(st, L, ldl, Wc, k, kc, n, sg, p0, bb, c0, T, stop, sink);
      }
    }
  }
  return hipGetLastError();
}

}  // namespace chm
