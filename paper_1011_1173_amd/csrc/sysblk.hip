// sysblk.hip -- blocked schedule of CholeskyModifyB for the fast evaluation
// mode.  Rows are processed in blocks of 64 and the columns of V in passes
// of up to 16.  One kernel launch per block b does all the work that becomes
// possible once block b-1 is finished:
//
//   workgroup 0 ("chain"):  applies the rotations of block b-1 to the 64
//     columns of block b (the head tile), then runs the rows of block b from
//     LDS and writes the block's rotation records for the next launch;
//   workgroups 1.. ("rest"): apply the rotations of block b-1 to the columns
//     to the right of block b, 64 columns each, concurrently with the chain.
//
// Every element goes through the same fast-mode operations (rotations.h) in
// the same order as in the per-row schedule, so both schedules give results
// that are identical bit for bit.
//
// The chain.  Algorithm 1 is serial through the rows: Compute(i, m) needs
// V_i after the Apply of rows 0..i-1 and L_ii after Compute(i, m-1).  Wave 0
// is a systolic pipeline over the columns of V: lane m runs Compute(i, m) at
// step t = i + m and passes the running radicand and 1/L_ii to lane m+1 with
// a DPP row shift.  Column j of the block needs the rotations of all earlier
// rows of the block before it becomes the diagonal:
//   * rows r < j - 2 are applied by three helper waves, one lane per column
//     j, in diagonal order: at step t the helper applies (r, m) with
//     r + m = t - 1, whose record wave 0 wrote to LDS at step t - 1; the
//     waves split the columns of V 6 + 5 + 5 and hand the partly rotated
//     L_rj on through LDS;
//   * the helper leaves V_j after row j - 3 in LDS, and lane m of wave 0
//     applies rows j - 2 and j - 1 itself at step j - 1 + m (the partly
//     rotated L_rj moving from lane m to lane m+1), so V_j is ready for
//     Compute(j, m) at the next step.
// Inside the step loop nothing touches global memory except the report of
// a failure.
//
// The apply tiles (head and rest).  A tile is 64 rows (the block) by 64
// columns; 16 lanes per column, lane g applies rotation g of row s - g at
// sub-step s, so the partly rotated L_rj moves to the next lane with a DPP
// row shift while each lane keeps its V_j[g] in a register.
//
// Failures.  After a failure at row r the contents of rows >= r are
// unspecified, so the kernels do not track the failure inside a block: a
// failing Compute records (index, code) and the row with atomic minima, and
// launches for later blocks (and later passes) skip the rows at or after it.
#include "rotations.h"

namespace chm {

namespace {

constexpr int kBR = 64;        // rows (and columns) of a block
constexpr int kKP = 16;        // columns of V per pass
constexpr int kCU = 2;         // rows wave 0 applies to the next column itself
constexpr int kThreads = 1024;

// Rotation record of this schedule: the Apply operands of (row, column m).
struct alignas(32) RotRec {
  double c;   // w / L_ii
  double s;   // V_i / L_ii
  double ic;  // L_ii / w
  double ss;  // sigma * s
};
static_assert(sizeof(RotRec) == sizeof(Coef), "record size");

// Original diagonal of a row, with the values its first Compute starts from.
struct DiagPre {
  double l, t, il, pad;  // L_ii, L_ii * L_ii, 1 / L_ii
};

struct SbLds {
  double Lb[kBR][kBR + 1];  // the block's upper triangle (original, then final)
  double A[kBR][kBR + 1];   // apply tile: rows of block b-1 x 64 columns
  RotRec R[kBR][kKP];       // records of block b-1 (apply), then of block b
  double H[kBR][kKP + 1];   // V of the block's columns: head result, then hand-off
  double X[2][2][kBR];      // helper h -> h+1, by step parity
  DiagPre dg[kBR];
  int64_t lim;              // first failing row known at launch
};

__device__ __forceinline__ double sb_shr1(double x, double fill) {
  const uint64_t b = __builtin_bit_cast(uint64_t, x);
  const uint64_t f = __builtin_bit_cast(uint64_t, fill);
  int lo = __builtin_amdgcn_update_dpp((int)(uint32_t)f, (int)(uint32_t)b, 0x111, 0xF, 0xF, false);
  int hi = __builtin_amdgcn_update_dpp((int)(uint32_t)(f >> 32), (int)(uint32_t)(b >> 32), 0x111,
                                       0xF, 0xF, false);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__device__ __forceinline__ int clamp_row(int r) { return r < 0 ? 0 : (r > kBR - 1 ? kBR - 1 : r); }

// Apply the records of rows [pa, pa + rows) to columns [j0, j0 + ncols).
// HEAD: V of those columns stays in sh.H; otherwise it goes back to W.
template <bool HEAD>
__device__ __forceinline__ void apply_tile(SbLds& sh, double* __restrict__ L, int64_t ldl,
                                           double* __restrict__ W, int64_t ldw, int kc,
                                           int64_t pa, int rows, int64_t j0, int ncols,
                                           const RotRec* __restrict__ T) {
  const int tid = threadIdx.x;
  const int c = tid >> 4, g = tid & 15;
  double a[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int idx = tid + q * kThreads, r = idx >> 6, cc = idx & 63;
    a[q] = (r < rows && cc < ncols) ? L[(pa + r) * ldl + j0 + cc] : 0.0;
  }
  RotRec rec;
  rec.c = 1.0; rec.s = 0.0; rec.ic = 1.0; rec.ss = 0.0;
  if (c < rows && g < kc) rec = T[(pa + c) * kKP + g];
  double w = (c < ncols && g < kc) ? W[(j0 + c) * ldw + g] : 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int idx = tid + q * kThreads;
    sh.A[idx >> 6][idx & 63] = a[q];
  }
  sh.R[c][g] = rec;
  __syncthreads();
  double xs = 0.0;
  const int S = rows + kc - 1;
  for (int s = 0; s < S; ++s) {
    const int r = s - g;
    const bool act = (g < kc) && (r >= 0) && (r < rows);
    const double xin = (g == 0) ? sh.A[clamp_row(s)][c] : xs;
    const RotRec cf = sh.R[clamp_row(r)][g];
    const double x = __builtin_fma(cf.ss, w, xin) * cf.ic;
    const double wn = __builtin_fma(-cf.s, x, cf.c * w);
    w = act ? wn : w;
    if (act && g == kc - 1) sh.A[r][c] = x;
    xs = sb_shr1(x, 0.0);
  }
  __syncthreads();
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int idx = tid + q * kThreads, r = idx >> 6, cc = idx & 63;
    if (r < rows && cc < ncols) L[(pa + r) * ldl + j0 + cc] = sh.A[r][cc];
  }
  if (HEAD) {
    if (g < kc) sh.H[c][g] = w;
  } else {
    if (c < ncols && g < kc) W[(j0 + c) * ldw + g] = w;
  }
}

// ------------------------------------------------------------------ chain
// Per-wave state lives in one register array laid out by the wave's role, so
// that the four roles share registers.
constexpr int kSt = 13;

// Wave 0 layout: st[0] radicand and st[1] 1/L_ii from lane m-1, st[2] L_ii
// of the next row (lane 0), st[3] V_i[m] for this step's Compute,
// st[4 .. 4+kCU) L_{r, i+1} for rows i-kCU+1..i rotated through columns < m,
// st[4+kCU .. 8+kCU) this lane's record of row i-1.
constexpr int kCsLf = 4, kCsPrev = 4 + kCU;
static_assert(kCU == 2, "wave 0 keeps one earlier record");
static_assert(kCsPrev + 4 <= kSt, "state size");

__device__ __forceinline__ void chain_init(SbLds& sh, double (&st)[kSt], int lane, int bbc) {
  const DiagPre d0 = sh.dg[0];
  st[0] = d0.t;
  st[1] = d0.il;
  st[2] = d0.l;
  st[3] = sh.H[0][lane & 15];
#pragma unroll
  for (int q = 0; q < kCU; ++q) {
    const int r = 1 - kCU + q;
    st[kCsLf + q] = (lane == 0 && r >= 0 && bbc > 1) ? sh.Lb[r < 0 ? 0 : r][1] : 0.0;
  }
  st[kCsPrev + 0] = 1.0;  // c
  st[kCsPrev + 1] = 0.0;  // s
  st[kCsPrev + 2] = 1.0;  // ic
  st[kCsPrev + 3] = 0.0;  // ss
  for (int u = kCsPrev + 4; u < kSt; ++u) st[u] = 0.0;
}

__device__ __forceinline__ void chain_step(SbLds& sh, double (&st)[kSt], int t, int m, int kc,
                                           int bbc, double sg, int64_t pc, int64_t kfull,
                                           int64_t m0, int64_t* __restrict__ info,
                                           int64_t* __restrict__ stop_row) {
  const int i = t - m;
  const bool cval = (m < kc) && (i >= 0) && (i < bbc);
  const int jj = i + 1;
  const bool jval = (m < kc) && (jj >= 1) && (jj < bbc);
  // LDS reads: the hand-off of column jj, lane 0's inputs of the next step
  double Wc = sh.H[clamp_row(jj)][m & 15];
  const DiagPre dn = sh.dg[clamp_row(t + 1)];
  double fill[kCU];
#pragma unroll
  for (int q = 0; q < kCU; ++q) {
    const int r = t + 2 - kCU + q, col = t + 2;
    const double f = sh.Lb[clamp_row(r)][clamp_row(col)];
    fill[q] = (r >= 0 && col < bbc) ? f : 0.0;
  }
  // Compute(i, m)
  const double tpi = st[0], ili = st[1];
  const double lin = (m == 0) ? st[2] : tpi * ili;
  const double v = st[3];
  const double tt = __builtin_fma(sg * v, v, tpi);
  const double y = rsqrt_refined(tt);
  const double ww = tt * y;
  const bool bad = (m == 0) && !(lin > 0.0);
  const bool npd = !bad && !(tt > 0.0);
  const bool ok = cval && !bad && !npd;
  RotRec cur;
  const double s = v * ili;
  cur.c = ok ? ww * ili : 1.0;
  cur.s = ok ? s : 0.0;
  cur.ic = ok ? lin * y : 1.0;
  cur.ss = ok ? sg * s : 0.0;
  const double t_out = ok ? tt : tpi, y_out = ok ? y : ili;
  if (cval && !ok) {
    const int64_t code = bad ? kCodeBadDiag : kCodeNotPD;
    atomicMin((unsigned long long*)info,
              (unsigned long long)info_key((pc + i) * kfull + m0 + m, code));
    atomicMin((unsigned long long*)stop_row, (unsigned long long)(pc + i));
  }
  if (cval) sh.R[i][m] = cur;
  if (ok && m == kc - 1) sh.Lb[i][i] = ww;
  // rows i-1 (record of the previous step) and i applied to column jj
  RotRec prev;
  prev.c = st[kCsPrev + 0];
  prev.s = st[kCsPrev + 1];
  prev.ic = st[kCsPrev + 2];
  prev.ss = st[kCsPrev + 3];
  double Lo[kCU];
#pragma unroll
  for (int q = 0; q < kCU; ++q) {
    const int r = i - kCU + 1 + q;
    const RotRec cf = (q == kCU - 1) ? cur : prev;
    const bool rv = jval && (r >= 0);
    const double x = __builtin_fma(cf.ss, Wc, st[kCsLf + q]) * cf.ic;
    const double wn = __builtin_fma(-cf.s, x, cf.c * Wc);
    Wc = rv ? wn : Wc;
    Lo[q] = rv ? x : st[kCsLf + q];
    if (rv && m == kc - 1) sh.Lb[r][jj] = x;
  }
  if (jval) st[3] = Wc;
  st[kCsPrev + 0] = cur.c;
  st[kCsPrev + 1] = cur.s;
  st[kCsPrev + 2] = cur.ic;
  st[kCsPrev + 3] = cur.ss;
  // to lane m+1 (lane 0 takes row t+1's originals)
#pragma unroll
  for (int q = 0; q < kCU; ++q) st[kCsLf + q] = sb_shr1(Lo[q], fill[q]);
  st[0] = sb_shr1(t_out, dn.t);
  st[1] = sb_shr1(y_out, dn.il);
  st[2] = dn.l;
}

// Helper wave layout (columns [MLO, MLO + CNT) of V, lane jj = block column):
// st[u] V_jj[MLO+u] after the rows applied so far, st[CNT+u] L_{r, jj} after
// rotation MLO+u (for the next step), st[2*CNT] the original L_{t, jj}
// (first helper).
template <int MLO, int CNT>
__device__ __forceinline__ void helper_init(SbLds& sh, double (&st)[kSt], int jj) {
  static_assert(2 * CNT + 1 <= kSt, "state size");
#pragma unroll
  for (int u = 0; u < kSt; ++u) st[u] = 0.0;
#pragma unroll
  for (int u = 0; u < CNT; ++u) st[u] = sh.H[jj][MLO + u];
  st[2 * CNT] = sh.Lb[0][jj];
}

template <int H, int MLO, int CNT>
__device__ __forceinline__ void helper_step(SbLds& sh, double (&st)[kSt], int t, int jj, int kc,
                                            int bbc) {
  RotRec cf[CNT];
#pragma unroll
  for (int u = 0; u < CNT; ++u) cf[u] = sh.R[clamp_row(t - 1 - MLO - u)][MLO + u];
  const double xin0 = (H == 0) ? st[2 * CNT] : sh.X[H > 0 ? H - 1 : 0][(t - 1) & 1][jj];
  double Lold[CNT];
#pragma unroll
  for (int u = 0; u < CNT; ++u) Lold[u] = st[CNT + u];
#pragma unroll
  for (int u = 0; u < CNT; ++u) {
    const int m = MLO + u, r = t - 1 - m;
    const bool act = (m < kc) && (r >= 0) && (r < jj - kCU) && (jj < bbc);
    const double lin = (u == 0) ? xin0 : Lold[u > 0 ? u - 1 : 0];
    const double x = __builtin_fma(cf[u].ss, st[u], lin) * cf[u].ic;
    const double wn = __builtin_fma(-cf[u].s, x, cf[u].c * st[u]);
    st[u] = act ? wn : st[u];
    st[CNT + u] = x;
    if (act && m == kc - 1) sh.Lb[r][jj] = x;
    if (act && r == jj - kCU - 1) sh.H[jj][m] = wn;
  }
  if (H < 2) sh.X[H < 2 ? H : 0][t & 1][jj] = st[2 * CNT - 1];
  if (H == 0) st[2 * CNT] = sh.Lb[clamp_row(t)][jj];
}

// Workgroup 0: head tile, then the chain of block [pc, pc + bbc).
__device__ __forceinline__ void chain_wg(SbLds& sh, double* __restrict__ L, int64_t ldl,
                                         double* __restrict__ W, int64_t ldw, int kc,
                                         int64_t kfull, int64_t m0, double sg, int64_t pc,
                                         int bbc, int64_t pa, RotRec* __restrict__ T,
                                         int64_t* __restrict__ info,
                                         int64_t* __restrict__ stop_row, int64_t lim) {
  const int tid = threadIdx.x;
  const bool head = pa >= 0 && pa < lim;
  if (pc >= lim) {
    // a failure in block b-1: finish its rows before the failure, nothing else
    if (head) apply_tile<true>(sh, L, ldl, W, ldw, kc, pa, (int)(lim - pa), pc, bbc, T);
    return;
  }
  double lt[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int idx = tid + q * kThreads, i = idx >> 6, j = idx & 63;
    lt[q] = (i < bbc && j < bbc && j >= i) ? L[(pc + i) * ldl + pc + j] : 0.0;
  }
  if (head) {
    const int rows = lim - pa < kBR ? (int)(lim - pa) : kBR;
    apply_tile<true>(sh, L, ldl, W, ldw, kc, pa, rows, pc, bbc, T);
  } else {
    const int c = tid >> 4, g = tid & 15;
    if (g < kc) sh.H[c][g] = c < bbc ? W[(pc + c) * ldw + g] : 0.0;
  }
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const int idx = tid + q * kThreads;
    sh.Lb[idx >> 6][idx & 63] = lt[q];
  }
  __syncthreads();
  if (tid < kBR) {
    const double l = sh.Lb[tid][tid];
    DiagPre d;
    d.l = l;
    d.t = l * l;
    d.il = 1.0 / l;
    d.pad = 0.0;
    sh.dg[tid] = d;
  }
  __syncthreads();
  if (tid >= 256) return;  // the chain uses waves 0..3; barriers count live waves only
  const int wv = tid >> 6, lane = tid & 63;
  double st[kSt];
  if (wv == 0) chain_init(sh, st, lane, bbc);
  else if (wv == 1) helper_init<0, 6>(sh, st, lane);
  else if (wv == 2) helper_init<6, 5>(sh, st, lane);
  else helper_init<11, 5>(sh, st, lane);
  __syncthreads();
  const int nsteps = bbc + kc - 1;
  for (int t0 = 0; t0 < nsteps; t0 += 2) {
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int t = t0 + u;
      if (t < nsteps) {
        if (wv == 0) chain_step(sh, st, t, lane, kc, bbc, sg, pc, kfull, m0, info, stop_row);
        else if (wv == 1) helper_step<0, 0, 6>(sh, st, t, lane, kc, bbc);
        else if (wv == 2) helper_step<1, 6, 5>(sh, st, t, lane, kc, bbc);
        else helper_step<2, 11, 5>(sh, st, t, lane, kc, bbc);
      }
      __syncthreads();
    }
  }
  // the block's triangle and its records
  for (int idx = tid; idx < kBR * kBR; idx += 256) {
    const int i = idx >> 6, j = idx & 63;
    if (i < bbc && j < bbc && j >= i) L[(pc + i) * ldl + pc + j] = sh.Lb[i][j];
  }
  for (int idx = tid; idx < kBR * kKP; idx += 256) {
    const int r = idx >> 4, m = idx & 15;
    if (r < bbc && m < kc) T[(pc + r) * kKP + m] = sh.R[r][m];
  }
}

__global__ __launch_bounds__(kThreads) void k_sb_block(
    double* __restrict__ L, int64_t ldl, double* __restrict__ W, int64_t ldw, int kc,
    int64_t kfull, int64_t m0, double sg, int64_t n, int64_t pc, int bbc, int64_t pa,
    RotRec* __restrict__ T, int64_t* __restrict__ info, int64_t* __restrict__ stop_row) {
  __shared__ SbLds sh;
  // one read of the failure row per workgroup, so that every wave takes the same path
  if (threadIdx.x == 0)
    sh.lim = __hip_atomic_load(stop_row, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  const int64_t lim = sh.lim;
  if (blockIdx.x == 0) {
    chain_wg(sh, L, ldl, W, ldw, kc, kfull, m0, sg, pc, bbc, pa, T, info, stop_row, lim);
  } else {
    if (pa < 0 || pa >= lim) return;
    const int64_t j0 = pc + bbc + (int64_t)(blockIdx.x - 1) * kBR;
    const int rows = lim - pa < kBR ? (int)(lim - pa) : kBR;
    const int ncols = n - j0 < kBR ? (int)(n - j0) : kBR;
    apply_tile<false>(sh, L, ldl, W, ldw, kc, pa, rows, j0, ncols, T);
  }
}

}  // namespace

// Fast blocked schedule: V columns in passes of 16, one launch per block of
// 64 rows.  W is the private copy of V (row stride k); T holds n x 16 records.
hipError_t run_sysblk(hipStream_t st, double* L, int64_t n, int64_t ldl, double* W, int64_t k,
                      double sg, Coef* T, int64_t* info, int64_t* stop, double* /*sink*/) {
  RotRec* R = reinterpret_cast<RotRec*>(T);
  for (int64_t m0 = 0; m0 < k; m0 += kKP) {
    const int kc = (int)((k - m0) < kKP ? (k - m0) : kKP);
    double* Wc = W + m0;
    for (int64_t pc = 0; pc < n; pc += kBR) {
      const int bbc = (int)((n - pc) < kBR ? (n - pc) : kBR);
      const int64_t pa = pc - kBR;  // previous block (always full), or < 0
      const int64_t rest = n - (pc + bbc);
      const unsigned grid = 1u + (pa >= 0 ? (unsigned)((rest + kBR - 1) / kBR) : 0u);
      hipLaunchKernelGGL(k_sb_block, dim3(grid), dim3(kThreads), 0, st, L, ldl, Wc, k, kc, k, m0,
                         sg, n, pc, bbc, pa, R, info, stop);
    }
  }
  return hipGetLastError();
}

}  // namespace chm
