// sysblk.hip -- blocked schedules of CholeskyModifyB for the fast
// evaluation mode.  Rows are processed in blocks of 64 and the columns of V
// in passes of up to 16.  The work of a block splits into its chain (the
// rows of the block: Compute, and the Apply inside its 64 x 64 triangle)
// and the Apply of its rows to the columns right of it.
//
// Single factor: one persistent launch per pass (the owner schedule,
// k_sb_owner).  Workgroup j, by the order in which workgroups start, owns
// the columns of block j: it applies blocks 0 .. j-1 to them in row order,
// each as the owner of that block publishes its records, then runs the
// chain of block j and publishes that block's records 4 rows at a time
// while the chain runs.  V of the owner's columns never leaves the
// workgroup, and the owner of block j+1 applies block j while its chain is
// still running, so the chains follow each other with only the last rows'
// Apply between them.
//
// Batches: one launch per block step (k_sb_batch).  Workgroup 0 of a
// factor's step applies block b-1 to the columns of block b, then runs the
// chain of block b and writes its records for the next launch; the other
// workgroups apply block b-1 to the columns right of block b.
//
// Every element goes through the same fast-mode operations (rotations.h) in
// the same order as in the per-row schedule, so all schedules give results
// that are identical bit for bit.
//
// The chain.  Algorithm 1 is serial through the rows: Compute(i, m) needs
// V_i after the Apply of rows 0..i-1 and L_ii after Compute(i, m-1).  Wave 0
// is a systolic pipeline over the columns of V: lane m runs Compute(i, m) at
// step t = i + m and passes the running radicand and 1/L_ii to lane m+1 with
// a DPP row shift.  Column j of the block needs the rotations of all earlier
// rows of the block before it becomes the diagonal:
//   * rows r < j - 2 are applied by six helper waves, one lane per column
//     j, in diagonal order: at step t a helper applies (r, m) with
//     r + m = t - 1, whose record wave 0 wrote to LDS at step t - 1; the
//     waves split the columns of V 3 + 3 + 3 + 3 + 2 + 2 and pass the partly
//     rotated L_rj on through LDS.  The workgroup's 8 waves are spread over
//     the 4 SIMDs round-robin, so wave 0 shares its SIMD only with wave 4,
//     which idles, and the helpers pair up on the other three.  After each rotation the helper publishes V_j[m]
//     (by step parity); the value after row j - 3 is the hand-off;
//   * lane m of wave 0 takes that hand-off and applies rows j - 2 and j - 1
//     itself at step j - 1 + m (the partly rotated L_rj moving from lane m
//     to lane m+1), so V_j is ready for Compute(j, m) at the next step.
// The helpers never test whether a rotation is theirs: rows before the
// block have identity records, and what they compute for rows >= j - 2 is
// never read.  Wave 0 tests only while its pipeline fills and drains.  The
// step loop touches no global memory; a failing Compute is remembered per
// lane and reported after the loop.
//
// The apply tiles.  A tile is 64 rows (a block) by 64 columns.  Lane g of a
// 16-lane group applies rotation g of row s - g at sub-step s to several
// columns (two in the batch form, four in the owner's), so each record read
// from LDS serves all of them; the partly rotated L_rj moves to lane g+1
// with a DPP row shift and each lane keeps its V_j[g] in registers.
//
// Failures.  After a failure at row r the contents of rows >= r are
// unspecified, so nothing inside a block depends on a failure: the first
// failure is recorded with atomic minima (index/code, row).  The batch
// form's launches for later blocks and passes skip the rows at or after
// it; the owner schedule simply carries on (every later value is
// unspecified) and the first failure stays the reported one.
#include "rotations.h"
#include "batch.h"

namespace chm {

namespace {

constexpr int kBR = 64;        // rows (and columns) of a block
constexpr int kKP = 16;        // columns of V per pass
constexpr int kThreads = 512;  // 8 waves, two per SIMD
constexpr int kPad = 16;       // identity record rows before the block
constexpr int kRRows = kPad + kBR + kKP;  // record rows -16 .. 79

// Rotation record of this schedule: the Apply operands of (row, column m).
struct alignas(32) RotRec {
  double c;   // w / L_ii
  double s;   // V_i / L_ii
  double ic;  // L_ii / w
  double ss;  // sigma * s
};
static_assert(sizeof(RotRec) == sizeof(Coef), "record size");

// Record as stored in the workspace between launches, in the storage type.
template <typename ST>
struct alignas(4 * sizeof(ST)) GRec {
  ST c, s, ic, ss;
};

// Original diagonal of a row, with the values its first Compute starts from.
struct DiagPre {
  double l, t, il, pad;  // L_ii, L_ii * L_ii, 1 / L_ii
};

// What wave 0 produces at its step of row i: L(i-1, i+1), L(i, i+1), L(i, i).
struct Band {
  double lo, hi, d, pad;
};

// Lane 0's other inputs at step t: the originals L(t-1, t+1) and L(t, t+1)
// for the rows wave 0 applies to column t+1.
struct Fill {
  double lo, hi;
};

struct SbLds {
  // first, so that every record is within the 64 KB reach of an LDS
  // instruction's immediate offset from a lane's base address
  RotRec R[kRRows][kKP];    // records by row + 16: identity / block rows / identity
  union {
    double Lb[kBR][kBR + 1];  // chain: the block's original upper triangle
    double A2[kBR][kBR + 1];  // batch rest workgroups: their second apply tile
    float A2f[kBR][kBR + 1];  // ... held in binary32 for FP32 storage
  };
  union {
    double A[kBR][kBR + 4];      // apply tile: rows of block b-1 x 64 columns
    float Af[kBR][kBR + 4];      // ... held in binary32 for FP32 storage
    double Lh[kPad + kBR][kBR];  // helper results after the last rotation, rows -16..63
  };
  double Hb[kKP][2][kBR];   // V_j[m] after each helper rotation, by step parity
  double X[5][2][kBR];      // helper h -> h+1, by step parity
  Band Lc[kRRows];          // wave 0 results by row + 16
  DiagPre dg[kRRows];       // by row; rows >= bbc unused
  Fill fl[kRRows];           // by step; steps with t + 1 >= bbc unused
  int64_t lim;              // first failing row known at launch
  int fail;                 // first failing (row * 16 + column) of the block
  int tk;                   // owner schedule: this workgroup's ticket
  int tmo;                  // owner schedule: a wait ran out of time
  int up[2];                // owner schedule: rows of the applied block staged, by round parity
};

// Row shift by D lanes within each 16-lane row (DPP row_shr:D); the first D
// lanes of a row take `fill`.
template <int D>
__device__ __forceinline__ double sb_shr(double x, double fill) {
  const uint64_t b = __builtin_bit_cast(uint64_t, x);
  const uint64_t f = __builtin_bit_cast(uint64_t, fill);
  int lo = __builtin_amdgcn_update_dpp((int)(uint32_t)f, (int)(uint32_t)b, 0x110 + D, 0xF, 0xF,
                                       false);
  int hi = __builtin_amdgcn_update_dpp((int)(uint32_t)(f >> 32), (int)(uint32_t)(b >> 32),
                                       0x110 + D, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

template <int D>
__device__ __forceinline__ float sb_shr(float x, float fill) {
  const int b = __builtin_bit_cast(int, x), f = __builtin_bit_cast(int, fill);
  return __builtin_bit_cast(float, __builtin_amdgcn_update_dpp(f, b, 0x110 + D, 0xF, 0xF, false));
}

__device__ __forceinline__ double sb_shr1(double x, double fill) { return sb_shr<1>(x, fill); }
__device__ __forceinline__ float sb_shr1(float x, float fill) { return sb_shr<1>(x, fill); }

__device__ __forceinline__ double fma_t(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_t(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

__device__ __forceinline__ int imin(int a, int b) { return a < b ? a : b; }
__device__ __forceinline__ int imax(int a, int b) { return a > b ? a : b; }

__device__ __forceinline__ RotRec identity_rec() {
  RotRec r;
  r.c = 1.0; r.s = 0.0; r.ic = 1.0; r.ss = 0.0;
  return r;
}

// Global inputs of a workgroup are loaded in two phases: every load is
// issued into registers first, then everything is stored to LDS, so that
// the loads cost one memory round trip instead of one per loop iteration.
constexpr int kRecPerThread = kRRows * kKP / kThreads;  // 3
constexpr int kTilePerThread = kBR * kBR / kThreads;    // 8

// Records of rows [p, p + rows) (columns m < kc) at row offset kPad, identity
// records everywhere else.
template <typename ST>
struct RecRegs {
  GRec<ST> g[kRecPerThread];
};

template <typename ST>
__device__ __forceinline__ void records_issue(RecRegs<ST>& rg, const GRec<ST>* __restrict__ T,
                                              int64_t p, int rows, int kc) {
#pragma unroll
  for (int q = 0; q < kRecPerThread; ++q) {
    const int idx = threadIdx.x + q * kThreads, rr = idx >> 4, m = idx & 15, r = rr - kPad;
    GRec<ST> g;
    g.c = (ST)1; g.s = (ST)0; g.ic = (ST)1; g.ss = (ST)0;
    if (r >= 0 && r < rows && m < kc) g = T[(p + r) * kKP + m];
    rg.g[q] = g;
  }
}

template <typename ST>
__device__ __forceinline__ void records_stage(SbLds& sh, const RecRegs<ST>& rg) {
#pragma unroll
  for (int q = 0; q < kRecPerThread; ++q) {
    const int idx = threadIdx.x + q * kThreads;
    RotRec rec;
    rec.c = rg.g[q].c; rec.s = rg.g[q].s; rec.ic = rg.g[q].ic; rec.ss = rg.g[q].ss;
    sh.R[idx >> 4][idx & 15] = rec;
  }
}

// An apply tile: rows [pa, pa + 64) x columns [j0, j0 + ncols) of L, loaded
// by all threads of the workgroup.
template <typename ST>
struct TileRegs {
  ST a[kTilePerThread];
};

template <typename ST>
__device__ __forceinline__ void tile_issue_a(TileRegs<ST>& tr, const ST* __restrict__ L,
                                             int64_t ldl, int64_t pa, int64_t j0, int ncols) {
  const int tid = threadIdx.x;
#pragma unroll
  for (int q = 0; q < kTilePerThread; ++q) {
    const int idx = tid + q * kThreads, r = idx >> 6, c = idx & 63;
    tr.a[q] = c < ncols ? L[(pa + r) * ldl + j0 + c] : (ST)0;
  }
}

// The apply tiles in the storage type: the Apply to other blocks' columns
// runs in ST, so the tile is kept in ST and no sub-step converts it.
template <typename ST> __device__ __forceinline__ ST* tile_a(SbLds& sh);
template <> __device__ __forceinline__ double* tile_a<double>(SbLds& sh) { return &sh.A[0][0]; }
template <> __device__ __forceinline__ float* tile_a<float>(SbLds& sh) { return &sh.Af[0][0]; }
template <typename ST> __device__ __forceinline__ ST* tile_a2(SbLds& sh);
template <> __device__ __forceinline__ double* tile_a2<double>(SbLds& sh) { return &sh.A2[0][0]; }
template <> __device__ __forceinline__ float* tile_a2<float>(SbLds& sh) { return &sh.A2f[0][0]; }
constexpr int kLdA = kBR + 4, kLdA2 = kBR + 1;  // row strides, in elements

template <typename ST>
__device__ __forceinline__ void tile_stage(SbLds& sh, const TileRegs<ST>& tr) {
  ST* const t = tile_a<ST>(sh);
#pragma unroll
  for (int q = 0; q < kTilePerThread; ++q) {
    const int idx = threadIdx.x + q * kThreads;
    t[(idx >> 6) * kLdA + (idx & 63)] = tr.a[q];
  }
}

// Records passed between the workgroups of one launch (the owner schedule
// below) are written and read with device-scope accesses, so that they are
// seen across the GPU's separate L2 caches.  A record field holding kEmpty (a
// signalling NaN, which no arithmetic result is) has not been written yet:
// the workspace is filled with it before the launch, so the data is its own
// "ready" flag and no fence or flag store is needed.
template <typename ST>
struct RecBits;
template <>
struct RecBits<double> {
  using U = uint64_t;
  static constexpr U kEmpty = 0x7FF4A5A5A5A5A5A5ull;
};
template <>
struct RecBits<float> {
  using U = uint32_t;
  static constexpr U kEmpty = 0x7FA5A5A5u;
};

template <typename ST>
__device__ __forceinline__ typename RecBits<ST>::U load_bits(const ST* p) {
  using U = typename RecBits<ST>::U;
  return __hip_atomic_load(reinterpret_cast<U*>(const_cast<ST*>(p)), __ATOMIC_RELAXED,
                           __HIP_MEMORY_SCOPE_AGENT);
}

template <typename ST>
__device__ __forceinline__ void publish_record(GRec<ST>* dst, const RotRec& r) {
  __hip_atomic_store(&dst->c, (ST)r.c, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&dst->s, (ST)r.s, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __hip_atomic_store(&dst->ic, (ST)r.ic, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// The Apply of a block to a tile of 64 columns runs on 256 threads (four
// waves, one per SIMD).  Lane (q, h, cs) = 16 q + 2 h + cs applies rotations
// 2h and 2h+1 of row s - h at sub-step s to the two columns 4 q + 2 cs and
// 4 q + 2 cs + 1: each pair of records read from LDS serves two columns, the
// partly rotated L_rj moves to lane h+1 of its column pair with a DPP shift
// by two lanes (the lanes of h = 0 take the next row of the tile), V_j[m]
// stays in a register, and the pipeline drains in 7 sub-steps.  The lane
// holding rotation kc - 1 leaves the final value in the tile.
constexpr int kOwnCols = 4;       // V values per apply lane: 2 rotations x 2 columns
constexpr int kOwnThreads = 256;  // apply lanes

// Column u (0, 1) and rotation k (0, 1) of apply lane lt; its V value of
// (rotation 2h + k, column) is w[2 k + u].
__device__ __forceinline__ int own_col(int lt, int u) { return 4 * (lt >> 4) + 2 * (lt & 1) + u; }
__device__ __forceinline__ int own_rot(int lt, int k) { return 2 * ((lt & 15) >> 1) + k; }

// V of apply lane lt's columns [j0, j0 + ncols), columns m < kc of V.
template <typename ST>
__device__ __forceinline__ void w2x2_load(ST (&w)[kOwnCols], const ST* __restrict__ W,
                                          int64_t ldw, int kc, int64_t j0, int ncols, int lt) {
#pragma unroll
  for (int k = 0; k < 2; ++k)
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int c = own_col(lt, u), m = own_rot(lt, k);
      w[2 * k + u] = (c < ncols && m < kc) ? W[(j0 + c) * ldw + m] : (ST)0;
    }
}

// One sub-step s of an apply lane: records qc (row s - h), the row that
// enters the lanes of h = 0 at the next sub-step in fc; loads the next
// records into qn and the row after into fn.  The tile is in LDS at `tile`
// with row stride LD.  Callers alternate two register sets, so that nothing
// is copied between sub-steps.
template <int SG, typename ST, int LD>
__device__ __forceinline__ void sub2x2(const ST* tile_in, ST* tile, const RotRec* rp,
                                       int s, int h, int c0, int hf, bool first,
                                       ST (&w)[kOwnCols], ST (&xin)[2], const RotRec (&qc)[2],
                                       RotRec (&qn)[2], const ST (&fc)[2], ST (&fn)[2]) {
  const int r = s - h;
  // s + 1 <= 71: record rows up to 87
  qn[0] = rp[(s + 1) * kKP];
  qn[1] = rp[(s + 1) * kKP + 1];
  if (h == 0) {
    const int rn2 = imin(s + 2, kBR - 1);
#pragma unroll
    for (int u = 0; u < 2; ++u) fn[u] = (ST)tile_in[rn2 * LD + c0 + u];
  }
  const ST ca = (ST)qc[0].c, sa = (ST)qc[0].s, ia = (ST)qc[0].ic;
  const ST cb = (ST)qc[1].c, sb = (ST)qc[1].s, ib = (ST)qc[1].ic;
  ST x1[2], x2[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    x1[u] = fma_t((ST)SG * sa, w[u], xin[u]) * ia;
    w[u] = fma_t(-sa, x1[u], ca * w[u]);
    x2[u] = fma_t((ST)SG * sb, w[2 + u], x1[u]) * ib;
    w[2 + u] = fma_t(-sb, x2[u], cb * w[2 + u]);
  }
  if (h == hf && r >= 0 && r < kBR) {
#pragma unroll
    for (int u = 0; u < 2; ++u) tile[r * LD + c0 + u] = first ? x1[u] : x2[u];
  }
#pragma unroll
  for (int u = 0; u < 2; ++u) xin[u] = sb_shr<2>(x2[u], fc[u]);
}

// Apply the records staged in sh.R (the block's 64 rows, identity records
// around them) to the 64 x 64 tile at `tile` (row stride LD), as apply lane
// lt of one half of the workgroup.  No barrier inside.  The arithmetic runs
// in the storage type ST (the records hold ST values).
template <int SG, typename ST, int KCF, int LD>
__device__ __forceinline__ void apply2x2(SbLds& sh, ST* tile, int kc_, int lt,
                                         ST (&w)[kOwnCols]) {
  const int kc = KCF ? KCF : kc_;
  const int h = (lt & 15) >> 1, c0 = own_col(lt, 0);
  const int hf = (kc - 1) >> 1;      // lane holding rotation kc - 1
  const bool first = (kc & 1) != 0;  // ... as the first of its pair
  const int S = kBR + hf;            // row 63 reaches lane hf at sub-step 63 + hf
  ST xin[2], fa[2], fb[2] = {(ST)0, (ST)0};
#pragma unroll
  for (int u = 0; u < 2; ++u) {
    xin[u] = (ST)tile[c0 + u];
    fa[u] = (ST)tile[LD + c0 + u];
  }
  const RotRec* rp = &sh.R[kPad - h][2 * h];
  RotRec qa[2] = {rp[0], rp[1]}, qb[2];
  int s = 0;
  for (; s + 2 <= S; s += 2) {
    sub2x2<SG, ST, LD>(tile, tile, rp, s, h, c0, hf, first, w, xin, qa, qb, fa, fb);
    sub2x2<SG, ST, LD>(tile, tile, rp, s + 1, h, c0, hf, first, w, xin, qb, qa, fb, fa);
  }
  if (s < S) sub2x2<SG, ST, LD>(tile, tile, rp, s, h, c0, hf, first, w, xin, qa, qb, fa, fb);
}

// ------------------------------------------------------------------ chain
// A helper wave's state lives in one register array laid out by its column
// range.
constexpr int kSt = 13;

// Wave 0's state, kept in separate scalars (an array would be carried
// through the step loop as one wide register tuple and copied whole at
// every step).
struct ChainState {
  double tp, il, lin;  // from lane m-1 (lane 0: the row's original diagonal):
                       // radicand, 1/L_ii and L_ii
  double v;            // V_i[m] for this step's Compute
  double lo, hi;       // L(i-1, i+1) and L(i, i+1) rotated through columns < m
  double pc, ps, pic;  // this lane's record {c, s, 1/c} of row i-1
};

__device__ __forceinline__ void chain_init(SbLds& sh, ChainState& g, int lane) {
  const DiagPre d0 = sh.dg[0];
  g.tp = d0.t;
  g.il = d0.il;
  g.lin = d0.l;
  g.v = sh.Hb[lane & 15][1][0];
  g.lo = sh.fl[0].lo;
  g.hi = sh.fl[0].hi;
  g.pc = 1.0;
  g.ps = 0.0;
  g.pic = 1.0;
}

// One step of wave 0.  All 64 lanes compute; lanes m >= kc carry garbage
// and send their LDS writes to rows nobody reads (record row kRRows - 1,
// band row 0).  CHECK: the pipeline is filling or draining (some lane has
// i < 0, or i + 1 >= bbc).
template <bool CHECK, int SG>
__device__ __forceinline__ void chain_step(SbLds& sh, ChainState& g, int t, int m, int kc,
                                           int bbc) {
  const int i = t - m;
  const int jj = i + 1;
  const bool act = m < kc;
  double Wc = sh.Hb[m & 15][(t - 1) & 1][jj & 63];
  const DiagPre dn = sh.dg[t + 1];  // t + 1 < 80
  const Fill fn = sh.fl[t + 1];
  // Compute(i, m)
  const double v = g.v;
  const double tt = __builtin_fma(SG * v, v, g.tp);
  const double y = rsqrt_refined(tt);
  const double ww = tt * y;
  const double s = v * g.il;
  const double c = ww * g.il;
  const double ic = g.lin * y;
  RotRec cur;
  cur.c = c; cur.s = s; cur.ic = ic; cur.ss = SG * s;
  const bool rec_ok = act && (!CHECK || (i >= 0 && i < bbc));
  sh.R[rec_ok ? i + kPad : kRRows - 1][m & 15] = cur;
  // rows i-1 (record of the previous step) and i applied to column jj
  const double x0 = __builtin_fma(SG * g.ps, Wc, g.lo) * g.pic;
  Wc = __builtin_fma(-g.ps, x0, g.pc * Wc);
  const double x1 = __builtin_fma(SG * s, Wc, g.hi) * ic;
  Wc = __builtin_fma(-s, x1, c * Wc);
  Band b;
  b.lo = x0; b.hi = x1; b.d = ww; b.pad = 0.0;
  sh.Lc[act ? (CHECK ? imax(imin(i + kPad, kRRows - 1), 0) : i + kPad) : 0] = b;
  if (CHECK) {
    const bool started = i >= 0;
    g.v = started ? Wc : v;
    g.pc = started ? c : 1.0;
    g.ps = started ? s : 0.0;
    g.pic = started ? ic : 1.0;
  } else {
    g.v = Wc;
    g.pc = c;
    g.ps = s;
    g.pic = ic;
  }
  // to lane m+1 (lane 0 takes row t+1's originals)
  g.lo = sb_shr1(x0, fn.lo);
  g.hi = sb_shr1(x1, fn.hi);
  g.tp = sb_shr1(tt, dn.t);
  g.il = sb_shr1(y, dn.il);
  g.lin = sb_shr1(ww, dn.l);  // L_ii after column m = t * y: what tp * il gives lane m+1
}

// Helper wave layout (columns [MLO, MLO + CNT) of V, lane jj = block column):
// st[u] V_jj[MLO+u] after the rows applied so far, st[CNT+u] L_{r, jj} after
// rotation MLO+u (input of the next step), st[2*CNT] the original L_{t, jj}
// (first helper only).
template <int MLO, int CNT>
__device__ __forceinline__ void helper_init(SbLds& sh, double (&st)[kSt], int jj) {
  static_assert(2 * CNT + 1 <= kSt, "state size");
#pragma unroll
  for (int u = 0; u < kSt; ++u) st[u] = 0.0;
#pragma unroll
  for (int u = 0; u < CNT; ++u) st[u] = sh.Hb[MLO + u][1][jj];
  st[2 * CNT] = sh.Lb[0][jj];
}

template <int H, int MLO, int CNT, int SG, int KCF>
__device__ __forceinline__ void helper_step(SbLds& sh, double (&st)[kSt], int t, int jj,
                                            int kc_) {
  const int kc = KCF ? KCF : kc_;
  double c[CNT], sn[CNT], ic[CNT];
#pragma unroll
  for (int u = 0; u < CNT; ++u) {
    // record row t - 1 - m + 16 lies in [0, 94): t < 80, m < 16
    const RotRec& cf = sh.R[t - 1 - MLO - u + kPad][MLO + u];
    c[u] = cf.c;
    sn[u] = cf.s;
    ic[u] = cf.ic;
  }
  const double xin0 = (H == 0) ? st[2 * CNT] : sh.X[H > 0 ? H - 1 : 0][(t - 1) & 1][jj];
  double Lold[CNT];
#pragma unroll
  for (int u = 0; u < CNT; ++u) Lold[u] = st[CNT + u];
#pragma unroll
  for (int u = 0; u < CNT; ++u) {
    const int m = MLO + u;
    if (m < kc) {
      const double lin = (u == 0) ? xin0 : Lold[u > 0 ? u - 1 : 0];
      const double x = __builtin_fma(SG * sn[u], st[u], lin) * ic[u];
      st[u] = __builtin_fma(-sn[u], x, c[u] * st[u]);
      st[CNT + u] = x;
      sh.Hb[m][t & 1][jj] = st[u];
      if (m == kc - 1) sh.Lh[imin(t - 1 - m + kPad, kPad + kBR - 1)][jj] = x;
    }
  }
  if (H < 5) sh.X[H < 5 ? H : 0][t & 1][jj] = st[2 * CNT - 1];
  if (H == 0) st[2 * CNT] = sh.Lb[imin(t, kBR - 1)][jj];
}

// Each role runs its own step loop; every loop passes the same number of
// barriers, one per step (the role is wave-uniform, so no wave enters
// another role's loop).
template <bool CHECK, int SG>
__device__ __forceinline__ void chain_steps(SbLds& sh, ChainState& g, int t0, int t1,
                                            int lane, int kc, int bbc) {
  for (int t = t0; t < t1; ++t) {
    chain_step<CHECK, SG>(sh, g, t, lane, kc, bbc);
    __syncthreads();
  }
}

template <int H, int MLO, int CNT, int SG, int KCF>
__device__ __forceinline__ void helper_steps(SbLds& sh, int nsteps, int lane, int kc) {
  double st[kSt];
  helper_init<MLO, CNT>(sh, st, lane);
  __syncthreads();
  for (int t = 0; t < nsteps; ++t) {
    helper_step<H, MLO, CNT, SG, KCF>(sh, st, t, lane, kc);
    __syncthreads();
  }
}

// LDS set-up of a chain that needs only the block's triangle (staged in
// sh.Lb): the helpers' transfer rows cleared, and each row's diagonal and
// lane 0's inputs.
__device__ __forceinline__ void chain_setup_tri(SbLds& sh, int bbc) {
  const int tid = threadIdx.x;
  for (int idx = tid; idx < 5 * kBR; idx += kThreads) sh.X[idx >> 6][1][idx & 63] = 0.0;
  if (tid == 0) sh.fail = 0x7fffffff;
  if (tid < kRRows) {
    const int r = tid < kBR ? tid : kBR - 1;
    const double l = sh.Lb[r][r];
    DiagPre d;
    d.l = l;
    d.t = l * l;
    d.il = 1.0 / l;
    d.pad = 0.0;
    sh.dg[tid] = d;
    // lane 0 at step t applies rows t-1 and t to column t+1
    Fill f;
    f.lo = (tid >= 1 && tid + 1 < bbc) ? sh.Lb[tid - 1][tid + 1] : 0.0;
    f.hi = (tid + 1 < bbc) ? sh.Lb[tid][tid + 1] : 0.0;
    sh.fl[tid] = f;
  }
}

// Identity records for the block's rows until wave 0 writes them.  (A full
// block could do without: every row a helper reads has been written by wave
// 0 one step earlier.)
__device__ __forceinline__ void chain_setup_records(SbLds& sh) {
  for (int idx = threadIdx.x; idx < kRRows * kKP; idx += kThreads) {
    if ((idx >> 4) >= kPad) sh.R[idx >> 4][idx & 15] = identity_rec();
  }
}

__device__ __forceinline__ void chain_setup(SbLds& sh, int bbc) {
  chain_setup_records(sh);
  chain_setup_tri(sh, bbc);
}

// Wave 4 (owner schedule): the records of rows [r0, r0 + 4) of block
// [pc, pc + 64), complete in sh.R, go to T for the owners of later blocks.
template <typename ST>
__device__ __forceinline__ void publish_rows(SbLds& sh, GRec<ST>* __restrict__ T, int64_t pc,
                                             int r0, int kc, int lane) {
  const int r = r0 + (lane >> 4), m = lane & 15;
  if (m < kc) publish_record(T + (pc + r) * kKP + m, sh.R[r + kPad][m]);
}

// The step loops of the chain of block [pc, pc + bbc); sh is set up and V of
// the block's columns is in sh.Hb parity 1.  pub (full blocks with a later
// block only): wave 4 publishes the records 4 rows at a time as they
// complete.  After barrier u of the loop (u = 0 .. nsteps) the rows up to
// u - kc are complete: row i's last record is written at step i + kc - 1.
template <int SG, typename ST, int KCF>
__device__ __forceinline__ void chain_loops(SbLds& sh, int kc, int bbc, bool pub,
                                            GRec<ST>* __restrict__ T, int64_t pc) {
  const int tid = threadIdx.x;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  // steady steps [s0, s1): every lane m < kc has i >= 0 and i + 1 < bbc
  const int nsteps = bbc + kc - 1;
  const int s0 = kc - 1, s1 = imax(kc - 1, bbc - 1);
  if (wv == 0) {
    ChainState g;
    chain_init(sh, g, lane);
    __syncthreads();
    chain_steps<true, SG>(sh, g, 0, s0, lane, kc, bbc);
    chain_steps<false, SG>(sh, g, s0, s1, lane, kc, bbc);
    chain_steps<true, SG>(sh, g, s1, nsteps, lane, kc, bbc);
  } else if (wv == 4) {
    // shares its SIMD with wave 0: passes the same barriers and publishes
    int q = 0;
    for (int u = 0; u <= nsteps; ++u) {
      __syncthreads();
      if (pub && q < kBR / 4 && u == 4 * q + 3 + kc) {
        publish_rows(sh, T, pc, 4 * q, kc, lane);
        ++q;
      }
    }
  } else if (wv == 1) {
    helper_steps<0, 0, 3, SG, KCF>(sh, nsteps, lane, kc);
  } else if (wv == 2) {
    helper_steps<1, 3, 3, SG, KCF>(sh, nsteps, lane, kc);
  } else if (wv == 3) {
    helper_steps<2, 6, 3, SG, KCF>(sh, nsteps, lane, kc);
  } else if (wv == 5) {
    helper_steps<3, 9, 3, SG, KCF>(sh, nsteps, lane, kc);
  } else if (wv == 6) {
    helper_steps<4, 12, 2, SG, KCF>(sh, nsteps, lane, kc);
  } else {
    helper_steps<5, 14, 2, SG, KCF>(sh, nsteps, lane, kc);
  }
}

// After the loops: the first failure of the block and the block's triangle.
// A Compute fails iff its radicand is not > 0 (then y, w and c are NaN) or,
// for column 0, the original diagonal is not > 0 (then c = w / L_ii is
// negative, infinite or NaN); every later Compute of the same row or of a
// later row may be garbage, none of an earlier row is.  So the failure is
// the first record whose c is not a finite positive number.
template <typename ST>
__device__ __forceinline__ void chain_finish(SbLds& sh, ST* __restrict__ L, int64_t ldl, int kc,
                                             int64_t kfull, int64_t m0, int64_t pc, int bbc,
                                             int64_t* __restrict__ info,
                                             int64_t* __restrict__ stop_row) {
  const int tid = threadIdx.x;
  for (int idx = tid; idx < kBR * kKP; idx += kThreads) {
    const int r = idx >> 4, m = idx & 15;
    if (r < bbc && m < kc) {
      const double c = sh.R[r + kPad][m].c;
      if (!(c > 0.0 && c < __builtin_huge_val())) atomicMin(&sh.fail, idx);
    }
  }
  __syncthreads();
  if (tid == 0 && sh.fail != 0x7fffffff) {
    const int r = sh.fail >> 4, m = sh.fail & 15;
    const int64_t code = (m == 0 && !(sh.dg[r].l > 0.0)) ? kCodeBadDiag : kCodeNotPD;
    atomicMin((unsigned long long*)info,
              (unsigned long long)info_key((pc + r) * kfull + m0 + m, code));
    atomicMin((unsigned long long*)stop_row, (unsigned long long)(pc + r));
  }
  // diagonal and two superdiagonals from wave 0, the rest from the helper
  // holding column kc - 1 of V
  for (int idx = tid; idx < kBR * kBR; idx += kThreads) {
    const int i = idx >> 6, j = idx & 63;
    if (i < bbc && j < bbc && j >= i) {
      double x;
      if (j == i) x = sh.Lc[i + kPad].d;
      else if (j == i + 1) x = sh.Lc[i + kPad].hi;
      else if (j == i + 2) x = sh.Lc[i + 1 + kPad].lo;
      else x = sh.Lh[i + kPad][j];
      L[(pc + i) * ldl + pc + j] = (ST)x;
    }
  }
}

// ------------------------------------------------------- launch per block
// Batched factors run one launch per step: workgroup 0 applies block b-1 to
// the columns of block b (the head tile, on waves 0-3), then runs the chain
// of block b and writes its records for the next launch; each other
// workgroup applies block b-1 to two of the 64-column tiles right of block
// b, one per half of its waves.
template <int SG, typename ST, int KCF>
__device__ __forceinline__ void chain_wg(SbLds& sh, ST* __restrict__ L, ST* __restrict__ La,
                                         int64_t ldl,
                                         ST* __restrict__ W, int64_t ldw, int kc_,
                                         int64_t kfull, int64_t m0, int64_t pc, int bbc,
                                         int64_t pa, GRec<ST>* __restrict__ T,
                                         int64_t* __restrict__ info,
                                         int64_t* __restrict__ stop_row, int64_t lim) {
  const int kc = KCF ? KCF : kc_;
  const int tid = threadIdx.x;
  const bool head = pa >= 0 && pa < lim;
  const int hrows = head ? (lim - pa < kBR ? (int)(lim - pa) : kBR) : 0;
  const bool chain = pc < lim;  // else a failure in block b-1: finish its rows only
  // issue every global load, then stage them in LDS
  RecRegs<ST> rg;
  records_issue(rg, T, pa, hrows, kc);  // all identity without a head tile
  TileRegs<ST> tr;
  ST wa[kOwnCols];
  if (head) {
    tile_issue_a(tr, La, ldl, pa, pc, bbc);
    if (tid < kOwnThreads) w2x2_load(wa, W, ldw, kc, pc, bbc, tid);
  }
  constexpr int kHbPerThread = kBR * kKP / kThreads;  // 2
  ST lt[kTilePerThread], wh[kHbPerThread];
  if (chain) {
#pragma unroll
    for (int q = 0; q < kTilePerThread; ++q) {
      const int idx = tid + q * kThreads, i = idx >> 6, j = idx & 63;
      lt[q] = (i < bbc && j < bbc && j >= i) ? L[(pc + i) * ldl + pc + j] : (ST)0;
    }
    if (!head) {
#pragma unroll
      for (int q = 0; q < kHbPerThread; ++q) {
        const int idx = tid + q * kThreads, c = idx >> 4, g = idx & 15;
        wh[q] = (g < kc && c < bbc) ? W[(pc + c) * ldw + g] : (ST)0;
      }
    }
  }
  records_stage(sh, rg);
  if (head) tile_stage(sh, tr);
  if (chain) {
#pragma unroll
    for (int q = 0; q < kTilePerThread; ++q) {
      const int idx = tid + q * kThreads;
      sh.Lb[idx >> 6][idx & 63] = (double)lt[q];
    }
    if (!head) {
#pragma unroll
      for (int q = 0; q < kHbPerThread; ++q) {
        const int idx = tid + q * kThreads;
        sh.Hb[idx & 15][1][idx >> 4] = (double)wh[q];
      }
    }
  }
  __syncthreads();
  if (head) {
    if (tid < kOwnThreads) apply2x2<SG, ST, KCF, kLdA>(sh, tile_a<ST>(sh), kc, tid, wa);
    __syncthreads();
    // the head tile's final values, and V of block b's columns for the chain
#pragma unroll
    for (int q = 0; q < kTilePerThread; ++q) {
      const int idx = tid + q * kThreads, r = idx >> 6, c = idx & 63;
      if (c < bbc) La[(pa + r) * ldl + pc + c] = tile_a<ST>(sh)[r * kLdA + c];
    }
    if (tid < kOwnThreads) {
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int m = own_rot(tid, k);
          if (m < kc) sh.Hb[m][1][own_col(tid, u)] = (double)wa[2 * k + u];
        }
    }
  }
  if (!chain) return;
  __syncthreads();
  chain_setup(sh, bbc);
  __syncthreads();
  chain_loops<SG, ST, KCF>(sh, kc, bbc, false, T, pc);
  chain_finish(sh, L, ldl, kc, kfull, m0, pc, bbc, info, stop_row);
  for (int idx = tid; idx < kBR * kKP; idx += kThreads) {
    const int r = idx >> 4, m = idx & 15;
    if (r < bbc && m < kc) {
      const RotRec& rec = sh.R[r + kPad][m];
      GRec<ST> g;
      g.c = (ST)rec.c; g.s = (ST)rec.s; g.ic = (ST)rec.ic; g.ss = (ST)rec.ss;
      T[(pc + r) * kKP + m] = g;
    }
  }
}

// One workgroup's share of the launch for block [pc, pc + bbc) of one factor:
// wg == 0 runs the chain, wg >= 1 applies block [pa, pa + 64) to tiles
// 2 (wg - 1) and 2 (wg - 1) + 1 right of block b (waves 0-3 the first, in
// sh.A, waves 4-7 the second, in sh.A2).
template <int SG, typename ST, int KCF>
__device__ __forceinline__ void block_work(SbLds& sh, ST* __restrict__ L, ST* __restrict__ La,
                                           int64_t ldl,
                                           ST* __restrict__ W, int64_t ldw, int kc,
                                           int64_t kfull, int64_t m0, int64_t n, int64_t pc,
                                           int bbc, int64_t pa, GRec<ST>* __restrict__ T,
                                           int64_t* __restrict__ info,
                                           int64_t* __restrict__ stop_row, int wg) {
  // one read of the failure row per workgroup, so that every wave takes the same path
  if (threadIdx.x == 0)
    sh.lim = __hip_atomic_load(stop_row, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  const int64_t lim = sh.lim;
  if (wg == 0) {
    chain_wg<SG, ST, KCF>(sh, L, La, ldl, W, ldw, kc, kfull, m0, pc, bbc, pa, T, info, stop_row,
                          lim);
  } else {
    if (pa < 0 || pa >= lim) return;
    const int tid = threadIdx.x, half = tid >> 8, lt = tid & (kOwnThreads - 1);
    const int64_t j0 = pc + bbc + (int64_t)(2 * (wg - 1) + half) * kBR;
    const int ncols = j0 < n ? (n - j0 < kBR ? (int)(n - j0) : kBR) : 0;
    RecRegs<ST> rg;
    records_issue(rg, T, pa, lim - pa < kBR ? (int)(lim - pa) : kBR, kc);
    constexpr int kHalfTile = kBR * kBR / kOwnThreads;  // 16 elements per thread
    ST ta[kHalfTile];
#pragma unroll
    for (int q = 0; q < kHalfTile; ++q) {
      const int idx = lt + q * kOwnThreads, r = idx >> 6, c = idx & 63;
      ta[q] = c < ncols ? La[(pa + r) * ldl + j0 + c] : (ST)0;
    }
    ST wa[kOwnCols];
    w2x2_load(wa, W, ldw, kc, j0, ncols, lt);
    records_stage(sh, rg);
    ST* const tile = half ? tile_a2<ST>(sh) : tile_a<ST>(sh);
    const int ld = half ? kLdA2 : kLdA;
#pragma unroll
    for (int q = 0; q < kHalfTile; ++q) {
      const int idx = lt + q * kOwnThreads;
      tile[(idx >> 6) * ld + (idx & 63)] = ta[q];
    }
    __syncthreads();
    if (ncols > 0) {
      if (half) apply2x2<SG, ST, KCF, kLdA2>(sh, tile_a2<ST>(sh), kc, lt, wa);
      else apply2x2<SG, ST, KCF, kLdA>(sh, tile_a<ST>(sh), kc, lt, wa);
    }
    __syncthreads();
    if (ncols > 0) {
#pragma unroll
      for (int q = 0; q < kHalfTile; ++q) {
        const int idx = lt + q * kOwnThreads, r = idx >> 6, c = idx & 63;
        if (c < ncols) La[(pa + r) * ldl + j0 + c] = tile[r * ld + c];
      }
#pragma unroll
      for (int k = 0; k < 2; ++k)
#pragma unroll
        for (int u = 0; u < 2; ++u) {
          const int c = own_col(lt, u), m = own_rot(lt, k);
          if (c < ncols && m < kc) W[(j0 + c) * ldw + m] = wa[2 * k + u];
        }
    }
  }
}

// ---------------------------------------------------------- owner schedule
// One launch per pass of 16 columns of V.  The workgroup with ticket j (the
// j-th to start) owns the columns of block j: it applies blocks 0 .. j-1 to
// them in row order, each as its owner publishes it, keeping V of its
// columns in registers, then runs the chain of block j itself and publishes
// the block's records 4 rows at a time while the chain runs.  A workgroup
// waits only for workgroups that started before it, so every wait ends; each
// wait is still bounded: all of a workgroup's waits end kWaitTicks after it
// started (then the launch reports kCodeTimeout and its results are void).
constexpr int64_t kWaitTicks = 500000000;  // steady-counter ticks (5 s at 100 MHz)

// The owner's apply runs on waves 0-3 (one per SIMD) with the two-rotation,
// two-column lanes of sub2x2.  Wave 4 fetches the records: it waits until a prefix of the next 16 rows
// has been published, stages those rows in sh.R and announces how far the
// staged rows go (sh.up, by round parity); the apply waves then run the
// sub-steps whose rows are all staged, while wave 4 fetches the next rows.
// Waves 5-7 only pass the rounds' barriers.

// Apply block [pb, pb + 64) (tile staged in sh.A, the caller has
// synchronised) to the owner's columns; w: an apply lane's V values.  next:
// block pb is the one just before the owner's own (its chain waits for this
// apply), so wave 4 polls without delay; the owners further right poll
// slowly, which keeps their reads of the same few records from crowding the
// memory channels.  Same operations, in the same order, as apply2x2.
template <int SG, typename ST, int KCF>
__device__ __forceinline__ void owner_apply(SbLds& sh, int kc_, int64_t pb,
                                            ST (&w)[kOwnCols],
                                            const GRec<ST>* __restrict__ T, int64_t deadline,
                                            bool next) {
  using U = typename RecBits<ST>::U;
  constexpr U kE = RecBits<ST>::kEmpty;
  const int kc = KCF ? KCF : kc_;
  const int tid = threadIdx.x;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  if (wv < 4) {
    const int h = (lane & 15) >> 1;
    const int c0 = own_col(tid, 0);
    const int hf = (kc - 1) >> 1;          // lane holding rotation kc - 1
    const bool first = (kc & 1) != 0;      // ... as the first of its pair
    const int S = kBR + hf;                // row 63 reaches lane hf at sub-step 63 + hf
    ST* const tile = tile_a<ST>(sh);
    constexpr int LD = kLdA;
    ST xin[2], fa[2], fb[2] = {(ST)0, (ST)0};  // fa, fb: only lanes h = 0 use them
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      xin[u] = (ST)tile[c0 + u];
      fa[u] = (ST)tile[LD + c0 + u];
    }
    // records of (row s - h, rotations 2h and 2h+1) at rp[s * kKP], rp[s * kKP + 1]
    const RotRec* rp = &sh.R[kPad - h][2 * h];
    int s = 0;
    for (int rd = 0;; ++rd) {
      __syncthreads();
      const int up = sh.up[rd & 1];
      const int lim = up >= kBR ? S : up;  // rows <= s - h < up are staged
      RotRec qa[2] = {rp[s * kKP], rp[s * kKP + 1]}, qb[2];
      for (; s + 2 <= lim; s += 2) {
        sub2x2<SG, ST, LD>(tile, tile, rp, s, h, c0, hf, first, w, xin, qa, qb, fa, fb);
        sub2x2<SG, ST, LD>(tile, tile, rp, s + 1, h, c0, hf, first, w, xin, qb, qa, fb, fa);
      }
      if (s < lim) {
        sub2x2<SG, ST, LD>(tile, tile, rp, s, h, c0, hf, first, w, xin, qa, qb, fa, fb);
        ++s;
        fa[0] = fb[0];
        fa[1] = fb[1];
      }
      if (up >= kBR) break;
    }
  } else if (wv == 4) {
    // lane holds rows up + 4 v + lane / 16 (v = 0..3) of the window, column m
    const int m = lane & 15, rl = lane >> 4;
    U f[4][3];
    auto fetch = [&](int up) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = up + 4 * v + rl;
        if (r < kBR && m < kc) {
          const GRec<ST>* src = T + (pb + r) * kKP + m;
          f[v][0] = load_bits(&src->c);
          f[v][1] = load_bits(&src->s);
          f[v][2] = load_bits(&src->ic);
        } else {
          f[v][0] = f[v][1] = f[v][2] = 0;  // nothing to wait for
        }
      }
    };
    // rows of the window (bit 4 v + group) whose records are all there
    auto ready_rows = [&]() {
      uint32_t full = 0;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const bool ok = f[v][0] != kE && f[v][1] != kE && f[v][2] != kE;
        const uint64_t b = __ballot(ok);
#pragma unroll
        for (int gq = 0; gq < 4; ++gq)
          if (((b >> (16 * gq)) & 0xFFFFull) == 0xFFFFull) full |= 1u << (4 * v + gq);
      }
      return full;
    };
    int up = 0;
    fetch(0);
    for (int rd = 0;; ++rd) {
      int nr = __builtin_ctz(~ready_rows());
      while (nr == 0) {
        if (wall_clock64() > deadline) {  // give up: stage what is there
          sh.tmo = 1;
          nr = 16;
          break;
        }
        if (next) __builtin_amdgcn_s_sleep(1);
        else __builtin_amdgcn_s_sleep(100);
        fetch(up);
        nr = __builtin_ctz(~ready_rows());
      }
      if (nr > kBR - up) nr = kBR - up;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = up + 4 * v + rl;
        if (4 * v + rl < nr && m < kc) {
          RotRec rec;
          rec.c = (double)__builtin_bit_cast(ST, f[v][0]);
          rec.s = (double)__builtin_bit_cast(ST, f[v][1]);
          rec.ic = (double)__builtin_bit_cast(ST, f[v][2]);
          rec.ss = 0.0;
          sh.R[kPad + r][m] = rec;
        }
      }
      up += nr;
      if (lane == 0) sh.up[rd & 1] = up;
      if (up < kBR) fetch(up);  // in flight while the apply waves run
      __syncthreads();
      if (up >= kBR) break;
    }
  } else {
    for (int rd = 0;; ++rd) {
      __syncthreads();
      if (sh.up[rd & 1] >= kBR) break;
    }
  }
}

template <int SG, typename ST, int KCF>
__global__ __launch_bounds__(kThreads) void k_sb_owner(
    ST* __restrict__ L, int64_t ldl, const ST* __restrict__ W, int64_t ldw, int kc_,
    int64_t kfull, int64_t m0, int64_t n, GRec<ST>* __restrict__ T,
    int64_t* __restrict__ info, int64_t* __restrict__ stop_row, int32_t* __restrict__ ticket) {
  __shared__ SbLds sh;
  const int kc = KCF ? KCF : kc_;
  const int tid = threadIdx.x;
  const int64_t deadline = wall_clock64() + kWaitTicks;
  if (tid == 0) {
    sh.tk = __hip_atomic_fetch_add(ticket, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    sh.tmo = 0;
  }
  __syncthreads();
  const int j = sh.tk;
  const int64_t pj = (int64_t)j * kBR;
  const int bbc = n - pj < kBR ? (int)(n - pj) : kBR;
  // every global input of the workgroup is issued before anything is staged:
  // the block's triangle, V of its columns and the first tile
  ST lt[kTilePerThread];
#pragma unroll
  for (int q = 0; q < kTilePerThread; ++q) {
    const int idx = tid + q * kThreads, i = idx >> 6, c = idx & 63;
    lt[q] = (i < bbc && c < bbc && c >= i) ? L[(pj + i) * ldl + pj + c] : (ST)0;
  }
  ST w[kOwnCols];
#pragma unroll
  for (int k = 0; k < 2; ++k)
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int c = own_col(tid, u), m = own_rot(tid, k);
      w[2 * k + u] = (tid < kOwnThreads && c < bbc && m < kc) ? W[(pj + c) * ldw + m] : (ST)0;
    }
  TileRegs<ST> tr;
  if (j > 0) tile_issue_a(tr, L, ldl, 0, pj, bbc);
#pragma unroll
  for (int q = 0; q < kTilePerThread; ++q) {
    const int idx = tid + q * kThreads;
    sh.Lb[idx >> 6][idx & 63] = (double)lt[q];
  }
  // identity records everywhere: the pad rows keep them, each block's rows
  // are overwritten as they arrive
  for (int idx = tid; idx < kRRows * kKP; idx += kThreads) sh.R[idx >> 4][idx & 15] = identity_rec();
  __syncthreads();
  chain_setup_tri(sh, bbc);  // needs only the triangle: done before the applies
  for (int b = 0; b < j; ++b) {
    __syncthreads();  // sh.A is free again
    tile_stage(sh, tr);
    if (b + 1 < j) tile_issue_a(tr, L, ldl, (int64_t)(b + 1) * kBR, pj, bbc);
    const int64_t pb = (int64_t)b * kBR;
    __syncthreads();
    owner_apply<SG, ST, KCF>(sh, kc, pb, w, T, deadline, b == j - 1);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kTilePerThread; ++q) {
      const int idx = tid + q * kThreads, r = idx >> 6, c = idx & 63;
      if (c < bbc) L[(pb + r) * ldl + pj + c] = tile_a<ST>(sh)[r * kLdA + c];
    }
  }
  // V of the block's columns, after all earlier rows, starts the chain
  if (tid < kOwnThreads) {
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int c = own_col(tid, u), m = own_rot(tid, k);
        if (m < kc) sh.Hb[m][1][c] = c < bbc ? (double)w[2 * k + u] : 0.0;
      }
  }
  if (bbc < kBR) chain_setup_records(sh);
  __syncthreads();
  chain_loops<SG, ST, KCF>(sh, kc, bbc, pj + kBR < n, T, pj);
  chain_finish(sh, L, ldl, kc, kfull, m0, pj, bbc, info, stop_row);
  if (tid == 0 && sh.tmo)
    atomicMin((unsigned long long*)info,
              (unsigned long long)info_key(pj * kfull + m0, kCodeTimeout));
}

// Records of one pass start out empty.
template <typename ST>
__global__ void k_owner_clear(GRec<ST>* __restrict__ T, int64_t words) {
  using U = typename RecBits<ST>::U;
  U* __restrict__ p = reinterpret_cast<U*>(T);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride)
    p[i] = RecBits<ST>::kEmpty;
}

// Batched form: the launch of step s holds, for every factor with more than
// s steps, the chain workgroup of its step s (workgroups [0, nent), longest
// factor first) and then all their rest workgroups.
__global__ __launch_bounds__(kThreads) void k_sb_batch(const BatchFactor* __restrict__ fac,
                                                       const BatchEntry* __restrict__ ent,
                                                       int nent) {
  __shared__ SbLds sh;
  const int x = (int)blockIdx.x;
  int e = x, wg = 0;
  if (x >= nent) {
    const int r = x - nent;  // rest workgroup r of the step: largest e with ent[e].rest0 <= r
    int lo = 0, hi = nent - 1;
    while (lo < hi) {
      const int mid = (lo + hi + 1) >> 1;
      if (ent[mid].rest0 <= r) lo = mid;
      else hi = mid - 1;
    }
    e = lo;
    wg = 1 + r - ent[lo].rest0;
  }
  const BatchEntry E = ent[e];
  const BatchFactor F = fac[E.f];
  if (F.dtype == kStoreF64) {
    double* L = (double*)E.Lc;
    double* La = (double*)E.La;
    double* W = (double*)F.W + E.m0;
    GRec<double>* T = (GRec<double>*)F.T;
    if (F.sigma > 0)
      block_work<1, double, 0>(sh, L, La, F.ldl, W, F.k, E.kc, F.k, E.m0, F.n, E.pc, E.bbc,
                               E.pa, T,
                               F.info, F.stop, wg);
    else
      block_work<-1, double, 0>(sh, L, La, F.ldl, W, F.k, E.kc, F.k, E.m0, F.n, E.pc, E.bbc,
                                E.pa, T,
                                F.info, F.stop, wg);
  } else {
    float* L = (float*)E.Lc;
    float* La = (float*)E.La;
    float* W = (float*)F.W + E.m0;
    GRec<float>* T = (GRec<float>*)F.T;
    if (F.sigma > 0)
      block_work<1, float, 0>(sh, L, La, F.ldl, W, F.k, E.kc, F.k, E.m0, F.n, E.pc, E.bbc,
                              E.pa, T,
                              F.info, F.stop, wg);
    else
      block_work<-1, float, 0>(sh, L, La, F.ldl, W, F.k, E.kc, F.k, E.m0, F.n, E.pc, E.bbc,
                               E.pa, T,
                               F.info, F.stop, wg);
  }
}

// Batched preparation: W <- V for every factor, info and stop row reset.
// Grid (chunks, factors).
__global__ void k_prepare_batch(const BatchFactor* __restrict__ fac) {
  const BatchFactor F = fac[blockIdx.y];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *F.info = INT64_MAX;
    *F.stop = INT64_MAX;
  }
  const int64_t words = F.n * F.k * (F.dtype == kStoreF64 ? 2 : 1);  // 4-byte words
  const uint32_t* __restrict__ src = (const uint32_t*)F.V;
  uint32_t* __restrict__ dst = (uint32_t*)F.W;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words; i += stride)
    dst[i] = src[i];
}

// One owner launch per pass; tickets[p] (zero before the first pass) counts
// the workgroups of pass p as they start.
template <typename ST>
hipError_t run_sysblk_t(hipStream_t st, ST* L, int64_t n, int64_t ldl, ST* W, int64_t k, int sg,
                        void* Tws, int64_t* info, int64_t* stop, int32_t* tickets) {
  GRec<ST>* R = reinterpret_cast<GRec<ST>*>(Tws);
  const int64_t nb = (n + kBR - 1) / kBR;
  const int64_t words = n * kKP * 4;
  const int64_t cblocks = (words + 255) / 256;
  const unsigned cgrid = (unsigned)(cblocks < 1024 ? cblocks : 1024);
  for (int64_t m0 = 0; m0 < k; m0 += kKP) {
    const int kc = (int)((k - m0) < kKP ? (k - m0) : kKP);
    hipLaunchKernelGGL(k_owner_clear<ST>, dim3(cgrid), dim3(256), 0, st, R, words);
    // full passes (16 columns of V) use a variant specialised on that width
    auto kern = sg > 0 ? (kc == kKP ? k_sb_owner<1, ST, kKP> : k_sb_owner<1, ST, 0>)
                       : (kc == kKP ? k_sb_owner<-1, ST, kKP> : k_sb_owner<-1, ST, 0>);
    hipLaunchKernelGGL(kern, dim3((unsigned)nb), dim3(kThreads), 0, st, L, ldl,
                       (const ST*)(W + m0), k, kc, k, m0, n, R, info, stop, tickets + m0 / kKP);
  }
  return hipGetLastError();
}

}  // namespace

// Batched launches: one preparation launch, then one launch per step.
hipError_t run_sysblk_batch_prepare(hipStream_t st, const BatchFactor* d_fac, int64_t count) {
  if (count > 0) {
    const unsigned fy = (unsigned)count;
    hipLaunchKernelGGL(k_prepare_batch, dim3(8, fy), dim3(256), 0, st, d_fac);
  }
  return hipGetLastError();
}

hipError_t run_sysblk_batch_step(hipStream_t st, const BatchFactor* d_fac,
                                 const BatchEntry* d_ent, const BatchStep& S) {
  if (S.nent > 0)
    hipLaunchKernelGGL(k_sb_batch, dim3((unsigned)(S.nent + S.nrest)), dim3(kThreads), 0, st,
                       d_fac, d_ent + S.off, (int)S.nent);
  return hipGetLastError();
}

hipError_t run_sysblk_batch(hipStream_t st, const BatchFactor* d_fac, int64_t count,
                            const BatchEntry* d_ent, const BatchStep* steps, int64_t nsteps) {
  hipError_t e = run_sysblk_batch_prepare(st, d_fac, count);
  for (int64_t s = 0; s < nsteps && e == hipSuccess; ++s)
    e = run_sysblk_batch_step(st, d_fac, d_ent, steps[s]);
  return e;
}

// Fast blocked schedule: V columns in passes of 16, one owner launch per
// pass.  W is the private copy of V (row stride k); T holds n x 16 records;
// tickets holds one zeroed int32 per pass.
hipError_t run_sysblk(hipStream_t st, double* L, int64_t n, int64_t ldl, double* W, int64_t k,
                      double sg, Coef* T, int64_t* info, int64_t* stop, int32_t* tickets) {
  return run_sysblk_t<double>(st, L, n, ldl, W, k, sg > 0 ? 1 : -1, T, info, stop, tickets);
}

// The same schedule with L, V and the records stored in FP32: the rows of a
// block (Compute and the Apply inside the block) run in FP64 from the FP32
// values, the Apply to other blocks' columns runs in FP32.
hipError_t run_sysblk_f32(hipStream_t st, float* L, int64_t n, int64_t ldl, float* W, int64_t k,
                          double sg, void* T, int64_t* info, int64_t* stop, int32_t* tickets) {
  return run_sysblk_t<float>(st, L, n, ldl, W, k, sg > 0 ? 1 : -1, T, info, stop, tickets);
}

}  // namespace chm
