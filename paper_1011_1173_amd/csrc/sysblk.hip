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
//   * rows r < j - 2 are applied by seven helper waves, one lane per column
//     j, in diagonal order: at step t a helper applies (r, m) with
//     r + m = t - 1, whose record wave 0 wrote to LDS at step t - 1; the
//     waves split the columns of V 3 + 3 + 3 + 2 + 2 + 2 + 1 and pass the
//     partly rotated L_rj on through LDS.  The workgroup's 8 waves are spread
//     over the 4 SIMDs round-robin (waves w and w + 4 on SIMD w), so each of
//     SIMDs 1-3 runs five columns and wave 0 shares SIMD 0 with the helper of
//     one column.  After each rotation the helper publishes V_j[m] (by step
//     parity); the value after row j - 3 is the hand-off;
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

// What lane 0 of the chain starts row r from: the row's original diagonal
// (the values its first Compute uses) and the originals L(r-1, r+1), L(r, r+1)
// of the two rows it applies to column r+1.  48 bytes, so that one step reads
// it with three LDS loads.
struct Feed {
  double t, il;  // L_rr * L_rr, 1 / L_rr
  double l, lo;  // L_rr, L(r-1, r+1)
  double hi;     // L(r, r+1)
  double pad;
};

// What wave 0 produces at its step of row i: L(i-1, i+1), L(i, i+1), L(i, i).
struct Band {
  double lo, hi, d, pad;
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
  double X[6][2][kBR];      // helper h -> h+1, by step parity
  Band Lc[kRRows];          // wave 0 results by row + 16
  Feed fd[kRRows];          // by row; rows >= bbc unused
  int64_t lim;              // first failing row known at launch
  int fail;                 // first failing (row * 16 + column) of the block
  int tk;                   // owner schedule: this workgroup's ticket
  int tmo;                  // owner schedule: a wait ran out of time
  int cnt[2][4];            // owner schedule: rows of each 16-row window of the applied
                            // block staged, by round parity
  int mst[2][4];            // owner schedule: what each staging wave found of the map in
                            // buffer 0 / 1 (kMapOk, kMapRot, kMapWait)
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

// One sub-step s of an apply lane: records qc (row s - h); loads the next
// records into qn.  The tile is in LDS at `tile` with row stride LD.  fc is
// the fill value of this sub-step's shift: row s + 1 of the tile, which the
// lanes of h = 0 take at the next sub-step; the sub-step reads row s + 2 into
// fn for the next one, so that each fill read has a whole sub-step to land
// (every lane reads it: one LDS broadcast per column pair costs less than
// masking the others off).  WRITE: the sub-step may finish a row (s >= hf;
// before, the lanes of h = hf still hold rows < 0), which lane h = hf stores;
// the rows read ahead are never the ones written.  DRAIN (s >= 63): the lanes
// of h = 0 enter rows past the tile, whose records are identity; they take 0,
// which such a rotation passes through exactly (a value read past the tile
// could be a NaN, and 0 * NaN would spoil V).  Callers alternate two record
// and fill sets, so that nothing is copied between sub-steps.
template <int SG, typename ST, int LD, bool WRITE, bool DRAIN>
__device__ __forceinline__ void sub2x2(ST* tile, const RotRec* rp, int s, int h, int c0,
                                       int hf, bool first, ST (&w)[kOwnCols], ST (&xin)[2],
                                       const RotRec (&qc)[2], RotRec (&qn)[2],
                                       const ST (&fc)[2], ST (&fn)[2]) {
  if (DRAIN) {
    fn[0] = fn[1] = (ST)0;
  } else {
    // row s + 2 (row 63 when that is past the tile: the next sub-step is
    // then a drain sub-step, which takes 0 instead)
    const int rn = imin(s + 2, kBR - 1);
#pragma unroll
    for (int u = 0; u < 2; ++u) fn[u] = tile[rn * LD + c0 + u];
  }
  // s + 1 <= 71: record rows up to 87
  qn[0] = rp[(s + 1) * kKP];
  qn[1] = rp[(s + 1) * kKP + 1];
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
  if (WRITE && h == hf) {
    const int r = s - hf;  // in [0, 64): s < 64 + hf
#pragma unroll
    for (int u = 0; u < 2; ++u) tile[r * LD + c0 + u] = first ? x1[u] : x2[u];
  }
#pragma unroll
  for (int u = 0; u < 2; ++u) xin[u] = sb_shr<2>(x2[u], DRAIN ? (ST)0 : fc[u]);
}

// Sub-steps [s, lim) of an apply lane (s is advanced); qa holds the records
// of sub-step s and, on return, those of sub-step lim.
template <int SG, typename ST, int LD>
__device__ __forceinline__ void sub2x2_run(ST* tile, const RotRec* rp, int& s, int lim, int h,
                                           int c0, int hf, bool first, ST (&w)[kOwnCols],
                                           ST (&xin)[2], RotRec (&qa)[2]) {
  RotRec qb[2];
  // the fill of sub-step s: row s + 1 of the tile (unused by drain sub-steps)
  ST fa[2], fb[2];
  {
    const int r1 = imin(s + 1, kBR - 1);
#pragma unroll
    for (int u = 0; u < 2; ++u) fa[u] = tile[r1 * LD + c0 + u];
  }
  for (; s < lim && s < hf; ++s) {  // no row is finished yet
    sub2x2<SG, ST, LD, false, false>(tile, rp, s, h, c0, hf, first, w, xin, qa, qb, fa, fb);
    qa[0] = qb[0];
    qa[1] = qb[1];
    fa[0] = fb[0];
    fa[1] = fb[1];
  }
  const int lmain = imin(lim, kBR - 1);  // sub-steps whose next row is in the tile
  for (; s + 2 <= lmain; s += 2) {
    sub2x2<SG, ST, LD, true, false>(tile, rp, s, h, c0, hf, first, w, xin, qa, qb, fa, fb);
    sub2x2<SG, ST, LD, true, false>(tile, rp, s + 1, h, c0, hf, first, w, xin, qb, qa, fb, fa);
  }
  if (s < lmain) {
    sub2x2<SG, ST, LD, true, false>(tile, rp, s, h, c0, hf, first, w, xin, qa, qb, fa, fb);
    ++s;
    qa[0] = qb[0];
    qa[1] = qb[1];
    fa[0] = fb[0];
    fa[1] = fb[1];
  }
  for (; s < lim; ++s) {  // the drain: at most hf + 1 sub-steps
    sub2x2<SG, ST, LD, true, true>(tile, rp, s, h, c0, hf, first, w, xin, qa, qb, fa, fb);
    qa[0] = qb[0];
    qa[1] = qb[1];
  }
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
  ST xin[2];
#pragma unroll
  for (int u = 0; u < 2; ++u) xin[u] = (ST)tile[c0 + u];
  const RotRec* rp = &sh.R[kPad - h][2 * h];
  RotRec qa[2] = {rp[0], rp[1]};
  int s = 0;
  sub2x2_run<SG, ST, LD>(tile, rp, s, S, h, c0, hf, first, w, xin, qa);
}

// ------------------------------------------------------------- block maps
// The Apply of one block (its 64 rows, kc <= 16 rotations each) to a column
// of the trailing matrix changes only the column's 64 entries in the block's
// rows and the column's 16 values of V (Algorithm 1, Apply), and it is
// linear in those 80 values with the same coefficients for every column: the
// block acts on each column as one 80 x 80 matrix, its map.  For an update
// the map is orthogonal (with 1/c and s/c as cosine and sine each rotation
// is a plane rotation); for a downdate it is a product of hyperbolic
// rotations.  An owner far behind the chain applies a block by its map -- a
// product of the map with the owner's 80 x 64 tile (64 rows of L, 16 rows of
// V) on the FP64 matrix cores -- instead of by the block's 1024 rotations
// one after the other; the workgroup that ran the block's chain builds the
// map once, by applying the block's rotations to the 80 unit vectors.
//
// The map's top-left 64 x 64 part is lower triangular (entry r of a column's
// result depends only on its entries <= r and on V), so 19 of its 25 16 x 16
// tiles are stored: the A operands of the v_mfma_f64_16x16x4 products that
// use them, 64 doubles each in lane order (lane l holds row l % 16, k index
// l / 16 of its operand), by row tile I (0..3: rows of L, 4: rows of V), then
// k-step.  The k-steps of row tile I < 4 are those of columns [0, 16 I + 16)
// of L and then the four of V; row tile 4 takes all 20.  k-step K, k index g
// is column 4 K + g of the 80 (rows of L, then of V): lane l of a product's
// output holds rows 4 r + l / 16 (r = 0..3) of column l % 16, which for row
// tile 4 is exactly the V operand the next block's k-steps 16 + r need from
// that lane, so V stays in registers from block to block.
//
// A map with an entry beyond kMapBound in magnitude (a downdate whose
// hyperbolic rotations grow vectors, or a block with a failed row) is marked
// unusable, and every owner applies that block by its rotations.
typedef double v4d __attribute__((ext_vector_type(4)));
constexpr int kMapPairs = 76;                // (row tile, k-step) operands stored
constexpr int kMapElems = kMapPairs * 64;    // doubles per map
constexpr int kLdM = kBR + kKP;              // row stride of the map being built
constexpr double kMapBound = 2.0;
constexpr int kNear = 3;                     // blocks before an owner's own applied by rotations
constexpr int kMinUses = 3;                  // a map is built only for this many owners or more

// Blocks [0, map_blocks(nb)) of a factor of nb blocks get maps: block b's
// map serves the owners of blocks b + kNear + 1 .. nb - 1.
__host__ __device__ constexpr int64_t map_blocks(int64_t nb) {
  return nb - kNear - kMinUses > 0 ? nb - kNear - kMinUses : 0;
}

// 8-byte words of a factor's map region: one map per block and pass.
__host__ __device__ constexpr int64_t map_words(int64_t n, int64_t k) {
  return ((k + kKP - 1) / kKP) * ((n + kBR - 1) / kBR) * kMapElems;
}
enum : int32_t { kMapOk = 1, kMapRot = 2, kMapWait = 3 };
// Map entries as published: a map region starts filled with kMapEmpty (a
// signalling NaN, which no arithmetic result is) and an unusable map is
// published as kMapRotate in every entry, so that, as with the rotation
// records, the data is its own ready flag and needs no fence or flag store.
constexpr uint64_t kMapEmpty = 0x7FF4A5A5A5A5A5A5ull;
constexpr uint64_t kMapRotate = 0x7FF4A5A5A5A5A5A6ull;

__host__ __device__ constexpr int map_base(int I) {
  return I == 0 ? 0 : I == 1 ? 8 : I == 2 ? 20 : I == 3 ? 36 : 56;
}
// k-steps of row tile I that take columns of L
__host__ __device__ constexpr int map_lk(int I) { return I < 4 ? 4 * (I + 1) : 16; }

// Row of the map and column (of the 80) of operand element (pair e, lane l).
__device__ __forceinline__ void map_entry(int e, int l, int& row, int& col) {
  const int I = e < 8 ? 0 : e < 20 ? 1 : e < 36 ? 2 : e < 56 ? 3 : 4;
  const int kl = e - map_base(I), g = l >> 4;
  row = 16 * I + (l & 15);
  col = kl < map_lk(I) ? 4 * kl + g : kBR + 4 * (kl - map_lk(I)) + g;
}

// Build the map of the block whose records are in sh.R (after its chain) and
// publish it: the 64 x 80 unit tile (its columns the unit vectors of the
// block's rows, then of V's rows) goes through the block's rotations on
// apply lanes 0 .. 319, the result is written in operand order with
// device-scope stores, and the map's state (usable or not) is stored after a
// device-scope fence.  Uses sh.Lh and sh.Hb; all threads of the workgroup.
template <int SG, int KCF>
__device__ __forceinline__ void map_build(SbLds& sh, int kc, double* __restrict__ Mg) {
  const int tid = threadIdx.x;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6);
  double* const tile = &sh.Lh[0][0];  // 64 x 80
  double* const vm = &sh.Hb[0][0][0];  // 16 x 80: V's rows of the result
  for (int idx = tid; idx < kBR * kLdM; idx += kThreads)
    tile[idx] = (idx / kLdM == idx % kLdM) ? 1.0 : 0.0;
  __syncthreads();
  // Waves 0-3 take the unit columns of the block's rows, 16 each; wave 7
  // (on the SIMD of wave 3, which has the least work) those of V.  Unit
  // column q < 64 stays zero, and V with it, until row q: wave c starts at
  // sub-step 16 c, where the lanes of h > 0 hold rows before its columns
  // (zero), so it skips the sub-steps that would only carry zeros.
  if (wv < 4 || wv == 7) {
    const int lt = wv < 4 ? tid : tid - 448 + kOwnThreads;
    const int s0 = wv < 4 ? 16 * wv : 0;
    const int kcc = KCF ? KCF : kc;
    const int h = (lt & 15) >> 1, c0 = own_col(lt, 0);
    const int hf = (kcc - 1) >> 1;
    const bool first = (kcc & 1) != 0;
    double w[kOwnCols];
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int u = 0; u < 2; ++u)
        w[2 * k + u] = own_col(lt, u) - kBR == own_rot(lt, k) ? 1.0 : 0.0;
    double xin[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) xin[u] = h == 0 ? tile[s0 * kLdM + c0 + u] : 0.0;
    const RotRec* rp = &sh.R[kPad - h][2 * h];
    RotRec qa[2] = {rp[s0 * kKP], rp[s0 * kKP + 1]};
    int s = s0;
    sub2x2_run<SG, double, kLdM>(tile, rp, s, kBR + hf, h, c0, hf, first, w, xin, qa);
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int u = 0; u < 2; ++u) vm[own_rot(lt, k) * kLdM + own_col(lt, u)] = w[2 * k + u];
  }
  __syncthreads();
  constexpr int kPer = (kMapElems + kThreads - 1) / kThreads;  // 10
  uint64_t v[kPer];
  bool bad = false;
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int idx = tid + q * kThreads;
    double x = 0.0;
    if (idx < kMapElems) {
      int row, col;
      map_entry(idx >> 6, idx & 63, row, col);
      x = row < kBR ? tile[row * kLdM + col] : vm[(row - kBR) * kLdM + col];
    }
    bad |= !(__builtin_fabs(x) <= kMapBound);
    v[q] = __builtin_bit_cast(uint64_t, x);
  }
  const bool rotate = __syncthreads_or(bad) != 0;
#pragma unroll
  for (int q = 0; q < kPer; ++q) {
    const int idx = tid + q * kThreads;
    if (idx < kMapElems)
      __hip_atomic_store(reinterpret_cast<uint64_t*>(Mg + idx), rotate ? kMapRotate : v[q],
                         __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
}

// Stage map Mb into LDS at dst: wave q of the four staging waves copies
// doubles [q * 1216, q * 1216 + 1216) once none of them is kMapEmpty any
// more (it polls, sleeping between polls; past the deadline it sets sh.tmo
// and gives up).  Returns kMapOk, or kMapRot for a map published as
// unusable (then nothing is copied); every staging wave finds the same.
// Every read is a device-scope load: the map region of a batch may hold an
// earlier batch's map (served batches reuse the workspace arena), and a
// cached copy of such a line is the one read that could see it.
constexpr int kMapPerWave = kMapElems / 4;  // 1216 = 19 x 64
__device__ __forceinline__ int map_stage(SbLds& sh, const double* Mb, double* dst,
                                         int64_t deadline, int q, int lane) {
  constexpr int kN = kMapPerWave / 64;
  const uint64_t* src = reinterpret_cast<const uint64_t*>(Mb + q * kMapPerWave) + lane;
  uint64_t v[kN];
  bool full = true;
#pragma unroll
  for (int i = 0; i < kN; ++i) {
    v[i] = __hip_atomic_load(const_cast<uint64_t*>(src + i * 64), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    full &= v[i] != kMapEmpty;
  }
  // the last entry of the quarter (one request per wave and poll) until it is
  // written, then the whole quarter until no entry is empty
  const uint64_t* last = reinterpret_cast<const uint64_t*>(Mb + (q + 1) * kMapPerWave) - 1;
  while (!__all(full)) {
    if (__all(__hip_atomic_load(const_cast<uint64_t*>(last), __ATOMIC_RELAXED,
                                __HIP_MEMORY_SCOPE_AGENT) != kMapEmpty)) {
      full = true;
#pragma unroll
      for (int i = 0; i < kN; ++i) {
        v[i] = __hip_atomic_load(const_cast<uint64_t*>(src + i * 64), __ATOMIC_RELAXED,
                                 __HIP_MEMORY_SCOPE_AGENT);
        full &= v[i] != kMapEmpty;
      }
      if (__all(full)) break;
    }
    if (wall_clock64() > deadline) {
      sh.tmo = 1;
      return kMapRot;
    }
    __builtin_amdgcn_s_sleep(20);
  }
  if (__builtin_amdgcn_readfirstlane((int)(v[0] == kMapRotate))) return kMapRot;
#pragma unroll
  for (int i = 0; i < kN; ++i) dst[q * kMapPerWave + i * 64 + lane] = __builtin_bit_cast(double, v[i]);
  return kMapOk;
}

// map_stage without waiting: kMapWait (nothing copied) if an entry of wave
// q's quarter is still empty.
__device__ __forceinline__ int map_try_stage(SbLds& sh, const double* Mb, double* dst, int q,
                                             int lane) {
  constexpr int kN = kMapPerWave / 64;
  const uint64_t* src = reinterpret_cast<const uint64_t*>(Mb + q * kMapPerWave) + lane;
  uint64_t v[kN];
  bool full = true;
#pragma unroll
  for (int i = 0; i < kN; ++i) {
    v[i] = __hip_atomic_load(const_cast<uint64_t*>(src + i * 64), __ATOMIC_RELAXED,
                             __HIP_MEMORY_SCOPE_AGENT);
    full &= v[i] != kMapEmpty;
  }
  if (!__all(full)) return kMapWait;
  if (__builtin_amdgcn_readfirstlane((int)(v[0] == kMapRotate))) return kMapRot;
#pragma unroll
  for (int i = 0; i < kN; ++i) dst[q * kMapPerWave + i * 64 + lane] = __builtin_bit_cast(double, v[i]);
  return kMapOk;
}

// B operands of the owner's tile (rows [pb, pb + 64), columns 16 ct ..
// 16 ct + 15 of those from pj, the first bbc in the factor) for one wave:
// bx[K] = row 4 K + lane / 16, column lane % 16.
template <typename ST>
__device__ __forceinline__ void map_tile_load(double (&bx)[16], const ST* __restrict__ L,
                                              int64_t ldl, int64_t pb, int64_t pj, int bbc,
                                              int ct, int lane) {
  const int g = lane >> 4, cl = 16 * ct + (lane & 15);
  const bool ok = cl < bbc;
#pragma unroll
  for (int K = 0; K < 16; ++K) bx[K] = ok ? (double)L[(pb + 4 * K + g) * ldl + pj + cl] : 0.0;
}

template <int I>
__device__ __forceinline__ void map_rows(const double* Mb, int lane, const double (&bx)[16],
                                         const double (&vx)[4], v4d& acc) {
  constexpr int nk = map_lk(I);
#pragma unroll
  for (int K = 0; K < nk; ++K)
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Mb[(map_base(I) + K) * 64 + lane], bx[K], acc, 0,
                                               0, 0);
#pragma unroll
  for (int q = 0; q < 4; ++q)
    acc = __builtin_amdgcn_mfma_f64_16x16x4f64(Mb[(map_base(I) + nk + q) * 64 + lane], vx[q],
                                               acc, 0, 0, 0);
}

// Row tiles I and J (map_lk(I) <= map_lk(J)) together, their products
// interleaved so that each accumulation chain's latency hides behind the
// other's.
template <int I, int J>
__device__ __forceinline__ void map_rows2(const double* Mb, int lane, const double (&bx)[16],
                                          const double (&vx)[4], v4d& ai, v4d& aj) {
  constexpr int ni = map_lk(I), nj = map_lk(J);
  static_assert(ni <= nj, "row tile order");
#pragma unroll
  for (int K = 0; K < ni; ++K) {
    ai = __builtin_amdgcn_mfma_f64_16x16x4f64(Mb[(map_base(I) + K) * 64 + lane], bx[K], ai, 0,
                                              0, 0);
    aj = __builtin_amdgcn_mfma_f64_16x16x4f64(Mb[(map_base(J) + K) * 64 + lane], bx[K], aj, 0,
                                              0, 0);
  }
#pragma unroll
  for (int K = ni; K < nj; ++K)
    aj = __builtin_amdgcn_mfma_f64_16x16x4f64(Mb[(map_base(J) + K) * 64 + lane], bx[K], aj, 0,
                                              0, 0);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    ai = __builtin_amdgcn_mfma_f64_16x16x4f64(Mb[(map_base(I) + ni + q) * 64 + lane], vx[q], ai,
                                              0, 0, 0);
    aj = __builtin_amdgcn_mfma_f64_16x16x4f64(Mb[(map_base(J) + nj + q) * 64 + lane], vx[q], aj,
                                              0, 0, 0);
  }
}

// Apply the map staged in LDS at Mb to the wave's 16 columns of the owner's
// tile, whose B operands are in bx (map_tile_load), one wave; the result
// rows go to L, and vx (V of those columns: lane l, element r is row
// 4 r + l / 16 of V, column l % 16) is updated in place.
template <typename ST>
__device__ __forceinline__ void map_apply(const double* Mb, const double (&bx)[16],
                                          ST* __restrict__ L, int64_t ldl, int64_t pb,
                                          int64_t pj, int bbc, int ct, int lane,
                                          double (&vx)[4]) {
  const int g = lane >> 4, cl = 16 * ct + (lane & 15);
  // two row tiles at a time (V's last: vx is an input of all five), each
  // stored at once, so that few accumulators and operands are live (the
  // scheduling barriers keep the compiler from hoisting every operand load
  // of the block)
  auto store = [&](int I, const v4d& acc) {
    if (cl < bbc) {
#pragma unroll
      for (int r = 0; r < 4; ++r) L[(pb + 16 * I + 4 * r + g) * ldl + pj + cl] = (ST)acc[r];
    }
  };
  const v4d z = {0.0, 0.0, 0.0, 0.0};
  v4d a = z, b = z;
  map_rows<0>(Mb, lane, bx, vx, a);
  store(0, a);
  __builtin_amdgcn_sched_barrier(0);
  a = z;
  map_rows2<1, 2>(Mb, lane, bx, vx, a, b);
  store(1, a);
  store(2, b);
  __builtin_amdgcn_sched_barrier(0);
  a = z;
  b = z;
  map_rows2<3, 4>(Mb, lane, bx, vx, a, b);
  store(3, a);
#pragma unroll
  for (int r = 0; r < 4; ++r) vx[r] = b[r];
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
  double bx0, bx1, bw; // band of the previous step, stored at the next one
};

__device__ __forceinline__ void chain_init(SbLds& sh, ChainState& g, int lane) {
  const Feed f0 = sh.fd[0];
  g.tp = f0.t;
  g.il = f0.il;
  g.lin = f0.l;
  g.v = sh.Hb[lane & 15][1][0];
  g.lo = f0.lo;
  g.hi = f0.hi;
  g.pc = 1.0;
  g.ps = 0.0;
  g.pic = 1.0;
  g.bx0 = g.bx1 = g.bw = 0.0;
}

// One step t of wave 0, lane m < kc (the wave runs with the other lanes
// masked off): Compute(i, m) for i = t - m, then the Apply of rows i-1 (the
// lane's record of the previous step) and i to column i+1, whose V_{i+1}[m]
// after rows < i-1 the helpers left in Hb at the previous step.  Reads state
// g, writes state o (the caller alternates two states, so nothing is copied
// between steps).  hb: this lane's Hb value for the step; rec, band: where
// the lane's record and band go (row i + 16); fn: row t+1's feed, the values
// lane 0 takes at the next step.
//
// FILL (the first kc - 1 steps): lanes with i < 0 have not started; they
// keep their state, write identity records into the pad rows before the
// block and pass identity values on.  In every other step each lane
// computes: lanes whose row i is at or after the block's last row compute
// rows nobody reads (their records and bands land in the pad rows after the
// block, their Hb reads stay inside LDS), and values of such rows only flow
// to rows after them.
template <bool FILL, int SG, typename RP, typename BP>
__device__ __forceinline__ void chain_step(const ChainState& g, ChainState& o, double Wc,
                                           const Feed fn, RP rec, BP band, bool started) {
  // the previous step's band: nobody reads it during the chain, so it is
  // stored here, where its LDS latency overlaps this step's Compute
  band[-1].lo = g.bx0;
  band[-1].hi = g.bx1;
  band[-1].d = g.bw;
  // Compute(i, m)
  const double v = g.v;
  const double tt = __builtin_fma(SG * v, v, g.tp);
  const double y = rsqrt_refined(tt);
  const double ww = tt * y;
  const double s = v * g.il;
  const double c = ww * g.il;
  const double ic = g.lin * y;
  // the record goes out as soon as it exists: the helpers read it after this
  // step's barrier, which waits for the store
  if (FILL) {
    rec->c = started ? c : 1.0;
    rec->s = started ? s : 0.0;
    rec->ic = started ? ic : 1.0;
  } else {
    rec->c = c;
    rec->s = s;
    rec->ic = ic;
  }
  __builtin_amdgcn_sched_barrier(0);
  o.tp = sb_shr1(tt, fn.t);
  o.il = sb_shr1(y, fn.il);
  o.lin = sb_shr1(ww, fn.l);  // L_ii after column m = t * y: what tp * il gives lane m+1
  // rows i-1 (record of the previous step) and i applied to column i+1
  const double x0 = __builtin_fma(SG * g.ps, Wc, g.lo) * g.pic;
  Wc = __builtin_fma(-g.ps, x0, g.pc * Wc);
  const double x1 = __builtin_fma(SG * s, Wc, g.hi) * ic;
  Wc = __builtin_fma(-s, x1, c * Wc);
  if (FILL) {
    o.v = started ? Wc : v;
    o.pc = started ? c : 1.0;
    o.ps = started ? s : 0.0;
    o.pic = started ? ic : 1.0;
  } else {
    o.v = Wc;
    o.pc = c;
    o.ps = s;
    o.pic = ic;
  }
  o.bx0 = x0;
  o.bx1 = x1;
  o.bw = ww;
  // to lane m+1 (lane 0 takes row t+1's originals)
  o.lo = sb_shr1(x0, fn.lo);
  o.hi = sb_shr1(x1, fn.hi);
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
  if (H < 6) sh.X[H < 6 ? H : 0][t & 1][jj] = st[2 * CNT - 1];
  if (H == 0) st[2 * CNT] = sh.Lb[imin(t, kBR - 1)][jj];
}

// LDS pointers that the compiler must keep in a register as they are (it
// would otherwise re-add the array's base address, which is too large for an
// LDS instruction's immediate offset, at every access).
template <typename T>
using lds_ptr = __attribute__((address_space(3))) T*;

template <typename T>
__device__ __forceinline__ lds_ptr<T> lds_pin(const void* p) {
  uint32_t a = (uint32_t)(uintptr_t)(lds_ptr<const char>)p;
  asm volatile("" : "+v"(a));
  return (lds_ptr<T>)(uintptr_t)a;
}

__device__ __forceinline__ Feed load_feed(lds_ptr<const Feed> p, int i) {
  const lds_ptr<const double> d = (lds_ptr<const double>)(p + i);
  Feed f;
  f.t = d[0];
  f.il = d[1];
  f.l = d[2];
  f.lo = d[3];
  f.hi = d[4];
  f.pad = 0.0;
  return f;
}

// Wave 0's step loop over steps [0, nsteps), one barrier per step; lanes
// m < kc compute, the others only pass the barriers.  Per lane the LDS
// addresses of step t are fixed offsets plus t: Hb[m][(t-1) & 1][t - m + 1],
// R[t - m + 16][m], Lc[t - m + 16], fd[t + 1].  Steps run in pairs with the
// two states alternating; the pairs start on an even step, so step parity
// (Hb's buffer) is known statically.  The feeds of a pair are read before
// its first step, so their load latency is hidden.
template <int SG>
__device__ __forceinline__ void chain_wave0(SbLds& sh, int m, int kc, int nsteps) {
  const bool act = m < kc;
  const int ml = m & 15;
  ChainState ga, gb;
  chain_init(sh, ga, ml);
  __syncthreads();
  // + t + 64 * parity of t-1
  lds_ptr<const double> hb = lds_pin<const double>(&sh.Hb[0][0][0] + 128 * ml + 1 - ml);
  lds_ptr<RotRec> rec = lds_pin<RotRec>(&sh.R[0][0] + kPad * kKP - (kKP - 1) * ml);  // + 16 t
  lds_ptr<Band> band = lds_pin<Band>(&sh.Lc[kPad] - ml);                            // + t
  lds_ptr<const Feed> fd = lds_pin<const Feed>(&sh.fd[1]);                          // + t
  int t = 0;
  // fill: steps [0, kc - 1), in pairs, then the odd one
  // No barrier may sit inside a branch on `act`: a wave with lanes on both
  // sides would execute both sides' barriers.
  for (; t + 2 <= kc - 1; t += 2) {
    const Feed f0 = load_feed(fd, 0), f1 = load_feed(fd, 1);
    if (act) chain_step<true, SG>(ga, gb, hb[64], f0, rec, band, t >= ml);
    __syncthreads();
    if (act) chain_step<true, SG>(gb, ga, hb[1], f1, rec + kKP, band + 1, t + 1 >= ml);
    __syncthreads();
    hb += 2; rec += 2 * kKP; band += 2; fd += 2;
  }
  if (t < kc - 1) {  // t even
    if (act) chain_step<true, SG>(ga, gb, hb[64], load_feed(fd, 0), rec, band, t >= ml);
    __syncthreads();
    ga = gb;
    ++t; hb += 1; rec += kKP; band += 1; fd += 1;
  }
  if (t < nsteps && (t & 1)) {  // align the pairs to an even step
    if (act) chain_step<false, SG>(ga, gb, hb[0], load_feed(fd, 0), rec, band, true);
    __syncthreads();
    ga = gb;
    ++t; hb += 1; rec += kKP; band += 1; fd += 1;
  }
  for (; t + 2 <= nsteps; t += 2) {
    const Feed f0 = load_feed(fd, 0), f1 = load_feed(fd, 1);
    if (act) chain_step<false, SG>(ga, gb, hb[64], f0, rec, band, true);
    __syncthreads();
    if (act) chain_step<false, SG>(gb, ga, hb[1], f1, rec + kKP, band + 1, true);
    __syncthreads();
    hb += 2; rec += 2 * kKP; band += 2; fd += 2;
  }
  if (t < nsteps) {
    if (act) chain_step<false, SG>(ga, gb, hb[64], load_feed(fd, 0), rec, band, true);
    __syncthreads();
    ga = gb;
    band += 1;
  }
  // the last step's band (read after the caller's next barrier)
  if (act) {
    band[-1].lo = ga.bx0;
    band[-1].hi = ga.bx1;
    band[-1].d = ga.bw;
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

template <typename ST>
__device__ __forceinline__ void publish_rows(SbLds& sh, GRec<ST>* __restrict__ T, int64_t pc,
                                             int r0, int kc, int lane);

// The helper on wave 4 (column 15 of V), which also publishes the block's
// records 4 rows at a time as they complete: after barrier u (u = t + 1
// after step t) the rows up to u - kc are complete.  The records are read
// from LDS right after that barrier and stored to T during the next step,
// when the read has long completed, so that the step does not wait for it.
template <int SG, typename ST, int KCF>
__device__ __forceinline__ void helper_steps_pub(SbLds& sh, int nsteps, int lane, int kc,
                                                 bool pub, GRec<ST>* __restrict__ T,
                                                 int64_t pc) {
  double st[kSt];
  helper_init<15, 1>(sh, st, lane);
  __syncthreads();
  // rows [rn, rn + 4) are read after step tn - 1, in groups of four as
  // each group is complete and the block's last four rows one by one, so
  // that the next owner can apply rows 60..62 before row 63 arrives
  int rn = 0, tn = pub ? 3 + kc : -1;
  bool have = false;
  RotRec rec;
  GRec<ST>* dst = T;
  for (int t = 0; t < nsteps; ++t) {
    helper_step<6, 15, 1, SG, KCF>(sh, st, t, lane, kc);
    if (have) publish_record(dst, rec);
    have = false;
    __syncthreads();
    if (t + 1 == tn) {
      const bool one = rn >= kBR - 4;
      const int r = rn + (one ? 0 : lane >> 4), m = lane & 15;
      rec = sh.R[r + kPad][m];
      dst = T + (pc + r) * kKP + m;
      have = m < kc && (!one || lane < 16);
      rn += one ? 1 : 4;
      tn = rn >= kBR ? -1 : rn < kBR - 4 ? rn + 3 + kc : rn + kc;
    }
  }
  if (have) publish_record(dst, rec);
}

// LDS set-up of a chain that needs only the block's triangle (staged in
// sh.Lb): the helpers' transfer rows cleared, and each row's diagonal and
// lane 0's inputs.
__device__ __forceinline__ void chain_setup_tri(SbLds& sh, int bbc) {
  const int tid = threadIdx.x;
  for (int idx = tid; idx < 6 * kBR; idx += kThreads) sh.X[idx >> 6][1][idx & 63] = 0.0;
  if (tid == 0) sh.fail = 0x7fffffff;
  if (tid < kRRows) {
    const int r = tid < kBR ? tid : kBR - 1;
    const double l = sh.Lb[r][r];
    Feed f;
    f.l = l;
    f.t = l * l;
    f.il = 1.0 / l;
    // lane 0 at step t applies rows t-1 and t to column t+1
    f.lo = (tid >= 1 && tid + 1 < bbc) ? sh.Lb[tid - 1][tid + 1] : 0.0;
    f.hi = (tid + 1 < bbc) ? sh.Lb[tid][tid + 1] : 0.0;
    f.pad = 0.0;
    sh.fd[tid] = f;
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
  const int nsteps = bbc + kc - 1;
  // columns of V per helper 3 3 3 2 2 2 1, so that each SIMD runs five
  // (waves w and w + 4 share SIMD w; wave 0 runs the Computes)
  if (wv == 0) {
    chain_wave0<SG>(sh, lane, kc, nsteps);
  } else if (wv == 4) {
    helper_steps_pub<SG, ST, KCF>(sh, nsteps, lane, kc, pub, T, pc);
  } else if (wv == 1) {
    helper_steps<0, 0, 3, SG, KCF>(sh, nsteps, lane, kc);
  } else if (wv == 2) {
    helper_steps<1, 3, 3, SG, KCF>(sh, nsteps, lane, kc);
  } else if (wv == 3) {
    helper_steps<2, 6, 3, SG, KCF>(sh, nsteps, lane, kc);
  } else if (wv == 5) {
    helper_steps<3, 9, 2, SG, KCF>(sh, nsteps, lane, kc);
  } else if (wv == 6) {
    helper_steps<4, 11, 2, SG, KCF>(sh, nsteps, lane, kc);
  } else {
    helper_steps<5, 13, 2, SG, KCF>(sh, nsteps, lane, kc);
  }
}

// After the loops: the first failure of the block and the block's triangle.
// A Compute fails iff its radicand is not > 0 (then y, w and c are NaN) or,
// for column 0, the original diagonal is not > 0 (then c = w / L_ii is
// negative, infinite or NaN); every later Compute of the same row or of a
// later row may be garbage, none of an earlier row is.  So the failure is
// the first record whose c is not a finite positive number.  store: the
// triangle goes to L; otherwise (another pass of the same block follows) it
// goes back to sh.Lb, rounded to the storage type as a store and reload
// would, so that the next pass starts from what L would hold.
template <typename ST>
__device__ __forceinline__ void chain_finish(SbLds& sh, ST* __restrict__ L, int64_t ldl, int kc,
                                             int64_t kfull, int64_t m0, int64_t pc, int bbc,
                                             int64_t* __restrict__ info,
                                             int64_t* __restrict__ stop_row, bool store = true) {
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
    const int64_t code = (m == 0 && !(sh.fd[r].l > 0.0)) ? kCodeBadDiag : kCodeNotPD;
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
      if (store) L[(pc + i) * ldl + pc + j] = (ST)x;
      else sh.Lb[i][j] = (double)(ST)x;
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
// two-column lanes of sub2x2.  Waves 4-7 fetch the records: wave 4 + w
// polls the records of rows [16 w, 16 w + 16) of the applied block, stages
// those that have been published in sh.R and counts how many rows of its
// window (a prefix) are staged.  In rounds separated by barriers, the apply
// waves run the sub-steps whose rows are all staged -- the rows before the
// first window that is not complete -- while the fetch waves stage more.
// Only the wave whose window is the first incomplete one waits for records
// to appear; a block whose records are all published (an owner far behind
// the chain) is staged in one round and applied without a barrier.

// Apply block [pb, pb + 64) (tile staged in sh.A, the caller has
// synchronised) to the owner's columns; w: an apply lane's V values.  next:
// block pb is the one just before the owner's own (its chain waits for this
// apply), so the waiting fetch wave polls without delay; the owners further
// right poll slowly, which keeps their reads of the same few records from
// crowding the memory channels.  Same operations, in the same order, as
// apply2x2.
template <int SG, typename ST, int KCF>
__device__ __forceinline__ void owner_apply(SbLds& sh, int kc_, int64_t pb,
                                            ST (&w)[kOwnCols],
                                            const GRec<ST>* __restrict__ T, int64_t deadline,
                                            bool next, int poll) {
  using U = typename RecBits<ST>::U;
  constexpr U kE = RecBits<ST>::kEmpty;
  const int kc = KCF ? KCF : kc_;
  const int tid = threadIdx.x;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  // rows staged before the first incomplete window, from the round's counts
  auto staged_prefix = [&](int par) {
    int up = 0;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int c = sh.cnt[par][q];
      up += c;
      if (c < 16) break;
    }
    return up;
  };
  if (wv < 4) {
    const int h = (lane & 15) >> 1;
    const int c0 = own_col(tid, 0);
    const int hf = (kc - 1) >> 1;          // lane holding rotation kc - 1
    const bool first = (kc & 1) != 0;      // ... as the first of its pair
    const int S = kBR + hf;                // row 63 reaches lane hf at sub-step 63 + hf
    ST* const tile = tile_a<ST>(sh);
    constexpr int LD = kLdA;
    ST xin[2];
#pragma unroll
    for (int u = 0; u < 2; ++u) xin[u] = (ST)tile[c0 + u];
    // records of (row s - h, rotations 2h and 2h+1) at rp[s * kKP], rp[s * kKP + 1]
    const RotRec* rp = &sh.R[kPad - h][2 * h];
    int s = 0;
    for (int rd = 0;; ++rd) {
      __syncthreads();
      const int up = staged_prefix(rd & 1);
      const int lim = up >= kBR ? S : up;  // rows <= s - h < up are staged
      RotRec qa[2] = {rp[s * kKP], rp[s * kKP + 1]};
      sub2x2_run<SG, ST, LD>(tile, rp, s, lim, h, c0, hf, first, w, xin, qa);
      if (up >= kBR) break;
    }
  } else {
    // fetch wave q: rows r0 + up_w + 4 v + lane / 16 (v = 0..3) of its
    // window [r0, r0 + 16), column m
    const int q = wv - 4, r0 = 16 * q;
    const int m = lane & 15, rl = lane >> 4;
    U f[4][3];
    auto fetch = [&](int upw) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = r0 + upw + 4 * v + rl;
        if (upw + 4 * v + rl < 16 && r < kBR && m < kc) {
          const GRec<ST>* src = T + (pb + r) * kKP + m;
          f[v][0] = load_bits(&src->c);
          f[v][1] = load_bits(&src->s);
          f[v][2] = load_bits(&src->ic);
        } else {
          f[v][0] = f[v][1] = f[v][2] = 0;  // nothing to wait for
        }
      }
    };
    // rows of the window's rest (bit 4 v + group) whose records are all there
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
    int upw = 0;          // rows of the window staged
    int known = 0;        // rows of the block staged before the first incomplete window
    fetch(0);
    for (int rd = 0;; ++rd) {
      if (upw < 16) {
        int nr = __builtin_ctz(~ready_rows());
        // the first incomplete window waits for at least one more row
        while (nr == 0 && known == r0 + upw) {
          if (wall_clock64() > deadline) {  // give up: stage what is there
            sh.tmo = 1;
            nr = 16;
            break;
          }
          if (next || poll == 0) __builtin_amdgcn_s_sleep(1);
          else if (poll == 1) __builtin_amdgcn_s_sleep(20);
          else __builtin_amdgcn_s_sleep(100);
          fetch(upw);
          nr = __builtin_ctz(~ready_rows());
        }
        if (sh.tmo) nr = 16;  // a wait ran out: every window counts as staged
        if (nr > 16 - upw) nr = 16 - upw;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int rr = upw + 4 * v + rl, r = r0 + rr;
          if (4 * v + rl < nr && r < kBR && m < kc) {
            RotRec rec;
            rec.c = (double)__builtin_bit_cast(ST, f[v][0]);
            rec.s = (double)__builtin_bit_cast(ST, f[v][1]);
            rec.ic = (double)__builtin_bit_cast(ST, f[v][2]);
            rec.ss = 0.0;
            sh.R[kPad + r][m] = rec;
          }
        }
        upw += nr;
        if (upw < 16) fetch(upw);  // in flight while the apply waves run
      }
      if (lane == 0) sh.cnt[rd & 1][q] = upw;
      __syncthreads();
      known = staged_prefix(rd & 1);
      if (known >= kBR) break;
    }
  }
}

// One factor as the owner kernels see it.  Pass p (columns 16p .. of V)
// keeps its records at T + p * n * 16 and the maps of its blocks at
// maps + p * nb * kMapElems (nb blocks); maps == nullptr: every block is
// applied by its rotations.
template <typename ST>
struct OwnF {
  ST* L;
  ST* W;  // private copy of V, row stride k
  GRec<ST>* T;
  double* maps;
  int64_t* info;
  int64_t* stop;
  int64_t n, k, ldl;
  int fuse;    // pass pairs share their far blocks' tiles
  double* vc;  // binary32 storage: V of the odd pass of each pair, n x 16 per pair
};

// V of apply lane tid's columns from rows m of buf[m * 64 + c] (the 16 x 64
// staging area in sh.Hb) and back: how V moves between the map layout and
// the rotation layout.
template <typename ST>
__device__ __forceinline__ void w_from_lds(ST (&w)[kOwnCols], const double* buf, int kc,
                                           int bbc, int tid) {
#pragma unroll
  for (int k = 0; k < 2; ++k)
#pragma unroll
    for (int u = 0; u < 2; ++u) {
      const int c = own_col(tid, u), m = own_rot(tid, k);
      w[2 * k + u] = (c < bbc && m < kc) ? (ST)buf[m * kBR + c] : (ST)0;
    }
}

template <typename ST>
__device__ __forceinline__ void w_to_lds(const ST (&w)[kOwnCols], double* buf, int tid) {
#pragma unroll
  for (int k = 0; k < 2; ++k)
#pragma unroll
    for (int u = 0; u < 2; ++u) buf[own_rot(tid, k) * kBR + own_col(tid, u)] = (double)w[2 * k + u];
}

// Pass `pass` of the owner of block j (the block's triangle is in sh.Lb):
// apply blocks 0 .. j-1 of this pass to the block's columns as their owners
// publish them, then the block's chain, publishing its records.  last: the
// triangle goes to L, else back to sh.Lb for the next pass.
template <int SG, typename ST, int KCF>
__device__ __forceinline__ void owner_pass(SbLds& sh, const OwnF<ST>& F, int j, int bbc,
                                           int pass, bool last, int64_t deadline, int poll,
                                           int& nfz) {
  const int tid = threadIdx.x;
  const int64_t m0 = (int64_t)pass * kKP;
  const int kc = KCF ? KCF : (int)(F.k - m0 < kKP ? F.k - m0 : kKP);
  const int64_t pj = (int64_t)j * kBR;
  GRec<ST>* const T = F.T + (int64_t)pass * F.n * kKP;
  ST* const W = F.W + m0;
  const int64_t ldw = F.k;
  const int wv = __builtin_amdgcn_readfirstlane(tid >> 6), lane = tid & 63;
  const int64_t nb = (F.n + kBR - 1) / kBR;
  // blocks [0, nfar) by their maps (blocks before j - kNear, whose maps are
  // built right after their chains, if they have maps at all), the rest by
  // their rotations.  Passes run in pairs: pass p (even) also applies the
  // maps of pass p + 1 (its "fused" blocks) while it has the tile at hand,
  // for blocks whose pass p + 1 map is published already, and leaves V of
  // pass p + 1 in the private copy; pass p + 1 then starts at block nfz.
  const int nfar = F.maps ? imax(0, imin(j - kNear, (int)map_blocks(nb))) : 0;
  // nfz < 0: the even pass before did not pair (V of this pass is in W)
  const bool carried = (pass & 1) && nfz >= 0;
  const int b0 = carried ? nfz : 0;
  const bool far = nfar > b0;
  const bool fuse = F.fuse && far && (pass & 1) == 0 && m0 + kKP < F.k;
  const int kc1 = fuse ? (int)(F.k - m0 - kKP < kKP ? F.k - m0 - kKP : kKP) : 0;
  if ((pass & 1) == 0) nfz = fuse ? 0 : -1;
  // where the odd pass of a pair finds its V: the private copy of V, or the
  // carry area (binary32 storage, whose private copy would round it)
  double* const vc = F.vc ? F.vc + (int64_t)(pass >> 1) * F.n * kKP : nullptr;
  const bool from_vc = carried && vc != nullptr;
  double* const maps = F.maps ? F.maps + (int64_t)pass * nb * kMapElems : nullptr;
  double* const maps1 = fuse ? maps + nb * kMapElems : nullptr;
  double* const vbuf = &sh.Hb[0][0][0];  // 16 x 64: V between the two layouts
  // every global input of the pass is issued before anything is staged: V
  // of the block's columns and the first tile
  ST w[kOwnCols];
  double vx[4];   // map layout (waves 0-3): row 4 r + lane / 16 of V, column 16 wv + lane % 16
  double vx1[4];  // ... of pass p + 1, while fusing
  if (far) {
    const int cl = 16 * wv + (lane & 15);
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      const int m = 4 * r + (lane >> 4);
      const bool ok = wv < 4 && cl < bbc && m < kc;
      vx[r] = !ok ? 0.0 : from_vc ? vc[(pj + cl) * kKP + m] : (double)W[(pj + cl) * ldw + m];
      vx1[r] = (wv < 4 && cl < bbc && m < kc1) ? (double)W[(pj + cl) * ldw + kKP + m] : 0.0;
    }
  } else {
#pragma unroll
    for (int k = 0; k < 2; ++k)
#pragma unroll
      for (int u = 0; u < 2; ++u) {
        const int c = own_col(tid, u), m = own_rot(tid, k);
        const bool ok = tid < kOwnThreads && c < bbc && m < kc;
        w[2 * k + u] = !ok ? (ST)0 : from_vc ? (ST)vc[(pj + c) * kKP + m] : W[(pj + c) * ldw + m];
      }
  }
  TileRegs<ST> tr;
  if (!far && nfar < j) tile_issue_a(tr, F.L, F.ldl, (int64_t)nfar * kBR, pj, bbc);
  // identity records everywhere: the pad rows keep them, each block's rows
  // are overwritten as they arrive (after the far blocks, whose maps are
  // staged where the records go)
  if (!far)
    for (int idx = tid; idx < kRRows * kKP; idx += kThreads) sh.R[idx >> 4][idx & 15] = identity_rec();
  __syncthreads();
  chain_setup_tri(sh, bbc);  // needs only the triangle: done before the applies
  if (far) {
    // Far blocks: waves 0-3 multiply a map (staged in LDS buffer ib) into
    // their columns while waves 4-7 stage the next map into the other
    // buffer; each wave 0-3 loads its B operands of the next tile during the
    // products.  The maps go in the order (b, pass p), then, while fusing,
    // (b, pass p + 1) on the same tile (stored after the first product,
    // read again from the cache).  A pass p map that is not usable makes
    // the workgroup apply that block by its rotations; a pass p + 1 map
    // that is not there yet (or not usable) ends the fusing.
    // map buffer ib: the apply tile's region (0) or the records' (1)
    auto mbuf = [&](int ib) -> double* { return ib ? &sh.R[0][0].c : &sh.Lh[0][0]; };
    // the staging waves' findings on the map of buffer ib, combined
    auto state = [&](int ib) {
      int ok = 1, rot = 0;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        const int v = sh.mst[ib][q];
        ok &= v == kMapOk;
        rot |= v == kMapRot;
      }
      return ok ? kMapOk : rot ? kMapRot : kMapWait;
    };
    double bx[16];
    int b = b0, sp = 0, ib = 0;  // the current map: block b, pass p + sp, in buffer ib
    bool fusing = fuse;
    if (wv >= 4) {
      sh.mst[0][wv - 4] = map_stage(sh, maps + (int64_t)b * kMapElems, mbuf(0), deadline, wv - 4,
                                    lane);
    } else {
      map_tile_load<ST>(bx, F.L, F.ldl, (int64_t)b * kBR, pj, bbc, wv, lane);
    }
    __syncthreads();
    while (b < nfar) {
      const int64_t pb = (int64_t)b * kBR;
      const int st = state(ib);
      if (sp == 1 && st != kMapOk) {
        // block b's pass p + 1 map is not there: pass p + 1 resumes here
        // (vx holds pass p + 1's V since the swap before this map)
        fusing = false;
        nfz = b;
        sp = 0;
        if (wv < 4) {
#pragma unroll
          for (int r = 0; r < 4; ++r) {
            const double t = vx[r];
            vx[r] = vx1[r];
            vx1[r] = t;
          }
        }
        if (++b >= nfar) break;
        // block b + 1's pass p map into the other buffer (the one just
        // applied), so that nobody rewrites the state being read
        if (wv >= 4) {
          sh.mst[ib ^ 1][wv - 4] = map_stage(sh, maps + (int64_t)b * kMapElems, mbuf(ib ^ 1),
                                             deadline, wv - 4, lane);
        } else {
          map_tile_load<ST>(bx, F.L, F.ldl, (int64_t)b * kBR, pj, bbc, wv, lane);
        }
        __syncthreads();
        ib ^= 1;
        continue;
      }
      if (st != kMapOk && fusing) {
        fusing = false;  // block b goes by its rotations: pass p + 1 resumes here
        nfz = b;
      }
      // the map after this one
      const int bn = (fusing && sp == 0) ? b : b + 1, sn = (fusing && sp == 0) ? 1 : 0;
      const bool more = bn < nfar;
      if (st == kMapOk) {
        if (wv < 4) {
          // one call site for both passes of a pair (the product is large):
          // vx holds the V of the map's pass, vx1 the other's
          map_apply<ST>(mbuf(ib), bx, F.L, F.ldl, pb, pj, bbc, wv, lane, vx);
          if (sp != sn) {
#pragma unroll
            for (int r = 0; r < 4; ++r) {
              const double t = vx[r];
              vx[r] = vx1[r];
              vx1[r] = t;
            }
          }
          if (more) map_tile_load<ST>(bx, F.L, F.ldl, (int64_t)bn * kBR, pj, bbc, wv, lane);
        } else if (more) {
          const double* src = (sn ? maps1 : maps) + (int64_t)bn * kMapElems;
          sh.mst[ib ^ 1][wv - 4] = sn ? map_try_stage(sh, src, mbuf(ib ^ 1), wv - 4, lane)
                                      : map_stage(sh, src, mbuf(ib ^ 1), deadline, wv - 4, lane);
        }
        __syncthreads();
      } else {
        // by the block's rotations (the map buffers are free: the next map
        // is staged afterwards); V to the rotation layout and back
        if (wv < 4) {
#pragma unroll
          for (int r = 0; r < 4; ++r) vbuf[(4 * r + (lane >> 4)) * kBR + 16 * wv + (lane & 15)] = vx[r];
        }
        for (int idx = tid; idx < kRRows * kKP; idx += kThreads)
          sh.R[idx >> 4][idx & 15] = identity_rec();
        TileRegs<ST> tf;
        tile_issue_a(tf, F.L, F.ldl, pb, pj, bbc);
        __syncthreads();
        if (tid < kOwnThreads) w_from_lds(w, vbuf, kc, bbc, tid);
        tile_stage(sh, tf);
        __syncthreads();
        owner_apply<SG, ST, KCF>(sh, kc, pb, w, T, deadline, false, poll);
        __syncthreads();
#pragma unroll
        for (int q = 0; q < kTilePerThread; ++q) {
          const int idx = tid + q * kThreads, r = idx >> 6, c = idx & 63;
          if (c < bbc) F.L[(pb + r) * F.ldl + pj + c] = tile_a<ST>(sh)[r * kLdA + c];
        }
        if (tid < kOwnThreads) w_to_lds(w, vbuf, tid);
        __syncthreads();
        if (wv < 4) {
#pragma unroll
          for (int r = 0; r < 4; ++r) vx[r] = vbuf[(4 * r + (lane >> 4)) * kBR + 16 * wv + (lane & 15)];
          if (more) map_tile_load<ST>(bx, F.L, F.ldl, (int64_t)bn * kBR, pj, bbc, wv, lane);
        } else if (more) {
          sh.mst[ib ^ 1][wv - 4] = map_stage(sh, maps + (int64_t)bn * kMapElems, mbuf(ib ^ 1),
                                             deadline, wv - 4, lane);
        }
        __syncthreads();
      }
      b = bn;
      sp = sn;
      ib ^= 1;
    }
    if (fusing) nfz = nfar;  // every far block's pass p + 1 map is applied
    if (fuse && wv < 4) {
      // V of pass p + 1 after blocks [0, nfz), for pass p + 1
      const int cl = 16 * wv + (lane & 15);
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const int m = 4 * r + (lane >> 4);
        if (cl < bbc && m < kc1) {
          if (F.vc) F.vc[(int64_t)(pass >> 1) * F.n * kKP + (pj + cl) * kKP + m] = vx1[r];
          else W[(pj + cl) * ldw + kKP + m] = (ST)vx1[r];
        }
      }
    }
    // V to the rotation layout for the rest; the records get their identity
    // pad rows back
    if (wv < 4) {
#pragma unroll
      for (int r = 0; r < 4; ++r) vbuf[(4 * r + (lane >> 4)) * kBR + 16 * wv + (lane & 15)] = vx[r];
    }
    for (int idx = tid; idx < kRRows * kKP; idx += kThreads) sh.R[idx >> 4][idx & 15] = identity_rec();
    if (j > nfar) tile_issue_a(tr, F.L, F.ldl, (int64_t)nfar * kBR, pj, bbc);
    __syncthreads();
    if (tid < kOwnThreads) w_from_lds(w, vbuf, kc, bbc, tid);
  }
  for (int b = nfar; b < j; ++b) {
    __syncthreads();  // sh.A is free again
    tile_stage(sh, tr);
    if (b + 1 < j) tile_issue_a(tr, F.L, F.ldl, (int64_t)(b + 1) * kBR, pj, bbc);
    const int64_t pb = (int64_t)b * kBR;
    __syncthreads();
    owner_apply<SG, ST, KCF>(sh, kc, pb, w, T, deadline, b == j - 1, poll);
    __syncthreads();
#pragma unroll
    for (int q = 0; q < kTilePerThread; ++q) {
      const int idx = tid + q * kThreads, r = idx >> 6, c = idx & 63;
      if (c < bbc) F.L[(pb + r) * F.ldl + pj + c] = tile_a<ST>(sh)[r * kLdA + c];
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
  __syncthreads();
  chain_loops<SG, ST, KCF>(sh, kc, bbc, pj + kBR < F.n, T, pj);
  chain_finish(sh, F.L, F.ldl, kc, F.k, m0, pj, bbc, F.info, F.stop, last);
  if (tid == 0 && sh.tmo)
    atomicMin((unsigned long long*)F.info,
              (unsigned long long)info_key(pj * F.k + m0, kCodeTimeout));
  // the block's map, for the owners of blocks j + kNear + 1 and later
  if (F.maps && j < map_blocks(nb)) {
    // the build's pipeline runs past the block's rows, where it must find
    // identity records: the chain's lanes that ran past the block left the
    // records of rows they computed for nothing there (of rotations that are
    // the identity only up to the near-zero V values they read)
    for (int idx = tid; idx < kKP * kKP; idx += kThreads)
      sh.R[kPad + kBR + (idx >> 4)][idx & 15] = identity_rec();
    __syncthreads();
    map_build<SG, KCF>(sh, kc, maps + (int64_t)j * kMapElems);
  }
  __syncthreads();
}

// Every pass of the owner of block j.  The passes of one block run in order;
// the owners of different blocks run their passes concurrently, so pass p+1
// of the factor trails pass p by about one block instead of starting after
// it: the chains of all passes together take about (blocks + passes - 1)
// block chains.
template <int SG, typename ST, bool SPEC16>
__device__ __forceinline__ void owner_item(SbLds& sh, const OwnF<ST>& F, int j, int poll) {
  const int tid = threadIdx.x;
  const int64_t deadline = wall_clock64() + kWaitTicks;
  const int64_t pj = (int64_t)j * kBR;
  const int bbc = F.n - pj < kBR ? (int)(F.n - pj) : kBR;
  if (tid == 0) sh.tmo = 0;
#pragma unroll
  for (int q = 0; q < kTilePerThread; ++q) {
    const int idx = tid + q * kThreads, i = idx >> 6, c = idx & 63;
    sh.Lb[i][c] = (i < bbc && c < bbc && c >= i) ? (double)F.L[(pj + i) * F.ldl + pj + c] : 0.0;
  }
  const int passes = (int)((F.k + kKP - 1) / kKP);
  int nfz = -1;  // far blocks of the odd pass applied by the even pass before it
  for (int p = 0; p < passes; ++p) {
    const bool last = p + 1 == passes;
    if (SPEC16 && F.k - (int64_t)p * kKP >= kKP)
      owner_pass<SG, ST, kKP>(sh, F, j, bbc, p, last, deadline, poll, nfz);
    else
      owner_pass<SG, ST, 0>(sh, F, j, bbc, p, last, deadline, poll, nfz);
  }
}

// Workgroups take owner items from a counter until none are left: item j
// owns the columns of block j.  An item waits only for items with lower
// numbers, which were taken earlier and are running or done, so every wait
// ends (each is still bounded, see kWaitTicks).
template <int SG, typename ST>
__global__ __launch_bounds__(kThreads) void k_sb_queue(OwnF<ST> F, int nitems,
                                                       int32_t* __restrict__ ticket) {
  __shared__ SbLds sh;
  for (;;) {
    if (threadIdx.x == 0)
      sh.tk = __hip_atomic_fetch_add(ticket, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int j = sh.tk;
    __syncthreads();
    if (j >= nitems) break;
    // every owner polls with the short sleep: one factor has at most one
    // owner per CU, and sleeping longer between polls measured slower
    owner_item<SG, ST, true>(sh, F, j, 0);
  }
}

// The owner item (block j, every pass) of one factor of a queued batch.
__device__ __forceinline__ void qbatch_item(SbLds& sh, const BatchFactor& B, int j, int poll) {
  if (B.dtype == kStoreF64) {
    OwnF<double> F;
    F.L = (double*)B.L;
    F.maps = (double*)B.maps;
    F.W = (double*)B.W;
    F.T = (GRec<double>*)B.T;
    F.info = B.info;
    F.stop = B.stop;
    F.n = B.n;
    F.k = B.k;
    F.ldl = B.ldl;
    F.fuse = 0;  // measured: no gain for queued batches
    F.vc = nullptr;
    if (B.sigma > 0) owner_item<1, double, true>(sh, F, j, poll);
    else owner_item<-1, double, true>(sh, F, j, poll);
  } else {
    OwnF<float> F;
    F.L = (float*)B.L;
    F.maps = (double*)B.maps;
    F.W = (float*)B.W;
    F.T = (GRec<float>*)B.T;
    F.info = B.info;
    F.stop = B.stop;
    F.n = B.n;
    F.k = B.k;
    F.ldl = B.ldl;
    F.fuse = 0;
    F.vc = nullptr;
    if (B.sigma > 0) owner_item<1, float, true>(sh, F, j, poll);
    else owner_item<-1, float, true>(sh, F, j, poll);
  }
}

// Batches: the same owner items over many factors, from one counter.  Item
// t of the batch is (factor items[t].f, block items[t].j); the host orders
// the items by block index, longest factor first within a block index, so
// an item waits only for items of its factor with lower numbers.  When a
// factor's last item finishes (its counter of unfinished items reaches
// zero), the factor's L and info word are final; with a done word, that
// workgroup copies the info word there (host-mapped memory) so that the
// host can complete the factor while the batch still runs.
__global__ __launch_bounds__(kThreads) void k_sb_qbatch(const BatchFactor* __restrict__ fac,
                                                        const QItem* __restrict__ items,
                                                        int nitems,
                                                        int32_t* __restrict__ ticket, int poll) {
  __shared__ SbLds sh;
  for (;;) {
    if (threadIdx.x == 0)
      sh.tk = __hip_atomic_fetch_add(ticket, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    __syncthreads();
    const int t = sh.tk;
    __syncthreads();
    if (t >= nitems) break;
    const QItem it = items[t];
    const BatchFactor B = fac[it.f];
    qbatch_item(sh, B, it.j, poll);  // ends with a barrier: every wave's stores are issued
    if (B.done != nullptr) {
      // Once the factor's last item is counted, the host may hand the factor
      // to a batch that runs beside this one.  Every wave waits for its own
      // stores and writes them back device-wide before the count goes down:
      // the barrier above only orders their issue, and one wave's fence does
      // not wait for stores the other waves still have in flight.
      __threadfence();
      __syncthreads();
    }
    if (threadIdx.x == 0 && B.done != nullptr) {
      if (__hip_atomic_fetch_add(B.left, -1, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT) == 1) {
        const int64_t info =
            __hip_atomic_load(B.info, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(B.done, info, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
      }
    }
  }
}

// Preparation of a queued batch (grid (chunks, factors)): W <- V, info and
// stop row reset, the records of every pass emptied; the batch's work
// counter reset by the first workgroup.
__global__ void k_prepare_qbatch(const BatchFactor* __restrict__ fac,
                                 int32_t* __restrict__ ticket) {
  const BatchFactor F = fac[blockIdx.y];
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    *F.info = INT64_MAX;
    *F.stop = INT64_MAX;
    if (blockIdx.y == 0) *ticket = 0;
    const int32_t items = (F.n == 0 || F.k == 0) ? 0 : (int32_t)((F.n + kBR - 1) / kBR);
    *F.left = items;
    // a factor without items is final now
    if (items == 0 && F.done != nullptr)
      __hip_atomic_store(F.done, (int64_t)INT64_MAX, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_SYSTEM);
  }
  const bool f64 = F.dtype == kStoreF64;
  const int64_t words = F.n * F.k * (f64 ? 2 : 1);  // 4-byte words
  const uint32_t* __restrict__ src = (const uint32_t*)F.V;
  uint32_t* __restrict__ dst = (uint32_t*)F.W;
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = i0; i < words; i += stride) dst[i] = src[i];
  // records: 16 per row and pass, 4 words of the storage type each
  const int64_t passes = (F.k + kKP - 1) / kKP;
  const int64_t rwords = F.n * kKP * 4 * passes;
  if (f64) {
    uint64_t* __restrict__ r = (uint64_t*)F.T;
    for (int64_t i = i0; i < rwords; i += stride) r[i] = RecBits<double>::kEmpty;
  } else {
    uint32_t* __restrict__ r = (uint32_t*)F.T;
    for (int64_t i = i0; i < rwords; i += stride) r[i] = RecBits<float>::kEmpty;
  }
  // no block map is built yet
  if (F.maps != nullptr) {
    uint64_t* __restrict__ m = (uint64_t*)F.maps;
    const int64_t mwords = map_words(F.n, F.k);
    for (int64_t i = i0; i < mwords; i += stride) m[i] = kMapEmpty;
  }
}

// Records of one pass start out empty.
template <typename ST>
__global__ void k_owner_clear(GRec<ST>* __restrict__ T, int64_t words,
                              double* __restrict__ maps, int64_t mwords) {
  using U = typename RecBits<ST>::U;
  U* __restrict__ p = reinterpret_cast<U*>(T);
  uint64_t* __restrict__ m = reinterpret_cast<uint64_t*>(maps);
  const int64_t stride = (int64_t)gridDim.x * blockDim.x;
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  for (int64_t i = i0; i < words; i += stride) p[i] = RecBits<ST>::kEmpty;
  for (int64_t i = i0; i < mwords; i += stride) m[i] = kMapEmpty;
}

// ------------------------------------------------------- latency probes
// The two latencies that bound one factor's time: the chain of a 64-row
// block (wave 0's Compute + Apply per step plus the helpers, one barrier per
// step) and the hand-off of a value from one workgroup to another through
// device-scope memory (how an owner learns of the records it waits for).
// Measurement only; nothing here is on the modification path.

// One workgroup runs the chain of `blocks` synthetic 64-row blocks with kc
// columns of V, back to back, everything in LDS (no global traffic), and
// writes out[0] = steady-counter ticks (100 MHz) summed over the chains and
// out[1] = shader-clock cycles summed over the chains.
template <int KCF>
__global__ __launch_bounds__(kThreads) void k_probe_chain(int kc, int blocks,
                                                           int64_t* __restrict__ out) {
  __shared__ SbLds sh;
  const int tid = threadIdx.x;
  // a well-conditioned upper triangle and small V values
  for (int idx = tid; idx < kBR * kBR; idx += kThreads) {
    const int i = idx >> 6, j = idx & 63;
    sh.Lb[i][j] = j < i ? 0.0 : (j == i ? 8.0 + 0.01 * i : 1e-3 * (double)((i + 2 * j) % 11 - 5));
  }
  constexpr int kHbPerThread = kBR * kKP / kThreads;  // 2
  double v0[kHbPerThread];
#pragma unroll
  for (int q = 0; q < kHbPerThread; ++q) {
    const int idx = tid + q * kThreads, m = idx & 15, c = idx >> 4;
    v0[q] = 1e-2 * (double)((3 * c + 5 * m) % 13 - 6);
  }
  int64_t ticks = 0, cyc = 0;
  for (int b = 0; b < blocks; ++b) {
#pragma unroll
    for (int q = 0; q < kHbPerThread; ++q) {
      const int idx = tid + q * kThreads;
      sh.Hb[idx & 15][1][idx >> 4] = v0[q];
    }
    __syncthreads();
    chain_setup(sh, kBR);
    __syncthreads();
    const int64_t w0 = wall_clock64(), c0 = clock64();
    chain_loops<1, double, KCF>(sh, kc, kBR, false, (GRec<double>*)nullptr, 0);
    __syncthreads();
    ticks += wall_clock64() - w0;
    cyc += clock64() - c0;
  }
  if (tid == 0) {
    out[0] = ticks;
    out[1] = cyc;
  }
}

// Workgroups 0 and `peer` pass a counter back and forth `rounds` times
// through device-scope stores and loads of two flag words (zero at launch);
// other workgroups exit at once.  Workgroups are dispatched to the XCDs
// round-robin, so peer = 1 crosses XCDs and peer = 8 stays on one.  Every
// wait is bounded: out[0] = steady-counter ticks for all rounds, out[1] = 1
// if a wait ran out.
__global__ void k_probe_handoff(int rounds, int peer, int32_t* __restrict__ flags,
                                int64_t* __restrict__ out) {
  const int wg = blockIdx.x;
  if ((wg != 0 && wg != peer) || threadIdx.x != 0) return;
  int32_t* mine = flags + (wg == 0 ? 0 : 32);  // separate cache lines
  int32_t* theirs = flags + (wg == 0 ? 32 : 0);
  const int64_t t0 = wall_clock64();
  const int64_t deadline = t0 + 100000000;  // 1 s
  int bad = 0;
  for (int r = 1; r <= rounds && !bad; ++r) {
    if (wg == 0) __hip_atomic_store(mine, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    while (__hip_atomic_load(theirs, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < r) {
      if (wall_clock64() > deadline) {
        bad = 1;
        break;
      }
    }
    if (wg != 0) __hip_atomic_store(mine, r, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  if (wg == 0) {
    out[0] = wall_clock64() - t0;
    out[1] = bad;
  }
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

// Compute units of the current device (cached per device): the owner
// kernels hold one workgroup per CU, so a grid of that many covers the GPU.
int owner_grid_limit() {
  static int cached[64] = {0};
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  if (cached[dev] == 0) {
    int cus = 0;
    if (hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0)
      cus = 256;
    cached[dev] = cus;
  }
  return cached[dev];
}

// One persistent owner launch per modification; tickets[0] is zero before
// it (the preparation launch clears it).  The records of every pass start
// out empty.
template <typename ST>
hipError_t run_sysblk_t(hipStream_t st, ST* L, int64_t n, int64_t ldl, ST* W, int64_t k, int sg,
                        void* Tws, int64_t* info, int64_t* stop, int32_t* tickets,
                        double* maps, double* carry) {
  GRec<ST>* R = reinterpret_cast<GRec<ST>*>(Tws);
  const int64_t nb = (n + kBR - 1) / kBR;
  const int64_t passes = (k + kKP - 1) / kKP;
  const int64_t words = n * kKP * 4 * passes;
  const int64_t mwords = maps ? map_words(n, k) : 0;
  const int64_t cblocks = (words + mwords + 255) / 256;
  const unsigned cgrid = (unsigned)(cblocks < 4096 ? cblocks : 4096);
  hipLaunchKernelGGL(k_owner_clear<ST>, dim3(cgrid), dim3(256), 0, st, R, words, maps, mwords);
  OwnF<ST> F;
  F.L = L;
  F.W = W;
  F.T = R;
  F.maps = maps;
  F.info = info;
  F.stop = stop;
  F.n = n;
  F.k = k;
  F.ldl = ldl;
  const int lim = owner_grid_limit();
  // pass pairs share the far blocks' tiles where owners start late enough
  // to find the later pass's maps published (more blocks than compute
  // units; measured: no gain below); V of the later pass is carried exactly,
  // in the private copy of V (binary64 storage) or in `carry`
  F.vc = sizeof(ST) == sizeof(double) ? nullptr : carry;
  F.fuse = (maps && nb > (int64_t)lim && (sizeof(ST) == sizeof(double) || carry)) ? 1 : 0;
  const unsigned grid = (unsigned)(nb < lim ? nb : lim);
  auto kern = sg > 0 ? k_sb_queue<1, ST> : k_sb_queue<-1, ST>;
  hipLaunchKernelGGL(kern, dim3(grid), dim3(kThreads), 0, st, F, (int)nb, tickets);
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

// A queued batch: the preparation launch and one persistent owner launch of
// `grid` workgroups (0: one per compute unit; never more than the items);
// poll: how long owners far from the chain sleep between polls (0..2).
hipError_t run_sysblk_qbatch(hipStream_t st, const BatchFactor* d_fac, int64_t count,
                             const QItem* d_items, int64_t nitems, int32_t* d_ticket, int grid,
                             int poll) {
  if (count <= 0) return hipSuccess;
  hipLaunchKernelGGL(k_prepare_qbatch, dim3(8, (unsigned)count), dim3(256), 0, st, d_fac,
                     d_ticket);
  if (nitems > 0) {
    int64_t g = grid > 0 ? grid : owner_grid_limit();
    if (g > nitems) g = nitems;
    hipLaunchKernelGGL(k_sb_qbatch, dim3((unsigned)g), dim3(kThreads), 0, st, d_fac, d_items,
                       (int)nitems, d_ticket, poll);
  }
  return hipGetLastError();
}

int compute_units() { return owner_grid_limit(); }

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
                      double sg, Coef* T, int64_t* info, int64_t* stop, int32_t* tickets,
                      double* maps) {
  return run_sysblk_t<double>(st, L, n, ldl, W, k, sg > 0 ? 1 : -1, T, info, stop, tickets, maps,
                              nullptr);
}

// The same schedule with L, V and the records stored in FP32: the rows of a
// block (Compute and the Apply inside the block) run in FP64 from the FP32
// values; the Apply to other blocks' columns runs in FP32 by rotations, in
// FP64 by block maps.
hipError_t run_sysblk_f32(hipStream_t st, float* L, int64_t n, int64_t ldl, float* W, int64_t k,
                          double sg, void* T, int64_t* info, int64_t* stop, int32_t* tickets,
                          double* maps, double* carry) {
  return run_sysblk_t<float>(st, L, n, ldl, W, k, sg > 0 ? 1 : -1, T, info, stop, tickets, maps,
                             carry);
}

// Latency probes (see k_probe_chain, k_probe_handoff): out[0] ns per chain
// step, out[1] ns per 64-row block's chain, out[2] / out[3] ns per one-way
// hand-off across XCDs / within one XCD.  Synchronous on `st`.
hipError_t run_probe_latency(hipStream_t st, int kc, int blocks, int rounds, double* out4,
                             int* timed_out) {
  void* buf = nullptr;
  hipError_t e = hipMalloc(&buf, 4096);
  if (e != hipSuccess) return e;
  int64_t* d_out = (int64_t*)buf;
  int32_t* flags = (int32_t*)((char*)buf + 1024);
  int64_t h[6] = {0, 0, 0, 0, 0, 0};
  *timed_out = 0;
  do {
    // the variant the owner schedule runs: specialised on 16 columns, or generic
    auto kern = kc == kKP ? k_probe_chain<kKP> : k_probe_chain<0>;
    hipLaunchKernelGGL(kern, dim3(1), dim3(kThreads), 0, st, kc, blocks, d_out);
    if ((e = hipGetLastError()) != hipSuccess) break;
    for (int peer : {1, 8}) {
      if ((e = hipMemsetAsync(flags, 0, 512, st)) != hipSuccess) break;
      hipLaunchKernelGGL(k_probe_handoff, dim3(peer + 1), dim3(64), 0, st, rounds, peer, flags,
                         d_out + (peer == 1 ? 2 : 4));
      if ((e = hipGetLastError()) != hipSuccess) break;
    }
    if (e != hipSuccess) break;
    if ((e = hipMemcpyAsync(h, d_out, sizeof(h), hipMemcpyDeviceToHost, st)) != hipSuccess) break;
    e = hipStreamSynchronize(st);
  } while (false);
  hipFree(buf);
  if (e != hipSuccess) return e;
  const int nsteps = kBR + kc - 1;
  out4[0] = 10.0 * (double)h[0] / ((double)blocks * nsteps);
  out4[1] = 10.0 * (double)h[0] / (double)blocks;
  out4[2] = 10.0 * (double)h[2] / (2.0 * rounds);
  out4[3] = 10.0 * (double)h[4] / (2.0 * rounds);
  *timed_out = (h[3] != 0 || h[5] != 0) ? 1 : 0;
  return hipSuccess;
}

}  // namespace chm
