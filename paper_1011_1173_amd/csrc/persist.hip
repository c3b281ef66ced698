// persist.hip -- single-launch streaming schedule of CholeskyModifyB (fast
// evaluation, FP64 storage, k <= 16 columns of V per pass).
//
// The serial dependence of Algorithm 1 runs through the rows: Compute(i, m)
// needs V_i after the Apply of rows 0..i-1, and Compute(i, m) also needs
// L_ii after Compute(i, m-1).  The Compute of row i, column m therefore
// happens at "step" t = i + m of a systolic pipeline whose lane m owns
// column m of V (lanes m >= k idle).  Everything else is arranged around
// that chain:
//
//   * Chain workgroup (block 0, NW = 4 waves in lock step, one barrier per
//     step).  Wave 0 runs Compute(i, m) in lane m at step i + m and passes
//     L_ii^2 and 1/L_ii to lane m+1 (DPP row shift).  A column j is brought
//     up to date by the chain workgroup for its last H rows before it becomes
//     the diagonal: wave w applies rows [j - hi_w, j - lo_w] to column j at
//     step j - 1 + m - w; the partly rotated V_j moves from wave w to wave
//     w-1 through LDS, the partly rotated L_rj moves from lane m to lane m+1
//     within a wave.  Wave 0 applies the newest rows (the newest being the row
//     whose Compute runs in the same step), so V_j is ready for Compute(j, m)
//     at the next step.
//   * Helper waves (all other blocks) own column tiles of 64 columns, one
//     thread per column, and apply to column j every row r < j - H, taking
//     the rotations in diagonal order (all (r, m) with r + m = d at once), so
//     a helper needs only the coefficients the chain has already published.
//     When row j - H - 1 has been applied for column m, the thread stores
//     V_j[m] into a hand-off buffer pre-filled with a sentinel; the chain
//     workgroup waits on the sentinel.
//
// Every Compute and Apply is the same arithmetic as in the fast blocked
// schedule and the rotations reach each element in the same order, so the
// two schedules give identical bits.
#include "rotations.h"

namespace chm {

// A signalling-NaN payload that no arithmetic result can produce.
constexpr uint64_t kSentinelBits = 0x7FF4C0FFEE5A1E57ull;

struct PersistArgs {
  double* L;
  int64_t ldl;
  int64_t n;
  const double* V;   // original V (row stride ldv), columns [m0, m0 + kc)
  int64_t ldv;
  int64_t m0;
  int kc;
  int64_t kfull;     // total columns (for failure indices)
  double sg;
  Coef* Td;          // coefficient table, diagonal-major: row d holds (d - m, m)
  const Coef* Tdr;   // the same memory, read side (helpers)
  int tdp;           // records per diagonal row (multiple of 4: 128-byte rows)
  double* Wh;        // hand-off buffer, n x kb
  int* progress;     // diagonals published by the chain
  int* tile_ctr;     // next helper tile
  int* abort_flag;   // set when a bounded wait gives up; everyone leaves
  int64_t* info;     // failure key
  int ntiles;
};

__device__ __forceinline__ double dpp_shr1(double x) {
  const uint64_t b = __builtin_bit_cast(uint64_t, x);
  int lo = (int)(uint32_t)b, hi = (int)(uint32_t)(b >> 32);
  // row_shr:1 within each row of 16 lanes; lane 0 of a row keeps garbage-free 0
  lo = __builtin_amdgcn_update_dpp(0, lo, 0x111, 0xF, 0xF, false);
  hi = __builtin_amdgcn_update_dpp(0, hi, 0x111, 0xF, 0xF, false);
  return __builtin_bit_cast(double, ((uint64_t)(uint32_t)hi << 32) | (uint32_t)lo);
}

__device__ __forceinline__ double load_dev(const double* p) {
  return __builtin_bit_cast(double, __hip_atomic_load((const uint64_t*)p, __ATOMIC_RELAXED,
                                                      __HIP_MEMORY_SCOPE_AGENT));
}
__device__ __forceinline__ void store_dev(double* p, double v) {
  __hip_atomic_store((uint64_t*)p, __builtin_bit_cast(uint64_t, v), __ATOMIC_RELAXED,
                     __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void store_coef_dev(Coef* p, const Coef& c) {
  store_dev(&p->c, c.c);
  store_dev(&p->s, c.s);
  store_dev(&p->ic, c.ic);
}
// Wait until every outstanding vector memory operation of this wave is done.
__device__ __forceinline__ void wait_vmem() { __builtin_amdgcn_s_waitcnt(0x0F70 & ~0x000F); }

template <int Q0, int Q, int NW>
struct ChainShape {
  static constexpr int H = Q0 + (NW - 1) * Q;  // rows applied by the chain workgroup
  static constexpr int QMAX = Q0 > Q ? Q0 : Q;
  __host__ __device__ static constexpr int nrows(int w) { return w == 0 ? Q0 : Q; }
  // column j gets rows [j - hi(w), j - hi(w) + nrows(w) - 1] from wave w
  __host__ __device__ static constexpr int hi(int w) { return w == 0 ? Q0 : Q0 + w * Q; }
};

constexpr int kRing = 64;  // rows kept in the LDS coefficient ring (>= H + NW + 1)
constexpr int kPublishEvery = 2;
// Bounded waits: a wait that exceeds this many polls (each with a short
// sleep, well over a second in total) records a timeout and every wave of
// the launch leaves; the host reports a runtime error instead of hanging.
constexpr int kSpinLimit = 1 << 21;

__device__ __forceinline__ void raise_abort(const PersistArgs& a) {
  __hip_atomic_store(a.abort_flag, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  atomicMin((unsigned long long*)a.info, (unsigned long long)info_key(0, kCodeTimeout));
}
__device__ __forceinline__ bool aborted(const PersistArgs& a) {
  return __hip_atomic_load(a.abort_flag, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0;
}

template <int KB, int Q0, int Q, int NW>
__device__ void chain_workgroup(const PersistArgs& a) {
  using S = ChainShape<Q0, Q, NW>;
  static_assert(S::H + NW + 1 <= kRing, "ring too small");
  __shared__ Coef ring[kRing][KB];
  __shared__ double wbuf[NW][2][64];
  __shared__ int s_stop;
  // abort request raised during step t, kept in slot t & 1: every wave reads
  // the slot of step t after the barrier that ends step t, and the slot is
  // written again only at step t + 2, after the next barrier
  __shared__ int s_abort[2];

  const int w = threadIdx.x >> 6;
  const int m = threadIdx.x & 63;
  const int kc = a.kc;
  const int64_t n = a.n, ldl = a.ldl;
  const double sg = a.sg;
  const int nr = S::nrows(w);
  const int hiw = S::hi(w);
  if (threadIdx.x == 0) {
    s_stop = (int)n;
    s_abort[0] = 0;
    s_abort[1] = 0;
  }
  __syncthreads();

  double Lf[S::QMAX];  // L_rj as received from lane m-1
#pragma unroll
  for (int q = 0; q < S::QMAX; ++q) Lf[q] = 0.0;
  double tp_in = 1.0, il_in = 1.0, vnext = 0.0;

  const int64_t t_end = n + kc - 2;
  for (int64_t t = 0; t <= t_end; ++t) {
    const int stop = s_stop;
    Coef cur;
    cur.c = 1.0; cur.s = 0.0; cur.ic = 1.0; cur.pad = 0.0;
    double t_out = tp_in, y_out = il_in;
    // ---------------------------------------------------------- Compute
    if (w == 0) {
      const int64_t i = t - m;
      const bool cval = (m < kc) && (i >= 0) && (i < n) && (i < stop);
      double tpi = tp_in, ili = il_in, lin;
      if (m == 0) {
        const double l0 = cval ? a.L[i * ldl + i] : 1.0;
        lin = l0;
        tpi = l0 * l0;
        ili = 1.0 / l0;
      } else {
        lin = tpi * ili;
      }
      const double v = (i == 0 && m < kc) ? a.V[a.m0 + m] : vnext;
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
          if (m == kc - 1) a.L[i * ldl + i] = ww;
        }
      }
      if (code) {
        atomicMin((unsigned long long*)a.info,
                  (unsigned long long)info_key(i * a.kfull + a.m0 + m, code));
        atomicMin(&s_stop, (int)i);
      }
      if (!cval) {
        t_out = tpi;
        y_out = ili;
      }
      if (m < KB) {
        const int64_t slot = (i >= 0 ? i : 0) & (kRing - 1);
        if (m < kc && i >= 0 && i < n) ring[slot][m] = cur;
      }
      if (m < kc) store_coef_dev(a.Td + t * a.tdp + m, cur);
    }
    // ---------------------------------------------------------- catch-up of column j
    const int64_t j = t + 1 - m + w;
    const bool jval = (m < kc) && (j >= 1) && (j < n);
    double Wc = 0.0;
    if (w == NW - 1) {
      if (jval) {
        const double* hp = a.Wh + j * KB + m;
        double x = load_dev(hp);
        int polls = 0;
        while (__builtin_bit_cast(uint64_t, x) == kSentinelBits) {
          if (++polls > kSpinLimit || ((polls & 1023) == 0 && aborted(a))) {
            raise_abort(a);
            s_abort[t & 1] = 1;
            break;
          }
          __builtin_amdgcn_s_sleep(1);
          x = load_dev(hp);
        }
        Wc = x;
      }
    } else if (t == 0) {
      // pipeline fill: every row upstream of wave w is negative for these
      // columns, so the column is still the original V
      Wc = jval ? a.V[j * a.ldv + a.m0 + m] : 0.0;
    } else {
      Wc = wbuf[w + 1][(t - 1) & 1][m];
    }
    double Lo[S::QMAX];
#pragma unroll
    for (int q = 0; q < S::QMAX; ++q) {
      Lo[q] = Lf[q];
      if (q < nr) {
        const int64_t r = j - hiw + q;
        const bool rv = jval && r >= 0 && r < stop;
        Coef cf;
        if (w == 0 && q == nr - 1) cf = cur;
        else cf = ring[(r >= 0 ? r : 0) & (kRing - 1)][m < KB ? m : 0];
        double lin = Lf[q];
        if (m == 0) lin = rv ? a.L[r * ldl + j] : 0.0;
        if (rv) {
          const double x = __builtin_fma(sg * cf.s, Wc, lin) * cf.ic;
          Wc = __builtin_fma(-cf.s, x, cf.c * Wc);
          Lo[q] = x;
          if (m == kc - 1) a.L[r * ldl + j] = x;
        } else {
          Lo[q] = lin;
        }
      }
    }
    if (w > 0) wbuf[w][t & 1][m] = Wc;
    else vnext = Wc;
    // ---------------------------------------------------------- systolic shifts
#pragma unroll
    for (int q = 0; q < S::QMAX; ++q)
      if (q < nr) Lf[q] = dpp_shr1(Lo[q]);
    if (w == 0) {
      tp_in = dpp_shr1(t_out);
      il_in = dpp_shr1(y_out);
    }
    // ---------------------------------------------------------- publish
    if (w == 0 && ((t % kPublishEvery) == kPublishEvery - 1 || t == t_end)) {
      wait_vmem();
      if (m == 0)
        __hip_atomic_store(a.progress, (int)(t + 1), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    if (s_abort[t & 1]) break;  // uniform: every wave reads the same slot
  }
}

template <int KB, int H>
__device__ void helper_wave(const PersistArgs& a) {
  const int lane = threadIdx.x & 63;
  const int kc = a.kc;
  const int64_t n = a.n, ldl = a.ldl;
  const double sg = a.sg;
  const Coef* __restrict__ Td = a.Tdr;
  int seen = 0;
  for (;;) {
    int tile = 0;
    if (lane == 0) tile = atomicAdd(a.tile_ctr, 1);
    tile = __shfl(tile, 0);
    if (tile >= a.ntiles) break;
    const int64_t j = (int64_t)tile * 64 + lane;
    const bool jv = j < n;
    const int64_t e = j - H;  // this thread applies rows [0, e) to column j
    double W[KB];
#pragma unroll
    for (int m = 0; m < KB; ++m) W[m] = (jv && m < kc) ? a.V[j * a.ldv + a.m0 + m] : 0.0;
    if (jv && e <= 0) {
#pragma unroll
      for (int m = 0; m < KB; ++m)
        if (m < kc) store_dev(a.Wh + j * KB + m, W[m]);
    }
    const int64_t jlast = ((int64_t)tile * 64 + 63 < n - 1) ? (int64_t)tile * 64 + 63 : n - 1;
    const int64_t dend = jlast - H - 1 + kc - 1;  // last diagonal with work in this tile
    double Lr[KB];
#pragma unroll
    for (int u = 0; u < KB; ++u) Lr[u] = 0.0;
    for (int64_t d0 = 0; d0 <= dend; d0 += KB) {
#pragma unroll
      for (int u = 0; u < KB; ++u) {
        const int64_t d = d0 + u;
        if (d > dend) break;
        int polls = 0;
        while (seen <= d) {
          seen = __hip_atomic_load(a.progress, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
          if (seen <= d) {
            if (++polls > kSpinLimit || ((polls & 255) == 0 && aborted(a))) {
              raise_abort(a);
              return;
            }
            __builtin_amdgcn_s_sleep(2);
          }
        }
#pragma unroll
        for (int m = 0; m < KB; ++m) {
          if (m >= kc) break;
          const int64_t r = d - m;
          if (r < 0) break;
          const int slot = ((u - m) % KB + KB) % KB;  // r mod KB (d0 is a multiple of KB)
          const bool act = jv && r < e;
          if (m == 0 && act) Lr[slot] = a.L[r * ldl + j];
          const Coef cf = Td[d * a.tdp + m];
          if (act) {
            const double x = __builtin_fma(sg * cf.s, W[m], Lr[slot]) * cf.ic;
            W[m] = __builtin_fma(-cf.s, x, cf.c * W[m]);
            Lr[slot] = x;
            if (m == kc - 1) a.L[r * ldl + j] = x;
            if (r == e - 1) store_dev(a.Wh + j * KB + m, W[m]);
          }
        }
      }
    }
  }
}

template <int KB, int Q0, int Q, int NW>
__global__ __launch_bounds__(256) void k_persist(PersistArgs a) {
  if (blockIdx.x == 0) {
    chain_workgroup<KB, Q0, Q, NW>(a);
  } else {
    helper_wave<KB, ChainShape<Q0, Q, NW>::H>(a);
  }
}

__global__ void k_persist_prepare(double* Wh, int64_t count, int* ctrl) {
  const int64_t i0 = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i0 == 0) {
    ctrl[0] = 0;  // progress
    ctrl[1] = 0;  // tile counter
    ctrl[2] = 0;  // abort
  }
  const double s = __builtin_bit_cast(double, kSentinelBits);
  for (int64_t i = i0; i < count; i += (int64_t)gridDim.x * blockDim.x) Wh[i] = s;
}

// ------------------------------------------------------------------ host side
constexpr int kQ0 = 2, kQ = 5, kNW = 4;
constexpr int kH = ChainShape<kQ0, kQ, kNW>::H;

template <int KB>
static hipError_t launch_persist_kb(hipStream_t st, const PersistArgs& a, int nblocks) {
  void* args[] = {(void*)&a};
  return hipLaunchCooperativeKernel((const void*)k_persist<KB, kQ0, kQ, kNW>, dim3(nblocks),
                                    dim3(256), args, 0, st);
}

static int persist_max_blocks(int kb) {
  static int cache[5] = {0, 0, 0, 0, 0};
  int idx = kb <= 1 ? 0 : kb <= 2 ? 1 : kb <= 4 ? 2 : kb <= 8 ? 3 : 4;
  if (cache[idx]) return cache[idx];
  int dev = 0, cus = 0, per = 0;
  hipGetDevice(&dev);
  hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const void* fn = idx == 0 ? (const void*)k_persist<1, kQ0, kQ, kNW>
                 : idx == 1 ? (const void*)k_persist<2, kQ0, kQ, kNW>
                 : idx == 2 ? (const void*)k_persist<4, kQ0, kQ, kNW>
                 : idx == 3 ? (const void*)k_persist<8, kQ0, kQ, kNW>
                            : (const void*)k_persist<16, kQ0, kQ, kNW>;
  hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, fn, 256, 0);
  cache[idx] = cus * (per > 0 ? per : 1);
  return cache[idx];
}

size_t persist_table_bytes(int64_t n, int64_t k) {
  const int64_t kc = k < 16 ? k : 16;
  const int64_t tdp = ((kc + 3) / 4) * 4;
  return (size_t)((n + kc + 1) * tdp) * sizeof(Coef);
}
size_t persist_handoff_bytes(int64_t n, int64_t k) {
  const int64_t kc = k < 16 ? k : 16;
  const int64_t kb = kc <= 1 ? 1 : kc <= 2 ? 2 : kc <= 4 ? 4 : kc <= 8 ? 8 : 16;
  return (size_t)(n * kb) * sizeof(double);
}

// One pass per 16 columns of V.  ctrl points at two ints (progress, tile counter).
hipError_t run_persist(hipStream_t st, double* L, int64_t n, int64_t ldl, const double* V,
                       int64_t k, double sg, Coef* Td, double* Wh, int* ctrl, int64_t* info) {
  for (int64_t m0 = 0; m0 < k; m0 += 16) {
    const int kc = (int)((k - m0) < 16 ? (k - m0) : 16);
    const int kb = kc <= 1 ? 1 : kc <= 2 ? 2 : kc <= 4 ? 4 : kc <= 8 ? 8 : 16;
    PersistArgs a;
    a.L = L; a.ldl = ldl; a.n = n; a.V = V; a.ldv = k; a.m0 = m0; a.kc = kc; a.kfull = k;
    a.sg = sg; a.Td = Td; a.Tdr = Td; a.tdp = ((kc + 3) / 4) * 4; a.Wh = Wh;
    a.progress = ctrl; a.tile_ctr = ctrl + 1; a.abort_flag = ctrl + 2; a.info = info;
    a.ntiles = (int)((n + 63) / 64);
    const int64_t cnt = n * kb;
    unsigned g = (unsigned)((cnt + 255) / 256);
    if (g < 1) g = 1;
    if (g > 2048) g = 2048;
    hipLaunchKernelGGL(k_persist_prepare, dim3(g), dim3(256), 0, st, Wh, cnt, ctrl);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    const int helpers_needed = (a.ntiles + 3) / 4;
    int nblocks = 1 + helpers_needed;
    const int maxb = persist_max_blocks(kb);
    if (nblocks > maxb) nblocks = maxb;
    if (nblocks < 2) nblocks = 2;
    switch (kb) {
      case 1: e = launch_persist_kb<1>(st, a, nblocks); break;
      case 2: e = launch_persist_kb<2>(st, a, nblocks); break;
      case 4: e = launch_persist_kb<4>(st, a, nblocks); break;
      case 8: e = launch_persist_kb<8>(st, a, nblocks); break;
      default: e = launch_persist_kb<16>(st, a, nblocks); break;
    }
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

}  // namespace chm
