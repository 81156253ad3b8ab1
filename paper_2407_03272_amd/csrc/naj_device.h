// Device code of the gfx950 accelerated-Jacobi solver.
//
// Matrix layout ("sliced rows of 64"): rows are grouped in slices of 64
// consecutive rows, one row per lane of a 64-wide wavefront.  A slice of
// width w (its longest row) stores w columns of 64 entries; entry k of the
// slice's lane l is at slice_ptr[s] + 64*k + l, so every load of a column
// step is one contiguous 256 B (indices) / 512 B (float64 values) access.
// Each row keeps its CSR order, so a lane's running sum adds the products in
// the same order as a row-by-row CSR product.  Padding entries have value 0
// and point at the row itself (always a valid, cache-hot address); in a slice
// of the column-offset form (below) they sit between a row's entries instead,
// at the offsets the row lacks, which adds zeros in the same order.
//
// All float arithmetic is compiled without contraction, so every product,
// sum and quotient is a separately rounded IEEE operation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <type_traits>

#include "naj_partition.h"

namespace naj {

constexpr int kWave = 64;
#ifndef NAJ_UNROLL
#define NAJ_UNROLL 4
#endif
// Column steps whose loads are issued together.  4 measured best on the 128^3
// Laplacian (fewer registers, more resident waves than 8 or 16).
constexpr int kUnroll = NAJ_UNROLL;

// Loads of matrix entries.  Ordinary cached loads measured faster than
// non-temporal ones for passes that fit the MALL; larger float64 passes use
// mat_ld<true> (below).  NAJ_NT_LOADS makes every such load non-temporal.
template <typename T>
__device__ __forceinline__ T stream_load(const T* p) {
#if defined(NAJ_NT_LOADS)
  return __builtin_nontemporal_load(p);
#else
  return *p;
#endif
}

// Matrix loads of the float64 iteration pass: non-temporal (NT) for systems whose pass does not fit the
// 256 MB MALL, so the streamed entries do not evict the gathered vectors; ordinary loads otherwise
// (the whole pass then stays in the MALL from one pass to the next).
template <bool NT, typename T>
__device__ __forceinline__ T mat_ld(const T* p) {
  if constexpr (NT)
    return __builtin_nontemporal_load(p);
  else
    return stream_load(p);
}

// PH_RESID64 and PH_INNER32 belong to the mixed-precision refinement loop.
enum Phase : int { PH_NORMB = 0, PH_ITER = 1, PH_CONFIRM = 2, PH_DONE = 3, PH_RESID64 = 4, PH_INNER32 = 5 };

enum : int { ST_OK = 0, ST_NOT_CONVERGED = 1, ST_EDEVICE = -3, ST_BREAKDOWN = -4, ST_CANCELLED = -5 };

// The scalar control reads the caller's cancel word once every this many passes (a read of host
// memory, kept off all other passes).
constexpr int kCancelEvery = 64;

constexpr int kRestartLogCap = 64;

// Control block of one solve.  The per-pass driver keeps two (by launch parity): workgroup 0 of a
// launch publishes the state it decided, which every workgroup of the next launch reads.  The
// single-workgroup and persistent drivers keep one, updated by one thread between passes.
struct Ctrl {
  double alpha;          // alpha_t of the pass about to run
  double beta;           // y = P + beta (P - R) for the pass about to run
  double nb;             // ||b||_2
  double relres;         // residual of the accepted iterate
  int t;                 // iteration index of the pass about to run (1-based)
  int K_re, K, ell;      // restart bookkeeping of Algorithm 2
  int iP, iR, iW;        // buffer roles: P = x^{t-1}, R = x^{t-2} (or y^t in the materialized form), W receives x^t
  int iYn;               // materialized form: buffer receiving y^{t+1}, -1 = none (beta_next == 0)
  double beta_next;      // materialized form: coefficient of y^{t+1} written by the pass about to run
  int beta_zero;         // beta == 0: y = P, R is not read
  int phase;
  int last_confirm;
  int status;
  int iterations;
  int result;            // buffer holding the answer, -1 = zero vector
  int restarts;
  int confirms;
  int pending_restart;   // restart decision held while a confirmation pass runs
  int hist_len;
  int timeout;           // set by a workgroup whose barrier wait timed out
  int passes;            // matrix passes run so far (including the norm of b)
  // mixed precision: the inner float32 solve reuses t, alpha, beta, K_re, K, ell,
  // iP/iR/iW (float32 buffers) and beta_zero above
  int zp;                // inner pass t = 1: the previous inner iterate is the zero vector
  int iX, iXn;           // float64 buffers: current x, next x (written by an updating residual pass)
  int iD;                // float32 buffer holding the inner result d of the pending update
  int update;            // the next residual pass applies x + d
  int outer;             // float64 residual passes done
  int inner_total;       // inner iterations summed over refinement steps
  int inner_restarts;    // inner restarts summed
  double nr;             // ||fl32(r)||_2 of the current inner right-hand side
  double best_mon;       // inner solve: best monitor value so far (for the stall rule)
  int best_t;            // inner solve: iteration of that value
  int restart_log[kRestartLogCap];
};

struct Barrier {
  unsigned long long count;   // arrivals of the persistent kernel's grid barrier (monotone over a solve)
  unsigned int epoch_done;    // last released barrier epoch
  unsigned int pad;
};

// Arrival counters of the per-pass kernel: one per L2 domain plus one on top,
// each on its own 4 KB page so the domains' atomics go to different channels.
constexpr int kMaxDomains = 8;
constexpr int kCounterStride = 1024;   // unsigned ints (4 KB)
constexpr int kCounterWords = (kMaxDomains + 1) * kCounterStride;

// Matrix in the solver's row order.  Rows [0, n_long) are long rows stored as
// CSR (lrowptr/lcol/lval), one wavefront per row; rows [row0, n) with
// row0 = n_long are stored in 64-row slices, one lane per row.
struct Sell {
  const int64_t* slice_ptr;   // [nslices+1]
  const int32_t* col;
  const double* val;
  const float* val32;
  int64_t n;
  int64_t nslices;
  int64_t row0;               // first row held by the slices (= n_long)
  int64_t n_long;
  const int64_t* dom_bounds;  // [nxcd+1] slice ranges of the L2 domains balanced by stored entries, or null
  const int64_t* lrowptr;     // [n_long+1]
  const int32_t* lcol;
  const int32_t* lrun;        // [n_long] c0 when a long row's columns are c0, c0 + 1, ... in stored order
                              // (a dense run: the passes form them instead of loading lcol), else -1; or null
  const double* lval;
  const float* lval32;
  const int32_t* soff;        // [nslices * kOffRec] column-offset records of the slices, or null
  // Per-wave item lists of the per-pass kernel (balanced on the sorted layout, a blocked slice order on
  // the regular layout), or null: wave w of the launch takes items witem[woff[w] .. woff[w+1]), an item
  // being long row r (< n_long) or slice it - n_long.  Built for one launch shape; null for every other
  // kernel.
  const int32_t* woff;
  const int32_t* witem;
};

// Column-offset form of a slice.  When every row r of a 64-row slice stores its entries at columns
// r + S[0] < r + S[1] < ... (a subsequence of one increasing offset list S common to the slice, as in
// a stencil), entry k of every lane has column r + S[k]: a row without offset S[k] holds an explicit
// zero there (which leaves its sums unchanged), and the slice's width is |S|.  The column indices
// then follow from S and are not loaded.  Record s holds |S| at [0] (0: ordinary slice) and S at
// [1 .. |S|].  The col array is filled either way, so code that loads columns reads the same values.
constexpr int kOffRec = 16;

// The records are written only when the system is created, so they are read through the scalar
// cache (constant address space): one scalar load per offset for the whole wavefront.
#define NAJ_CONST __attribute__((address_space(4)))
using OffPtr = const NAJ_CONST int32_t*;

__device__ __forceinline__ OffPtr slice_offsets(const Sell& A, int64_t s) {
  if (!A.soff) return nullptr;
  const OffPtr r = (OffPtr)(A.soff + s * kOffRec);
  return r[0] ? r + 1 : nullptr;
}

// Column index of column step k of a slice's lane: formed from the slice's offsets (OFF) or loaded.
template <bool OFF, bool NT = false>
__device__ __forceinline__ int slice_col(const int32_t* __restrict__ cp, OffPtr so, int32_t row, int k) {
  if constexpr (OFF)
    return row + so[k];
  else
    return mat_ld<NT>(cp + k * kWave);
}

// Which J a pass applies (template parameter JM of the pass functions):
//  0  J of eq. (J-diag), recomputed from the row's values as its absolute sum;
//  1  the caller's diagonal D (stored as 1/D);
//  2  the block-diagonal J of eq. (J-blkdiag) with blocks of `jblock` consecutive rows
//     (regular layout only), applied through its stored inverse blocks.
constexpr int kJRowSum = 0, kJUser = 1, kJBlock = 2;
constexpr int kMaxJBlock = 8;

struct SolveArgs {
  Sell A;
  const double* dinv;         // non-null: caller's diagonal (as 1/D); null: J from the row
  const double* jinv;         // block J: inverse blocks, row r of a block holding row r of its inverse
  const float* jinv32;        // the same in float32 (inner solves)
  int jblock;                 // block J: rows per block (1, 2, 4 or 8; divides 64)
  int stop_obj;               // 1: stop on the objective gap |f(x) - f*| / (1 + |f*|) (float64 solves)
  double fstar;               // f* of that stop
  double fscale;              // 1 + |f*|
  const double* b;
  double* buf0;
  double* buf1;
  double* buf2;
  double* buf3;               // materialized form: the second y buffer
  double* part;               // [2][G][kPartStride] (the single-launch drivers use the first half)
  Ctrl* ctrl;                 // [2]: the per-pass driver's states after even / odd launches
  Barrier* bar;
  unsigned int* counters;     // [kCounterWords], zero between passes
  double* hist;
  double* trace;
  int hist_cap;
  int trace_cap;
  double tol;
  int max_iter;
  int restart;
  int confirm_gap;
  int k0;
  int nxcd;                   // workgroups are spread round-robin over this many L2 domains
  long long spin_ticks;       // barrier wait limit in wall-clock ticks
  // mixed precision
  int precision;              // 0 float64, 1 float32 inner solve + float64 refinement
  int max_refine;
  int inner_stall;
  double inner_tol;
  float* f0;                  // three float32 inner iterates
  float* f1;
  float* f2;
  float* f3;
  float* r32;                 // float32 right-hand side of the inner solve
  int ymode;                  // materialized momentum form (y written by each pass, one gathered vector)
  int ypar;                   // materialized form in the float32 inner phase: the two y buffers alternate
                              // with the pass count (batches: every right-hand side of a system reads y
                              // from the same buffer in a pass)
  const int* cancel;          // host-visible cancel word of the solve (nonzero: stop), or null
};

// How a pass forms y^t and whether it writes y^{t+1}.
//  two-iterate form: y = P + beta (P - R) at every use (R = x^{t-2}); nothing extra written.
//  materialized form (ym): y^t was written by the previous pass into R (or is P when bz), and this
//  pass writes y^{t+1} = x^t + beta_next (x^t - x^{t-1}) into Yn (when Yn is not null); if the
//  restart test then fires, that y^{t+1} is simply not used.  One gathered vector instead of two.
template <typename T>
struct Momentum {
  const T* R;
  T* Yn;
  T beta;
  T beta_next;
  bool bz;        // y^t = x^{t-1} = P
  bool ym;
};

__device__ __forceinline__ double wave_sum(double v) {
  // xor butterfly: every lane ends with the same value (additions commute)
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ double* pick(const SolveArgs& a, int i) {
  return i == 0 ? a.buf0 : (i == 1 ? a.buf1 : (i == 2 ? a.buf2 : a.buf3));
}

__device__ __forceinline__ float* pickf(const SolveArgs& a, int i) {
  return i == 0 ? a.f0 : (i == 1 ? a.f1 : (i == 2 ? a.f2 : a.f3));
}

__device__ __forceinline__ int wave_id() { return __builtin_amdgcn_readfirstlane(threadIdx.x / kWave); }

using WaveRange = SliceRange;

// z = J^{-1} g on the rows of one slice for the block-diagonal J.  A block's nb rows are nb
// consecutive lanes (nb divides 64 and slices start at multiples of 64), so the lane of row r
// reads the block's g values from its neighbours and adds J^{-1}_{r,k} g_k for k = 0, 1, ...
// in that order.  Entry k of the lane's row of the inverse is at jinv[(s * nb + k) * 64 + lane]
// (one coalesced 64-lane load per k).  Every lane of the wavefront must call this (shuffles);
// lanes past the last row pass g = 0.
template <typename T>
__device__ __forceinline__ T block_apply(const T* __restrict__ jinv, int64_t s, int lane, int nb, T g) {
  const T* __restrict__ jp = jinv + (size_t)s * nb * kWave + lane;
  T jk[kMaxJBlock];
#pragma unroll
  for (int k = 0; k < kMaxJBlock; ++k)
    if (k < nb) jk[k] = jp[k * kWave];
  const int first = lane & ~(nb - 1);
  T z = T(0);
#pragma unroll
  for (int k = 0; k < kMaxJBlock; ++k)
    if (k < nb) {
      const T gk = __shfl(g, first + k, kWave);
      z = (k == 0) ? jk[k] * gk : z + jk[k] * gk;
    }
  return z;
}

template <int BS>
__device__ __forceinline__ WaveRange wave_range(const Sell& A, int nxcd) {
  return slice_range(A.nslices, nxcd, (int)gridDim.x, (int)blockIdx.x, wave_id(), BS / kWave, A.dom_bounds);
}

template <typename T>
__device__ __forceinline__ T abs_of(T v) {
  if constexpr (sizeof(T) == 4)
    return fabsf(v);
  else
    return fabs(v);
}

// One lane's sums over its slice's column steps in the fused pass, in stored order:
// acc = sum_k v_k y_{c_k} and asum = sum_k |v_k|, with y = P + beta (P - R) (two-iterate form),
// y = R (materialized form), y = P (bz) or y = 0 (zy).  OFF: the slice's columns come from its
// offsets.  The two column sources are separate instances so each keeps its own register budget.
template <bool OFF, bool YM, bool NT, typename T, typename V = T>
__device__ __forceinline__ void fused_row_sums(const int32_t* __restrict__ cp, OffPtr so,
                                               int32_t row, const V* __restrict__ vp, int width,
                                               const T* __restrict__ P, const T* __restrict__ R, T beta, bool bz,
                                               bool zy, T& acc, T& asum) {
  for (int k0 = 0; k0 < width; k0 += kUnroll) {
    int c[kUnroll];
    V v[kUnroll];   // stored values (float with the float32 copy of a float64 pass), widened where used
    T y[kUnroll];
#pragma unroll
    for (int j = 0; j < kUnroll; ++j)
      if (k0 + j < width) {
        c[j] = slice_col<OFF, NT>(cp, so, row, k0 + j);
        v[j] = mat_ld<NT>(vp + (k0 + j) * kWave);
      }
    if (zy) {
#pragma unroll
      for (int j = 0; j < kUnroll; ++j) y[j] = T(0);
    } else if (bz) {
#pragma unroll
      for (int j = 0; j < kUnroll; ++j)
        if (k0 + j < width) y[j] = P[c[j]];
    } else if (YM) {
#pragma unroll
      for (int j = 0; j < kUnroll; ++j)
        if (k0 + j < width) y[j] = R[c[j]];
    } else {
      T pj[kUnroll], rj[kUnroll];
#pragma unroll
      for (int j = 0; j < kUnroll; ++j)
        if (k0 + j < width) {
          pj[j] = P[c[j]];
          rj[j] = R[c[j]];
        }
#pragma unroll
      for (int j = 0; j < kUnroll; ++j)
        if (k0 + j < width) y[j] = pj[j] + beta * (pj[j] - rj[j]);
    }
#pragma unroll
    for (int j = 0; j < kUnroll; ++j)
      if (k0 + j < width) {
        const T vj = (T)v[j];
        acc = acc + vj * y[j];
        asum = asum + abs_of(vj);
      }
  }
}

// One lane's sum_k v_k x_{c_k} over its slice (OFF as above); with D, x = X + (double)D at every
// gathered column.
template <bool OFF, typename V = double>
__device__ __forceinline__ double resid_row_sum(const int32_t* __restrict__ cp, OffPtr so,
                                                int32_t row, const V* __restrict__ vp, int width,
                                                const double* __restrict__ X, const float* __restrict__ D) {
  double acc = 0.0;
  for (int k0 = 0; k0 < width; k0 += kUnroll) {
    int c[kUnroll];
    V v[kUnroll];
    double xj[kUnroll];
#pragma unroll
    for (int j = 0; j < kUnroll; ++j)
      if (k0 + j < width) {
        c[j] = slice_col<OFF>(cp, so, row, k0 + j);
        v[j] = stream_load(vp + (k0 + j) * kWave);
      }
    if (D) {
      float dj[kUnroll];
#pragma unroll
      for (int j = 0; j < kUnroll; ++j)
        if (k0 + j < width) {
          xj[j] = X[c[j]];
          dj[j] = D[c[j]];
        }
#pragma unroll
      for (int j = 0; j < kUnroll; ++j)
        if (k0 + j < width) xj[j] = xj[j] + (double)dj[j];
    } else {
#pragma unroll
      for (int j = 0; j < kUnroll; ++j)
        if (k0 + j < width) xj[j] = X[c[j]];
    }
#pragma unroll
    for (int j = 0; j < kUnroll; ++j)
      if (k0 + j < width) acc = acc + (double)v[j] * xj[j];
  }
  return acc;
}

// One slice of the fused pass: u = Q y, g = u - b, x = y - J^{-1} g, d = x - P,
// with y = P + beta (P - R) formed at every gathered column (y = P when bz).
// V32: the values are read from the float32 copy, which holds every value exactly (checked when the
// system is created), and widened to float64 where they are used: the same arithmetic on 4-byte loads.
template <int JM, bool YM, bool NT = false, bool V32 = false>
__device__ __forceinline__ void iter_slice(const SolveArgs& a, int64_t s, int lane, const double* __restrict__ P,
                                           const Momentum<double>& m, double* __restrict__ W, double& ps, double& pgg,
                                           double& psabs) {
  const double* __restrict__ R = m.R;
  const double beta = m.beta;
  const bool bz = m.bz;
  constexpr bool ym = YM;
  const int64_t base = a.A.slice_ptr[s];
  const int width = (int)((a.A.slice_ptr[s + 1] - base) >> 6);
  const int64_t row = a.A.row0 + s * kWave + lane;
  const bool live = row < a.A.n;
  const int64_t rr = live ? row : 0;
  // own-row operands do not depend on the column loop: issue them first
  const double Pi = P[rr];
  const double Ri = bz ? 0.0 : R[rr];
  const double bi = a.b[rr];
  const double di = (JM == 1) ? a.dinv[rr] : 0.0;
  const int32_t* __restrict__ cp = a.A.col + base + lane;
  const OffPtr so = slice_offsets(a.A, s);
  double acc = 0.0, asum = 0.0;
  if constexpr (V32) {
    const float* __restrict__ vp = a.A.val32 + base + lane;
    if (so)
      fused_row_sums<true, YM, NT, double, float>(cp, so, (int32_t)rr, vp, width, P, R, beta, bz, false, acc, asum);
    else
      fused_row_sums<false, YM, NT, double, float>(cp, so, (int32_t)rr, vp, width, P, R, beta, bz, false, acc, asum);
  } else {
    const double* __restrict__ vp = a.A.val + base + lane;
    if (so)
      fused_row_sums<true, YM, NT>(cp, so, (int32_t)rr, vp, width, P, R, beta, bz, false, acc, asum);
    else
      fused_row_sums<false, YM, NT>(cp, so, (int32_t)rr, vp, width, P, R, beta, bz, false, acc, asum);
  }
  double z = 0.0;
  if constexpr (JM == kJBlock) z = block_apply(a.jinv, s, lane, a.jblock, live ? acc - bi : 0.0);
  if (live) {
    const double yi = bz ? Pi : (ym ? Ri : Pi + beta * (Pi - Ri));
    const double g = acc - bi;
    const double dv = (JM == 1) ? di : 1.0 / (asum == 0.0 ? 1.0 : asum);
    const double xi = (JM == kJBlock) ? yi - z : yi - dv * g;
    W[row] = xi;
    const double d = xi - Pi;
    if (YM && m.Yn) m.Yn[row] = xi + m.beta_next * d;
    const double gd = g * d;
    ps = ps + gd;
    // monitor: ||Q y - b||^2, or with the objective stop f(y) = sum_i y_i (u_i / 2 - b_i)
    pgg = pgg + (a.stop_obj ? yi * (0.5 * acc - bi) : g * g);
    psabs = psabs + fabs(gd);
  }
}

// One slice of r = b - Q x; accumulates ||r||^2 (with obj: f(x) = sum_i x_i ((Q x)_i / 2 - b_i))
// and optionally stores r.  V32 as in iter_slice.
template <bool V32 = false>
__device__ __forceinline__ void resid_slice(const Sell& A, int64_t s, int lane, const double* __restrict__ X,
                                            const double* __restrict__ b, double* __restrict__ out, double& prr,
                                            bool obj = false) {
  const int64_t base = A.slice_ptr[s];
  const int width = (int)((A.slice_ptr[s + 1] - base) >> 6);
  const int64_t row = A.row0 + s * kWave + lane;
  const bool live = row < A.n;
  const double bi = b[live ? row : 0];
  const int32_t* __restrict__ cp = A.col + base + lane;
  const OffPtr so = slice_offsets(A, s);
  const int32_t rw = (int32_t)(live ? row : 0);
  double acc;
  if constexpr (V32) {
    const float* __restrict__ vp = A.val32 + base + lane;
    acc = so ? resid_row_sum<true, float>(cp, so, rw, vp, width, X, nullptr)
             : resid_row_sum<false, float>(cp, so, rw, vp, width, X, nullptr);
  } else {
    const double* __restrict__ vp = A.val + base + lane;
    acc = so ? resid_row_sum<true>(cp, so, rw, vp, width, X, nullptr) : resid_row_sum<false>(cp, so, rw, vp, width, X, nullptr);
  }
  if (live) {
    const double r = bi - acc;
    if (out) out[row] = r;
    prr = prr + (obj ? X[row] * (0.5 * acc - bi) : r * r);
  }
}

// One slice of the float32 inner pass (mixed precision): the same step as
// iter_slice on Q d = r32 with float32 values, vectors and row sums; the
// restart inner product and the monitor are accumulated in float64 from
// exactly converted float32 operands.  zp: the previous iterate is zero.
template <int JM, bool YM, bool NT = false>
__device__ __forceinline__ void inner_slice(const SolveArgs& a, int64_t s, int lane, const float* __restrict__ P,
                                            const Momentum<float>& m, float* __restrict__ W, bool zp, double& ps,
                                            double& pgg, double& psabs) {
  const float* __restrict__ R = m.R;
  const float beta = m.beta;
  const bool bz = m.bz;
  constexpr bool ym = YM;
  const int64_t base = a.A.slice_ptr[s];
  const int width = (int)((a.A.slice_ptr[s + 1] - base) >> 6);
  const int64_t row = a.A.row0 + s * kWave + lane;
  const bool live = row < a.A.n;
  const int64_t rr = live ? row : 0;
  const float Pi = zp ? 0.0f : P[rr];
  const float Ri = (zp || bz) ? 0.0f : R[rr];
  const float bi = a.r32[rr];
  const double di = (JM == 1) ? a.dinv[rr] : 0.0;
  const int32_t* __restrict__ cp = a.A.col + base + lane;
  const OffPtr so = slice_offsets(a.A, s);
  const float* __restrict__ vp = a.A.val32 + base + lane;
  float acc = 0.0f, asum = 0.0f;
  if (so)
    fused_row_sums<true, YM, NT>(cp, so, (int32_t)rr, vp, width, P, R, beta, bz, zp, acc, asum);
  else
    fused_row_sums<false, YM, NT>(cp, so, (int32_t)rr, vp, width, P, R, beta, bz, zp, acc, asum);
  float z = 0.0f;
  if constexpr (JM == kJBlock) z = block_apply(a.jinv32, s, lane, a.jblock, live ? acc - bi : 0.0f);
  if (live) {
    const float yi = (zp || bz) ? Pi : (ym ? Ri : Pi + beta * (Pi - Ri));
    const float g = acc - bi;
    const float dv = (JM == 1) ? (float)di : 1.0f / (asum == 0.0f ? 1.0f : asum);
    const float xi = (JM == kJBlock) ? yi - z : yi - dv * g;
    W[row] = xi;
    const float d = xi - Pi;
    if (YM && m.Yn) m.Yn[row] = xi + m.beta_next * d;
    const double g64 = (double)g, d64 = (double)d;
    const double gd = g64 * d64;
    ps = ps + gd;
    pgg = pgg + g64 * g64;
    psabs = psabs + fabs(gd);
  }
}

// One slice of the float64 residual pass of the refinement loop: with D != null
// the iterate is first updated, x_new = X + (double)D (formed at every gathered
// column, stored for the own rows in Xn); then r = b - Q x_new in float64,
// r32 = fl32(r), and ||r||^2, ||r32||^2 are accumulated.  V32 as in iter_slice.
template <bool V32 = false>
__device__ __forceinline__ void resid_mixed_slice(const SolveArgs& a, int64_t s, int lane, const double* __restrict__ X,
                                                  const float* __restrict__ D, double* __restrict__ Xn, double& prr,
                                                  double& pr32) {
  const int64_t base = a.A.slice_ptr[s];
  const int width = (int)((a.A.slice_ptr[s + 1] - base) >> 6);
  const int64_t row = a.A.row0 + s * kWave + lane;
  const bool live = row < a.A.n;
  const int64_t rr = live ? row : 0;
  const double bi = a.b[rr];
  const double xi0 = X[rr];
  const float di0 = D ? D[rr] : 0.0f;
  const int32_t* __restrict__ cp = a.A.col + base + lane;
  const OffPtr so = slice_offsets(a.A, s);
  double acc;
  if constexpr (V32) {
    const float* __restrict__ vp = a.A.val32 + base + lane;
    acc = so ? resid_row_sum<true, float>(cp, so, (int32_t)rr, vp, width, X, D)
             : resid_row_sum<false, float>(cp, so, (int32_t)rr, vp, width, X, D);
  } else {
    const double* __restrict__ vp = a.A.val + base + lane;
    acc = so ? resid_row_sum<true>(cp, so, (int32_t)rr, vp, width, X, D)
             : resid_row_sum<false>(cp, so, (int32_t)rr, vp, width, X, D);
  }
  if (live) {
    if (D) Xn[row] = xi0 + (double)di0;
    const double r = bi - acc;
    const float r32 = (float)r;
    a.r32[row] = r32;
    prr = prr + r * r;
    const double r64 = (double)r32;
    pr32 = pr32 + r64 * r64;
  }
}

// ---------------------------------------------------------------------------
// Long rows: one wavefront per row.  Lane l adds the row's entries l, l+64,
// l+128, ... in turn, then the lanes are combined by the xor butterfly: a fixed
// order (repeatable), though not the row's stored order.
constexpr int kLongUnroll = 4;

__device__ __forceinline__ float wave_sum_f(float v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

// The dense-run start of long row r (see Sell::lrun), or -1.
__device__ __forceinline__ int32_t long_run(const Sell& A, int64_t r) { return A.lrun ? A.lrun[r] : -1; }

// sum_k v_k * y(c_k) and sum_k |v_k| over [s, e); Y maps a column to its (already formed) y value.
// NT: the row's entries are loaded non-temporally (see mat_ld).  RUN: the columns are run + (k - s)
// (a dense run), formed instead of loaded; the products and their order are the same either way.
template <bool RUN, typename T, typename VT, typename YF, bool NT>
__device__ __forceinline__ void long_row_sums_in(const int32_t* __restrict__ col, const VT* __restrict__ val,
                                                 int64_t s, int64_t e, int lane, YF yof, T& acc, T& asum,
                                                 int32_t run) {
  acc = (T)0;
  asum = (T)0;
  for (int64_t k = s + lane; k < e; k += (int64_t)kWave * kLongUnroll) {
    int c[kLongUnroll];
    VT v[kLongUnroll];   // widened where used, so the loads stay in flight together
    T y[kLongUnroll];
#pragma unroll
    for (int q = 0; q < kLongUnroll; ++q)
      if (k + q * kWave < e) {
        if constexpr (RUN) c[q] = run + (int)(k + q * kWave - s);
        else c[q] = mat_ld<NT>(col + k + q * kWave);
        v[q] = mat_ld<NT>(val + k + q * kWave);
      }
#pragma unroll
    for (int q = 0; q < kLongUnroll; ++q)
      if (k + q * kWave < e) y[q] = yof(c[q]);
#pragma unroll
    for (int q = 0; q < kLongUnroll; ++q)
      if (k + q * kWave < e) {
        const T vq = (T)v[q];
        acc = acc + vq * y[q];
        asum = asum + (vq < (T)0 ? -vq : vq);
      }
  }
}

template <typename T, typename VT, typename YF, bool NT = false>
__device__ __forceinline__ void long_row_sums(const int32_t* __restrict__ col, const VT* __restrict__ val, int64_t s,
                                              int64_t e, int lane, YF yof, T& acc, T& asum, int32_t run = -1) {
  if (run >= 0) long_row_sums_in<true, T, VT, YF, NT>(col, val, s, e, lane, yof, acc, asum, run);
  else long_row_sums_in<false, T, VT, YF, NT>(col, val, s, e, lane, yof, acc, asum, run);
}

template <int JM, bool YM, bool NT = false, bool V32 = false>
__device__ __forceinline__ void iter_long(const SolveArgs& a, int64_t r, int lane, const double* __restrict__ P,
                                          const Momentum<double>& m, double* __restrict__ W, double& ps, double& pgg,
                                          double& psabs) {
  const double* __restrict__ R = m.R;
  const double beta = m.beta;
  const bool bz = m.bz;
  constexpr bool ym = YM;
  double acc, asum;
  const int64_t s = a.A.lrowptr[r], e = a.A.lrowptr[r + 1];
  auto fP = [&](int c) { return P[c]; };
  auto fR = [&](int c) { return R[c]; };
  auto fY = [&](int c) { const double p = P[c]; return p + beta * (p - R[c]); };
  using VT = std::conditional_t<V32, float, double>;
  const VT* __restrict__ lv;
  if constexpr (V32)
    lv = a.A.lval32;
  else
    lv = a.A.lval;
  if (bz)
    long_row_sums<double, VT, decltype(fP), NT>(a.A.lcol, lv, s, e, lane, fP, acc, asum, long_run(a.A, r));
  else if (ym)
    long_row_sums<double, VT, decltype(fR), NT>(a.A.lcol, lv, s, e, lane, fR, acc, asum, long_run(a.A, r));
  else
    long_row_sums<double, VT, decltype(fY), NT>(a.A.lcol, lv, s, e, lane, fY, acc, asum, long_run(a.A, r));
  acc = wave_sum(acc);
  asum = wave_sum(asum);
  if (lane == 0) {
    const double Pi = P[r];
    const double yi = bz ? Pi : (ym ? R[r] : Pi + beta * (Pi - R[r]));
    const double g = acc - a.b[r];
    const double dv = (JM == 1) ? a.dinv[r] : 1.0 / (asum == 0.0 ? 1.0 : asum);
    const double xi = yi - dv * g;
    W[r] = xi;
    const double dd = xi - Pi;
    if (YM && m.Yn) m.Yn[r] = xi + m.beta_next * dd;
    const double gd = g * dd;
    ps = ps + gd;
    pgg = pgg + (a.stop_obj ? yi * (0.5 * acc - a.b[r]) : g * g);
    psabs = psabs + fabs(gd);
  }
}

template <bool V32 = false>
__device__ __forceinline__ void resid_long(const Sell& A, int64_t r, int lane, const double* __restrict__ X,
                                           const double* __restrict__ b, double* __restrict__ out, double& prr,
                                           bool obj = false) {
  double acc, asum;
  if constexpr (V32)
    long_row_sums<double>(A.lcol, A.lval32, A.lrowptr[r], A.lrowptr[r + 1], lane, [&](int c) { return X[c]; }, acc,
                          asum, long_run(A, r));
  else
    long_row_sums<double>(A.lcol, A.lval, A.lrowptr[r], A.lrowptr[r + 1], lane, [&](int c) { return X[c]; }, acc, asum,
                          long_run(A, r));
  acc = wave_sum(acc);
  if (lane == 0) {
    const double res = b[r] - acc;
    if (out) out[r] = res;
    prr = prr + (obj ? X[r] * (0.5 * acc - b[r]) : res * res);
  }
}

template <int JM, bool YM, bool NT = false>
__device__ __forceinline__ void inner_long(const SolveArgs& a, int64_t r, int lane, const float* __restrict__ P,
                                           const Momentum<float>& m, float* __restrict__ W, bool zp, double& ps,
                                           double& pgg, double& psabs) {
  const float* __restrict__ R = m.R;
  const float beta = m.beta;
  const bool bz = m.bz;
  constexpr bool ym = YM;
  float acc, asum;
  const int64_t s = a.A.lrowptr[r], e = a.A.lrowptr[r + 1];
  auto f0 = [&](int c) { (void)c; return 0.0f; };
  auto fP = [&](int c) { return P[c]; };
  auto fR = [&](int c) { return R[c]; };
  auto fY = [&](int c) { const float p = P[c]; return p + beta * (p - R[c]); };
  if (zp)
    long_row_sums<float, float, decltype(f0), NT>(a.A.lcol, a.A.lval32, s, e, lane, f0, acc, asum, long_run(a.A, r));
  else if (bz)
    long_row_sums<float, float, decltype(fP), NT>(a.A.lcol, a.A.lval32, s, e, lane, fP, acc, asum, long_run(a.A, r));
  else if (ym)
    long_row_sums<float, float, decltype(fR), NT>(a.A.lcol, a.A.lval32, s, e, lane, fR, acc, asum, long_run(a.A, r));
  else
    long_row_sums<float, float, decltype(fY), NT>(a.A.lcol, a.A.lval32, s, e, lane, fY, acc, asum, long_run(a.A, r));
  acc = wave_sum_f(acc);
  asum = wave_sum_f(asum);
  if (lane == 0) {
    const float Pi = zp ? 0.0f : P[r];
    const float yi = (zp || bz) ? Pi : (ym ? R[r] : Pi + beta * (Pi - R[r]));
    const float g = acc - a.r32[r];
    const float dv = (JM == 1) ? (float)a.dinv[r] : 1.0f / (asum == 0.0f ? 1.0f : asum);
    const float xi = yi - dv * g;
    W[r] = xi;
    const float dd = xi - Pi;
    if (YM && m.Yn) m.Yn[r] = xi + m.beta_next * dd;
    const double g64 = (double)g, d64 = (double)dd;
    const double gd = g64 * d64;
    ps = ps + gd;
    pgg = pgg + g64 * g64;
    psabs = psabs + fabs(gd);
  }
}

template <bool V32 = false>
__device__ __forceinline__ void resid_mixed_long(const SolveArgs& a, int64_t r, int lane, const double* __restrict__ X,
                                                 const float* __restrict__ D, double* __restrict__ Xn, double& prr,
                                                 double& pr32) {
  double acc, asum;
  const int64_t s = a.A.lrowptr[r], e = a.A.lrowptr[r + 1];
  using VT = std::conditional_t<V32, float, double>;
  const VT* __restrict__ lv;
  if constexpr (V32)
    lv = a.A.lval32;
  else
    lv = a.A.lval;
  if (D)
    long_row_sums<double>(a.A.lcol, lv, s, e, lane, [&](int c) { return X[c] + (double)D[c]; }, acc, asum,
                          long_run(a.A, r));
  else
    long_row_sums<double>(a.A.lcol, lv, s, e, lane, [&](int c) { return X[c]; }, acc, asum, long_run(a.A, r));
  acc = wave_sum(acc);
  if (lane == 0) {
    if (D) Xn[r] = X[r] + (double)D[r];
    const double res = a.b[r] - acc;
    const float r32 = (float)res;
    a.r32[r] = r32;
    prr = prr + res * res;
    const double r64 = (double)r32;
    pr32 = pr32 + r64 * r64;
  }
}

// Long rows handed out round-robin over every wave of the grid (heaviest first).
template <int BS>
struct LongRange {
  int64_t first, step;
  __device__ __forceinline__ LongRange() {
    first = (int64_t)blockIdx.x * (BS / kWave) + wave_id();
    step = (int64_t)gridDim.x * (BS / kWave);
  }
};

// Sum three per-thread values over the workgroup in a fixed order; result valid in thread 0.
template <int BS>
__device__ __forceinline__ void block_sum3(double& a, double& b, double& c, double (*sh)[BS / kWave]) {
  constexpr int WPB = BS / kWave;
  a = wave_sum(a);
  b = wave_sum(b);
  c = wave_sum(c);
  const int wave = threadIdx.x / kWave, lane = threadIdx.x % kWave;
  if (lane == 0) {
    sh[0][wave] = a;
    sh[1][wave] = b;
    sh[2][wave] = c;
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    a = sh[0][0];
    b = sh[1][0];
    c = sh[2][0];
    for (int i = 1; i < WPB; ++i) {
      a = a + sh[0][i];
      b = b + sh[1][i];
      c = c + sh[2][i];
    }
  }
}

// Per-workgroup partial sums live at part[4*w + k], k = 0, 1, 2 (32 B per workgroup); the per-pass
// driver keeps two such arrays, for launches of even and odd index.
constexpr int kPartStride = 4;

// Sums of the G workgroups' partials in a fixed order (lane l adds slots l, l+64, ...
// in turn, then the lanes are combined by the xor butterfly); every lane gets
// the result.  Loads are issued four slots at a time before any is used.
__device__ __forceinline__ void grid_sum3(const double* __restrict__ part, int G, int lane, double& r0, double& r1,
                                          double& r2) {
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  int i = lane;
  for (; i + 3 * kWave < G; i += 4 * kWave) {
    double v[4][3];
#pragma unroll
    for (int q = 0; q < 4; ++q)
#pragma unroll
      for (int k = 0; k < 3; ++k) v[q][k] = part[(size_t)(i + q * kWave) * kPartStride + k];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      s0 = s0 + v[q][0];
      s1 = s1 + v[q][1];
      s2 = s2 + v[q][2];
    }
  }
  for (; i < G; i += kWave) {
    const double* p = part + (size_t)i * kPartStride;
    const double a0 = p[0], a1 = p[1], a2 = p[2];
    s0 = s0 + a0;
    s1 = s1 + a1;
    s2 = s2 + a2;
  }
  r0 = wave_sum(s0);
  r1 = wave_sum(s1);
  r2 = wave_sum(s2);
}

}  // namespace naj
