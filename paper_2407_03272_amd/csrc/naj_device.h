// Device code of the gfx950 accelerated-Jacobi solver.
//
// Matrix layout ("sliced rows of 64"): rows are grouped in slices of 64
// consecutive rows, one row per lane of a 64-wide wavefront.  A slice of
// width w (its longest row) stores w columns of 64 entries; entry k of the
// slice's lane l is at slice_ptr[s] + 64*k + l, so every load of a column
// step is one contiguous 256 B (indices) / 512 B (float64 values) access.
// Each row keeps its CSR order, so a lane's running sum adds the products in
// the same order as a row-by-row CSR product.  Padding entries have value 0
// and point at the row itself (always a valid, cache-hot address).
//
// All float arithmetic is compiled without contraction, so every product,
// sum and quotient is a separately rounded IEEE operation.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace naj {

constexpr int kWave = 64;
constexpr int kBlock = 256;
constexpr int kWavesPerBlock = kBlock / kWave;

enum Phase : int { PH_NORMB = 0, PH_ITER = 1, PH_CONFIRM = 2, PH_DONE = 3 };

enum : int { ST_OK = 0, ST_NOT_CONVERGED = 1, ST_EDEVICE = -3, ST_BREAKDOWN = -4 };

constexpr int kRestartLogCap = 64;

// Control block of one solve: written only by the workgroup that arrives
// last at a grid barrier, read by every workgroup after it.
struct Ctrl {
  double alpha;          // alpha_t of the pass about to run
  double beta;           // y = P + beta (P - R) for the pass about to run
  double nb;             // ||b||_2
  double relres;         // residual of the accepted iterate
  int t;                 // iteration index of the pass about to run (1-based)
  int K_re, K, ell;      // restart bookkeeping of Algorithm 2
  int iP, iR, iW;        // buffer roles: P = x^{t-1}, R = x^{t-2}, W receives x^t
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
  int restart_log[kRestartLogCap];
};

struct Barrier {
  unsigned long long count;   // arrivals, monotone over the solve
  unsigned int epoch_done;    // last released barrier epoch
  unsigned int pad;
};

struct Sell {
  const int64_t* slice_ptr;   // [nslices+1]
  const int32_t* col;
  const double* val;
  const float* val32;
  int64_t n;
  int64_t nslices;
};

struct SolveArgs {
  Sell A;
  const double* dinv;         // non-null: caller's diagonal (as 1/D); null: J from the row
  const double* b;
  double* buf0;
  double* buf1;
  double* buf2;
  double* part;               // [3 * G]
  Ctrl* ctrl;
  Barrier* bar;
  double* hist;
  double* trace;
  int hist_cap;
  int trace_cap;
  double tol;
  int max_iter;
  int restart;
  int confirm_gap;
  int nxcd;                   // workgroups are spread round-robin over this many L2 domains
  long long spin_ticks;       // barrier wait limit in wall-clock ticks
};

__device__ __forceinline__ double wave_sum(double v) {
  // xor butterfly: every lane ends with the same value (additions commute)
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) v += __shfl_xor(v, off, 64);
  return v;
}

__device__ __forceinline__ double* pick(const SolveArgs& a, int i) {
  return i == 0 ? a.buf0 : (i == 1 ? a.buf1 : a.buf2);
}

// Slice range owned by one wave: the slices of an L2 domain are contiguous,
// and the domain's waves sweep them together so neighbouring rows are read
// close in time on the same L2.
struct WaveRange {
  int64_t first, end, step;
};

__device__ __forceinline__ WaveRange wave_range(int64_t nslices, int nxcd) {
  const int G = gridDim.x;
  const int w = blockIdx.x;
  const int dom = w % nxcd;
  const int j = w / nxcd;
  const int per_dom = G / nxcd;
  const int64_t lo = nslices * dom / nxcd;
  const int64_t hi = nslices * (dom + 1) / nxcd;
  const int wave = threadIdx.x / kWave;
  WaveRange r;
  r.first = lo + (int64_t)j * kWavesPerBlock + wave;
  r.end = hi;
  r.step = (int64_t)per_dom * kWavesPerBlock;
  return r;
}

// One slice of the fused pass: u = Q y, g = u - b, x = y - J^{-1} g, d = x - P.
template <bool USER_D>
__device__ __forceinline__ void iter_slice(const SolveArgs& a, int64_t s, int lane, const double* __restrict__ P,
                                           const double* __restrict__ R, double* __restrict__ W, double beta,
                                           bool bz, double& ps, double& pgg, double& psabs) {
  const int64_t base = a.A.slice_ptr[s];
  const int width = (int)((a.A.slice_ptr[s + 1] - base) >> 6);
  const int32_t* __restrict__ cp = a.A.col + base + lane;
  const double* __restrict__ vp = a.A.val + base + lane;
  double acc = 0.0, asum = 0.0;
  int k = 0;
  if (bz) {
    for (; k + 4 <= width; k += 4) {
      const int c0 = __builtin_nontemporal_load(cp + (k + 0) * kWave);
      const int c1 = __builtin_nontemporal_load(cp + (k + 1) * kWave);
      const int c2 = __builtin_nontemporal_load(cp + (k + 2) * kWave);
      const int c3 = __builtin_nontemporal_load(cp + (k + 3) * kWave);
      const double v0 = __builtin_nontemporal_load(vp + (k + 0) * kWave);
      const double v1 = __builtin_nontemporal_load(vp + (k + 1) * kWave);
      const double v2 = __builtin_nontemporal_load(vp + (k + 2) * kWave);
      const double v3 = __builtin_nontemporal_load(vp + (k + 3) * kWave);
      const double y0 = P[c0], y1 = P[c1], y2 = P[c2], y3 = P[c3];
      acc = acc + v0 * y0; asum = asum + fabs(v0);
      acc = acc + v1 * y1; asum = asum + fabs(v1);
      acc = acc + v2 * y2; asum = asum + fabs(v2);
      acc = acc + v3 * y3; asum = asum + fabs(v3);
    }
    for (; k < width; ++k) {
      const int c = __builtin_nontemporal_load(cp + k * kWave);
      const double v = __builtin_nontemporal_load(vp + k * kWave);
      acc = acc + v * P[c];
      asum = asum + fabs(v);
    }
  } else {
    for (; k + 4 <= width; k += 4) {
      const int c0 = __builtin_nontemporal_load(cp + (k + 0) * kWave);
      const int c1 = __builtin_nontemporal_load(cp + (k + 1) * kWave);
      const int c2 = __builtin_nontemporal_load(cp + (k + 2) * kWave);
      const int c3 = __builtin_nontemporal_load(cp + (k + 3) * kWave);
      const double v0 = __builtin_nontemporal_load(vp + (k + 0) * kWave);
      const double v1 = __builtin_nontemporal_load(vp + (k + 1) * kWave);
      const double v2 = __builtin_nontemporal_load(vp + (k + 2) * kWave);
      const double v3 = __builtin_nontemporal_load(vp + (k + 3) * kWave);
      const double p0 = P[c0], p1 = P[c1], p2 = P[c2], p3 = P[c3];
      const double r0 = R[c0], r1 = R[c1], r2 = R[c2], r3 = R[c3];
      const double y0 = p0 + beta * (p0 - r0);
      const double y1 = p1 + beta * (p1 - r1);
      const double y2 = p2 + beta * (p2 - r2);
      const double y3 = p3 + beta * (p3 - r3);
      acc = acc + v0 * y0; asum = asum + fabs(v0);
      acc = acc + v1 * y1; asum = asum + fabs(v1);
      acc = acc + v2 * y2; asum = asum + fabs(v2);
      acc = acc + v3 * y3; asum = asum + fabs(v3);
    }
    for (; k < width; ++k) {
      const int c = __builtin_nontemporal_load(cp + k * kWave);
      const double v = __builtin_nontemporal_load(vp + k * kWave);
      const double p = P[c];
      const double y = p + beta * (p - R[c]);
      acc = acc + v * y;
      asum = asum + fabs(v);
    }
  }
  const int64_t row = s * kWave + lane;
  if (row < a.A.n) {
    const double Pi = P[row];
    const double yi = bz ? Pi : Pi + beta * (Pi - R[row]);
    const double g = acc - a.b[row];
    double dv;
    if (USER_D) {
      dv = a.dinv[row];
    } else {
      dv = 1.0 / (asum == 0.0 ? 1.0 : asum);
    }
    const double xi = yi - dv * g;
    W[row] = xi;
    const double d = xi - Pi;
    const double gd = g * d;
    ps = ps + gd;
    pgg = pgg + g * g;
    psabs = psabs + fabs(gd);
  }
}

// One slice of r = b - Q x; accumulates ||r||^2 and optionally stores r.
__device__ __forceinline__ void resid_slice(const Sell& A, int64_t s, int lane, const double* __restrict__ X,
                                            const double* __restrict__ b, double* __restrict__ out, double& prr) {
  const int64_t base = A.slice_ptr[s];
  const int width = (int)((A.slice_ptr[s + 1] - base) >> 6);
  const int32_t* __restrict__ cp = A.col + base + lane;
  const double* __restrict__ vp = A.val + base + lane;
  double acc = 0.0;
  int k = 0;
  for (; k + 4 <= width; k += 4) {
    const int c0 = cp[(k + 0) * kWave], c1 = cp[(k + 1) * kWave], c2 = cp[(k + 2) * kWave], c3 = cp[(k + 3) * kWave];
    const double v0 = vp[(k + 0) * kWave], v1 = vp[(k + 1) * kWave], v2 = vp[(k + 2) * kWave], v3 = vp[(k + 3) * kWave];
    const double x0 = X[c0], x1 = X[c1], x2 = X[c2], x3 = X[c3];
    acc = acc + v0 * x0;
    acc = acc + v1 * x1;
    acc = acc + v2 * x2;
    acc = acc + v3 * x3;
  }
  for (; k < width; ++k) acc = acc + vp[k * kWave] * X[cp[k * kWave]];
  const int64_t row = s * kWave + lane;
  if (row < A.n) {
    const double r = b[row] - acc;
    if (out) out[row] = r;
    prr = prr + r * r;
  }
}

// Sum three per-thread values over the workgroup in a fixed order; result valid in thread 0.
__device__ __forceinline__ void block_sum3(double& a, double& b, double& c, double (*sh)[kWavesPerBlock]) {
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
    for (int i = 1; i < kWavesPerBlock; ++i) {
      a = a + sh[0][i];
      b = b + sh[1][i];
      c = c + sh[2][i];
    }
  }
}

// Sum part[k*G + 0 .. k*G + G-1] in a fixed order with one wavefront.
__device__ __forceinline__ double grid_sum_fixed(const double* part, int k, int G, int lane) {
  double v = 0.0;
  for (int i = lane; i < G; i += kWave) v = v + __hip_atomic_load(part + (size_t)k * G + i, __ATOMIC_RELAXED,
                                                                     __HIP_MEMORY_SCOPE_AGENT);
  return wave_sum(v);
}

}  // namespace naj
