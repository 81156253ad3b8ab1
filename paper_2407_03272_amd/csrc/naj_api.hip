// C ABI of the gfx950 accelerated-Jacobi solver (declared in include/naj.h).
//
// Host side: validates the CSR input on the device, builds the sliced-row
// layout, owns all device memory of a system, and launches the persistent
// solve kernel cooperatively (all workgroups resident, so the grid barrier
// inside it is safe).
#include <hip/hip_runtime.h>

#include <algorithm>
#include <climits>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <string>
#include <vector>

#include "../../include/naj.h"
#include "naj_device.h"
#include "naj_solve.h"
#include "naj_batch.h"
#include "naj_lists.h"
#include <map>
#include <mutex>
#include <queue>
#include <thread>
#include <unordered_map>

using namespace naj;

namespace {

thread_local std::string g_err;

naj_status fail(naj_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof buf, fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

#define HIP_TRY(expr)                                                                        \
  do {                                                                                       \
    hipError_t e_ = (expr);                                                                  \
    if (e_ != hipSuccess) {                                                                  \
      return fail(e_ == hipErrorOutOfMemory ? NAJ_ENOMEM : NAJ_EDEVICE, "%s failed: %s (%s:%d)", #expr, \
                  hipGetErrorString(e_), __FILE__, __LINE__);                                \
    }                                                                                        \
  } while (0)

int env_int(const char* name, int dflt) {
  const char* v = getenv(name);
  if (!v || !*v) return dflt;
  return atoi(v);
}

// ---------------------------------------------------------------------------- setup kernels

__global__ void k_check_rowptr(const int32_t* rowptr, int64_t n, int64_t nnz, int* flag) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    if (rowptr[i] > rowptr[i + 1]) atomicOr(flag, 1);
    if (i == 0 && rowptr[0] != 0) atomicOr(flag, 2);
    if (i == n - 1 && (int64_t)rowptr[n] != nnz) atomicOr(flag, 4);
  }
}

__global__ void k_check_cols(const int32_t* colidx, int64_t nnz, int64_t n, int* flag) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nnz; i += (int64_t)gridDim.x * blockDim.x) {
    const int32_t c = colidx[i];
    if (c < 0 || (int64_t)c >= n) atomicOr(flag, 8);
  }
}

__global__ void k_check_vals(const double* vals, int64_t nnz, int* flag) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < nnz; i += (int64_t)gridDim.x * blockDim.x) {
    if (!(fabs(vals[i]) < __builtin_inf())) atomicOr(flag, 32);
  }
}

// Flags (64) a stored value that its float32 copy does not hold exactly (widening the copy back, as the
// passes that read it do, must give the value itself).
__global__ void k_check_exact32(const double* v, const float* v32, int64_t count, int* flag) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x) {
    if ((double)v32[i] != v[i]) atomicOr(flag, 64);
  }
}

__global__ void k_check_D(const double* D, int64_t n, double* dinv, int* flag) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const double d = D[i];
    if (!(d > 0.0) || !(d < __builtin_inf())) atomicOr(flag, 16);
    dinv[i] = 1.0 / d;
  }
}

// ---------------------------------------------------------------- block-diagonal J, eq. (J-blkdiag)

// Largest eigenvalue of a symmetric NB x NB matrix (overwritten) by the cyclic Jacobi method:
// sweeps of plane rotations over all index pairs, each rotation chosen to zero one
// off-diagonal pair, until the off-diagonal part is below 1e-16 of the diagonal (Golub and
// Van Loan, Matrix Computations, Section 8.5).
template <int NB>
__device__ double sym_max_eig(double (&A)[NB][NB]) {
  for (int sweep = 0; sweep < 40; ++sweep) {
    double off = 0.0, dg = 0.0;
    for (int p = 0; p < NB; ++p) {
      dg = dg + A[p][p] * A[p][p];
      for (int q = p + 1; q < NB; ++q) off = off + A[p][q] * A[p][q];
    }
    if (off <= 1e-32 * dg) break;
    for (int p = 0; p < NB - 1; ++p)
      for (int q = p + 1; q < NB; ++q) {
        const double apq = A[p][q];
        if (apq == 0.0) continue;
        const double tau = (A[q][q] - A[p][p]) / (2.0 * apq);
        const double t = (tau >= 0.0 ? 1.0 : -1.0) / (fabs(tau) + sqrt(1.0 + tau * tau));
        const double c = 1.0 / sqrt(1.0 + t * t);
        const double sn = t * c;
        for (int k = 0; k < NB; ++k) {   // columns p, q of A G
          const double akp = A[k][p], akq = A[k][q];
          A[k][p] = c * akp - sn * akq;
          A[k][q] = sn * akp + c * akq;
        }
        for (int k = 0; k < NB; ++k) {   // rows p, q of G^T (A G)
          const double apk = A[p][k], aqk = A[q][k];
          A[p][k] = c * apk - sn * aqk;
          A[q][k] = sn * apk + c * aqk;
        }
      }
  }
  double m = A[0][0];
  for (int p = 1; p < NB; ++p) m = fmax(m, A[p][p]);
  return m;
}

// One thread per block of NB consecutive rows (block i holds rows NB i .. NB i + NB - 1 below n):
// J^{i,i} = Q^{i,i} + sum_{j != i} ||Q^{i,j}||_2 I (eq. (J-blkdiag)), a zero diagonal entry
// replaced by 1 (as for the diagonal J), identity rows past n; then its inverse by Cholesky,
// stored in the layout block_apply reads, in float64 and float32.  ||Q^{i,j}||_2 is the square
// root of the largest eigenvalue of Q^{i,j}^T Q^{i,j} (a sum of outer products of the block's
// rows restricted to block j), and the coupled blocks j are visited in increasing order.
// Flag 64: a block is not positive definite (so Q is not positive semidefinite).
template <int NB>
__global__ void k_block_jinv(const int32_t* rowptr, const int32_t* colidx, const double* vals, int64_t n,
                             int64_t nblocks, double* jinv, float* jinv32, int* flag) {
  const int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (i >= nblocks) return;
  const int64_t r0 = i * NB;
  const int ni = (int)(n - r0 < NB ? (n - r0 > 0 ? n - r0 : 0) : NB);
  double J[NB][NB];
  for (int p = 0; p < NB; ++p)
    for (int q = 0; q < NB; ++q) J[p][q] = 0.0;
  for (int r = 0; r < ni; ++r)
    for (int e = rowptr[r0 + r]; e < rowptr[r0 + r + 1]; ++e) {
      const int64_t c = colidx[e];
      if (c / NB == i) J[r][c - r0] = J[r][c - r0] + vals[e];
    }
  double shift = 0.0;
  int64_t jprev = -1;
  for (;;) {
    int64_t jn = INT64_MAX;
    for (int r = 0; r < ni; ++r)
      for (int e = rowptr[r0 + r]; e < rowptr[r0 + r + 1]; ++e) {
        const int64_t j = colidx[e] / NB;
        if (j != i && j > jprev && j < jn) jn = j;
      }
    if (jn == INT64_MAX) break;
    double A[NB][NB];
    for (int p = 0; p < NB; ++p)
      for (int q = 0; q < NB; ++q) A[p][q] = 0.0;
    for (int r = 0; r < ni; ++r) {
      double m[NB];
      for (int q = 0; q < NB; ++q) m[q] = 0.0;
      for (int e = rowptr[r0 + r]; e < rowptr[r0 + r + 1]; ++e) {
        const int64_t c = colidx[e];
        if (c / NB == jn) m[c - jn * NB] = m[c - jn * NB] + vals[e];
      }
      for (int p = 0; p < NB; ++p)
        for (int q = 0; q < NB; ++q) A[p][q] = A[p][q] + m[p] * m[q];
    }
    shift = shift + sqrt(sym_max_eig<NB>(A));
    jprev = jn;
  }
  for (int k = 0; k < NB; ++k) {
    if (k < ni) {
      J[k][k] = J[k][k] + shift;
      if (J[k][k] == 0.0) J[k][k] = 1.0;
    } else {
      for (int q = 0; q < NB; ++q) J[k][q] = J[q][k] = 0.0;
      J[k][k] = 1.0;
    }
  }
  bool pd = true;   // Cholesky J = L L^T, L in the lower triangle
  for (int j = 0; j < NB; ++j) {
    double d = J[j][j];
    for (int k = 0; k < j; ++k) d = d - J[j][k] * J[j][k];
    if (!(d > 0.0)) {
      pd = false;
      d = 1.0;
    }
    const double l = sqrt(d);
    J[j][j] = l;
    for (int r = j + 1; r < NB; ++r) {
      double v = J[r][j];
      for (int k = 0; k < j; ++k) v = v - J[r][k] * J[j][k];
      J[r][j] = v / l;
    }
  }
  if (!pd) atomicOr(flag, 64);
  const int64_t sl = r0 / kWave;
  const int lane0 = (int)(r0 % kWave);
  for (int k = 0; k < NB; ++k) {   // column k of the inverse: L y = e_k, then L^T z = y
    double z[NB];
    for (int r = 0; r < NB; ++r) {
      double v = r == k ? 1.0 : 0.0;
      for (int q = 0; q < r; ++q) v = v - J[r][q] * z[q];
      z[r] = v / J[r][r];
    }
    for (int r = NB - 1; r >= 0; --r) {
      double v = z[r];
      for (int q = r + 1; q < NB; ++q) v = v - J[q][r] * z[q];
      z[r] = v / J[r][r];
    }
    for (int r = 0; r < NB; ++r) {
      const size_t at = ((size_t)sl * NB + k) * kWave + lane0 + r;
      jinv[at] = z[r];
      jinv32[at] = (float)z[r];
    }
  }
}

// out[row * nb + k] = entry k of row `row` of the block inverse (caller layout).
__global__ void k_block_jinv_out(const double* jinv, int64_t n, int nb, double* out) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (t >= n * nb) return;
  const int64_t row = t / nb;
  const int k = (int)(t % nb);
  out[t] = jinv[((size_t)(row / kWave) * nb + k) * kWave + row % kWave];
}

// Width of each 64-row slice (rows row0 + 64 s + lane) = its longest row.
__global__ void k_slice_width(const int32_t* rowptr, int64_t row0, int64_t n, int64_t nslices, int32_t* width) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t s = t / kWave;
  const int64_t row = row0 + t;
  int len = row < n ? rowptr[row + 1] - rowptr[row] : 0;
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) len = max(len, __shfl_xor(len, off, 64));
  if ((threadIdx.x % kWave) == 0 && s < nslices) width[s] = len;
}

__device__ __forceinline__ long long wave_min_ll(long long v) {
#pragma unroll
  for (int off = 32; off >= 1; off >>= 1) {
    const long long o = __shfl_xor(v, off, 64);
    v = o < v ? o : v;
  }
  return v;
}

// Dense runs of the long rows: lrun[r] = c0 when row r's columns, in stored order, are c0, c0 + 1, ...,
// else -1.  One wavefront per row (blockDim is a multiple of 64, so r is the same across a wavefront).
__global__ void k_long_runs(const int64_t* lrowptr, const int32_t* lcol, int64_t nlong, int32_t* lrun) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t r = t / kWave;
  if (r >= nlong) return;
  const int lane = (int)(t % kWave);
  const int64_t s = lrowptr[r], e = lrowptr[r + 1];
  const int32_t c0 = lcol[s];   // a long row holds more than 128 entries
  bool run = true;
  for (int64_t k = s + lane; k < e; k += kWave) run = run && (int64_t)lcol[k] - c0 == k - s;
  run = __all(run) != 0;
  if (lane == 0) lrun[r] = run ? c0 : -1;
}

// Column-offset records of the slices of the regular layout (rows 64 s + lane).  One wavefront per
// slice merges its rows' offsets (column - row) into the increasing list S.  The slice qualifies when
// all 64 rows exist, every row's offsets increase strictly (so its entries, in stored order, take
// increasing positions of S), |S| < kOffRec, and row + S[k] lies in [0, n) for every lane and k.
// rec[0] = |S|, or 0 when the slice does not qualify.  Every loop ends: a row's scan is bounded by
// its length, and each merge step either stops or advances the lanes holding the minimum.
__global__ void k_slice_offsets(const int32_t* rowptr, const int32_t* colidx, int64_t n, int64_t nslices,
                                int32_t* soff) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t s = t / kWave;   // the same for the whole wavefront (blockDim is a multiple of 64)
  if (s >= nslices) return;
  const int lane = (int)(t % kWave);
  const int64_t row = s * kWave + lane;
  int32_t* rec = soff + s * kOffRec;
  const bool live = row < n;
  int64_t p = live ? rowptr[row] : 0;
  const int64_t e = live ? rowptr[row + 1] : 0;
  bool mono = true;
  for (int64_t q = p + 1; q < e; ++q) mono = mono && colidx[q] > colidx[q - 1];
  bool good = __all(live && mono) != 0;
  int cnt = 0;
  while (good) {
    const long long cur = p < e ? (long long)colidx[p] - row : LLONG_MAX;
    const long long m = wave_min_ll(cur);
    if (m == LLONG_MAX) break;
    const bool inr = row + m >= 0 && row + m < n;
    if (cnt == kOffRec - 1 || !__all(inr)) {
      good = false;
      break;
    }
    if (lane == 0) rec[1 + cnt] = (int32_t)m;
    ++cnt;
    if (cur == m) ++p;
  }
  if (lane == 0) rec[0] = good ? cnt : 0;
}

// Fills the slices: rows row0 + 64 s + lane.  An ordinary slice stores a row's entries in its first
// positions and pads with zeros pointing at the row itself; a slice in the column-offset form (its
// record's count > 0, regular layout) stores entry k of a row at column row + S[k], taking the row's
// next stored entry when its column matches and an explicit zero otherwise.
__global__ void k_sell_fill(const int32_t* rowptr, const int32_t* colidx, const double* vals, int64_t row0, int64_t n,
                            int64_t nslices, const int64_t* slice_ptr, const int32_t* soff, int32_t* col, double* val,
                            float* val32) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  const int64_t s = t / kWave;
  if (s >= nslices) return;
  const int lane = (int)(t % kWave);
  const int64_t row = row0 + t;
  const int64_t base = slice_ptr[s];
  const int width = (int)((slice_ptr[s + 1] - base) / kWave);
  const int64_t r0 = row < n ? rowptr[row] : 0;
  const int len = row < n ? (int)(rowptr[row + 1] - r0) : 0;
  const int32_t self = row < n ? (int32_t)row : 0;
  const int32_t* rec = soff ? soff + s * kOffRec : nullptr;
  if (rec && rec[0] > 0) {   // every lane of such a slice holds a row (row < n)
    int p = 0;
    for (int k = 0; k < width; ++k) {
      const int64_t dst = base + (int64_t)k * kWave + lane;
      const int32_t c = (int32_t)(row + rec[1 + k]);
      col[dst] = c;
      if (p < len && colidx[r0 + p] == c) {
        const double v = vals[r0 + p];
        val[dst] = v;
        val32[dst] = (float)v;
        ++p;
      } else {
        val[dst] = 0.0;
        val32[dst] = 0.0f;
      }
    }
    return;
  }
  for (int k = 0; k < width; ++k) {
    const int64_t dst = base + (int64_t)k * kWave + lane;
    if (k < len) {
      const double v = vals[r0 + k];
      col[dst] = colidx[r0 + k];
      val[dst] = v;
      val32[dst] = (float)v;
    } else {
      col[dst] = self;
      val[dst] = 0.0;
      val32[dst] = 0.0f;
    }
  }
}

// Symmetric renumbering: new row i is old row perm[i]; its entries keep their
// stored order, with columns renamed through iperm.  One wavefront per row.
__global__ void k_permute_rows(const int32_t* rowptr, const int32_t* colidx, const double* vals, int64_t n,
                               const int32_t* perm, const int32_t* iperm, const int64_t* new_rowptr, int32_t* new_col,
                               double* new_val) {
  const int lane = threadIdx.x % kWave;
  const int64_t w0 = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = (int64_t)gridDim.x * blockDim.x / kWave;
  for (int64_t i = w0; i < n; i += nw) {
    const int32_t o = perm[i];
    const int64_t s = rowptr[o], e = rowptr[o + 1], d = new_rowptr[i];
    for (int64_t k = s + lane; k < e; k += kWave) {
      new_col[d + (k - s)] = iperm[colidx[k]];
      new_val[d + (k - s)] = vals[k];
    }
  }
}

__global__ void k_fill_ones(double* p, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 1.0;
}

__global__ void k_to_float(const double* in, float* out, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = (float)in[i];
}

// out[i] = in[perm[i]] (into the solver's row order)
__global__ void k_gather(const double* in, const int32_t* perm, double* out, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[i] = in[perm[i]];
}

// out[perm[i]] = in[i] (back to the caller's row order)
__global__ void k_scatter(const double* in, const int32_t* perm, double* out, int64_t n) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    out[perm[i]] = in[i];
}

// J of the long rows, summed in the order the solve kernels use.
__global__ void k_long_abs_sum(Sell A, double* out) {
  const int lane = threadIdx.x % kWave;
  const int64_t w0 = (blockIdx.x * (int64_t)blockDim.x + threadIdx.x) / kWave;
  const int64_t nw = (int64_t)gridDim.x * blockDim.x / kWave;
  for (int64_t r = w0; r < A.n_long; r += nw) {
    double acc, asum;
    long_row_sums<double>(A.lcol, A.lval, A.lrowptr[r], A.lrowptr[r + 1], lane, [](int) { return 0.0; }, acc, asum,
                          long_run(A, r));
    asum = wave_sum(asum);
    if (lane == 0) out[r] = asum == 0.0 ? 1.0 : asum;
  }
}

// J of eq. (J-diag) as the row absolute sum in row order (equal for PSD Q), zero rows -> 1.
__global__ void k_row_abs_sum(Sell A, const double* dinv, double* out) {
  const int64_t t = blockIdx.x * (int64_t)blockDim.x + threadIdx.x;
  if (dinv) {
    if (t < A.n) out[t] = 1.0 / dinv[t];
    return;
  }
  const int64_t s = t / kWave;
  const int64_t row = A.row0 + t;
  if (s >= A.nslices || row >= A.n) return;
  const int lane = (int)(t % kWave);
  const int64_t base = A.slice_ptr[s];
  const int width = (int)((A.slice_ptr[s + 1] - base) / kWave);
  double asum = 0.0;
  for (int k = 0; k < width; ++k) asum = asum + fabs(A.val[base + (int64_t)k * kWave + lane]);
  out[row] = asum == 0.0 ? 1.0 : asum;
}

constexpr int kAux = 256;   // block size of the stand-alone one-pass kernels

// One fused pass (stand-alone form of the solve kernel's iteration pass).
template <int JM>
__global__ void __launch_bounds__(kAux) k_step64(SolveArgs a, const double* P, const double* R, double beta,
                                                 int bz, double* W) {
  __shared__ double sh[3][kAux / kWave];
  double p0 = 0.0, p1 = 0.0, p2 = 0.0;
  Momentum<double> m;
  m.R = R;
  m.Yn = nullptr;
  m.beta = beta;
  m.beta_next = 0.0;
  m.bz = bz != 0;
  m.ym = false;
  pass_iter64<JM, kAux, false>(a, P, m, W, p0, p1, p2);
  block_sum3<kAux>(p0, p1, p2, sh);
  if (threadIdx.x == 0) {
    double* slot = a.part + (size_t)blockIdx.x * kPartStride;
    slot[0] = p0;
    slot[1] = p1;
    slot[2] = p2;
  }
}

__global__ void __launch_bounds__(kAux) k_resid64(Sell A, int nxcd, const double* X, const double* b, double* out,
                                                  double* part, int obj) {
  __shared__ double sh[3][kAux / kWave];
  double p0 = 0.0, p1 = 0.0, p2 = 0.0;
  pass_resid64<kAux>(A, nxcd, X, b, out, p0, obj != 0);
  block_sum3<kAux>(p0, p1, p2, sh);
  if (threadIdx.x == 0) {
    double* slot = part + (size_t)blockIdx.x * kPartStride;
    slot[0] = p0;
    slot[1] = 0.0;
    slot[2] = 0.0;
  }
}

// Fixed-order sums of the G workgroups' three partials into out[0..2].
__global__ void k_reduce_fixed(const double* part, int G, double* out) {
  double r0, r1, r2;
  grid_sum3(part, G, threadIdx.x, r0, r1, r2);
  if (threadIdx.x == 0) {
    out[0] = r0;
    out[1] = r1;
    out[2] = r2;
  }
}

// Streaming probes of the attainable HBM rate (naj_bandwidth_probe).  The buffer is cut into blocks of
// 16 KB (256 threads x four 16-byte words), taken by the workgroups in turn (block j, j + grid, ...):
// each thread keeps its four accesses of a block in flight, 4 KB apart, so a workgroup's requests fall
// in one 16 KB region.  This order streamed fastest among those measured on the MI355X: 16 KB blocks
// read at 7.27 TB/s with non-temporal loads (6.53 TB/s plain), where a grid-stride sweep whose thread
// accesses lie a whole grid apart read at 5.3-5.9 TB/s and 4 KB blocks with one access in flight at
// 3.1.  MODE 0 reads src with non-temporal loads (the xor of the words is stored only if it equals a
// constant no real input produces, so the loads stay), 1 copies src to dst (non-temporal loads and
// stores), 2 writes dst.
constexpr int kProbeBlock = 256;
constexpr int kProbeInFlight = 4;
constexpr int kProbeWgPerCu = 3;
typedef unsigned int u32x4 __attribute__((ext_vector_type(4)));

template <int MODE>
__global__ void __launch_bounds__(kProbeBlock) k_bw_probe(const u32x4* __restrict__ src, u32x4* __restrict__ dst,
                                                          int64_t n16) {
  constexpr int64_t kWords = (int64_t)kProbeBlock * kProbeInFlight;   // 16-byte words per block
  const int64_t nblk = (n16 + kWords - 1) / kWords;
  uint32_t acc = 0;
  for (int64_t blk = blockIdx.x; blk < nblk; blk += gridDim.x) {
    const int64_t i0 = blk * kWords + threadIdx.x;
    if (i0 + (kProbeInFlight - 1) * kProbeBlock < n16) {
      if constexpr (MODE == 2) {
#pragma unroll
        for (int q = 0; q < kProbeInFlight; ++q) {
          const uint32_t v = (uint32_t)(i0 + q * kProbeBlock);
          dst[i0 + q * kProbeBlock] = u32x4{v, v + 1u, v + 2u, v + 3u};
        }
      } else {
        u32x4 w[kProbeInFlight];
#pragma unroll
        for (int q = 0; q < kProbeInFlight; ++q) w[q] = __builtin_nontemporal_load(src + i0 + q * kProbeBlock);
#pragma unroll
        for (int q = 0; q < kProbeInFlight; ++q) {
          if constexpr (MODE == 0)
            acc ^= w[q].x ^ w[q].y ^ w[q].z ^ w[q].w;
          else
            __builtin_nontemporal_store(w[q], dst + i0 + q * kProbeBlock);
        }
      }
    } else {   // the last, partial block
      for (int64_t i = i0; i < n16; i += kProbeBlock) {
        if constexpr (MODE == 0) {
          const u32x4 w = src[i];
          acc ^= w.x ^ w.y ^ w.z ^ w.w;
        } else if constexpr (MODE == 1) {
          dst[i] = src[i];
        } else {
          const uint32_t v = (uint32_t)i;
          dst[i] = u32x4{v, v + 1u, v + 2u, v + 3u};
        }
      }
    }
  }
  if constexpr (MODE == 0)
    if (acc == 0x9E3779B9u) dst[0] = u32x4{acc, acc, acc, acc};
}

}  // namespace

// ---------------------------------------------------------------------------- system object

namespace naj {

// First-fit allocation of ranges of [0, size) with a coalescing free list, all on the
// host.  Used for a pool of device memory and for a table of work items.
struct RangeAlloc {
  size_t size = 0;
  size_t in_use = 0;
  std::map<size_t, size_t> free_;            // offset -> length
  std::unordered_map<size_t, size_t> used_;  // offset -> length

  void reset(size_t n) {
    size = n;
    in_use = 0;
    free_.clear();
    used_.clear();
    if (n) free_[0] = n;
  }
  bool alloc(size_t len, size_t* off) {
    for (auto it = free_.begin(); it != free_.end(); ++it) {
      if (it->second < len) continue;
      *off = it->first;
      const size_t rest = it->second - len;
      free_.erase(it);
      if (rest) free_[*off + len] = rest;
      used_[*off] = len;
      in_use += len;
      return true;
    }
    return false;
  }
  void release(size_t off) {
    auto u = used_.find(off);
    if (u == used_.end()) return;
    size_t start = off, len = u->second;
    used_.erase(u);
    in_use -= len;
    auto next = free_.lower_bound(start);
    if (next != free_.end() && next->first == start + len) {   // merge with the following range
      len += next->second;
      next = free_.erase(next);
    }
    if (next != free_.begin()) {                               // and with the preceding one
      auto prev = std::prev(next);
      if (prev->first + prev->second == start) {
        start = prev->first;
        len += prev->second;
        free_.erase(prev);
      }
    }
    free_[start] = len;
  }
  size_t largest_free() const {
    size_t m = 0;
    for (const auto& kv : free_) m = std::max(m, kv.second);
    return m;
  }
};

// A sub-allocator over one device allocation (256-byte granules): allocation and release
// are host bookkeeping only, so they never synchronize the device.  A serving loop draws
// every buffer of its requests from one.
struct Pool {
  static constexpr size_t kAlign = 256;
  char* base = nullptr;
  RangeAlloc ranges;

  hipError_t init(size_t bytes) {
    const size_t n = (bytes + kAlign - 1) / kAlign;
    hipError_t e = hipMalloc((void**)&base, n * kAlign);
    if (e != hipSuccess) {
      base = nullptr;
      return e;
    }
    ranges.reset(n);
    return hipSuccess;
  }
  void* alloc(size_t bytes) {
    size_t off = 0;
    if (!ranges.alloc(std::max<size_t>(1, (bytes + kAlign - 1) / kAlign), &off)) return nullptr;
    return base + off * kAlign;
  }
  void release(void* p) {
    if (p) ranges.release((size_t)((char*)p - base) / kAlign);
  }
  size_t size() const { return ranges.size * kAlign; }
  size_t in_use() const { return ranges.in_use * kAlign; }
  size_t largest_free() const { return ranges.largest_free() * kAlign; }
};

}  // namespace naj

// Scratch of the allocation-free solve (naj_solve_noalloc), for callers that cannot allocate device
// memory: the control block, the grid-barrier words, the arrival counters, the per-workgroup partial
// sums and an 8-double reduction slot of one solve, at fixed offsets in one static array.  Each
// device holds its own copy for the life of the process.  Host code must never pass `scratch`
// itself to a kernel (that is a host-side stand-in): it takes the device address from
// hipGetSymbolAddress once per device (noalloc_scratch) and uses that.
constexpr size_t kNoAllocCtrlOff = 0;       // two control blocks
constexpr size_t kNoAllocBarOff = 1024;
constexpr size_t kNoAllocScalOff = 1280;
constexpr size_t kNoAllocCountersOff = 4096;
constexpr size_t kNoAllocPartOff = kNoAllocCountersOff + sizeof(unsigned int) * kCounterWords;
constexpr int kNoAllocMaxGrid = 4096;   // workgroups whose partial sums fit
constexpr size_t kNoAllocBytes = kNoAllocPartOff + 2 * sizeof(double) * kPartStride * kNoAllocMaxGrid;
constexpr int kNoAllocMaxDevices = 64;
static_assert(2 * sizeof(Ctrl) <= kNoAllocBarOff - kNoAllocCtrlOff, "control blocks exceed their scratch slot");
static_assert(sizeof(Barrier) <= kNoAllocScalOff - kNoAllocBarOff, "barrier exceeds its scratch slot");
static_assert(kNoAllocScalOff + 8 * sizeof(double) <= kNoAllocCountersOff, "reduction slot exceeds its scratch slot");
static_assert(kNoAllocPartOff % 256 == 0, "partial sums must stay 256-byte aligned");

static __device__ __align__(256) unsigned char scratch[kNoAllocBytes];

struct naj_system {
  int device = 0;
  int64_t n = 0, nnz = 0;
  int64_t nslices = 0, stored = 0;
  int64_t* slice_ptr = nullptr;
  int32_t* col = nullptr;
  double* val = nullptr;
  float* val32 = nullptr;
  double* dinv = nullptr;          // caller's D as 1/D (solver row order), or null
  int jblock = 0;                  // > 0: block-diagonal J with blocks of jblock rows (regular layout)
  double* jinv = nullptr;          // its inverse blocks, [nslices * jblock * 64] (see block_apply)
  float* jinv32 = nullptr;
  // row order: with the irregular layout rows are renumbered by decreasing length
  int32_t* perm = nullptr;         // solver row i is caller row perm[i]; null = identity
  double* bperm = nullptr;         // b in solver row order (irregular layout only)
  int64_t n_long = 0;              // rows handled one wavefront per row
  int64_t* lrowptr = nullptr;
  int32_t* lcol = nullptr;
  int32_t* lrun = nullptr;         // [n_long] dense-run starts of the long rows (see Sell::lrun), or null
  int64_t run_nnz = 0;             // nonzeros of the dense-run long rows
  double* lval = nullptr;
  float* lval32 = nullptr;
  int layout = 0;                  // 0 = slices in caller order; 1 = sorted slices + long rows
  int32_t* soff = nullptr;         // column-offset records [nslices * kOffRec] (regular layout), or null
  int64_t off_slices = 0;          // slices stored in the column-offset form
  int64_t reach = 0;               // largest column - row offset of an offset-form slice (regular layout)
  int64_t off_nnz = 0;             // the caller's nonzeros in those slices
  std::vector<int64_t> hslice;     // host copy of slice_ptr (for the domain split)
  std::vector<int64_t> hlong;      // host copy of lrowptr (for the balanced item lists)
  int32_t* woff[2] = {nullptr, nullptr};    // item lists of the per-pass kernel for the float64 and mixed
  int32_t* witem[2] = {nullptr, nullptr};   // launch shapes (build_wave_items, build_blocked_items)
  int wgrid[2] = {0, 0}, wbs[2] = {0, 0};   // the launch shape each list was built for
  int64_t* dom_bounds = nullptr;   // [nxcd+1] device copy of the balanced domain split
  double* vec[4] = {nullptr, nullptr, nullptr, nullptr};   // x buffers; the 4th only in the materialized form
  float* fvec[5] = {nullptr, nullptr, nullptr, nullptr, nullptr};   // mixed: 4 inner iterates + r32 (lazy)
  int ymode = 0;                   // materialized momentum form (irregular layout: one gathered vector)
  int nt = 0;                      // float64 iteration passes load matrix entries non-temporally
  int nt_mx = 0;                   // the same for the float32 inner passes of mixed solves
  int val_exact32 = 0;             // every stored value is exact in float32: the float64 per-pass kernels
                                   // read the float32 copy (4 bytes per entry) and widen it where used
  double* part = nullptr;          // 3 * max_grid
  Ctrl* ctrl = nullptr;
  Barrier* bar = nullptr;
  unsigned int* counters = nullptr;
  double* hist = nullptr;
  int hist_cap_dev = 0;
  double* trace = nullptr;
  int trace_cap_dev = 0;
  double* scal = nullptr;          // small device scratch for reductions
  int max_grid = 0;                // largest grid of any driver (sizes the partial-sum array)
  int aux_grid = 0;                // grid of the stand-alone 256-thread one-pass kernels
  int grid = 0;                    // grid of the solve driver in use
  int grid_mx = 0;                 // grid of the per-pass driver in mixed-precision solves
  int mode = 0;                    // kModePass / kModeSmall / kModePersistent
  int pass_bs = 256;               // block size of the per-pass kernel
  int pass_bs_mx = 512;            // the same in mixed-precision solves
  int nxcd = 1;
  int cus = 0;
  long long spin_ticks = 0;
  int64_t bytes = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  int* hflag = nullptr;            // pinned host words: [0], [1] the phase word of the chunks in flight,
                                   // [2] the cancel word (naj_cancel), read by the solve's scalar control
  Pool* pool = nullptr;            // device memory source (null: the runtime allocator)
  bool lean = false;               // matrix only: no single-solve workspace (batch and server members)
};

namespace {

hipError_t sys_malloc(naj_system* s, void** p, size_t bytes) {
  if (s->pool) {
    *p = s->pool->alloc(bytes);
    return *p ? hipSuccess : hipErrorOutOfMemory;
  }
  return hipMalloc(p, bytes);
}

void sys_free(naj_system* s, void* p) {
  if (!p) return;
  if (s->pool) s->pool->release(p);
  else (void)hipFree(p);
}

template <typename T>
naj_status dev_alloc(naj_system* s, T** p, size_t count) {
  if (count == 0) count = 1;
  hipError_t e = sys_malloc(s, (void**)p, count * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(e == hipErrorOutOfMemory ? NAJ_ENOMEM : NAJ_EDEVICE, "hipMalloc(%zu bytes): %s", count * sizeof(T),
                hipGetErrorString(e));
  }
  s->bytes += (int64_t)(count * sizeof(T));
  return NAJ_OK;
}

void free_system(naj_system* s) {
  if (!s) return;
  for (void* p : {(void*)s->slice_ptr, (void*)s->col, (void*)s->val, (void*)s->val32, (void*)s->dinv, (void*)s->jinv, (void*)s->jinv32, (void*)s->perm,
                  (void*)s->dom_bounds, (void*)s->bperm, (void*)s->lrowptr, (void*)s->lcol, (void*)s->lrun, (void*)s->lval,
                  (void*)s->lval32, (void*)s->part, (void*)s->ctrl, (void*)s->bar, (void*)s->counters, (void*)s->hist,
                  (void*)s->trace, (void*)s->scal, (void*)s->soff, (void*)s->woff[0], (void*)s->witem[0],
                  (void*)s->woff[1], (void*)s->witem[1]})
    sys_free(s, p);
  for (auto& v : s->vec) sys_free(s, v);
  for (auto& v : s->fvec) sys_free(s, v);
  if (s->ev0) (void)hipEventDestroy(s->ev0);
  if (s->ev1) (void)hipEventDestroy(s->ev1);
  if (s->hflag) (void)hipHostFree(s->hflag);
  delete s;
}

int blocks_for(int64_t work, int per_block) {
  int64_t b = (work + per_block - 1) / per_block;
  if (b < 1) b = 1;
  if (b > 65535LL * 16) b = 65535LL * 16;
  return (int)b;
}

constexpr int kModePass = 0, kModeSmall = 1, kModePersistent = 2;
constexpr int64_t kMallBytes = 256ll << 20;   // MI355X Infinity Cache (MALL)
constexpr int kSmallBlock = 1024;

// J of a system: its stored block inverse, the caller's D, or the row sums.
int jm_of(const naj_system* s) { return s->jblock > 0 ? kJBlock : (s->dinv ? kJUser : kJRowSum); }

// Per-pass kernel instances: J mode, block size, momentum form, non-temporal matrix loads and the phases
// of float64 (PS = kPhasesFp64) or mixed-precision (kPhasesMixed) solves.
template <bool YM, int PS, bool V32>
const void* pass_kernel_ym(int jm, int bs) {
  if (bs == 1024)
    return jm ? (const void*)k_pass64<kJUser, 1024, YM, false, PS, V32>
              : (const void*)k_pass64<kJRowSum, 1024, YM, false, PS, V32>;
  if (bs == 512)
    return jm ? (const void*)k_pass64<kJUser, 512, YM, false, PS, V32>
              : (const void*)k_pass64<kJRowSum, 512, YM, false, PS, V32>;
  return jm ? (const void*)k_pass64<kJUser, 256, YM, false, PS, V32> : (const void*)k_pass64<kJRowSum, 256, YM, false, PS, V32>;
}

template <int PS, bool V32>
const void* pass_kernel_ps(int jm, int bs, bool ym, bool nt) {
  if constexpr (V32) {
    if (nt && bs == 512 && !ym)
      return jm ? (const void*)k_pass64<kJUser, 512, false, true, PS, true>
                : (const void*)k_pass64<kJRowSum, 512, false, true, PS, true>;
  }
  if (nt && bs == 256) {
    if (jm == kJBlock) return (const void*)k_pass64<kJBlock, 256, false, true, PS, V32>;
    if (ym)
      return jm ? (const void*)k_pass64<kJUser, 256, true, true, PS, V32>
                : (const void*)k_pass64<kJRowSum, 256, true, true, PS, V32>;
    return jm ? (const void*)k_pass64<kJUser, 256, false, true, PS, V32>
              : (const void*)k_pass64<kJRowSum, 256, false, true, PS, V32>;
  }
  if (jm == kJBlock) {
    if (bs == 1024) return (const void*)k_pass64<kJBlock, 1024, false, false, PS, V32>;
    if (bs == 512) return (const void*)k_pass64<kJBlock, 512, false, false, PS, V32>;
    return (const void*)k_pass64<kJBlock, 256, false, false, PS, V32>;
  }
  return ym ? pass_kernel_ym<true, PS, V32>(jm, bs) : pass_kernel_ym<false, PS, V32>(jm, bs);
}

// A block-J system always uses the regular layout in the two-iterate form.
// nt: the iteration passes load matrix entries non-temporally (instances for the 256-thread pass, and
// for the 512-thread two-iterate pass with 4-byte values; other shapes load them as usual).
// v32: the float64 passes read the float32 copy of the values, which holds every value exactly.
const void* pass_kernel(int jm, int bs, bool ym, bool nt, bool mixed, bool v32) {
  if (v32)
    return mixed ? pass_kernel_ps<kPhasesMixed, true>(jm, bs, ym, nt) : pass_kernel_ps<kPhasesFp64, true>(jm, bs, ym, nt);
  return mixed ? pass_kernel_ps<kPhasesMixed, false>(jm, bs, ym, nt) : pass_kernel_ps<kPhasesFp64, false>(jm, bs, ym, nt);
}

// LDS-resident single-workgroup solve: 32 n bytes of vectors must fit beside the kernel's own LDS.
constexpr int64_t kLdsMaxN = 4800;

const void* solve_lds_kernel(int jm) {
  if (jm == kJBlock) return (const void*)k_solve_lds<kJBlock, kSmallBlock>;
  return jm ? (const void*)k_solve_lds<kJUser, kSmallBlock> : (const void*)k_solve_lds<kJRowSum, kSmallBlock>;
}

const void* solve_kernel(int jm, bool ym) {
  if (jm == kJBlock) return (const void*)k_solve64<kJBlock, kSmallBlock, false>;
  if (ym) return jm ? (const void*)k_solve64<kJUser, kSmallBlock, true> : (const void*)k_solve64<kJRowSum, kSmallBlock, true>;
  return jm ? (const void*)k_solve64<kJUser, kSmallBlock, false> : (const void*)k_solve64<kJRowSum, kSmallBlock, false>;
}

naj_status choose_grid(naj_system* s, hipStream_t st) {
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, s->device));
  s->cus = prop.multiProcessorCount;
  // Contiguous slice ranges per L2 domain keep the gathers of neighbouring rows in one L2.  A
  // sorted layout (rows renumbered by length: power-law graphs) has no such locality to keep,
  // and one global round-robin of slices measured 6 % faster there than balanced domain ranges.
  int nxcd = env_int("NAJ_NXCD", (s->cus % 8 == 0 && s->layout == 0) ? 8 : 1);
  if (nxcd < 1) nxcd = 1;
  if (nxcd > kMaxDomains) nxcd = kMaxDomains;
  s->nxcd = nxcd;
  // 256 threads x 3 per CU measured best for 8-byte values on the 128^3 Laplacian; with 4-byte values
  // (exact in float32) 512 x 3 on regular layouts: 128^3 31.4 against 33.2 us per pass, 160^3 54.0
  // against 72.1 (more waves in flight for the smaller loads, as for the float32 inner pass).  512
  // threads only once their grid is full (a wave per slice or long row at three workgroups per CU):
  // below that, 256-thread workgroups spread the same waves over twice as many workgroups and CUs.
  // Measured, float64 solves/s with 256 / 512 threads: 64x64 301 / 272, 32^3 455 / 407, 64^3 (4096
  // slices) 198 / 195, 96^3 (13,824 slices) 84 / 88; mixed: 324 / 296, 550 / 495, 219 / 208, 88 / 109.
  // A block-J pass (89 VGPRs: five waves per SIMD) cannot hold three 512-thread workgroups per CU.
  const bool full512 = s->nslices + s->n_long >= (int64_t)3 * s->cus * (512 / kWave);
  const int bs_default = (s->val_exact32 && s->layout == 0 && full512 && !s->jblock) ? 512 : 256;
  int bs = env_int("NAJ_BS", bs_default);
  if (bs != 256 && bs != 512 && bs != 1024) bs = bs_default;
  s->pass_bs = bs;
  // three workgroups per CU for 256 threads, and for 512 threads with 4-byte values (the measured
  // shapes above); otherwise 512 x 1 or 1024 x 1
  const int per_cu_default =
      (bs == 256 || (bs == 512 && s->val_exact32 && s->layout == 0 && !s->jblock)) ? 3 : 2 * 256 / bs;
  const int per_cu = std::max(1, env_int("NAJ_WG_PER_CU", per_cu_default));
  int g = per_cu * s->cus;
  // NAJ_GRID: an explicit float64 grid (at most the resident limit of the launch shape), for sweeps
  if (getenv("NAJ_GRID")) g = std::max(1, std::min(env_int("NAJ_GRID", g), g));
  g -= g % nxcd;
  if (g < nxcd) g = nxcd;
  // no more workgroups than give each wave one slice or one long row
  const int wpb = bs / kWave;
  int64_t want = (s->nslices + s->n_long + wpb - 1) / wpb;
  want = ((want + nxcd - 1) / nxcd) * nxcd;
  s->max_grid = (int)std::max<int64_t>(nxcd, std::min<int64_t>(g, want));
  // One workgroup only for small systems.  A single-workgroup pass costs about 3.8 us plus 0.15 us per
  // slice (its waves take the slices in turn); a pass of the per-pass driver costs about 7.3 us up to a
  // few thousand slices (the launch and the decision at the start of every workgroup).  Measured on 2D
  // and 3D Poisson systems (float64 solves/s, one workgroup against one launch per pass): 16x16 1539 /
  // 935, 32x32 586 / 467, 64x64 167 / 291, 16^3 454 / 863, 128x128 31 / 176; the cooperative
  // persistent driver was slower than one of the two at every size.
  const int small_slices = env_int("NAJ_SMALL_SLICES", 24);
  const int force = env_int("NAJ_MODE", -1);
  s->mode = (s->nslices + s->n_long / 4 <= small_slices && s->nnz <= (1 << 21)) ? kModeSmall : kModePass;
  if (force >= 0 && force <= 2) s->mode = force;
  s->grid = s->max_grid;
  if (s->mode == kModeSmall) s->grid = 1;
  {
    // Mixed-precision solves: the float32 inner pass moves 8 instead of 12 bytes per stored entry
    // (4 with the column-offset form) and needs more waves in flight on regular layouts: 512 threads
    // x 3 per CU measured best on the 128^3 Laplacian (25.8 against 35.4 us per pass with the float64
    // shape) and on 160^3 (40.7 against 61.4 us).  The sorted layout's gather-bound pass keeps the
    // float64 shape (Chung-Lu n = 2^22: 728 against 800 us per pass).  Small systems keep 256 threads
    // (the float64 rule above).
    const int bsm_default = (s->layout == 0 && full512) ? 512 : 256;
    int bsm = env_int("NAJ_BS_MIXED", bsm_default);
    if (bsm != 256 && bsm != 512 && bsm != 1024) bsm = bsm_default;
    s->pass_bs_mx = bsm;
    int gm = std::max(1, env_int("NAJ_WG_PER_CU_MIXED", 3)) * s->cus;
    gm -= gm % nxcd;
    if (gm < nxcd) gm = nxcd;
    const int wpbm = bsm / kWave;
    int64_t wantm = (s->nslices + s->n_long + wpbm - 1) / wpbm;
    wantm = ((wantm + nxcd - 1) / nxcd) * nxcd;
    s->grid_mx = (int)std::max<int64_t>(nxcd, std::min<int64_t>(gm, wantm));
    s->max_grid = std::max(s->max_grid, s->grid_mx);
  }
  if (s->mode == kModePersistent) {
    int coop = 0;
    HIP_TRY(hipDeviceGetAttribute(&coop, hipDeviceAttributeCooperativeLaunch, s->device));
    if (!coop) return fail(NAJ_EDEVICE, "device %d does not support cooperative launches", s->device);
    int occ = 0;
    HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, solve_kernel(jm_of(s), s->ymode != 0), kSmallBlock, 0));
    int resident = occ * s->cus;
    resident -= resident % nxcd;
    if (resident < nxcd) return fail(NAJ_EDEVICE, "persistent solve kernel cannot be resident");
    const int wpb1 = kSmallBlock / kWave;
    int64_t w1 = (s->nslices + s->n_long + wpb1 - 1) / wpb1;
    w1 = ((w1 + nxcd - 1) / nxcd) * nxcd;
    s->grid = (int)std::max<int64_t>(nxcd, std::min<int64_t>(resident, w1));
    s->max_grid = std::max(s->max_grid, s->grid);
  }
  {
    int ga = 8 * s->cus;
    ga -= ga % nxcd;
    int64_t wa = (s->nslices + s->n_long + kAux / kWave - 1) / (kAux / kWave);
    wa = ((wa + nxcd - 1) / nxcd) * nxcd;
    s->aux_grid = (int)std::max<int64_t>(nxcd, std::min<int64_t>(std::max(ga, nxcd), wa));
    s->max_grid = std::max(s->max_grid, s->aux_grid);
  }
  if (nxcd > 1 && s->nslices >= nxcd && env_int("NAJ_BALANCE", s->layout == 1 ? 1 : 0)) {
    // L2 domains get contiguous slice ranges of equal weight: stored entries (12 B each in
    // float64) plus the 64 rows' vector traffic (about 4 streams of 8 B per row).  Sorted
    // (irregular) layouts only: regular slices are equal to within a few percent.
    std::vector<int64_t> wpre(s->nslices + 1), bounds(nxcd + 1);
    for (int64_t i = 0; i <= s->nslices; ++i) wpre[i] = s->hslice[i] * 12 / kWave + i * 32;
    balanced_bounds(wpre.data(), s->nslices, nxcd, bounds.data());
    naj_status rc = dev_alloc(s, &s->dom_bounds, (size_t)nxcd + 1);
    if (rc != NAJ_OK) return rc;
    HIP_TRY(hipMemcpyAsync(s->dom_bounds, bounds.data(), sizeof(int64_t) * (nxcd + 1), hipMemcpyHostToDevice, st));
    HIP_TRY(hipStreamSynchronize(st));   // bounds is a local
  }
  int khz = 0;
  HIP_TRY(hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, s->device));
  if (khz <= 0) khz = 100000;
  s->spin_ticks = (long long)khz * 1000LL * (long long)std::max(1, env_int("NAJ_SPIN_SECONDS", 4));
  // a tiny limit makes every barrier wait give up: lets a test force the timeout path from the host
  if (getenv("NAJ_SPIN_TICKS")) s->spin_ticks = std::max(0, env_int("NAJ_SPIN_TICKS", 0));
  return NAJ_OK;
}

naj_status ensure_hist(naj_system* s, int hist_cap, int trace_cap) {
  if (hist_cap > s->hist_cap_dev) {
    sys_free(s, s->hist);
    s->hist = nullptr;
    s->hist_cap_dev = 0;
    naj_status st = dev_alloc(s, &s->hist, (size_t)hist_cap);
    if (st != NAJ_OK) return st;
    s->hist_cap_dev = hist_cap;
  }
  if (trace_cap > s->trace_cap_dev) {
    sys_free(s, s->trace);
    s->trace = nullptr;
    s->trace_cap_dev = 0;
    naj_status st = dev_alloc(s, &s->trace, (size_t)trace_cap * 2);
    if (st != NAJ_OK) return st;
    s->trace_cap_dev = trace_cap;
  }
  return NAJ_OK;
}

Sell sell_of(const naj_system* s) {
  Sell A;
  A.slice_ptr = s->slice_ptr;
  A.col = s->col;
  A.val = s->val;
  A.val32 = s->val32;
  A.n = s->n;
  A.nslices = s->nslices;
  A.row0 = s->n_long;
  A.dom_bounds = s->dom_bounds;
  A.n_long = s->n_long;
  A.lrowptr = s->lrowptr;
  A.lcol = s->lcol;
  A.lrun = s->lrun;
  A.lval = s->lval;
  A.lval32 = s->lval32;
  A.soff = s->soff;
  A.woff = nullptr;
  A.witem = nullptr;
  return A;
}

naj_status check_opts(const naj_opts& o) {
  if (!(o.tol > 0.0) || !std::isfinite(o.tol)) return fail(NAJ_EINVAL, "tol must be finite and > 0 (got %g)", o.tol);
  if (o.max_iter < 1) return fail(NAJ_EINVAL, "max_iter must be >= 1 (got %d)", o.max_iter);
  if (o.k0 < 2) return fail(NAJ_EINVAL, "k0 must be >= 2 (got %d)", o.k0);
  if (o.confirm_gap < 1) return fail(NAJ_EINVAL, "confirm_gap must be >= 1 (got %d)", o.confirm_gap);
  if (o.precision != NAJ_FP64 && o.precision != NAJ_MIXED) return fail(NAJ_EINVAL, "unknown precision %d", o.precision);
  if (o.precision == NAJ_MIXED) {
    if (!(o.inner_tol > 0.0 && o.inner_tol < 1.0)) return fail(NAJ_EINVAL, "inner_tol must be in (0,1)");
    if (o.max_refine < 1) return fail(NAJ_EINVAL, "max_refine must be >= 1");
  }
  if (o.inner_stall < 1) return fail(NAJ_EINVAL, "inner_stall must be >= 1 (got %d)", o.inner_stall);
  if (o.stop != NAJ_STOP_RELRES && o.stop != NAJ_STOP_OBJECTIVE) return fail(NAJ_EINVAL, "unknown stop %d", o.stop);
  if (o.stop == NAJ_STOP_OBJECTIVE) {
    if (o.precision != NAJ_FP64) return fail(NAJ_EINVAL, "the objective-gap stop is a float64 option");
    if (!(std::fabs(o.fstar) < HUGE_VAL)) return fail(NAJ_EINVAL, "fstar must be finite");
  }
  return NAJ_OK;
}

// Per-solve scratch of the single-solve drivers: control block, grid-barrier words, arrival
// counters, per-workgroup partial sums and a small reduction slot.  naj_solve uses the system's
// own (allocated at creation); naj_solve_noalloc points it into the static device array below.
struct SolveScratch {
  Ctrl* ctrl;
  Barrier* bar;
  unsigned int* counters;
  double* part;
  double* scal;
};

SolveScratch own_scratch(naj_system* s) { return SolveScratch{s->ctrl, s->bar, s->counters, s->part, s->scal}; }

// Device address of `scratch` on device `dev` (current), looked up once per device and kept.
std::mutex g_noalloc_mu;
char* g_noalloc_ptr[kNoAllocMaxDevices] = {};

naj_status noalloc_scratch(int dev, SolveScratch* w) {
  if (dev < 0 || dev >= kNoAllocMaxDevices) return fail(NAJ_EINVAL, "device %d out of range", dev);
  char* base = nullptr;
  {
    std::lock_guard<std::mutex> lk(g_noalloc_mu);
    if (!g_noalloc_ptr[dev]) {
      void* p = nullptr;
      const hipError_t e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
      if (e != hipSuccess || !p)
        return fail(NAJ_EDEVICE, "hipGetSymbolAddress(scratch) on device %d: %s", dev, hipGetErrorString(e));
      g_noalloc_ptr[dev] = (char*)p;
    }
    base = g_noalloc_ptr[dev];
  }
  w->ctrl = (Ctrl*)(base + kNoAllocCtrlOff);
  w->bar = (Barrier*)(base + kNoAllocBarOff);
  w->scal = (double*)(base + kNoAllocScalOff);
  w->counters = (unsigned int*)(base + kNoAllocCountersOff);
  w->part = (double*)(base + kNoAllocPartOff);
  return NAJ_OK;
}

SolveArgs make_args(naj_system* s, const double* b, const naj_opts& o, const SolveScratch& w) {
  SolveArgs a;
  a.A = sell_of(s);
  a.dinv = s->dinv;
  a.jinv = s->jinv;
  a.jinv32 = s->jinv32;
  a.jblock = s->jblock;
  a.b = b;
  a.buf0 = s->vec[0];
  a.buf1 = s->vec[1];
  a.buf2 = s->vec[2];
  a.buf3 = s->vec[3];
  a.ymode = s->ymode;
  a.ypar = 0;
  a.part = w.part;
  a.ctrl = w.ctrl;
  a.bar = w.bar;
  a.counters = w.counters;
  a.hist = s->hist;
  a.trace = s->trace;
  a.hist_cap = s->hist_cap_dev;
  a.trace_cap = s->trace_cap_dev;
  a.tol = o.tol;
  a.max_iter = o.max_iter;
  a.restart = o.restart ? 1 : 0;
  a.confirm_gap = o.confirm_gap;
  a.k0 = o.k0;
  a.precision = o.precision == NAJ_MIXED ? 1 : 0;
  a.max_refine = o.max_refine;
  a.inner_stall = o.inner_stall;
  a.inner_tol = o.inner_tol;
  a.stop_obj = o.stop == NAJ_STOP_OBJECTIVE ? 1 : 0;
  a.fstar = o.fstar;
  a.fscale = 1.0 + std::fabs(o.fstar);
  a.f0 = s->fvec[0];
  a.f1 = s->fvec[1];
  a.f2 = s->fvec[2];
  a.f3 = s->fvec[3];
  a.r32 = s->fvec[4];
  a.nxcd = s->nxcd;
  a.spin_ticks = s->spin_ticks;
  a.cancel = s->hflag ? s->hflag + 2 : nullptr;
  return a;
}

// ||b - Q x||^2 into *rr (with obj: f(x) = <x, Q x>/2 - <b, x> instead), fixed-order sums.
naj_status residual_norm2(naj_system* s, const double* x, const double* b, double* out, double* rr,
                          hipStream_t st, bool obj, const SolveScratch& w) {
  const int G = s->aux_grid;
  hipLaunchKernelGGL(k_resid64, dim3(G), dim3(kAux), 0, st, sell_of(s), s->nxcd, x, b, out, w.part, obj ? 1 : 0);
  HIP_TRY(hipGetLastError());
  hipLaunchKernelGGL(k_reduce_fixed, dim3(1), dim3(kWave), 0, st, w.part, G, w.scal);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(rr, w.scal, sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return NAJ_OK;
}



// Rows longer than this go to the one-wavefront-per-row part of the irregular layout.
constexpr int kLongRow = 128;

// Builds the matrix layout from the caller's (validated) device CSR.  Regular
// matrices keep the caller's row order in 64-row slices.  When that would pad
// the slices heavily (rows of very different lengths, e.g. power-law graphs),
// rows are renumbered by decreasing length (a symmetric permutation; each
// row keeps its stored entry order), rows longer than kLongRow are kept as
// CSR for one-wavefront-per-row processing, and the rest go to slices.
naj_status build_layout(naj_system* s, const int32_t* rowptr, const int32_t* colidx, const double* vals,
                        hipStream_t st) {
  const int64_t n = s->n;
  std::vector<int32_t> hrp(n + 1);
  HIP_TRY(hipMemcpyAsync(hrp.data(), rowptr, sizeof(int32_t) * (n + 1), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  int64_t plain_stored = 0;
  int maxlen = 0;
  for (int64_t sl = 0; sl * kWave < n; ++sl) {
    int w = 0;
    for (int64_t r = sl * kWave; r < std::min<int64_t>(n, (sl + 1) * kWave); ++r) w = std::max(w, hrp[r + 1] - hrp[r]);
    plain_stored += (int64_t)w * kWave;
    maxlen = std::max(maxlen, w);
  }
  int layout = plain_stored > (int64_t)(1.3 * (double)std::max<int64_t>(s->nnz, n)) ? 1 : 0;
  // Long rows on average (a dense-row system such as the Section 4.1 matrix): one wavefront per row
  // streams them with all 64 lanes instead of one lane per row over few slices.
  if (s->nnz >= (1 << 20) && s->nnz > (int64_t)kLongRow * n) layout = 1;
  const int forced = env_int("NAJ_LAYOUT", -1);
  if (forced == 0 || forced == 1) layout = forced;
  if (s->jblock) layout = 0;   // a block J's rows must stay consecutive
  s->layout = layout;

  const int32_t* src_rp = rowptr;
  const int32_t* src_col = colidx;
  const double* src_val = vals;
  // Temporaries of the sorted layout, released on every exit (an early error return included, so a
  // failed build inside a server pool gives their memory back).  The stream is drained first: a
  // kernel enqueued before the failure may still read them.
  struct Temps {
    naj_system* s;
    hipStream_t st;
    int64_t* new_rp_d = nullptr;
    int32_t* tmp_col = nullptr;
    double* tmp_val = nullptr;
    int32_t* tmp_rp32 = nullptr;
    int32_t* iperm_d = nullptr;
    double* dtmp = nullptr;
    ~Temps() {
      if (new_rp_d || tmp_col || tmp_val || tmp_rp32 || iperm_d || dtmp) (void)hipStreamSynchronize(st);
      for (void* p : {(void*)new_rp_d, (void*)tmp_col, (void*)tmp_val, (void*)tmp_rp32, (void*)iperm_d, (void*)dtmp})
        sys_free(s, p);
    }
  } tmp{s, st};
  std::vector<int32_t> hrp2;
  naj_status rc = NAJ_OK;
  if (layout == 1) {
    // counting sort by decreasing length (stable)
    std::vector<int64_t> cnt((size_t)maxlen + 2, 0);
    for (int64_t r = 0; r < n; ++r) cnt[(size_t)(maxlen - (hrp[r + 1] - hrp[r]))] += 1;
    int64_t acc = 0;
    for (auto& c : cnt) {
      const int64_t t = c;
      c = acc;
      acc += t;
    }
    std::vector<int32_t> perm(n), iperm(n);
    for (int64_t r = 0; r < n; ++r) {
      const int64_t pos = cnt[(size_t)(maxlen - (hrp[r + 1] - hrp[r]))]++;
      perm[pos] = (int32_t)r;
      iperm[r] = (int32_t)pos;
    }
    std::vector<int64_t> nrp(n + 1);
    nrp[0] = 0;
    int64_t nlong = 0;
    for (int64_t i = 0; i < n; ++i) {
      const int len = hrp[perm[i] + 1] - hrp[perm[i]];
      nrp[i + 1] = nrp[i] + len;
      if (len > kLongRow) nlong = i + 1;
    }
    s->n_long = nlong;
    hrp2.resize(n + 1);
    for (int64_t i = 0; i <= n; ++i) hrp2[i] = (int32_t)nrp[i];
    rc = dev_alloc(s, &s->perm, (size_t)n);
    if (rc != NAJ_OK) return rc;
    HIP_TRY(sys_malloc(s, (void**)&tmp.iperm_d, sizeof(int32_t) * n));
    HIP_TRY(sys_malloc(s, (void**)&tmp.new_rp_d, sizeof(int64_t) * (n + 1)));
    HIP_TRY(sys_malloc(s, (void**)&tmp.tmp_rp32, sizeof(int32_t) * (n + 1)));
    HIP_TRY(sys_malloc(s, (void**)&tmp.tmp_col, sizeof(int32_t) * std::max<int64_t>(1, s->nnz)));
    HIP_TRY(sys_malloc(s, (void**)&tmp.tmp_val, sizeof(double) * std::max<int64_t>(1, s->nnz)));
    HIP_TRY(hipMemcpyAsync(s->perm, perm.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(tmp.iperm_d, iperm.data(), sizeof(int32_t) * n, hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(tmp.new_rp_d, nrp.data(), sizeof(int64_t) * (n + 1), hipMemcpyHostToDevice, st));
    HIP_TRY(hipMemcpyAsync(tmp.tmp_rp32, hrp2.data(), sizeof(int32_t) * (n + 1), hipMemcpyHostToDevice, st));
    hipLaunchKernelGGL(k_permute_rows, dim3(blocks_for(n * kWave, kAux)), dim3(kAux), 0, st, rowptr, colidx, vals, n,
                       s->perm, tmp.iperm_d, tmp.new_rp_d, tmp.tmp_col, tmp.tmp_val);
    HIP_TRY(hipGetLastError());
    if (s->dinv) {   // caller's diagonal into solver order
      HIP_TRY(sys_malloc(s, (void**)&tmp.dtmp, sizeof(double) * n));
      hipLaunchKernelGGL(k_gather, dim3(blocks_for(n, kAux)), dim3(kAux), 0, st, s->dinv, s->perm, tmp.dtmp, n);
      HIP_TRY(hipGetLastError());
      HIP_TRY(hipMemcpyAsync(s->dinv, tmp.dtmp, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    }
    // long rows: the prefix of the renumbered CSR
    const int64_t lnnz = nrp[nlong];
    rc = dev_alloc(s, &s->lrowptr, (size_t)nlong + 1);
    if (rc == NAJ_OK) rc = dev_alloc(s, &s->lcol, (size_t)lnnz);
    if (rc == NAJ_OK) rc = dev_alloc(s, &s->lval, (size_t)lnnz);
    if (rc == NAJ_OK) rc = dev_alloc(s, &s->lval32, (size_t)lnnz);
    if (rc == NAJ_OK) rc = dev_alloc(s, &s->bperm, (size_t)n);
    if (rc != NAJ_OK) return rc;
    HIP_TRY(hipMemcpyAsync(s->lrowptr, nrp.data(), sizeof(int64_t) * (nlong + 1), hipMemcpyHostToDevice, st));
    s->hlong.assign(nrp.begin(), nrp.begin() + nlong + 1);
    if (lnnz > 0) {
      HIP_TRY(hipMemcpyAsync(s->lcol, tmp.tmp_col, sizeof(int32_t) * lnnz, hipMemcpyDeviceToDevice, st));
      HIP_TRY(hipMemcpyAsync(s->lval, tmp.tmp_val, sizeof(double) * lnnz, hipMemcpyDeviceToDevice, st));
      hipLaunchKernelGGL(k_to_float, dim3(blocks_for(lnnz, kAux)), dim3(kAux), 0, st, s->lval, s->lval32, lnnz);
      HIP_TRY(hipGetLastError());
      if (nlong > 0 && env_int("NAJ_LONG_RUNS", 1)) {
        rc = dev_alloc(s, &s->lrun, (size_t)nlong);
        if (rc != NAJ_OK) return rc;
        hipLaunchKernelGGL(k_long_runs, dim3(blocks_for(nlong * kWave, kAux)), dim3(kAux), 0, st, s->lrowptr, s->lcol,
                           nlong, s->lrun);
        HIP_TRY(hipGetLastError());
        std::vector<int32_t> hrun((size_t)nlong);
        HIP_TRY(hipMemcpyAsync(hrun.data(), s->lrun, sizeof(int32_t) * nlong, hipMemcpyDeviceToHost, st));
        HIP_TRY(hipStreamSynchronize(st));
        for (int64_t r = 0; r < nlong; ++r)
          if (hrun[(size_t)r] >= 0) s->run_nnz += nrp[r + 1] - nrp[r];
      }
    }
    src_rp = tmp.tmp_rp32;
    src_col = tmp.tmp_col;
    src_val = tmp.tmp_val;
  }
  // slices over rows [n_long, n)
  const int64_t row0 = s->n_long;
  s->nslices = (n - row0 + kWave - 1) / kWave;
  const std::vector<int32_t>& rp = layout == 1 ? hrp2 : hrp;
  // column-offset records (regular layout): a slice takes the offset form when it qualifies and its
  // offset list is no longer than its longest row, so the layout stores no more entries than without
  // the form (the batch passes, which load every column index, read the same bytes either way)
  std::vector<int32_t> hsoff;
  if (layout == 0 && s->nslices > 0 && env_int("NAJ_OFFSETS", 1)) {
    rc = dev_alloc(s, &s->soff, (size_t)s->nslices * kOffRec);
    if (rc != NAJ_OK) return rc;
    hipLaunchKernelGGL(k_slice_offsets, dim3(blocks_for(s->nslices * kWave, kAux)), dim3(kAux), 0, st, rowptr, colidx,
                       n, s->nslices, s->soff);
    HIP_TRY(hipGetLastError());
    hsoff.resize((size_t)s->nslices * kOffRec);
    HIP_TRY(hipMemcpyAsync(hsoff.data(), s->soff, sizeof(int32_t) * hsoff.size(), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipStreamSynchronize(st));
  }
  s->off_slices = 0;
  s->off_nnz = 0;
  std::vector<int64_t> hp(s->nslices + 1);
  hp[0] = 0;
  for (int64_t sl = 0; sl < s->nslices; ++sl) {
    int w = 0;
    const int64_t ra = row0 + sl * kWave, rb = std::min<int64_t>(n, row0 + (sl + 1) * kWave);
    for (int64_t r = ra; r < rb; ++r) w = std::max(w, rp[r + 1] - rp[r]);
    if (!hsoff.empty()) {
      int32_t& cnt = hsoff[(size_t)sl * kOffRec];
      if (cnt > 0 && cnt <= w) {
        w = cnt;
        s->off_slices += 1;
        s->reach = std::max<int64_t>(s->reach, hsoff[(size_t)sl * kOffRec + cnt]);
        s->off_nnz += (int64_t)rp[rb] - rp[ra];
      } else {
        cnt = 0;
      }
    }
    hp[sl + 1] = hp[sl] + (int64_t)w * kWave;
  }
  if (!hsoff.empty()) {
    if (s->off_slices == 0) {
      sys_free(s, s->soff);
      s->soff = nullptr;
      s->bytes -= (int64_t)(hsoff.size() * sizeof(int32_t));
    } else {
      HIP_TRY(hipMemcpyAsync(s->soff, hsoff.data(), sizeof(int32_t) * hsoff.size(), hipMemcpyHostToDevice, st));
    }
  }
  s->stored = hp[s->nslices] + (layout == 1 ? (int64_t)rp[row0] : 0);
  rc = dev_alloc(s, &s->slice_ptr, (size_t)s->nslices + 1);
  if (rc == NAJ_OK) rc = dev_alloc(s, &s->col, (size_t)hp[s->nslices]);
  if (rc == NAJ_OK) rc = dev_alloc(s, &s->val, (size_t)hp[s->nslices]);
  if (rc == NAJ_OK) rc = dev_alloc(s, &s->val32, (size_t)hp[s->nslices]);
  if (rc != NAJ_OK) return rc;
  HIP_TRY(hipMemcpyAsync(s->slice_ptr, hp.data(), sizeof(int64_t) * (s->nslices + 1), hipMemcpyHostToDevice, st));
  s->hslice = hp;
  if (s->nslices > 0) {
    hipLaunchKernelGGL(k_sell_fill, dim3(blocks_for(s->nslices * kWave, kAux)), dim3(kAux), 0, st, src_rp, src_col,
                       src_val, row0, n, s->nslices, s->slice_ptr, s->soff, s->col, s->val, s->val32);
    HIP_TRY(hipGetLastError());
  }
  HIP_TRY(hipStreamSynchronize(st));
  return NAJ_OK;   // the temporaries are released by tmp's destructor
}

// Balanced item lists of the per-pass kernel on the sorted layout, for the launch shape (grid, bs).
// There the long rows and the slices come in decreasing length, so striding them over the waves gives
// the first waves of every round the longest items; a CU's three workgroups then carry unequal work,
// and the pass ends with the most loaded CU (Chung-Lu n = 2^22: the most loaded CU holds 13 % more
// than the mean).  The lists assign items longest first, each to the wave with the least work so far
// (ties to the lowest wave), and every wave sweeps its items in increasing order.  An item's cost is
// its rounds of 256 stored entries (four column steps of a slice's 64 lanes, or four 64-entry chunks of
// a long row), plus one for its row operands.  Measured on that graph: 892.6 -> 847.0 us per float64
// pass, 709.8 -> 659.2 us per float32 inner pass, answers unchanged bit for bit.  Weighting a long
// row's rounds by 0.2-0.75 or 1.5-2, or breaking ties across the CUs' dispatch slots, was slower.
naj_status build_wave_items(naj_system* s, int which, int grid, int bs, hipStream_t st) {
  const int waves = grid * (bs / kWave);
  const int64_t nlong = s->n_long, nitems = s->n_long + s->nslices;
  if (nitems <= 0 || nitems >= INT32_MAX || (int64_t)s->hlong.size() != nlong + 1 ||
      (int64_t)s->hslice.size() != s->nslices + 1)
    return NAJ_OK;   // no lists: the kernel strides items over the waves
  std::vector<int64_t> cost((size_t)nitems);
  for (int64_t r = 0; r < nlong; ++r) cost[(size_t)r] = (s->hlong[r + 1] - s->hlong[r] + 255) / 256 + 1;
  for (int64_t sl = 0; sl < s->nslices; ++sl) {
    const int64_t width = (s->hslice[sl + 1] - s->hslice[sl]) / kWave;
    cost[(size_t)(nlong + sl)] = (width + kUnroll - 1) / kUnroll + 1;
  }
  std::vector<int32_t> off, items;
  balanced_wave_lists(cost, waves, off, items);
  naj_status rc = dev_alloc(s, &s->woff[which], (size_t)waves + 1);
  if (rc == NAJ_OK) rc = dev_alloc(s, &s->witem[which], (size_t)nitems);
  if (rc != NAJ_OK) return rc;
  HIP_TRY(hipMemcpyAsync(s->woff[which], off.data(), sizeof(int32_t) * off.size(), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(s->witem[which], items.data(), sizeof(int32_t) * items.size(), hipMemcpyHostToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  s->wgrid[which] = grid;
  s->wbs[which] = bs;
  return NAJ_OK;
}

// Blocked item lists of the per-pass kernel on the regular layout, for the launch shape (grid, bs).
// Rows gather the vector up to `reach` rows away (a 3D stencil: one plane), so a vector line is first
// fetched for the rows one band of ceil(reach / 64) slices before its own and last used one band after.
// Swept in slice order, the data a domain streams between those uses is two whole bands, which on large
// 3D grids outgrows an L2.  The lists cut every band into blocks of `blk` slices and visit one block
// through all of the domain's bands before the next, so the reuse spans two blocks instead.  Each domain
// keeps its contiguous slice range (its workgroups run on one XCD), and its waves take the blocked
// order in turn.  Only the order of the slices changes: every row is computed as before.  The float64
// instances that read 4-byte values take these lists (their iteration and confirmation passes).
// Measured, float64 us per pass against slice order with blocks of 32 slices (flat from 8 to 36):
// 128^3 31.34 -> 29.82, 160^3 53.58 -> 50.54, 192^3 111.51 -> 109.80, 96^3 17.86 -> 17.47, 64^3
// 10.26 -> 10.10; answers identical bit for bit.
naj_status build_blocked_items(naj_system* s, int which, int grid, int bs, int64_t blk, hipStream_t st) {
  const int wpb = bs / kWave;
  const int waves = grid * wpb;
  const int64_t ns = s->nslices;
  const int64_t band = (s->reach + kWave - 1) / kWave;
  if (ns <= 0 || ns + s->n_long >= INT32_MAX || blk <= 0 || band <= blk || s->n_long != 0) return NAJ_OK;
  std::vector<int32_t> off, items;
  if (!blocked_wave_lists(ns, s->n_long, band, blk, s->nxcd, grid, wpb, off, items)) return NAJ_OK;
  if ((int64_t)items.size() != ns) return fail(NAJ_EDEVICE, "blocked item lists cover %lld of %lld slices",
                                              (long long)items.size(), (long long)ns);
  naj_status rc = dev_alloc(s, &s->woff[which], (size_t)waves + 1);
  if (rc == NAJ_OK) rc = dev_alloc(s, &s->witem[which], (size_t)ns);
  if (rc != NAJ_OK) return rc;
  HIP_TRY(hipMemcpyAsync(s->woff[which], off.data(), sizeof(int32_t) * off.size(), hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(s->witem[which], items.data(), sizeof(int32_t) * items.size(), hipMemcpyHostToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  s->wgrid[which] = grid;
  s->wbs[which] = bs;
  return NAJ_OK;
}

// Runs the solve kernels on `st` for the prepared control blocks; ev0/ev1 bracket them.  *final
// receives the control block that holds the finished solve's state.
naj_status run_solve(naj_system* s, SolveArgs& a, const naj_opts& o, hipStream_t st, Ctrl** final) {
  const int ud = jm_of(s);
  void* kargs[] = {&a};
  *final = a.ctrl;
  if (s->mode == kModeSmall && !s->ymode && s->n <= kLdsMaxN && env_int("NAJ_LDS", 1)) {
    const void* fn = solve_lds_kernel(ud);
    const size_t bytes = (size_t)32 * s->n;
    HIP_TRY(hipFuncSetAttribute(fn, hipFuncAttributeMaxDynamicSharedMemorySize, (int)bytes));
    HIP_TRY(hipEventRecord(s->ev0, st));
    HIP_TRY(hipLaunchKernel(fn, dim3(1), dim3(kSmallBlock), kargs, bytes, st));
    HIP_TRY(hipEventRecord(s->ev1, st));
    return NAJ_OK;
  }
  if (s->mode == kModeSmall) {
    HIP_TRY(hipEventRecord(s->ev0, st));
    HIP_TRY(hipLaunchKernel(solve_kernel(ud, s->ymode != 0), dim3(1), dim3(kSmallBlock), kargs, 0, st));
    HIP_TRY(hipEventRecord(s->ev1, st));
    return NAJ_OK;
  }
  if (s->mode == kModePersistent) {
    HIP_TRY(hipEventRecord(s->ev0, st));
    HIP_TRY(hipLaunchCooperativeKernel(solve_kernel(ud, s->ymode != 0), dim3(s->grid), dim3(kSmallBlock), kargs, 0, st));
    HIP_TRY(hipEventRecord(s->ev1, st));
    return NAJ_OK;
  }
  // One launch per pass, enqueued in chunks of 4-8.  The chunk's last launch stores the phase it
  // published in a pinned host word (workgroup 0, after its decision); the host marks the word pending
  // before enqueuing the chunk and, while the next chunk runs, waits for the word of the previous one.
  // No event or copy sits between the launches, and a finished solve leaves at most two chunks of
  // launches behind it (each copies the finished state forward in a few microseconds).  Launch k takes
  // its index parity as an argument: it publishes its control state in ctrl[k & 1] (see k_pass64).
  const bool mx = o.precision == NAJ_MIXED;
  const void* fn = pass_kernel(ud, mx ? s->pass_bs_mx : s->pass_bs, s->ymode != 0, mx ? s->nt_mx != 0 : s->nt != 0, mx,
                               s->val_exact32 != 0);
  const dim3 grid(mx ? s->grid_mx : s->grid), block(mx ? s->pass_bs_mx : s->pass_bs);
  // passes: norm of b + iterations + confirmations (at most one per confirm_gap iterations, plus one),
  // and the launch that takes the last decision
  const int64_t max_pass = o.precision == NAJ_MIXED
                               ? 3 + (int64_t)(o.max_refine + 1) * (1 + (int64_t)o.max_iter)
                               : 3 + (int64_t)o.max_iter + (int64_t)o.max_iter / std::max(1, o.confirm_gap) + 1;
  constexpr int kPending = -1;   // no phase has this value
  // Waits for chunk slot `slot`'s phase word.  The stream is asked now and then: an error it reports,
  // or a drained stream with the word still pending, ends the solve with NAJ_EDEVICE.
  auto wait_word = [&](int slot, int* phase) -> naj_status {
    for (int64_t spin = 1;; ++spin) {
      const int v = __atomic_load_n(&s->hflag[slot], __ATOMIC_ACQUIRE);
      if (v != kPending) {
        *phase = v;
        return NAJ_OK;
      }
      if (spin % 1024 == 0) {
        const hipError_t e = hipStreamQuery(st);
        if (e == hipSuccess) {
          const int w = __atomic_load_n(&s->hflag[slot], __ATOMIC_ACQUIRE);
          if (w != kPending) {
            *phase = w;
            return NAJ_OK;
          }
          return fail(NAJ_EDEVICE, "the pass launches finished without publishing their phase");
        }
        if (e != hipErrorNotReady) return fail(NAJ_EDEVICE, "solve stream: %s", hipGetErrorString(e));
        std::this_thread::yield();
      }
    }
  };
  int64_t launched = 0;
  int chunk = 4, cur = 0, prev = -1;
  int kidx = 0;
  int* flag = nullptr;
  SolveArgs ap = a;   // with the balanced item lists built for this launch shape, if any
  for (int w = 0; w < 2; ++w)
    if (s->witem[w] && s->wgrid[w] == (int)grid.x && s->wbs[w] == (int)block.x) {
      ap.A.woff = s->woff[w];
      ap.A.witem = s->witem[w];
      break;
    }
  void* pargs[] = {&ap, &kidx, &flag};
  HIP_TRY(hipEventRecord(s->ev0, st));
  for (;;) {
    const int64_t n_now = std::min<int64_t>(chunk, max_pass - launched);
    __atomic_store_n(&s->hflag[cur], kPending, __ATOMIC_RELEASE);
    for (int64_t i = 0; i < n_now; ++i) {
      const int64_t k = launched + i;
      kidx = k == 0 ? 0 : 2 - (int)(k & 1);   // the kernel needs only k > 0 and the parity of k
      flag = i + 1 == n_now ? &s->hflag[cur] : nullptr;
      HIP_TRY(hipLaunchKernel(fn, grid, block, pargs, 0, st));
    }
    launched += n_now;
    *final = a.ctrl + ((launched - 1) & 1);
    int phase = 0;
    if (prev >= 0) {
      const naj_status rc = wait_word(prev, &phase);
      if (rc != NAJ_OK) return rc;
      if (phase == PH_DONE) break;
    }
    if (launched >= max_pass) {
      const naj_status rc = wait_word(cur, &phase);
      if (rc != NAJ_OK) return rc;
      if (phase == PH_DONE) break;
      return fail(NAJ_EDEVICE, "solve did not finish within %lld passes", (long long)launched);
    }
    prev = cur;
    cur ^= 1;
    chunk = std::min(chunk * 2, 8);
  }
  HIP_TRY(hipEventRecord(s->ev1, st));
  return NAJ_OK;
}

}  // namespace

// ============================================================================ batch

struct naj_batch {
  int device = 0;
  int nsys = 0, ninst = 0, ntiles = 0, grid = 0;
  std::vector<naj_system*> systems;
  std::vector<int> nrhs, inst0;
  naj_opts opts;
  BatchSys* d_sys = nullptr;
  BatchTile* d_tiles = nullptr;
  int* d_active = nullptr;              // active item list [ntiles] and its length
  int* d_nactive = nullptr;
  int* d_sact = nullptr;                // active system list [nsys] and its length
  int* d_nsact = nullptr;
  PassView* d_vt = nullptr;             // pass views, kMaxRhs per system
  unsigned int* d_done = nullptr;
  Ctrl* d_ctrl = nullptr;
  std::vector<BatchSys> h_sys;          // host copy of the per-system records (device pointers)
  std::vector<void*> bufs;
  unsigned int* hdone = nullptr;        // pinned, 2 slots
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  int graph_len = 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr, evc[2] = {nullptr, nullptr};
  BatchArgs args;
  int64_t bytes = 0;
  std::vector<int> tile_slices;
};

namespace {

// ---- tile sizes: a process-wide table keyed by system features (never by the batch)
struct TuneKey {
  int layout, log2n, nnz_row, nrhs, precision;
  bool operator<(const TuneKey& o) const {
    return std::tie(layout, log2n, nnz_row, nrhs, precision) < std::tie(o.layout, o.log2n, o.nnz_row, o.nrhs, o.precision);
  }
};
std::mutex g_tune_mu;
std::map<TuneKey, int> g_tune;

TuneKey tune_key(const naj_system* s, int nrhs, int precision) {
  int l2 = 0;
  while ((1LL << (l2 + 1)) <= s->n) ++l2;
  return TuneKey{s->layout, l2, (int)((s->nnz + s->n / 2) / s->n), nrhs, precision};
}

// Slices per item (one wavefront's unit of work) for a system: the tuned value if one is
// recorded for its features, else a default of 2, never more than the system has.
int tile_slices_for(const naj_system* s, int nrhs, int precision) {
  int t = 2;
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    auto it = g_tune.find(tune_key(s, nrhs, precision));
    if (it != g_tune.end()) t = it->second;
  }
  if (s->nslices > 0 && t > s->nslices) t = (int)s->nslices;
  return std::max(1, t);
}

void free_batch(naj_batch* bt) {
  if (!bt) return;
  if (bt->exec) (void)hipGraphExecDestroy(bt->exec);
  if (bt->graph) (void)hipGraphDestroy(bt->graph);
  if (bt->cap) (void)hipStreamDestroy(bt->cap);
  for (void* p : bt->bufs) (void)hipFree(p);   // every device allocation of the batch, once
  if (bt->hdone) (void)hipHostFree(bt->hdone);
  if (bt->ev0) (void)hipEventDestroy(bt->ev0);
  if (bt->ev1) (void)hipEventDestroy(bt->ev1);
  for (auto& e : bt->evc)
    if (e) (void)hipEventDestroy(e);
  delete bt;
}

template <typename T>
naj_status batch_alloc(naj_batch* bt, T** p, size_t count) {
  if (count == 0) count = 1;
  hipError_t e = hipMalloc((void**)p, count * sizeof(T));
  if (e != hipSuccess) {
    *p = nullptr;
    return fail(e == hipErrorOutOfMemory ? NAJ_ENOMEM : NAJ_EDEVICE, "hipMalloc(%zu bytes): %s", count * sizeof(T),
                hipGetErrorString(e));
  }
  bt->bufs.push_back(*p);
  bt->bytes += (int64_t)(count * sizeof(T));
  return NAJ_OK;
}

naj_status batch_build(naj_batch* bt, hipStream_t st) {
  const naj_opts& o = bt->opts;
  const bool mixed = o.precision == NAJ_MIXED;
  std::vector<BatchSys>& hs = bt->h_sys;
  hs.assign(bt->nsys, BatchSys{});
  std::vector<BatchTile> ht;
  bt->ninst = 0;
  bt->inst0.assign(bt->nsys, 0);
  bt->tile_slices.assign(bt->nsys, 0);
  for (int i = 0; i < bt->nsys; ++i) {
    naj_system* s = bt->systems[i];
    const int T = tile_slices_for(s, bt->nrhs[i], o.precision);
    bt->tile_slices[i] = T;
    BatchSys& S = hs[i];
    S.A = sell_of(s);
    S.A.dom_bounds = nullptr;
    S.dinv = s->dinv;
    S.nrhs = bt->nrhs[i];
    S.tol = o.tol;
    S.lk = 0;
    while ((1 << S.lk) < S.nrhs) ++S.lk;
    S.tile0 = (int)ht.size();
    // several right-hand sides: the materialized form (one gathered vector per pass)
    S.ymode = S.nrhs > 1 ? 1 : s->ymode;
    bt->inst0[i] = bt->ninst;
    bt->ninst += bt->nrhs[i];
    const int lt = 4;   // long rows per item
    for (int64_t l = 0; l < s->n_long; l += lt)
      ht.push_back(BatchTile{i, 0, 0, (int)l, (int)std::min<int64_t>(s->n_long, l + lt)});
    for (int64_t sl = 0; sl < s->nslices; sl += T)
      ht.push_back(BatchTile{i, (int)sl, (int)std::min<int64_t>(s->nslices, sl + T), 0, 0});
    if ((int)ht.size() == S.tile0) ht.push_back(BatchTile{i, 0, 0, 0, 0});
    S.ntiles = (int)ht.size() - S.tile0;
  }
  bt->ntiles = (int)ht.size();
  naj_status rc = NAJ_OK;
  if ((rc = batch_alloc(bt, &bt->d_sys, (size_t)bt->nsys)) != NAJ_OK) return rc;
  if ((rc = batch_alloc(bt, &bt->d_tiles, (size_t)bt->ntiles)) != NAJ_OK) return rc;
  if ((rc = batch_alloc(bt, &bt->d_active, (size_t)bt->ntiles)) != NAJ_OK) return rc;
  if ((rc = batch_alloc(bt, &bt->d_nactive, (size_t)64)) != NAJ_OK) return rc;
  if ((rc = batch_alloc(bt, &bt->d_sact, (size_t)bt->nsys)) != NAJ_OK) return rc;
  if ((rc = batch_alloc(bt, &bt->d_nsact, (size_t)64)) != NAJ_OK) return rc;
  if ((rc = batch_alloc(bt, &bt->d_done, (size_t)64)) != NAJ_OK) return rc;
  if ((rc = batch_alloc(bt, &bt->d_vt, (size_t)bt->nsys * kMaxRhs)) != NAJ_OK) return rc;
  if ((rc = batch_alloc(bt, &bt->d_ctrl, (size_t)bt->ninst)) != NAJ_OK) return rc;
  for (int i = 0; i < bt->nsys; ++i) {
    naj_system* s = bt->systems[i];
    BatchSys& S = hs[i];
    const size_t nv = (size_t)s->n << S.lk;
    S.ctrl = bt->d_ctrl + bt->inst0[i];
    S.vt = bt->d_vt + (size_t)i * kMaxRhs;
    // every byte offset into the vector blocks must fit 32 bits
    if (nv * sizeof(double) * 4 >= (1ull << 32))
      return fail(NAJ_EINVAL, "system %d: n x right-hand sides too large for a batch (solve it alone)", i);
    S.xs = (uint32_t)(nv * sizeof(double));
    S.fs = (uint32_t)(nv * sizeof(float));
    S.xb = nullptr;
    S.fb = nullptr;
    // float64 iterates: mixed refinement keeps x and x + d (2 buffers), float64 solves 3 (+1 materialized y)
    if ((rc = batch_alloc(bt, &S.xb, nv * (mixed ? 2 : 3 + S.ymode))) != NAJ_OK) return rc;
    if (mixed && (rc = batch_alloc(bt, &S.fb, nv * 5)) != NAJ_OK) return rc;
    if ((rc = batch_alloc(bt, &S.b, nv)) != NAJ_OK) return rc;
    if ((rc = batch_alloc(bt, &S.part, (size_t)kPartStride * S.ntiles * S.nrhs)) != NAJ_OK) return rc;
  }
  HIP_TRY(hipMemcpyAsync(bt->d_sys, hs.data(), sizeof(BatchSys) * bt->nsys, hipMemcpyHostToDevice, st));
  HIP_TRY(hipMemcpyAsync(bt->d_tiles, ht.data(), sizeof(BatchTile) * bt->ntiles, hipMemcpyHostToDevice, st));
  HIP_TRY(hipStreamSynchronize(st));
  // grid: every resident workgroup, at most one wavefront per item
  int occ = 0, cus = 0;
  int kpmax = 1;
  for (const BatchSys& S : hs) kpmax = std::max(kpmax, 1 << S.lk);
  const void* pass_fn = batch_pass_kernel(mixed, kpmax);
  HIP_TRY(hipOccupancyMaxActiveBlocksPerMultiprocessor(&occ, pass_fn, kBatchBlock, 0));
  hipDeviceProp_t prop;
  HIP_TRY(hipGetDeviceProperties(&prop, bt->device));
  cus = prop.multiProcessorCount;
  occ = std::min(std::max(1, occ), std::max(1, env_int("NAJ_BATCH_WG_PER_CU", occ)));
  bt->grid = std::max(1, std::min((bt->ntiles + kBatchWaves - 1) / kBatchWaves, occ * cus));
  BatchArgs& A = bt->args;
  A.tiles = bt->d_tiles;
  A.sys = bt->d_sys;
  A.nsys = bt->nsys;
  A.active = bt->d_active;
  A.nactive = bt->d_nactive;
  A.sact = bt->d_sact;
  A.nsact = bt->d_nsact;
  A.done = bt->d_done;
  A.slot_done = nullptr;
  A.nxcd = std::max(1, std::min(kMaxDomains, env_int("NAJ_NXCD", (cus % 8 == 0) ? 8 : 1)));
  A.tol = o.tol;
  A.inner_tol = o.inner_tol;
  A.max_iter = o.max_iter;
  A.restart = o.restart ? 1 : 0;
  A.confirm_gap = o.confirm_gap;
  A.k0 = o.k0;
  A.precision = mixed ? 1 : 0;
  A.max_refine = o.max_refine;
  A.inner_stall = o.inner_stall;
  // a chunk of passes captured once as a graph and replayed: the active lists are rebuilt
  // at the head of each chunk, then graph_len passes (item kernel + decision kernel) run
  if (bt->exec) {
    (void)hipGraphExecDestroy(bt->exec);
    bt->exec = nullptr;
  }
  if (bt->graph) {
    (void)hipGraphDestroy(bt->graph);
    bt->graph = nullptr;
  }
  bt->graph_len = std::max(1, env_int("NAJ_GRAPH_LEN", 8));
  HIP_TRY(hipStreamBeginCapture(bt->cap, hipStreamCaptureModeThreadLocal));
  hipLaunchKernelGGL(k_batch_compact, dim3(1), dim3(kCompactBlock), 0, bt->cap, bt->args);
  for (int q = 0; q < bt->graph_len; ++q) {
    void* kargs[] = {&bt->args};
    HIP_TRY(hipLaunchKernel(pass_fn, dim3(bt->grid), dim3(kBatchBlock), kargs, 0, bt->cap));
    hipLaunchKernelGGL(k_batch_decide, dim3(bt->nsys), dim3(kDecideBlock), 0, bt->cap, bt->args);
  }
  HIP_TRY(hipStreamEndCapture(bt->cap, &bt->graph));
  HIP_TRY(hipGraphInstantiate(&bt->exec, bt->graph, nullptr, nullptr, 0));
  return NAJ_OK;
}

}  // namespace

extern "C" {

void naj_opts_default(naj_opts* o) {
  if (!o) return;
  o->tol = 1e-8;
  o->max_iter = 20000;
  o->restart = 1;
  o->k0 = 2;
  o->confirm_gap = 8;
  o->precision = NAJ_FP64;
  o->inner_tol = 1e-4;
  o->max_refine = 50;
  o->inner_stall = 200;
  o->stop = NAJ_STOP_RELRES;
  o->pad_ = 0;
  o->fstar = 0.0;
}

const char* naj_last_error(void) { return g_err.c_str(); }

const char* naj_version(void) { return "naj 0.1 gfx950"; }

// System creation; with a pool every device buffer comes from it, and a lean system holds the
// matrix only (its right-hand sides are solved by a batch or a server).
static naj_status create_system_impl(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* colidx,
                                     const double* vals, const double* D, void* stream, Pool* pool, bool lean,
                                     naj_system** out, int jblock = 0) {
  g_err.clear();
  (void)hipGetLastError();   // drop a stale error left by unrelated earlier runtime calls
  if (!out) return fail(NAJ_EINVAL, "out is NULL");
  *out = nullptr;
  if (n < 1 || n >= (1LL << 31) - 64) return fail(NAJ_EINVAL, "n must be in [1, 2^31-64) (got %lld)", (long long)n);
  if (nnz < 0 || nnz >= (1LL << 31)) return fail(NAJ_EINVAL, "nnz must be in [0, 2^31) (got %lld)", (long long)nnz);
  if (!rowptr || (nnz > 0 && (!colidx || !vals))) return fail(NAJ_EINVAL, "null CSR pointer");
  hipStream_t st = (hipStream_t)stream;
  if (jblock != 0 && jblock != 1 && jblock != 2 && jblock != 4 && jblock != 8)
    return fail(NAJ_EINVAL, "block must be 1, 2, 4 or 8 (got %d)", jblock);
  if (jblock && D) return fail(NAJ_EINVAL, "a block J and a caller diagonal D exclude each other");
  naj_system* s = new naj_system();
  s->pool = pool;
  s->lean = lean;
  s->jblock = jblock;
  naj_status rc = NAJ_OK;
  int* flag = nullptr;
  int hflag = 0;
#define STEP(x)              \
  do {                       \
    rc = (x);                \
    if (rc != NAJ_OK) goto bad; \
  } while (0)
#define HSTEP(expr)                                                                                   \
  do {                                                                                                \
    hipError_t e_ = (expr);                                                                           \
    if (e_ != hipSuccess) {                                                                           \
      rc = fail(e_ == hipErrorOutOfMemory ? NAJ_ENOMEM : NAJ_EDEVICE, "%s: %s", #expr, hipGetErrorString(e_)); \
      goto bad;                                                                                       \
    }                                                                                                 \
  } while (0)
  HSTEP(hipGetDevice(&s->device));
  s->n = n;
  s->nnz = nnz;
  HSTEP(sys_malloc(s, (void**)&flag, sizeof(int)));
  HSTEP(hipMemsetAsync(flag, 0, sizeof(int), st));
  hipLaunchKernelGGL(k_check_rowptr, dim3(blocks_for(n, kAux)), dim3(kAux), 0, st, rowptr, n, nnz, flag);
  HSTEP(hipGetLastError());
  HSTEP(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  HSTEP(hipStreamSynchronize(st));
  if (hflag) {
    rc = fail(NAJ_EINVAL, "invalid rowptr (flags 0x%x: 1 decreasing, 2 rowptr[0]!=0, 4 rowptr[n]!=nnz)", hflag);
    goto bad;
  }
  if (nnz > 0) {
    hipLaunchKernelGGL(k_check_cols, dim3(blocks_for(nnz, kAux)), dim3(kAux), 0, st, colidx, nnz, n, flag);
    HSTEP(hipGetLastError());
    hipLaunchKernelGGL(k_check_vals, dim3(blocks_for(nnz, kAux)), dim3(kAux), 0, st, vals, nnz, flag);
    HSTEP(hipGetLastError());
  }
  if (D) {
    STEP(dev_alloc(s, &s->dinv, (size_t)n));
    hipLaunchKernelGGL(k_check_D, dim3(blocks_for(n, kAux)), dim3(kAux), 0, st, D, n, s->dinv, flag);
    HSTEP(hipGetLastError());
  }
  HSTEP(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
  HSTEP(hipStreamSynchronize(st));
  if (hflag) {
    rc = fail(NAJ_EINVAL, "invalid input (flags 0x%x: 8 column index out of range, 16 D not finite and > 0, "
              "32 value not finite)", hflag);
    goto bad;
  }
  STEP(build_layout(s, rowptr, colidx, vals, st));
  // 4-byte values for the float64 passes when every stored value is exact in float32 (graph Laplacians
  // with integer weights, stencils, the Section 4.1 matrix): the same products and sums on half the
  // value bytes.  NAJ_VALUES32=0 keeps the 8-byte values.  A block J keeps its inverse blocks in float64
  // (128^3, 8-row blocks: 59.4 -> 45.8 us per float64 pass, the pass then fitting the MALL).
  if (env_int("NAJ_VALUES32", 1)) {
    HSTEP(hipMemsetAsync(flag, 0, sizeof(int), st));
    const int64_t ns = s->nslices > 0 ? (int64_t)s->hslice[s->nslices] : 0;
    if (ns > 0) {
      hipLaunchKernelGGL(k_check_exact32, dim3(blocks_for(ns, kAux)), dim3(kAux), 0, st, s->val, s->val32, ns, flag);
      HSTEP(hipGetLastError());
    }
    const int64_t nl = s->n_long > 0 ? (int64_t)s->hlong[s->n_long] : 0;
    if (nl > 0) {
      hipLaunchKernelGGL(k_check_exact32, dim3(blocks_for(nl, kAux)), dim3(kAux), 0, st, s->lval, s->lval32, nl, flag);
      HSTEP(hipGetLastError());
    }
    HSTEP(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    HSTEP(hipStreamSynchronize(st));
    s->val_exact32 = hflag == 0 ? 1 : 0;
    hflag = 0;
    HSTEP(hipMemsetAsync(flag, 0, sizeof(int), st));
  }
  s->ymode = env_int("NAJ_YMODE", s->layout == 1 ? 1 : 0) ? 1 : 0;
  if (jblock) {   // eq. (J-blkdiag): inverse blocks from the caller's CSR
    s->ymode = 0;
    const int64_t nblk = s->nslices * kWave / jblock;
    STEP(dev_alloc(s, &s->jinv, (size_t)(s->nslices * kWave * jblock)));
    STEP(dev_alloc(s, &s->jinv32, (size_t)(s->nslices * kWave * jblock)));
    const dim3 g(blocks_for(nblk, 64)), b(64);
    if (jblock == 1) hipLaunchKernelGGL(k_block_jinv<1>, g, b, 0, st, rowptr, colidx, vals, n, nblk, s->jinv, s->jinv32, flag);
    if (jblock == 2) hipLaunchKernelGGL(k_block_jinv<2>, g, b, 0, st, rowptr, colidx, vals, n, nblk, s->jinv, s->jinv32, flag);
    if (jblock == 4) hipLaunchKernelGGL(k_block_jinv<4>, g, b, 0, st, rowptr, colidx, vals, n, nblk, s->jinv, s->jinv32, flag);
    if (jblock == 8) hipLaunchKernelGGL(k_block_jinv<8>, g, b, 0, st, rowptr, colidx, vals, n, nblk, s->jinv, s->jinv32, flag);
    HSTEP(hipGetLastError());
    HSTEP(hipMemcpyAsync(&hflag, flag, sizeof(int), hipMemcpyDeviceToHost, st));
    HSTEP(hipStreamSynchronize(st));
    if (hflag) {
      rc = fail(NAJ_EINVAL, "a diagonal block of the block J is not positive definite (Q is not PSD)");
      goto bad;
    }
  }
  STEP(choose_grid(s, st));
  {
    // A float64 iteration pass larger than the 256 MB MALL streams its matrix entries with
    // non-temporal loads, so they do not evict the gathered vectors (160^3: 92.7 -> 83.1 us per pass;
    // the Section 4.1 system n = 6000: 95.5 -> 89.4 us; Chung-Lu n = 2^22: 911 -> 892 us; 192^3 with
    // 4-byte values, 512 threads: 124.7 -> 111.6 us).  A pass that fits keeps ordinary loads: the whole
    // pass then stays in the MALL between passes (128^3: 36.9 us, 46.5 us with non-temporal loads;
    // with 4-byte values 128^3 31.2 against 38.3 us, 160^3 54.3 against 67.7 us).
    const int64_t pass_bytes = (s->val_exact32 ? 4 : 8) * s->stored + 4 * (s->stored - s->off_nnz - s->run_nnz) + 32 * n +
                               8 * (int64_t)jblock * n;
    s->nt = env_int("NAJ_NT", pass_bytes > kMallBytes ? 1 : 0) ? 1 : 0;
    // the same rule for the float32 inner pass of mixed solves (4-byte values, float32 vectors and r32):
    // mixed 192^3 (about 340 MB) 69.3 -> 63.8 ms per solve with non-temporal loads; 160^3 (197 MB) keeps
    // ordinary loads (30.8 against 37.7 ms)
    const int64_t inner_bytes =
        4 * s->stored + 4 * (s->stored - s->off_nnz - s->run_nnz) + 20 * n + 4 * (int64_t)jblock * n;
    s->nt_mx = env_int("NAJ_NT_MIXED", inner_bytes > kMallBytes ? 1 : 0) ? 1 : 0;
  }
  if (!lean) {   // workspace of the single-solve drivers
    if (s->layout == 1 && s->mode == kModePass && env_int("NAJ_WAVE_LISTS", 1)) {
      STEP(build_wave_items(s, 0, s->grid, s->pass_bs, st));
      if (s->grid_mx != s->grid || s->pass_bs_mx != s->pass_bs)
        STEP(build_wave_items(s, 1, s->grid_mx, s->pass_bs_mx, st));
    }
    // float64 passes only: the float32 inner pass of mixed solves measured no faster with the blocked
    // order (128^3 25.8 -> 25.6 us, 160^3 41.5 -> 42.0, 192^3 81.5 -> 82.2)
    // not with a block J: its 128^3 pass (8-row blocks) measured 45.8 us in slice order, 47.1 blocked
    if (s->layout == 0 && s->mode == kModePass && s->val_exact32 && !jblock)
      STEP(build_blocked_items(s, 0, s->grid, s->pass_bs, env_int("NAJ_BLOCK", 32), st));
    for (int i = 0; i < 3 + s->ymode; ++i) STEP(dev_alloc(s, &s->vec[i], (size_t)n));
    STEP(dev_alloc(s, &s->part, (size_t)2 * kPartStride * s->max_grid));
    STEP(dev_alloc(s, &s->ctrl, 2));
    STEP(dev_alloc(s, &s->bar, 1));
    STEP(dev_alloc(s, &s->counters, (size_t)kCounterWords));
    HSTEP(hipMemsetAsync(s->counters, 0, sizeof(unsigned int) * kCounterWords, st));
    STEP(dev_alloc(s, &s->scal, 8));
    HSTEP(hipEventCreate(&s->ev0));
    HSTEP(hipEventCreate(&s->ev1));
    HSTEP(hipHostMalloc((void**)&s->hflag, 4 * sizeof(int), hipHostMallocDefault));
    for (int i = 0; i < 4; ++i) s->hflag[i] = 0;
  }
  HSTEP(hipStreamSynchronize(st));
  sys_free(s, flag);
  *out = s;
  return NAJ_OK;
bad:
  (void)hipStreamSynchronize(st);   // kernels enqueued before the failure may still use the memory freed below
  if (flag) sys_free(s, flag);
  free_system(s);
  return rc;
#undef STEP
#undef HSTEP
}

naj_status naj_create_system(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* colidx, const double* vals,
                             const double* D, void* stream, naj_system** out) {
  return create_system_impl(n, nnz, rowptr, colidx, vals, D, stream, nullptr, false, out);
}

naj_status naj_create_system_blockj(int64_t n, int64_t nnz, const int32_t* rowptr, const int32_t* colidx,
                                    const double* vals, int32_t block, void* stream, naj_system** out) {
  if (block < 1) {
    g_err.clear();
    return fail(NAJ_EINVAL, "block must be 1, 2, 4 or 8 (got %d)", block);
  }
  return create_system_impl(n, nnz, rowptr, colidx, vals, nullptr, stream, nullptr, false, out, block);
}

naj_status naj_block_inverse(naj_system* s, double* out, void* stream) {
  g_err.clear();
  (void)hipGetLastError();
  if (!s || !out) return fail(NAJ_EINVAL, "null argument");
  if (s->jblock == 0) return fail(NAJ_EINVAL, "the system uses a diagonal J (no block inverse)");
  hipStream_t st = (hipStream_t)stream;
  const int64_t cnt = s->n * s->jblock;
  hipLaunchKernelGGL(k_block_jinv_out, dim3(blocks_for(cnt, kAux)), dim3(kAux), 0, st, s->jinv, s->n, s->jblock, out);
  HIP_TRY(hipGetLastError());
  return NAJ_OK;
}

void naj_destroy_system(naj_system* s) {
  if (!s) return;
  (void)hipDeviceSynchronize();
  free_system(s);
}

naj_status naj_system_info(const naj_system* s, int64_t* n, int64_t* nnz, int64_t* device_bytes, int32_t* layout,
                           int64_t* stored_entries) {
  if (!s) return fail(NAJ_EINVAL, "system is NULL");
  if (n) *n = s->n;
  if (nnz) *nnz = s->nnz;
  if (device_bytes) *device_bytes = s->bytes;
  if (layout) *layout = s->layout;
  if (stored_entries) *stored_entries = s->stored;
  return NAJ_OK;
}

naj_status naj_system_value_bytes(const naj_system* s, int32_t* bytes) {
  if (!s || !bytes) return fail(NAJ_EINVAL, "system and bytes are required");
  *bytes = s->val_exact32 ? 4 : 8;
  return NAJ_OK;
}

naj_status naj_system_offset_slices(const naj_system* s, int64_t* offset_slices, int64_t* nslices,
                                    int64_t* offset_nnz) {
  if (!s) return fail(NAJ_EINVAL, "system is NULL");
  if (offset_slices) *offset_slices = s->off_slices;
  if (nslices) *nslices = s->nslices;
  if (offset_nnz) *offset_nnz = s->off_nnz + s->run_nnz;
  return NAJ_OK;
}

// The body of naj_solve and naj_solve_noalloc: w is the per-solve scratch; with may_alloc false
// nothing is allocated (no history buffers; mixed precision needs the float32 vectors already).
static naj_status solve_impl(naj_system* s, const double* b, const double* x0, const naj_opts* opts, double* x,
                             naj_result* res, double* hist, int32_t hist_cap, int32_t* restart_log, int32_t log_cap,
                             double* trace, int32_t trace_cap, hipStream_t st, const SolveScratch& w,
                             bool may_alloc) {
  naj_opts o;
  if (opts) o = *opts; else naj_opts_default(&o);
  naj_status rc = check_opts(o);
  if (rc != NAJ_OK) return rc;
  if ((hist && hist_cap < 0) || (trace && trace_cap < 0) || (restart_log && log_cap < 0))
    return fail(NAJ_EINVAL, "negative capacity");
  if (may_alloc) {
    rc = ensure_hist(s, hist ? hist_cap : 0, trace ? trace_cap : 0);
    if (rc != NAJ_OK) return rc;
    if (o.precision == NAJ_MIXED && !s->fvec[0]) {
      for (int i = 0; i < 5; ++i) {
        if (i == 3 && !s->ymode) continue;
        rc = dev_alloc(s, &s->fvec[i], (size_t)s->n);
        if (rc != NAJ_OK) return rc;
      }
    }
  } else if (o.precision == NAJ_MIXED && !s->fvec[0]) {
    return fail(NAJ_EINVAL, "mixed precision needs the system's float32 work vectors, which the first mixed "
                            "naj_solve on it allocates; this entry point allocates nothing");
  }
  const double* b_in = b;
  if (s->perm) {   // into the solver's row order
    hipLaunchKernelGGL(k_gather, dim3(blocks_for(s->n, kAux * 4)), dim3(kAux), 0, st, b, s->perm, s->bperm, s->n);
    HIP_TRY(hipGetLastError());
    b_in = s->bperm;
    if (x0) {
      hipLaunchKernelGGL(k_gather, dim3(blocks_for(s->n, kAux * 4)), dim3(kAux), 0, st, x0, s->perm, s->vec[0], s->n);
      HIP_TRY(hipGetLastError());
    }
  } else if (x0) {
    HIP_TRY(hipMemcpyAsync(s->vec[0], x0, sizeof(double) * s->n, hipMemcpyDeviceToDevice, st));
  }
  if (!x0) HIP_TRY(hipMemsetAsync(s->vec[0], 0, sizeof(double) * s->n, st));
  hipLaunchKernelGGL(k_solve_init, dim3(1), dim3(64), 0, st, w.ctrl, w.bar, w.counters, o.k0, s->ymode);
  HIP_TRY(hipGetLastError());
  // a cancel request applies to the solve that is running: one left from before this solve is dropped
  // (the stream is idle here for this system's work: every entry point returns after its stream work)
  __atomic_store_n(&s->hflag[2], 0, __ATOMIC_RELEASE);
  SolveArgs a = make_args(s, b_in, o, w);
  if (!hist || !may_alloc) a.hist = nullptr, a.hist_cap = 0;
  else a.hist_cap = std::min(hist_cap, s->hist_cap_dev);
  if (!trace || !may_alloc) a.trace = nullptr, a.trace_cap = 0;
  else a.trace_cap = std::min(trace_cap, s->trace_cap_dev);
  Ctrl* fin = nullptr;
  rc = run_solve(s, a, o, st, &fin);
  if (rc != NAJ_OK) return rc;
  hipLaunchKernelGGL(k_copy_result, dim3(blocks_for(s->n, kAux * 4)), dim3(kAux), 0, st, fin, s->vec[0],
                     s->vec[1], s->vec[2], x, s->perm, s->n);
  HIP_TRY(hipGetLastError());
  Ctrl hc;
  HIP_TRY(hipMemcpyAsync(&hc, fin, sizeof(Ctrl), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  const int hl = std::min(hc.hist_len, a.hist_cap);
  if (a.hist && hl > 0) HIP_TRY(hipMemcpy(hist, s->hist, sizeof(double) * hl, hipMemcpyDeviceToHost));
  const int tl = std::min(o.precision == NAJ_MIXED ? hc.outer : hc.hist_len, a.trace_cap);
  if (a.trace && tl > 0) HIP_TRY(hipMemcpy(trace, s->trace, sizeof(double) * 2 * tl, hipMemcpyDeviceToHost));
  int nlog = std::min(hc.restarts, (int)kRestartLogCap);
  if (restart_log) {
    nlog = std::min(nlog, (int)log_cap);
    for (int i = 0; i < nlog; ++i) restart_log[i] = hc.restart_log[i];
  }
  res->status = hc.status;
  res->iterations = hc.iterations;
  res->restarts = hc.restarts;
  res->confirmations = hc.confirms;
  res->relres = hc.relres;
  if (o.precision == NAJ_MIXED) {
    res->iterations = hc.inner_total;
    res->restarts = hc.inner_restarts;
    res->confirmations = hc.outer;
  }
  res->hist_len = a.hist ? std::max(hl, 0) : 0;
  res->nrestart_log = restart_log ? nlog : 0;
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, s->ev0, s->ev1));
  res->kernel_ms = ms;
  res->passes = hc.passes;
  res->grid = (s->mode == kModePass && o.precision == NAJ_MIXED) ? s->grid_mx : s->grid;
  if (hc.timeout) {
    res->status = NAJ_EDEVICE;
    return fail(NAJ_EDEVICE, "grid barrier wait timed out inside the solve kernel");
  }
  res->objgap = __builtin_nan("");
  const bool obj = o.stop == NAJ_STOP_OBJECTIVE;
  if (obj && hc.status == ST_OK) res->objgap = hc.nb > 0.0 ? hc.relres : 0.0;
  if ((obj || hc.status == ST_NOT_CONVERGED || hc.status == ST_BREAKDOWN || hc.status == ST_CANCELLED) &&
      hc.result >= 0 && hc.nb > 0.0) {
    double rr = 0.0;   // residual of the returned iterate, in the solver's row order
    rc = residual_norm2(s, s->vec[hc.result], b_in, nullptr, &rr, st, false, w);
    if (rc != NAJ_OK) return rc;
    res->relres = std::sqrt(rr) / hc.nb;
    if (obj && hc.status != ST_OK) {   // the objective gap of the returned iterate
      double fx = 0.0;
      rc = residual_norm2(s, s->vec[hc.result], b_in, nullptr, &fx, st, true, w);
      if (rc != NAJ_OK) return rc;
      res->objgap = std::fabs(fx - o.fstar) / (1.0 + std::fabs(o.fstar));
    }
  }
  if (hc.status == ST_BREAKDOWN) return fail(NAJ_EBREAKDOWN, "NaN/Inf in a reduction at iteration %d", hc.iterations);
  if (hc.status == ST_CANCELLED) return fail(NAJ_ECANCELLED, "cancelled after %d passes", hc.passes);
  return (naj_status)hc.status;
}

naj_status naj_bandwidth_probe(int32_t mode, const void* src, void* dst, int64_t bytes, int32_t reps,
                               double* ms, void* stream) {
  g_err.clear();
  (void)hipGetLastError();
  if (mode < 0 || mode > 2) return fail(NAJ_EINVAL, "mode must be 0 (read), 1 (copy) or 2 (write)");
  if (bytes < 16 || bytes % 16 != 0) return fail(NAJ_EINVAL, "bytes must be a positive multiple of 16");
  if (reps < 1 || !ms) return fail(NAJ_EINVAL, "reps >= 1 and ms are required");
  if ((mode != 2 && !src) || !dst) return fail(NAJ_EINVAL, "src (modes 0, 1) and dst are required");
  if (((uintptr_t)src | (uintptr_t)dst) % 16 != 0) return fail(NAJ_EINVAL, "src and dst must be 16-byte aligned");
  hipStream_t st = (hipStream_t)stream;
  int dev = 0, cus = 0;
  HIP_TRY(hipGetDevice(&dev));
  HIP_TRY(hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev));
  const int64_t n16 = bytes / 16;
  const int64_t nblk = (n16 + (int64_t)kProbeBlock * kProbeInFlight - 1) / ((int64_t)kProbeBlock * kProbeInFlight);
  const int grid = (int)std::max<int64_t>(1, std::min<int64_t>((int64_t)cus * kProbeWgPerCu, nblk));
  const u32x4* s4 = (const u32x4*)src;
  u32x4* d4 = (u32x4*)dst;
  auto launch = [&]() {
    if (mode == 0) hipLaunchKernelGGL(k_bw_probe<0>, dim3(grid), dim3(kProbeBlock), 0, st, s4, d4, n16);
    else if (mode == 1) hipLaunchKernelGGL(k_bw_probe<1>, dim3(grid), dim3(kProbeBlock), 0, st, s4, d4, n16);
    else hipLaunchKernelGGL(k_bw_probe<2>, dim3(grid), dim3(kProbeBlock), 0, st, s4, d4, n16);
  };
  launch();   // warm-up
  HIP_TRY(hipGetLastError());
  hipEvent_t e0 = nullptr, e1 = nullptr;
  HIP_TRY(hipEventCreate(&e0));
  HIP_TRY(hipEventCreate(&e1));
  HIP_TRY(hipEventRecord(e0, st));
  for (int r = 0; r < reps; ++r) launch();
  HIP_TRY(hipEventRecord(e1, st));
  HIP_TRY(hipEventSynchronize(e1));
  float t = 0.f;
  const hipError_t e = hipEventElapsedTime(&t, e0, e1);
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  HIP_TRY(e);
  *ms = (double)t / reps;
  return NAJ_OK;
}

naj_status naj_cancel(naj_system* s) {
  if (!s) return fail(NAJ_EINVAL, "system is NULL");
  if (!s->hflag) return fail(NAJ_EINVAL, "the system belongs to a server and has no single-solve state");
  __atomic_store_n(&s->hflag[2], 1, __ATOMIC_RELEASE);
  return NAJ_OK;
}

naj_status naj_solve(naj_system* s, const double* b, const double* x0, const naj_opts* opts, double* x,
                     naj_result* res, double* hist, int32_t hist_cap, int32_t* restart_log, int32_t log_cap,
                     double* trace, int32_t trace_cap, void* stream) {
  g_err.clear();
  (void)hipGetLastError();   // drop a stale error left by unrelated earlier runtime calls
  if (!s) return fail(NAJ_EINVAL, "system is NULL");
  if (!b || !x || !res) return fail(NAJ_EINVAL, "b, x and res are required");
  if (x == b) return fail(NAJ_EINVAL, "x must not alias b");
  HIP_TRY(hipSetDevice(s->device));
  return solve_impl(s, b, x0, opts, x, res, hist, hist_cap, restart_log, log_cap, trace, trace_cap,
                    (hipStream_t)stream, own_scratch(s), true);
}

naj_status naj_solve_noalloc(naj_system* s, const double* b, const double* x0, const naj_opts* opts, double* x,
                             naj_result* res, int32_t* restart_log, int32_t log_cap, void* stream) {
  g_err.clear();
  (void)hipGetLastError();
  if (!s) return fail(NAJ_EINVAL, "system is NULL");
  if (!b || !x || !res) return fail(NAJ_EINVAL, "b, x and res are required");
  if (x == b) return fail(NAJ_EINVAL, "x must not alias b");
  if (s->lean) return fail(NAJ_EINVAL, "the system belongs to a server and has no single-solve vectors");
  if (s->max_grid > kNoAllocMaxGrid)
    return fail(NAJ_EINVAL, "the system's drivers use %d workgroups; the static scratch holds partial sums for %d",
                s->max_grid, kNoAllocMaxGrid);
  HIP_TRY(hipSetDevice(s->device));
  SolveScratch w;
  naj_status rc = noalloc_scratch(s->device, &w);
  if (rc != NAJ_OK) return rc;
  return solve_impl(s, b, x0, opts, x, res, nullptr, 0, restart_log, log_cap, nullptr, 0, (hipStream_t)stream, w,
                    false);
}

naj_status naj_step(naj_system* s, const double* p, const double* r, double beta, const double* b, double* x,
                    double* red, void* stream) {
  g_err.clear();
  (void)hipGetLastError();   // drop a stale error left by unrelated earlier runtime calls
  if (!s || !p || !b || !x || !red) return fail(NAJ_EINVAL, "null argument");
  if (x == p || x == r || x == b) return fail(NAJ_EINVAL, "x must not alias p, r or b");
  if (beta != 0.0 && !r) return fail(NAJ_EINVAL, "r is required when beta != 0");
  hipStream_t st = (hipStream_t)stream;
  naj_opts o;
  naj_opts_default(&o);
  SolveArgs a = make_args(s, b, o, own_scratch(s));
  const int G = s->aux_grid;
  const int bz = beta == 0.0 ? 1 : 0;
  const double* P = p;
  const double* R = bz ? p : r;
  double* W = x;
  if (s->perm) {   // run in the solver's row order
    const dim3 g1(blocks_for(s->n, kAux * 4)), b1(kAux);
    hipLaunchKernelGGL(k_gather, g1, b1, 0, st, p, s->perm, s->vec[0], s->n);
    if (!bz) hipLaunchKernelGGL(k_gather, g1, b1, 0, st, r, s->perm, s->vec[1], s->n);
    hipLaunchKernelGGL(k_gather, g1, b1, 0, st, b, s->perm, s->bperm, s->n);
    HIP_TRY(hipGetLastError());
    P = s->vec[0];
    R = bz ? s->vec[0] : s->vec[1];
    W = s->vec[2];
    a.b = s->bperm;
  }
  if (s->jblock > 0)
    hipLaunchKernelGGL(k_step64<kJBlock>, dim3(G), dim3(kAux), 0, st, a, P, R, beta, bz, W);
  else if (s->dinv)
    hipLaunchKernelGGL(k_step64<kJUser>, dim3(G), dim3(kAux), 0, st, a, P, R, beta, bz, W);
  else
    hipLaunchKernelGGL(k_step64<kJRowSum>, dim3(G), dim3(kAux), 0, st, a, P, R, beta, bz, W);
  HIP_TRY(hipGetLastError());
  if (s->perm) {
    hipLaunchKernelGGL(k_scatter, dim3(blocks_for(s->n, kAux * 4)), dim3(kAux), 0, st, W, s->perm, x, s->n);
    HIP_TRY(hipGetLastError());
  }
  hipLaunchKernelGGL(k_reduce_fixed, dim3(1), dim3(kWave), 0, st, s->part, G, s->scal);
  HIP_TRY(hipGetLastError());
  HIP_TRY(hipMemcpyAsync(red, s->scal, 3 * sizeof(double), hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  return NAJ_OK;
}

naj_status naj_residual(naj_system* s, const double* x, const double* b, double* out, double* rr, void* stream) {
  g_err.clear();
  if (!s || !x || !b || !rr) return fail(NAJ_EINVAL, "null argument");
  hipStream_t st = (hipStream_t)stream;
  if (!s->perm) return residual_norm2(s, x, b, out, rr, st, false, own_scratch(s));
  const dim3 g1(blocks_for(s->n, kAux * 4)), b1(kAux);
  hipLaunchKernelGGL(k_gather, g1, b1, 0, st, x, s->perm, s->vec[0], s->n);
  hipLaunchKernelGGL(k_gather, g1, b1, 0, st, b, s->perm, s->bperm, s->n);
  HIP_TRY(hipGetLastError());
  naj_status rc = residual_norm2(s, s->vec[0], s->bperm, out ? s->vec[1] : nullptr, rr, st, false, own_scratch(s));
  if (rc != NAJ_OK) return rc;
  if (out) {
    hipLaunchKernelGGL(k_scatter, g1, b1, 0, st, s->vec[1], s->perm, out, s->n);
    HIP_TRY(hipGetLastError());
    HIP_TRY(hipStreamSynchronize(st));
  }
  return NAJ_OK;
}

naj_status naj_diagonal(naj_system* s, double* out, void* stream) {
  g_err.clear();
  if (!s || !out) return fail(NAJ_EINVAL, "null argument");
  if (s->jblock) return fail(NAJ_EINVAL, "the system uses a block J (read it with naj_block_inverse)");
  hipStream_t st = (hipStream_t)stream;
  double* dst = s->perm ? s->vec[0] : out;
  hipLaunchKernelGGL(k_row_abs_sum, dim3(blocks_for(std::max<int64_t>(s->n, s->nslices * kWave), kAux)), dim3(kAux), 0,
                     st, sell_of(s), s->dinv, dst);
  HIP_TRY(hipGetLastError());
  if (!s->dinv && s->n_long > 0) {
    hipLaunchKernelGGL(k_long_abs_sum, dim3(blocks_for(s->n_long * kWave, kAux)), dim3(kAux), 0, st, sell_of(s), dst);
    HIP_TRY(hipGetLastError());
  }
  if (s->perm) {
    hipLaunchKernelGGL(k_scatter, dim3(blocks_for(s->n, kAux * 4)), dim3(kAux), 0, st, dst, s->perm, out, s->n);
    HIP_TRY(hipGetLastError());
  }
  HIP_TRY(hipStreamSynchronize(st));
  return NAJ_OK;
}


naj_status naj_batch_create(int32_t nsys, naj_system* const* systems, const int32_t* nrhs, const naj_opts* opts,
                            void* stream, naj_batch** out) {
  g_err.clear();
  if (!out) return fail(NAJ_EINVAL, "out is NULL");
  *out = nullptr;
  if (nsys < 1 || !systems || !nrhs) return fail(NAJ_EINVAL, "need nsys >= 1, systems and nrhs");
  naj_opts o;
  if (opts) o = *opts; else naj_opts_default(&o);
  naj_status rc = check_opts(o);
  if (rc != NAJ_OK) return rc;
  if (o.stop != NAJ_STOP_RELRES) return fail(NAJ_EINVAL, "batches stop on the relative residual only");
  int dev = 0;
  HIP_TRY(hipGetDevice(&dev));
  for (int i = 0; i < nsys; ++i) {
    if (!systems[i]) return fail(NAJ_EINVAL, "system %d is NULL", i);
    if (nrhs[i] < 1 || nrhs[i] > kMaxRhs) return fail(NAJ_EINVAL, "nrhs[%d] = %d outside [1, %d]", i, nrhs[i], kMaxRhs);
    if (systems[i]->device != dev) return fail(NAJ_EINVAL, "system %d lives on another device", i);
    if (systems[i]->jblock) return fail(NAJ_EINVAL, "system %d uses a block J (single solves only)", i);
  }
  naj_batch* bt = new naj_batch();
  bt->device = dev;
  bt->nsys = nsys;
  bt->systems.assign(systems, systems + nsys);
  bt->nrhs.assign(nrhs, nrhs + nsys);
  bt->opts = o;
  hipStream_t st = (hipStream_t)stream;
  hipError_t e = hipStreamCreateWithFlags(&bt->cap, hipStreamNonBlocking);
  if (e == hipSuccess) e = hipEventCreate(&bt->ev0);
  if (e == hipSuccess) e = hipEventCreate(&bt->ev1);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&bt->evc[0], hipEventDisableTiming);
  if (e == hipSuccess) e = hipEventCreateWithFlags(&bt->evc[1], hipEventDisableTiming);
  if (e == hipSuccess) e = hipHostMalloc((void**)&bt->hdone, 2 * sizeof(unsigned int), hipHostMallocDefault);
  if (e != hipSuccess) {
    free_batch(bt);
    return fail(NAJ_EDEVICE, "batch setup: %s", hipGetErrorString(e));
  }
  rc = batch_build(bt, st);
  if (rc != NAJ_OK) {
    free_batch(bt);
    return rc;
  }
  *out = bt;
  return NAJ_OK;
}

void naj_batch_destroy(naj_batch* bt) {
  if (!bt) return;
  (void)hipDeviceSynchronize();
  free_batch(bt);
}

naj_status naj_batch_info(const naj_batch* bt, int32_t* ntiles, int32_t* grid, int64_t* device_bytes) {
  if (!bt) return fail(NAJ_EINVAL, "batch is NULL");
  if (ntiles) *ntiles = bt->ntiles;
  if (grid) *grid = bt->grid;
  if (device_bytes) *device_bytes = bt->bytes;
  return NAJ_OK;
}

naj_status naj_batch_solve(naj_batch* bt, const double* const* b, const double* const* x0, double* const* x,
                           naj_result* res, void* stream) {
  g_err.clear();
  (void)hipGetLastError();   // drop a stale error left by unrelated earlier runtime calls
  if (!bt || !b || !x || !res) return fail(NAJ_EINVAL, "batch, b, x and res are required");
  for (int i = 0; i < bt->nsys; ++i)
    if (!b[i] || !x[i]) return fail(NAJ_EINVAL, "b[%d] and x[%d] are required", i, i);
  hipStream_t st = (hipStream_t)stream;
  HIP_TRY(hipSetDevice(bt->device));
  const naj_opts& o = bt->opts;
  hipLaunchKernelGGL(k_batch_init, dim3(bt->nsys), dim3(kMaxRhs), 0, st, bt->args);
  HIP_TRY(hipGetLastError());
  for (int i = 0; i < bt->nsys; ++i) {
    naj_system* s = bt->systems[i];
    const BatchSys& S = bt->h_sys[i];
    const int kp = 1 << S.lk;
    const dim3 g1(blocks_for(s->n * kp, kAux * 4)), b1(kAux);
    hipLaunchKernelGGL(k_batch_load, g1, b1, 0, st, b[i], S.nrhs, kp, s->perm, s->n, S.b);
    hipLaunchKernelGGL(k_batch_load, g1, b1, 0, st, x0 ? x0[i] : nullptr, S.nrhs, kp, s->perm, s->n, S.xb);
  }
  HIP_TRY(hipGetLastError());
  // passes: graph replays, the host checking the previous replay's done count while the next runs
  const int64_t per_inst = o.precision == NAJ_MIXED
                               ? 2 + (int64_t)(o.max_refine + 1) * (1 + (int64_t)o.max_iter)
                               : 2 + (int64_t)o.max_iter + (int64_t)o.max_iter / std::max(1, o.confirm_gap) + 1;
  const int64_t max_replays = per_inst / bt->graph_len + 2;
  int64_t replays = 0;
  int cur = 0, prev = -1;
  bool finished = false;
  HIP_TRY(hipEventRecord(bt->ev0, st));
  for (;;) {
    HIP_TRY(hipGraphLaunch(bt->exec, st));
    ++replays;
    HIP_TRY(hipMemcpyAsync(&bt->hdone[cur], bt->d_done, sizeof(unsigned int), hipMemcpyDeviceToHost, st));
    HIP_TRY(hipEventRecord(bt->evc[cur], st));
    if (prev >= 0) {
      HIP_TRY(hipEventSynchronize(bt->evc[prev]));
      if ((int)bt->hdone[prev] >= bt->ninst) {
        finished = true;
        break;
      }
    }
    if (replays >= max_replays) {
      HIP_TRY(hipEventSynchronize(bt->evc[cur]));
      finished = (int)bt->hdone[cur] >= bt->ninst;
      break;
    }
    prev = cur;
    cur ^= 1;
  }
  HIP_TRY(hipEventRecord(bt->ev1, st));
  if (!finished) return fail(NAJ_EDEVICE, "batch did not finish within %lld passes", (long long)replays * bt->graph_len);
  for (int i = 0; i < bt->nsys; ++i) {
    naj_system* s = bt->systems[i];
    const int k = bt->nrhs[i];
    hipLaunchKernelGGL(k_batch_store, dim3(blocks_for(s->n * k, kAux * 4)), dim3(kAux), 0, st, bt->d_sys, i, k, s->perm,
                       s->n, x[i]);
  }
  HIP_TRY(hipGetLastError());
  std::vector<Ctrl> hc(bt->ninst);
  HIP_TRY(hipMemcpyAsync(hc.data(), bt->d_ctrl, sizeof(Ctrl) * bt->ninst, hipMemcpyDeviceToHost, st));
  HIP_TRY(hipStreamSynchronize(st));
  float ms = 0.f;
  HIP_TRY(hipEventElapsedTime(&ms, bt->ev0, bt->ev1));
  naj_status worst = NAJ_OK;
  for (int q = 0; q < bt->ninst; ++q) {
    const Ctrl& c = hc[q];
    naj_result& r = res[q];
    r.status = c.status;
    r.iterations = o.precision == NAJ_MIXED ? c.inner_total : c.iterations;
    r.restarts = o.precision == NAJ_MIXED ? c.inner_restarts : c.restarts;
    r.confirmations = o.precision == NAJ_MIXED ? c.outer : c.confirms;
    r.relres = c.relres;
    r.hist_len = 0;
    r.nrestart_log = 0;
    r.kernel_ms = ms;
    r.passes = c.passes;
    r.grid = bt->grid;
    if (c.status < 0 && (worst >= 0 || c.status < worst)) worst = (naj_status)c.status;
    if (worst >= 0 && c.status == ST_NOT_CONVERGED) worst = NAJ_NOT_CONVERGED;
  }
  if (worst == NAJ_EBREAKDOWN) return fail(NAJ_EBREAKDOWN, "NaN/Inf in a reduction of at least one instance");
  return worst;
}

// Times each candidate tile size on one system solved alone (a batch of one) for `passes`
// passes of the batch kernel, and records the fastest for the system's features.
naj_status naj_autotune_tiles(naj_system* s, int32_t nrhs, const naj_opts* opts, int32_t passes, void* stream,
                              int32_t* best_tile) {
  g_err.clear();
  if (!s || nrhs < 1 || nrhs > kMaxRhs) return fail(NAJ_EINVAL, "bad system or nrhs");
  naj_opts o;
  if (opts) o = *opts; else naj_opts_default(&o);
  o.max_iter = std::max(1, passes);
  o.tol = 1e-300;
  o.inner_tol = 1e-300 < o.inner_tol ? o.inner_tol : 1e-4;
  o.max_refine = 1;   // mixed: one inner solve of `passes` iterations between two residual passes
  const int cands[] = {1, 2, 4, 8, 16};
  // Each item size is timed on copies of the system batched together, about 1 M rows in flight
  // (at most 64 copies): a moderately loaded GPU, between a batch's full start and its tail of a
  // few long-running systems.  Measured on the 512-system finite-element batch, the sizes picked
  // this way ran it as fast as the best single size for every system (4 slices); picks from the
  // system alone (the most, smallest items) were 12 % slower, from 4 M rows in flight 8 %, and
  // from the sum of relative times over several regimes 2-4 %.  NAJ_TUNE_ROWS lists other
  // regimes (rows in flight, 0 = the system alone; the score adds relative times).
  std::vector<int> Rs;
  {
    const char* e = getenv("NAJ_TUNE_ROWS");
    std::string spec = e ? e : "1048576";
    size_t pos = 0;
    while (pos <= spec.size()) {
      size_t c = spec.find(',', pos);
      if (c == std::string::npos) c = spec.size();
      const long long rows = atoll(spec.substr(pos, c - pos).c_str());
      Rs.push_back(rows <= 0 ? 1 : (int)std::max<int64_t>(1, std::min<int64_t>(64, rows / std::max<int64_t>(1, s->n))));
      pos = c + 1;
    }
  }
  int R = 1;
  for (int r : Rs) R = std::max(R, r);
  hipStream_t st = (hipStream_t)stream;
  double* dbuf = nullptr;
  HIP_TRY(hipMalloc((void**)&dbuf, sizeof(double) * s->n * nrhs * (1 + R)));
  HIP_TRY(hipMemsetAsync(dbuf, 0, sizeof(double) * s->n * nrhs * (1 + R), st));
  hipLaunchKernelGGL(k_fill_ones, dim3(blocks_for(s->n * nrhs, kAux * 4)), dim3(kAux), 0, st, dbuf, s->n * nrhs);
  const TuneKey key = tune_key(s, nrhs, o.precision);
  std::vector<naj_result> res((size_t)nrhs * R);
  std::vector<naj_system*> arr(R, s);
  std::vector<int32_t> k(R, nrhs);
  std::vector<const double*> bb(R, dbuf);
  std::vector<double*> xx(R);
  for (int r = 0; r < R; ++r) xx[r] = dbuf + (size_t)s->n * nrhs * (1 + r);
  std::vector<int> tried;
  std::vector<std::vector<float>> times;
  for (int T : cands) {
    if (T > std::max<int64_t>(1, s->nslices) && T != cands[0]) break;
    {
      std::lock_guard<std::mutex> g(g_tune_mu);
      g_tune[key] = T;
    }
    std::vector<float> ms(Rs.size(), 1e30f);
    for (size_t regime = 0; regime < Rs.size(); ++regime) {
      const int copies = Rs[regime];
      naj_batch* bt = nullptr;
      naj_status rc = naj_batch_create(copies, arr.data(), k.data(), &o, stream, &bt);
      if (rc != NAJ_OK) {
        (void)hipFree(dbuf);
        return rc;
      }
      for (int rep = 0; rep < 2; ++rep) {
        rc = naj_batch_solve(bt, bb.data(), nullptr, xx.data(), res.data(), stream);
        if (rc < 0 && rc != NAJ_EBREAKDOWN) {
          naj_batch_destroy(bt);
          (void)hipFree(dbuf);
          return rc;
        }
        ms[regime] = std::min(ms[regime], (float)res[0].kernel_ms);
      }
      naj_batch_destroy(bt);
    }
    tried.push_back(T);
    times.push_back(ms);
  }
  int best = tried[0];
  float best_score = 1e30f;
  for (size_t i = 0; i < tried.size(); ++i) {
    float score = 0.0f;
    for (size_t r = 0; r < Rs.size(); ++r) {
      float m = 1e30f;
      for (size_t q = 0; q < tried.size(); ++q) m = std::min(m, times[q][r]);
      score += times[i][r] / m;
    }
    if (score < best_score) {
      best_score = score;
      best = tried[i];
    }
  }
  {
    std::lock_guard<std::mutex> g(g_tune_mu);
    g_tune[key] = best;
  }
  (void)hipFree(dbuf);
  if (best_tile) *best_tile = best;
  return NAJ_OK;
}

// Tile-size table: one "layout log2n nnz_per_row nrhs precision tile" line per entry.
naj_status naj_tune_save(const char* path) {
  if (!path) return fail(NAJ_EINVAL, "path is NULL");
  FILE* f = fopen(path, "w");
  if (!f) return fail(NAJ_EINVAL, "cannot write %s", path);
  std::lock_guard<std::mutex> g(g_tune_mu);
  for (const auto& kv : g_tune)
    fprintf(f, "%d %d %d %d %d %d\n", kv.first.layout, kv.first.log2n, kv.first.nnz_row, kv.first.nrhs,
            kv.first.precision, kv.second);
  fclose(f);
  return NAJ_OK;
}

naj_status naj_tune_load(const char* path) {
  if (!path) return fail(NAJ_EINVAL, "path is NULL");
  FILE* f = fopen(path, "r");
  if (!f) return fail(NAJ_EINVAL, "cannot read %s", path);
  TuneKey k;
  int t = 0;
  std::lock_guard<std::mutex> g(g_tune_mu);
  while (fscanf(f, "%d %d %d %d %d %d", &k.layout, &k.log2n, &k.nnz_row, &k.nrhs, &k.precision, &t) == 6)
    if (t >= 1 && t <= 4096) g_tune[k] = t;
  fclose(f);
  return NAJ_OK;
}

}  // extern "C"

#include "naj_server_impl.h"
