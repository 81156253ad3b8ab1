/*
 * naj_oracle_omp.c -- CPU oracle of the float64 accelerated Jacobi-type method, threaded over rows.
 *
 * TEST INFRASTRUCTURE ONLY.  This is a second, multi-core copy of the plain oracle (naj_oracle.py's
 * accelerated_jacobi), written in C with OpenMP so that the CPU baseline can be timed as a whole solve on
 * every host core.  Only the test suite and the CPU-baseline leg of the benchmark load it; the product
 * path never does, and it shares no code with the HIP library.
 *
 * What it computes (Liang, Pang, Toh, Yang, arXiv 2407.03272):
 *   Algorithm 3 (Section 3) with the diagonal J of eq. (J-diag), J_kk = Q_kk + sum_{j != k} |Q_kj|,
 *   taken as the row absolute sum in stored order (equal for positive semidefinite Q; a zero row
 *   gets J_kk = 1):
 *       x^t = y^t - J^{-1} (Q y^t - b)                              (the Jacobi-type step)
 *       restart when IsRestart and t > K_re + K_l and <Q y^t - b, x^t - x^{t-1}> >= 0:
 *           K_re = t, K_{l+1} = 2 K_l, alpha_{t+1} = 1, y^{t+1} = x^{t-1}, x^t = x^{t-1}   (Algorithm 2)
 *       otherwise alpha_{t+1} = (1 + sqrt(1 + 4 alpha_t^2)) / 2,
 *           y^{t+1} = x^t + (alpha_t - 1)/alpha_{t+1} (x^t - x^{t-1})                  (Algorithm 1)
 *   from x^0 = y^1, alpha_1 = 1, K_re = 0.  Stop rule as the Python oracle: the monitor ||Q y^t - b|| / ||b||
 *   (free with the step); when it is <= tol (and at least confirm_gap iterations after the previous
 *   check) the residual of x^t is computed and the run stops if it is <= tol; a monitor <= tol at t = 1
 *   returns x^0 with 0 iterations.  The momentum step is x + beta * d with d = x - x^{t-1}.
 *
 * Arithmetic: each row's product adds its stored entries in order in float64, and every step is the
 * same sequence of IEEE operations as the Python oracle's (build with -ffp-contract=off), so the
 * iterates are identical whenever the restart and stop decisions are.  The reductions (restart inner
 * product, norms) add per-thread partials over contiguous row blocks in thread order: a fixed order for
 * a given thread count, which may round differently from the Python oracle's library dot products.
 */
#include <math.h>
#include <stdint.h>
#include <stdlib.h>
#include <string.h>

#include <omp.h>

#define NAJ_ORACLE_OK 0
#define NAJ_ORACLE_NOT_CONVERGED 1
#define NAJ_ORACLE_EINVAL (-1)
#define NAJ_ORACLE_ENOMEM (-2)
#define NAJ_ORACLE_BREAKDOWN (-4)

#define MAX_THREADS 1024

/* alpha_{t+1} from alpha_t (Algorithm 1). */
static double alpha_next(double alpha) { return (1.0 + sqrt(1.0 + 4.0 * alpha * alpha)) / 2.0; }

/* Row range [*lo, *hi) of thread `tid` of `nt` (contiguous blocks). */
static void rows_of(int64_t n, int tid, int nt, int64_t* lo, int64_t* hi) {
  *lo = n * tid / nt;
  *hi = n * (tid + 1) / nt;
}

/* sum of per-thread partials in thread order */
static double sum_partials(const double* part, int nt) {
  double s = 0.0;
  for (int i = 0; i < nt; ++i) s = s + part[i];
  return s;
}

/* ||b - Q x||^2 with per-thread partials */
static double resid_norm2(int64_t n, const int32_t* rp, const int32_t* ci, const double* va, const double* x,
                          const double* b, int nt, double* part) {
#pragma omp parallel num_threads(nt)
  {
    const int tid = omp_get_thread_num();
    int64_t lo, hi;
    rows_of(n, tid, nt, &lo, &hi);
    double acc = 0.0;
    for (int64_t i = lo; i < hi; ++i) {
      double u = 0.0;
      for (int32_t k = rp[i]; k < rp[i + 1]; ++k) u = u + va[k] * x[ci[k]];
      const double r = b[i] - u;
      acc = acc + r * r;
    }
    part[tid] = acc;
  }
  return sum_partials(part, nt);
}

/*
 * Solve Q x = b (host CSR, float64) by Algorithm 3.
 *   x0            : starting point or NULL (zero)
 *   nthreads      : threads to use (<= 0: OpenMP's default)
 *   x             : [n] answer (the accepted x^t, or the last iterate x^{t-1} when not converged)
 *   iterations    : t of the accepted x^t (0 = x^0 accepted)
 *   nrestarts     : restarts fired; restart_log[0 .. min(nrestarts, log_cap)) their iterations
 *   hist          : monitor per iteration (hist_cap entries at most), may be NULL
 *   hist_len      : entries of the monitor written
 *   relres        : ||b - Q x|| / ||b|| of the returned x when it was confirmed or computed, else NaN
 *   seconds       : wall time of the iteration loop (setup of J and the buffers excluded)
 *   threads_used  : the thread count of the parallel regions
 * Returns NAJ_ORACLE_OK, NAJ_ORACLE_NOT_CONVERGED, NAJ_ORACLE_BREAKDOWN, or a negative error.
 */
int naj_oracle_solve(int64_t n, const int32_t* rowptr, const int32_t* colidx, const double* vals, const double* b,
                     const double* x0, double tol, int32_t max_iter, int32_t restart, int32_t k0,
                     int32_t confirm_gap, int32_t nthreads, double* x, int32_t* iterations, int32_t* nrestarts,
                     int32_t* restart_log, int32_t log_cap, double* hist, int32_t hist_cap, int32_t* hist_len,
                     double* relres, double* seconds, int32_t* threads_used) {
  if (n < 1 || !rowptr || !b || !x || !iterations || !nrestarts || !hist_len || !relres || !seconds ||
      !threads_used || max_iter < 1 || k0 < 2 || confirm_gap < 1 || !(tol > 0.0))
    return NAJ_ORACLE_EINVAL;
  int nt = nthreads > 0 ? nthreads : omp_get_max_threads();
  if (nt > MAX_THREADS) nt = MAX_THREADS;
  if (nt > n) nt = (int)n;
  *threads_used = nt;
  *iterations = 0;
  *nrestarts = 0;
  *hist_len = 0;
  *relres = NAN;
  *seconds = 0.0;

  double* dinv = (double*)malloc(sizeof(double) * n);
  double* y = (double*)malloc(sizeof(double) * n);
  double* xp = (double*)malloc(sizeof(double) * n);   /* x^{t-1} */
  double* xn = (double*)malloc(sizeof(double) * n);   /* x^t */
  double part0[MAX_THREADS], part1[MAX_THREADS];
  if (!dinv || !y || !xp || !xn) {
    free(dinv), free(y), free(xp), free(xn);
    return NAJ_ORACLE_ENOMEM;
  }
  int status = NAJ_ORACLE_NOT_CONVERGED;
  double nb2;
  /* J of eq. (J-diag) as the row absolute sum in stored order, zero rows -> 1; x^0; ||b||^2 */
#pragma omp parallel num_threads(nt)
  {
    const int tid = omp_get_thread_num();
    int64_t lo, hi;
    rows_of(n, tid, nt, &lo, &hi);
    double acc = 0.0;
    for (int64_t i = lo; i < hi; ++i) {
      double a = 0.0;
      for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k) a = a + fabs(vals[k]);
      if (a == 0.0) a = 1.0;
      dinv[i] = 1.0 / a;
      const double v = x0 ? x0[i] : 0.0;
      xp[i] = v;
      y[i] = v;
      acc = acc + b[i] * b[i];
    }
    part0[tid] = acc;
  }
  nb2 = sum_partials(part0, nt);
  const double nb = sqrt(nb2);
  if (nb == 0.0) {
    memset(x, 0, sizeof(double) * n);
    *relres = 0.0;
    free(dinv), free(y), free(xp), free(xn);
    return NAJ_ORACLE_OK;
  }

  const double t0 = omp_get_wtime();
  double alpha = 1.0;
  int64_t K_re = 0, K = k0;
  int64_t last_confirm = -((int64_t)1 << 62);
  for (int32_t t = 1; t <= max_iter; ++t) {
    /* x^t = y^t - J^{-1}(Q y^t - b) and the partial sums of ||g||^2 and <g, x^t - x^{t-1}> */
#pragma omp parallel num_threads(nt)
    {
      const int tid = omp_get_thread_num();
      int64_t lo, hi;
      rows_of(n, tid, nt, &lo, &hi);
      double s = 0.0, gg = 0.0;
      for (int64_t i = lo; i < hi; ++i) {
        double u = 0.0;
        for (int32_t k = rowptr[i]; k < rowptr[i + 1]; ++k) u = u + vals[k] * y[colidx[k]];
        const double g = u - b[i];
        const double xi = y[i] - dinv[i] * g;
        xn[i] = xi;
        const double d = xi - xp[i];
        s = s + g * d;
        gg = gg + g * g;
      }
      part0[tid] = s;
      part1[tid] = gg;
    }
    const double s = sum_partials(part0, nt);
    const double mon = sqrt(sum_partials(part1, nt)) / nb;
    if (hist && t - 1 < hist_cap) {
      hist[t - 1] = mon;
      *hist_len = t;
    }
    if (!isfinite(mon)) {
      memcpy(x, xp, sizeof(double) * n);
      *iterations = t;
      status = NAJ_ORACLE_BREAKDOWN;
      break;
    }
    if (t == 1 && mon <= tol) {   /* y^1 = x^0 already meets the tolerance */
      memcpy(x, xp, sizeof(double) * n);
      *iterations = 0;
      *relres = mon;
      status = NAJ_ORACLE_OK;
      break;
    }
    if (mon <= tol && t >= last_confirm + confirm_gap) {
      const double rho = sqrt(resid_norm2(n, rowptr, colidx, vals, xn, b, nt, part0)) / nb;
      last_confirm = t;
      if (rho <= tol) {
        memcpy(x, xn, sizeof(double) * n);
        *iterations = t;
        *relres = rho;
        status = NAJ_ORACLE_OK;
        break;
      }
    }
    if (!isfinite(s)) {
      memcpy(x, xp, sizeof(double) * n);
      *iterations = t;
      status = NAJ_ORACLE_BREAKDOWN;
      break;
    }
    double an;
    if (restart && t > K_re + K && s >= 0.0) {
      /* restart branch: y^{t+1} = x^{t-1}; x^t := x^{t-1} (x^{t-1} stays the previous iterate) */
      K_re = t;
      K = 2 * K;
      if (*nrestarts < log_cap && restart_log) restart_log[*nrestarts] = t;
      *nrestarts += 1;
      an = 1.0;
      memcpy(y, xp, sizeof(double) * n);
    } else {
      /* momentum branch: y^{t+1} = x^t + beta_t (x^t - x^{t-1}) */
      an = alpha_next(alpha);
      const double beta = (alpha - 1.0) / an;
#pragma omp parallel for num_threads(nt) schedule(static)
      for (int64_t i = 0; i < n; ++i) {
        const double d = xn[i] - xp[i];
        y[i] = xn[i] + beta * d;
      }
      double* tmp = xp;
      xp = xn;
      xn = tmp;
    }
    alpha = an;
    if (t == max_iter) {
      memcpy(x, xp, sizeof(double) * n);
      *iterations = max_iter;
      status = NAJ_ORACLE_NOT_CONVERGED;
      *relres = sqrt(resid_norm2(n, rowptr, colidx, vals, x, b, nt, part0)) / nb;
    }
  }
  *seconds = omp_get_wtime() - t0;
  free(dinv), free(y), free(xp), free(xn);
  return status;
}
