// Persistent single-system solve kernel: every iteration of Algorithm 3 is
// one fused pass over the matrix followed by one grid barrier.  The
// workgroup that arrives last at the barrier reduces the per-workgroup
// partial sums in a fixed order and takes the scalar decisions of
// Algorithm 2 (restart test, alpha/beta, prohibition period, stopping), then
// releases the others.  Restarts never move data: they only change which of
// the three vector buffers plays x^{t-1}, x^{t-2} and x^t in the next pass.
#pragma once

#include "naj_device.h"

namespace naj {

__device__ __forceinline__ int ld_i(const int* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ double ld_d(const double* p) {
  return __hip_atomic_load(p, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Scalar control after an iteration pass that did not stop: the restart test and the
// restart/momentum branches of Algorithm 2.
__device__ inline void apply_step(const SolveArgs& a, Ctrl* c, bool restart) {
  const int t = c->t;
  if (restart) {
    c->K_re = t;
    c->K = c->K < (1 << 29) ? 2 * c->K : c->K;
    c->ell += 1;
    if (c->restarts < kRestartLogCap) c->restart_log[c->restarts] = t;
    c->restarts += 1;
    c->alpha = 1.0;
    c->beta = 0.0;
    c->beta_zero = 1;
    // y^{t+1} = x^{t-1} = P and x^t := x^{t-1}: the roles stay as they are
  } else {
    const double alpha = c->alpha;
    const double an = (1.0 + sqrt(1.0 + 4.0 * alpha * alpha)) / 2.0;
    const double beta = (alpha - 1.0) / an;
    c->alpha = an;
    c->beta = beta;
    c->beta_zero = beta == 0.0 ? 1 : 0;
    const int p = c->iP, r = c->iR, w = c->iW;
    c->iP = w;   // x^t becomes the previous iterate
    c->iR = p;   // x^{t-1} becomes the one before
    c->iW = r;   // the oldest buffer receives the next iterate
  }
  if (t >= a.max_iter) {
    c->status = ST_NOT_CONVERGED;
    c->iterations = a.max_iter;
    c->result = c->iP;
    c->relres = __builtin_nan("");
    c->phase = PH_DONE;
  } else {
    c->t = t + 1;
    c->phase = PH_ITER;
  }
}

// Runs on one thread of the last-arriving workgroup.
__device__ inline void control_update(const SolveArgs& a, Ctrl* c, double r0, double r1, double r2) {
  const int phase = c->phase;
  if (phase == PH_NORMB) {
    const double nb = sqrt(r0);
    c->nb = nb;
    if (!(nb < __builtin_inf())) {          // NaN or Inf in b
      c->status = ST_BREAKDOWN;
      c->iterations = 0;
      c->result = c->iP;
      c->phase = PH_DONE;
    } else if (nb == 0.0) {
      c->status = ST_OK;
      c->iterations = 0;
      c->result = -1;
      c->relres = 0.0;
      c->phase = PH_DONE;
    } else {
      c->phase = PH_ITER;
    }
    return;
  }
  if (phase == PH_ITER) {
    const int t = c->t;
    const double s = r0, gg = r1, sabs = r2;
    const double mon = sqrt(gg) / c->nb;
    if (a.hist && t - 1 < a.hist_cap) a.hist[t - 1] = mon;
    if (a.trace && t - 1 < a.trace_cap) {
      a.trace[2 * (t - 1)] = s;
      a.trace[2 * (t - 1) + 1] = sabs;
    }
    c->hist_len = t;
    if (!(mon < __builtin_inf()) || !(fabs(s) < __builtin_inf())) {
      c->status = ST_BREAKDOWN;
      c->iterations = t;
      c->result = c->iP;
      c->phase = PH_DONE;
      return;
    }
    if (t == 1 && mon <= a.tol) {           // y^1 = x^0 already meets the tolerance
      c->status = ST_OK;
      c->iterations = 0;
      c->result = c->iP;
      c->relres = mon;
      c->phase = PH_DONE;
      return;
    }
    const bool restart = a.restart && (t > c->K_re + c->K) && (s >= 0.0);
    if (mon <= a.tol && t >= c->last_confirm + a.confirm_gap) {
      c->last_confirm = t;
      c->pending_restart = restart ? 1 : 0;
      c->phase = PH_CONFIRM;                // residual of x^t (buffer W) next
      return;
    }
    apply_step(a, c, restart);
    return;
  }
  if (phase == PH_CONFIRM) {
    const double rho = sqrt(r0) / c->nb;
    c->confirms += 1;
    if (rho <= a.tol) {
      c->status = ST_OK;
      c->iterations = c->t;
      c->result = c->iW;
      c->relres = rho;
      c->phase = PH_DONE;
      return;
    }
    apply_step(a, c, c->pending_restart != 0);
  }
}

template <bool USER_D>
__global__ void __launch_bounds__(kBlock) k_solve64(SolveArgs a) {
  __shared__ double sh[3][kWavesPerBlock];
  __shared__ int s_phase, s_iP, s_iR, s_iW, s_bz, s_last, s_stop;
  __shared__ double s_beta;
  const int G = gridDim.x;
  const int lane = threadIdx.x % kWave;
  const WaveRange wr = wave_range(a.A.nslices, a.nxcd);
  unsigned int epoch = 0;

  for (;;) {
    if (threadIdx.x == 0) {
      s_phase = ld_i(&a.ctrl->phase);
      s_iP = ld_i(&a.ctrl->iP);
      s_iR = ld_i(&a.ctrl->iR);
      s_iW = ld_i(&a.ctrl->iW);
      s_bz = ld_i(&a.ctrl->beta_zero);
      s_beta = ld_d(&a.ctrl->beta);
    }
    __syncthreads();
    const int phase = s_phase;
    if (phase == PH_DONE) break;
    double p0 = 0.0, p1 = 0.0, p2 = 0.0;
    if (phase == PH_ITER) {
      const double* P = pick(a, s_iP);
      const double* R = pick(a, s_iR);
      double* W = pick(a, s_iW);
      const double beta = s_beta;
      const bool bz = s_bz != 0;
      for (int64_t s = wr.first; s < wr.end; s += wr.step) iter_slice<USER_D>(a, s, lane, P, R, W, beta, bz, p0, p1, p2);
    } else if (phase == PH_CONFIRM) {
      const double* X = pick(a, s_iW);
      for (int64_t s = wr.first; s < wr.end; s += wr.step) resid_slice(a.A, s, lane, X, a.b, nullptr, p0);
    } else {  // PH_NORMB
      for (int64_t s = wr.first; s < wr.end; s += wr.step) {
        const int64_t row = s * kWave + lane;
        if (row < a.A.n) {
          const double v = a.b[row];
          p0 = p0 + v * v;
        }
      }
    }
    block_sum3(p0, p1, p2, sh);
    ++epoch;
    if (threadIdx.x == 0) {
      a.part[0 * (size_t)G + blockIdx.x] = p0;
      a.part[1 * (size_t)G + blockIdx.x] = p1;
      a.part[2 * (size_t)G + blockIdx.x] = p2;
      __threadfence();
      const unsigned long long old = __hip_atomic_fetch_add(&a.bar->count, 1ULL, __ATOMIC_ACQ_REL,
                                                            __HIP_MEMORY_SCOPE_AGENT);
      s_last = (old == (unsigned long long)epoch * (unsigned long long)G - 1ULL) ? 1 : 0;
      s_stop = 0;
    }
    __syncthreads();
    if (s_last) {
      if (threadIdx.x < kWave) {
        __threadfence();
        const double r0 = grid_sum_fixed(a.part, 0, G, lane);
        const double r1 = grid_sum_fixed(a.part, 1, G, lane);
        const double r2 = grid_sum_fixed(a.part, 2, G, lane);
        if (lane == 0) {
          control_update(a, a.ctrl, r0, r1, r2);
          __threadfence();
          __hip_atomic_store(&a.bar->epoch_done, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    } else if (threadIdx.x == 0) {
      const long long t0 = wall_clock64();
      unsigned int spins = 0;
      while (__hip_atomic_load(&a.bar->epoch_done, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < epoch) {
        __builtin_amdgcn_s_sleep(1);
        if ((++spins & 255u) == 0u) {
          if (ld_i(&a.ctrl->timeout) != 0 || wall_clock64() - t0 > a.spin_ticks) {
            __hip_atomic_store(&a.ctrl->timeout, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_stop = 1;
            break;
          }
        }
      }
      __threadfence();
    }
    __syncthreads();
    if (s_stop) break;
  }
}

// Clears the control block and the barrier before a solve.
__global__ void k_solve_init(Ctrl* c, Barrier* bar, int k0) {
  if (threadIdx.x == 0 && blockIdx.x == 0) {
    c->alpha = 1.0;
    c->beta = 0.0;
    c->nb = 0.0;
    c->relres = __builtin_nan("");
    c->t = 1;
    c->K_re = 0;
    c->K = k0;
    c->ell = 0;
    c->iP = 0;
    c->iR = 1;
    c->iW = 2;
    c->beta_zero = 1;
    c->phase = PH_NORMB;
    c->last_confirm = -(1 << 30);
    c->status = ST_EDEVICE;
    c->iterations = 0;
    c->result = 0;
    c->restarts = 0;
    c->confirms = 0;
    c->pending_restart = 0;
    c->hist_len = 0;
    c->timeout = 0;
    for (int i = 0; i < kRestartLogCap; ++i) c->restart_log[i] = 0;
    bar->count = 0ULL;
    bar->epoch_done = 0u;
    bar->pad = 0u;
  }
}

// Copies the buffer the control block names as the answer into x (zeros for -1).
__global__ void k_copy_result(const Ctrl* c, const double* b0, const double* b1, const double* b2, double* x,
                              int64_t n) {
  const int r = c->result;
  const double* src = r == 0 ? b0 : (r == 1 ? b1 : b2);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[i] = r < 0 ? 0.0 : src[i];
}

}  // namespace naj
