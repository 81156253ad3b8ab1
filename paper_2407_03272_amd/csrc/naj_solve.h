// Solve kernels.  Every iteration of Algorithm 3 is one fused pass over the
// matrix (product, Jacobi-type step and the partial sums of the restart
// inner product and the residual monitor) followed by one scalar decision:
// the restart test and the restart/momentum branches of Algorithm 2, or the
// stopping test.  The decision is taken from the per-workgroup partial sums
// added in a fixed order, so every run of the same system takes the same
// decisions.  Restarts never move data: they only change which of three
// vector buffers plays x^{t-1}, x^{t-2} and x^t in the next pass.
//
// Two drivers share the pass:
//  * k_pass64: one launch per pass (every system above about 24 slices).
//    Kernel boundaries order the passes; every workgroup of launch k takes
//    the decision after pass k-1 itself, at its start.
//  * k_solve64: one persistent launch per solve.  With a single workgroup
//    the passes are separated by workgroup barriers only (tiny systems);
//    with several co-resident workgroups by a counting grid barrier (an
//    option, NAJ_MODE=2).
#pragma once

#include "naj_device.h"

namespace naj {

constexpr double kStallArm = 0.5;   // inner monitor level from which the stall test applies

__device__ __forceinline__ double alpha_next(double alpha) { return (1.0 + sqrt(1.0 + 4.0 * alpha * alpha)) / 2.0; }

// Materialized momentum form: after the roles of a pass are settled, fix the
// coefficient of y^{t+1} the next pass writes, (alpha_t - 1)/alpha_{t+1} with
// alpha_t = c->alpha (the value Algorithm 2 uses if that pass does not restart),
// and the buffer receiving it (-1 when the coefficient is 0: then y^{t+1} = x^t).
__device__ inline void ymode_plan_next(Ctrl* c) {
  const double bn = (c->alpha - 1.0) / alpha_next(c->alpha);
  c->beta_next = bn;
  c->iYn = bn == 0.0 ? -1 : (c->beta_zero ? 2 : (c->iR == 2 ? 3 : 2));
}

// The same with the y buffers chosen by the parity of the pass count (consecutive inner passes
// alternate between buffers 2 and 3, so the buffer read is never the one written).
__device__ inline void ymode_plan_parity(Ctrl* c) {
  const double bn = (c->alpha - 1.0) / alpha_next(c->alpha);
  c->beta_next = bn;
  c->iYn = bn == 0.0 ? -1 : 2 + (c->passes & 1);
}

// Roles after a pass that did not restart, materialized form: x^t becomes the previous
// iterate, and y^{t+1} is the buffer just written (or x^t itself).
__device__ inline void ymode_advance(Ctrl* c) {
  const int p = c->iP;
  c->iP = c->iW;
  c->iW = p;
  if (c->iYn >= 0) {
    c->iR = c->iYn;
    c->beta_zero = 0;
  } else {
    c->beta_zero = 1;
  }
}

// Scalar control after an iteration pass that did not stop: the restart and
// momentum branches of Algorithm 2, then the iteration cap.
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
    const double an = alpha_next(alpha);
    const double beta = (alpha - 1.0) / an;
    c->alpha = an;
    c->beta = beta;
    if (a.ymode) {
      ymode_advance(c);
    } else {
      c->beta_zero = beta == 0.0 ? 1 : 0;
      const int p = c->iP, r = c->iR, w = c->iW;
      c->iP = w;   // x^t becomes the previous iterate
      c->iR = p;   // x^{t-1} becomes the one before
      c->iW = r;   // the oldest buffer receives the next iterate
    }
  }
  if (a.ymode) ymode_plan_next(c);
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

// Mixed precision, after a float64 residual pass (refinement step k = c->outer):
// accept x, give up, or start a float32 inner solve of Q d = fl32(r) from d = 0.
__device__ inline void mixed_after_residual(const SolveArgs& a, Ctrl* c, double rr, double r32sq, bool side) {
  if (c->update) {               // the pass wrote x + d into iXn: it is the current iterate now
    const int t = c->iX;
    c->iX = c->iXn;
    c->iXn = t;
    c->update = 0;
  }
  const int k = c->outer;
  const double rho = sqrt(rr) / c->nb;
  c->outer = k + 1;
  if (side && a.hist && k < a.hist_cap) a.hist[k] = rho;
  c->hist_len = k + 1;
  c->relres = rho;
  c->result = c->iX;
  if (!(rho < __builtin_inf())) {
    c->status = ST_BREAKDOWN;
    c->phase = PH_DONE;
    return;
  }
  if (rho <= a.tol) {
    c->status = ST_OK;
    c->phase = PH_DONE;
    return;
  }
  c->nr = sqrt(r32sq);
  if (k >= a.max_refine || c->nr == 0.0) {   // refinement budget spent, or nothing left to correct in float32
    c->status = ST_NOT_CONVERGED;
    c->phase = PH_DONE;
    return;
  }
  c->t = 1;
  c->alpha = 1.0;
  c->beta = 0.0;
  c->beta_zero = 1;
  c->zp = 1;
  c->best_mon = __builtin_inf();
  c->best_t = 0;
  c->K_re = 0;
  c->K = a.k0;
  c->ell = 0;
  if (a.ymode) {
    c->iP = 0;
    c->iW = 1;
    c->iR = 2;
    ymode_plan_next(c);
  } else {
    c->iP = 0;
    c->iR = 1;
    c->iW = 2;
  }
  c->phase = PH_INNER32;
}

__device__ inline void mixed_finish_inner(const SolveArgs& a, Ctrl* c, int d_buf, int its, bool side) {
  const int k = c->outer - 1;
  if (side && a.trace && k < a.trace_cap) {
    a.trace[2 * k] = (double)its;
    a.trace[2 * k + 1] = (double)c->ell;
  }
  c->inner_total += its;
  c->inner_restarts += c->ell;
  c->iD = d_buf;
  c->update = 1;
  c->phase = PH_RESID64;
}

// Mixed precision, after a float32 inner pass: the inner solve's stop test, then
// the restart test and the restart/momentum branches of Algorithm 2.
__device__ inline void mixed_after_inner(const SolveArgs& a, Ctrl* c, double s, double gg, double sabs, bool side) {
  (void)sabs;
  const int t = c->t;
  const double mon = sqrt(gg) / c->nr;
  if (!(mon < __builtin_inf()) || !(fabs(s) < __builtin_inf())) {
    c->status = ST_BREAKDOWN;
    c->result = c->iX;
    c->phase = PH_DONE;
    return;
  }
  if (mon <= a.inner_tol) {
    mixed_finish_inner(a, c, c->iW, t, side);     // d = x^t
    return;
  }
  if (mon <= 0.9 * c->best_mon) {
    c->best_mon = mon;
    c->best_t = t;
  }
  // the stall test applies once the monitor has halved (before that a plateau is the slow
  // start on a smooth right-hand side, not the float32 rounding level)
  if (a.inner_stall > 0 && c->best_mon <= kStallArm && t - c->best_t >= a.inner_stall) {
    mixed_finish_inner(a, c, c->iW, t, side);     // stalled at the float32 rounding level: d = x^t
    return;
  }
  const bool restart = a.restart && (t > c->K_re + c->K) && (s >= 0.0);
  if (restart) {
    c->K_re = t;
    c->K = c->K < (1 << 29) ? 2 * c->K : c->K;
    c->ell += 1;
    c->alpha = 1.0;
    c->beta = 0.0;
    c->beta_zero = 1;
  } else {
    const double alpha = c->alpha;
    const double an = alpha_next(alpha);
    const double beta = (alpha - 1.0) / an;
    c->alpha = an;
    c->beta = beta;
    if (a.ymode) {
      ymode_advance(c);
    } else {
      c->beta_zero = beta == 0.0 ? 1 : 0;
      const int p = c->iP, r = c->iR, w = c->iW;
      c->iP = w;
      c->iR = p;
      c->iW = r;
    }
    c->zp = 0;
  }
  if (a.ymode) {
    if (a.ypar) ymode_plan_parity(c);
    else ymode_plan_next(c);
  }
  if (t >= a.max_iter) {
    mixed_finish_inner(a, c, c->iP, a.max_iter, side);   // d = the last iterate
    return;
  }
  c->t = t + 1;
}

// A cancel request (a nonzero word in host-visible memory, written by the caller's host thread) ends the
// solve at the pass boundary where it is seen, after that pass's decision: the result is the float64
// iterate the solve holds (x^{t-1} role, or the refinement's current x), as for the iteration cap.
__device__ inline void check_cancel(const SolveArgs& a, Ctrl* c) {
  if (!a.cancel || c->phase == PH_DONE || (c->passes % kCancelEvery) != 0) return;
  if (__hip_atomic_load(a.cancel, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM) == 0) return;
  c->status = ST_CANCELLED;
  if (a.precision) {
    c->result = c->iX;
  } else {
    c->result = c->iP;
    c->iterations = c->t - 1;
  }
  c->relres = __builtin_nan("");
  c->phase = PH_DONE;
}

__device__ inline void control_update_pass(const SolveArgs& a, Ctrl* c, double r0, double r1, double r2, bool side);

// The decision after a pass, from its three reduced sums, then the cancel check.  One thread runs
// it.  With side false only the control state is updated: the residual history, the trace and the
// cancel word are left to the one copy of the decision whose state is published (see k_pass64).
__device__ inline void control_update(const SolveArgs& a, Ctrl* c, double r0, double r1, double r2,
                                      bool side = true) {
  control_update_pass(a, c, r0, r1, r2, side);
  if (side) check_cancel(a, c);
}

// The decision after a pass, from its three reduced sums.
__device__ inline void control_update_pass(const SolveArgs& a, Ctrl* c, double r0, double r1, double r2, bool side) {
  const int phase = c->phase;
  c->passes += 1;
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
      c->phase = a.precision ? PH_RESID64 : PH_ITER;
    }
    return;
  }
  if (phase == PH_RESID64) {
    mixed_after_residual(a, c, r0, r1, side);
    return;
  }
  if (phase == PH_INNER32) {
    mixed_after_inner(a, c, r0, r1, r2, side);
    return;
  }
  if (phase == PH_ITER) {
    const int t = c->t;
    const double s = r0, gg = r1, sabs = r2;
    // monitor at y^t: relative residual, or relative objective gap (gg then holds f(y^t))
    const double mon = a.stop_obj ? fabs(gg - a.fstar) / a.fscale : sqrt(gg) / c->nb;
    if (side && a.hist && t - 1 < a.hist_cap) a.hist[t - 1] = mon;
    if (side && a.trace && t - 1 < a.trace_cap) {
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
    const double rho = a.stop_obj ? fabs(r0 - a.fstar) / a.fscale : sqrt(r0) / c->nb;
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

// Control fields a pass needs, staged in LDS by thread 0.
struct PassView {
  int phase, iP, iR, iW, bz, zp, iX, iXn, iD, update, iYn;
  double beta, beta_next;
};

__device__ __forceinline__ void load_view(const Ctrl* c, PassView* v) {
  v->phase = c->phase;
  v->iP = c->iP;
  v->iR = c->iR;
  v->iW = c->iW;
  v->bz = c->beta_zero;
  v->beta = c->beta;
  v->zp = c->zp;
  v->iX = c->iX;
  v->iXn = c->iXn;
  v->iD = c->iD;
  v->update = c->update;
  v->iYn = c->iYn;
  v->beta_next = c->beta_next;
}

// The rows one wave takes in a pass.  With an item list (A.witem, built for this launch shape: balanced
// lists on the sorted layout, blocked slice orders on the regular layout) the wave sweeps its own list
// of long rows and slices; otherwise the long rows are strided over every wave of the grid, then the
// wave takes its slice range.  `longs` is false where the kernel instance has no long-row path (block
// J, whose layout has no long rows).  LISTS: the instance carries the list path: the materialized-
// momentum instances, which the sorted layout runs, and the float64 passes of the instances that read
// 4-byte values (the others keep their register budget and ignore the lists).
template <int BS, bool LISTS, class LongFn, class SliceFn>
__device__ __forceinline__ void for_wave_items(const Sell& A, int nxcd, bool longs, LongFn&& fl, SliceFn&& fs) {
  if (LISTS && A.witem) {
    const NAJ_CONST int32_t* off = (const NAJ_CONST int32_t*)A.woff;
    const NAJ_CONST int32_t* item = (const NAJ_CONST int32_t*)A.witem;
    const int w = (int)blockIdx.x * (BS / kWave) + wave_id();
    const int e = off[w + 1];
    for (int i = off[w]; i < e; ++i) {
      const int64_t it = item[i];
      if (it < A.n_long) {
        if (longs) fl(it);
      } else {
        fs(it - A.n_long);
      }
    }
    return;
  }
  if (longs) {
    const LongRange<BS> lr;
    for (int64_t r = lr.first; r < A.n_long; r += lr.step) fl(r);
  }
  const WaveRange wr = wave_range<BS>(A, nxcd);
  for (int64_t s = wr.first; s < wr.end; s += wr.step) fs(s);
}

// The workgroup's share of one float64 iteration pass (long rows, then slices).  YM: the
// materialized momentum form (a compile-time choice, so the two-iterate kernel carries none
// of the materialized form's code).
template <int JM, int BS, bool YM, bool NT = false, bool V32 = false>
__device__ __forceinline__ void pass_iter64(const SolveArgs& a, const double* P, const Momentum<double>& m, double* W,
                                            double& p0, double& p1, double& p2) {
  const int lane = threadIdx.x % kWave;
  // a block J uses the regular layout: no long rows
  for_wave_items<BS, YM || V32>(
      a.A, a.nxcd, JM != kJBlock,
      [&](int64_t r) {
        if constexpr (JM != kJBlock) iter_long<JM, YM, NT, V32>(a, r, lane, P, m, W, p0, p1, p2);
      },
      [&](int64_t s) { iter_slice<JM, YM, NT, V32>(a, s, lane, P, m, W, p0, p1, p2); });
}

// The workgroup's share of r = b - Q X (float64); ||r||^2 in p0 (with obj: f(X)).
template <int BS, bool LISTS = false, bool V32 = false>
__device__ __forceinline__ void pass_resid64(const Sell& A, int nxcd, const double* X, const double* b, double* out,
                                             double& p0, bool obj = false) {
  const int lane = threadIdx.x % kWave;
  for_wave_items<BS, LISTS>(
      A, nxcd, true, [&](int64_t r) { resid_long<V32>(A, r, lane, X, b, out, p0, obj); },
      [&](int64_t s) { resid_slice<V32>(A, s, lane, X, b, out, p0, obj); });
}

// Phases a kernel instance carries (template parameter PS of run_pass and k_pass64): every phase, or
// those of float64 solves only (norm of b, iteration, confirmation), or those of mixed-precision solves
// only (norm of b, float64 residual, float32 inner pass).  An instance's register budget is that of
// the heaviest phase it carries.
constexpr int kPhasesAll = 0, kPhasesFp64 = 1, kPhasesMixed = 2;

// The workgroup's share of one pass; partial sums in p0..p2 (per thread).
template <int JM, int BS, bool YM, bool NT = false, int PS = kPhasesAll, bool V32 = false>
__device__ __forceinline__ void run_pass(const SolveArgs& a, const PassView& v, double& p0, double& p1,
                                         double& p2) {
  const int lane = threadIdx.x % kWave;
  constexpr bool F64 = PS != kPhasesMixed, MX = PS != kPhasesFp64;
  if (F64 && v.phase == PH_ITER) {
    Momentum<double> m;
    m.R = pick(a, v.iR);
    m.Yn = (YM && v.iYn >= 0) ? pick(a, v.iYn) : nullptr;
    m.beta = v.beta;
    m.beta_next = v.beta_next;
    m.bz = v.bz != 0;
    m.ym = YM;
    pass_iter64<JM, BS, YM, NT, V32>(a, pick(a, v.iP), m, pick(a, v.iW), p0, p1, p2);
  } else if (F64 && v.phase == PH_CONFIRM) {
    pass_resid64<BS, YM || V32, V32>(a.A, a.nxcd, pick(a, v.iW), a.b, nullptr, p0, a.stop_obj != 0);
  } else if (MX && v.phase == PH_INNER32) {
    const float* P = pickf(a, v.iP);
    float* W = pickf(a, v.iW);
    Momentum<float> m;
    m.R = pickf(a, v.iR);
    m.Yn = (YM && v.iYn >= 0) ? pickf(a, v.iYn) : nullptr;
    m.beta = (float)v.beta;
    m.beta_next = (float)v.beta_next;
    m.bz = v.bz != 0;
    m.ym = YM;
    const bool zp = v.zp != 0;
    for_wave_items<BS, YM>(
        a.A, a.nxcd, JM != kJBlock,
        [&](int64_t r) {
          if constexpr (JM != kJBlock) inner_long<JM, YM, NT>(a, r, lane, P, m, W, zp, p0, p1, p2);
        },
        [&](int64_t s) { inner_slice<JM, YM, NT>(a, s, lane, P, m, W, zp, p0, p1, p2); });
  } else if (MX && v.phase == PH_RESID64) {
    const double* X = pick(a, v.iX);
    const float* D = v.update ? pickf(a, v.iD) : nullptr;
    double* Xn = v.update ? pick(a, v.iXn) : nullptr;
    for_wave_items<BS, YM>(
        a.A, a.nxcd, true, [&](int64_t r) { resid_mixed_long<V32>(a, r, lane, X, D, Xn, p0, p1); },
        [&](int64_t s) { resid_mixed_slice<V32>(a, s, lane, X, D, Xn, p0, p1); });
  } else if (v.phase == PH_NORMB) {  // every row, flat
    for (int64_t i = (int64_t)blockIdx.x * BS + threadIdx.x; i < a.A.n; i += (int64_t)gridDim.x * BS) {
      const double x = a.b[i];
      p0 = p0 + x * x;
    }
  }
}

// Sums of the G per-workgroup partial sums of a pass, in a fixed order: thread i adds slots i, i + BS,
// i + 2 BS, ... in turn, then the workgroup's threads are combined by block_sum3.  Every workgroup that
// runs it gets the same three values (in thread 0).  issue() starts the loads of up to four slots per
// thread, so that they travel together with the other loads at the start of a launch; combine() adds
// them (and, for G > 4 BS, loads and adds the slots in groups of four itself).
template <int BS>
struct PartSums {
  double v[4][3];

  __device__ __forceinline__ void issue(const double* __restrict__ part, int G) {
    if (G > 4 * BS) return;
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int j = threadIdx.x + q * BS;
#pragma unroll
      for (int k = 0; k < 3; ++k) v[q][k] = j < G ? part[(size_t)j * kPartStride + k] : 0.0;
    }
  }

  __device__ __forceinline__ void combine(const double* __restrict__ part, int G, double& r0, double& r1,
                                          double& r2, double (*sh)[BS / kWave]) {
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    if (G <= 4 * BS) {
#pragma unroll
      for (int q = 0; q < 4; ++q)
        if ((int)threadIdx.x + q * BS < G) {
          s0 = s0 + v[q][0];
          s1 = s1 + v[q][1];
          s2 = s2 + v[q][2];
        }
    } else {
      int i = threadIdx.x;
      for (; i + 3 * BS < G; i += 4 * BS) {
        double w[4][3];
#pragma unroll
        for (int q = 0; q < 4; ++q)
#pragma unroll
          for (int k = 0; k < 3; ++k) w[q][k] = part[(size_t)(i + q * BS) * kPartStride + k];
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          s0 = s0 + w[q][0];
          s1 = s1 + w[q][1];
          s2 = s2 + w[q][2];
        }
      }
      for (; i < G; i += BS) {
        const double* p = part + (size_t)i * kPartStride;
        const double a0 = p[0], a1 = p[1], a2 = p[2];
        s0 = s0 + a0;
        s1 = s1 + a1;
        s2 = s2 + a2;
      }
    }
    r0 = s0;
    r1 = s1;
    r2 = s2;
    block_sum3<BS>(r0, r1, r2, sh);
  }
};

// One pass per launch; launch k of a solve (k = 0, 1, ...) runs pass k.  The scalar decision after
// pass k-1 is taken at the start of launch k by every workgroup, each from the same two inputs: the
// control state C_{k-1} (in ctrl[(k-1) & 1]; launch 0 reads the initial state from ctrl[1]) and the
// per-workgroup partial sums of pass k-1 (in the half (k-1) & 1 of part), added in one fixed order.
// So every workgroup reaches the same state C_k without waiting for any other workgroup of its own
// launch: the kernel boundary between launches k-1 and k is the only synchronization.  Workgroup 0
// alone publishes C_k into ctrl[k & 1] (read by launch k+1 and by the host) and writes the residual
// history, the trace and the cancel decision.  A cancel therefore reaches only workgroup 0's copy
// of C_k; the other workgroups may still run pass k, into buffers that are not the result, and
// launch k+1 reads the published state.  Launches after the solve has finished copy the finished
// state forward and return.
// The launch passes k itself for k < 3 and any value of the same parity above 0 beyond (only k > 0
// and k & 1 matter).  With `flag` set, workgroup 0 also stores the phase of C_k there (a host-visible
// word the host polls instead of copying the control block back).
// Instances: J mode, block size, momentum form (YM), non-temporal matrix loads (NT), the phases carried
// (PS), and V32: the float64 passes read the float32 copy of the values, which the host uses only when
// that copy holds every value exactly (the products are then those of the 8-byte values).
template <int JM, int BS, bool YM, bool NT = false, int PS = kPhasesAll, bool V32 = false>
__global__ void __launch_bounds__(BS) k_pass64(SolveArgs a, int k, int* flag) {
  __shared__ double sh[3][BS / kWave];
  __shared__ PassView v;
  __shared__ Ctrl c;
  const int G = gridDim.x;
  const int prev = (k + 1) & 1;
  // the partial sums' loads and the control block's go out together: one memory round trip
  const double* __restrict__ part_prev = a.part + (size_t)prev * G * kPartStride;
  PartSums<BS> ps;
  if (k > 0) ps.issue(part_prev, G);
  {
    const uint32_t* src = (const uint32_t*)(a.ctrl + prev);
    uint32_t* dst = (uint32_t*)&c;
    for (int i = threadIdx.x; i < (int)(sizeof(Ctrl) / 4); i += BS) dst[i] = src[i];
  }
  double r0 = 0.0, r1 = 0.0, r2 = 0.0;
  if (k > 0) ps.combine(part_prev, G, r0, r1, r2, sh);
  __syncthreads();
  if (threadIdx.x == 0) {
    if (k > 0 && c.phase != PH_DONE) control_update(a, &c, r0, r1, r2, blockIdx.x == 0);
    load_view(&c, &v);
  }
  __syncthreads();
  if (blockIdx.x == 0) {
    const uint32_t* src = (const uint32_t*)&c;
    uint32_t* dst = (uint32_t*)(a.ctrl + (k & 1));
    for (int i = threadIdx.x; i < (int)(sizeof(Ctrl) / 4); i += BS) dst[i] = src[i];
    if (flag && threadIdx.x == 0) __hip_atomic_store(flag, v.phase, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_SYSTEM);
  }
  if (v.phase == PH_DONE) return;
  double p0 = 0.0, p1 = 0.0, p2 = 0.0;
  run_pass<JM, BS, YM, NT, PS, V32>(a, v, p0, p1, p2);
  block_sum3<BS>(p0, p1, p2, sh);
  if (threadIdx.x == 0) {
    double* slot = a.part + ((size_t)(k & 1) * G + blockIdx.x) * kPartStride;
    slot[0] = p0;
    slot[1] = p1;
    slot[2] = p2;
  }
}

// One persistent launch per solve (see the file comment).
template <int JM, int BS, bool YM>
__global__ void __launch_bounds__(BS) k_solve64(SolveArgs a) {
  __shared__ double sh[3][BS / kWave];
  __shared__ PassView v;
  __shared__ int s_last, s_stop;
  const int G = gridDim.x;
  const int lane = threadIdx.x % kWave;
  unsigned int epoch = 0;
  for (;;) {
    if (threadIdx.x == 0) {
      if (G == 1) {
        load_view(a.ctrl, &v);
      } else {
        v.phase = __hip_atomic_load(&a.ctrl->phase, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        v.iP = __hip_atomic_load(&a.ctrl->iP, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        v.iR = __hip_atomic_load(&a.ctrl->iR, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        v.iW = __hip_atomic_load(&a.ctrl->iW, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        v.bz = __hip_atomic_load(&a.ctrl->beta_zero, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        v.beta = __hip_atomic_load(&a.ctrl->beta, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        v.zp = __hip_atomic_load(&a.ctrl->zp, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        v.iX = __hip_atomic_load(&a.ctrl->iX, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        v.iXn = __hip_atomic_load(&a.ctrl->iXn, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        v.iD = __hip_atomic_load(&a.ctrl->iD, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        v.update = __hip_atomic_load(&a.ctrl->update, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        v.iYn = __hip_atomic_load(&a.ctrl->iYn, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        v.beta_next = __hip_atomic_load(&a.ctrl->beta_next, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
    }
    __syncthreads();
    if (v.phase == PH_DONE) break;
    double p0 = 0.0, p1 = 0.0, p2 = 0.0;
    run_pass<JM, BS, YM>(a, v, p0, p1, p2);
    block_sum3<BS>(p0, p1, p2, sh);
    if (G == 1) {
      // single workgroup: every wave runs on this CU, a workgroup barrier orders the passes
      if (threadIdx.x == 0) control_update(a, a.ctrl, p0, p1, p2);
      __syncthreads();
      continue;
    }
    ++epoch;
    if (threadIdx.x == 0) {
      double* slot = a.part + (size_t)blockIdx.x * kPartStride;
      slot[0] = p0;
      slot[1] = p1;
      slot[2] = p2;
      const unsigned long long old =
          __hip_atomic_fetch_add(&a.bar->count, 1ULL, __ATOMIC_ACQ_REL, __HIP_MEMORY_SCOPE_AGENT);
      s_last = (old == (unsigned long long)epoch * (unsigned long long)G - 1ULL) ? 1 : 0;
      s_stop = 0;
    }
    __syncthreads();
    if (s_last) {
      if (threadIdx.x < kWave) {
        double r0, r1, r2;
        grid_sum3(a.part, G, lane, r0, r1, r2);
        if (lane == 0) {
          control_update(a, a.ctrl, r0, r1, r2);
          __hip_atomic_store(&a.bar->epoch_done, epoch, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    } else if (threadIdx.x == 0) {
      const long long t0 = wall_clock64();
      unsigned int spins = 0;
      while (__hip_atomic_load(&a.bar->epoch_done, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) < epoch) {
        __builtin_amdgcn_s_sleep(1);
        if (a.spin_ticks == 0 || (++spins & 255u) == 0u) {
          if (a.spin_ticks == 0 ||
              __hip_atomic_load(&a.ctrl->timeout, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != 0 ||
              wall_clock64() - t0 > a.spin_ticks) {
            __hip_atomic_store(&a.ctrl->timeout, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            s_stop = 1;
            break;
          }
        }
      }
    }
    __syncthreads();
    if (s_stop) break;
  }
}

// Clears the control blocks, the barrier and the arrival counters before a solve.  ctrl[0] and
// ctrl[1] both receive the initial state: the single-launch drivers use ctrl[0]; the per-pass driver
// reads the state before its first launch from ctrl[1].
__global__ void k_solve_init(Ctrl* ctrl, Barrier* bar, unsigned int* counters, int k0, int ymode) {
  for (int i = threadIdx.x; i <= kMaxDomains; i += blockDim.x) counters[(size_t)i * kCounterStride] = 0u;
  if (threadIdx.x < 2 && blockIdx.x == 0) {
    Ctrl* c = ctrl + threadIdx.x;
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
    c->passes = 0;
    c->zp = 0;
    c->iX = 0;
    c->iXn = 1;
    c->iD = 0;
    c->update = 0;
    c->outer = 0;
    c->inner_total = 0;
    c->inner_restarts = 0;
    c->nr = 0.0;
    c->iYn = -1;
    c->beta_next = 0.0;
    if (ymode) {   // x buffers 0/1, y buffers 2/3
      c->iP = 0;
      c->iW = 1;
      c->iR = 2;
      ymode_plan_next(c);
    }
    for (int i = 0; i < kRestartLogCap; ++i) c->restart_log[i] = 0;
    if (threadIdx.x == 0) {
      bar->count = 0ULL;
      bar->epoch_done = 0u;
      bar->pad = 0u;
    }
  }
}

// Copies the buffer the control block names as the answer into x (zeros for -1).
// With perm (irregular layout) the solver's row i is the caller's row perm[i].
__global__ void k_copy_result(const Ctrl* c, const double* b0, const double* b1, const double* b2, double* x,
                              const int32_t* perm, int64_t n) {
  const int r = c->result;
  const double* src = r == 0 ? b0 : (r == 1 ? b1 : b2);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    x[perm ? perm[i] : i] = r < 0 ? 0.0 : src[i];
}

// Copies the phase word (for the host's stop check) into a small host-visible slot.
__global__ void k_peek_phase(const Ctrl* c, int* dst) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *dst = c->phase;
}

// Small systems whose vectors fit in LDS: one workgroup runs the whole solve with the three
// iterates, b and the control block in LDS (the matrix stays in global memory and L2).  The
// gathers and the scalar control then pay LDS latency instead of L2 latency, which is what
// bounds a pass of a system this small.  The pass functions take generic pointers, so they
// run unchanged on the LDS copies.  On exit the iterates and the control block are written
// back, so the host reads the answer as after the other drivers.  Two-iterate form only.
template <int JM, int BS>
__global__ void __launch_bounds__(BS) k_solve_lds(SolveArgs a) {
  extern __shared__ double lds[];   // [4 n]: iterates 0, 1, 2, then b
  __shared__ double sh[3][BS / kWave];
  __shared__ PassView v;
  __shared__ Ctrl c;
  const int64_t n = a.A.n;
  for (int64_t i = threadIdx.x; i < n; i += BS) {
    lds[i] = a.buf0[i];
    lds[3 * n + i] = a.b[i];
  }
  if (threadIdx.x == 0) c = *a.ctrl;
  __syncthreads();
  SolveArgs al = a;
  al.buf0 = lds;
  al.buf1 = lds + n;
  al.buf2 = lds + 2 * n;
  al.b = lds + 3 * n;
  al.ctrl = &c;
  for (;;) {
    if (threadIdx.x == 0) load_view(&c, &v);
    __syncthreads();
    if (v.phase == PH_DONE) break;
    double p0 = 0.0, p1 = 0.0, p2 = 0.0;
    run_pass<JM, BS, false>(al, v, p0, p1, p2);
    block_sum3<BS>(p0, p1, p2, sh);
    if (threadIdx.x == 0) control_update(al, &c, p0, p1, p2);
    __syncthreads();
  }
  for (int64_t i = threadIdx.x; i < n; i += BS) {
    a.buf0[i] = lds[i];
    a.buf1[i] = lds[n + i];
    a.buf2[i] = lds[2 * n + i];
  }
  if (threadIdx.x == 0) *a.ctrl = c;
}

}  // namespace naj
