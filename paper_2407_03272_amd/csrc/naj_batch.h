// Batched solves: many systems, several right-hand sides each, advanced
// together one pass per launch.
//
// Every (system, right-hand side) pair is an independent solve instance with
// its own control block and vector buffers, running the same Algorithm 3 (or
// the mixed-precision refinement) as a single solve.  The work of a pass is a
// list of tiles; a tile is a range of one system's slices (and of its long
// rows).  A workgroup takes a tile and, slice by slice, advances every active
// instance of that system, so the slice's matrix entries are fetched from
// memory once and reused from cache for the other right-hand sides.  The last
// tile of a system to finish adds the tiles' partial sums in tile order and
// takes each instance's scalar decision.  Tiles and their order depend only on
// the system, so an instance's result does not depend on which other systems
// share the batch.
#pragma once

#include "naj_solve.h"

namespace naj {

constexpr int kMaxRhs = 8;      // right-hand sides per system in one batch
constexpr int kBatchBlock = 256;

struct BatchSys {
  Sell A;
  const double* dinv;
  int inst0, ninst;             // instances of this system
  int tile0, ntiles;            // tiles of this system
  unsigned int* counter;        // arrivals of this system's tiles in the current pass
  int ymode;
};

struct BatchInst {
  Ctrl* ctrl;
  double* x[4];
  float* f[5];
  double* b;                    // right-hand side in the system's row order
  double* part;                 // [kPartStride * ntiles of the system]
};

struct BatchTile {
  int sys;
  int s0, s1;                   // slices [s0, s1)
  int l0, l1;                   // long rows [l0, l1)
};

struct BatchArgs {
  const BatchTile* tiles;
  int ntiles;
  const BatchSys* sys;
  const BatchInst* inst;
  unsigned int* done;           // instances that have finished (status set)
  // options shared by the batch
  double tol;
  double inner_tol;
  int max_iter;
  int restart;
  int confirm_gap;
  int k0;
  int precision;
  int max_refine;
  int inner_stall;
};

__device__ __forceinline__ SolveArgs batch_args(const BatchArgs& ba, const BatchSys& S, const BatchInst& I) {
  SolveArgs a;
  a.A = S.A;
  a.dinv = S.dinv;
  a.b = I.b;
  a.buf0 = I.x[0];
  a.buf1 = I.x[1];
  a.buf2 = I.x[2];
  a.buf3 = I.x[3];
  a.part = I.part;
  a.ctrl = I.ctrl;
  a.bar = nullptr;
  a.counters = nullptr;
  a.hist = nullptr;
  a.trace = nullptr;
  a.hist_cap = 0;
  a.trace_cap = 0;
  a.tol = ba.tol;
  a.max_iter = ba.max_iter;
  a.restart = ba.restart;
  a.confirm_gap = ba.confirm_gap;
  a.k0 = ba.k0;
  a.nxcd = 1;
  a.spin_ticks = 0;
  a.precision = ba.precision;
  a.max_refine = ba.max_refine;
  a.inner_stall = ba.inner_stall;
  a.inner_tol = ba.inner_tol;
  a.f0 = I.f[0];
  a.f1 = I.f[1];
  a.f2 = I.f[2];
  a.f3 = I.f[3];
  a.r32 = I.f[4];
  a.ymode = S.ymode;
  return a;
}

// One slice (or one long row) of one instance, in the phase its view says.
template <bool USER_D>
__device__ __forceinline__ void batch_slice(const SolveArgs& a, const PassView& v, int64_t s, bool is_long, int lane,
                                            double& p0, double& p1, double& p2) {
  if (v.phase == PH_ITER) {
    Momentum<double> m;
    m.R = pick(a, v.iR);
    m.Yn = (a.ymode && v.iYn >= 0) ? pick(a, v.iYn) : nullptr;
    m.beta = v.beta;
    m.beta_next = v.beta_next;
    m.bz = v.bz != 0;
    m.ym = a.ymode != 0;
    if (is_long) iter_long<USER_D>(a, s, lane, pick(a, v.iP), m, pick(a, v.iW), p0, p1, p2);
    else iter_slice<USER_D>(a, s, lane, pick(a, v.iP), m, pick(a, v.iW), p0, p1, p2);
  } else if (v.phase == PH_CONFIRM) {
    if (is_long) resid_long(a.A, s, lane, pick(a, v.iW), a.b, nullptr, p0);
    else resid_slice(a.A, s, lane, pick(a, v.iW), a.b, nullptr, p0);
  } else if (v.phase == PH_INNER32) {
    Momentum<float> m;
    m.R = pickf(a, v.iR);
    m.Yn = (a.ymode && v.iYn >= 0) ? pickf(a, v.iYn) : nullptr;
    m.beta = (float)v.beta;
    m.beta_next = (float)v.beta_next;
    m.bz = v.bz != 0;
    m.ym = a.ymode != 0;
    if (is_long) inner_long<USER_D>(a, s, lane, pickf(a, v.iP), m, pickf(a, v.iW), v.zp != 0, p0, p1, p2);
    else inner_slice<USER_D>(a, s, lane, pickf(a, v.iP), m, pickf(a, v.iW), v.zp != 0, p0, p1, p2);
  } else if (v.phase == PH_RESID64) {
    const double* X = pick(a, v.iX);
    const float* D = v.update ? pickf(a, v.iD) : nullptr;
    double* Xn = v.update ? pick(a, v.iXn) : nullptr;
    if (is_long) resid_mixed_long(a, s, lane, X, D, Xn, p0, p1);
    else resid_mixed_slice(a, s, lane, X, D, Xn, p0, p1);
  } else if (v.phase == PH_NORMB) {
    if (is_long) {
      if (lane == 0) {
        const double x = a.b[s];
        p0 = p0 + x * x;
      }
    } else {
      const int64_t row = a.A.row0 + s * kWave + lane;
      if (row < a.A.n) {
        const double x = a.b[row];
        p0 = p0 + x * x;
      }
    }
  }
}

template <bool USER_D>
__device__ inline void batch_tile(const BatchArgs& ba, const BatchSys& S, const BatchTile& T, const PassView* views,
                                  double (*acc)[3][kBatchBlock]) {
  const int lane = threadIdx.x % kWave;
  const int wave = wave_id();
  constexpr int WPB = kBatchBlock / kWave;
  // long rows of the tile, then slices, each wave taking every WPB-th one; for every unit
  // all active instances in turn (the matrix entries are reused from cache)
  const int nlong = T.l1 - T.l0;
  const int nsl = T.s1 - T.s0;
  for (int u = wave; u < nlong + nsl; u += WPB) {
    const bool is_long = u < nlong;
    const int64_t s = is_long ? (int64_t)T.l0 + u : (int64_t)T.s0 + (u - nlong);
    for (int j = 0; j < S.ninst; ++j) {
      if (views[j].phase == PH_DONE) continue;
      const SolveArgs a = batch_args(ba, S, ba.inst[S.inst0 + j]);
      double p0 = 0.0, p1 = 0.0, p2 = 0.0;
      batch_slice<USER_D>(a, views[j], s, is_long, lane, p0, p1, p2);
      acc[j][0][threadIdx.x] += p0;
      acc[j][1][threadIdx.x] += p1;
      acc[j][2][threadIdx.x] += p2;
    }
  }
}

// One pass of every active instance of the batch.
__global__ void __launch_bounds__(kBatchBlock) k_batch_pass(BatchArgs ba) {
  __shared__ PassView views[kMaxRhs];
  __shared__ double acc[kMaxRhs][3][kBatchBlock];
  __shared__ double sh[3][kBatchBlock / kWave];
  __shared__ int s_active, s_last;
  for (int t = blockIdx.x; t < ba.ntiles; t += gridDim.x) {
    const BatchTile T = ba.tiles[t];
    const BatchSys& S = ba.sys[T.sys];
    if (threadIdx.x == 0) s_active = 0;
    __syncthreads();
    if (threadIdx.x < S.ninst) {
      load_view(ba.inst[S.inst0 + threadIdx.x].ctrl, &views[threadIdx.x]);
      if (views[threadIdx.x].phase != PH_DONE) atomicAdd(&s_active, 1);
    }
    for (int j = 0; j < S.ninst; ++j) {
      acc[j][0][threadIdx.x] = 0.0;
      acc[j][1][threadIdx.x] = 0.0;
      acc[j][2][threadIdx.x] = 0.0;
    }
    __syncthreads();
    if (s_active == 0) continue;   // uniform: every instance of this system has finished
    if (S.dinv) batch_tile<true>(ba, S, T, views, acc);
    else batch_tile<false>(ba, S, T, views, acc);
    __syncthreads();
    // per-instance workgroup sums (fixed order), written through to the coherence point
    for (int j = 0; j < S.ninst; ++j) {
      if (views[j].phase == PH_DONE) continue;
      double p0 = acc[j][0][threadIdx.x], p1 = acc[j][1][threadIdx.x], p2 = acc[j][2][threadIdx.x];
      block_sum3<kBatchBlock>(p0, p1, p2, sh);
      if (threadIdx.x == 0) {
        double* slot = ba.inst[S.inst0 + j].part + (size_t)(t - S.tile0) * kPartStride;
        __hip_atomic_store(slot + 0, p0, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(slot + 1, p1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(slot + 2, p2, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      }
      __syncthreads();
    }
    if (threadIdx.x == 0) {
      wait_stores_complete();
      const unsigned int old = __hip_atomic_fetch_add(S.counter, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      s_last = old == (unsigned int)(S.ntiles - 1) ? 1 : 0;
      if (s_last) __hip_atomic_store(S.counter, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    __syncthreads();
    if (s_last && threadIdx.x < kWave) {
      __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      const int lane = threadIdx.x;
      for (int j = 0; j < S.ninst; ++j) {
        if (views[j].phase == PH_DONE) continue;
        const BatchInst& I = ba.inst[S.inst0 + j];
        double r0, r1, r2;
        grid_sum3(I.part, S.ntiles, lane, r0, r1, r2);
        if (lane == 0) {
          const SolveArgs a = batch_args(ba, S, I);
          control_update(a, I.ctrl, r0, r1, r2);
          if (I.ctrl->phase == PH_DONE) __hip_atomic_fetch_add(ba.done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        }
      }
    }
    __syncthreads();
  }
}

// Per solve: clear every instance's control block (as k_solve_init), the tile counters and the done counter.
__global__ void k_batch_init(BatchArgs ba, int nsys, int ninst) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i < ninst) {
    // the instance's system, for its row-order mode
    int sidx = 0;
    for (int q = 0; q < nsys; ++q)
      if (ba.sys[q].inst0 <= i) sidx = q;
    Ctrl* c = ba.inst[i].ctrl;
    c->alpha = 1.0;
    c->beta = 0.0;
    c->nb = 0.0;
    c->relres = __builtin_nan("");
    c->t = 1;
    c->K_re = 0;
    c->K = ba.k0;
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
    if (ba.sys[sidx].ymode) {
      c->iP = 0;
      c->iW = 1;
      c->iR = 2;
      ymode_plan_next(c);
    }
    for (int q = 0; q < kRestartLogCap; ++q) c->restart_log[q] = 0;
  }
  if (i < nsys) *ba.sys[i].counter = 0u;
  if (i == 0) *ba.done = 0u;
}

// Right-hand sides and starting points into the instances' buffers (row-interleaved n x k
// caller layout -> one vector per instance, in the system's row order).
__global__ void k_batch_load(const double* src, int k, int j, const int32_t* perm, int64_t n, double* dst) {
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t o = perm ? perm[i] : i;
    dst[i] = src ? src[o * k + j] : 0.0;
  }
}

// Answer of one instance back into the caller's row-interleaved x.
__global__ void k_batch_store(const Ctrl* c, const double* b0, const double* b1, const double* b2, int k, int j,
                              const int32_t* perm, int64_t n, double* x) {
  const int r = c->result;
  const double* src = r == 0 ? b0 : (r == 1 ? b1 : b2);
  for (int64_t i = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t o = perm ? perm[i] : i;
    x[o * k + j] = r < 0 ? 0.0 : src[i];
  }
}

}  // namespace naj
