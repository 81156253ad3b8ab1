// Batched solves: many systems, several right-hand sides each, advanced
// together one pass per launch.
//
// Every (system, right-hand side) pair is an independent solve instance with
// its own control block running the same Algorithm 3 (or the mixed-precision
// refinement) as a single solve.  The vectors of a system's k right-hand
// sides are stored row-interleaved with kp = the power of two >= k entries per
// row: element (row, j) at row * kp + j, so the k values of a gathered column
// are adjacent in memory.
//
// The work of a pass is a list of items; an item is a range of one system's
// slices (or of its long rows) and is done by one wavefront.  The wavefronts of
// an L2 domain take consecutive items of the list in turn, so the rows being
// worked on in a domain form one compact band and the vector entries that
// neighbouring rows gather stay in that domain's L2.  Each item writes its
// partial sums per right-hand side to its own slot; a second kernel then adds a
// system's slots in item order and takes each instance's scalar decision.
// Items, their order and every summation order depend only on the system and
// its number of right-hand sides, so an instance's result does not depend on
// which other systems share the batch.  The per-row arithmetic is that of the
// single-solve pass, so on the regular layout an instance's iterates equal a
// single solve's bit for bit.
#pragma once

#include <type_traits>

#include "naj_solve.h"

namespace naj {

constexpr int kMaxRhs = 8;      // right-hand sides per system in one batch
constexpr int kBatchBlock = 256;
constexpr int kBatchWaves = kBatchBlock / kWave;
#ifndef NAJ_BATCH_UNROLL
#define NAJ_BATCH_UNROLL 4
#endif
// Column steps whose loads a lane issues together (the last group of a slice reloads
// its last column in the unused steps, so every group issues all its loads at once).
constexpr int kBatchUnroll = NAJ_BATCH_UNROLL;

struct BatchSys {
  Sell A;
  const double* dinv;           // caller's 1/D (system row order) or null
  double* xb;                   // float64 vectors: 4 buffers of n x kp (interleaved), xs bytes apart
  float* fb;                    // float32 vectors (mixed): 4 buffers + fl32(r), fs bytes apart
  uint32_t xs, fs;              // bytes per float64 / float32 buffer (every offset fits 32 bits)
  double* b;                    // right-hand sides, n x kp, in the system's row order
  double* part;                 // [nrhs][ntiles][kPartStride]
  Ctrl* ctrl;                   // [nrhs]
  PassView* vt;                 // [kMaxRhs] the pass view of each right-hand side (done beyond nrhs)
  double tol;                   // relative residual tolerance of this system's right-hand sides
  int gen;                      // tag written to slot_done when every instance has finished
  int lk, nrhs;                 // log2 of the lanes per row (kp = 1 << lk), right-hand sides
  int tile0, ntiles;
  int ymode;
};

struct BatchTile {             // one item of work
  int sys;
  int s0, s1;                   // slices [s0, s1)
  int l0, l1;                   // long rows [l0, l1)
};

struct BatchArgs {
  const BatchTile* tiles;
  const BatchSys* sys;
  int nsys;
  int* active;                  // items of the systems with an unfinished instance
  int* nactive;
  int* sact;                    // those systems
  int* nsact;
  unsigned int* done;           // instances that have finished (status set)
  int* slot_done;               // per system: set once all its instances have finished (null: not kept)
  int nxcd;                     // L2 domains the workgroups are spread over
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

// The fields of SolveArgs that the scalar control reads.
__device__ __forceinline__ SolveArgs batch_ctrl_args(const BatchArgs& ba, const BatchSys& S) {
  SolveArgs a = {};
  a.tol = S.tol;
  a.max_iter = ba.max_iter;
  a.restart = ba.restart;
  a.confirm_gap = ba.confirm_gap;
  a.k0 = ba.k0;
  a.precision = ba.precision;
  a.max_refine = ba.max_refine;
  a.inner_stall = ba.inner_stall;
  a.inner_tol = ba.inner_tol;
  a.ymode = S.ymode;
  a.ypar = 1;
  return a;
}

// Device-memory pointers.  The batch's pointers are read from a table in memory,
// so the compiler cannot tell their address space; marking them global gives the
// global load/store forms (a uniform base register plus a 32-bit lane offset)
// instead of flat accesses.
#define NAJ_GLOBAL __attribute__((address_space(1)))

template <typename T>
__device__ __forceinline__ const NAJ_GLOBAL T* gptr(const T* p) {
  return (const NAJ_GLOBAL T*)p;
}

// Matrix entries are read once per pass: with NAJ_BATCH_NT they bypass the caches'
// replacement order (non-temporal), leaving L2 to the gathered vector entries.
template <typename T>
__device__ __forceinline__ T mat_load(const NAJ_GLOBAL T* p) {
#if defined(NAJ_BATCH_NT)
  return __builtin_nontemporal_load(p);
#else
  return *p;
#endif
}

// Element access at a byte offset from a buffer block: the buffer role of the lane's
// instance times the buffer size, plus the element's offset.
template <typename T>
__device__ __forceinline__ T ld_at(const T* base, uint32_t off) {
  return *(const NAJ_GLOBAL T*)((const NAJ_GLOBAL char*)base + off);
}
template <typename T>
__device__ __forceinline__ void st_at(T* base, uint32_t off, T v) {
  *(NAJ_GLOBAL T*)((NAJ_GLOBAL char*)base + off) = v;
}

// Sum over the lanes of the same right-hand side (xor butterfly over the row bits of the
// lane index); every lane gets its right-hand side's sum.  Needs every lane of the wave.
template <typename T>
__device__ __forceinline__ T rhs_sum(T v, int kp) {
  for (int off = kWave / 2; off >= kp; off >>= 1) v += __shfl_xor(v, off, kWave);
  return v;
}

// Wave-uniform copies of values read from memory.  The batch tables live in device
// memory that the kernel also writes, so the compiler loads them into vector
// registers and cannot tell they are the same in every lane; reading the first
// lane puts them in scalar registers (uniform branches, scalar address bases).
__device__ __forceinline__ int uni(int x) { return __builtin_amdgcn_readfirstlane(x); }
__device__ __forceinline__ uint32_t uni(uint32_t x) { return (uint32_t)__builtin_amdgcn_readfirstlane((int)x); }
__device__ __forceinline__ int64_t uni(int64_t x) {
  const uint32_t lo = uni((uint32_t)(uint64_t)x), hi = uni((uint32_t)((uint64_t)x >> 32));
  return (int64_t)(((uint64_t)hi << 32) | lo);
}
template <typename T>
__device__ __forceinline__ T* uni(T* p) {
  return (T*)(uintptr_t)uni((int64_t)(uintptr_t)p);
}

// A system's record, read once per tile into scalar registers.
__device__ __forceinline__ BatchSys uniform_sys(const BatchSys& g) {
  BatchSys S;
  S.A.slice_ptr = uni(g.A.slice_ptr);
  S.A.col = uni(g.A.col);
  S.A.val = uni(g.A.val);
  S.A.val32 = uni(g.A.val32);
  S.A.n = uni(g.A.n);
  S.A.nslices = uni(g.A.nslices);
  S.A.row0 = uni(g.A.row0);
  S.A.n_long = uni(g.A.n_long);
  S.A.dom_bounds = nullptr;
  S.A.lrowptr = uni(g.A.lrowptr);
  S.A.lcol = uni(g.A.lcol);
  S.A.lval = uni(g.A.lval);
  S.A.lval32 = uni(g.A.lval32);
  S.A.soff = uni(g.A.soff);
  S.dinv = uni(g.dinv);
  S.xb = uni(g.xb);
  S.fb = uni(g.fb);
  S.tol = __builtin_bit_cast(double, uni(__builtin_bit_cast(int64_t, g.tol)));
  S.xs = uni(g.xs);
  S.fs = uni(g.fs);
  S.b = uni(g.b);
  S.part = uni(g.part);
  S.ctrl = uni(g.ctrl);
  S.vt = uni(g.vt);
  S.lk = uni(g.lk);
  S.nrhs = uni(g.nrhs);
  S.tile0 = uni(g.tile0);
  S.ntiles = uni(g.ntiles);
  S.ymode = uni(g.ymode);
  S.gen = uni(g.gen);
  return S;
}

// ---------------------------------------------------------------------------
// Rows of a slice: unit `sub` of slice s covers rows sub * (64/kp) ... of the
// slice; lane l takes row l / kp of the unit and right-hand side l % kp.

struct UnitRow {
  int rl;          // row within the slice
  int64_t row;     // row in the system's order
  bool live;
  int64_t rr;      // row, or 0 for a dead lane (any valid address)
  __device__ __forceinline__ UnitRow(const Sell& A, int64_t s, int sub, int lane, int lk) {
    rl = (sub << (6 - lk)) + (lane >> lk);
    row = A.row0 + s * kWave + rl;
    live = row < A.n;
    rr = live ? row : 0;
  }
};

// Byte offset of element (row, j) of an interleaved vector of E-byte entries.
template <int E>
__device__ __forceinline__ uint32_t elem(int64_t row, int lk, uint32_t j) {
  return ((((uint32_t)row) << lk) + j) * (uint32_t)E;
}

// The per-lane choices of a pass (restart just taken, first inner pass, pending
// update) differ between right-hand sides, so they are made by selects, never by
// branches inside the column loop: every lane issues the same loads (a lane that
// does not need an operand reads a valid, cached address) and keeps what it needs.

// Float64 iteration (Algorithm 3 step and partial sums), as iter_slice.
__device__ __forceinline__ void unit_iter(const BatchSys& S, int64_t s, int sub, int lane, const PassView& v,
                                          double& ps, double& pgg, double& psabs) {
  const int lk = S.lk;
  const uint32_t j = lane & ((1 << lk) - 1);
  const UnitRow u(S.A, s, sub, lane, lk);
  const double* X = S.xb;
  const bool bz = v.bz != 0, ym = S.ymode != 0;
  const uint32_t oP = (uint32_t)v.iP * S.xs, oW = (uint32_t)v.iW * S.xs;
  const uint32_t oR = bz ? oP : (uint32_t)v.iR * S.xs;          // bz: R is not used
  const bool yn = S.ymode && v.iYn >= 0;
  const uint32_t oY = yn ? (uint32_t)v.iYn * S.xs : 0u;
  const double beta = v.beta;
  const int64_t base = uni(gptr(S.A.slice_ptr)[s]);
  const int width = (int)((uni(gptr(S.A.slice_ptr)[s + 1]) - base) >> 6);
  const uint32_t ei = elem<8>(u.rr, lk, j);
  const double Pi = ld_at(X, oP + ei);
  const double Ri = ld_at(X, oR + ei);
  const double bi = ld_at((const double*)S.b, ei);
  const double di = S.dinv ? gptr(S.dinv)[u.rr] : 0.0;
  const NAJ_GLOBAL int32_t* cp = gptr(S.A.col) + base + u.rl;
  const OffPtr so = slice_offsets(S.A, s);   // every row of such a slice is live
  const int32_t rowc = (int32_t)u.rr;
  const NAJ_GLOBAL double* vp = gptr(S.A.val) + base + u.rl;
  double acc = 0.0, asum = 0.0;
  // U column steps: all loads issued before any is used; entries added in column order
  auto step = [&](auto U_, int k0) {
    constexpr int U = decltype(U_)::value;
    int cr[U];
    double w[U], y[U];
    if (so) {   // past the slice width: reuse the last column (cached), not added
#pragma unroll
      for (int q = 0; q < U; ++q) cr[q] = rowc + so[k0 + q < width ? k0 + q : width - 1];
    } else {
#pragma unroll
      for (int q = 0; q < U; ++q) cr[q] = mat_load(cp + (k0 + q < width ? k0 + q : width - 1) * kWave);
    }
#pragma unroll
    for (int q = 0; q < U; ++q) w[q] = mat_load(vp + (k0 + q < width ? k0 + q : width - 1) * kWave);
    if (ym) {   // materialized form: y^t is P (bz) or R, one gathered vector
      const uint32_t oG = bz ? oP : oR;
#pragma unroll
      for (int q = 0; q < U; ++q) y[q] = ld_at(X, oG + elem<8>(cr[q], lk, j));
    } else {
      double pj[U], rj[U];
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const uint32_t o = elem<8>(cr[q], lk, j);
        pj[q] = ld_at(X, oP + o);
        rj[q] = ld_at(X, oR + o);
      }
#pragma unroll
      for (int q = 0; q < U; ++q) y[q] = bz ? pj[q] : pj[q] + beta * (pj[q] - rj[q]);
    }
#pragma unroll
    for (int q = 0; q < U; ++q)
      if (k0 + q < width) {
        acc = acc + w[q] * y[q];
        asum = asum + fabs(w[q]);
      }
  };
  for (int k0 = 0; k0 < width; k0 += kBatchUnroll) step(std::integral_constant<int, kBatchUnroll>{}, k0);
  if (u.live) {
    const double yi = bz ? Pi : (ym ? Ri : Pi + beta * (Pi - Ri));
    const double g = acc - bi;
    const double dv = S.dinv ? di : 1.0 / (asum == 0.0 ? 1.0 : asum);
    const double xi = yi - dv * g;
    st_at(S.xb, oW + ei, xi);
    const double d = xi - Pi;
    if (yn) st_at(S.xb, oY + ei, xi + v.beta_next * d);
    const double gd = g * d;
    ps = ps + gd;
    pgg = pgg + g * g;
    psabs = psabs + fabs(gd);
  }
}

// Float32 inner iteration of the refinement loop, as inner_slice.
__device__ __forceinline__ void unit_inner(const BatchSys& S, int64_t s, int sub, int lane, const PassView& v,
                                           double& ps, double& pgg, double& psabs) {
  const int lk = S.lk;
  const uint32_t j = lane & ((1 << lk) - 1);
  const UnitRow u(S.A, s, sub, lane, lk);
  const float* F = S.fb;
  const bool bz = v.bz != 0, ym = S.ymode != 0, zp = v.zp != 0;
  const uint32_t oP = (uint32_t)v.iP * S.fs, oW = (uint32_t)v.iW * S.fs;
  const uint32_t oR = bz ? oP : (uint32_t)v.iR * S.fs;
  const bool yn = S.ymode && v.iYn >= 0;
  const uint32_t oY = yn ? (uint32_t)v.iYn * S.fs : 0u;
  const uint32_t oB = 4u * S.fs;
  const float beta = (float)v.beta;
  const int64_t base = uni(gptr(S.A.slice_ptr)[s]);
  const int width = (int)((uni(gptr(S.A.slice_ptr)[s + 1]) - base) >> 6);
  const uint32_t ei = elem<4>(u.rr, lk, j);
  const float Pi = zp ? 0.0f : ld_at(F, oP + ei);
  const float Ri = zp ? 0.0f : ld_at(F, oR + ei);
  const float bi = ld_at(F, oB + ei);
  const double di = S.dinv ? gptr(S.dinv)[u.rr] : 0.0;
  const NAJ_GLOBAL int32_t* cp = gptr(S.A.col) + base + u.rl;
  const OffPtr so = slice_offsets(S.A, s);   // every row of such a slice is live
  const int32_t rowc = (int32_t)u.rr;
  const NAJ_GLOBAL float* vp = gptr(S.A.val32) + base + u.rl;
  float acc = 0.0f, asum = 0.0f;
  auto step = [&](auto U_, int k0) {
    constexpr int U = decltype(U_)::value;
    int cr[U];
    float w[U], y[U];
    if (so) {   // past the slice width: reuse the last column (cached), not added
#pragma unroll
      for (int q = 0; q < U; ++q) cr[q] = rowc + so[k0 + q < width ? k0 + q : width - 1];
    } else {
#pragma unroll
      for (int q = 0; q < U; ++q) cr[q] = mat_load(cp + (k0 + q < width ? k0 + q : width - 1) * kWave);
    }
#pragma unroll
    for (int q = 0; q < U; ++q) w[q] = mat_load(vp + (k0 + q < width ? k0 + q : width - 1) * kWave);
    if (ym) {
      const uint32_t oG = bz ? oP : oR;
#pragma unroll
      for (int q = 0; q < U; ++q) y[q] = zp ? 0.0f : ld_at(F, oG + elem<4>(cr[q], lk, j));
    } else {
      float pj[U], rj[U];
#pragma unroll
      for (int q = 0; q < U; ++q) {
        const uint32_t o = elem<4>(cr[q], lk, j);
        pj[q] = ld_at(F, oP + o);
        rj[q] = ld_at(F, oR + o);
      }
#pragma unroll
      for (int q = 0; q < U; ++q) y[q] = zp ? 0.0f : (bz ? pj[q] : pj[q] + beta * (pj[q] - rj[q]));
    }
#pragma unroll
    for (int q = 0; q < U; ++q)
      if (k0 + q < width) {
        acc = acc + w[q] * y[q];
        asum = asum + fabsf(w[q]);
      }
  };
  for (int k0 = 0; k0 < width; k0 += kBatchUnroll) step(std::integral_constant<int, kBatchUnroll>{}, k0);
  if (u.live) {
    const float yi = (zp || bz) ? Pi : (ym ? Ri : Pi + beta * (Pi - Ri));
    const float g = acc - bi;
    const float dv = S.dinv ? (float)di : 1.0f / (asum == 0.0f ? 1.0f : asum);
    const float xi = yi - dv * g;
    st_at(S.fb, oW + ei, xi);
    const float d = xi - Pi;
    if (yn) st_at(S.fb, oY + ei, xi + (float)v.beta_next * d);
    const double g64 = (double)g, d64 = (double)d;
    const double gd = g64 * d64;
    ps = ps + gd;
    pgg = pgg + g64 * g64;
    psabs = psabs + fabs(gd);
  }
}

// Confirmation pass: ||b - Q x||^2 with x the instance's W buffer, as resid_slice.
__device__ __forceinline__ void unit_resid(const BatchSys& S, int64_t s, int sub, int lane, const PassView& v,
                                           double& prr) {
  const int lk = S.lk;
  const uint32_t j = lane & ((1 << lk) - 1);
  const UnitRow u(S.A, s, sub, lane, lk);
  const double* X = S.xb;
  const uint32_t oX = (uint32_t)v.iW * S.xs;
  const int64_t base = uni(gptr(S.A.slice_ptr)[s]);
  const int width = (int)((uni(gptr(S.A.slice_ptr)[s + 1]) - base) >> 6);
  const double bi = ld_at((const double*)S.b, elem<8>(u.rr, lk, j));
  const NAJ_GLOBAL int32_t* cp = gptr(S.A.col) + base + u.rl;
  const OffPtr so = slice_offsets(S.A, s);   // every row of such a slice is live
  const int32_t rowc = (int32_t)u.rr;
  const NAJ_GLOBAL double* vp = gptr(S.A.val) + base + u.rl;
  double acc = 0.0;
  auto step = [&](auto U_, int k0) {
    constexpr int U = decltype(U_)::value;
    int cr[U];
    double w[U], xj[U];
    if (so) {   // past the slice width: reuse the last column (cached), not added
#pragma unroll
      for (int q = 0; q < U; ++q) cr[q] = rowc + so[k0 + q < width ? k0 + q : width - 1];
    } else {
#pragma unroll
      for (int q = 0; q < U; ++q) cr[q] = mat_load(cp + (k0 + q < width ? k0 + q : width - 1) * kWave);
    }
#pragma unroll
    for (int q = 0; q < U; ++q) w[q] = mat_load(vp + (k0 + q < width ? k0 + q : width - 1) * kWave);
#pragma unroll
    for (int q = 0; q < U; ++q) xj[q] = ld_at(X, oX + elem<8>(cr[q], lk, j));
#pragma unroll
    for (int q = 0; q < U; ++q)
      if (k0 + q < width) acc = acc + w[q] * xj[q];
  };
  for (int k0 = 0; k0 < width; k0 += kBatchUnroll) step(std::integral_constant<int, kBatchUnroll>{}, k0);
  if (u.live) {
    const double r = bi - acc;
    prr = prr + r * r;
  }
}

// Float64 residual pass of the refinement loop (with the pending x + d update), as
// resid_mixed_slice.
__device__ __forceinline__ void unit_resid_mixed(const BatchSys& S, int64_t s, int sub, int lane, const PassView& v,
                                                 double& prr, double& pr32) {
  const int lk = S.lk;
  const uint32_t j = lane & ((1 << lk) - 1);
  const UnitRow u(S.A, s, sub, lane, lk);
  const double* X = S.xb;
  const float* F = S.fb;
  const bool up = v.update != 0;
  const uint32_t oX = (uint32_t)v.iX * S.xs, oXn = (uint32_t)v.iXn * S.xs, oD = (uint32_t)v.iD * S.fs;
  const uint32_t oB = 4u * S.fs;
  const int64_t base = uni(gptr(S.A.slice_ptr)[s]);
  const int width = (int)((uni(gptr(S.A.slice_ptr)[s + 1]) - base) >> 6);
  const uint32_t e4 = elem<4>(u.rr, lk, j);
  const double bi = ld_at((const double*)S.b, 2u * e4);
  const double xi0 = ld_at(X, oX + 2u * e4);
  const float di0 = ld_at(F, oD + e4);
  const NAJ_GLOBAL int32_t* cp = gptr(S.A.col) + base + u.rl;
  const OffPtr so = slice_offsets(S.A, s);   // every row of such a slice is live
  const int32_t rowc = (int32_t)u.rr;
  const NAJ_GLOBAL double* vp = gptr(S.A.val) + base + u.rl;
  double acc = 0.0;
  auto step = [&](auto U_, int k0) {
    constexpr int U = decltype(U_)::value;
    int cr[U];
    double w[U], xj[U];
    float dj[U];
    if (so) {   // past the slice width: reuse the last column (cached), not added
#pragma unroll
      for (int q = 0; q < U; ++q) cr[q] = rowc + so[k0 + q < width ? k0 + q : width - 1];
    } else {
#pragma unroll
      for (int q = 0; q < U; ++q) cr[q] = mat_load(cp + (k0 + q < width ? k0 + q : width - 1) * kWave);
    }
#pragma unroll
    for (int q = 0; q < U; ++q) w[q] = mat_load(vp + (k0 + q < width ? k0 + q : width - 1) * kWave);
#pragma unroll
    for (int q = 0; q < U; ++q) {
      const uint32_t o = elem<4>(cr[q], lk, j);
      xj[q] = ld_at(X, oX + 2u * o);
      dj[q] = ld_at(F, oD + o);
    }
#pragma unroll
    for (int q = 0; q < U; ++q)
      if (k0 + q < width) {
        const double xq = up ? xj[q] + (double)dj[q] : xj[q];
        acc = acc + w[q] * xq;
      }
  };
  for (int k0 = 0; k0 < width; k0 += kBatchUnroll) step(std::integral_constant<int, kBatchUnroll>{}, k0);
  if (u.live) {
    if (up) st_at(S.xb, oXn + 2u * e4, xi0 + (double)di0);
    const double r = bi - acc;
    const float r32 = (float)r;
    st_at(S.fb, oB + e4, r32);
    prr = prr + r * r;
    const double r64 = (double)r32;
    pr32 = pr32 + r64 * r64;
  }
}

__device__ __forceinline__ void unit_normb(const BatchSys& S, int64_t s, int sub, int lane, double& p0) {
  const int lk = S.lk;
  const UnitRow u(S.A, s, sub, lane, lk);
  if (u.live) {
    const double x = ld_at((const double*)S.b, elem<8>(u.row, lk, lane & ((1 << lk) - 1)));
    p0 = p0 + x * x;
  }
}

// ---------------------------------------------------------------------------
// Long rows: one wavefront per row and all its right-hand sides; lane l adds the
// entries l / kp, l / kp + 64/kp, ... for right-hand side l % kp, and the lanes
// of a right-hand side are then combined by the xor butterfly (a fixed order).
// Each function runs with every lane of the wave (the butterfly needs them all);
// only lanes with `mine` set write or add to their sums.

template <typename T, typename VT, typename YF>
__device__ __forceinline__ void long_sums_kp(const int32_t* colp, const VT* valp, int64_t s, int64_t e, int lane,
                                             int lk, YF yof, T& acc, T& asum) {
  const NAJ_GLOBAL int32_t* col = gptr(colp);
  const NAJ_GLOBAL VT* val = gptr(valp);
  const int RS = kWave >> lk;   // entries per step
  T a = (T)0, b = (T)0;
  for (int64_t k = s + (lane >> lk); k < e; k += (int64_t)RS * kLongUnroll) {
    int c[kLongUnroll];
    T w[kLongUnroll], y[kLongUnroll];
#pragma unroll
    for (int q = 0; q < kLongUnroll; ++q)
      if (k + q * RS < e) {
        c[q] = col[k + q * RS];
        w[q] = (T)val[k + q * RS];
      }
#pragma unroll
    for (int q = 0; q < kLongUnroll; ++q)
      if (k + q * RS < e) y[q] = yof(c[q]);
#pragma unroll
    for (int q = 0; q < kLongUnroll; ++q)
      if (k + q * RS < e) {
        a = a + w[q] * y[q];
        b = b + (w[q] < (T)0 ? -w[q] : w[q]);
      }
  }
  acc = rhs_sum(a, 1 << lk);
  asum = rhs_sum(b, 1 << lk);
}

__device__ __forceinline__ void long_iter(const BatchSys& S, int64_t r, int lane, const PassView& v, bool mine,
                                          double& ps, double& pgg, double& psabs) {
  const int lk = S.lk;
  const uint32_t j = lane & ((1 << lk) - 1);
  const double* X = S.xb;
  const bool bz = v.bz != 0, ym = S.ymode != 0;
  const uint32_t oP = (uint32_t)v.iP * S.xs, oW = (uint32_t)v.iW * S.xs;
  const uint32_t oR = bz ? oP : (uint32_t)v.iR * S.xs;
  const bool yn = S.ymode && v.iYn >= 0;
  const uint32_t oY = yn ? (uint32_t)v.iYn * S.xs : 0u;
  const double beta = v.beta;
  double acc, asum;
  long_sums_kp<double>(S.A.lcol, S.A.lval, uni(gptr(S.A.lrowptr)[r]), uni(gptr(S.A.lrowptr)[r + 1]), lane, lk,
                       [&](int c) {
                         const uint32_t o = elem<8>(c, lk, j);
                         const double p = ld_at(X, oP + o), q = ld_at(X, oR + o);
                         return bz ? p : (ym ? q : p + beta * (p - q));
                       },
                       acc, asum);
  if (mine && lane < (1 << lk)) {
    const uint32_t ei = elem<8>(r, lk, j);
    const double Pi = ld_at(X, oP + ei);
    const double Ri = ld_at(X, oR + ei);
    const double yi = bz ? Pi : (ym ? Ri : Pi + beta * (Pi - Ri));
    const double g = acc - ld_at((const double*)S.b, ei);
    const double dv = S.dinv ? gptr(S.dinv)[r] : 1.0 / (asum == 0.0 ? 1.0 : asum);
    const double xi = yi - dv * g;
    st_at(S.xb, oW + ei, xi);
    const double dd = xi - Pi;
    if (yn) st_at(S.xb, oY + ei, xi + v.beta_next * dd);
    const double gd = g * dd;
    ps = ps + gd;
    pgg = pgg + g * g;
    psabs = psabs + fabs(gd);
  }
}

__device__ __forceinline__ void long_inner(const BatchSys& S, int64_t r, int lane, const PassView& v, bool mine,
                                           double& ps, double& pgg, double& psabs) {
  const int lk = S.lk;
  const uint32_t j = lane & ((1 << lk) - 1);
  const float* F = S.fb;
  const bool bz = v.bz != 0, ym = S.ymode != 0, zp = v.zp != 0;
  const uint32_t oP = (uint32_t)v.iP * S.fs, oW = (uint32_t)v.iW * S.fs;
  const uint32_t oR = bz ? oP : (uint32_t)v.iR * S.fs;
  const bool yn = S.ymode && v.iYn >= 0;
  const uint32_t oY = yn ? (uint32_t)v.iYn * S.fs : 0u;
  const float beta = (float)v.beta;
  float acc, asum;
  long_sums_kp<float>(S.A.lcol, S.A.lval32, uni(gptr(S.A.lrowptr)[r]), uni(gptr(S.A.lrowptr)[r + 1]), lane, lk,
                      [&](int c) {
                        const uint32_t o = elem<4>(c, lk, j);
                        const float p = ld_at(F, oP + o), q = ld_at(F, oR + o);
                        return zp ? 0.0f : (bz ? p : (ym ? q : p + beta * (p - q)));
                      },
                      acc, asum);
  if (mine && lane < (1 << lk)) {
    const uint32_t ei = elem<4>(r, lk, j);
    const float Pi = zp ? 0.0f : ld_at(F, oP + ei);
    const float Ri = zp ? 0.0f : ld_at(F, oR + ei);
    const float yi = (zp || bz) ? Pi : (ym ? Ri : Pi + beta * (Pi - Ri));
    const float g = acc - ld_at(F, 4u * S.fs + ei);
    const float dv = S.dinv ? (float)gptr(S.dinv)[r] : 1.0f / (asum == 0.0f ? 1.0f : asum);
    const float xi = yi - dv * g;
    st_at(S.fb, oW + ei, xi);
    const float dd = xi - Pi;
    if (yn) st_at(S.fb, oY + ei, xi + (float)v.beta_next * dd);
    const double g64 = (double)g, d64 = (double)dd;
    const double gd = g64 * d64;
    ps = ps + gd;
    pgg = pgg + g64 * g64;
    psabs = psabs + fabs(gd);
  }
}

__device__ __forceinline__ void long_resid(const BatchSys& S, int64_t r, int lane, const PassView& v, bool mine,
                                           double& prr) {
  const int lk = S.lk;
  const uint32_t j = lane & ((1 << lk) - 1);
  const double* X = S.xb;
  const uint32_t oX = (uint32_t)v.iW * S.xs;
  double acc, asum;
  long_sums_kp<double>(S.A.lcol, S.A.lval, uni(gptr(S.A.lrowptr)[r]), uni(gptr(S.A.lrowptr)[r + 1]), lane, lk,
                       [&](int c) { return ld_at(X, oX + elem<8>(c, lk, j)); }, acc, asum);
  if (mine && lane < (1 << lk)) {
    const double res = ld_at((const double*)S.b, elem<8>(r, lk, j)) - acc;
    prr = prr + res * res;
  }
}

__device__ __forceinline__ void long_resid_mixed(const BatchSys& S, int64_t r, int lane, const PassView& v, bool mine,
                                                 double& prr, double& pr32) {
  const int lk = S.lk;
  const uint32_t j = lane & ((1 << lk) - 1);
  const double* X = S.xb;
  const float* F = S.fb;
  const bool up = v.update != 0;
  const uint32_t oX = (uint32_t)v.iX * S.xs, oXn = (uint32_t)v.iXn * S.xs, oD = (uint32_t)v.iD * S.fs;
  double acc, asum;
  long_sums_kp<double>(S.A.lcol, S.A.lval, uni(gptr(S.A.lrowptr)[r]), uni(gptr(S.A.lrowptr)[r + 1]), lane, lk,
                       [&](int c) {
                         const uint32_t o = elem<4>(c, lk, j);
                         const double x = ld_at(X, oX + 2u * o);
                         const float d = ld_at(F, oD + o);
                         return up ? x + (double)d : x;
                       },
                       acc, asum);
  if (mine && lane < (1 << lk)) {
    const uint32_t e4 = elem<4>(r, lk, j);
    if (up) st_at(S.xb, oXn + 2u * e4, ld_at(X, oX + 2u * e4) + (double)ld_at(F, oD + e4));
    const double res = ld_at((const double*)S.b, 2u * e4) - acc;
    const float r32 = (float)res;
    st_at(S.fb, 4u * S.fs + e4, r32);
    prr = prr + res * res;
    const double r64 = (double)r32;
    pr32 = pr32 + r64 * r64;
  }
}

// ---------------------------------------------------------------------------
// Float32 inner pass over slices, one lane per row (two-iterate form).  A
// wavefront takes a whole 64-row slice and the right-hand sides of the system G at
// a time: the matrix entries of a column are loaded once per row, and the G values
// of a gathered row (adjacent in the interleaved layout) come in one vector load.
// The state of each right-hand side (phase, roles, momentum) is the same in every
// lane, so every per-right-hand-side choice is uniform.  In the two-iterate form the
// roles are a rotation of the three buffers, fixed by the buffer of P alone
// (R = P + 1, W = P + 2, mod 3); restarts fall at different iterations for different
// right-hand sides, so a group can mix rotations: then all three buffers are loaded
// and each right-hand side picks its own by bit masks.

template <int G>
__device__ __forceinline__ void ld_vec(const float* base, uint32_t off, float (&o)[G]) {
  const NAJ_GLOBAL char* p = (const NAJ_GLOBAL char*)base + off;
  if constexpr (G == 8) {
    typedef float v4 __attribute__((ext_vector_type(4)));
    const v4 t = *(const NAJ_GLOBAL v4*)p;
    const v4 u = *(const NAJ_GLOBAL v4*)(p + 16);
    o[0] = t.x;
    o[1] = t.y;
    o[2] = t.z;
    o[3] = t.w;
    o[4] = u.x;
    o[5] = u.y;
    o[6] = u.z;
    o[7] = u.w;
  } else if constexpr (G == 4) {
    typedef float v4 __attribute__((ext_vector_type(4)));
    const v4 t = *(const NAJ_GLOBAL v4*)p;
    o[0] = t.x;
    o[1] = t.y;
    o[2] = t.z;
    o[3] = t.w;
  } else if constexpr (G == 2) {
    typedef float v2 __attribute__((ext_vector_type(2)));
    const v2 t = *(const NAJ_GLOBAL v2*)p;
    o[0] = t.x;
    o[1] = t.y;
  } else {
    o[0] = *(const NAJ_GLOBAL float*)p;
  }
}

template <int G>
__device__ __forceinline__ void st_vec(float* base, uint32_t off, const float (&v)[G]) {
  NAJ_GLOBAL char* p = (NAJ_GLOBAL char*)base + off;
  if constexpr (G == 8) {
    typedef float v4 __attribute__((ext_vector_type(4)));
    v4 t, u;
    t.x = v[0];
    t.y = v[1];
    t.z = v[2];
    t.w = v[3];
    u.x = v[4];
    u.y = v[5];
    u.z = v[6];
    u.w = v[7];
    *(NAJ_GLOBAL v4*)p = t;
    *(NAJ_GLOBAL v4*)(p + 16) = u;
  } else if constexpr (G == 4) {
    typedef float v4 __attribute__((ext_vector_type(4)));
    v4 t;
    t.x = v[0];
    t.y = v[1];
    t.z = v[2];
    t.w = v[3];
    *(NAJ_GLOBAL v4*)p = t;
  } else if constexpr (G == 2) {
    typedef float v2 __attribute__((ext_vector_type(2)));
    v2 t;
    t.x = v[0];
    t.y = v[1];
    *(NAJ_GLOBAL v2*)p = t;
  } else {
    *(NAJ_GLOBAL float*)p = v[0];
  }
}

__device__ __forceinline__ float uni_f(float x) { return __builtin_bit_cast(float, uni(__builtin_bit_cast(int, x))); }

// a_s for a uniform s in {0, 1, 2}, by bit masks (no branch, no indexed array)
__device__ __forceinline__ float sel3(float a0, float a1, float a2, int s) {
  const int m0 = -(int)(s == 0), m1 = -(int)(s == 1), m2 = -(int)(s == 2);
  return __builtin_bit_cast(float, (__builtin_bit_cast(int, a0) & m0) | (__builtin_bit_cast(int, a1) & m1) |
                                       (__builtin_bit_cast(int, a2) & m2));
}

// Uniform state of right-hand sides j0 .. j0+G-1 for the float32 inner pass.
template <int G>
struct InnerGroup {
  int act;          // bit q: right-hand side j0+q is in the inner phase
  int all;          // every right-hand side of the group is active
  int bz, zp;       // bit q: y = P (restart / first step); previous iterate zero
  int needR;        // some active right-hand side reads R
  int rot;          // the common buffer of P when all active right-hand sides share it, else -1
  int sig[G];       // buffer of P per right-hand side
  float beta[G];
};

template <int G>
__device__ __forceinline__ InnerGroup<G> inner_group(const PassView* views, int j0) {   // views: the view table
  InnerGroup<G> g;
  g.act = g.bz = g.zp = g.needR = 0;
  int sigs = 0, s0 = 0;
#pragma unroll
  for (int q = 0; q < G; ++q) {
    const NAJ_GLOBAL PassView& v = gptr(views)[j0 + q];
    const bool on = uni(v.phase) == PH_INNER32;
    g.sig[q] = uni(v.iP);
    g.beta[q] = uni_f((float)v.beta);
    const bool bz = uni(v.bz) != 0, zp = uni(v.zp) != 0;
    if (!on) continue;
    g.act |= 1 << q;
    if (bz) g.bz |= 1 << q;
    if (zp) g.zp |= 1 << q;
    if (!bz && !zp) g.needR = 1;
    sigs |= 1 << g.sig[q];
    s0 = g.sig[q];
  }
  g.all = g.act == (1 << G) - 1;
  g.rot = (sigs & (sigs - 1)) == 0 ? s0 : -1;
  return g;
}

// Row form: the matrix entries of `chunk` columns are loaded at once, then their gathers go
// `unroll` columns at a time, so a slice takes few dependent memory round trips.  Measured on
// 64 3D finite-element systems of 40k rows: with 8 right-hand sides per lane the registers
// bound the resident waves, and 4 columns one at a time (123 VGPRs, 4 waves per SIMD) beat
// 8 two at a time by 9 %; with one right-hand side, 8 columns four at a time beat two at a
// time by 7 %.
template <int G>
struct RowShape {
  static constexpr int chunk = G >= 8 ? 4 : 8;
  static constexpr int unroll = G >= 8 ? 1 : (G == 1 ? 4 : 2);
};
#ifndef NAJ_ROW_GROUP
#define NAJ_ROW_GROUP 8
#endif
// Right-hand sides a lane carries at once in the row form (8 measured best for 8
// right-hand sides: one pass over the row's columns instead of two).
constexpr int kRowGroup = NAJ_ROW_GROUP;

// P and R values of every right-hand side of the group at interleaved offset e.
template <int G>
__device__ __forceinline__ void roles_at(const float* F, uint32_t fs, uint32_t e, const InnerGroup<G>& g,
                                         float (&P)[G], float (&R)[G]) {
  if (g.rot >= 0) {   // one rotation for the whole group: two vector loads
    ld_vec<G>(F, (uint32_t)g.rot * fs + e, P);
    if (g.needR) {
      ld_vec<G>(F, (uint32_t)(g.rot == 2 ? 0 : g.rot + 1) * fs + e, R);
    } else {
#pragma unroll
      for (int q = 0; q < G; ++q) R[q] = 0.0f;
    }
  } else {
    float t0[G], t1[G], t2[G];
    ld_vec<G>(F, e, t0);
    ld_vec<G>(F, fs + e, t1);
    ld_vec<G>(F, 2u * fs + e, t2);
#pragma unroll
    for (int q = 0; q < G; ++q) {
      int sp = g.sig[q];
      asm volatile("" : "+s"(sp));   // recompute the masks here rather than keep them all live
      const int sr = sp == 2 ? 0 : sp + 1;
      P[q] = sel3(t0[q], t1[q], t2[q], sp);
      R[q] = sel3(t0[q], t1[q], t2[q], sr);
    }
  }
}

template <int G>
__device__ __forceinline__ void slice_inner_rows(const BatchSys& S, int64_t s, int lane, int j0, const InnerGroup<G>& g,
                                                 double (&ps)[G], double (&pgg)[G]) {
  constexpr int U = RowShape<G>::unroll;
  constexpr int kRowChunk = RowShape<G>::chunk;
  const int lk = S.lk;
  const int64_t row = S.A.row0 + s * kWave + lane;
  const bool live = row < S.A.n;
  const int64_t rr = live ? row : 0;
  const float* F = S.fb;
  const uint32_t fs = S.fs;
  const int64_t base = uni(gptr(S.A.slice_ptr)[s]);
  const int width = (int)((uni(gptr(S.A.slice_ptr)[s + 1]) - base) >> 6);
  const uint32_t eo = elem<4>(rr, lk, (uint32_t)j0);
  float Pi[G], Ri[G], bi[G];
  roles_at<G>(F, fs, eo, g, Pi, Ri);
  ld_vec<G>(F, 4u * fs + eo, bi);
  const double di = S.dinv ? gptr(S.dinv)[rr] : 0.0;
  const NAJ_GLOBAL int32_t* cp = gptr(S.A.col) + base + lane;
  const OffPtr so = slice_offsets(S.A, s);   // every row of such a slice is live
  const int32_t rowc = (int32_t)rr;
  const NAJ_GLOBAL float* vp = gptr(S.A.val32) + base + lane;
  float acc[G];
#pragma unroll
  for (int q = 0; q < G; ++q) acc[q] = 0.0f;
  float asum = 0.0f;
  for (int k0 = 0; k0 < width; k0 += kRowChunk) {
    int cr[kRowChunk];
    float w[kRowChunk];
    if (so) {   // past the slice width: reuse the last column (cached), not added
#pragma unroll
      for (int u = 0; u < kRowChunk; ++u) cr[u] = rowc + so[k0 + u < width ? k0 + u : width - 1];
    } else {
#pragma unroll
      for (int u = 0; u < kRowChunk; ++u) cr[u] = mat_load(cp + (k0 + u < width ? k0 + u : width - 1) * kWave);
    }
#pragma unroll
    for (int u = 0; u < kRowChunk; ++u) w[u] = mat_load(vp + (k0 + u < width ? k0 + u : width - 1) * kWave);
#pragma unroll
    for (int u0 = 0; u0 < kRowChunk; u0 += U) {
      if (k0 + u0 >= width) break;
      float pj[U][G], rj[U][G];
#pragma unroll
      for (int u = 0; u < U; ++u) roles_at<G>(F, fs, elem<4>(cr[u0 + u], lk, (uint32_t)j0), g, pj[u], rj[u]);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (k0 + u0 + u >= width) break;
        asum = asum + fabsf(w[u0 + u]);
#pragma unroll
        for (int q = 0; q < G; ++q) {
          if (!((g.act >> q) & 1)) continue;
          float y;
          if ((g.zp >> q) & 1) y = 0.0f;
          else if ((g.bz >> q) & 1) y = pj[u][q];
          else y = pj[u][q] + g.beta[q] * (pj[u][q] - rj[u][q]);
          acc[q] = acc[q] + w[u0 + u] * y;
        }
      }
    }
  }
  if (live) {
    const float dv = S.dinv ? (float)di : 1.0f / (asum == 0.0f ? 1.0f : asum);
    float xo[G];
#pragma unroll
    for (int q = 0; q < G; ++q) {
      const bool zp = (g.zp >> q) & 1, bz = (g.bz >> q) & 1;
      const float P0 = zp ? 0.0f : Pi[q];
      const float R0 = (zp || bz) ? 0.0f : Ri[q];
      const float yi = (zp || bz) ? P0 : P0 + g.beta[q] * (P0 - R0);
      const float gr = acc[q] - bi[q];
      const float xi = yi - dv * gr;
      xo[q] = xi;
      if ((g.act >> q) & 1) {
        const float d = xi - P0;
        const double g64 = (double)gr, d64 = (double)d;
        ps[q] = ps[q] + g64 * d64;
        pgg[q] = pgg[q] + g64 * g64;
      }
    }
    if (g.all && g.rot >= 0) {   // one W buffer for the group: one vector store
      st_vec<G>(S.fb, (uint32_t)(g.rot == 0 ? 2 : g.rot - 1) * fs + elem<4>(row, lk, (uint32_t)j0), xo);
    } else {
#pragma unroll
      for (int q = 0; q < G; ++q)
        if ((g.act >> q) & 1) {
          const int sw = g.sig[q] == 0 ? 2 : g.sig[q] - 1;
          st_at(S.fb, (uint32_t)sw * fs + elem<4>(row, lk, (uint32_t)(j0 + q)), xo[q]);
        }
    }
  }
}

// Materialized form of the row-form inner pass (systems of mixed batches with several
// right-hand sides; with one, the two-iterate form measured faster when many systems run
// together, the extra y store outweighing the halved gathers): the pass
// gathers y^t from one buffer and writes y^{t+1} = x^t + beta_next (x^t - x^{t-1}) for the
// next pass, one gathered vector instead of two.  The y buffers (roles 2 and 3) alternate
// with the system's pass count, which is the same for all its right-hand sides, so every
// right-hand side that reads y in a pass reads the same buffer and a gathered row's G
// values come in one vector load.  Right-hand sides right after a restart (y = P = x^{t-1})
// or at an inner solve's first step (y = 0) take their values by selects; the iterates
// alternate between roles 0 and 1.
template <int G>
struct InnerGroupY {
  int act;          // bit q: right-hand side j0+q is in the inner phase
  int all;          // every right-hand side of the group is active
  int bz, zp;       // bit q: y = P; previous iterate zero (y = 0)
  int ybuf;         // y buffer of the right-hand sides that read y (-1: none reads y)
  int ymix;         // they do not share one buffer (then both are loaded and selected)
  int prot;         // common P buffer of the active right-hand sides, -1 if they differ
  int wyn;          // buffer receiving y^{t+1} (-1: no active right-hand side writes one)
  int yb[G];        // y buffer per right-hand side
  int psig[G];      // P buffer per right-hand side (0 or 1)
  float bnext[G];
};

template <int G>
__device__ __forceinline__ InnerGroupY<G> inner_group_y(const PassView* views, int j0) {
  InnerGroupY<G> g;
  g.act = g.bz = g.zp = 0;
  g.ybuf = g.wyn = -1;
  g.ymix = 0;
  int psigs = 0, p0 = 0;
#pragma unroll
  for (int q = 0; q < G; ++q) {
    const NAJ_GLOBAL PassView& v = gptr(views)[j0 + q];
    const bool on = uni(v.phase) == PH_INNER32;
    g.psig[q] = uni(v.iP) & 1;
    g.yb[q] = uni(v.iR) == 3 ? 3 : 2;
    g.bnext[q] = uni_f((float)v.beta_next);
    const bool bz = uni(v.bz) != 0, zp = uni(v.zp) != 0;
    const int yn = uni(v.iYn);
    if (!on) continue;
    g.act |= 1 << q;
    if (bz) g.bz |= 1 << q;
    if (zp) g.zp |= 1 << q;
    if (!bz && !zp) {
      if (g.ybuf >= 0 && g.ybuf != g.yb[q]) g.ymix = 1;
      g.ybuf = g.yb[q];
    }
    if (yn >= 0) g.wyn = yn;
    psigs |= 1 << g.psig[q];
    p0 = g.psig[q];
  }
  g.all = g.act == (1 << G) - 1;
  g.prot = (psigs & (psigs - 1)) == 0 ? p0 : -1;
  return g;
}

// y values of the group's right-hand sides at interleaved offset e.
template <int G>
__device__ __forceinline__ void y_at(const float* F, uint32_t fs, uint32_t e, const InnerGroupY<G>& g,
                                     float (&y)[G]) {
  float yv[G], pv[G];
  if (g.ybuf >= 0 && !g.ymix) {
    ld_vec<G>(F, (uint32_t)g.ybuf * fs + e, yv);
  } else if (g.ymix) {
    float t2[G], t3[G];
    ld_vec<G>(F, 2u * fs + e, t2);
    ld_vec<G>(F, 3u * fs + e, t3);
#pragma unroll
    for (int q = 0; q < G; ++q) yv[q] = g.yb[q] == 3 ? t3[q] : t2[q];
  } else {
#pragma unroll
    for (int q = 0; q < G; ++q) yv[q] = 0.0f;
  }
  if (g.bz) {
    if (g.prot >= 0) {
      ld_vec<G>(F, (uint32_t)g.prot * fs + e, pv);
    } else {
      float t0[G], t1[G];
      ld_vec<G>(F, e, t0);
      ld_vec<G>(F, fs + e, t1);
#pragma unroll
      for (int q = 0; q < G; ++q) pv[q] = g.psig[q] ? t1[q] : t0[q];
    }
  } else {
#pragma unroll
    for (int q = 0; q < G; ++q) pv[q] = 0.0f;
  }
#pragma unroll
  for (int q = 0; q < G; ++q) y[q] = ((g.zp >> q) & 1) ? 0.0f : (((g.bz >> q) & 1) ? pv[q] : yv[q]);
}

template <int G>
__device__ __forceinline__ void slice_inner_rows_ym(const BatchSys& S, int64_t s, int lane, int j0,
                                                    const InnerGroupY<G>& g, double (&ps)[G], double (&pgg)[G]) {
  constexpr int U = RowShape<G>::unroll;
  constexpr int kRowChunk = RowShape<G>::chunk;
  const int lk = S.lk;
  const int64_t row = S.A.row0 + s * kWave + lane;
  const bool live = row < S.A.n;
  const int64_t rr = live ? row : 0;
  const float* F = S.fb;
  const uint32_t fs = S.fs;
  const int64_t base = uni(gptr(S.A.slice_ptr)[s]);
  const int width = (int)((uni(gptr(S.A.slice_ptr)[s + 1]) - base) >> 6);
  const uint32_t eo = elem<4>(rr, lk, (uint32_t)j0);
  const NAJ_GLOBAL int32_t* cp = gptr(S.A.col) + base + lane;
  const OffPtr so = slice_offsets(S.A, s);   // every row of such a slice is live
  const int32_t rowc = (int32_t)rr;
  const NAJ_GLOBAL float* vp = gptr(S.A.val32) + base + lane;
  float acc[G];
#pragma unroll
  for (int q = 0; q < G; ++q) acc[q] = 0.0f;
  float asum = 0.0f;
  for (int k0 = 0; k0 < width; k0 += kRowChunk) {
    int cr[kRowChunk];
    float w[kRowChunk];
    if (so) {   // past the slice width: reuse the last column (cached), not added
#pragma unroll
      for (int u = 0; u < kRowChunk; ++u) cr[u] = rowc + so[k0 + u < width ? k0 + u : width - 1];
    } else {
#pragma unroll
      for (int u = 0; u < kRowChunk; ++u) cr[u] = mat_load(cp + (k0 + u < width ? k0 + u : width - 1) * kWave);
    }
#pragma unroll
    for (int u = 0; u < kRowChunk; ++u) w[u] = mat_load(vp + (k0 + u < width ? k0 + u : width - 1) * kWave);
#pragma unroll
    for (int u0 = 0; u0 < kRowChunk; u0 += U) {
      if (k0 + u0 >= width) break;
      float yj[U][G];
#pragma unroll
      for (int u = 0; u < U; ++u) y_at<G>(F, fs, elem<4>(cr[u0 + u], lk, (uint32_t)j0), g, yj[u]);
#pragma unroll
      for (int u = 0; u < U; ++u) {
        if (k0 + u0 + u >= width) break;
        asum = asum + fabsf(w[u0 + u]);
#pragma unroll
        for (int q = 0; q < G; ++q)
          if ((g.act >> q) & 1) acc[q] = acc[q] + w[u0 + u] * yj[u][q];
      }
    }
  }
  // own-row operands after the column loop (fewer registers live across it)
  float Pi[G], yi[G], bi[G];
  if (g.prot >= 0) {
    ld_vec<G>(F, (uint32_t)g.prot * fs + eo, Pi);
  } else {
    float t0[G], t1[G];
    ld_vec<G>(F, eo, t0);
    ld_vec<G>(F, fs + eo, t1);
#pragma unroll
    for (int q = 0; q < G; ++q) Pi[q] = g.psig[q] ? t1[q] : t0[q];
  }
  y_at<G>(F, fs, eo, g, yi);
  ld_vec<G>(F, 4u * fs + eo, bi);
  const double di = S.dinv ? gptr(S.dinv)[rr] : 0.0;
  if (live) {
    const float dv = S.dinv ? (float)di : 1.0f / (asum == 0.0f ? 1.0f : asum);
    float xo[G], yo[G];
#pragma unroll
    for (int q = 0; q < G; ++q) {
      const float P0 = ((g.zp >> q) & 1) ? 0.0f : Pi[q];
      const float gr = acc[q] - bi[q];
      const float xi = yi[q] - dv * gr;
      const float d = xi - P0;
      xo[q] = xi;
      yo[q] = xi + g.bnext[q] * d;
      if ((g.act >> q) & 1) {
        const double g64 = (double)gr, d64 = (double)d;
        ps[q] = ps[q] + g64 * d64;
        pgg[q] = pgg[q] + g64 * g64;
      }
    }
    const uint32_t er = elem<4>(row, lk, (uint32_t)j0);
    if (g.all && g.prot >= 0) {   // one W buffer for the group: one vector store
      st_vec<G>(S.fb, (uint32_t)(1 - g.prot) * fs + er, xo);
    } else {
#pragma unroll
      for (int q = 0; q < G; ++q)
        if ((g.act >> q) & 1) st_at(S.fb, (uint32_t)(1 - g.psig[q]) * fs + er + 4u * q, xo[q]);
    }
    // y^{t+1} for the whole group: a right-hand side that does not use it next pass (not
    // active, or restarting) never reads this slot before rewriting it
    if (g.wyn >= 0) st_vec<G>(S.fb, (uint32_t)g.wyn * fs + er, yo);
  }
}

// The slices of an item in the row form, every right-hand side of the inner phase; the
// wave's sums for right-hand side j are added to lane j's p0, p1.
template <int KP, bool YM>
__device__ __forceinline__ void tile_inner_rows(const BatchSys& S, const BatchTile& T, const PassView* views, int lane,
                                                double& p0, double& p1) {
  constexpr int G = KP < kRowGroup ? KP : kRowGroup;
  constexpr int NG = KP / G;
  using Group = typename std::conditional<YM, InnerGroupY<G>, InnerGroup<G>>::type;
  Group grp[NG];
#pragma unroll
  for (int gi = 0; gi < NG; ++gi) {
    if constexpr (YM) grp[gi] = inner_group_y<G>(views, gi * G);
    else grp[gi] = inner_group<G>(views, gi * G);
  }
  double a[NG][G], b[NG][G];
#pragma unroll
  for (int gi = 0; gi < NG; ++gi)
#pragma unroll
    for (int q = 0; q < G; ++q) a[gi][q] = b[gi][q] = 0.0;
  for (int64_t s = T.s0; s < T.s1; ++s) {
#pragma unroll
    for (int gi = 0; gi < NG; ++gi)
      if (grp[gi].act) {
        if constexpr (YM) slice_inner_rows_ym<G>(S, s, lane, gi * G, grp[gi], a[gi], b[gi]);
        else slice_inner_rows<G>(S, s, lane, gi * G, grp[gi], a[gi], b[gi]);
      }
  }
#pragma unroll
  for (int gi = 0; gi < NG; ++gi)
#pragma unroll
    for (int q = 0; q < G; ++q) {
      const double sa = wave_sum(a[gi][q]), sb = wave_sum(b[gi][q]);
      if (lane == gi * G + q) {
        p0 = p0 + sa;
        p1 = p1 + sb;
      }
    }
}

// An item's units of one phase: its long rows with every lane (the lanes of the phase
// keep the results), then its slices (kp units of 64/kp rows each) with the lanes of
// the phase only.  A lane adds its long rows, then its slice rows, in order.
template <int PH>
__device__ __forceinline__ void item_phase(const BatchSys& S, const BatchTile& T, int lane, const PassView& v,
                                           double& p0, double& p1, double& p2) {
  const int lk = S.lk;
  const bool mine = v.phase == PH;
  for (int64_t r = T.l0; r < T.l1; ++r) {
    if (PH == PH_ITER) long_iter(S, r, lane, v, mine, p0, p1, p2);
    if (PH == PH_INNER32) long_inner(S, r, lane, v, mine, p0, p1, p2);
    if (PH == PH_RESID64) long_resid_mixed(S, r, lane, v, mine, p0, p1);
    if (PH == PH_CONFIRM) long_resid(S, r, lane, v, mine, p0);
    if (PH == PH_NORMB && mine && lane < (1 << lk)) {
      const double x = ld_at((const double*)S.b, elem<8>(r, lk, (uint32_t)lane));
      p0 = p0 + x * x;
    }
  }
  if (mine && PH != PH_INNER32) {   // float32 inner slices run in the row form
    const int nu = (T.s1 - T.s0) << lk;
    for (int u = 0; u < nu; ++u) {
      const int64_t s = (int64_t)T.s0 + (u >> lk);
      const int sub = u & ((1 << lk) - 1);
      if (PH == PH_ITER) unit_iter(S, s, sub, lane, v, p0, p1, p2);
      if (PH == PH_INNER32) unit_inner(S, s, sub, lane, v, p0, p1, p2);
      if (PH == PH_RESID64) unit_resid_mixed(S, s, sub, lane, v, p0, p1);
      if (PH == PH_CONFIRM) unit_resid(S, s, sub, lane, v, p0);
      if (PH == PH_NORMB) unit_normb(S, s, sub, lane, p0);
    }
  }
}

// One item for every lane's instance, one phase after another (each phase present among
// the system's right-hand sides runs once; MIXED selects the phases of the refinement
// loop, else those of the float64 solve).  Leaves right-hand side j's sums in lane j.
template <bool MIXED, int KPMAX>
__device__ __forceinline__ void batch_item(const BatchSys& S, const BatchTile& T, const PassView& v, int lane,
                                           double& p0, double& p1, double& p2) {
  const int kp = 1 << S.lk;
  p0 = p1 = p2 = 0.0;
  if (MIXED) {
    if (__any(v.phase == PH_RESID64)) item_phase<PH_RESID64>(S, T, lane, v, p0, p1, p2);
    if (__any(v.phase == PH_INNER32))
      item_phase<PH_INNER32>(S, T, lane, v, p0, p1, p2);   // long rows (and slices, materialized form)
  } else {
    if (__any(v.phase == PH_ITER)) item_phase<PH_ITER>(S, T, lane, v, p0, p1, p2);
    if (__any(v.phase == PH_CONFIRM)) item_phase<PH_CONFIRM>(S, T, lane, v, p0, p1, p2);
  }
  if (__any(v.phase == PH_NORMB)) item_phase<PH_NORMB>(S, T, lane, v, p0, p1, p2);
  // long-row sums sit in lanes < kp only, slice sums in every lane: the butterfly over the
  // row bits gives lane j < kp the wave's sum for right-hand side j either way
  p0 = rhs_sum(p0, kp);
  p1 = rhs_sum(p1, kp);
  p2 = rhs_sum(p2, kp);
  if (MIXED && __any(v.phase == PH_INNER32)) {
    // float32 inner slices in the row form (materialized form for several right-hand
    // sides: mixed batches set it for every such system); a right-hand side is in one
    // phase only, so one of the two terms added to lane j is zero
    if (KPMAX >= 8 && kp == 8) tile_inner_rows<(KPMAX >= 8 ? 8 : 1), true>(S, T, S.vt, lane, p0, p1);
    else if (KPMAX >= 4 && kp == 4) tile_inner_rows<(KPMAX >= 4 ? 4 : 1), true>(S, T, S.vt, lane, p0, p1);
    else if (KPMAX >= 2 && kp == 2) tile_inner_rows<(KPMAX >= 2 ? 2 : 1), true>(S, T, S.vt, lane, p0, p1);
    else if (S.ymode) tile_inner_rows<1, true>(S, T, S.vt, lane, p0, p1);
    else tile_inner_rows<1, false>(S, T, S.vt, lane, p0, p1);
  }
}

// One pass of every active instance of the batch.  Each wavefront takes items of the
// active list on its own (no workgroup barrier): the list is cut into one contiguous
// range per L2 domain, and the domain's wavefronts take its items in turn.  The next
// item's index and descriptor are loaded while the current one is worked on.  KPMAX is
// the most right-hand-side lanes of any system (the row form's registers grow with it,
// so a kernel for one right-hand side per system stays lean).
template <bool MIXED, int KPMAX>
__global__ void __launch_bounds__(kBatchBlock) k_batch_pass(BatchArgs ba) {
  const int lane = threadIdx.x % kWave;
  const int nact = uni(*gptr(ba.nactive));
  const SliceRange r = slice_range(nact, ba.nxcd, (int)gridDim.x, (int)blockIdx.x, wave_id(), kBatchWaves);
  int sys = -1;
  BatchSys S;
  PassView v;
  bool live = false;
  int p = (int)r.first;
  int t = p < r.end ? uni(gptr(ba.active)[p]) : 0;
  while (p < r.end) {
    const int pn = p + (int)r.step;
    const int tn = pn < r.end ? gptr(ba.active)[pn] : 0;   // in flight during this item
    const NAJ_GLOBAL BatchTile& Tg = gptr(ba.tiles)[t];
    BatchTile T;
    T.sys = uni(Tg.sys);
    T.s0 = uni(Tg.s0);
    T.s1 = uni(Tg.s1);
    T.l0 = uni(Tg.l0);
    T.l1 = uni(Tg.l1);
    if (T.sys != sys) {   // consecutive items mostly share a system: its record and views are kept
      sys = T.sys;
      S = uniform_sys(ba.sys[sys]);
      const NAJ_GLOBAL PassView& g = gptr(S.vt)[lane & ((1 << S.lk) - 1)];
      v.phase = g.phase;
      v.iP = g.iP;
      v.iR = g.iR;
      v.iW = g.iW;
      v.bz = g.bz;
      v.zp = g.zp;
      v.iX = g.iX;
      v.iXn = g.iXn;
      v.iD = g.iD;
      v.update = g.update;
      v.iYn = g.iYn;
      v.beta = g.beta;
      v.beta_next = g.beta_next;
      live = __any(v.phase != PH_DONE);
    }
    if (live) {
      double p0, p1, p2;
      batch_item<MIXED, KPMAX>(S, T, v, lane, p0, p1, p2);
      if (lane < S.nrhs && v.phase != PH_DONE) {
        double* slot = S.part + ((size_t)lane * S.ntiles + (t - S.tile0)) * kPartStride;
        slot[0] = p0;
        slot[1] = p1;
        slot[2] = p2;
      }
    }
    p = pn;
    t = uni(tn);
  }
}

// The pass kernel for a precision and the most right-hand-side lanes of any system.
inline const void* batch_pass_kernel(bool mixed, int kpmax) {
  if (!mixed) return (const void*)k_batch_pass<false, 8>;
  if (kpmax <= 1) return (const void*)k_batch_pass<true, 1>;
  if (kpmax <= 2) return (const void*)k_batch_pass<true, 2>;
  if (kpmax <= 4) return (const void*)k_batch_pass<true, 4>;
  return (const void*)k_batch_pass<true, 8>;
}

// After a pass: for every system with an unfinished instance (one workgroup each), the
// items' partial sums of each instance, the scalar decision, and the view of the next pass.
// The workgroup's 8 wavefronts are shared out among the right-hand-side lanes kp (the power
// of two >= k): 8/kp wavefronts per right-hand side, so the instances decide concurrently and
// a system with one right-hand side adds its items with all 8.  Wavefront part q of a
// right-hand side adds items q*64 + l, q*64 + l + 64*8/kp, ... in lane l, then a fixed
// butterfly over the lanes, then the parts are added in order q = 0, 1, ...; the order
// depends only on the system's item count and right-hand-side count.
constexpr int kDecideBlock = kWave * kMaxRhs;

__global__ void __launch_bounds__(kDecideBlock) k_batch_decide(BatchArgs ba) {
  __shared__ double ws[kDecideBlock / kWave][3];
  const int nsact = uni(*gptr(ba.nsact));
  if ((int)blockIdx.x >= nsact) return;
  const int sys = uni(gptr(ba.sact)[blockIdx.x]);
  const BatchSys S = uniform_sys(ba.sys[sys]);
  const int w = wave_id();
  const int wpr = (kDecideBlock / kWave) >> S.lk;   // wavefronts per right-hand side
  const int j = w / wpr, q = w % wpr;
  const int lane = (int)threadIdx.x % kWave;
  const bool act = j < S.nrhs && uni(gptr(S.vt)[j].phase) != PH_DONE;
  double r0 = 0.0, r1 = 0.0, r2 = 0.0;
  if (act) {
    const NAJ_GLOBAL double* part = gptr(S.part) + (size_t)j * S.ntiles * kPartStride;
#pragma unroll 4
    for (int i = q * kWave + lane; i < S.ntiles; i += wpr * kWave) {
      r0 = r0 + part[(size_t)i * kPartStride + 0];
      r1 = r1 + part[(size_t)i * kPartStride + 1];
      r2 = r2 + part[(size_t)i * kPartStride + 2];
    }
    r0 = wave_sum(r0);
    r1 = wave_sum(r1);
    r2 = wave_sum(r2);
  }
  if (lane == 0) {
    ws[w][0] = r0;
    ws[w][1] = r1;
    ws[w][2] = r2;
  }
  __syncthreads();
  if (act && q == 0 && lane == 0) {
    double s0 = ws[w][0], s1 = ws[w][1], s2 = ws[w][2];
    for (int k = 1; k < wpr; ++k) {
      s0 = s0 + ws[w + k][0];
      s1 = s1 + ws[w + k][1];
      s2 = s2 + ws[w + k][2];
    }
    const SolveArgs a = batch_ctrl_args(ba, S);
    Ctrl* c = S.ctrl + j;
    control_update(a, c, s0, s1, s2);
    load_view(c, S.vt + j);
    if (c->phase == PH_DONE) __hip_atomic_fetch_add(ba.done, 1u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();   // the views written above are visible to the workgroup
  if (ba.slot_done && threadIdx.x == 0) {
    bool all = true;
    for (int k = 0; k < S.nrhs; ++k) all = all && S.vt[k].phase == PH_DONE;
    if (all) ba.slot_done[sys] = S.gen;
  }
}

// The active lists: the systems with an unfinished instance, and their items, in system
// order.  One workgroup; systems are taken in chunks of its size.
constexpr int kCompactBlock = 1024;

__global__ void __launch_bounds__(kCompactBlock) k_batch_compact(BatchArgs ba) {
  __shared__ int off[kCompactBlock];
  __shared__ int flag[kCompactBlock];
  __shared__ int base, sbase;
  if (threadIdx.x == 0) base = sbase = 0;
  __syncthreads();
  for (int c0 = 0; c0 < ba.nsys; c0 += kCompactBlock) {
    const int i = c0 + (int)threadIdx.x;
    int cnt = 0;
    if (i < ba.nsys) {
      const BatchSys& S = ba.sys[i];
      bool act = false;
      for (int j = 0; j < S.nrhs; ++j) act = act || S.vt[j].phase != PH_DONE;
      cnt = act ? S.ntiles : 0;
    }
    off[threadIdx.x] = cnt;
    flag[threadIdx.x] = cnt > 0 ? 1 : 0;
    __syncthreads();
    // inclusive scans of the item counts and of the active flags
    for (int d = 1; d < kCompactBlock; d <<= 1) {
      const int add = (int)threadIdx.x >= d ? off[threadIdx.x - d] : 0;
      const int addf = (int)threadIdx.x >= d ? flag[threadIdx.x - d] : 0;
      __syncthreads();
      off[threadIdx.x] += add;
      flag[threadIdx.x] += addf;
      __syncthreads();
    }
    const int b0 = base, sb0 = sbase;
    const int hi = min(kCompactBlock, ba.nsys - c0);
    if ((int)threadIdx.x < hi && cnt > 0) ba.sact[sb0 + flag[threadIdx.x] - 1] = i;
    // the whole workgroup writes the item ids of one system after another
    for (int q = 0; q < hi; ++q) {
      const int start = q ? off[q - 1] : 0, end = off[q];
      if (start == end) continue;
      const int tile0 = ba.sys[c0 + q].tile0;
      for (int k = start + (int)threadIdx.x; k < end; k += kCompactBlock) ba.active[b0 + k] = tile0 + (k - start);
    }
    __syncthreads();
    if (threadIdx.x == 0) {
      base = b0 + off[hi - 1];
      sbase = sb0 + flag[hi - 1];
    }
    __syncthreads();
  }
  if (threadIdx.x == 0) {
    *ba.nactive = base;
    *ba.nsact = sbase;
  }
}

// Control block of instance j of a system at the start of a solve (as k_solve_init), and
// its first pass view.
__device__ inline void batch_ctrl_start(const BatchArgs& ba, const BatchSys& S, int j) {
  Ctrl* c = S.ctrl + j;
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
  c->best_mon = __builtin_inf();
  c->best_t = 0;
  c->iYn = -1;
  c->beta_next = 0.0;
  if (S.ymode) {
    c->iP = 0;
    c->iW = 1;
    c->iR = 2;
    ymode_plan_next(c);
  }
  for (int q = 0; q < kRestartLogCap; ++q) c->restart_log[q] = 0;
  load_view(c, S.vt + j);
}

__device__ inline void batch_view_done(const BatchSys& S, int j) {
  PassView v = {};
  v.phase = PH_DONE;
  S.vt[j] = v;
}

// Per solve: start every instance's control block and clear the done counter.  One
// workgroup of kMaxRhs threads per system.
__global__ void k_batch_init(BatchArgs ba) {
  const int i = blockIdx.x;
  if (i >= ba.nsys) return;
  const BatchSys& S = ba.sys[i];
  const int j = threadIdx.x;
  if (i == 0 && j == 0) *ba.done = 0u;
  if (j >= kMaxRhs) return;
  if (j < S.nrhs) batch_ctrl_start(ba, S, j);
  else batch_view_done(S, j);
}

// Serving loop: a request enters slot `slot`: its record, its work items (long rows four
// per item, then `tslices` slices per item) and its control blocks.  Runs on the pass
// stream between chunks of passes, so the next active-list rebuild picks the slot up.
__global__ void k_server_admit(BatchArgs ba, int slot, BatchSys rec, int tslices, int nlt) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    const_cast<BatchSys*>(ba.sys)[slot] = rec;
    ba.slot_done[slot] = 0;
  }
  if (i < kMaxRhs) {
    if (i < rec.nrhs) batch_ctrl_start(ba, rec, i);
    else batch_view_done(rec, i);
  }
  if (i < rec.ntiles) {
    BatchTile t;
    t.sys = slot;
    if (i < nlt) {
      t.s0 = t.s1 = 0;
      t.l0 = i * 4;
      t.l1 = (int)min((int64_t)t.l0 + 4, rec.A.n_long);
    } else {
      t.l0 = t.l1 = 0;
      t.s0 = (i - nlt) * tslices;
      t.s1 = (int)min((int64_t)t.s0 + tslices, rec.A.nslices);
    }
    const_cast<BatchTile*>(ba.tiles)[rec.tile0 + i] = t;
  }
}

// Serving loop: a slot is emptied (no instance, so the active-list rebuild skips it).
__global__ void k_server_clear(BatchArgs ba, int slot) {
  if (threadIdx.x == 0 && blockIdx.x == 0) const_cast<BatchSys*>(ba.sys)[slot].nrhs = 0;
}

// Right-hand sides (or starting points) of one system into its interleaved buffer:
// caller layout n x k row-interleaved in caller row order -> n x kp in the system's order.
__global__ void k_batch_load(const double* src, int k, int kp, const int32_t* perm, int64_t n, double* dst) {
  const int64_t total = n * kp;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = q / kp;
    const int j = (int)(q % kp);
    const int64_t o = perm ? perm[i] : i;
    dst[q] = (src && j < k) ? src[o * k + j] : 0.0;
  }
}

// Answers of one system back into the caller's row-interleaved x (each right-hand
// side from the buffer its control block names).
__global__ void k_batch_store(const BatchSys* sys, int si, int k, const int32_t* perm, int64_t n, double* x) {
  const BatchSys& S = sys[si];
  const int64_t total = n * k;
  for (int64_t q = blockIdx.x * (int64_t)blockDim.x + threadIdx.x; q < total; q += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = q / k;
    const int j = (int)(q % k);
    const int r = S.ctrl[j].result;
    const int64_t o = perm ? perm[i] : i;
    x[o * k + j] = r < 0 ? 0.0 : ld_at((const double*)S.xb, (uint32_t)r * S.xs + elem<8>(i, S.lk, (uint32_t)j));
  }
}

}  // namespace naj
