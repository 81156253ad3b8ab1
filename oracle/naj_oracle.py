"""CPU oracle for the accelerated Jacobi-type method with adaptive restart.

TEST INFRASTRUCTURE ONLY.  This module is the plain, slow reference that the
GPU path is checked against.  Only the test suite, the smoke check and the
CPU-baseline leg of the benchmark may import it; the product path never does.
It shares no code with the HIP library: every step below is written from the
paper (Liang, Pang, Toh, Yang, "Nesterov's accelerated Jacobi-type methods for
large-scale symmetric positive semidefinite linear systems", arXiv 2407.03272).

What it computes
----------------
For a consistent system Q x = b with Q symmetric positive semidefinite
(Section 1, eq. (eq-linear-sys)), Algorithm 3 (Section 3) runs Algorithm 2's
accelerated, restarted template with the proximal matrix S = J - Q, which
turns the proximal subproblem of Algorithm 1 into the Jacobi-type step

    x^t = y^t + J^{-1} (b - Q y^t)            (Section 3, the displayed update)

with J the diagonal of eq. (J-diag): J_kk = Q_kk + sum_{j != k} |Q_kj|.  The
momentum step is y^{t+1} = x^t + beta_t (x^t - x^{t-1}) with
beta_t = (alpha_t - 1)/alpha_{t+1} and alpha_{t+1} = (1 + sqrt(1 + 4 alpha_t^2))/2
(Algorithm 1).  The restart test of Algorithm 2/3 fires when
t > K_re + K_l and <Q y^t - b, x^t - x^{t-1}> >= 0; it sets K_re = t,
K_{l+1} = 2 K_l, l = l + 1, alpha_{t+1} = 1, y^{t+1} = x^{t-1} and
x^t = x^{t-1}.

Readings where the paper leaves a choice open (all shared with the GPU path
by specification, not by code):

* x^0 defaults to 0; K_0 defaults to 2 (the paper only requires K_0 >= 2).
* Stopping: by default on the relative residual ||b - Q x^t|| / ||b|| <= tol.
  The residual at y^t, ||Q y^t - b||, comes free with the step and is the
  monitor; when it is <= tol the residual at x^t is computed (one extra
  product) and the run stops if that is <= tol.  After a failed
  confirmation the next one waits ``confirm_gap`` iterations.  At t = 1,
  y^1 = x^0, so a monitor <= tol returns x^0 with 0 iterations.
  With ``stop="objective"`` the criterion is the paper's own (Section 4):
  |f(x^t) - f*| / (1 + |f*|) <= tol with f* given.  The monitor is then the
  same gap at y^t, f(y^t) = sum_i y_i (u_i / 2 - b_i) with u = Q y^t (free
  with the step), and the confirmation evaluates f(x^t) with one extra
  product.  Since x^t minimizes f + ||. - y^t||_S^2 / 2 (Lemma 1),
  f(x^t) <= f(y^t): a monitor <= tol implies the criterion at x^t in exact
  arithmetic, and the stop can come a few iterations after the first x^t
  that meets it.
* A restart iteration counts as an iteration (its product was spent).
* The table of update rules in Section 4 writes Q x^t in the accelerated
  Jacobi row; Algorithm 3 writes Q y^t, which is what is done here.
* A row of Q that is entirely zero gives J_kk = 0; J_kk := 1 is used there.
* The momentum step is formed as x + beta*d with d = x - x_prev (equal to
  (1+beta) x - beta x_prev in exact arithmetic).
* The diagonal of eq. (J-diag) equals the row absolute sum sum_j |Q_kj|
  because Q_kk >= 0 for a positive semidefinite Q; it is computed that way.
"""
from __future__ import annotations

import math
from dataclasses import dataclass, field
from decimal import Decimal, getcontext
from typing import Callable, Iterable

import numpy as np
import scipy.sparse as sp

STATUS_OK = 0
STATUS_NOT_CONVERGED = 1
STATUS_BREAKDOWN = -4

# The stall test of the float32 inner solve applies once its monitor has halved.
STALL_ARM = 0.5


def csr(rowptr, colidx, vals, dtype=np.float64) -> sp.csr_matrix:
    n = len(rowptr) - 1
    return sp.csr_matrix((np.asarray(vals, dtype=dtype), np.asarray(colidx), np.asarray(rowptr)),
                         shape=(n, n))


def jacobi_diagonal(Q: sp.csr_matrix) -> np.ndarray:
    """Diagonal J of eq. (J-diag), Section 3: J_kk = Q_kk + sum_{j != k} |Q_kj|.

    Computed as the row absolute sums |Q| 1 (a row-by-row sum in stored
    order, in Q's own precision), which is the same quantity for PSD Q.
    A zero row gives J_kk = 0, replaced by 1.
    """
    absQ = abs(Q)
    J = np.asarray(absQ @ np.ones(Q.shape[0], dtype=Q.dtype))
    J = J.copy()
    J[J == 0] = 1
    return J


def block_jacobi_blocks(Q: sp.csr_matrix, nb: int) -> np.ndarray:
    """Diagonal blocks of the block-diagonal J of eq. (J-blkdiag), Section 3.

    The rows are partitioned into s = ceil(n / nb) blocks of nb consecutive
    rows (Section 3's partition of Q into blocks Q^{i,j} with n_i rows; here
    n_i = nb, the last block keeping the n - (s-1) nb rows that remain), and

        J^{i,i} = Q^{i,i} + sum_{j != i} ||Q^{i,j}||_2 I_{n_i}.

    The spectral norms are taken by the library SVD of each nonzero
    off-diagonal block, and added to the shift in increasing j.  A zero
    diagonal entry of J^{i,i} (a zero row of Q in a block coupled to no other
    block) is replaced by 1, as for the diagonal J.  Returns an array of shape
    (s, nb, nb); rows and columns of the last block beyond n are those of the
    identity.
    """
    n = Q.shape[0]
    s = -(-n // nb)
    C = Q.tocoo()
    r, c, v = C.row.astype(np.int64), C.col.astype(np.int64), C.data.astype(np.float64)
    bi, bj = r // nb, c // nb
    Jb = np.zeros((s, nb, nb))
    diag = bi == bj
    np.add.at(Jb, (bi[diag], r[diag] % nb, c[diag] % nb), v[diag])
    off = ~diag
    key = bi[off] * s + bj[off]
    keys, grp = np.unique(key, return_inverse=True)
    M = np.zeros((len(keys), nb, nb))
    np.add.at(M, (grp, r[off] % nb, c[off] % nb), v[off])
    norms = np.linalg.norm(M, ord=2, axis=(1, 2)) if len(keys) else np.zeros(0)
    shift = np.zeros(s)
    for g, k in enumerate(keys):          # keys ascend in (i, j): each shift sums its norms in increasing j
        i = int(k // s)
        shift[i] = shift[i] + norms[g]
    for i in range(s):
        ni = min(nb, n - i * nb)
        for k in range(ni):
            Jb[i, k, k] = Jb[i, k, k] + shift[i]
            if Jb[i, k, k] == 0.0:
                Jb[i, k, k] = 1.0
        for k in range(ni, nb):
            Jb[i, k, k] = 1.0
    return Jb


def block_solve(Jb: np.ndarray, g: np.ndarray) -> np.ndarray:
    """z = J^{-1} g for the block-diagonal J: one dense solve per block (library LU)."""
    s, nb, _ = Jb.shape
    n = g.shape[0]
    gp = np.zeros(s * nb)
    gp[:n] = g
    return np.linalg.solve(Jb, gp.reshape(s, nb, 1))[:, :, 0].reshape(-1)[:n]


def block_matrix(Jb: np.ndarray, n: int) -> np.ndarray:
    """The dense n x n block-diagonal J assembled from its blocks (small systems only)."""
    s, nb, _ = Jb.shape
    J = np.zeros((s * nb, s * nb))
    for i in range(s):
        J[i * nb:(i + 1) * nb, i * nb:(i + 1) * nb] = Jb[i]
    return J[:n, :n]


def objective(Q: sp.csr_matrix, b: np.ndarray, x: np.ndarray) -> float:
    """f(x) = 1/2 <x, Q x> - <b, x>, eq. (eq-qp)."""
    return 0.5 * float(x @ (Q @ x)) - float(b @ x)


def alpha_next(alpha: float) -> float:
    """alpha_{t+1} = (1 + sqrt(1 + 4 alpha_t^2)) / 2 (Algorithm 1)."""
    return (1.0 + math.sqrt(1.0 + 4.0 * alpha * alpha)) / 2.0


def fused_step(rowptr, colidx, vals, p, r, beta, b, D=None, jblock=None):
    """One pass of Algorithm 3's row update with the momentum point formed from two iterates.

    y = p + beta (p - r) (y = p when beta == 0; Algorithm 1, momentum step),
    x = y + J^{-1}(b - Q y) (Section 3 update; J of eq. (J-diag), the caller's
    D, or the block J of eq. (J-blkdiag) with blocks of ``jblock`` rows), and the reductions the restart
    test and the monitor use: s = <Q y - b, x - p>, gg = ||Q y - b||^2,
    sabs = sum |(Q y - b)_i (x - p)_i|.  Returns (x, s, gg, sabs).
    """
    Q = csr(rowptr, colidx, vals)
    p = np.asarray(p, dtype=np.float64)
    y = p.copy() if beta == 0.0 else p + beta * (p - np.asarray(r, dtype=np.float64))
    g = Q @ y - np.asarray(b, dtype=np.float64)
    if jblock is not None:
        x = y - block_solve(block_jacobi_blocks(Q, jblock), g)
    else:
        J = jacobi_diagonal(Q) if D is None else np.asarray(D, dtype=np.float64)
        dinv = 1.0 / J
        x = y - dinv * g
    d = x - p
    return x, float(g @ d), float(g @ g), float(np.abs(g * d).sum())


@dataclass
class OracleResult:
    x: np.ndarray
    iterations: int
    status: int
    hist: list = field(default_factory=list)          # ||Q y^t - b|| / ||b||, t = 1..T
    restarts: list = field(default_factory=list)      # iterations t at which a restart fired
    s_log: list = field(default_factory=list)         # <Q y^t - b, x^t - x^{t-1}>
    sabs_log: list = field(default_factory=list)      # sum_i |g_i d_i| (scale of s_t, for near-tie checks)
    confirms: list = field(default_factory=list)      # (t, ||b - Q x^t|| / ||b||)
    relres: float = float("nan")                      # residual of the returned x (when computed)
    objgap: float = float("nan")                      # objective stop: |f(x) - f*| / (1 + |f*|) of the returned x


def accelerated_jacobi(rowptr, colidx, vals, b, x0=None, *, tol: float = 1e-8, max_iter: int = 5000,
                       restart: bool = True, k0: int = 2, D: np.ndarray | None = None,
                       confirm_gap: int = 8, forced_restarts: Iterable[int] | None = None,
                       callback: Callable | None = None, jblock: int | None = None,
                       stop: str = "relres", fstar: float | None = None) -> OracleResult:
    """Algorithm 3 (Section 3) with diagonal J, in float64.

    ``restart`` is the IsRestart switch of Algorithm 3 (False gives Algorithm 1
    with S = J - Q).  ``D`` replaces J when given (Remark 1 allows any
    invertible J with J - Q PSD).  ``jblock`` selects the block-diagonal J of
    eq. (J-blkdiag) with blocks of that many consecutive rows (Algorithm 3 with
    its block update).  ``stop="objective"`` with ``fstar`` stops on the
    relative objective gap of Section 4 (see the module notes); the result's
    ``relres`` is then still the relative residual of the returned x and
    ``objgap`` its gap.  ``forced_restarts``, when given, replaces
    the restart test by that exact set of iterations (used to replay a run
    whose restart test was a numerical tie).  ``callback(t, info)`` sees every
    iteration's vectors (used by invariant tests).
    """
    Q = csr(rowptr, colidx, vals)
    n = Q.shape[0]
    b = np.asarray(b, dtype=np.float64)
    if jblock is not None:
        Jb = block_jacobi_blocks(Q, jblock)

        def jinv_apply(g):
            return block_solve(Jb, g)
    else:
        J = jacobi_diagonal(Q) if D is None else np.asarray(D, dtype=np.float64).copy()
        dinv = 1.0 / J

        def jinv_apply(g):
            return dinv * g
    x0 = np.zeros(n) if x0 is None else np.asarray(x0, dtype=np.float64).copy()
    forced = None if forced_restarts is None else set(int(t) for t in forced_restarts)

    res = OracleResult(x=x0.copy(), iterations=0, status=STATUS_OK)
    nb = float(np.linalg.norm(b))
    if nb == 0.0:
        res.x = np.zeros(n)
        res.relres = 0.0
        res.objgap = 0.0 if stop == "objective" else float("nan")
        return res
    if stop == "objective":
        if fstar is None:
            raise ValueError("the objective stop needs f*")
        fscale = 1.0 + abs(float(fstar))

        def monitor(y, u, g):
            # f(y) = <y, Q y>/2 - <b, y> = sum_i y_i (u_i/2 - b_i), eq. (eq-qp)
            return abs(float(y @ (0.5 * u - b)) - fstar) / fscale

        def check(x):
            return abs(float(x @ (0.5 * (Q @ x) - b)) - fstar) / fscale
    elif stop == "relres":
        def monitor(y, u, g):
            return float(np.linalg.norm(g)) / nb

        def check(x):
            return float(np.linalg.norm(b - Q @ x)) / nb
    else:
        raise ValueError(f"unknown stop {stop!r}")

    def finish(x):
        res.x = x
        if stop == "objective":
            res.objgap = check(x)
            res.relres = float(np.linalg.norm(b - Q @ x)) / nb

    # Algorithm 3 input: x^0 = y^1, alpha_1 = 1, l = 0, K_0, K_re = 0
    x_prev = x0.copy()
    y = x0.copy()
    alpha = 1.0
    K_re, K, ell = 0, int(k0), 0
    last_confirm = -(1 << 62)
    for t in range(1, max_iter + 1):
        # Jacobi-type step of Section 3: x^t = y^t + J^{-1}(b - Q y^t)
        u = Q @ y
        g = u - b
        x = y - jinv_apply(g)
        mon = monitor(y, u, g)
        res.hist.append(mon)
        if not math.isfinite(mon):
            res.x, res.iterations, res.status = x_prev, t, STATUS_BREAKDOWN
            return res
        if t == 1 and mon <= tol:
            res.x, res.iterations, res.relres = x0, 0, mon
            finish(x0)
            return res
        if mon <= tol and t >= last_confirm + confirm_gap:
            rho = check(x)
            last_confirm = t
            res.confirms.append((t, rho))
            if rho <= tol:
                res.x, res.iterations, res.relres = x, t, rho
                finish(x)
                if callback is not None:
                    callback(t, dict(x=x, y=y, x_prev=x_prev, alpha=alpha, restarted=False, final=True))
                return res
        # restart test of Algorithm 2/3: <Q y^t - b, x^t - x^{t-1}> >= 0 past the prohibition period
        d = x - x_prev
        s = float(g @ d)
        res.s_log.append(s)
        res.sabs_log.append(float(np.abs(g * d).sum()))
        if not math.isfinite(s):
            res.x, res.iterations, res.status = x_prev, t, STATUS_BREAKDOWN
            return res
        if forced is not None:
            do_restart = t in forced
        else:
            do_restart = restart and t > K_re + K and s >= 0.0
        if callback is not None:
            callback(t, dict(x=x, y=y, x_prev=x_prev, alpha=alpha, restarted=do_restart, final=False))
        if do_restart:
            # restart branch: K_re = t, K_{l+1} = 2 K_l, l += 1, alpha_{t+1} = 1, y^{t+1} = x^{t-1}, x^t = x^{t-1}
            K_re = t
            K = 2 * K
            ell += 1
            res.restarts.append(t)
            a_next = 1.0
            y = x_prev.copy()
        else:
            # momentum branch: alpha_{t+1}, y^{t+1} = x^t + beta_t (x^t - x^{t-1})
            a_next = alpha_next(alpha)
            beta = (alpha - 1.0) / a_next
            y = x + beta * d
            x_prev = x
        alpha = a_next
    res.x, res.iterations, res.status = x_prev, max_iter, STATUS_NOT_CONVERGED
    res.relres = float(np.linalg.norm(b - Q @ x_prev)) / nb
    finish(x_prev)
    return res


@dataclass
class MixedResult:
    x: np.ndarray
    status: int
    outer: int                                   # FP64 residual evaluations
    inner_total: int                             # FP32 inner iterations summed over refinement steps
    relres_hist: list = field(default_factory=list)   # ||b - Q x_k|| / ||b|| per refinement step
    inner_iters: list = field(default_factory=list)
    inner_restarts: list = field(default_factory=list)


def block_apply_fp32(jinv32: np.ndarray, g: np.ndarray) -> np.ndarray:
    """z = fl32(J^{-1}) g in float32 for the block-diagonal J, block by block.

    ``jinv32[i, r, k]`` is entry (r, k) of fl32((J^{i,i})^{-1}); each z_r adds the
    products of its block's columns k = 0, 1, ... in that order, in float32.
    """
    f32 = np.float32
    s, nb, _ = jinv32.shape
    n = g.shape[0]
    gp = np.zeros(s * nb, dtype=f32)
    gp[:n] = g
    G = gp.reshape(s, nb)
    z = (jinv32[:, :, 0] * G[:, 0:1]).astype(f32)
    for k in range(1, nb):
        z = (z + (jinv32[:, :, k] * G[:, k:k + 1]).astype(f32)).astype(f32)
    return z.reshape(-1)[:n]


def inner_solve_fp32(Q32: sp.csr_matrix, dinv32: np.ndarray, r32: np.ndarray, *, inner_tol: float,
                     max_iter: int, restart: bool, k0: int, stall: int = 200, log: list | None = None):
    """Algorithm 3 on Q d = r in float32 from d^0 = 0 with float64 reductions.

    ``dinv32`` is the float32 diagonal of J^{-1}, or, for the block J of
    eq. (J-blkdiag), the stack of float32 inverse blocks (``block_apply_fp32``).

    The product, the Jacobi-type step and the momentum step are float32
    operations (float32 accumulation in the row sums; the momentum coefficient
    rounded to float32).  The restart inner product and the monitor norm are
    accumulated in float64 from the exactly converted float32 operands.  The
    solve stops when ||Q y^t - r|| / ||r|| <= inner_tol and returns x^t; or,
    once the recorded best monitor value is <= STALL_ARM, when the monitor has
    not fallen below 0.9 times that best value for ``stall`` iterations
    (float32 rounding of the row sums bounds how far the float32 residual can
    fall, about eps32 times the condition number) and returns x^t; or returns
    the last iterate after ``max_iter`` iterations.  The best value is updated
    only when the monitor falls to 0.9 times it or below.  Before the monitor
    has halved, a plateau is the slow start of the method on a smooth
    right-hand side (it lasts about the square root of the condition number),
    not the float32 floor, so the stall test is not applied.
    ``log``, when given, receives the monitor value of every iteration (for tests).
    Returns (d, iterations, restarts, finite).
    """
    n = Q32.shape[0]
    f32 = np.float32
    r64 = r32.astype(np.float64)
    nr = math.sqrt(float(r64 @ r64))
    x_prev = np.zeros(n, dtype=f32)
    y = np.zeros(n, dtype=f32)
    alpha = 1.0
    K_re, K = 0, int(k0)
    restarts = []
    best, best_t = math.inf, 0
    for t in range(1, max_iter + 1):
        u = Q32 @ y
        g = (u - r32).astype(f32)
        x = (y - (dinv32 * g if dinv32.ndim == 1 else block_apply_fp32(dinv32, g))).astype(f32)
        g64 = g.astype(np.float64)
        mon = math.sqrt(float(g64 @ g64)) / nr
        if log is not None:
            log.append(mon)
        d = (x - x_prev).astype(f32)
        s = float(g64 @ d.astype(np.float64))
        if not (math.isfinite(mon) and math.isfinite(s)):
            return x_prev, t, restarts, False
        if mon <= inner_tol:
            return x, t, restarts, True
        if mon <= 0.9 * best:
            best, best_t = mon, t
        if stall > 0 and best <= STALL_ARM and t - best_t >= stall:
            return x, t, restarts, True
        if restart and t > K_re + K and s >= 0.0:
            K_re, K = t, 2 * K
            restarts.append(t)
            a_next = 1.0
            y = x_prev.copy()
        else:
            a_next = alpha_next(alpha)
            beta = f32((alpha - 1.0) / a_next)
            y = (x + beta * d).astype(f32)
            x_prev = x
        alpha = a_next
    return x_prev, max_iter, restarts, True


def accelerated_jacobi_mixed(rowptr, colidx, vals, b, x0=None, *, tol: float = 1e-8, max_refine: int = 50,
                             inner_tol: float = 1e-4, inner_max_iter: int = 20000, restart: bool = True,
                             k0: int = 2, D: np.ndarray | None = None, inner_stall: int = 200,
                             jblock: int | None = None) -> MixedResult:
    """Float32 inner Algorithm 3 inside float64 iterative refinement.

    Outer step k = 0, 1, ...: r_k = b - Q x_k with float64 values and
    accumulation; stop when ||r_k|| / ||b|| <= tol, or (NOT_CONVERGED) when k
    reaches ``max_refine`` or fl32(r_k) is zero; otherwise solve Q d = fl32(r_k)
    approximately with ``inner_solve_fp32`` (float32 copy of Q, J from the
    float32 row absolute sums, or fl32(1/D) for a caller diagonal, or for the
    block J of eq. (J-blkdiag) with blocks of ``jblock`` rows fl32 of the
    float64 inverse of each block) and set
    x_{k+1} = x_k + d in float64.  A non-finite inner reduction ends the solve
    with BREAKDOWN and x_k.  The refinement loop is not part of the paper; the
    paper's algorithm is the inner solver.
    """
    Q = csr(rowptr, colidx, vals)
    Q32 = csr(rowptr, colidx, np.asarray(vals, dtype=np.float32), dtype=np.float32)
    n = Q.shape[0]
    if jblock is not None:
        dinv32 = np.linalg.inv(block_jacobi_blocks(Q, jblock)).astype(np.float32)
    elif D is None:
        J32 = jacobi_diagonal(Q32)
        dinv32 = (np.float32(1.0) / J32).astype(np.float32)
    else:
        dinv32 = (1.0 / np.asarray(D, dtype=np.float64)).astype(np.float32)
    b = np.asarray(b, dtype=np.float64)
    x = np.zeros(n) if x0 is None else np.asarray(x0, dtype=np.float64).copy()
    nb = float(np.linalg.norm(b))
    out = MixedResult(x=x, status=STATUS_OK, outer=0, inner_total=0)
    if nb == 0.0:
        out.x = np.zeros(n)
        return out
    for k in range(max_refine + 1):
        r = b - Q @ x
        rho = float(np.linalg.norm(r)) / nb
        out.outer += 1
        out.relres_hist.append(rho)
        out.x = x
        if not math.isfinite(rho):
            out.status = STATUS_BREAKDOWN
            return out
        if rho <= tol:
            return out
        r32 = r.astype(np.float32)
        if k == max_refine or not np.any(r32):
            break
        d, it, rs, finite = inner_solve_fp32(Q32, dinv32, r32, inner_tol=inner_tol, max_iter=inner_max_iter,
                                             restart=restart, k0=k0, stall=inner_stall)
        out.inner_total += it
        out.inner_iters.append(it)
        out.inner_restarts.append(rs)
        if not finite:
            out.status = STATUS_BREAKDOWN
            return out
        x = x + d.astype(np.float64)
    out.status = STATUS_NOT_CONVERGED
    return out


# ----------------------------------------------------------------------------
# Section 4.1 worked example, reduced to two scalars
# ----------------------------------------------------------------------------

def sdd_scalar_run(n: int, *, tol: float = 1e-8, max_iter: int = 5000, restart: bool = True, k0: int = 2,
                   confirm_gap: int = 8, digits: int = 60, stop: str = "relres"):
    """Algorithm 3 on the Section 4.1 system in high-precision scalar arithmetic.

    Q = (n+1) I - 1 1^T, b = 1, x^0 = 0.  Q 1 = 1, so every iterate is a
    multiple of the all-ones vector: y^t = eta_t 1, x^t = xi_t 1.  With
    J = (2n - 1) I from eq. (J-diag):  Q y^t - b = (eta_t - 1) 1,
    xi_t = eta_t - (eta_t - 1)/(2n - 1), the restart inner product is
    n (eta_t - 1)(xi_t - xi_{t-1}), ||Q y^t - b||/||b|| = |eta_t - 1| and
    ||b - Q x^t||/||b|| = |1 - xi_t|.  With ``stop="objective"``: x* = 1,
    f* = -n/2 and f(eta 1) - f* = n (eta - 1)^2 / 2, so the monitor and the
    confirmation are n (eta_t - 1)^2 / (2 + n) and n (xi_t - 1)^2 / (2 + n).
    Same control flow and readings as ``accelerated_jacobi``; arithmetic in
    ``digits``-digit decimals.
    Returns dict(iterations, status, restarts, xi (list), hist (list), xhat (list)); xi holds the
    accepted x^t of every iteration (x^{t-1} after a restart), xhat the computed Jacobi-type step.
    """
    getcontext().prec = digits
    one = Decimal(1)
    J = Decimal(2 * n - 1)
    tol_d = Decimal(repr(tol))
    xi_prev = Decimal(0)
    eta = Decimal(0)
    alpha = one
    K_re, K = 0, k0
    last_confirm = -(1 << 62)
    restarts, xis, hist, xhat = [], [], [], []
    obj = stop == "objective"
    fs = Decimal(n) / (Decimal(2) + Decimal(n))

    def gap(v):
        return fs * (v - one) * (v - one) if obj else abs(v - one)

    for t in range(1, max_iter + 1):
        g = eta - one
        xi = eta - g / J
        xhat.append(xi)
        mon = gap(eta)
        hist.append(mon)
        if t == 1 and mon <= tol_d:
            return dict(iterations=0, status=STATUS_OK, restarts=restarts, xi=[Decimal(0)], hist=hist, xhat=xhat)
        if mon <= tol_d and t >= last_confirm + confirm_gap:
            last_confirm = t
            if gap(xi) <= tol_d:
                xis.append(xi)
                return dict(iterations=t, status=STATUS_OK, restarts=restarts, xi=xis, hist=hist, xhat=xhat)
        d = xi - xi_prev
        s = Decimal(n) * g * d
        if restart and t > K_re + K and s >= 0:
            K_re, K = t, 2 * K
            restarts.append(t)
            a_next = one
            eta = xi_prev
            xis.append(xi_prev)
        else:
            a_next = (one + (one + 4 * alpha * alpha).sqrt()) / 2
            beta = (alpha - one) / a_next
            eta = xi + beta * d
            xi_prev = xi
            xis.append(xi)
        alpha = a_next
    return dict(iterations=max_iter, status=STATUS_NOT_CONVERGED, restarts=restarts, xi=xis, hist=hist, xhat=xhat)


# ----------------------------------------------------------------------------
# plain definitions the limits are checked against
# ----------------------------------------------------------------------------

def dense_solution_spd(rowptr, colidx, vals, b) -> np.ndarray:
    """x* = Q^{-1} b by dense Cholesky (small SPD systems only)."""
    Q = csr(rowptr, colidx, vals).toarray()
    L = np.linalg.cholesky(Q)
    z = np.linalg.solve(L, b)
    return np.linalg.solve(L.T, z)


def dense_limit_spsd(rowptr, colidx, vals, b, x0, J=None) -> np.ndarray:
    """The solution the method converges to on a consistent singular system (small systems only).

    Each step is J-affine and N^T Q = 0, N^T b = 0 for a null-space basis N, so
    N^T J x^t = N^T J x^0 for every t (follows from the update of Section 3).
    The limit is therefore x_p - N (N^T J N)^{-1} N^T J (x_p - x^0), with
    x_p = Q^+ b the minimum-norm solution.  ``J`` is the diagonal (a vector) or
    a dense symmetric J (the block-diagonal J of eq. (J-blkdiag)).
    """
    Qs = csr(rowptr, colidx, vals)
    Q = Qs.toarray()
    if J is None:
        J = jacobi_diagonal(Qs)
    w, V = np.linalg.eigh(Q)
    thr = 1e-9 * max(1.0, abs(w).max())
    N = V[:, np.abs(w) <= thr]
    xp = np.linalg.pinv(Q, rcond=1e-12, hermitian=True) @ b
    if N.shape[1] == 0:
        return xp
    JN = J[:, None] * N if np.ndim(J) == 1 else J @ N
    c = np.linalg.solve(N.T @ JN, JN.T @ (xp - x0))
    return xp - N @ c
