"""Pins for the CPU oracle: each test checks the oracle against something the
paper or plain mathematics fixes, not against the oracle itself.

Citations name the paper's sections, equations, lemmas and theorems
(arXiv 2407.03272).
"""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from paper_2407_03272_amd import workloads as W

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _tiny_spd(n=60, seed=3):
    return W.random_spd(n, 0.08, seed)


def _tiny_laplacian(n=60, seed=5):
    rowptr, colidx, vals, u, v = W.random_laplacian(n, 0.06, seed, weighted=True)
    return rowptr, colidx, vals


def _dense(rowptr, colidx, vals):
    return O.csr(rowptr, colidx, vals).toarray()


def _record(rowptr, colidx, vals, b, **kw):
    """Run the oracle and keep every iterate (x^t after the restart branch, y^t, alpha_t)."""
    rec = []

    def cb(t, info):
        rec.append(dict(t=t, x=info["x"].copy(), y=info["y"].copy(), x_prev=info["x_prev"].copy(),
                        alpha=info["alpha"], restarted=info["restarted"]))
    res = O.accelerated_jacobi(rowptr, colidx, vals, b, callback=cb, **kw)
    return res, rec


# ---------------------------------------------------------------- eq. (J-diag)

@pytest.mark.parametrize("maker", [_tiny_spd, _tiny_laplacian])
def test_jacobi_diagonal_is_eq_J_diag(maker):
    """J_kk = Q_kk + sum_{j!=k} |Q_kj| (eq. (J-diag)), written out with a dense double loop."""
    rowptr, colidx, vals = maker()
    Q = _dense(rowptr, colidx, vals)
    n = Q.shape[0]
    ref = np.empty(n)
    for k in range(n):
        acc = Q[k, k]
        for j in range(n):
            if j != k:
                acc += abs(Q[k, j])
        ref[k] = acc if acc != 0 else 1.0
    J = O.jacobi_diagonal(O.csr(rowptr, colidx, vals))
    np.testing.assert_allclose(J, ref, rtol=1e-14, atol=0)


@pytest.mark.parametrize("maker", [_tiny_spd, _tiny_laplacian])
def test_S_is_psd_and_J_positive(maker):
    """With no zero row, S = J - Q is PSD and J is positive definite (Section 3, after eq. (J-blkdiag))."""
    rowptr, colidx, vals = maker()
    Q = _dense(rowptr, colidx, vals)
    J = O.jacobi_diagonal(O.csr(rowptr, colidx, vals))
    assert (J > 0).all()
    lam = np.linalg.eigvalsh(np.diag(J) - Q)
    assert lam.min() >= -1e-12 * np.abs(Q).max()


def test_diag_of_Q_can_break_S_psd():
    """Using diag(Q) as J can make S indefinite (Section 4.3 remark): a bipartite Laplacian shows it."""
    # path graph on 4 vertices (bipartite): lambda_max(L) > 2 max deg ... S = diag(L) - L has eigenvalue < 0
    u = np.array([0, 1, 2]); v = np.array([1, 2, 3])
    rowptr, colidx, vals = W._laplacian_from_edges(4, u, v)
    Q = _dense(rowptr, colidx, vals)
    S_bad = np.diag(np.diag(Q)) - Q
    assert np.linalg.eigvalsh(S_bad).min() < -1e-3
    J = O.jacobi_diagonal(O.csr(rowptr, colidx, vals))
    assert np.linalg.eigvalsh(np.diag(J) - Q).min() >= -1e-12


# ---------------------------------------------------------------- product and step

def test_spmv_exact_on_integer_matrix():
    """Integer Q and small-integer y: every row sum is exact in float64, so the product must equal a brute-force loop."""
    rowptr, colidx, vals = W.poisson_dirichlet((7, 5, 3))
    n = len(rowptr) - 1
    rng = np.random.default_rng(0)
    y = rng.integers(-50, 50, n).astype(np.float64)
    ref = np.zeros(n)
    for i in range(n):
        for k in range(rowptr[i], rowptr[i + 1]):
            ref[i] += vals[k] * y[colidx[k]]
    got = O.csr(rowptr, colidx, vals) @ y
    assert np.array_equal(got, ref)


@pytest.mark.parametrize("maker", [_tiny_spd, _tiny_laplacian])
def test_step_solves_proximal_subproblem(maker):
    """Lemma 1's optimality condition with S = J - Q: Q x^t - b + S (x^t - y^t) = 0 at every iteration
    (x^t is the argmin of the proximal subproblem of Algorithms 1/2; Section 3 turns it into the Jacobi-type step)."""
    rowptr, colidx, vals = maker()
    Q = _dense(rowptr, colidx, vals)
    J = O.jacobi_diagonal(O.csr(rowptr, colidx, vals))
    S = np.diag(J) - Q
    b = W.rhs_in_range(rowptr, colidx, vals, 11)
    res, rec = _record(rowptr, colidx, vals, b, tol=1e-12, max_iter=300)
    assert len(rec) > 50
    for r in rec:
        resid = Q @ r["x"] - b + S @ (r["x"] - r["y"])
        scale = np.abs(Q) @ np.abs(r["x"]) + np.abs(b) + np.abs(S) @ (np.abs(r["x"]) + np.abs(r["y"]))
        assert np.all(np.abs(resid) <= 1e-13 * scale + 1e-300)


def test_alpha_recurrence_identities():
    """alpha_0 = 0, alpha_1 = 1: alpha_{t-1}^2 = alpha_t(alpha_t - 1) (Lemma 2 proof) and alpha_t >= (t+1)/2 (Theorem 1 proof)."""
    a = [0.0, 1.0]
    for _ in range(2000):
        a.append(O.alpha_next(a[-1]))
    for t in range(1, len(a)):
        assert a[t - 1] ** 2 == pytest.approx(a[t] * (a[t] - 1.0), rel=1e-12, abs=1e-15)
        assert a[t] >= (t + 1) / 2


# ---------------------------------------------------------------- Lemma 2 / Theorem 1 (no restart)

def _fstar_and_xstar(rowptr, colidx, vals, b):
    Q = _dense(rowptr, colidx, vals)
    xs = np.linalg.pinv(Q, rcond=1e-12, hermitian=True) @ b
    fs = 0.5 * xs @ Q @ xs - b @ xs
    return Q, xs, fs


@pytest.mark.parametrize("maker", [_tiny_spd, _tiny_laplacian])
def test_lyapunov_nonincreasing_and_theorem1(maker):
    """Algorithm 1 (IsRestart = False): E_t = alpha_t^2 (f(x^t) - f*) + 1/2 <w^t, S w^t> is non-increasing
    (Lemma 2) and 0 <= f(x^t) - f* <= 2 ||x^0 - x*||_S^2 / (t+1)^2 (Theorem 1)."""
    rowptr, colidx, vals = maker()
    b = W.rhs_in_range(rowptr, colidx, vals, 21)
    Q, xs, fs = _fstar_and_xstar(rowptr, colidx, vals, b)
    J = O.jacobi_diagonal(O.csr(rowptr, colidx, vals))
    S = np.diag(J) - Q
    rng = np.random.default_rng(1)
    x0 = rng.standard_normal(Q.shape[0])
    res, rec = _record(rowptr, colidx, vals, b, x0=x0, tol=1e-300, max_iter=400, restart=False)
    f = lambda x: 0.5 * x @ Q @ x - b @ x
    scale = abs(fs) + 1.0
    d0 = x0 - xs
    bound0 = 2 * (d0 @ S @ d0)
    E_prev = 0.5 * d0 @ S @ d0  # E_0 with alpha_0 = 0 and w^0 = x^0 - x*
    for r in rec:
        t, a, x, xp = r["t"], r["alpha"], r["x"], r["x_prev"]
        gap = f(x) - fs
        assert gap >= -1e-12 * scale
        assert gap <= bound0 / (t + 1) ** 2 + 1e-12 * scale
        w = a * x - (a - 1.0) * xp - xs
        E = a * a * gap + 0.5 * w @ S @ w
        assert E <= E_prev + 1e-10 * (scale + E_prev)
        E_prev = E


def test_lemma3_no_restart_descent():
    """Without restarts f(x^t) <= f(x^0) for all t (Lemma 3, first claim)."""
    rowptr, colidx, vals = _tiny_spd(80, 9)
    b = W.rhs_in_range(rowptr, colidx, vals, 4)
    Q = _dense(rowptr, colidx, vals)
    x0 = np.random.default_rng(2).standard_normal(Q.shape[0])
    f = lambda x: 0.5 * x @ Q @ x - b @ x
    res, rec = _record(rowptr, colidx, vals, b, x0=x0, tol=1e-300, max_iter=300, restart=False)
    f0 = f(x0)
    for r in rec:
        assert f(r["x"]) <= f0 + 1e-12 * (abs(f0) + 1)


# ---------------------------------------------------------------- restart: Lemma 3, Theorem 2, schedule

@pytest.mark.parametrize("k0", [2, 3, 8])
def test_restart_schedule_and_theorem2(k0):
    """Algorithm 2/3 with restart on an SPD system:
    * epoch-start values f(x^{l,0}) are non-increasing and f(x^{l,k}) <= f(x^{l,0}) (Lemma 3);
    * f(x^t) - f* <= 2 R^2 (log2 t)^2 / t^2 for t >= 2 (Theorem 2), R^2 = sup over the level set of
      ||x - x*||_S^2 = 2 (f(x^0) - f*) lambda_max(Q^{-1/2} S Q^{-1/2});
    * restarts only past the prohibition period: gap since the last restart > K_0 2^l, and
      l <= log2(t + 2) - 1 (Theorem 2 proof);
    * every restart saw <Q y^t - b, x^t - x^{t-1}> >= 0 and no eligible iteration skipped one (the restart test of Algorithm 2)."""
    rowptr, colidx, vals = _tiny_spd(120, 17)
    Q = _dense(rowptr, colidx, vals)
    rng = np.random.default_rng(3)
    xs = rng.standard_normal(Q.shape[0])
    b = Q @ xs
    fs = 0.5 * xs @ Q @ xs - b @ xs
    J = O.jacobi_diagonal(O.csr(rowptr, colidx, vals))
    S = np.diag(J) - Q
    x0 = np.zeros_like(b)
    f = lambda x: 0.5 * x @ Q @ x - b @ x
    res, rec = _record(rowptr, colidx, vals, b, x0=x0, tol=1e-13, max_iter=3000, restart=True, k0=k0)
    assert len(res.restarts) >= 2
    w, V = np.linalg.eigh(Q)
    Qmh = V @ np.diag(w ** -0.5) @ V.T
    R2 = 2 * (f(x0) - fs) * np.linalg.eigvalsh(Qmh @ S @ Qmh).max()
    scale = abs(fs) + 1
    epoch_start = f(x0)
    starts = [epoch_start]
    K_re, K, ell = 0, k0, 0
    for r in rec:
        t = r["t"]
        g = Q @ r["y"] - b
        s = g @ (r["x"] - r["x_prev"])
        tie = abs(s) <= 64 * len(b) * np.finfo(float).eps * np.abs(g * (r["x"] - r["x_prev"])).sum()
        eligible = t > K_re + K
        if r["restarted"]:
            assert eligible and (s >= 0 or tie)
            assert t - K_re > k0 * 2 ** ell
            K_re, K, ell = t, 2 * K, ell + 1
            assert ell <= math.log2(t + 2) - 1 + 1e-12
            xt = r["x_prev"]  # x^t := x^{t-1}
            new_start = f(xt)
            assert new_start <= starts[-1] + 1e-12 * scale
            starts.append(new_start)
        else:
            xt = r["x"]
            if eligible and not tie:
                assert s < 0
            assert f(xt) <= starts[-1] + 1e-12 * scale
        if t >= 2:
            assert f(xt) - fs <= 2 * R2 * math.log2(t) ** 2 / t ** 2 + 1e-12 * scale


# ---------------------------------------------------------------- limits

@pytest.mark.parametrize("seed", [0, 1, 2])
def test_limit_matches_cholesky_on_spd(seed):
    """On SPD systems the run converges to Q^{-1} b (dense Cholesky); error <= cond(Q) * tol."""
    rowptr, colidx, vals = W.random_spd(150, 0.05, 100 + seed)
    rng = np.random.default_rng(seed)
    b = rng.standard_normal(150)
    res = O.accelerated_jacobi(rowptr, colidx, vals, b, tol=1e-12, max_iter=50000)
    assert res.status == O.STATUS_OK
    xc = O.dense_solution_spd(rowptr, colidx, vals, b)
    kappa = np.linalg.cond(_dense(rowptr, colidx, vals))
    assert np.linalg.norm(res.x - xc) / np.linalg.norm(xc) <= kappa * 1e-12 * 4
    assert res.relres <= 1e-12


def test_limit_on_singular_laplacian_and_invariant():
    """Consistent singular Laplacian with a random x^0: sum_k J_k x_k^t is constant on every connected
    component at every t (the step is J-affine and N^T b = 0), and the limit is the pseudoinverse
    solution shifted to that invariant (Section 4.2 defines the Laplacian; Q 1 = 0)."""
    n = 80
    rowptr, colidx, vals, u, v = W.random_laplacian(n, 0.04, 33, weighted=False)
    Qs = O.csr(rowptr, colidx, vals)
    Q = Qs.toarray()
    assert np.abs(Q @ np.ones(n)).max() == 0.0
    from scipy.sparse.csgraph import connected_components
    ncomp, lab = connected_components(sp.csr_matrix((np.ones(len(u)), (u, v)), shape=(n, n)), directed=False)
    assert ncomp >= 2  # the invariant must hold per component
    b = W.mean_zero_per_component(n, u, v, np.random.default_rng(4).standard_normal(n))
    x0 = np.random.default_rng(5).standard_normal(n)
    J = O.jacobi_diagonal(Qs)
    inv0 = np.bincount(lab, weights=J * x0, minlength=ncomp)
    res, rec = _record(rowptr, colidx, vals, b, x0=x0, tol=1e-11, max_iter=20000)
    assert res.status == O.STATUS_OK
    for r in rec[::7]:
        xt = r["x_prev"] if r["restarted"] else r["x"]
        inv = np.bincount(lab, weights=J * xt, minlength=ncomp)
        np.testing.assert_allclose(inv, inv0, rtol=0, atol=1e-10 * (1 + np.abs(inv0).max()))
    xl = O.dense_limit_spsd(rowptr, colidx, vals, b, x0, J)
    assert np.linalg.norm(res.x - xl) / np.linalg.norm(xl) < 1e-7


# ---------------------------------------------------------------- Section 4.1 worked example

@pytest.mark.parametrize("n", [1000, 2000])
@pytest.mark.parametrize("restart", [True, False])
def test_sdd_vector_run_matches_scalar_reduction(n, restart):
    """Section 4.1 system Q = (n+1)I - 11^T, b = 1, x* = 1: the float64 sparse run must follow the
    two-scalar reduction computed in 60-digit decimals (same iteration count, same restarts,
    x^t = xi_t 1) and end near x* = 1."""
    sys_ = W.sdd_system(n)
    ref = O.sdd_scalar_run(n, tol=1e-8, max_iter=5000, restart=restart)
    res = O.accelerated_jacobi(sys_.rowptr, sys_.colidx, sys_.vals, sys_.b, tol=1e-8, max_iter=5000,
                               restart=restart)
    assert res.iterations == ref["iterations"]
    assert res.restarts == ref["restarts"]
    xi = float(ref["xi"][-1])
    assert np.abs(res.x - xi).max() <= 1e-10 * abs(xi)
    assert res.status == ref["status"]
    if res.status == O.STATUS_OK:
        assert np.abs(res.x - 1.0).max() <= 1e-8


def test_sdd_scalar_reduction_closed_form():
    """The scalar reduction's fixed point is the known solution x* = 1 (Section 4.1), and with restart
    it needs fewer iterations than without (the section's qualitative claim)."""
    for n in (1000, 3000):
        on = O.sdd_scalar_run(n, tol=1e-10)
        off = O.sdd_scalar_run(n, tol=1e-10, restart=False)
        assert on["status"] == O.STATUS_OK
        assert abs(float(on["xi"][-1]) - 1.0) <= 1e-10
        assert on["iterations"] < off["iterations"]


# ---------------------------------------------------------------- algebraic invariances

def test_power_of_two_scaling_is_bitwise_invariant():
    """(2^k Q, 2^k b) scales J by 2^k, so x^t = y^t + J^{-1}(b - Q y^t) is unchanged bit for bit."""
    s = W.poisson2d_64()
    a = O.accelerated_jacobi(s.rowptr, s.colidx, s.vals, s.b, tol=1e-8, max_iter=3000)
    c = O.accelerated_jacobi(s.rowptr, s.colidx, s.vals * 8.0, s.b * 8.0, tol=1e-8, max_iter=3000)
    assert a.iterations == c.iterations and a.restarts == c.restarts
    assert np.array_equal(a.x, c.x)


def test_forced_schedule_replays_bitwise():
    """Replaying a run with its own restart schedule forced gives the identical result (near-tie replay tool)."""
    s = W.poisson2d_64()
    a = O.accelerated_jacobi(s.rowptr, s.colidx, s.vals, s.b, tol=1e-8, max_iter=3000)
    c = O.accelerated_jacobi(s.rowptr, s.colidx, s.vals, s.b, tol=1e-8, max_iter=3000,
                             forced_restarts=a.restarts)
    assert a.iterations == c.iterations and np.array_equal(a.x, c.x)


def test_restart_beats_no_restart_on_poisson():
    """Adaptive restart reduces iterations (Section 2.2 motivation; Section 4.1 observation)."""
    s = W.poisson2d_64()
    a = O.accelerated_jacobi(s.rowptr, s.colidx, s.vals, s.b, tol=1e-8, max_iter=20000)
    c = O.accelerated_jacobi(s.rowptr, s.colidx, s.vals, s.b, tol=1e-8, max_iter=20000, restart=False)
    assert a.status == c.status == O.STATUS_OK
    assert a.iterations < c.iterations


# ---------------------------------------------------------------- edge cases of the readings

def test_zero_rhs_and_converged_start():
    s = W.poisson2d_64()
    r = O.accelerated_jacobi(s.rowptr, s.colidx, s.vals, np.zeros(s.n), tol=1e-8)
    assert r.iterations == 0 and r.status == O.STATUS_OK and not r.x.any()
    r2 = O.accelerated_jacobi(s.rowptr, s.colidx, s.vals, s.b, x0=s.xstar, tol=1e-8)
    assert r2.iterations == 0 and np.array_equal(r2.x, s.xstar)


def test_zero_row_keeps_component_and_inconsistent_rhs_does_not_converge():
    """A zero row gets J_kk = 1: with b_k = 0 the component stays at x^0_k; with b_k != 0 the system is
    inconsistent (b not in range(Q), excluded by Section 1) and the run ends NOT_CONVERGED."""
    rowptr, colidx, vals, u, v = W.random_laplacian(40, 0.1, 8)
    deg = np.diff(rowptr)
    Q = O.csr(rowptr, colidx, vals)
    # make vertex 0 isolated by removing its edges
    A = Q.tolil()
    for j in A.rows[0][:]:
        if j != 0:
            A[0, j] = 0; A[j, 0] = 0; A[j, j] -= 1
    A[0, 0] = 0
    A = A.tocsr(); A.eliminate_zeros(); A.sort_indices()
    rp, ci, va = A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data
    assert rp[1] - rp[0] == 0 and deg[0] > 1
    b = W.rhs_in_range(rp, ci, va, 3)
    x0 = np.full(40, 0.25)
    r = O.accelerated_jacobi(rp, ci, va, b, x0=x0, tol=1e-9, max_iter=20000)
    assert r.status == O.STATUS_OK and r.x[0] == 0.25
    b2 = b.copy(); b2[0] = 1.0
    r2 = O.accelerated_jacobi(rp, ci, va, b2, x0=x0, tol=1e-9, max_iter=500)
    assert r2.status == O.STATUS_NOT_CONVERGED


def test_nan_rhs_is_breakdown():
    s = W.poisson2d_64()
    b = s.b.copy(); b[5] = np.nan
    r = O.accelerated_jacobi(s.rowptr, s.colidx, s.vals, b, tol=1e-8)
    assert r.status == O.STATUS_BREAKDOWN


# ---------------------------------------------------------------- mixed precision (refinement around the paper's solver)

def test_mixed_refinement_reaches_fp64_tolerance():
    """Float32 inner Algorithm 3 + float64 refinement reaches ||b - Qx||/||b|| <= 1e-8 (checked by an
    independent float64 product) and agrees with the float64 solve to the conditioning level."""
    s = W.poisson_system((24, 24, 24), 7)
    m = O.accelerated_jacobi_mixed(s.rowptr, s.colidx, s.vals, s.b, tol=1e-8)
    assert m.status == O.STATUS_OK
    Q = O.csr(s.rowptr, s.colidx, s.vals)
    assert np.linalg.norm(s.b - Q @ m.x) / np.linalg.norm(s.b) <= 1e-8
    f = O.accelerated_jacobi(s.rowptr, s.colidx, s.vals, s.b, tol=1e-8, max_iter=20000)
    assert np.linalg.norm(m.x - f.x) / np.linalg.norm(f.x) < 1e-6
    assert m.outer >= 2 and all(it > 0 for it in m.inner_iters)


def test_mixed_on_singular_laplacian_modulo_nullspace():
    n = 3000
    s = W.chung_lu_laplacian(n, 16, 2.5, seed=71, b_seed=72)
    m = O.accelerated_jacobi_mixed(s.rowptr, s.colidx, s.vals, s.b, tol=1e-8)
    assert m.status == O.STATUS_OK
    Q = O.csr(s.rowptr, s.colidx, s.vals)
    assert np.linalg.norm(s.b - Q @ m.x) / np.linalg.norm(s.b) <= 1e-8
