"""Pins for the oracle's block-diagonal J (eq. (J-blkdiag), Section 3) and Algorithm 3 run with it.

Each test checks the oracle against a closed form, a brute-force computation with a
different routine, or a statement the paper proves (Lemma 1, Theorem 1, the J-affine
invariant on singular systems), not against the oracle itself.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import oracle as O
from paper_2407_03272_amd import workloads as W

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


def _tiny_spd(n=61, seed=3):
    return W.random_spd(n, 0.08, seed)


def _tiny_laplacian(n=61, seed=5):
    rowptr, colidx, vals, u, v = W.random_laplacian(n, 0.06, seed, weighted=True)
    return rowptr, colidx, vals


def _fe(n=300, seed=9):
    s = W.fe_p1_system(n, 2, seed, nrhs=1)
    return s.rowptr, s.colidx, s.vals


def _brute_blocks(Q, nb):
    """J^{i,i} = Q^{i,i} + sum_{j != i} ||Q^{i,j}||_2 I by a loop over every block pair, with the
    spectral norm as the square root of the largest eigenvalue of M^T M (eigvalsh, not an SVD)."""
    n = Q.shape[0]
    s = -(-n // nb)
    out = []
    for i in range(s):
        ri = slice(i * nb, min(n, (i + 1) * nb))
        shift = 0.0
        for j in range(s):
            if j == i:
                continue
            M = Q[ri, j * nb:min(n, (j + 1) * nb)]
            if np.any(M):
                shift += float(np.sqrt(np.linalg.eigvalsh(M.T @ M).max()))
        out.append(Q[ri, ri] + shift * np.eye(ri.stop - ri.start))
    return out


def test_block_size_one_is_eq_J_diag():
    """With 1 x 1 blocks, ||Q^{i,j}||_2 = |Q_ij|, so eq. (J-blkdiag) is eq. (J-diag) (written as a loop)."""
    rowptr, colidx, vals = _tiny_spd()
    Q = O.csr(rowptr, colidx, vals).toarray()
    ref = np.array([Q[k, k] + sum(abs(Q[k, j]) for j in range(Q.shape[0]) if j != k) for k in range(Q.shape[0])])
    Jb = O.block_jacobi_blocks(O.csr(rowptr, colidx, vals), 1)
    np.testing.assert_allclose(Jb[:, 0, 0], ref, rtol=1e-14, atol=0)


def test_closed_form_1d_laplacian_ragged():
    """1D Dirichlet Laplacian tridiag(-1, 2, -1), n = 18, blocks of 4 (last block 2 rows): each coupling
    block holds a single -1 (norm 1), so J^{i,i} = T_{n_i} + (number of neighbouring blocks) I."""
    n, nb = 18, 4
    Q = sp.diags([-np.ones(n - 1), 2 * np.ones(n), -np.ones(n - 1)], [-1, 0, 1], format="csr")
    Jb = O.block_jacobi_blocks(Q, nb)
    s = 5
    assert Jb.shape == (s, nb, nb)
    for i in range(s):
        ni = min(nb, n - i * nb)
        T = 2 * np.eye(ni) - np.eye(ni, k=1) - np.eye(ni, k=-1)
        neighbours = (i > 0) + (i < s - 1)
        np.testing.assert_array_equal(Jb[i, :ni, :ni], T + neighbours * np.eye(ni))
        np.testing.assert_array_equal(Jb[i, ni:, ni:], np.eye(nb - ni))       # identity padding
        assert not np.any(Jb[i, :ni, ni:]) and not np.any(Jb[i, ni:, :ni])


def test_closed_form_section41_matrix():
    """Q = (n+1) I - 1 1^T (Section 4.1): Q^{i,j} = -1 (n_i x n_j) has norm sqrt(n_i n_j)."""
    n, nb = 10, 4
    Q = sp.csr_matrix((n + 1) * np.eye(n) - np.ones((n, n)))
    Jb = O.block_jacobi_blocks(Q, nb)
    sizes = [4, 4, 2]
    for i, ni in enumerate(sizes):
        shift = sum(np.sqrt(ni * nj) for j, nj in enumerate(sizes) if j != i)
        ref = (n + 1) * np.eye(ni) - np.ones((ni, ni)) + shift * np.eye(ni)
        np.testing.assert_allclose(Jb[i, :ni, :ni], ref, rtol=1e-15, atol=1e-14)


@pytest.mark.parametrize("maker", [_tiny_spd, _tiny_laplacian, _fe])
@pytest.mark.parametrize("nb", [2, 4, 8, 16])
def test_blocks_match_brute_force_and_S_psd(maker, nb):
    """Blocks equal the brute-force eq. (J-blkdiag); S = J - Q is PSD and J is PD (Section 3's claim for a
    Q without zero rows)."""
    rowptr, colidx, vals = maker()
    Qs = O.csr(rowptr, colidx, vals)
    Q = Qs.toarray()
    n = Q.shape[0]
    Jb = O.block_jacobi_blocks(Qs, nb)
    for i, ref in enumerate(_brute_blocks(Q, nb)):
        ni = ref.shape[0]
        np.testing.assert_allclose(Jb[i, :ni, :ni], ref, rtol=1e-13, atol=1e-13 * np.abs(ref).max())
    J = O.block_matrix(Jb, n)
    assert np.linalg.eigvalsh(J - Q).min() >= -1e-12 * np.abs(Q).max()
    assert np.linalg.eigvalsh(J).min() > 0


def test_block_solve_is_J_inverse():
    rowptr, colidx, vals = _tiny_spd()
    Qs = O.csr(rowptr, colidx, vals)
    Jb = O.block_jacobi_blocks(Qs, 8)
    J = O.block_matrix(Jb, Qs.shape[0])
    g = np.random.default_rng(2).standard_normal(Qs.shape[0])
    np.testing.assert_allclose(J @ O.block_solve(Jb, g), g, rtol=0, atol=1e-13 * np.abs(g).max())


def _record(rowptr, colidx, vals, b, **kw):
    rec = []

    def cb(t, info):
        rec.append(dict(t=t, x=info["x"].copy(), y=info["y"].copy(), x_prev=info["x_prev"].copy(),
                        alpha=info["alpha"], restarted=info["restarted"]))
    res = O.accelerated_jacobi(rowptr, colidx, vals, b, callback=cb, **kw)
    return res, rec


@pytest.mark.parametrize("maker", [_tiny_spd, _tiny_laplacian])
def test_block_step_solves_proximal_subproblem(maker):
    """Lemma 1 with the block S = J - Q: Q x^t - b + S (x^t - y^t) = 0 at every iteration."""
    rowptr, colidx, vals = maker()
    Qs = O.csr(rowptr, colidx, vals)
    Q = Qs.toarray()
    S = O.block_matrix(O.block_jacobi_blocks(Qs, 8), Q.shape[0]) - Q
    b = W.rhs_in_range(rowptr, colidx, vals, 11)
    res, rec = _record(rowptr, colidx, vals, b, tol=1e-12, max_iter=300, jblock=8)
    assert len(rec) > 50
    for r in rec:
        resid = Q @ r["x"] - b + S @ (r["x"] - r["y"])
        scale = np.abs(Q) @ np.abs(r["x"]) + np.abs(b) + np.abs(S) @ (np.abs(r["x"]) + np.abs(r["y"]))
        assert np.all(np.abs(resid) <= 1e-12 * scale + 1e-300)


@pytest.mark.parametrize("maker", [_tiny_spd, _tiny_laplacian])
def test_block_theorem1_bound(maker):
    """Algorithm 1 with the block S: 0 <= f(x^t) - f* <= 2 ||x^0 - x*||_S^2 / (t+1)^2 (Theorem 1)."""
    rowptr, colidx, vals = maker()
    b = W.rhs_in_range(rowptr, colidx, vals, 21)
    Qs = O.csr(rowptr, colidx, vals)
    Q = Qs.toarray()
    xs = np.linalg.pinv(Q, rcond=1e-12, hermitian=True) @ b
    fs = 0.5 * xs @ Q @ xs - b @ xs
    S = O.block_matrix(O.block_jacobi_blocks(Qs, 4), Q.shape[0]) - Q
    x0 = np.random.default_rng(1).standard_normal(Q.shape[0])
    res, rec = _record(rowptr, colidx, vals, b, x0=x0, tol=1e-300, max_iter=400, restart=False, jblock=4)
    d0 = x0 - xs
    bound0 = 2 * (d0 @ S @ d0)
    scale = abs(fs) + 1.0
    for r in rec:
        gap = 0.5 * r["x"] @ Q @ r["x"] - b @ r["x"] - fs
        assert -1e-12 * scale <= gap <= bound0 / (r["t"] + 1) ** 2 + 1e-12 * scale


@pytest.mark.parametrize("nb", [4, 16])
def test_block_limit_spd_and_singular_invariant(nb):
    """SPD: the run reaches the Cholesky solution.  Singular Laplacian from a random x^0: N^T J x^t stays
    N^T J x^0 for the block J, and the limit is the pseudoinverse solution shifted to that invariant."""
    rowptr, colidx, vals = _tiny_spd()
    b = np.random.default_rng(3).standard_normal(len(rowptr) - 1)
    res = O.accelerated_jacobi(rowptr, colidx, vals, b, tol=1e-12, max_iter=20000, jblock=nb)
    xs = O.dense_solution_spd(rowptr, colidx, vals, b)
    assert res.status == O.STATUS_OK
    assert np.linalg.norm(res.x - xs) / np.linalg.norm(xs) < 1e-9

    n = 80
    rowptr, colidx, vals, u, v = W.random_laplacian(n, 0.04, 33, weighted=False)
    Qs = O.csr(rowptr, colidx, vals)
    b = W.mean_zero_per_component(n, u, v, np.random.default_rng(4).standard_normal(n))
    x0 = np.random.default_rng(5).standard_normal(n)
    J = O.block_matrix(O.block_jacobi_blocks(Qs, nb), n)
    w, V = np.linalg.eigh(Qs.toarray())
    N = V[:, np.abs(w) <= 1e-9 * np.abs(w).max()]
    assert N.shape[1] >= 2
    inv0 = N.T @ J @ x0
    res, rec = _record(rowptr, colidx, vals, b, x0=x0, tol=1e-11, max_iter=40000, jblock=nb)
    assert res.status == O.STATUS_OK
    for r in rec[::11]:
        xt = r["x_prev"] if r["restarted"] else r["x"]
        np.testing.assert_allclose(N.T @ J @ xt, inv0, rtol=0, atol=1e-9 * (1 + np.abs(inv0).max()))
    xl = O.dense_limit_spsd(rowptr, colidx, vals, b, x0, J)
    assert np.linalg.norm(res.x - xl) / np.linalg.norm(xl) < 1e-7


def test_block_apply_fp32_is_sequential_float32_sum():
    """z_r = sum_k fl32(J^{-1})_{rk} g_k added in increasing k in float32, checked by a per-row loop."""
    rng = np.random.default_rng(6)
    n, nb = 23, 8
    jinv = rng.standard_normal((3, nb, nb)).astype(np.float32)
    g = rng.standard_normal(n).astype(np.float32)
    z = O.block_apply_fp32(jinv, g)
    gp = np.zeros(24, dtype=np.float32)
    gp[:n] = g
    for r in range(n):
        i, rr = divmod(r, nb)
        acc = np.float32(jinv[i, rr, 0] * gp[i * nb])
        for k in range(1, nb):
            acc = np.float32(acc + np.float32(jinv[i, rr, k] * gp[i * nb + k]))
        assert z[r] == acc


def test_block_mixed_reaches_fp64_tolerance():
    """Float32 inner solves with fl32 of the block inverse inside float64 refinement reach 1e-8 (by an
    independent float64 product) and agree with the float64 block solve to the conditioning level."""
    s = W.poisson_system((16, 16, 16), 7)
    m = O.accelerated_jacobi_mixed(s.rowptr, s.colidx, s.vals, s.b, tol=1e-8, jblock=8)
    assert m.status == O.STATUS_OK
    Q = O.csr(s.rowptr, s.colidx, s.vals)
    assert np.linalg.norm(s.b - Q @ m.x) / np.linalg.norm(s.b) <= 1e-8
    f = O.accelerated_jacobi(s.rowptr, s.colidx, s.vals, s.b, tol=1e-8, max_iter=20000, jblock=8)
    assert f.status == O.STATUS_OK
    assert np.linalg.norm(m.x - f.x) / np.linalg.norm(f.x) < 1e-6
