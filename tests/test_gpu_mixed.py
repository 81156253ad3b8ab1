"""GPU parity of the mixed-precision path (float32 inner Algorithm 3 inside float64 refinement).

The mixed oracle (oracle.accelerated_jacobi_mixed) performs the same float32
and float64 operations in the same order per row, so with the same inner
restart and stop decisions the GPU result is expected to be bit-identical;
the bar checked is relative 1e-10 against the mixed oracle, plus the
float64 relative residual <= 1e-8 recomputed by the oracle's own product,
and the error against the float64 oracle solution (stated per case).
"""
import numpy as np
import pytest

import oracle as O
from paper_2407_03272_amd import workloads as W

pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def naj():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2407_03272_amd import naj as N
    N.load()
    return N


def _say(*a):
    print("[gpu-case]", *a, flush=True)


def _kappa_dirichlet(m):
    """Condition number of the Dirichlet Laplacian with m interior points per side: cot^2(pi / (2(m+1)))."""
    return 1.0 / np.tan(np.pi / (2 * (m + 1))) ** 2


def _compare_mixed(naj, sysm, rowptr, colidx, vals, b, *, x0=None, D=None, tol=1e-8, inner_tol=1e-4,
                   max_refine=50, max_iter=20000, **kw):
    orc = O.accelerated_jacobi_mixed(rowptr, colidx, vals, b, x0=x0, D=D, tol=tol, inner_tol=inner_tol,
                                     max_refine=max_refine, inner_max_iter=max_iter, **kw)
    x, info = sysm.solve(b, x0=x0, precision=naj.NAJ_MIXED, tol=tol, inner_tol=inner_tol, max_refine=max_refine,
                         max_iter=max_iter, trace=True, hist_cap=max_refine + 2, **kw)
    xg = x.cpu().numpy()
    assert info.status == orc.status
    assert info.confirmations == orc.outer
    its = [int(v) for v in info.trace[:, 0]]
    assert its[:len(orc.inner_iters)] == orc.inner_iters
    assert info.iterations == orc.inner_total
    np.testing.assert_allclose(info.hist, orc.relres_hist, rtol=1e-8, atol=1e-14)
    scale = max(np.abs(orc.x).max(), 1e-300)
    assert np.abs(xg - orc.x).max() / scale <= 1e-10
    Q = O.csr(rowptr, colidx, vals)
    rel = np.linalg.norm(b - Q @ xg) / np.linalg.norm(b)
    return orc, info, xg, rel


@pytest.mark.parametrize("mode", ["0", "1"])
def test_mixed_poisson2d(naj, mode, monkeypatch):
    _say("mixed poisson2d driver", mode)
    monkeypatch.setenv("NAJ_MODE", mode)
    s = W.poisson2d_64()
    sysm = naj.System(s.rowptr, s.colidx, s.vals)
    monkeypatch.delenv("NAJ_MODE")
    orc, info, xg, rel = _compare_mixed(naj, sysm, s.rowptr, s.colidx, s.vals, s.b)
    assert info.status == 0 and rel <= 1e-8
    assert np.array_equal(xg, orc.x)
    f = O.accelerated_jacobi(s.rowptr, s.colidx, s.vals, s.b, tol=1e-8, max_iter=20000)
    err = np.linalg.norm(xg - f.x) / np.linalg.norm(f.x)
    _say(f"mixed vs float64 oracle solution: rel err {err:.2e}, refinement steps {info.confirmations}, "
         f"inner iterations {info.iterations}")
    # both solutions meet relres 1e-8, so they differ by at most about 2 cond(Q) 1e-8
    assert err <= 2 * _kappa_dirichlet(64) * 1e-8


def test_mixed_ragged_spd_and_user_diagonal(naj):
    _say("mixed ragged spd, user D")
    rowptr, colidx, vals = W.random_spd(1000, 0.02, 5)
    b = np.random.default_rng(11).standard_normal(1000)
    sysm = naj.System(rowptr, colidx, vals)
    orc, info, xg, rel = _compare_mixed(naj, sysm, rowptr, colidx, vals, b, tol=1e-9, inner_tol=1e-5)
    assert info.status == 0 and rel <= 1e-9
    J = O.jacobi_diagonal(O.csr(rowptr, colidx, vals))
    sysd = naj.System(rowptr, colidx, vals, D=1.1 * J)
    orc, info, xg, rel = _compare_mixed(naj, sysd, rowptr, colidx, vals, b, D=1.1 * J, tol=1e-9)
    assert info.status == 0 and rel <= 1e-9


def _modulo_nullspace(rowptr, colidx, vals, x):
    """Remove the J-weighted mean of x on every connected component (the null space of a graph Laplacian)."""
    import scipy.sparse as sp
    from scipy.sparse.csgraph import connected_components
    n = len(rowptr) - 1
    A = sp.csr_matrix((np.ones(len(colidx)), colidx, rowptr), shape=(n, n))
    ncomp, lab = connected_components(A, directed=False)
    J = O.jacobi_diagonal(O.csr(rowptr, colidx, vals))
    m = np.bincount(lab, weights=J * x, minlength=ncomp) / np.bincount(lab, weights=J, minlength=ncomp)
    return x - m[lab]


def test_mixed_singular_laplacian(naj):
    """Singular Chung-Lu Laplacian (power-law degrees; rows longer than 128 go one wavefront per row and sum in
    another order, so float32 rounding differs from the oracle's): the bar is the float64 relative residual
    <= 1e-8 recomputed by the oracle, the refinement step count within one of the mixed oracle's, and the error
    against the float64 oracle solution modulo the null space (per-component J-weighted means removed)."""
    _say("mixed singular chung-lu n=3000")
    s = W.chung_lu_laplacian(3000, 16, 2.5, seed=71, b_seed=72)
    sysm = naj.System(s.rowptr, s.colidx, s.vals)
    x, info = sysm.solve(s.b, precision=naj.NAJ_MIXED, trace=True, hist_cap=64)
    m = O.accelerated_jacobi_mixed(s.rowptr, s.colidx, s.vals, s.b, tol=1e-8)
    xg = x.cpu().numpy()
    Q = O.csr(s.rowptr, s.colidx, s.vals)
    rel = np.linalg.norm(s.b - Q @ xg) / np.linalg.norm(s.b)
    assert info.status == 0 and rel <= 1e-8
    assert abs(info.confirmations - m.outer) <= 1
    f = O.accelerated_jacobi(s.rowptr, s.colidx, s.vals, s.b, tol=1e-10, max_iter=20000)
    dg = _modulo_nullspace(s.rowptr, s.colidx, s.vals, xg)
    df = _modulo_nullspace(s.rowptr, s.colidx, s.vals, f.x)
    err = np.linalg.norm(dg - df) / np.linalg.norm(df)
    _say(f"chung-lu mixed: relres {rel:.2e}, error vs float64 modulo null space {err:.2e}")
    assert err < 1e-5


def test_mixed_edge_cases(naj):
    _say("mixed edge cases")
    s = W.poisson2d_64()
    sysm = naj.System(s.rowptr, s.colidx, s.vals)
    x, info = sysm.solve(np.zeros(s.n), precision=naj.NAJ_MIXED)
    assert info.status == 0 and not x.cpu().numpy().any()
    x, info = sysm.solve(s.b, x0=s.xstar, precision=naj.NAJ_MIXED)     # already converged: one residual pass
    assert info.status == 0 and info.confirmations == 1 and info.iterations == 0
    x, info = sysm.solve(s.b, precision=naj.NAJ_MIXED, max_refine=1, tol=1e-14)
    assert info.status == naj.NAJ_NOT_CONVERGED and info.confirmations == 2
    with pytest.raises(naj.NajError):
        sysm.solve(s.b, precision=naj.NAJ_MIXED, inner_tol=2.0)


def test_mixed_full_size(naj):
    """128^3 Laplacian in the benchmark's launch configuration: relative residual <= 1e-8 by the oracle's own
    float64 product, and the error against the stored float64 oracle solution (sampled entries)."""
    import json
    import os
    _say("mixed 128^3")
    c2 = W.poisson3d_128()
    sysm = naj.System(c2.rowptr, c2.colidx, c2.vals)
    x, info = sysm.solve(c2.b, precision=naj.NAJ_MIXED, trace=True, hist_cap=64)
    xg = x.cpu().numpy()
    assert info.status == 0
    Q = O.csr(c2.rowptr, c2.colidx, c2.vals)
    rel = np.linalg.norm(c2.b - Q @ xg) / np.linalg.norm(c2.b)
    assert rel <= 1e-8 and rel == pytest.approx(info.relres, rel=1e-6)
    ref = [r for r in json.load(open(os.path.join(os.path.dirname(__file__), "golden", "oracle_runs.json")))["runs"]
           if r["name"] == "laplace3d_128"][0]
    idx, sx = np.asarray(ref["sample_idx"]), np.asarray(ref["sample_x"])
    err = np.abs(xg[idx] - sx).max() / np.abs(sx).max()
    _say(f"128^3 mixed: refinement steps {info.confirmations}, inner iterations {info.iterations}, "
         f"relres {rel:.2e}, max sampled rel err vs float64 oracle {err:.2e}")
    assert err <= 2 * _kappa_dirichlet(128) * 1e-8
