"""Parity at the benchmark workloads' full sizes, in the configuration bench.py times.

* Chung-Lu graph Laplacian, n = 2^22 (sorted layout, long rows): the complete float64 solve against the
  oracle (every restart decision checked along the GPU's trajectory by the near-tie rule of tie_rule.py,
  iterates within 1e-10), and the mixed solve to relres 1e-8 by the oracle's product, its error against the
  float64 oracle's answer stated and bounded after removing each connected component's J-weighted mean
  (the method keeps that mean at its starting value on every component, so answers of the singular system
  are compared modulo its null space).
* The 512-system finite-element batch, 8 right-hand sides each, with autotuned work items: every one of the
  4096 instances reaches relres 1e-8 by an independent float64 product, and sampled regular-layout
  instances equal the mixed oracle bit for bit (the oracle computes them one by one).

* The 160^3 and 192^3 Laplacians (in and beyond the MALL, too large for the oracle's complete run): relres
  by an independent host product, and bit-for-bit agreement of the iterates with the slice order (160^3)
  and with the 8-byte slice-order solve (192^3).

The 128^3 Laplacian at full size is covered in test_gpu_parity.py against a stored oracle run.
"""
import os

import numpy as np
import pytest

import oracle as O
import tie_rule as TR
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


def _component_mean_free(rowptr, colidx, vals, x):
    """x minus its J-weighted mean (J = absolute row sums, 1 on zero rows) on each connected component."""
    import scipy.sparse as sps
    from scipy.sparse.csgraph import connected_components
    n = len(rowptr) - 1
    A = sps.csr_matrix((np.abs(vals), colidx, rowptr), shape=(n, n))
    J = np.asarray(A.sum(axis=1)).ravel()
    J[J == 0] = 1.0
    nc, lab = connected_components(A, directed=False)
    mean = np.bincount(lab, weights=J * x, minlength=nc) / np.bincount(lab, weights=J, minlength=nc)
    return x - mean[lab]


def test_chunglu_4m_full_size(naj):
    _say("full size: Chung-Lu n=2^22")
    s = W.chung_lu_laplacian()
    sysm = naj.System(s.rowptr, s.colidx, s.vals)
    assert sysm.info()["layout"] == 1
    x, info = sysm.solve(s.b, tol=1e-8, max_iter=20000, trace=True)
    orc = O.accelerated_jacobi(s.rowptr, s.colidx, s.vals, s.b, tol=1e-8, max_iter=20000)
    if info.restart_log != orc.restarts or info.iterations != orc.iterations:
        orc = O.accelerated_jacobi(s.rowptr, s.colidx, s.vals, s.b, tol=1e-8, max_iter=20000,
                                   forced_restarts=info.restart_log)
    # long rows sum in another order, so the iterates are not bit-identical: the GPU's restart inner
    # products must agree with the oracle's to 1e-6 of sum|g_i d_i|, and any decision that differs must be
    # a tie (|s_t| <= 4 n eps sum|g_i d_i| + the measured difference)
    ties = TR.check_decisions(orc, info.restart_log, info.trace, s.n, agree=1e-6)
    _say(f"  decisions checked over {len(orc.s_log)} iterations, ties {ties}, largest |s_gpu - s|/sum|gd| "
         f"{TR.max_sum_difference(orc, info.trace):.2e}")
    assert info.status == orc.status == O.STATUS_OK
    assert info.iterations == orc.iterations
    xg = x.cpu().numpy()
    assert np.abs(xg - orc.x).max() <= 1e-10 * np.abs(orc.x).max()
    Q = O.csr(s.rowptr, s.colidx, s.vals)
    assert np.linalg.norm(s.b - Q @ xg) / np.linalg.norm(s.b) <= 1e-8
    xm, im = sysm.solve(s.b, tol=1e-8, precision=naj.NAJ_MIXED)
    assert im.status == 0
    xmh = xm.cpu().numpy()
    assert np.linalg.norm(s.b - Q @ xmh) / np.linalg.norm(s.b) <= 1e-8
    # the mixed answer against the float64 oracle's, modulo the null space
    pm = _component_mean_free(s.rowptr, s.colidx, s.vals, xmh)
    po = _component_mean_free(s.rowptr, s.colidx, s.vals, orc.x)
    err = float(np.linalg.norm(pm - po) / np.linalg.norm(po))
    _say(f"  iterations {info.iterations}, restarts {info.restart_log}; mixed inner {im.iterations}, "
         f"error of the mixed answer against the float64 oracle (modulo the null space) {err:.2e}")
    assert err <= 1e-5
    sysm.close()


def test_fe_batch_512_full_size(naj):
    _say("full size: 512-system finite-element batch x 8 right-hand sides")
    import torch
    systems = W.fe_batch(512, nrhs=8, workers=min(16, os.cpu_count() or 1))
    syss = [naj.System(x.rowptr, x.colidx, x.vals) for x in systems]
    reps = {}
    for x, sm in zip(systems, syss):
        reps.setdefault((sm.info()["layout"], int(np.log2(x.n)), int(round(x.nnz / x.n))), sm)
    for sm in reps.values():
        naj.autotune_tiles(sm, 8, passes=20, precision=naj.NAJ_MIXED)
    _say(f"  autotuned {len(reps)} feature keys")
    bs = [torch.as_tensor(x.b).cuda() for x in systems]
    bt = naj.Batch(syss, [8] * len(syss), tol=1e-8, max_iter=20000, precision=naj.NAJ_MIXED)
    xs, infos, ms = bt.solve(bs)
    _say(f"  batch solve {ms:.0f} ms")
    worst = 0.0
    for i, (x, xg) in enumerate(zip(systems, xs)):
        X = xg.cpu().numpy().reshape(x.n, 8)
        B = np.asarray(x.b).reshape(x.n, 8)
        R = B - O.csr(x.rowptr, x.colidx, x.vals) @ X
        rel = np.linalg.norm(R, axis=0) / np.linalg.norm(B, axis=0)
        assert all(v.status == 0 for v in infos[8 * i:8 * i + 8]), i
        worst = max(worst, float(rel.max()))
    assert worst <= 1e-8, worst
    # sampled instances, computed one by one by the oracle (the smallest regular-layout systems)
    small = sorted((x.n, i) for i, x in enumerate(systems) if syss[i].info()["layout"] == 0)[:6]
    for _, i in small:
        x = systems[i]
        X = xs[i].cpu().numpy().reshape(x.n, 8)
        for j in (0, 7):
            bj = np.ascontiguousarray(np.asarray(x.b).reshape(x.n, 8)[:, j])
            m = O.accelerated_jacobi_mixed(x.rowptr, x.colidx, x.vals, bj, tol=1e-8)
            assert infos[8 * i + j].iterations == m.inner_total, (i, j)
            assert np.array_equal(X[:, j], m.x), (i, j)
    _say(f"  worst relres {worst:.2e}; {len(small) * 2} sampled instances equal the mixed oracle")
    bt.close()
    for sm in syss:
        sm.close()


def test_laplace3d_160_in_the_mall(naj):
    """The 160^3 Laplacian (4.1 M rows; with 4-byte values its pass fits the MALL and keeps ordinary loads)
    in the configuration bench.py times: relres <= 1e-8 by an independent host product, and the blocked
    slice order's iterates equal the slice order's bit for bit."""
    import scipy.sparse as sp
    _say("160^3 float64 at full size, bench configuration")
    s = W.poisson_system((160, 160, 160), 1006)
    out = []
    for blk in ("32", "0"):
        os.environ["NAJ_BLOCK"] = blk
        try:
            sysm = naj.System(s.rowptr, s.colidx, s.vals)
        finally:
            del os.environ["NAJ_BLOCK"]
        x, info = sysm.solve(s.b, tol=1e-8, max_iter=20000, hist_cap=0)
        out.append((x.cpu().numpy(), info))
        sysm.close()
    (xb, ib), (x0, i0) = out
    assert ib.status == 0 and ib.grid == 768 and ib.iterations == i0.iterations and ib.restart_log == i0.restart_log
    assert np.array_equal(xb, x0)
    q = sp.csr_matrix((s.vals, s.colidx, s.rowptr), shape=(s.n, s.n))
    assert np.linalg.norm(s.b - q @ xb) / np.linalg.norm(s.b) <= 1e-8 * (1 + 1e-6)


def test_laplace3d_192_beyond_the_mall(naj, monkeypatch):
    """The 192^3 Laplacian (7.08 M rows, the pass beyond the 256 MiB MALL) in the configuration bench.py
    times (4-byte value reads, blocked slice order, non-temporal matrix loads, 512 x 3): relres <= 1e-8 by
    an independent host product of the caller's CSR, and the same iterates and schedule, bit for bit, as
    the solve that reads 8-byte values in slice order (its own launch shape and loads)."""
    import scipy.sparse as sp
    _say("192^3 float64 at full size, bench configuration")
    s = W.poisson_system((192, 192, 192), 1007)
    sysm = naj.System(s.rowptr, s.colidx, s.vals)
    assert sysm.info()["value_bytes"] == 4
    x, info = sysm.solve(s.b, tol=1e-8, max_iter=20000, hist_cap=0)
    x = x.cpu().numpy()
    sysm.close()
    assert info.status == 0 and info.grid == 768
    q = sp.csr_matrix((s.vals, s.colidx, s.rowptr), shape=(s.n, s.n))
    assert np.linalg.norm(s.b - q @ x) / np.linalg.norm(s.b) <= 1e-8 * (1 + 1e-6)
    _say("192^3 float64 with 8-byte values in slice order")
    monkeypatch.setenv("NAJ_VALUES32", "0")
    sysm = naj.System(s.rowptr, s.colidx, s.vals)
    monkeypatch.delenv("NAJ_VALUES32")
    assert sysm.info()["value_bytes"] == 8
    x8, i8 = sysm.solve(s.b, tol=1e-8, max_iter=20000, hist_cap=0)
    sysm.close()
    assert i8.iterations == info.iterations and i8.restart_log == info.restart_log
    assert np.array_equal(x8.cpu().numpy(), x)
