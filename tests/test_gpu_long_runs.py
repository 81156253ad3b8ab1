"""Long rows whose columns form one run c0, c0 + 1, ... (dense rows) form their column indices instead
of loading them.  The products and their order are unchanged, so every solve equals the same solve with
the form off (NAJ_LONG_RUNS=0) bit for bit."""
import numpy as np
import pytest
import scipy.sparse as sp

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


def _mixed_runs_system():
    """The Section 4.1 matrix (n + 1) I - 1 1^T, n = 600 (every row long), with rows 100-199 storing their
    columns in decreasing order: 500 rows are runs, 100 are not (same row lengths, so the sorted layout
    keeps the row order)."""
    s = W.sdd_system(600)
    colidx, vals = s.colidx.copy(), s.vals.copy()
    for r in range(100, 200):
        a, b = s.rowptr[r], s.rowptr[r + 1]
        colidx[a:b] = colidx[a:b][::-1]
        vals[a:b] = vals[a:b][::-1]
    return s, colidx, vals


@pytest.mark.parametrize("precision", [0, 1])
def test_long_runs_are_bitwise(naj, monkeypatch, precision):
    _say("dense-run long rows against loaded columns, precision", precision)
    s, colidx, vals = _mixed_runs_system()
    out = []
    for runs in ("1", "0"):
        monkeypatch.setenv("NAJ_LONG_RUNS", runs)
        monkeypatch.setenv("NAJ_LAYOUT", "1")   # rows of 600 entries: long rows (one wavefront each)
        sysm = naj.System(s.rowptr, colidx, vals)
        monkeypatch.delenv("NAJ_LONG_RUNS")
        monkeypatch.delenv("NAJ_LAYOUT")
        inf = sysm.info()
        assert inf["layout"] == 1
        assert inf["offset_nnz"] == (500 * 600 if runs == "1" else 0)
        x, info = sysm.solve(s.b, tol=1e-8, max_iter=20000, precision=precision, hist_cap=0)
        out.append((x.cpu().numpy(), info))
        sysm.close()
    (x1, i1), (x0, i0) = out
    assert i1.status == 0 and i1.iterations == i0.iterations and i1.restart_log == i0.restart_log
    assert i1.relres == i0.relres
    assert np.array_equal(x1, x0)
    # the residual by an independent host product of the caller's CSR
    q = sp.csr_matrix((vals, colidx, s.rowptr), shape=(s.n, s.n))
    assert np.linalg.norm(s.b - q @ x1) / np.linalg.norm(s.b) <= 1e-8 * (1 + 1e-6)


def test_long_runs_capped(naj, monkeypatch):
    """An iteration cap: the confirmation reads the last iterate's residual through the run form too."""
    _say("dense-run long rows, iteration cap")
    s, colidx, vals = _mixed_runs_system()
    res = []
    for runs in ("1", "0"):
        monkeypatch.setenv("NAJ_LONG_RUNS", runs)
        monkeypatch.setenv("NAJ_LAYOUT", "1")   # rows of 600 entries: long rows (one wavefront each)
        sysm = naj.System(s.rowptr, colidx, vals)
        monkeypatch.delenv("NAJ_LONG_RUNS")
        monkeypatch.delenv("NAJ_LAYOUT")
        x, info = sysm.solve(s.b, tol=1e-12, max_iter=7, hist_cap=0)
        res.append((x.cpu().numpy(), info))
        sysm.close()
    assert res[0][1].status == naj.NAJ_NOT_CONVERGED and res[0][1].relres == res[1][1].relres
    assert np.array_equal(res[0][0], res[1][0])
