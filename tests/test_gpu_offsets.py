"""The column-offset form of the sliced layout against the oracle and against the ordinary form.

A slice whose 64 rows all store their entries at columns row + S[k] of one increasing offset list S
(a stencil) forms its column indices from S instead of loading them.  A row that lacks an offset holds
an explicit zero at that position.  Adding a zero product leaves every running sum unchanged, so a
system in this form must give the oracle's results bit for bit, and exactly the results of the same
system built with the form switched off (NAJ_OFFSETS=0).
"""
import numpy as np
import pytest

import oracle as O
from offset_rule import expected_offset_slices
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


def _check_count(sysm, rowptr, colidx):
    c, z = expected_offset_slices(rowptr, colidx)
    info = sysm.info()
    assert (info["offset_slices"], info["offset_nnz"]) == (c, z)


def _pair(naj, monkeypatch, rowptr, colidx, vals):
    """The system with the offset form (default) and without it."""
    on = naj.System(rowptr, colidx, vals)
    _check_count(on, rowptr, colidx)
    monkeypatch.setenv("NAJ_OFFSETS", "0")
    off = naj.System(rowptr, colidx, vals)
    monkeypatch.delenv("NAJ_OFFSETS")
    assert off.info()["offset_slices"] == 0
    assert on.info()["stored_entries"] == off.info()["stored_entries"]
    # the form costs one 64-byte record per slice, kept only when some slice takes it
    extra = 64 * on.info()["nslices"] if on.info()["offset_slices"] else 0
    assert on.info()["device_bytes"] - off.info()["device_bytes"] == extra
    return on, off


def _same_solve(on, off, b, **kw):
    x1, i1 = on.solve(b, **kw)
    x2, i2 = off.solve(b, **kw)
    assert i1.status == i2.status and i1.iterations == i2.iterations
    assert i1.restart_log == i2.restart_log
    assert np.array_equal(x1.cpu().numpy(), x2.cpu().numpy())
    assert np.array_equal(np.asarray(i1.hist), np.asarray(i2.hist))
    return x1.cpu().numpy(), i1


def test_poisson2d_offset_slices_bitwise(naj, monkeypatch):
    """64x64 Poisson: one grid line per slice.  The first and last lines would gather outside [0, n)
    through the -1 / +1 offsets their corner rows lack, so 62 of the 64 slices take the form; the
    single-workgroup drivers (vectors in LDS, and in global memory) run it."""
    _say("offset form, poisson 2d")
    s = W.poisson2d_64()
    monkeypatch.setenv("NAJ_MODE", "1")     # the single-workgroup driver (the default takes it up to 24 slices)
    on, off = _pair(naj, monkeypatch, s.rowptr, s.colidx, s.vals)
    monkeypatch.delenv("NAJ_MODE")
    assert on.info()["offset_slices"] == 62 and on.info()["nslices"] == 64
    orc = O.accelerated_jacobi(s.rowptr, s.colidx, s.vals, s.b, tol=1e-8, max_iter=20000)
    for lds in ("1", "0"):
        monkeypatch.setenv("NAJ_LDS", lds)
        x, info = _same_solve(on, off, s.b, tol=1e-8, max_iter=20000)
        assert info.iterations == orc.iterations and info.restart_log == orc.restarts
        assert np.array_equal(x, orc.x)
    monkeypatch.delenv("NAJ_LDS")
    m = O.accelerated_jacobi_mixed(s.rowptr, s.colidx, s.vals, s.b, tol=1e-8)
    x, info = _same_solve(on, off, s.b, tol=1e-8, precision=naj.NAJ_MIXED)
    assert info.iterations == m.inner_total and np.array_equal(x, m.x)


def test_poisson3d_offset_form_per_pass_driver(naj, monkeypatch):
    """40^3 Poisson on the per-pass driver: float64, objective stop and mixed solves equal those of the
    ordinary form, and the float64 solve equals the oracle; the one-step, residual and diagonal kernels
    match the oracle too."""
    _say("offset form, poisson 3d 40^3")
    s = W.poisson_system((40, 40, 40), 12)
    on, off = _pair(naj, monkeypatch, s.rowptr, s.colidx, s.vals)
    ns = on.info()["nslices"]
    assert ns - 2 * (1600 // 64 + 1) <= on.info()["offset_slices"] < ns
    x, info = _same_solve(on, off, s.b, tol=1e-8, max_iter=20000)
    assert info.grid > 1   # the per-pass driver: the one this size gets at creation
    orc = O.accelerated_jacobi(s.rowptr, s.colidx, s.vals, s.b, tol=1e-8, max_iter=20000)
    if info.restart_log == orc.restarts:
        assert info.iterations == orc.iterations and np.array_equal(x, orc.x)
    else:
        assert np.abs(x - orc.x).max() <= 1e-10 * np.abs(orc.x).max()
    x0 = np.random.default_rng(4).standard_normal(s.n)
    _same_solve(on, off, s.b, x0=x0, tol=1e-8, max_iter=20000)
    _same_solve(on, off, s.b, tol=1e-8, precision=naj.NAJ_MIXED)
    Q = O.csr(s.rowptr, s.colidx, s.vals)
    fstar = -0.5 * float(s.b @ orc.x)
    _same_solve(on, off, s.b, tol=1e-9, stop=naj.NAJ_STOP_OBJECTIVE, fstar=fstar, max_iter=20000)
    rng = np.random.default_rng(5)
    p, r = rng.standard_normal(s.n), rng.standard_normal(s.n)
    xg, (s_, gg, sabs) = on.step(p, r, 0.3, s.b)
    xo, so, ggo, sabso = O.fused_step(s.rowptr, s.colidx, s.vals, p, r, 0.3, s.b)
    assert np.array_equal(xg.cpu().numpy(), xo)
    assert gg == pytest.approx(ggo, rel=1e-12) and s_ == pytest.approx(so, rel=1e-10, abs=1e-12 * sabso)
    res, rr = on.residual(p, s.b, want_vector=True)
    assert np.array_equal(res.cpu().numpy(), s.b - Q @ p)
    assert np.array_equal(on.diagonal().cpu().numpy(), O.jacobi_diagonal(Q))
    for h in (on, off):
        h.close()


def test_unsorted_row_keeps_its_slice_ordinary(naj, monkeypatch):
    """A row whose stored columns do not increase cannot take positions of S in stored order: its slice
    stays ordinary, every other qualifying slice takes the form, and the solve equals the ordinary
    form's bit for bit and the oracle's within 1e-10 (the oracle's sparse product may visit the reversed
    row in another order)."""
    _say("offset form, one unsorted row")
    s = W.poisson2d_64()
    rowptr, colidx, vals = s.rowptr.copy(), s.colidx.copy(), s.vals.copy()
    r = 1000
    a, e = rowptr[r], rowptr[r + 1]
    colidx[a:e] = colidx[a:e][::-1].copy()
    vals[a:e] = vals[a:e][::-1].copy()
    on, off = _pair(naj, monkeypatch, rowptr, colidx, vals)
    assert on.info()["offset_slices"] == 61
    orc = O.accelerated_jacobi(rowptr, colidx, vals, s.b, tol=1e-8, max_iter=20000)
    x, info = _same_solve(on, off, s.b, tol=1e-8, max_iter=20000)
    assert info.iterations == orc.iterations and info.restart_log == orc.restarts
    assert np.abs(x - orc.x).max() <= 1e-10 * np.abs(orc.x).max()


def test_no_pattern_no_offset_slices(naj, monkeypatch):
    """Random sparsity has no common offsets; the sorted layout never uses the form; finite-element
    systems on jittered grids get the slices the host rule predicts."""
    _say("offset form absent / FE")
    rowptr, colidx, vals = W.random_spd(1000, 0.02, 5)
    sm = naj.System(rowptr, colidx, vals)
    assert sm.info()["offset_slices"] == 0
    # the records were dropped and no longer count as the system's device memory
    monkeypatch.setenv("NAJ_OFFSETS", "0")
    assert naj.System(rowptr, colidx, vals).info()["device_bytes"] == sm.info()["device_bytes"]
    monkeypatch.delenv("NAJ_OFFSETS")
    for x in W.fe_batch(6, nrhs=1, workers=1):
        sm = naj.System(x.rowptr, x.colidx, x.vals)
        _check_count(sm, x.rowptr, x.colidx)
        assert sm.info()["offset_slices"] > 0
        sm.close()
    c = W.chung_lu_laplacian(1 << 13, 16, 2.5, seed=46, b_seed=47)
    i = naj.System(c.rowptr, c.colidx, c.vals).info()
    assert i["layout"] == 1 and i["offset_slices"] == 0


def test_batch_on_offset_systems_is_unchanged(naj, monkeypatch):
    """Batches load every column index; systems built with the form give the same answers bit for bit."""
    _say("offset form, batch")
    import torch
    systems = [W.poisson_system((20, 20, 20), 31, nrhs=4), W.poisson_system((48, 48), 32, nrhs=4)]
    res = []
    for flag in ("1", "0"):
        monkeypatch.setenv("NAJ_OFFSETS", flag)
        syss = [naj.System(x.rowptr, x.colidx, x.vals) for x in systems]
        monkeypatch.delenv("NAJ_OFFSETS")
        assert (syss[0].info()["offset_slices"] > 0) == (flag == "1")
        bs = [torch.as_tensor(x.b).cuda() for x in systems]
        for prec in (naj.NAJ_FP64, naj.NAJ_MIXED):
            bt = naj.Batch(syss, [4, 4], tol=1e-8, max_iter=20000, precision=prec)
            xs, infos, _ = bt.solve(bs)
            res.append(([x.cpu().numpy() for x in xs], [(i.status, i.iterations) for i in infos]))
            bt.close()
    for a, b in ((res[0], res[2]), (res[1], res[3])):
        assert a[1] == b[1]
        assert all(np.array_equal(u, v) for u, v in zip(a[0], b[0]))
