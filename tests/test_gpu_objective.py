"""GPU parity of the objective-gap stop (the paper's criterion, Section 4) against the CPU oracle.

The monitor f(y^t) and the confirmation f(x^t) are fixed-order sums on the GPU and library
sums in the oracle, so a stop decision may differ only where the gap lies within float64's
resolution of f at the tolerance; otherwise iterations, restarts and iterates agree as in the
relative-residual parity tests.
"""
import ctypes

import numpy as np
import pytest
import scipy.sparse.linalg as spla

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


def _fstar_spd(rowptr, colidx, vals, b):
    """f* = -<b, Q^{-1} b>/2 by a sparse direct solve."""
    Q = O.csr(rowptr, colidx, vals).tocsc()
    xs = spla.spsolve(Q, b)
    return -0.5 * float(b @ xs)


def _compare(naj, rowptr, colidx, vals, b, fstar, *, tol=1e-10, res_=1e-14, rtol=1e-10, **kw):
    orc = O.accelerated_jacobi(rowptr, colidx, vals, b, tol=tol, stop="objective", fstar=fstar, **kw)
    sysm = naj.System(rowptr, colidx, vals)
    x, info = sysm.solve(b, tol=tol, stop=naj.NAJ_STOP_OBJECTIVE, fstar=fstar, **kw)
    sysm.close()
    assert info.status == orc.status
    if info.iterations != orc.iterations:
        # a stop decision differing only at a float64 tie of the gap with tol
        t = min(info.iterations, orc.iterations)
        assert abs(orc.hist[t - 1] - tol) <= res_ or any(abs(r - tol) <= res_ for _, r in orc.confirms), \
            (info.iterations, orc.iterations)
        return info, orc, None
    assert info.restart_log == orc.restarts[:64]
    xg = x.cpu().numpy()
    assert np.abs(xg - orc.x).max() <= rtol * np.abs(orc.x).max()
    np.testing.assert_allclose(info.hist, orc.hist, rtol=1e-6, atol=res_)
    assert info.objgap == pytest.approx(orc.objgap, rel=1e-6, abs=res_)
    assert info.relres == pytest.approx(orc.relres, rel=1e-9)
    return info, orc, xg


def test_objective_stop_section41(naj):
    """The paper's worked example at its tolerance 1e-10: x* = 1, f* = -n/2."""
    for n in (1000, 2000):
        _say("objective stop, Section 4.1 system", n)
        s = W.sdd_system(n)
        res_ = 4 * np.finfo(float).eps * n ** 1.5
        info, orc, xg = _compare(naj, s.rowptr, s.colidx, s.vals, s.b, -n / 2, res_=res_)
        assert info.status == 0 and info.objgap <= 1e-10 + res_


@pytest.mark.parametrize("case", ["poisson2d", "spd_ragged", "poisson3d_40"])
def test_objective_stop_matches_oracle(naj, case):
    _say("objective stop", case)
    if case == "poisson2d":
        s = W.poisson2d_64()
        rowptr, colidx, vals, b = s.rowptr, s.colidx, s.vals, s.b
    elif case == "spd_ragged":
        rowptr, colidx, vals = W.random_spd(1000, 0.02, 5)
        b = np.random.default_rng(3).standard_normal(1000)
    else:
        s = W.poisson_system((40, 40, 40), 12)
        rowptr, colidx, vals, b = s.rowptr, s.colidx, s.vals, s.b
    fstar = _fstar_spd(rowptr, colidx, vals, b)
    info, orc, xg = _compare(naj, rowptr, colidx, vals, b, fstar, max_iter=20000)
    assert info.status == 0
    # the returned x meets the paper's criterion by an independent float64 evaluation
    Q = O.csr(rowptr, colidx, vals)
    xr = xg if xg is not None else orc.x
    assert abs(0.5 * xr @ (Q @ xr) - b @ xr - fstar) / (1 + abs(fstar)) <= 1e-10 * (1 + 1e-6)


def test_objective_stop_sorted_layout_singular(naj):
    """A singular Chung-Lu Laplacian (sorted layout, long rows): f* from a tight float64 solve."""
    _say("objective stop, Chung-Lu")
    s = W.chung_lu_laplacian(1 << 15, 16, 2.5, seed=46, b_seed=47)
    ref = O.accelerated_jacobi(s.rowptr, s.colidx, s.vals, s.b, tol=1e-13, max_iter=20000)
    Q = O.csr(s.rowptr, s.colidx, s.vals)
    fstar = 0.5 * ref.x @ (Q @ ref.x) - s.b @ ref.x
    info, orc, xg = _compare(naj, s.rowptr, s.colidx, s.vals, s.b, fstar, tol=1e-10, rtol=1e-9, max_iter=20000)
    assert info.status == 0


def test_objective_not_converged_reports_gap(naj):
    _say("objective stop, iteration cap")
    s = W.poisson2d_64()
    fstar = _fstar_spd(s.rowptr, s.colidx, s.vals, s.b)
    orc = O.accelerated_jacobi(s.rowptr, s.colidx, s.vals, s.b, tol=1e-12, max_iter=50, stop="objective",
                               fstar=fstar)
    sysm = naj.System(s.rowptr, s.colidx, s.vals)
    x, info = sysm.solve(s.b, tol=1e-12, max_iter=50, stop=naj.NAJ_STOP_OBJECTIVE, fstar=fstar)
    assert info.status == orc.status == O.STATUS_NOT_CONVERGED
    assert np.array_equal(x.cpu().numpy(), orc.x)
    assert info.objgap == pytest.approx(orc.objgap, rel=1e-9)
    assert info.relres == pytest.approx(orc.relres, rel=1e-12)
    sysm.close()


def test_objective_stop_errors(naj):
    _say("objective stop errors")
    s = W.poisson2d_64()
    sysm = naj.System(s.rowptr, s.colidx, s.vals)
    with pytest.raises(naj.NajError):
        sysm.solve(s.b, stop=naj.NAJ_STOP_OBJECTIVE, fstar=-1.0, precision=naj.NAJ_MIXED)
    with pytest.raises(naj.NajError):
        sysm.solve(s.b, stop=7)
    with pytest.raises(naj.NajError):
        naj.Batch([sysm], [1], stop=naj.NAJ_STOP_OBJECTIVE)
    # the default stop leaves objgap unset
    _, info = sysm.solve(s.b)
    assert np.isnan(info.objgap)
    sysm.close()
