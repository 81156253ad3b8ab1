"""Systems whose stored values are all exact in float32 run their float64 passes on the float32 copy of the
values (4-byte loads, widened to float64 where used).  That computes exactly what the 8-byte values do:
every solve equals the same solve with NAJ_VALUES32=0 bit for bit (iterate, schedule, residual), with the
launch shape held equal so that the value storage is the only difference.  Systems with any value that
float32 does not hold keep 8 bytes.
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


def _make(naj, monkeypatch, s, values32, layout=None):
    monkeypatch.setenv("NAJ_VALUES32", "1" if values32 else "0")
    monkeypatch.setenv("NAJ_BS", "256")
    monkeypatch.setenv("NAJ_BS_MIXED", "256")
    if layout is not None:
        monkeypatch.setenv("NAJ_LAYOUT", str(layout))
    sysm = naj.System(s.rowptr, s.colidx, s.vals)
    for v in ("NAJ_VALUES32", "NAJ_BS", "NAJ_BS_MIXED", "NAJ_LAYOUT"):
        monkeypatch.delenv(v, raising=False)
    return sysm


def _pair_solves(naj, monkeypatch, s, layout=None, **opts):
    out = []
    for v32 in (True, False):
        sysm = _make(naj, monkeypatch, s, v32, layout)
        assert sysm.info()["value_bytes"] == (4 if v32 else 8)
        x, info = sysm.solve(s.b, **opts)
        out.append((x.cpu().numpy(), info))
        sysm.close()
    (x4, i4), (x8, i8) = out
    assert i4.status == i8.status and i4.iterations == i8.iterations and i4.restart_log == i8.restart_log
    assert i4.relres == i8.relres or (np.isnan(i4.relres) and np.isnan(i8.relres))
    assert np.array_equal(x4, x8)
    return x4, i4


CASES = {
    "poisson2d_64": lambda: W.poisson2d_64(),
    "laplace3d_40": lambda: W.poisson_system((40, 40, 40), 12),
    "chunglu_2e15": lambda: W.chung_lu_laplacian(1 << 15, 16, 2.5, seed=81, b_seed=82),
}


@pytest.mark.parametrize("case", list(CASES))
@pytest.mark.parametrize("precision", [0, 1])
def test_values32_is_bitwise(naj, monkeypatch, case, precision):
    _say("float32-stored values against 8-byte values:", case, "precision", precision)
    s = CASES[case]()
    x, info = _pair_solves(naj, monkeypatch, s, tol=1e-8, max_iter=20000, precision=precision, hist_cap=0)
    assert info.status == 0
    if case != "chunglu_2e15" and precision == 0:
        # regular layouts: the oracle's answer, bit for bit
        orc = O.accelerated_jacobi(s.rowptr, s.colidx, s.vals, s.b, tol=1e-8, max_iter=20000)
        assert info.iterations == orc.iterations and np.array_equal(x, orc.x)


def test_values32_long_rows_and_cap(naj, monkeypatch):
    """The Section 4.1 system on the sorted layout (every row long: the long-row path reads the float32
    copy), then an iteration cap (the residual of the last iterate on the confirmation path)."""
    _say("float32-stored values, SDD n=600 all rows long")
    s = W.sdd_system(600)
    _pair_solves(naj, monkeypatch, s, layout=1, tol=1e-8, max_iter=5000)
    _pair_solves(naj, monkeypatch, s, layout=1, tol=1e-12, max_iter=7)


def test_inexact_values_keep_8_bytes(naj, monkeypatch):
    _say("values that float32 does not hold")
    rowptr, colidx, vals = W.random_spd(1003, 0.01, 5)
    sysm = naj.System(rowptr, colidx, vals)
    assert sysm.info()["value_bytes"] == 8
    sysm.close()
    s = W.poisson_system((40, 40, 40), 12)
    vals = s.vals.copy()
    vals[12345] += 1e-9                     # one value with no float32 twin
    sysm = naj.System(s.rowptr, s.colidx, vals)
    assert sysm.info()["value_bytes"] == 8
    sysm.close()
    sysm = naj.System(s.rowptr, s.colidx, s.vals)
    assert sysm.info()["value_bytes"] == 4
    sysm.close()


@pytest.mark.parametrize("precision", [0, 1])
def test_values32_nontemporal_512(naj, monkeypatch, precision):
    """The 512-thread pass with 4-byte values and non-temporal matrix loads (taken by regular systems whose
    pass exceeds the MALL) against the same launch with ordinary loads: bit for bit."""
    _say("float32-stored values, 512 threads, non-temporal loads, precision", precision)
    s = W.poisson_system((40, 40, 40), 12)
    out = []
    for nt in ("1", "0"):
        for v, val in (("NAJ_NT", nt), ("NAJ_NT_MIXED", nt), ("NAJ_BS", "512"), ("NAJ_BS_MIXED", "512")):
            monkeypatch.setenv(v, val)
        sysm = naj.System(s.rowptr, s.colidx, s.vals)
        for v in ("NAJ_NT", "NAJ_NT_MIXED", "NAJ_BS", "NAJ_BS_MIXED"):
            monkeypatch.delenv(v)
        assert sysm.info()["value_bytes"] == 4
        x, info = sysm.solve(s.b, tol=1e-8, max_iter=20000, precision=precision, hist_cap=0)
        out.append((x.cpu().numpy(), info))
        sysm.close()
    (x1, i1), (x0, i0) = out
    assert i1.status == 0 and i1.iterations == i0.iterations and i1.restart_log == i0.restart_log
    assert np.array_equal(x1, x0)


def _blocked_pair(naj, monkeypatch, s, blk, **opts):
    out = []
    for b in (blk, 0):
        monkeypatch.setenv("NAJ_BLOCK", str(b))
        sysm = naj.System(s.rowptr, s.colidx, s.vals)
        monkeypatch.delenv("NAJ_BLOCK")
        x, info = sysm.solve(s.b, **opts)
        out.append((x.cpu().numpy(), info, sysm.info()["device_bytes"]))
        sysm.close()
    (xb, ib, db), (x0, i0, d0) = out
    assert db > d0, "the blocked item lists were not built"
    assert ib.status == i0.status and ib.iterations == i0.iterations and ib.restart_log == i0.restart_log
    # every row is computed as before, so the iterates agree bit for bit; the reductions add other rows'
    # partial sums per workgroup, so a reported norm may differ in its last bits
    assert np.array_equal(xb, x0)
    assert abs(ib.relres - i0.relres) <= 1e-12 * abs(i0.relres)
    return xb, ib


@pytest.mark.parametrize("shape", [(40, 40, 40), (37, 29, 48)])
def test_blocked_slice_order_is_bitwise(naj, monkeypatch, shape):
    """Float64 passes that visit the slices in column blocks through the planes (item lists on the
    regular layout) compute every row as the slice order does: the same iterates bit for bit and the same
    schedule, through the relres stop, the objective stop and an iteration cap (confirmation on the last
    iterate); a mixed solve of a system that holds such lists runs its own order and is unchanged."""
    _say("blocked slice order against slice order:", shape)
    s = W.poisson_system(shape, 13)
    x, info = _blocked_pair(naj, monkeypatch, s, 8, tol=1e-8, max_iter=20000, hist_cap=0)
    assert info.status == 0
    orc = O.accelerated_jacobi(s.rowptr, s.colidx, s.vals, s.b, tol=1e-8, max_iter=20000)
    assert info.iterations == orc.iterations and np.array_equal(x, orc.x)
    _blocked_pair(naj, monkeypatch, s, 8, tol=1e-12, max_iter=9, hist_cap=0)
    # f* = -<b, x*>/2 from the oracle's answer (any value serves: both solves take the same one)
    _blocked_pair(naj, monkeypatch, s, 5, tol=1e-10, max_iter=20000, hist_cap=0, stop=naj.NAJ_STOP_OBJECTIVE,
                  fstar=-0.5 * float(s.b @ orc.x))
    _blocked_pair(naj, monkeypatch, s, 8, tol=1e-8, max_iter=20000, hist_cap=0, precision=1)
    # a caller's starting point (seeded, not the iterate of another solve)
    x0 = np.random.default_rng(29).standard_normal(s.n)
    _blocked_pair(naj, monkeypatch, s, 8, x0=x0, tol=1e-8, max_iter=20000, hist_cap=0)


@pytest.mark.parametrize("precision", [0, 1])
def test_values32_block_j(naj, monkeypatch, precision):
    """A block-diagonal J (eq. (J-blkdiag), 8-row blocks) on 4-byte values: its inverse blocks stay float64,
    and the solve equals the 8-byte one bit for bit."""
    _say("float32-stored values with a block J, precision", precision)
    s = W.poisson_system((32, 24, 40), 17)
    out = []
    for v32 in ("1", "0"):
        monkeypatch.setenv("NAJ_VALUES32", v32)
        sysm = naj.System(s.rowptr, s.colidx, s.vals, jblock=8)
        monkeypatch.delenv("NAJ_VALUES32")
        assert sysm.info()["value_bytes"] == (4 if v32 == "1" else 8)
        x, info = sysm.solve(s.b, tol=1e-8, max_iter=20000, precision=precision, hist_cap=0)
        out.append((x.cpu().numpy(), info, sysm.block_inverse().cpu().numpy()))
        sysm.close()
    (x4, i4, j4), (x8, i8, j8) = out
    assert i4.status == 0 and i4.iterations == i8.iterations and i4.restart_log == i8.restart_log
    assert np.array_equal(j4, j8)
    assert np.array_equal(x4, x8)


def test_blocked_slice_order_other_domains(naj, monkeypatch):
    """The blocked lists for another split into L2 domains (3) and a grid of 150 workgroups: still the
    slice order's iterates bit for bit."""
    _say("blocked slice order, 3 domains, grid 150")
    s = W.poisson_system((40, 40, 40), 13)
    for v, val in (("NAJ_NXCD", "3"), ("NAJ_GRID", "150")):
        monkeypatch.setenv(v, val)
    x, info = _blocked_pair(naj, monkeypatch, s, 8, tol=1e-8, max_iter=20000, hist_cap=0)
    assert info.status == 0 and info.grid == 150
