"""naj_solve_noalloc (scratch in the library's static device array) against naj_solve.

Both run the same kernels with the same grids and summation orders, so every output must be
bit-identical: x, iterations, restarts and the restart log, confirmations, relres, status.  Each
pair of checks runs two allocation-free solves in a row, the second on a smaller system, so the
second call finds the first one's contents in the static array.
"""
import numpy as np
import pytest

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


def _same(naj, sysm, s, **opts):
    """naj_solve and naj_solve_noalloc on the same system and options: identical outputs."""
    import torch
    out_a = torch.empty(s.n, dtype=torch.float64, device="cuda:0")
    out_b = torch.empty(s.n, dtype=torch.float64, device="cuda:0")
    xa, ia = sysm.solve(s.b, out=out_a, hist_cap=0, **opts)
    xb, ib = sysm.solve_noalloc(s.b, out=out_b, **opts)
    torch.cuda.synchronize()
    assert np.array_equal(xa.cpu().numpy(), xb.cpu().numpy()), s.name
    for f in ("status", "iterations", "restarts", "confirmations", "passes", "grid"):
        assert getattr(ia, f) == getattr(ib, f), (s.name, f, getattr(ia, f), getattr(ib, f))
    assert ia.restart_log == ib.restart_log
    assert ia.relres == ib.relres or (np.isnan(ia.relres) and np.isnan(ib.relres))
    assert len(ib.hist) == 0
    return ib


def test_noalloc_float64_large_then_small(naj):
    big = W.poisson_system((40, 40, 40), 12)
    small = W.poisson_system((24, 24), 5)    # 9 slices: the single-workgroup driver
    sb = naj.System(big.rowptr, big.colidx, big.vals)
    ss = naj.System(small.rowptr, small.colidx, small.vals)
    for rep in range(2):
        _say(f"noalloc float64 40^3 (per-pass driver), round {rep}")
        ib = _same(naj, sb, big, tol=1e-8, max_iter=20000)
        assert ib.status == 0 and ib.relres <= 1e-8
        _say(f"noalloc float64 24x24 (single workgroup), round {rep}")
        i2 = _same(naj, ss, small, tol=1e-8, max_iter=20000)
        assert i2.status == 0 and i2.relres <= 1e-8
    _say("noalloc float64 capped (not converged: residual of the last iterate from the static scratch)")
    ib = _same(naj, sb, big, tol=1e-8, max_iter=50)
    assert ib.status == naj.NAJ_NOT_CONVERGED
    sb.close()
    ss.close()


def test_noalloc_blocked_slice_order(naj):
    """A 3D grid whose planes (2288 rows) exceed a 32-slice block: its float64 passes sweep the blocked
    item lists, which the allocation-free solve reads from the system as naj_solve does."""
    blk = W.poisson_system((52, 44, 48), 16)
    small = W.poisson_system((24, 24), 5)
    sb = naj.System(blk.rowptr, blk.colidx, blk.vals)
    ss = naj.System(small.rowptr, small.colidx, small.vals)
    for rep in range(2):
        _say(f"noalloc float64 52x44x48 (blocked slice order), round {rep}")
        ib = _same(naj, sb, blk, tol=1e-8, max_iter=20000)
        assert ib.status == 0 and ib.relres <= 1e-8
        _say(f"noalloc float64 24x24 after it, round {rep}")
        _same(naj, ss, small, tol=1e-8, max_iter=20000)
    sb.close()
    ss.close()


def test_noalloc_sorted_layout_and_x0(naj):
    c = W.chung_lu_laplacian(1 << 15, 16, 2.5, seed=81, b_seed=82)
    d = W.chung_lu_laplacian(1 << 12, 16, 2.5, seed=83, b_seed=84)
    sc = naj.System(c.rowptr, c.colidx, c.vals)
    sd = naj.System(d.rowptr, d.colidx, d.vals)
    assert sc.info()["layout"] == 1
    _say("noalloc sorted layout 2^15 then 2^12")
    _same(naj, sc, c, tol=1e-8, max_iter=20000)
    _same(naj, sd, d, tol=1e-8, max_iter=20000)
    _say("noalloc with a starting point")
    import torch
    x0 = torch.as_tensor(np.random.default_rng(85).standard_normal(c.n)).cuda()
    xa, ia = sc.solve(c.b, x0=x0, hist_cap=0, tol=1e-8)
    xb, ib = sc.solve_noalloc(c.b, x0=x0, tol=1e-8)
    assert np.array_equal(xa.cpu().numpy(), xb.cpu().numpy())
    assert ia.iterations == ib.iterations and ia.restart_log == ib.restart_log
    sc.close()
    sd.close()


def test_noalloc_mixed(naj):
    big = W.poisson_system((40, 40, 40), 13)
    small = W.poisson_system((20, 20), 14)
    sb = naj.System(big.rowptr, big.colidx, big.vals)
    ss = naj.System(small.rowptr, small.colidx, small.vals)
    _say("noalloc mixed before the float32 vectors exist: refused")
    with pytest.raises(naj.NajError) as e:
        sb.solve_noalloc(big.b, precision=naj.NAJ_MIXED)
    assert e.value.status == naj.NAJ_EINVAL
    _say("noalloc mixed 40^3 then 20x20")
    ib = _same(naj, sb, big, tol=1e-8, precision=naj.NAJ_MIXED)     # naj_solve allocates them first
    assert ib.status == 0 and ib.relres <= 1e-8
    i2 = _same(naj, ss, small, tol=1e-8, precision=naj.NAJ_MIXED)
    assert i2.status == 0 and i2.relres <= 1e-8
    sb.close()
    ss.close()


def test_noalloc_errors(naj):
    s = W.poisson_system((10, 10), 15)
    sm = naj.System(s.rowptr, s.colidx, s.vals)
    with pytest.raises(naj.NajError) as e:
        sm.solve_noalloc(s.b, tol=-1.0)
    assert e.value.status == naj.NAJ_EINVAL
    sm.close()
