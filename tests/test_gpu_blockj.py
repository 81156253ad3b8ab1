"""GPU parity of the block-diagonal J (eq. (J-blkdiag), Section 3) against the CPU oracle.

The setup (block norms, inverse blocks) and each iteration's block application round
differently from the oracle's library solves, so iterates agree to a tolerance rather than
bit for bit: inverse blocks within 1e-12 of the oracle's, iterates within 1e-10 (float64),
and mixed-precision answers at relative residual 1e-8 by the oracle's float64 product.
"""
import ctypes

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


def _case(name):
    if name == "spd_ragged":
        return W.random_spd(1003, 0.01, 5)                    # n % 8 != 0: ragged last block
    if name == "poisson2d":
        s = W.poisson_system((17, 13), 3)
        return s.rowptr, s.colidx, s.vals
    if name == "fe2d":
        s = W.fe_p1_system(900, 2, 41, nrhs=1)
        return s.rowptr, s.colidx, s.vals
    if name == "laplacian":
        rowptr, colidx, vals, _, _ = W.random_laplacian(777, 0.01, 6)
        return rowptr, colidx, vals
    raise KeyError(name)


def _oracle_inverse_rows(rowptr, colidx, vals, nb):
    Jb = O.block_jacobi_blocks(O.csr(rowptr, colidx, vals), nb)
    inv = np.linalg.inv(Jb)
    n = len(rowptr) - 1
    return inv.reshape(-1, nb)[:n]       # row r: row r - i*nb of block i's inverse


@pytest.mark.parametrize("case", ["spd_ragged", "poisson2d", "fe2d", "laplacian"])
@pytest.mark.parametrize("nb", [1, 2, 4, 8])
def test_block_inverse_matches_oracle(naj, case, nb):
    _say("block inverse", case, nb)
    rowptr, colidx, vals = _case(case)
    sysm = naj.System(rowptr, colidx, vals, jblock=nb)
    got = sysm.block_inverse().cpu().numpy()
    ref = _oracle_inverse_rows(rowptr, colidx, vals, nb)
    scale = np.abs(ref).max()
    assert np.abs(got - ref).max() <= 1e-12 * scale
    sysm.close()


def test_block_size_one_matches_diagonal_J(naj):
    """1 x 1 blocks: the block inverse is 1/J of eq. (J-diag) to rounding."""
    rowptr, colidx, vals = _case("spd_ragged")
    sysm = naj.System(rowptr, colidx, vals, jblock=1)
    got = sysm.block_inverse().cpu().numpy()[:, 0]
    ref = 1.0 / O.jacobi_diagonal(O.csr(rowptr, colidx, vals))
    np.testing.assert_allclose(got, ref, rtol=1e-14, atol=0)


@pytest.mark.parametrize("case", ["spd_ragged", "fe2d", "laplacian"])
@pytest.mark.parametrize("beta", [0.0, 0.37])
def test_block_step_matches_oracle(naj, case, beta):
    _say("block step", case, beta)
    rowptr, colidx, vals = _case(case)
    n = len(rowptr) - 1
    rng = np.random.default_rng(7)
    p, r, b = rng.standard_normal(n), rng.standard_normal(n), rng.standard_normal(n)
    sysm = naj.System(rowptr, colidx, vals, jblock=8)
    x, (s_, gg, sabs) = sysm.step(p, r, beta, b)
    xo, so, ggo, sabso = O.fused_step(rowptr, colidx, vals, p, r, beta, b, jblock=8)
    xg = x.cpu().numpy()
    assert np.abs(xg - xo).max() <= 1e-13 * np.abs(xo).max()
    assert s_ == pytest.approx(so, rel=1e-11, abs=1e-11 * sabso)
    assert gg == pytest.approx(ggo, rel=1e-13)
    assert sabs == pytest.approx(sabso, rel=1e-11)
    sysm.close()


# The GPU applies the inverse blocks from its own Cholesky factor, the oracle an LU solve of each block,
# so the iterates agree to rounding only: the restart inner products must agree to 1e-6 of sum|g_i d_i|
# (tie_rule), and a decision that differs must be a tie.
AGREE_BLOCK = 1e-6


def _compare_block_solve(naj, rowptr, colidx, vals, b, nb, *, rtol=1e-10, **kw):
    n = len(rowptr) - 1
    orc = O.accelerated_jacobi(rowptr, colidx, vals, b, jblock=nb, **kw)
    sysm = naj.System(rowptr, colidx, vals, jblock=nb)
    x, info = sysm.solve(b, trace=True, **kw)
    if info.restart_log != orc.restarts[:64] or info.iterations != orc.iterations:
        orc = O.accelerated_jacobi(rowptr, colidx, vals, b, jblock=nb, forced_restarts=info.restart_log, **kw)
    ties = TR.check_decisions(orc, info.restart_log, info.trace, n, k0=kw.get("k0", 2), agree=AGREE_BLOCK)
    _say(f"  decisions checked over {len(orc.s_log)} iterations, ties {ties}, largest |s_gpu - s|/sum|gd| "
         f"{TR.max_sum_difference(orc, info.trace):.2e}")
    assert info.status == orc.status == O.STATUS_OK
    assert info.iterations == orc.iterations, (info.iterations, orc.iterations)
    xg = x.cpu().numpy()
    err = np.abs(xg - orc.x).max() / np.abs(orc.x).max()
    assert err <= rtol, err
    Q = O.csr(rowptr, colidx, vals)
    assert np.linalg.norm(b - Q @ xg) / np.linalg.norm(b) <= kw.get("tol", 1e-8)
    sysm.close()
    return info, orc


@pytest.mark.parametrize("case", ["spd_ragged", "poisson2d", "fe2d"])
@pytest.mark.parametrize("nb", [2, 8])
def test_block_solve_matches_oracle_small(naj, case, nb):
    """Small systems (the single-workgroup driver)."""
    _say("block solve small", case, nb)
    rowptr, colidx, vals = _case(case)
    b = np.random.default_rng(11).standard_normal(len(rowptr) - 1)
    info, orc = _compare_block_solve(naj, rowptr, colidx, vals, b, nb, tol=1e-8)
    _say(f"  iterations {info.iterations} restarts {info.restart_log}")


@pytest.mark.parametrize("nb", [4, 8])
def test_block_solve_matches_oracle_per_pass_driver(naj, nb):
    """A system above the single-workgroup limit (one launch per pass), with a singular case."""
    _say("block solve per-pass", nb)
    s = W.poisson_system((40, 40, 40), 12)
    _compare_block_solve(naj, s.rowptr, s.colidx, s.vals, s.b, nb, tol=1e-8)
    lap = W.chung_lu_laplacian(1 << 15, 16, 2.5, seed=46, b_seed=47)
    _compare_block_solve(naj, lap.rowptr, lap.colidx, lap.vals, lap.b, nb, tol=1e-8, max_iter=20000)


@pytest.mark.parametrize("case", ["poisson3d", "fe2d"])
def test_block_mixed_reaches_tolerance(naj, case):
    _say("block mixed", case)
    if case == "poisson3d":
        s = W.poisson_system((40, 40, 40), 13)
        rowptr, colidx, vals, b = s.rowptr, s.colidx, s.vals, s.b
    else:
        rowptr, colidx, vals = _case("fe2d")
        b = np.random.default_rng(3).standard_normal(len(rowptr) - 1)
    sysm = naj.System(rowptr, colidx, vals, jblock=8)
    x, info = sysm.solve(b, tol=1e-8, precision=naj.NAJ_MIXED)
    assert info.status == 0
    Q = O.csr(rowptr, colidx, vals)
    xg = x.cpu().numpy()
    assert np.linalg.norm(b - Q @ xg) / np.linalg.norm(b) <= 1e-8
    f = O.accelerated_jacobi(rowptr, colidx, vals, b, tol=1e-8, max_iter=20000, jblock=8)
    assert np.linalg.norm(xg - f.x) / np.linalg.norm(f.x) < 1e-5
    m = O.accelerated_jacobi_mixed(rowptr, colidx, vals, b, tol=1e-8, jblock=8)
    _say(f"  inner iterations gpu {info.iterations} oracle {m.inner_total}; refinements {info.confirmations} {m.outer}")
    sysm.close()


def test_block_errors(naj):
    _say("block errors")
    import torch
    lib = naj.load()
    rowptr, colidx, vals = _case("poisson2d")
    dev = [torch.as_tensor(np.asarray(a)).cuda() for a in (rowptr, colidx, vals)]
    h = ctypes.c_void_p()
    n, nnz = len(rowptr) - 1, len(colidx)
    for bad in (0, 3, 16):
        st = lib.naj_create_system_blockj(n, nnz, dev[0].data_ptr(), dev[1].data_ptr(), dev[2].data_ptr(), bad,
                                          None, ctypes.byref(h))
        assert st == naj.NAJ_EINVAL and not h.value
    # a symmetric matrix that is not PSD: its only block is itself, so Cholesky fails
    q = [np.array([0, 2, 4], dtype=np.int32), np.array([0, 1, 0, 1], dtype=np.int32),
         np.array([1.0, 2.0, 2.0, 1.0])]
    with pytest.raises(naj.NajError) as e:
        naj.System(*q, jblock=2)
    assert e.value.status == naj.NAJ_EINVAL
    sysm = naj.System(rowptr, colidx, vals, jblock=4)
    with pytest.raises(naj.NajError):
        sysm.diagonal()
    with pytest.raises(naj.NajError):
        naj.Batch([sysm], [1])
    plain = naj.System(rowptr, colidx, vals)
    with pytest.raises(naj.NajError):
        plain.block_inverse()
    sysm.close()
    plain.close()
