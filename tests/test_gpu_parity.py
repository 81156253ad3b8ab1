"""GPU parity: the HIP path (through the C ABI) against the CPU oracle on the same seeded inputs.

Bar (float64): iterates within relative 1e-10 of the oracle's; with the same
restart schedule the elementwise arithmetic is the same sequence of IEEE
operations on both sides, so the iterates are expected to be equal bit for
bit, and the tests check that where the matrix makes it certain.  Reductions
(restart inner product, norms) sum in a different order, so a restart or stop
decision may differ only at a numerical tie; the near-tie rule replays the
oracle with the GPU's schedule in that case.
"""
import hashlib
import json
import os

import numpy as np
import pytest

import oracle as O
import tie_rule as TR
from paper_2407_03272_amd import workloads as W

pytestmark = pytest.mark.gpu

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module")
def naj():
    import torch
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    from paper_2407_03272_amd import naj as N
    N.load()
    return N


def _say(*a):
    print("[gpu-case]", *a, flush=True)


# Agreement of the GPU's restart inner products with the oracle's on paths whose iterates are not
# bit-identical (long rows of the sorted layout sum in another order): |s^GPU - s| <= AGREE_LONG * sum|g d|.
AGREE_LONG = 1e-6


def _compare_solve(naj, sysm, rowptr, colidx, vals, b, *, x0=None, D=None, rtol=1e-10, bitwise=False,
                   agree=None, **kw):
    """The GPU solve against the oracle.  Every restart decision is checked along the GPU's trajectory
    (tie_rule): the oracle replayed with the GPU's schedule must make the same decision at every
    iteration unless the restart inner product is a numerical tie, and the GPU's inner products must
    agree with the oracle's to within `agree` (default 4 n eps: the rounding of the sum alone)."""
    orc = O.accelerated_jacobi(rowptr, colidx, vals, b, x0=x0, D=D, **kw)
    x, info = sysm.solve(b, x0=x0, trace=True, **kw)
    xg = x.cpu().numpy()
    n = len(rowptr) - 1
    if info.restart_log != orc.restarts or info.iterations != orc.iterations:
        orc = O.accelerated_jacobi(rowptr, colidx, vals, b, x0=x0, D=D, forced_restarts=info.restart_log, **kw)
    ties = TR.check_decisions(orc, info.restart_log, info.trace, n, k0=kw.get("k0", 2),
                              restart=kw.get("restart", True), agree=agree)
    _say(f"  decisions checked over {len(orc.s_log)} iterations, ties {ties}, largest |s_gpu - s|/sum|gd| "
         f"{TR.max_sum_difference(orc, info.trace):.2e}")
    assert info.status == orc.status
    assert info.iterations == orc.iterations
    assert info.restart_log == orc.restarts[:64]
    scale = max(np.abs(orc.x).max(), 1e-300)
    err = np.abs(xg - orc.x).max() / scale
    assert err <= rtol, err
    if bitwise:
        assert np.array_equal(xg, orc.x)
    # monitor history: same values up to summation order
    h = np.asarray(orc.hist)
    assert len(info.hist) == len(h)
    np.testing.assert_allclose(info.hist, h, rtol=1e-9, atol=1e-13)
    return orc, info, xg


# --------------------------------------------------------------------------- single fused pass

@pytest.mark.parametrize("case", ["poisson2d", "spd_ragged", "laplacian", "sdd"])
@pytest.mark.parametrize("beta", [0.0, 0.37])
def test_step_matches_oracle(naj, case, beta):
    _say("step", case, beta)
    rng = np.random.default_rng(7)
    if case == "poisson2d":
        s = W.poisson2d_64(); rowptr, colidx, vals = s.rowptr, s.colidx, s.vals
    elif case == "spd_ragged":
        rowptr, colidx, vals = W.random_spd(1000, 0.02, 5)       # n % 64 != 0, rows of 5..40 entries
    elif case == "laplacian":
        rowptr, colidx, vals, _, _ = W.random_laplacian(777, 0.01, 6)
    else:
        s = W.sdd_system(300); rowptr, colidx, vals = s.rowptr, s.colidx, s.vals
    n = len(rowptr) - 1
    p, r, b = rng.standard_normal(n), rng.standard_normal(n), rng.standard_normal(n)
    sysm = naj.System(rowptr, colidx, vals)
    x, (s_, gg, sabs) = sysm.step(p, r, beta, b)
    xo, so, ggo, sabso = O.fused_step(rowptr, colidx, vals, p, r, beta, b)
    assert np.array_equal(x.cpu().numpy(), xo)          # identical operation sequence per row
    assert s_ == pytest.approx(so, rel=1e-12, abs=1e-12 * sabso)
    assert gg == pytest.approx(ggo, rel=1e-13)
    assert sabs == pytest.approx(sabso, rel=1e-13)
    sysm.close()


def test_diagonal_and_residual(naj):
    _say("diagonal/residual")
    rowptr, colidx, vals = W.random_spd(1000, 0.02, 9)
    sysm = naj.System(rowptr, colidx, vals)
    J = sysm.diagonal().cpu().numpy()
    assert np.array_equal(J, O.jacobi_diagonal(O.csr(rowptr, colidx, vals)))
    rng = np.random.default_rng(1)
    x, b = rng.standard_normal(1000), rng.standard_normal(1000)
    r, rr = sysm.residual(x, b, want_vector=True)
    ref = b - O.csr(rowptr, colidx, vals) @ x
    assert np.array_equal(r.cpu().numpy(), ref)
    assert rr == pytest.approx(float(ref @ ref), rel=1e-13)
    D = 1.5 * J
    sysd = naj.System(rowptr, colidx, vals, D=D)
    assert np.array_equal(sysd.diagonal().cpu().numpy(), 1.0 / (1.0 / D))


# --------------------------------------------------------------------------- whole solves

def test_solve_poisson2d_matches_oracle_bitwise(naj):
    _say("solve poisson2d 64x64")
    s = W.poisson2d_64()
    sysm = naj.System(s.rowptr, s.colidx, s.vals)
    orc, info, xg = _compare_solve(naj, sysm, s.rowptr, s.colidx, s.vals, s.b, tol=1e-8, max_iter=20000,
                                   bitwise=True)
    assert info.iterations == 449 and info.restart_log == [184, 335]
    assert info.relres <= 1e-8


@pytest.mark.parametrize("mode,lds", [("0", "1"), ("1", "1"), ("1", "0"), ("2", "1")])
def test_every_driver_matches_oracle(naj, mode, lds, monkeypatch):
    """The solve drivers (one launch per pass / one workgroup with the vectors in LDS / one workgroup on
    global memory / cooperative persistent grid) share the pass and must all reproduce the oracle's run,
    on a regular and on a ragged matrix."""
    _say("driver", mode, "lds", lds)
    monkeypatch.setenv("NAJ_MODE", mode)
    s = W.poisson2d_64()
    sysm = naj.System(s.rowptr, s.colidx, s.vals)
    rowptr, colidx, vals = W.random_spd(1000, 0.02, 5)
    sysr = naj.System(rowptr, colidx, vals)
    monkeypatch.delenv("NAJ_MODE")
    monkeypatch.setenv("NAJ_LDS", lds)      # read by each solve
    _compare_solve(naj, sysm, s.rowptr, s.colidx, s.vals, s.b, tol=1e-8, max_iter=20000, bitwise=True)
    b = np.random.default_rng(3).standard_normal(1000)
    _compare_solve(naj, sysr, rowptr, colidx, vals, b, tol=1e-9, max_iter=20000)
    x, info = sysm.solve(s.b, tol=1e-8, precision=naj.NAJ_MIXED)
    m = O.accelerated_jacobi_mixed(s.rowptr, s.colidx, s.vals, s.b, tol=1e-8)
    assert info.status == 0 and info.iterations == m.inner_total
    assert np.array_equal(x.cpu().numpy(), m.x)
    monkeypatch.delenv("NAJ_LDS")


def test_solve_without_restart_is_algorithm1(naj):
    _say("solve no restart, capped")
    s = W.poisson2d_64()
    sysm = naj.System(s.rowptr, s.colidx, s.vals)
    orc, info, xg = _compare_solve(naj, sysm, s.rowptr, s.colidx, s.vals, s.b, tol=1e-8, max_iter=300,
                                   restart=False, bitwise=True)
    assert info.status == naj.NAJ_NOT_CONVERGED and info.iterations == 300
    assert info.relres == pytest.approx(orc.relres, rel=1e-9)


@pytest.mark.parametrize("k0", [2, 5, 32])
def test_solve_ragged_spd(naj, k0):
    _say("solve ragged spd k0", k0)
    rowptr, colidx, vals = W.random_spd(1000, 0.02, 5)
    b = np.random.default_rng(k0).standard_normal(1000)
    sysm = naj.System(rowptr, colidx, vals)
    _compare_solve(naj, sysm, rowptr, colidx, vals, b, tol=1e-9, max_iter=20000, k0=k0)


def test_solve_singular_laplacian_with_x0(naj):
    _say("solve singular laplacian, x0")
    rowptr, colidx, vals, u, v = W.random_laplacian(1500, 0.004, 12)
    n = 1500
    b = W.mean_zero_per_component(n, u, v, np.random.default_rng(3).standard_normal(n))
    x0 = np.random.default_rng(4).standard_normal(n)
    sysm = naj.System(rowptr, colidx, vals)
    _compare_solve(naj, sysm, rowptr, colidx, vals, b, x0=x0, tol=1e-8, max_iter=20000)


def test_solve_user_diagonal(naj):
    _say("solve user D")
    s = W.poisson_system((20, 17, 9), 55)
    J = O.jacobi_diagonal(O.csr(s.rowptr, s.colidx, s.vals))
    D = J * 1.25
    sysm = naj.System(s.rowptr, s.colidx, s.vals, D=D)
    _compare_solve(naj, sysm, s.rowptr, s.colidx, s.vals, s.b, D=D, tol=1e-8, max_iter=20000, bitwise=True)


def test_solve_sdd_section41_follows_fixture(naj):
    _say("solve SDD n=1000 (Section 4.1)")
    runs = json.load(open(os.path.join(GOLD, "sdd_trajectories.json")))["runs"]
    ref = [r for r in runs if r["n"] == 1000 and r["tol"] == 1e-8 and r["restart"]][0]
    s = W.sdd_system(1000)
    sysm = naj.System(s.rowptr, s.colidx, s.vals)
    x, info = sysm.solve(s.b, tol=1e-8, max_iter=5000)
    assert info.iterations == ref["iterations"] and info.restart_log == ref["restarts"]
    assert np.abs(x.cpu().numpy() - float(ref["xi_final"])).max() <= 1e-10


def test_edge_cases(naj):
    _say("edge cases")
    s = W.poisson2d_64()
    sysm = naj.System(s.rowptr, s.colidx, s.vals)
    x, info = sysm.solve(np.zeros(s.n))
    assert info.status == 0 and info.iterations == 0 and not x.cpu().numpy().any()
    x, info = sysm.solve(s.b, x0=s.xstar)                   # monitor at y^1 = x^0 already below tol
    assert info.iterations == 0 and np.array_equal(x.cpu().numpy(), s.xstar)
    bad = s.b.copy(); bad[17] = np.nan
    x, info = sysm.solve(bad)
    assert info.status == naj.NAJ_EBREAKDOWN
    with pytest.raises(naj.NajError):
        sysm.solve(s.b, tol=-1.0)
    with pytest.raises(naj.NajError):
        sysm.solve(s.b, k0=1)
    # tiny systems: one row, and n = 65 (one full slice plus a ragged one)
    one = naj.System(np.array([0, 1]), np.array([0]), np.array([4.0]))
    x, info = one.solve(np.array([2.0]))
    assert info.status == 0 and x.cpu().numpy()[0] == 0.5
    rp, ci, va = W.poisson_dirichlet((13, 5))
    b = np.random.default_rng(0).standard_normal(65)
    s65 = naj.System(rp, ci, va)
    _compare_solve(naj, s65, rp, ci, va, b, tol=1e-10, max_iter=5000, bitwise=True)


@pytest.mark.parametrize("mode", ["0", "2"])
def test_edge_cases_launch_drivers(naj, mode, monkeypatch):
    """The edge cases on the one-launch-per-pass driver (whose decision after a pass is taken at the start of
    the next launch) and on the cooperative persistent driver: a zero right-hand side (decided after the
    norm pass), a converged start, NaN in b, an iteration cap of 1 and of 2."""
    _say("edge cases, driver", mode)
    monkeypatch.setenv("NAJ_MODE", mode)
    s = W.poisson2d_64()
    sysm = naj.System(s.rowptr, s.colidx, s.vals)
    monkeypatch.delenv("NAJ_MODE")
    x, info = sysm.solve(np.zeros(s.n))
    assert info.status == 0 and info.iterations == 0 and not x.cpu().numpy().any()
    x, info = sysm.solve(s.b, x0=s.xstar)
    assert info.iterations == 0 and np.array_equal(x.cpu().numpy(), s.xstar)
    bad = s.b.copy(); bad[17] = np.nan
    x, info = sysm.solve(bad)
    assert info.status == naj.NAJ_EBREAKDOWN
    for cap in (1, 2):
        x, info = sysm.solve(s.b, tol=1e-8, max_iter=cap)
        orc = O.accelerated_jacobi(s.rowptr, s.colidx, s.vals, s.b, tol=1e-8, max_iter=cap)
        assert info.status == naj.NAJ_NOT_CONVERGED and info.iterations == cap
        assert np.array_equal(x.cpu().numpy(), orc.x)
    sysm.close()


def test_zero_row_gpu_matches_oracle(naj):
    """A zero row (an isolated vertex) gets J_kk = 1.  With b_k = 0 the component stays at x^0_k and the
    run converges; with b_k != 0 the system is inconsistent (b outside range(Q), excluded by Section 1)
    and the run ends NOT_CONVERGED at the cap.  Both runs equal the oracle's bit for bit."""
    _say("zero row: consistent and inconsistent right-hand sides")
    rowptr, colidx, vals, u, v = W.random_laplacian(40, 0.1, 8)
    Q = O.csr(rowptr, colidx, vals)
    A = Q.tolil()
    for j in A.rows[0][:]:          # isolate vertex 0
        if j != 0:
            A[0, j] = 0; A[j, 0] = 0; A[j, j] -= 1
    A[0, 0] = 0
    A = A.tocsr(); A.eliminate_zeros(); A.sort_indices()
    rp, ci, va = A.indptr.astype(np.int32), A.indices.astype(np.int32), A.data
    assert rp[1] - rp[0] == 0
    b = W.rhs_in_range(rp, ci, va, 3)
    x0 = np.full(40, 0.25)
    sysm = naj.System(rp, ci, va)
    orc, info, xg = _compare_solve(naj, sysm, rp, ci, va, b, x0=x0, tol=1e-9, max_iter=20000, bitwise=True)
    assert info.status == 0 and xg[0] == 0.25
    b2 = b.copy(); b2[0] = 1.0
    orc2, info2, xg2 = _compare_solve(naj, sysm, rp, ci, va, b2, x0=x0, tol=1e-9, max_iter=500, bitwise=True)
    assert info2.status == orc2.status == naj.NAJ_NOT_CONVERGED and info2.iterations == 500
    rel = np.linalg.norm(b2 - O.csr(rp, ci, va) @ xg2) / np.linalg.norm(b2)
    assert rel >= 1.0 / np.linalg.norm(b2) * (1 - 1e-12)      # row 0 keeps its residual b_0
    assert info2.relres == pytest.approx(rel, rel=1e-10)
    sysm.close()


def test_invalid_csr_rejected(naj):
    _say("invalid csr")
    rp, ci, va = W.poisson_dirichlet((8, 8))
    ci2 = ci.copy(); ci2[10] = 64
    with pytest.raises(naj.NajError, match="column index"):
        naj.System(rp, ci2, va)
    rp2 = rp.copy(); rp2[5] = rp2[6] + 1
    with pytest.raises(naj.NajError, match="rowptr"):
        naj.System(rp2, ci, va)
    with pytest.raises(naj.NajError, match="D not finite"):
        naj.System(rp, ci, va, D=-np.ones(64))


def test_barrier_timeout_path_exits_cleanly(naj, monkeypatch):
    """Force every barrier wait to give up at once (host-set limit of 0 ticks): the kernel must exit and the
    call must report a device error, not hang."""
    _say("forced barrier timeout")
    s = W.poisson2d_64()
    monkeypatch.setenv("NAJ_SPIN_TICKS", "0")
    monkeypatch.setenv("NAJ_MODE", "2")          # the cooperative persistent driver has the grid barrier
    sysm = naj.System(s.rowptr, s.colidx, s.vals)
    monkeypatch.delenv("NAJ_SPIN_TICKS")
    monkeypatch.delenv("NAJ_MODE")
    with pytest.raises(naj.NajError, match="timed out"):
        sysm.solve(s.b)
    sysm.close()
    ok = naj.System(s.rowptr, s.colidx, s.vals)
    x, info = ok.solve(s.b)
    assert info.status == 0 and info.iterations == 449


def test_repeat_solves_are_bitwise_deterministic(naj):
    _say("determinism")
    rowptr, colidx, vals = W.random_spd(3000, 0.005, 21)
    b = np.random.default_rng(2).standard_normal(3000)
    sysm = naj.System(rowptr, colidx, vals)
    x1, i1 = sysm.solve(b, trace=True)
    x2, i2 = sysm.solve(b, trace=True)
    assert np.array_equal(x1.cpu().numpy(), x2.cpu().numpy())
    assert np.array_equal(i1.trace, i2.trace) and np.array_equal(i1.hist, i2.hist)


# --------------------------------------------------------------------------- full size (3D 128^3)

@pytest.fixture(scope="module")
def c2():
    return W.poisson3d_128()


def test_full_size_first_iterations_elementwise(naj, c2):
    """At the full 128^3 size, in the benchmark's launch configuration: the first 12 iterations (one restart
    window, two momentum steps with beta > 0) elementwise against the oracle."""
    _say("128^3 first iterations")
    sysm = naj.System(c2.rowptr, c2.colidx, c2.vals)
    x, info = sysm.solve(c2.b, tol=1e-8, max_iter=12)
    orc = O.accelerated_jacobi(c2.rowptr, c2.colidx, c2.vals, c2.b, tol=1e-8, max_iter=12)
    assert info.status == naj.NAJ_NOT_CONVERGED and info.restart_log == orc.restarts
    assert np.array_equal(x.cpu().numpy(), orc.x)
    np.testing.assert_allclose(info.hist, orc.hist, rtol=1e-12)


def test_full_size_solve_matches_stored_oracle_run(naj, c2):
    """Full 128^3 solve against the oracle's stored complete run: same iteration count and restarts, the whole
    x bit-identical (its SHA-256 against the stored one; sampled entries within 1e-10 as well), and the
    residual of the returned x recomputed by the oracle's product."""
    _say("128^3 full solve")
    ref = [r for r in json.load(open(os.path.join(GOLD, "oracle_runs.json")))["runs"] if r["name"] == "laplace3d_128"][0]
    sysm = naj.System(c2.rowptr, c2.colidx, c2.vals)
    x, info = sysm.solve(c2.b, tol=1e-8, max_iter=20000)
    xg = x.cpu().numpy()
    assert info.status == 0
    assert info.iterations == ref["iterations"] and info.restart_log == ref["restarts"]
    idx = np.asarray(ref["sample_idx"])
    sx = np.asarray(ref["sample_x"])
    assert np.abs(xg[idx] - sx).max() <= 1e-10 * np.abs(sx).max()
    # the whole vector, bit for bit: same restart schedule and the same IEEE operations per row
    assert hashlib.sha256(np.ascontiguousarray(xg, dtype="<f8").tobytes()).hexdigest() == ref["x_sha256"]
    np.testing.assert_allclose(info.hist, ref["hist"], rtol=1e-9)
    Q = O.csr(c2.rowptr, c2.colidx, c2.vals)
    rel = np.linalg.norm(c2.b - Q @ xg) / np.linalg.norm(c2.b)
    assert rel <= 1e-8 and rel == pytest.approx(info.relres, rel=1e-6)


# --------------------------------------------------------------------------- irregular rows (sorted layout)

def test_irregular_layout_chung_lu(naj):
    """Power-law Chung-Lu Laplacian (n = 2^15, mean degree 16, max degree ~700): rows renumbered by decreasing
    length, rows longer than 128 processed one wavefront per row.  Iterates within 1e-10 of the oracle (long
    rows sum in a different order, so not bit-identical); the step, residual and diagonal kernels too."""
    _say("irregular chung-lu 2^15")
    s = W.chung_lu_laplacian(1 << 15, 16, 2.5, seed=81, b_seed=82)
    sysm = naj.System(s.rowptr, s.colidx, s.vals)
    info = sysm.info()
    assert info["layout"] == 1
    assert info["stored_entries"] <= 1.05 * s.nnz
    _compare_solve(naj, sysm, s.rowptr, s.colidx, s.vals, s.b, tol=1e-8, max_iter=20000, agree=AGREE_LONG)
    rng = np.random.default_rng(5)
    p, r = rng.standard_normal(s.n), rng.standard_normal(s.n)
    x, (s_, gg, sabs) = sysm.step(p, r, 0.3, s.b)
    xo, so, ggo, sabso = O.fused_step(s.rowptr, s.colidx, s.vals, p, r, 0.3, s.b)
    np.testing.assert_allclose(x.cpu().numpy(), xo, rtol=1e-12, atol=1e-12 * np.abs(xo).max())
    assert gg == pytest.approx(ggo, rel=1e-12)
    J = sysm.diagonal().cpu().numpy()
    np.testing.assert_allclose(J, O.jacobi_diagonal(O.csr(s.rowptr, s.colidx, s.vals)), rtol=1e-14)
    res, rr = sysm.residual(p, s.b, want_vector=True)
    ref = s.b - O.csr(s.rowptr, s.colidx, s.vals) @ p
    np.testing.assert_allclose(res.cpu().numpy(), ref, rtol=1e-12, atol=1e-12 * np.abs(ref).max())


@pytest.mark.parametrize("precision,bs_mixed", [(0, None), (1, None), (1, "512")])
def test_balanced_wave_lists_are_bitwise(naj, monkeypatch, precision, bs_mixed):
    """The sorted layout's per-pass kernel takes its long rows and slices from per-wave lists balanced on the
    host (longest first to the least-loaded wave).  Every row is computed as with the strided assignment,
    so the iterates are bit-identical; only the grouping of the partial sums differs (the same schedule
    here).  Float64 and mixed precision, against the same system built without the lists; with 512-thread
    mixed launches the mixed solve uses a second list built for that launch shape."""
    _say("balanced wave lists on/off, chung-lu 2^15, precision", precision, "mixed block", bs_mixed)
    s = W.chung_lu_laplacian(1 << 15, 16, 2.5, seed=81, b_seed=82)
    out = []
    for lists in ("0", "1"):
        monkeypatch.setenv("NAJ_WAVE_LISTS", lists)
        if bs_mixed:
            monkeypatch.setenv("NAJ_BS_MIXED", bs_mixed)
        sysm = naj.System(s.rowptr, s.colidx, s.vals)
        monkeypatch.delenv("NAJ_WAVE_LISTS")
        if bs_mixed:
            monkeypatch.delenv("NAJ_BS_MIXED")
        assert sysm.info()["layout"] == 1
        x, info = sysm.solve(s.b, tol=1e-8, max_iter=20000, precision=precision)
        assert info.status == 0
        out.append((x.cpu().numpy(), info, sysm.info()))
        sysm.close()
    (x0, i0, d0), (x1, i1, d1) = out
    # the lists exist: 4 bytes per item (long rows and slices) per launch shape, plus the offsets
    tables = 2 if bs_mixed else 1
    assert d1["device_bytes"] - d0["device_bytes"] >= 4 * tables * d1["nslices"]
    assert i0.iterations == i1.iterations and i0.restart_log == i1.restart_log
    assert np.array_equal(x0, x1)


def test_sorted_layout_forced_on_regular_rows_is_bitwise(naj, monkeypatch):
    """The renumbering keeps each row's stored order, so with no long rows the result is bit-identical."""
    _say("forced sorted layout, poisson 2d")
    monkeypatch.setenv("NAJ_LAYOUT", "1")
    s = W.poisson2d_64()
    sysm = naj.System(s.rowptr, s.colidx, s.vals)
    monkeypatch.delenv("NAJ_LAYOUT")
    assert sysm.info()["layout"] == 1
    _compare_solve(naj, sysm, s.rowptr, s.colidx, s.vals, s.b, tol=1e-8, max_iter=20000, bitwise=True)
    x0 = np.random.default_rng(2).standard_normal(s.n)
    _compare_solve(naj, sysm, s.rowptr, s.colidx, s.vals, s.b, x0=x0, tol=1e-8, max_iter=20000, bitwise=True)


def test_sorted_layout_all_rows_long(naj, monkeypatch):
    """Section 4.1 system with every row long (n = 600 > 128 entries per row): all rows one wavefront each."""
    _say("forced sorted layout, SDD n=600")
    monkeypatch.setenv("NAJ_LAYOUT", "1")
    s = W.sdd_system(600)
    sysm = naj.System(s.rowptr, s.colidx, s.vals)
    monkeypatch.delenv("NAJ_LAYOUT")
    ref = O.sdd_scalar_run(600, tol=1e-8)
    x, info = sysm.solve(s.b, tol=1e-8, max_iter=5000)
    assert info.iterations == ref["iterations"] and info.restart_log == ref["restarts"]
    assert np.abs(x.cpu().numpy() - float(ref["xi"][-1])).max() <= 1e-10


def test_irregular_user_diagonal_and_mixed(naj):
    _say("irregular: user D + mixed")
    s = W.chung_lu_laplacian(1 << 14, 16, 2.5, seed=91, b_seed=92)
    J = O.jacobi_diagonal(O.csr(s.rowptr, s.colidx, s.vals))
    sysd = naj.System(s.rowptr, s.colidx, s.vals, D=1.2 * J)
    _compare_solve(naj, sysd, s.rowptr, s.colidx, s.vals, s.b, D=1.2 * J, tol=1e-8, max_iter=20000,
                   agree=AGREE_LONG)
    sysm = naj.System(s.rowptr, s.colidx, s.vals)
    x, info = sysm.solve(s.b, precision=naj.NAJ_MIXED, trace=True, hist_cap=64)
    m = O.accelerated_jacobi_mixed(s.rowptr, s.colidx, s.vals, s.b, tol=1e-8)
    assert info.status == 0 and m.status == 0
    Q = O.csr(s.rowptr, s.colidx, s.vals)
    xg = x.cpu().numpy()
    assert np.linalg.norm(s.b - Q @ xg) / np.linalg.norm(s.b) <= 1e-8
    # long rows sum in another order, so refinement steps may differ by one at most
    assert abs(info.confirmations - m.outer) <= 1


@pytest.mark.parametrize("mode", ["0", "1"])
def test_materialized_momentum_form_is_bitwise(naj, mode, monkeypatch):
    """Each pass writing y^{t+1} = x^t + beta_t (x^t - x^{t-1}) (used unless the restart test fires) gives the
    same iterates bit for bit as forming y inside the gather; float64 and mixed precision."""
    _say("materialized y, driver", mode)
    monkeypatch.setenv("NAJ_YMODE", "1")
    monkeypatch.setenv("NAJ_MODE", mode)
    s = W.poisson2d_64()
    sysm = naj.System(s.rowptr, s.colidx, s.vals)
    monkeypatch.delenv("NAJ_YMODE")
    monkeypatch.delenv("NAJ_MODE")
    _compare_solve(naj, sysm, s.rowptr, s.colidx, s.vals, s.b, tol=1e-8, max_iter=20000, bitwise=True)
    orc = O.accelerated_jacobi(s.rowptr, s.colidx, s.vals, s.b, tol=1e-8, max_iter=300, restart=False)
    x, info = sysm.solve(s.b, tol=1e-8, max_iter=300, restart=False)
    assert np.array_equal(x.cpu().numpy(), orc.x)
    m = O.accelerated_jacobi_mixed(s.rowptr, s.colidx, s.vals, s.b, tol=1e-8)
    x, info = sysm.solve(s.b, precision=naj.NAJ_MIXED)
    assert info.iterations == m.inner_total and np.array_equal(x.cpu().numpy(), m.x)


def test_nontemporal_pass_is_bitwise(naj, monkeypatch):
    """Systems whose float64 pass exceeds the 256 MB MALL load matrix entries non-temporally (a separate
    kernel instance), and so do mixed solves whose float32 inner pass exceeds it (256-thread launch shape).
    Forced at creation on a 40^3 Poisson system with the 256-thread mixed launch shape, the float64, block-J,
    mixed and block-J mixed solves equal the ordinary instances' bit for bit, the float64 solve equals the
    oracle's and the mixed solve the mixed oracle's; forced on a Chung-Lu Laplacian (sorted layout, long
    rows), the float64 and mixed solves equal the ordinary passes' bit for bit."""
    _say("non-temporal pass, poisson 40^3")
    s = W.poisson_system((40, 40, 40), 12)
    out = []
    for flag in ("1", "0"):
        monkeypatch.setenv("NAJ_NT", flag)
        monkeypatch.setenv("NAJ_NT_MIXED", flag)
        monkeypatch.setenv("NAJ_BS_MIXED", "256")     # the launch shape that has the non-temporal instances
        sysm = naj.System(s.rowptr, s.colidx, s.vals)
        sysb = naj.System(s.rowptr, s.colidx, s.vals, jblock=4)
        for v in ("NAJ_NT", "NAJ_NT_MIXED", "NAJ_BS_MIXED"):
            monkeypatch.delenv(v)
        x, info = sysm.solve(s.b, tol=1e-8, max_iter=20000)
        xb, ib = sysb.solve(s.b, tol=1e-8, max_iter=20000)
        xm, im = sysm.solve(s.b, tol=1e-8, precision=naj.NAJ_MIXED)
        xbm, ibm = sysb.solve(s.b, tol=1e-8, precision=naj.NAJ_MIXED)
        assert info.grid > 1 and info.status == 0 and ib.status == 0 and im.status == 0 and ibm.status == 0
        out.append((x.cpu().numpy(), info.iterations, info.restart_log, xb.cpu().numpy(), ib.iterations,
                    xm.cpu().numpy(), im.iterations, xbm.cpu().numpy(), ibm.iterations))
        sysm.close()
        sysb.close()
    assert np.array_equal(out[0][0], out[1][0]) and out[0][1:3] == out[1][1:3]
    assert np.array_equal(out[0][3], out[1][3]) and out[0][4] == out[1][4]
    assert np.array_equal(out[0][5], out[1][5]) and out[0][6] == out[1][6]
    assert np.array_equal(out[0][7], out[1][7]) and out[0][8] == out[1][8]
    orc = O.accelerated_jacobi(s.rowptr, s.colidx, s.vals, s.b, tol=1e-8, max_iter=20000)
    if out[0][2] == orc.restarts:
        assert out[0][1] == orc.iterations and np.array_equal(out[0][0], orc.x)
    else:
        assert np.abs(out[0][0] - orc.x).max() <= 1e-10 * np.abs(orc.x).max()
    m = O.accelerated_jacobi_mixed(s.rowptr, s.colidx, s.vals, s.b, tol=1e-8)
    assert out[0][6] == m.inner_total and np.array_equal(out[0][5], m.x)
    # the sorted layout (materialized form, long rows one wavefront each) with and without the loads
    c = W.chung_lu_laplacian(1 << 15, 16, 2.5, seed=81, b_seed=82)
    res = []
    for flag in ("1", "0"):
        monkeypatch.setenv("NAJ_NT", flag)
        monkeypatch.setenv("NAJ_NT_MIXED", flag)
        sysm = naj.System(c.rowptr, c.colidx, c.vals)
        monkeypatch.delenv("NAJ_NT")
        monkeypatch.delenv("NAJ_NT_MIXED")
        assert sysm.info()["layout"] == 1
        x, info = sysm.solve(c.b, tol=1e-8, max_iter=20000)
        xm, im = sysm.solve(c.b, tol=1e-8, precision=naj.NAJ_MIXED)
        assert info.status == 0 and info.grid > 1 and im.status == 0
        res.append((x.cpu().numpy(), info.iterations, info.restart_log, xm.cpu().numpy(), im.iterations))
        sysm.close()
    assert np.array_equal(res[0][0], res[1][0]) and res[0][1:3] == res[1][1:3]
    assert np.array_equal(res[0][3], res[1][3]) and res[0][4] == res[1][4]
