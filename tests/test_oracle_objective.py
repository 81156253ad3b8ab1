"""Pins for the oracle's objective-gap stop (the paper's criterion, Section 4):
|f(x^t) - f*| / (1 + |f*|) <= tol with f(x) = <x, Q x>/2 - <b, x> (eq. (eq-qp)).

Checked against the Section 4.1 worked example reduced to two scalars in 60-digit
arithmetic, and against a dense recomputation of every iterate's objective.
"""
import numpy as np
import pytest

import oracle as O
from paper_2407_03272_amd import workloads as W

pytestmark = pytest.mark.filterwarnings("ignore::RuntimeWarning")


@pytest.mark.parametrize("n", [1000, 2000])
@pytest.mark.parametrize("restart", [True, False])
def test_sdd_objective_stop_matches_scalar_reduction(n, restart):
    """Q = (n+1) I - 1 1^T, b = 1: x* = 1, f* = -n/2.  The float64 run with the paper's tolerance 1e-10
    follows the exact two-scalar recurrence (same restarts, same iterates) and stops where it does,
    unless the exact gap at the crossing lies within float64's resolution of f (terms of size n that
    cancel in the dense row sums), where the two may stop one apart."""
    s = W.sdd_system(n)
    r = O.accelerated_jacobi(s.rowptr, s.colidx, s.vals, s.b, tol=1e-10, max_iter=5000, restart=restart,
                             stop="objective", fstar=-n / 2)
    sc = O.sdd_scalar_run(n, tol=1e-10, max_iter=5000, restart=restart, stop="objective")
    assert r.status == O.STATUS_OK and sc["status"] == O.STATUS_OK
    # float64 resolution of the scaled gap: each dense row sum of n terms of size up to n carries about
    # eps n^{3/2} of rounding, f adds n such rows and the gap divides by 1 + n/2
    res_ = 4 * np.finfo(float).eps * n ** 1.5
    if r.iterations != sc["iterations"]:
        t = min(r.iterations, sc["iterations"])
        assert abs(r.iterations - sc["iterations"]) == 1
        assert abs(float(sc["hist"][t - 1]) - 1e-10) <= res_
    # the exact trajectory up to the float64 run's stop
    full = O.sdd_scalar_run(n, tol=0.0, max_iter=r.iterations, restart=restart, stop="objective")
    assert [t for t in full["restarts"] if t < r.iterations] == r.restarts
    xi = float(full["xhat"][r.iterations - 1])
    np.testing.assert_allclose(r.x, xi, rtol=1e-10, atol=0)
    # the returned x meets the criterion, computed from the closed form n (xi - 1)^2 / (2 + n)
    assert n * (xi - 1.0) ** 2 / (2.0 + n) <= 1e-10 + res_
    assert r.objgap == pytest.approx(n * (xi - 1.0) ** 2 / (2.0 + n), abs=res_)


def _dense_f(Q, b):
    return lambda v: 0.5 * v @ Q @ v - b @ v


@pytest.mark.parametrize("kind", ["spd", "laplacian"])
def test_objective_stop_is_first_monitor_crossing(kind):
    """Every iterate's objective recomputed densely: f(x^t) <= f(y^t) (x^t minimizes f + ||. - y^t||_S^2/2,
    Lemma 1), the run stops at the first t whose gap at y^t is <= tol, and the returned x^t meets the
    paper's criterion."""
    if kind == "spd":
        rowptr, colidx, vals = W.random_spd(120, 0.05, 3)
        Qs = O.csr(rowptr, colidx, vals)
        b = np.random.default_rng(2).standard_normal(120)
    else:
        rowptr, colidx, vals, u, v = W.random_laplacian(120, 0.05, 4, weighted=True)
        Qs = O.csr(rowptr, colidx, vals)
        b = W.mean_zero_per_component(120, u, v, np.random.default_rng(2).standard_normal(120))
    Q = Qs.toarray()
    xs = np.linalg.pinv(Q, rcond=1e-12, hermitian=True) @ b
    f = _dense_f(Q, b)
    fstar = f(xs)
    tol = 1e-10
    rec = []
    res = O.accelerated_jacobi(rowptr, colidx, vals, b, tol=tol, max_iter=20000, stop="objective", fstar=fstar,
                               callback=lambda t, info: rec.append((t, info["x"].copy(), info["y"].copy())))
    assert res.status == O.STATUS_OK
    scale = 1.0 + abs(fstar)
    slack = 1e-13 * (abs(fstar) + 1.0)
    for t, x, y in rec:
        assert f(x) <= f(y) + slack
    gaps_y = [abs(f(y) - fstar) / scale for _, _, y in rec]
    first = next(i for i, gy in enumerate(gaps_y) if gy <= tol * (1 + 1e-6))
    assert rec[first][0] in (res.iterations, res.iterations - 1) or abs(gaps_y[first] - tol) < 1e-3 * tol
    assert abs(f(res.x) - fstar) / scale <= tol * (1 + 1e-6)
    assert res.objgap == pytest.approx(abs(f(res.x) - fstar) / scale, rel=1e-3, abs=1e-14)


def test_objective_stop_needs_fstar():
    rowptr, colidx, vals = W.random_spd(30, 0.1, 1)
    with pytest.raises(ValueError):
        O.accelerated_jacobi(rowptr, colidx, vals, np.ones(30), stop="objective")
