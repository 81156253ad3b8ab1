"""Stored fixtures: the paper's Section 4.1 setup and the trajectories the oracle's
scalar reduction produced for it (written by tests/golden/make_sdd_golden.py)."""
import json
import os

import numpy as np
import pytest

import oracle as O
from paper_2407_03272_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def _runs():
    return json.load(open(os.path.join(GOLD, "sdd_trajectories.json")))["runs"]


def test_setup_fixture_matches_generator():
    """The generator's Section 4.1 system is the one the paper prints: diagonal n, off-diagonal -1, b = 1,
    and x* = 1 solves it exactly."""
    setup = json.load(open(os.path.join(GOLD, "sdd_paper_setup.json")))
    assert setup["sizes_n"] == [1000, 2000, 3000, 4000, 5000, 6000]
    s = W.sdd_system(50)
    Q = O.csr(s.rowptr, s.colidx, s.vals).toarray()
    assert np.array_equal(np.diag(Q), np.full(50, 50.0))
    assert np.array_equal(Q - np.diag(np.diag(Q)), -(np.ones((50, 50)) - np.eye(50)))
    assert np.array_equal(Q @ np.ones(50), s.b)
    J = O.jacobi_diagonal(O.csr(s.rowptr, s.colidx, s.vals))
    assert np.array_equal(J, np.full(50, 2 * 50 - 1.0))


@pytest.mark.parametrize("idx", [0, 2, 5, 8])
def test_trajectory_fixture_is_current(idx):
    r = _runs()[idx]
    f = O.sdd_scalar_run(r["n"], tol=r["tol"], max_iter=5000, restart=r["restart"])
    assert f["iterations"] == r["iterations"] and f["restarts"] == r["restarts"] and f["status"] == r["status"]


def test_vector_oracle_follows_fixture_n1000():
    for r in _runs():
        if r["n"] != 1000 or not r["restart"]:
            continue
        s = W.sdd_system(1000)
        res = O.accelerated_jacobi(s.rowptr, s.colidx, s.vals, s.b, tol=r["tol"], max_iter=5000)
        assert res.restarts == r["restarts"]
        if r["tol"] >= 1e-8:
            assert res.iterations == r["iterations"]
            assert np.abs(res.x - float(r["xi_final"])).max() <= 1e-10
        else:
            # 1e-10 sits at the float64 rounding floor of ||b - Qx|| for these dense rows
            # (about n * eps * (2n - 1) / sqrt(n) per entry), so the float64 run may need a few more
            # confirmations than the exact reduction; it can never stop earlier.
            assert res.iterations >= r["iterations"]
            assert np.abs(res.x - 1.0).max() <= 1e-9
