"""Host tests of the near-tie rule (tie_rule.py) that the GPU parity tests apply to restart decisions."""
from types import SimpleNamespace

import numpy as np
import pytest

import oracle as O
import tie_rule as TR
from paper_2407_03272_amd import workloads as W


def test_k_state_follows_algorithm2():
    # restarts at 5 and 12 with K_0 = 2: K_re = 0, K = 2 through t = 5; then K_re = 5, K = 4; then 12, 8
    ks = TR.k_state([5, 12], 14, 2)
    assert ks[0] == (0, 2) and ks[4] == (0, 2)
    assert ks[5] == (5, 4) and ks[11] == (5, 4)
    assert ks[12] == (12, 8) and ks[13] == (12, 8)


def _run():
    s = W.poisson_system((16, 16), 3)
    r = O.accelerated_jacobi(s.rowptr, s.colidx, s.vals, s.b, tol=1e-10, max_iter=5000)
    assert len(r.restarts) >= 2
    return s, r


def test_identical_runs_have_no_ties():
    s, r = _run()
    trace = np.stack([r.s_log, r.sabs_log], axis=1)
    assert TR.check_decisions(r, r.restarts, trace, s.n) == []
    assert TR.max_sum_difference(r, trace) == 0.0


def test_a_skipped_restart_that_is_not_a_tie_fails():
    s, r = _run()
    sched = r.restarts[1:]                  # the GPU "missed" the first restart
    f = O.accelerated_jacobi(s.rowptr, s.colidx, s.vals, s.b, tol=1e-10, max_iter=5000, forced_restarts=sched)
    trace = np.stack([f.s_log, f.sabs_log], axis=1)
    with pytest.raises(AssertionError):
        TR.check_decisions(f, sched, trace, s.n)


def test_an_extra_restart_that_is_not_a_tie_fails():
    s, r = _run()
    t_extra = r.restarts[0] + 1             # inside the prohibition window after the first restart
    sched = sorted(r.restarts + [t_extra])
    f = O.accelerated_jacobi(s.rowptr, s.colidx, s.vals, s.b, tol=1e-10, max_iter=5000, forced_restarts=sched)
    trace = np.stack([f.s_log, f.sabs_log], axis=1)
    with pytest.raises(AssertionError):
        TR.check_decisions(f, sched, trace, s.n)


def test_a_tie_is_accepted_and_reported():
    # a hand-made record: at t = 4 the oracle's s is within 4 n eps of zero and the GPU decided the other way
    n = 1000
    eps = np.finfo(float).eps
    s_log = [-1.0, -1.0, -1.0, 2 * n * eps * 1.0, -1.0, -1.0]
    sabs = [1.0] * 6
    orc = SimpleNamespace(s_log=s_log, sabs_log=sabs)
    trace = np.stack([np.array(s_log), np.array(sabs)], axis=1)
    # the oracle's own test restarts at t = 4 (s >= 0, 4 > 0 + 2); the GPU did not
    assert TR.check_decisions(orc, [], trace, n) == [4]
    # the same decision difference with |s| well outside the band is rejected
    s_log2 = list(s_log)
    s_log2[3] = 1e-3
    orc2 = SimpleNamespace(s_log=s_log2, sabs_log=sabs)
    with pytest.raises(AssertionError):
        TR.check_decisions(orc2, [], np.stack([np.array(s_log2), np.array(sabs)], axis=1), n)


def test_a_wrong_gpu_sum_cannot_widen_the_band():
    # the GPU's s differs from the oracle's by more than `agree`: rejected even without a decision difference
    n = 1000
    orc = SimpleNamespace(s_log=[-1.0, -0.5, -0.25], sabs_log=[1.0, 1.0, 1.0])
    trace = np.array([[-1.0, 1.0], [-0.5 + 1e-3, 1.0], [-0.25, 1.0]])
    with pytest.raises(AssertionError):
        TR.check_decisions(orc, [], trace, n)
    assert TR.check_decisions(orc, [], trace, n, agree=1e-2) == []
