"""The near-tie rule for comparing the GPU's restart decisions with the oracle's.

The restart test of Algorithm 2 (Section 2.2) is the sign of s_t = <Q y^t - b, x^t - x^{t-1}>, a sum
of n products that the GPU and the oracle add in different orders.  Two correct implementations can
therefore disagree about the sign only when |s_t| lies within the rounding of that sum, a numerical
tie.  The rule is checked along the GPU's own trajectory: the oracle is replayed with the GPU's
restart schedule forced, and at every iteration t the oracle's restart test (t > K_re + K and
s_t >= 0, with K_re and K following the GPU's schedule) must give the GPU's decision, unless

    |s_t| <= 4 n eps sum_i |g_i d_i| + |s_t^GPU - s_t|

(the sum's rounding bound with headroom, plus the measured difference between the two computed
values).  The measured difference itself must stay within `agree * sum_i |g_i d_i|` at every
iteration, so a wrong GPU sum cannot widen the band: agree = 4 n eps where the iterates are
bit-identical (only the order of the sum differs), a documented larger value where they are not
(long rows summed in another order, a block J applied through its explicit inverse).
"""
import numpy as np


def k_state(schedule, t_max: int, k0: int):
    """K_re and K in force at each iteration 1..t_max when restarts fire at `schedule` (Algorithm 2:
    a restart at t sets K_re = t and doubles K)."""
    fired = set(int(t) for t in schedule)
    K_re, K = 0, int(k0)
    out = []
    for t in range(1, t_max + 1):
        out.append((K_re, K))
        if t in fired:
            K_re, K = t, 2 * K
    return out


def check_decisions(orc_forced, gpu_schedule, gpu_trace, n: int, *, k0: int = 2, restart: bool = True,
                    agree: float | None = None):
    """Check every restart decision of a GPU run against the oracle replayed on its trajectory.

    orc_forced   : oracle result of the run with forced_restarts=gpu_schedule
    gpu_schedule : iterations at which the GPU restarted
    gpu_trace    : (T, 2) array of the GPU's s_t and sum|g_i d_i| per iteration
    Returns the iterations where the two decisions differ (each one a tie under the rule).
    Raises AssertionError on a difference that is not a tie or on a sum outside `agree`."""
    eps = np.finfo(float).eps
    band = 4 * n * eps
    agree = band if agree is None else agree
    s_o = np.asarray(orc_forced.s_log, dtype=np.float64)
    a_o = np.asarray(orc_forced.sabs_log, dtype=np.float64)
    tr = np.asarray(gpu_trace, dtype=np.float64).reshape(-1, 2)
    T = min(len(s_o), len(tr))
    assert T > 0 or len(s_o) == 0, "no trace to compare"
    fired = set(int(t) for t in gpu_schedule)
    ks = k_state(gpu_schedule, len(s_o), k0)
    ties = []
    for t in range(1, len(s_o) + 1):
        s, sabs = s_o[t - 1], a_o[t - 1]
        diff = abs(tr[t - 1, 0] - s) if t <= T else 0.0
        if t <= T:
            assert diff <= agree * sabs + 1e-300, (t, tr[t - 1, 0], s, sabs, agree)
        K_re, K = ks[t - 1]
        oracle_restarts = restart and t > K_re + K and s >= 0.0
        if oracle_restarts != (t in fired):
            assert abs(s) <= band * sabs + diff, (t, s, sabs, diff, oracle_restarts)
            ties.append(t)
    return ties


def max_sum_difference(orc_forced, gpu_trace) -> float:
    """Largest |s_t^GPU - s_t| / sum_i |g_i d_i| over the iterations both record (for reporting)."""
    s_o = np.asarray(orc_forced.s_log, dtype=np.float64)
    a_o = np.asarray(orc_forced.sabs_log, dtype=np.float64)
    tr = np.asarray(gpu_trace, dtype=np.float64).reshape(-1, 2)
    T = min(len(s_o), len(tr))
    if T == 0:
        return 0.0
    return float(np.max(np.abs(tr[:T, 0] - s_o[:T]) / np.maximum(a_o[:T], 1e-300)))
