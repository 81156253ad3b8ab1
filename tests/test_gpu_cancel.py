"""naj_cancel: a solve stopped from another host thread ends at a pass boundary with NAJ_ECANCELLED.

The stopped float64 solve returns the iterate it held, which is exactly what the same solve returns
when its iteration cap is the number of iterations it had run (bit for bit), with the residual of that
iterate.  Covered on the per-pass driver, the single-workgroup driver and a mixed-precision solve; a
request made while no solve runs is dropped.
"""
import threading
import time

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


def _cancelled_solve(sysm, b, delay, **opts):
    """Run sysm.solve in a thread and cancel it after `delay` seconds; returns (x, info, seconds)."""
    out = {}

    def work():
        t0 = time.perf_counter()
        out["r"] = sysm.solve(b, hist_cap=0, **opts)
        out["t"] = time.perf_counter() - t0

    th = threading.Thread(target=work)
    th.start()
    time.sleep(delay)
    sysm.cancel()
    th.join(timeout=60)
    assert not th.is_alive(), "the cancelled solve did not return"
    x, info = out["r"]
    return x, info, out["t"]


@pytest.mark.parametrize("shape", [(64, 64, 64), (24, 24)])   # the per-pass and the single-workgroup driver
def test_cancel_float64(naj, shape):
    s = W.poisson_system(shape, 21)
    sysm = naj.System(s.rowptr, s.colidx, s.vals)
    cap = 200000
    _say(f"cancel float64 {shape}")
    x, info, dt = _cancelled_solve(sysm, s.b, 0.2, tol=1e-300, max_iter=cap)
    _say(f"  status {info.status} after {info.iterations} iterations, {info.passes} passes, {dt:.2f} s")
    assert info.status == naj.NAJ_ECANCELLED
    assert 0 < info.iterations < cap
    xg = x.cpu().numpy()
    assert np.isfinite(xg).all()
    rel = np.linalg.norm(s.b - O.csr(s.rowptr, s.colidx, s.vals) @ xg) / np.linalg.norm(s.b)
    assert info.relres == pytest.approx(rel, rel=1e-8)
    # the iterate held at the cancel is the one the iteration cap returns there
    x2, info2 = sysm.solve(s.b, hist_cap=0, tol=1e-300, max_iter=info.iterations)
    assert info2.status == naj.NAJ_NOT_CONVERGED and info2.iterations == info.iterations
    assert np.array_equal(x2.cpu().numpy(), xg)
    sysm.close()


def test_cancel_mixed_and_stale_request(naj):
    s = W.poisson_system((64, 64, 64), 22)
    sysm = naj.System(s.rowptr, s.colidx, s.vals)
    _say("cancel mixed 64^3")
    x, info, dt = _cancelled_solve(sysm, s.b, 0.2, tol=1e-300, precision=naj.NAJ_MIXED, max_refine=100000)
    _say(f"  status {info.status} after {info.iterations} inner iterations, {info.confirmations} residual passes, "
         f"{dt:.2f} s")
    assert info.status == naj.NAJ_ECANCELLED
    xg = x.cpu().numpy()
    rel = np.linalg.norm(s.b - O.csr(s.rowptr, s.colidx, s.vals) @ xg) / np.linalg.norm(s.b)
    assert np.isfinite(xg).all() and rel < 1e-4
    assert info.relres == pytest.approx(rel, rel=1e-6)
    _say("a request made while no solve runs is dropped")
    sysm.cancel()
    x, info = sysm.solve(s.b, hist_cap=0, tol=1e-8)
    assert info.status == 0 and info.relres <= 1e-8
    sysm.close()
