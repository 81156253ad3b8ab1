"""Serving at the benchmark's configuration on a prefix of its request trace.

The first 300 requests of the seeded serving trace (finite-element systems and 3D Laplacians up to
n = 1M, one right-hand side, tolerance 1e-6 or 1e-8 each) go through a server with the benchmark's
budget, slot count and options, admitted as slots and memory free up.  Every answer must meet its
own tolerance by an independent float64 product, and sampled requests (regular layouts) must equal
the mixed oracle's answer bit for bit.
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


def test_serving_trace_prefix(naj):
    print("[gpu-case] serving trace, first 300 requests", flush=True)
    reqs = W.serve_trace(300, workers=8)
    srv = naj.Server(8192 << 20, 64, max_rhs=1, precision=naj.NAJ_MIXED, tol=1e-8, max_iter=20000)
    pending = list(range(len(reqs)))
    tickets, out = {}, {}
    turns = 0
    while len(out) < len(reqs):
        while pending:
            r = reqs[pending[0]]
            t = srv.admit(r["sys"].rowptr, r["sys"].colidx, r["sys"].vals, r["b"], tol=r["tol"])
            if t is None:
                break
            tickets[t] = pending.pop(0)
        for t in srv.step(1):
            x, infos = srv.result(t)
            out[tickets[t]] = (x.cpu().numpy(), infos[0])
        turns += 1
        assert turns < 2_000_000
    srv.close()
    worst = 0.0
    for i, r in enumerate(reqs):
        x, info = out[i]
        s = r["sys"]
        rel = np.linalg.norm(r["b"] - O.csr(s.rowptr, s.colidx, s.vals) @ x) / np.linalg.norm(r["b"])
        assert info.status == 0 and rel <= r["tol"], (i, rel, r["tol"])
        worst = max(worst, rel / r["tol"])
    small = sorted((r["sys"].n, i) for i, r in enumerate(reqs))[:8]
    for _, i in small:
        r = reqs[i]
        s = r["sys"]
        m = O.accelerated_jacobi_mixed(s.rowptr, s.colidx, s.vals, r["b"], tol=r["tol"])
        assert out[i][1].iterations == m.inner_total, i
        assert np.array_equal(out[i][0], m.x), i
    print(f"[gpu-case]   300 answers within their tolerances (worst relres / tol {worst:.3f}); "
          f"8 sampled requests equal the mixed oracle", flush=True)
