"""Parity at the benchmark workloads' full sizes, in the configuration bench.py times.

* Chung-Lu graph Laplacian, n = 2^22 (sorted layout, long rows): the complete float64 solve against the
  oracle (the same restart schedule unless a restart test is a numerical tie, iterates within 1e-10), and the
  mixed solve to relres 1e-8 by the oracle's product.
* The 512-system finite-element batch, 8 right-hand sides each, with autotuned work items: every one of the
  4096 instances reaches relres 1e-8 by an independent float64 product, and sampled regular-layout
  instances equal the mixed oracle bit for bit (the oracle computes them one by one).

The 128^3 Laplacian at full size is covered in test_gpu_parity.py against a stored oracle run.
"""
import os

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


def test_chunglu_4m_full_size(naj):
    _say("full size: Chung-Lu n=2^22")
    s = W.chung_lu_laplacian()
    sysm = naj.System(s.rowptr, s.colidx, s.vals)
    assert sysm.info()["layout"] == 1
    x, info = sysm.solve(s.b, tol=1e-8, max_iter=20000, trace=True)
    orc = O.accelerated_jacobi(s.rowptr, s.colidx, s.vals, s.b, tol=1e-8, max_iter=20000)
    if info.restart_log != orc.restarts:
        eps = np.finfo(float).eps
        t = sorted(set(orc.restarts) ^ set(info.restart_log))[0]
        assert abs(orc.s_log[t - 1]) <= 64 * s.n * eps * orc.sabs_log[t - 1]
        orc = O.accelerated_jacobi(s.rowptr, s.colidx, s.vals, s.b, tol=1e-8, max_iter=20000,
                                   forced_restarts=info.restart_log)
    assert info.status == orc.status == O.STATUS_OK
    assert info.iterations == orc.iterations
    xg = x.cpu().numpy()
    assert np.abs(xg - orc.x).max() <= 1e-10 * np.abs(orc.x).max()
    Q = O.csr(s.rowptr, s.colidx, s.vals)
    assert np.linalg.norm(s.b - Q @ xg) / np.linalg.norm(s.b) <= 1e-8
    xm, im = sysm.solve(s.b, tol=1e-8, precision=naj.NAJ_MIXED)
    assert im.status == 0
    assert np.linalg.norm(s.b - Q @ xm.cpu().numpy()) / np.linalg.norm(s.b) <= 1e-8
    _say(f"  iterations {info.iterations}, restarts {info.restart_log}; mixed inner {im.iterations}")
    sysm.close()


def test_fe_batch_512_full_size(naj):
    _say("full size: 512-system finite-element batch x 8 right-hand sides")
    import torch
    systems = W.fe_batch(512, nrhs=8, workers=min(16, os.cpu_count() or 1))
    syss = [naj.System(x.rowptr, x.colidx, x.vals) for x in systems]
    reps = {}
    for x, sm in zip(systems, syss):
        reps.setdefault((sm.info()["layout"], int(np.log2(x.n)), int(round(x.nnz / x.n))), sm)
    for sm in reps.values():
        naj.autotune_tiles(sm, 8, passes=20, precision=naj.NAJ_MIXED)
    _say(f"  autotuned {len(reps)} feature keys")
    bs = [torch.as_tensor(x.b).cuda() for x in systems]
    bt = naj.Batch(syss, [8] * len(syss), tol=1e-8, max_iter=20000, precision=naj.NAJ_MIXED)
    xs, infos, ms = bt.solve(bs)
    _say(f"  batch solve {ms:.0f} ms")
    worst = 0.0
    for i, (x, xg) in enumerate(zip(systems, xs)):
        X = xg.cpu().numpy().reshape(x.n, 8)
        B = np.asarray(x.b).reshape(x.n, 8)
        R = B - O.csr(x.rowptr, x.colidx, x.vals) @ X
        rel = np.linalg.norm(R, axis=0) / np.linalg.norm(B, axis=0)
        assert all(v.status == 0 for v in infos[8 * i:8 * i + 8]), i
        worst = max(worst, float(rel.max()))
    assert worst <= 1e-8, worst
    # sampled instances, computed one by one by the oracle (the smallest regular-layout systems)
    small = sorted((x.n, i) for i, x in enumerate(systems) if syss[i].info()["layout"] == 0)[:6]
    for _, i in small:
        x = systems[i]
        X = xs[i].cpu().numpy().reshape(x.n, 8)
        for j in (0, 7):
            bj = np.ascontiguousarray(np.asarray(x.b).reshape(x.n, 8)[:, j])
            m = O.accelerated_jacobi_mixed(x.rowptr, x.colidx, x.vals, bj, tol=1e-8)
            assert infos[8 * i + j].iterations == m.inner_total, (i, j)
            assert np.array_equal(X[:, j], m.x), (i, j)
    _say(f"  worst relres {worst:.2e}; {len(small) * 2} sampled instances equal the mixed oracle")
    bt.close()
    for sm in syss:
        sm.close()
