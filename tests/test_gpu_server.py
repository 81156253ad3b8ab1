"""GPU tests of the serving loop (naj_server_*): continuous batching of independent requests.

Each request's answer must be bit-identical to the same request served alone (its work
split and summation orders depend only on its system), meet its own tolerance by the
oracle's float64 product, and, on the regular layout, equal the mixed oracle's answer.
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


def _say(*a):
    print("[gpu-case]", *a, flush=True)


def _requests():
    """(system, b with k columns, tol) for a mix of shapes, sizes and tolerances."""
    out = []
    s = W.fe_p1_system(900, 2, 41, nrhs=3)
    out.append((s, s.b, 1e-8))
    s = W.fe_p1_system(2000, 3, 42, nrhs=1)
    out.append((s, s.b, 1e-6))
    s = W.poisson_system((30, 20), 43, nrhs=2)
    out.append((s, s.b, 1e-8))
    rowptr, colidx, vals = W.random_spd(700, 0.02, 44)
    b = np.random.default_rng(45).standard_normal(700)
    out.append((W.CsrSystem(rowptr, colidx, vals, b, name="spd700"), b, 1e-7))
    s = W.chung_lu_laplacian(4096, 16, 2.5, seed=46, b_seed=47)
    out.append((s, s.b, 1e-8))
    s = W.poisson_system((12, 12, 12), 48, nrhs=1)
    out.append((s, s.b, 1e-6))
    return out


def _serve(naj, reqs, budget=256 << 20, slots=16, stagger=True):
    """Admit the requests (half at once, the rest while the first ones run) and collect answers."""
    srv = naj.Server(budget, slots, precision=naj.NAJ_MIXED)
    tickets, results = {}, {}
    order = list(range(len(reqs)))
    first = order[: len(order) // 2] if stagger else order
    rest = order[len(first):]
    for i in first:
        s, b, tol = reqs[i]
        t = srv.admit(s.rowptr, s.colidx, s.vals, b, tol=tol)
        assert t is not None
        tickets[t] = i
    steps = 0
    while len(results) < len(reqs):
        if rest and steps == 2:   # join while the others are on the device
            for i in rest:
                s, b, tol = reqs[i]
                t = srv.admit(s.rowptr, s.colidx, s.vals, b, tol=tol)
                assert t is not None
                tickets[t] = i
            rest = []
        for t in srv.step(1):
            x, infos = srv.result(t)
            results[tickets[t]] = (x.cpu().numpy(), infos)
        steps += 1
        assert steps < 200000
    srv.close()
    return results


def test_server_alone_equals_mix(naj):
    _say("server: mix vs alone")
    reqs = _requests()
    mix = _serve(naj, reqs)
    for i, (s, b, tol) in enumerate(reqs):
        alone = _serve(naj, [reqs[i]], stagger=False)[0]
        xm, im = mix[i]
        xa, ia = alone
        assert np.array_equal(xm, xa), s.name
        assert [v.iterations for v in im] == [v.iterations for v in ia]
        assert [v.confirmations for v in im] == [v.confirmations for v in ia]
        Q = O.csr(s.rowptr, s.colidx, s.vals)
        X = xm.reshape(s.n, -1)
        B = np.asarray(b).reshape(s.n, -1)
        for j in range(B.shape[1]):
            assert im[j].status == 0
            rel = np.linalg.norm(B[:, j] - Q @ X[:, j]) / np.linalg.norm(B[:, j])
            assert rel <= tol, (s.name, j, rel)
        _say(f"{s.name}: k {B.shape[1]} tol {tol:g} inner iterations {[v.iterations for v in im]}")


def test_server_matches_mixed_oracle(naj):
    """Regular layout: the served answer is the mixed oracle's, bit for bit."""
    _say("server vs mixed oracle")
    reqs = [r for r in _requests() if r[0].name.startswith(("fe", "poisson"))]
    got = _serve(naj, reqs)
    for i, (s, b, tol) in enumerate(reqs):
        X = got[i][0].reshape(s.n, -1)
        B = np.asarray(b).reshape(s.n, -1)
        for j in range(B.shape[1]):
            m = O.accelerated_jacobi_mixed(s.rowptr, s.colidx, s.vals, np.ascontiguousarray(B[:, j]), tol=tol)
            assert got[i][1][j].iterations == m.inner_total
            assert np.array_equal(X[:, j], m.x), (s.name, j)


def test_server_budget_queues_requests(naj):
    """With a budget for one request at a time, the second waits (busy) until the first is taken."""
    _say("server budget")
    s1 = W.poisson_system((40, 40, 40), 51, nrhs=1)
    s2 = W.poisson_system((40, 40, 40), 52, nrhs=1)
    srv = naj.Server(12 << 20, 4, precision=naj.NAJ_MIXED)
    t1 = srv.admit(s1.rowptr, s1.colidx, s1.vals, s1.b)
    assert t1 is not None
    assert srv.admit(s2.rowptr, s2.colidx, s2.vals, s2.b) is None      # busy: budget in use
    x1 = None
    while x1 is None:
        for t in srv.step(1):
            assert t == t1
            x1, i1 = srv.result(t)
    assert srv.info()["slots_used"] == 0 and srv.info()["bytes_used"] == 0
    t2 = srv.admit(s2.rowptr, s2.colidx, s2.vals, s2.b)
    assert t2 is not None
    x2 = None
    while x2 is None:
        for t in srv.step(1):
            x2, i2 = srv.result(t)
    for s, x, inf in ((s1, x1, i1), (s2, x2, i2)):
        Q = O.csr(s.rowptr, s.colidx, s.vals)
        xx = x.cpu().numpy()
        assert inf[0].status == 0
        assert np.linalg.norm(s.b - Q @ xx) / np.linalg.norm(s.b) <= 1e-8
    srv.close()


def test_server_errors(naj):
    _say("server errors")
    srv = naj.Server(4 << 20, 2, precision=naj.NAJ_MIXED)
    big = W.poisson_system((60, 60, 60), 61, nrhs=1)
    with pytest.raises(naj.NajError) as e:
        srv.admit(big.rowptr, big.colidx, big.vals, big.b)                 # can never fit the budget
    assert e.value.status == naj.NAJ_ENOMEM
    s = W.poisson_system((10, 10), 62, nrhs=1)
    with pytest.raises(naj.NajError):
        srv.admit(s.rowptr, s.colidx, s.vals, np.zeros((s.n, 9)))          # too many right-hand sides
    t = srv.admit(s.rowptr, s.colidx, s.vals, s.b)
    with pytest.raises(naj.NajError) as e:
        srv.result(t)                                                       # not finished: nothing run yet
    assert e.value.status == naj.NAJ_EBUSY
    done = []
    while not done:
        done = srv.step(1)
    x, inf = srv.result(done[0])
    assert inf[0].status == 0
    with pytest.raises(KeyError):
        srv.result(done[0])                                                 # taken already
    srv.close()


def test_server_failed_layout_build_returns_budget(naj):
    """A sorted-layout request whose build runs out of budget (while its temporaries are held) is
    refused as busy and gives back every byte it took; with no other request admitted the same
    request is an error (it can never fit), not a busy server."""
    _say("server: failed sorted-layout build")
    a = W.poisson_system((16, 16), 71, nrhs=1)
    c = W.chung_lu_laplacian(4096, 16, 2.5, seed=72, b_seed=73)
    probe = naj.Server(64 << 20, 4, precision=naj.NAJ_MIXED)
    ta = probe.admit(a.rowptr, a.colidx, a.vals, a.b)
    assert ta is not None
    used_a = probe.info()["bytes_used"]
    probe.close()
    # the admission estimate for c (matrix 16 B per nonzero, vectors 52 B per row in mixed precision)
    # fits the free budget, but the sorted layout's build needs its temporaries and slices on top
    need_c = 16 * c.nnz + 52 * c.n
    budget = used_a + need_c + (192 << 10)
    srv = naj.Server(budget, 4, precision=naj.NAJ_MIXED)
    ta = srv.admit(a.rowptr, a.colidx, a.vals, a.b)
    assert ta is not None
    before = srv.info()["bytes_used"]
    assert before == used_a
    assert srv.admit(c.rowptr, c.colidx, c.vals, c.b) is None             # busy: the build ran out of budget
    assert srv.info()["bytes_used"] == before                              # nothing kept from the failed build
    assert srv.info()["slots_used"] == 1
    x = None
    while x is None:
        for t in srv.step(1):
            x, inf = srv.result(t)
    assert inf[0].status == 0
    assert srv.info()["bytes_used"] == 0
    with pytest.raises(naj.NajError) as e:
        srv.admit(c.rowptr, c.colidx, c.vals, c.b)                         # alone it still cannot fit
    assert e.value.status == naj.NAJ_ENOMEM
    assert srv.info()["bytes_used"] == 0
    srv.close()
