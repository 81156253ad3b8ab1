"""GPU parity of the batched form: many systems, several right-hand sides each, one set of passes.

Each (system, right-hand side) instance runs its own Algorithm 3; it is checked against the oracle run on
that right-hand side (iterates within 1e-10, bit-identical where the rows are regular), and an instance's
result must be bit-identical whether its system is solved alone or inside a larger batch.
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


def _systems():
    """A mix: 2D/3D FE (regular layout), a Poisson grid, a ragged SPD, a power-law Laplacian (sorted layout)."""
    out = []
    out.append((W.fe_p1_system(900, 2, 11, nrhs=3), 3))
    out.append((W.fe_p1_system(2000, 3, 12, nrhs=8), 8))
    p = W.poisson_system((30, 20), 13, nrhs=2)
    out.append((p, 2))
    rowptr, colidx, vals = W.random_spd(700, 0.02, 14)
    b = np.random.default_rng(15).standard_normal((700, 1))
    out.append((W.CsrSystem(rowptr, colidx, vals, b, name="spd700"), 1))
    cl = W.chung_lu_laplacian(4096, 16, 2.5, seed=16, b_seed=17, nrhs=4)
    out.append((cl, 4))
    return out


def _col(b, j, k):
    return b[:, j] if (b.ndim == 2 and k >= 1) else b


@pytest.fixture(scope="module")
def mix(naj):
    items = _systems()
    syss = [naj.System(s.rowptr, s.colidx, s.vals) for s, _ in items]
    return items, syss


def test_batch_fp64_matches_oracle_per_instance(naj, mix):
    _say("batch fp64 vs oracle")
    items, syss = mix
    batch = naj.Batch(syss, [k for _, k in items], tol=1e-8, max_iter=20000)
    xs, infos, ms = batch.solve([s.b for s, _ in items])
    q = 0
    for (s, k), x in zip(items, xs):
        xg = x.cpu().numpy().reshape(s.n, -1)
        regular = naj.System(s.rowptr, s.colidx, s.vals).info()["layout"] == 0
        for j in range(k):
            bj = np.ascontiguousarray(_col(s.b, j, k))
            orc = O.accelerated_jacobi(s.rowptr, s.colidx, s.vals, bj, tol=1e-8, max_iter=20000)
            inf = infos[q]
            assert inf.status == 0
            if inf.iterations != orc.iterations:       # only a numerical tie may change a decision
                t = min(inf.iterations, orc.iterations)
                assert abs(orc.s_log[t - 1]) <= 4 * s.n * np.finfo(float).eps * orc.sabs_log[t - 1]
            else:
                err = np.abs(xg[:, j] - orc.x).max() / np.abs(orc.x).max()
                assert err <= 1e-10, (s.name, j, err)
                if regular:
                    assert np.array_equal(xg[:, j], orc.x), (s.name, j)
            q += 1
    _say(f"batch of {len(items)} systems / {q} instances: {ms:.2f} ms, tiles {batch.info()['ntiles']}")


def test_batch_alone_equals_in_mix(naj, mix):
    """An instance's answer and iteration count do not depend on the rest of the batch."""
    _say("alone vs mix")
    items, syss = mix
    big = naj.Batch(syss, [k for _, k in items], tol=1e-8, max_iter=20000)
    xs_mix, inf_mix, _ = big.solve([s.b for s, _ in items])
    q = 0
    for i, ((s, k), sysm) in enumerate(zip(items, syss)):
        alone = naj.Batch([sysm], [k], tol=1e-8, max_iter=20000)
        xs_a, inf_a, _ = alone.solve([s.b])
        assert np.array_equal(xs_a[0].cpu().numpy(), xs_mix[i].cpu().numpy()), s.name
        for j in range(k):
            assert inf_a[j].iterations == inf_mix[q + j].iterations
            assert inf_a[j].restarts == inf_mix[q + j].restarts
        q += k
        alone.close()
    # and in a different order, with a subset
    sub = naj.Batch([syss[3], syss[0]], [items[3][1], items[0][1]], tol=1e-8, max_iter=20000)
    xs_s, _, _ = sub.solve([items[3][0].b, items[0][0].b])
    assert np.array_equal(xs_s[0].cpu().numpy(), xs_mix[3].cpu().numpy())
    assert np.array_equal(xs_s[1].cpu().numpy(), xs_mix[0].cpu().numpy())


def test_batch_mixed_precision(naj, mix):
    _say("batch mixed")
    items, syss = mix
    batch = naj.Batch(syss, [k for _, k in items], tol=1e-8, precision=naj.NAJ_MIXED)
    xs, infos, ms = batch.solve([s.b for s, _ in items])
    q = 0
    for (s, k), x in zip(items, xs):
        xg = x.cpu().numpy().reshape(s.n, -1)
        Q = O.csr(s.rowptr, s.colidx, s.vals)
        regular = naj.System(s.rowptr, s.colidx, s.vals).info()["layout"] == 0
        for j in range(k):
            bj = np.ascontiguousarray(_col(s.b, j, k))
            rel = np.linalg.norm(bj - Q @ xg[:, j]) / np.linalg.norm(bj)
            assert infos[q].status == 0 and rel <= 1e-8, (s.name, j, rel)
            if regular:
                m = O.accelerated_jacobi_mixed(s.rowptr, s.colidx, s.vals, bj, tol=1e-8)
                assert infos[q].iterations == m.inner_total
                assert np.array_equal(xg[:, j], m.x), (s.name, j)
            q += 1
    _say(f"mixed batch: {ms:.2f} ms")


def test_batch_x0_zero_rhs_and_max_iter(naj):
    _say("batch edge cases")
    s = W.poisson_system((16, 16), 21, nrhs=3)
    b = s.b.copy()
    b[:, 1] = 0.0
    sysm = naj.System(s.rowptr, s.colidx, s.vals)
    x0 = np.random.default_rng(1).standard_normal((s.n, 3))
    bt = naj.Batch([sysm], [3], tol=1e-9, max_iter=20000)
    xs, infos, _ = bt.solve([b], x0s=[x0])
    xg = xs[0].cpu().numpy()
    for j in range(3):
        orc = O.accelerated_jacobi(s.rowptr, s.colidx, s.vals, np.ascontiguousarray(b[:, j]),
                                   x0=np.ascontiguousarray(x0[:, j]), tol=1e-9, max_iter=20000)
        assert infos[j].iterations == orc.iterations
        assert np.array_equal(xg[:, j], orc.x)
    capped = naj.Batch([sysm], [3], tol=1e-12, max_iter=25)
    xs, infos, _ = capped.solve([s.b])
    assert all(i.status == naj.NAJ_NOT_CONVERGED and i.iterations == 25 for i in infos)
    with pytest.raises(naj.NajError):
        naj.Batch([sysm], [9])


def test_autotune_records_a_tile_size(naj, tmp_path):
    _say("autotune")
    s = W.fe_p1_system(3000, 2, 31, nrhs=4)
    sysm = naj.System(s.rowptr, s.colidx, s.vals)
    best = naj.autotune_tiles(sysm, 4, passes=20)
    assert best in (1, 2, 4, 8, 16)
    path = str(tmp_path / "tiles.txt")
    naj.tune_save(path)
    text = open(path).read()
    assert text.strip().endswith(str(best))
    naj.tune_load(path)
    bt = naj.Batch([sysm], [4], tol=1e-8)
    xs, infos, _ = bt.solve([s.b])
    Q = O.csr(s.rowptr, s.colidx, s.vals)
    xg = xs[0].cpu().numpy()
    for j in range(4):
        assert np.linalg.norm(s.b[:, j] - Q @ xg[:, j]) / np.linalg.norm(s.b[:, j]) <= 1e-8
