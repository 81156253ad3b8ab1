"""Pins for the multi-core C oracle (oracle/naj_oracle_omp.c), the CPU baseline's solver.

It must run the same float64 Algorithm 3 as the Python oracle, which the other oracle tests pin to the
paper: on the same inputs the iterates are bit-identical whenever the restart and stop decisions agree
(they differ only in how the reductions are summed), and it reproduces the Section 4.1 worked example
stored in tests/golden/sdd_trajectories.json.
"""
import json
import os

import numpy as np
import pytest

import oracle as O
from oracle import cpu_omp as C
from paper_2407_03272_amd import workloads as W

GOLD = os.path.join(os.path.dirname(__file__), "golden")


@pytest.fixture(scope="module", autouse=True)
def _built():
    if not os.path.exists(C.LIB):
        import subprocess
        subprocess.run(C.GCC_CMD, check=True)


@pytest.mark.parametrize("threads", [1, 4])
def test_poisson_64_bit_identical_to_python_oracle(threads):
    """The 64 x 64 Poisson system: same iterations, restarts, monitor history (to rounding) and answer
    bit for bit, on one and on four threads."""
    s = W.poisson2d_64()
    ref = O.accelerated_jacobi(s.rowptr, s.colidx, s.vals, s.b, tol=1e-8, max_iter=20000)
    got = C.solve(s.rowptr, s.colidx, s.vals, s.b, tol=1e-8, max_iter=20000, threads=threads)
    assert got.status == 0 and got.threads == threads
    assert got.iterations == ref.iterations and got.restarts == ref.restarts
    assert np.array_equal(got.x, ref.x)
    assert np.allclose(got.hist, ref.hist, rtol=1e-12, atol=0)
    assert got.relres <= 1e-8 and abs(got.relres - ref.relres) <= 1e-14


def test_singular_laplacian_from_random_start():
    rowptr, colidx, vals, u, v = W.random_laplacian(300, 0.02, 17, weighted=True)
    b = W.rhs_in_range(rowptr, colidx, vals, 18)
    x0 = np.random.default_rng(19).standard_normal(300)
    ref = O.accelerated_jacobi(rowptr, colidx, vals, b, x0=x0, tol=1e-9, max_iter=20000)
    got = C.solve(rowptr, colidx, vals, b, x0=x0, tol=1e-9, max_iter=20000, threads=3)
    assert got.status == ref.status == 0
    assert got.iterations == ref.iterations and got.restarts == ref.restarts
    assert np.array_equal(got.x, ref.x)


def test_restart_off_and_iteration_cap():
    """Algorithm 1 (no restart) capped before convergence: NOT_CONVERGED with the last iterate, as the
    Python oracle returns it."""
    rowptr, colidx, vals = W.random_spd(200, 0.05, 23)
    b = np.random.default_rng(24).standard_normal(200)
    ref = O.accelerated_jacobi(rowptr, colidx, vals, b, tol=1e-14, max_iter=60, restart=False)
    got = C.solve(rowptr, colidx, vals, b, tol=1e-14, max_iter=60, restart=False, threads=2)
    assert got.status == ref.status == 1 and got.iterations == 60
    assert np.array_equal(got.x, ref.x)
    assert abs(got.relres - ref.relres) <= 1e-13


def test_section41_worked_example():
    """The Section 4.1 system (n+1) I - 1 1^T, b = 1, n = 1000: the restarts and the stopping iteration of the
    stored exact two-scalar run, and x = xi_t 1."""
    runs = json.load(open(os.path.join(GOLD, "sdd_trajectories.json")))["runs"]
    r = next(q for q in runs if q["n"] == 1000 and q["restart"] and q["tol"] == 1e-8)
    s = W.sdd_system(1000)
    got = C.solve(s.rowptr, s.colidx, s.vals, s.b, tol=r["tol"], max_iter=5000, threads=4)
    assert got.status == 0 and got.iterations == r["iterations"] and got.restarts == r["restarts"]
    assert np.abs(got.x - float(r["xi_final"])).max() <= 1e-10


def test_zero_rhs_and_converged_start():
    s = W.poisson_system((9, 7), 5)
    got = C.solve(s.rowptr, s.colidx, s.vals, np.zeros(s.n), threads=2)
    assert got.status == 0 and got.iterations == 0 and not got.x.any()
    xs = s.xstar
    got = C.solve(s.rowptr, s.colidx, s.vals, s.b, x0=xs, tol=1e-8, threads=2)
    assert got.status == 0 and got.iterations == 0 and np.array_equal(got.x, xs)
