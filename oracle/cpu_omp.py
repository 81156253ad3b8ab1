"""ctypes front end of the multi-core C oracle (naj_oracle_omp.c).

TEST INFRASTRUCTURE ONLY, like the rest of this package: the test suite and the benchmark's
CPU-baseline leg use it; the product path never does.  ``liboracle_omp.so`` is compiled from
naj_oracle_omp.c by the repository's build step (gcc -O2 -fopenmp -ffp-contract=off).
"""
from __future__ import annotations

import ctypes
import os
from dataclasses import dataclass, field

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "naj_oracle_omp.c")
LIB = os.path.join(HERE, "liboracle_omp.so")
GCC_CMD = ["gcc", "-O2", "-std=c11", "-fopenmp", "-ffp-contract=off", "-fPIC", "-shared", "-o", LIB, SRC, "-lm"]

_lib = None


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(LIB):
            raise RuntimeError(f"{LIB} is missing: run the build step (__graft_entry__.build())")
        lib = ctypes.CDLL(LIB)
        P = ctypes.c_void_p
        I32, I64, D = ctypes.c_int32, ctypes.c_int64, ctypes.c_double
        lib.naj_oracle_solve.restype = ctypes.c_int
        lib.naj_oracle_solve.argtypes = [I64, P, P, P, P, P, D, I32, I32, I32, I32, I32, P, P, P, P, I32, P, I32,
                                         P, P, P, P]
        _lib = lib
    return _lib


@dataclass
class OmpResult:
    x: np.ndarray
    status: int
    iterations: int
    restarts: list = field(default_factory=list)
    hist: np.ndarray = field(default_factory=lambda: np.zeros(0))
    relres: float = float("nan")
    seconds: float = 0.0
    threads: int = 0


def solve(rowptr, colidx, vals, b, x0=None, *, tol: float = 1e-8, max_iter: int = 5000, restart: bool = True,
          k0: int = 2, confirm_gap: int = 8, threads: int = 0, hist_cap: int | None = None) -> OmpResult:
    """Algorithm 3 (float64, diagonal J of eq. (J-diag)) on ``threads`` host threads (0: OpenMP default)."""
    lib = _load()
    rp = np.ascontiguousarray(rowptr, dtype=np.int32)
    ci = np.ascontiguousarray(colidx, dtype=np.int32)
    va = np.ascontiguousarray(vals, dtype=np.float64)
    bb = np.ascontiguousarray(b, dtype=np.float64)
    n = rp.size - 1
    xx0 = None if x0 is None else np.ascontiguousarray(x0, dtype=np.float64)
    x = np.zeros(n)
    cap = max_iter if hist_cap is None else hist_cap
    hist = np.zeros(max(1, cap))
    rlog = np.zeros(64, dtype=np.int32)
    its, nres, hlen, used = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    rel, sec = ctypes.c_double(), ctypes.c_double()

    def p(a):
        return None if a is None else a.ctypes.data_as(ctypes.c_void_p)
    st = lib.naj_oracle_solve(n, p(rp), p(ci), p(va), p(bb), p(xx0), float(tol), int(max_iter), int(bool(restart)),
                              int(k0), int(confirm_gap), int(threads), p(x), ctypes.byref(its), ctypes.byref(nres),
                              p(rlog), 64, p(hist) if cap > 0 else None, cap, ctypes.byref(hlen), ctypes.byref(rel),
                              ctypes.byref(sec), ctypes.byref(used))
    if st < 0 and st != -4:
        raise RuntimeError(f"naj_oracle_solve failed with status {st}")
    return OmpResult(x=x, status=st, iterations=its.value, restarts=rlog[:min(nres.value, 64)].tolist(),
                     hist=hist[:hlen.value].copy(), relres=rel.value, seconds=sec.value, threads=used.value)
