"""Writes oracle_runs.json: the CPU oracle's complete runs on the two Laplacian
workloads (2D 64x64 Poisson, 3D 128^3 Laplacian), so GPU tests at full size can
compare without re-running the slow oracle: iterations, restarts, confirmations,
the monitor history, sampled entries of x and the SHA-256 of the whole x (its
float64 values, little-endian, in row order).  Calls only oracle/ and the seeded
input generators.  Run from the repository root (takes about a minute):
    python tests/golden/make_oracle_runs.py
"""
import hashlib
import json
import os
import sys

import numpy as np

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

import oracle as O  # noqa: E402
from paper_2407_03272_amd import workloads as W  # noqa: E402

SAMPLE_SEED = 4242
NSAMPLE = 4096


def run(name, sysobj, **kw):
    r = O.accelerated_jacobi(sysobj.rowptr, sysobj.colidx, sysobj.vals, sysobj.b, **kw)
    rng = np.random.default_rng(SAMPLE_SEED)
    idx = np.sort(rng.choice(sysobj.n, size=min(NSAMPLE, sysobj.n), replace=False))
    return {"name": name, "opts": kw, "n": sysobj.n, "nnz": sysobj.nnz, "iterations": r.iterations,
            "status": r.status, "restarts": r.restarts, "confirms": r.confirms, "relres": r.relres,
            "hist": r.hist, "sample_idx": idx.tolist(), "sample_x": r.x[idx].tolist(),
            "x_sha256": hashlib.sha256(np.ascontiguousarray(r.x, dtype="<f8").tobytes()).hexdigest()}


def main():
    out = {"_source": "written by tests/golden/make_oracle_runs.py (oracle.accelerated_jacobi on "
                      "paper_2407_03272_amd.workloads inputs)", "runs": []}
    c1 = W.poisson2d_64()
    out["runs"].append(run("poisson2d_64x64", c1, tol=1e-8, max_iter=20000))
    out["runs"].append(run("poisson2d_64x64_norestart", c1, tol=1e-8, max_iter=20000, restart=False))
    c2 = W.poisson3d_128()
    out["runs"].append(run("laplace3d_128", c2, tol=1e-8, max_iter=20000))
    with open(os.path.join(HERE, "oracle_runs.json"), "w") as f:
        json.dump(out, f)


if __name__ == "__main__":
    main()
