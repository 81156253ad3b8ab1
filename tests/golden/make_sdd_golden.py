"""Writes sdd_trajectories.json: Algorithm 3 on the Section 4.1 system, reduced to
two scalars and run in 60-digit decimals by the oracle (oracle.sdd_scalar_run).

Inputs are the paper's own parameters (sdd_paper_setup.json); the stopping rule
is the relative residual with the monitor/confirm reading of the oracle, with
x^0 = 0 and K_0 = 2.  Run from the repository root:
    python tests/golden/make_sdd_golden.py
"""
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, os.path.dirname(os.path.dirname(HERE)))

from oracle import sdd_scalar_run  # noqa: E402


def main():
    setup = json.load(open(os.path.join(HERE, "sdd_paper_setup.json")))
    out = {"_source": "written by tests/golden/make_sdd_golden.py from oracle.sdd_scalar_run; "
                      "system and sizes from arXiv 2407.03272 Section 4.1",
           "k0": 2, "confirm_gap": 8, "x0": 0, "maxiter": setup["maxiter"], "runs": []}
    for n in setup["sizes_n"]:
        for tol in (1e-8, 1e-10):
            for restart in (True, False):
                r = sdd_scalar_run(n, tol=tol, max_iter=setup["maxiter"], restart=restart, k0=2, confirm_gap=8)
                out["runs"].append({"n": n, "tol": tol, "restart": restart, "iterations": r["iterations"],
                                    "status": r["status"], "restarts": r["restarts"],
                                    "xi_final": str(r["xi"][-1])})
    with open(os.path.join(HERE, "sdd_trajectories.json"), "w") as f:
        json.dump(out, f, indent=1)


if __name__ == "__main__":
    main()
