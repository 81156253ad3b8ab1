"""A process that exits with a system, a batch and a server still open ends cleanly.

Device memory must not be freed from finalizers during interpreter shutdown (the HIP runtime, and
a profiler attached to it, may already be gone then); the binding releases live handles from an
exit hook instead.  The child below leaves all three open and must exit with status 0.
"""
import os
import subprocess
import sys

import pytest

pytestmark = pytest.mark.gpu

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))

CHILD = r"""
import sys
sys.path.insert(0, {root!r})
import torch
from paper_2407_03272_amd import naj
from paper_2407_03272_amd import workloads as W
s = W.poisson_system((24, 24), 7)
sysm = naj.System(s.rowptr, s.colidx, s.vals)
x, info = sysm.solve(s.b, tol=1e-8, max_iter=5000, hist_cap=0)
assert info.status == 0, info
bt = naj.Batch([sysm], [1], tol=1e-8, max_iter=5000)
xs, infos, _ = bt.solve([torch.as_tensor(s.b)])
assert infos[0].status == 0
srv = naj.Server(64 << 20, 4, max_rhs=1, tol=1e-8, max_iter=5000)
t = srv.admit(s.rowptr, s.colidx, s.vals, s.b, tol=1e-8)
assert t is not None
torch.cuda.synchronize()
print("child: leaving a system, a batch and a server open", flush=True)
"""


def test_exit_with_open_handles():
    print("[gpu-case] child process exits with open handles", flush=True)
    r = subprocess.run([sys.executable, "-c", CHILD.format(root=ROOT)], capture_output=True, text=True, timeout=120)
    assert "leaving a system" in r.stdout, (r.stdout, r.stderr)
    assert r.returncode == 0, (r.returncode, r.stderr[-2000:])
