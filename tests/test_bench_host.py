"""Host-side checks of bench.py: the byte models behind the roofline figures, and the one-GPU contract.

The yardstick (values + int32 columns of every nonzero, row pointers, four vector streams) is the figure the
roofline fraction is computed from; the layout's own bytes drop the column indices of nonzeros held in
column-offset slices.
"""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_yardstick_bytes_of_the_benchmark_workloads():
    n, nnz = 128 ** 3, 128 ** 3 + 6 * 127 * 128 ** 2          # 7-point Dirichlet Laplacian on 128^3
    assert nnz == 14_581_760
    assert bench.bytes_per_iteration(n, nnz) == 250_478_596
    assert bench.bytes_per_iteration(n, nnz, s_v=4, s_x=4) == 158_597_124
    assert bench.bytes_per_iteration(n, nnz, jb=8) == 250_478_596 + 8 * 8 * n
    n1, nnz1 = 160 ** 3, 160 ** 3 + 6 * 159 * 160 ** 2
    assert bench.bytes_per_iteration(n1, nnz1) == 489_676_804
    n0, nnz0 = 64 * 64, 5 * 64 * 64 - 4 * 64                  # 5-point Poisson on 64x64
    assert bench.bytes_per_iteration(n0, nnz0) == 390_148


def test_layout_bytes_drop_the_offset_slices_columns():
    n, nnz = 128 ** 3, 14_581_760
    assert bench.bytes_per_iteration(n, nnz, nnz_off=14_581_122) == 192_154_108
    assert bench.bytes_per_iteration(n, nnz, nnz_off=0) == bench.bytes_per_iteration(n, nnz)
    assert bench.bytes_per_residual(n, nnz) - bench.bytes_per_residual(n, nnz, 1000) == 4000
    assert bench.bytes_per_refinement_residual(n, nnz) == 12 * nnz + 4 * (n + 1) + 32 * n


def test_value_bytes_as_read():
    """With the float32 copy of exact values the float64 passes read 4 bytes per value: the yardstick's s_v
    is those 4 bytes (vectors stay 8), for the iteration and residual passes and for whole solves."""
    n, nnz = 128 ** 3, 14_581_760
    assert bench.bytes_per_iteration(n, nnz, s_v=4) == 192_151_556
    assert bench.bytes_per_iteration(n, nnz, s_v=4, nnz_off=14_581_122) == 133_827_068
    n2, nnz2 = 192 ** 3, 192 ** 3 + 6 * 191 * 192 ** 2
    assert nnz2 == 49_324_032
    assert bench.bytes_per_iteration(n2, nnz2, s_v=4) == 649_396_228
    assert bench.bytes_per_residual(n, nnz) - bench.bytes_per_residual(n, nnz, s_v=4) == 4 * nnz

    class Info:
        iterations, passes, confirmations = 731, 733, 1
    assert (bench.solve_bytes(n, nnz, Info, mixed=False, vb=4)
            == 8 * n + 731 * 192_151_556 + bench.bytes_per_residual(n, nnz, s_v=4))


def test_traffic_records_match_their_keys():
    """A committed counter record is reported only for the pass kernel sources, grid and value size it was
    taken with."""
    import json
    path = os.path.join(ROOT, "profiles", "k_pass64_laplace3d_128_traffic.json")
    rec = json.load(open(path))
    assert bench.measured_traffic("laplace3d_128", rec["grid"], rec["value_bytes"]) == (
        rec["traffic_bytes_per_pass"] if rec["kernel_source_sha256"] == bench.kernel_source_hash() else None)
    assert bench.measured_traffic("laplace3d_128", rec["grid"] + 8, rec["value_bytes"]) is None
    assert bench.measured_traffic("laplace3d_128", rec["grid"], 12 - rec["value_bytes"]) is None
    assert bench.measured_traffic("no_such_workload") is None
    # comments do not enter the key
    src = {"naj_device.h": "int a; // x\n/* y */ int b;\n", "naj_solve.h": "", "naj_partition.h": ""}
    src2 = {"naj_device.h": "int a; // changed\n/* also changed */ int b;\n", "naj_solve.h": "", "naj_partition.h": ""}
    assert bench.kernel_source_hash(src.__getitem__) == bench.kernel_source_hash(src2.__getitem__)


def test_residency_label():
    """A pass is called MALL-resident when the bytes it moves fit the 256 MiB MALL."""
    assert bench.residency({"layout_bytes_per_launch": 133_827_068}).startswith("MALL-resident")
    assert bench.residency({"layout_bytes_per_launch": 261_534_956}).startswith("MALL-resident")
    assert bench.residency({"layout_bytes_per_launch": 452_102_652}).startswith("beyond the MALL")
    assert bench.residency({"layout_bytes_per_launch": 256 << 20}).startswith("MALL-resident")
    assert bench.residency({"layout_bytes_per_launch": (256 << 20) + 1}).startswith("beyond")


def test_solve_bytes_count_every_pass():
    class Info:
        iterations, passes, confirmations = 731, 733, 3
    n, nnz = 128 ** 3, 14_581_760
    fp64 = bench.solve_bytes(n, nnz, Info, mixed=False)
    assert fp64 == 8 * n + 731 * bench.bytes_per_iteration(n, nnz) + 1 * bench.bytes_per_residual(n, nnz)
    mixed = bench.solve_bytes(n, nnz, Info, mixed=True)
    assert mixed == (8 * n + 731 * bench.bytes_per_iteration(n, nnz, s_v=4, s_x=4)
                     + 3 * bench.bytes_per_refinement_residual(n, nnz))


def test_more_than_one_gpu_exits_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120)
    assert r.returncode != 0
    assert "one GPU" in r.stderr and r.stdout.strip() == ""
