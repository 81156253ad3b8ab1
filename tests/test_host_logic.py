"""Host logic compiled for the CPU: the slice-to-wave partition every solve kernel uses and the per-wave
item lists of the per-pass kernel."""
import os
import shutil
import subprocess

import pytest

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(os.path.dirname(HERE), "paper_2407_03272_amd", "csrc")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_partition_covers_every_slice_once(tmp_path):
    exe = tmp_path / "test_partition"
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", CSRC, os.path.join(HERE, "host", "test_partition.cpp"),
                    "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    assert out.startswith("ok")


@pytest.mark.skipif(shutil.which("g++") is None, reason="needs g++")
def test_item_lists(tmp_path):
    """The per-wave item lists of the per-pass kernel (balanced and blocked), built on the host."""
    exe = tmp_path / "test_lists"
    subprocess.run(["g++", "-std=c++17", "-O1", "-I", CSRC, os.path.join(HERE, "host", "test_lists.cpp"),
                    "-o", str(exe)], check=True)
    out = subprocess.run([str(exe)], check=True, capture_output=True, text=True).stdout
    assert out.startswith("ok"), out
