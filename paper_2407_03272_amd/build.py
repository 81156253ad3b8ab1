"""Build step: compiles the HIP sources into the in-tree C-ABI library libnaj.so (gfx950).

    python -m paper_2407_03272_amd.build
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libnaj.so")
SOURCES = ["naj_api.hip"]
HEADERS = ["naj_device.h", "naj_solve.h", "naj_partition.h", "naj_batch.h", "naj_server_impl.h", "naj_lists.h"]

HIPCC_FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-ffp-contract=off",                      # every float op separately rounded
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wno-unused-command-line-argument",
]


def hipcc() -> str:
    for cand in (os.environ.get("HIPCC"), "/opt/rocm/bin/hipcc", shutil.which("hipcc")):
        if cand and os.path.exists(cand):
            return cand
    raise RuntimeError("hipcc not found")


def build(verbose: bool = True, out: str | None = None, defines: tuple = ()) -> str:
    srcs = [os.path.join(CSRC, s) for s in SOURCES]
    lib = out or LIB
    tmp = lib + ".tmp"
    cmd = [hipcc(), *HIPCC_FLAGS, *[f"-D{d}" for d in defines], "-I", os.path.join(os.path.dirname(PKG), "include"),
           "-o", tmp, *srcs]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True, cwd=CSRC)
    os.replace(tmp, lib)
    return lib


if __name__ == "__main__":
    build()
    sys.exit(0)
