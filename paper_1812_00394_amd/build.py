"""Builds libfvlbm.so for gfx950 in-tree (paper_1812_00394_amd/_lib/).

    python -m paper_1812_00394_amd.build          # or __graft_entry__.build()

hipcc cross-compiles without a GPU.  Packed FP32 instructions are disabled for all device code.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
LIBDIR = os.path.join(HERE, "_lib")
LIB = os.path.join(LIBDIR, "libfvlbm.so")
BUILD = os.path.join(HERE, "_build")

ARCH = os.environ.get("FVLBM_ARCH", "gfx950")
HIPCC = shutil.which("hipcc") or "/opt/rocm/bin/hipcc"
COMMON = ["-O3", "-std=c++17", "-fPIC", "-Wall", "-Wno-unused-function"]
DEVICE = [f"--offload-arch={ARCH}", "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
          "-munsafe-fp-atomics"]


def _run(cmd):
    print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)


def build(verbose: bool = True) -> str:
    os.makedirs(LIBDIR, exist_ok=True)
    os.makedirs(BUILD, exist_ok=True)
    objs = []
    mesh_o = os.path.join(BUILD, "mesh.o")
    _run([HIPCC, *COMMON, "-x", "c++", "-c", os.path.join(CSRC, "mesh.cpp"), "-o", mesh_o])
    objs.append(mesh_o)
    dev_o = os.path.join(BUILD, "fvlbm.o")
    _run([HIPCC, *COMMON, *DEVICE, "-x", "hip", "-c", os.path.join(CSRC, "fvlbm.hip"), "-o", dev_o])
    objs.append(dev_o)
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs, "-lpthread"])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
