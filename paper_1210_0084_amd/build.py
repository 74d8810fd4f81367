"""Builds libslicq.so (HIP kernels for gfx950 + FP64 host plan + C ABI) in-tree.

Run ``python -m paper_1210_0084_amd.build``; ``__graft_entry__.build()`` calls
``build()``. Compiles every time it is called.
"""
from __future__ import annotations

import os
import shutil
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "libslicq.so")
BUILD_DIR = os.path.join(HERE, "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"

# Packed FP32 instructions are disabled on purpose: the compiler would form
# them from ordinary float code.
HIP_FLAGS = [
    "-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-ffp-contract=fast", "-Wall", "-Wno-unused-result",
    f"-I{os.path.join(ROOT, 'include')}",
]
HOST_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-ffp-contract=off", "-Wall"]


def _run(cmd):
    print("+", " ".join(cmd), flush=True)
    subprocess.check_call(cmd)


def build(verbose: bool = True) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    plan_o = os.path.join(BUILD_DIR, "plan.o")
    api_o = os.path.join(BUILD_DIR, "api.o")
    _run(["g++", *HOST_FLAGS, "-c", os.path.join(CSRC, "plan.cpp"), "-o", plan_o])
    _run([HIPCC, *HIP_FLAGS, "-c", os.path.join(CSRC, "api.hip"), "-o", api_o])
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", "-fPIC", f"--offload-arch={ARCH}", api_o, plan_o, "-o", tmp])
    shutil.move(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build()
    sys.exit(0)
