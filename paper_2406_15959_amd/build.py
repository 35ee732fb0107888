"""Build libelmddm.so in-tree for gfx950 with hipcc.

Usage: python -m paper_2406_15959_amd.build
"""
from __future__ import annotations

import os
import subprocess
import sys

PKG = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(PKG)
CSRC = os.path.join(PKG, "csrc")
LIB = os.path.join(PKG, "libelmddm.so")
TEST_LIB = os.path.join(PKG, "libelmddm_testhooks.so")
SOURCES = ["kernels.hip", "linalg.cpp", "plan.cpp", "mlp.hip", "testhooks.cpp"]
LIB_OBJS = ["kernels", "linalg", "plan", "mlp"]
TEST_OBJS = ["kernels", "linalg", "testhooks"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
# Packed FP32 ops are disabled for all device code.
FLAGS = [
    "-O3", "-std=c++17", "-fPIC", "--offload-arch=gfx950",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-Wall", "-Wno-unused-function", "-Wno-unused-command-line-argument",
    "-I" + os.path.join(ROOT, "include"),
]


def _link(objs, out, verbose):
    tmp = out + ".tmp"
    cmd = [HIPCC, "-shared", "-fPIC", "--offload-arch=gfx950"] + objs + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.run(cmd, check=True)
    os.replace(tmp, out)


def build_library(verbose: bool = False) -> str:
    """Compile every source and link libelmddm.so and the test-hooks library."""
    obj_dir = os.path.join(PKG, "_build")
    os.makedirs(obj_dir, exist_ok=True)
    objs = {}
    for src in SOURCES:
        stem = os.path.splitext(src)[0]
        obj = os.path.join(obj_dir, stem + ".o")
        cmd = [HIPCC] + FLAGS + ["-x", "hip", "-c", os.path.join(CSRC, src), "-o", obj]
        if verbose:
            print(" ".join(cmd), flush=True)
        subprocess.run(cmd, check=True)
        objs[stem] = obj
    _link([objs[k] for k in LIB_OBJS], LIB, verbose)
    _link([objs[k] for k in TEST_OBJS], TEST_LIB, verbose)
    return LIB


if __name__ == "__main__":
    build_library(verbose="-q" not in sys.argv)
    print(LIB)
