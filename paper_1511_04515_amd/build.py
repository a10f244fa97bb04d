"""Builds libexpri.so (the C-ABI library with its gfx950 kernels) in-tree.

    python -m paper_1511_04515_amd.build        # or build() from Python

Every HIP translation unit is compiled for gfx950 only, with packed FP32
instructions disabled.  The host-only symbolic analysis is plain C++.
"""
from __future__ import annotations

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
INCLUDE = os.path.join(os.path.dirname(HERE), "include")
LIB = os.path.join(HERE, "libexpri.so")
BUILD_DIR = os.path.join(os.path.dirname(HERE), "_build")

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
ARCH = "gfx950"
HIP_FLAGS = ["-O3", "-std=c++17", "-fPIC", f"--offload-arch={ARCH}",
             "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
             "-Wall", "-Wno-unused-function"]
CXX_FLAGS = ["-O2", "-std=c++17", "-fPIC", "-Wall"]

SOURCES = [("engine.hip", "hip"), ("controller.hip", "hip"), ("expri_api.cpp", "hip"), ("symbolic.cpp", "cxx"),
           ("symbolic_capi.cpp", "cxx")]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("build step failed: " + " ".join(cmd[:3]) + " ...")
    return r


def build(verbose: bool = False) -> str:
    os.makedirs(BUILD_DIR, exist_ok=True)
    objs = []
    for src, kind in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(BUILD_DIR, src + ".o")
        if kind == "hip":
            cmd = [HIPCC, *HIP_FLAGS, "-I", INCLUDE, "-I", CSRC, "-x", "hip", "-c", path, "-o", obj]
        else:
            cmd = ["g++", *CXX_FLAGS, "-I", CSRC, "-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd))
        _run(cmd)
        objs.append(obj)
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv))
