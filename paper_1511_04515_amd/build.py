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
           ("symbolic_capi.cpp", "cxx"), ("frontal.cpp", "cxx"), ("grid.hip", "hip"), ("grid_engine.cpp", "hip")]


def _run(cmd):
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0:
        sys.stderr.write(r.stdout + r.stderr)
        raise RuntimeError("build step failed: " + " ".join(cmd[:3]) + " ...")
    return r


def _stale(src: str, obj: str) -> bool:
    """True when obj is missing or older than its source or any header."""
    if not os.path.exists(obj):
        return True
    t = os.path.getmtime(obj)
    deps = [src] + [os.path.join(d, f) for d in (CSRC, INCLUDE) for f in os.listdir(d)
                    if f.endswith((".hpp", ".h"))]
    return any(os.path.getmtime(f) > t for f in deps)


def build(verbose: bool = False, incremental: bool = False) -> str:
    """Compiles every translation unit (in parallel) and links libexpri.so.
    incremental=True skips objects newer than every source and header."""
    from concurrent.futures import ThreadPoolExecutor
    os.makedirs(BUILD_DIR, exist_ok=True)
    objs, cmds = [], []
    for src, kind in SOURCES:
        path = os.path.join(CSRC, src)
        obj = os.path.join(BUILD_DIR, src + ".o")
        if kind == "hip":
            cmd = [HIPCC, *HIP_FLAGS, "-I", INCLUDE, "-I", CSRC, "-x", "hip", "-c", path, "-o", obj]
        else:
            cmd = ["g++", *CXX_FLAGS, "-I", CSRC, "-c", path, "-o", obj]
        if verbose:
            print(" ".join(cmd))
        if not incremental or _stale(path, obj):
            cmds.append(cmd)
        objs.append(obj)
    if cmds:
        with ThreadPoolExecutor(max_workers=min(len(cmds), max(1, os.cpu_count() or 1))) as ex:
            list(ex.map(_run, cmds))
    tmp = LIB + ".tmp"
    _run([HIPCC, "-shared", f"--offload-arch={ARCH}", "-o", tmp, *objs])
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    print(build(verbose="-v" in sys.argv, incremental="-i" in sys.argv))
