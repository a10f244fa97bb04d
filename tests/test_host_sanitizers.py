"""The host-side symbolic and multifrontal analyses under AddressSanitizer and
UndefinedBehaviorSanitizer (CPU only): tests/host_check.cpp and the analysis
sources are built with g++ -fsanitize=address,undefined, and the check runs
on an RC mesh, an inverter chain (with its solve schedules) and a small
power grid (multifrontal analysis).  Any out-of-bounds access, leak or
undefined behaviour aborts the check."""
import os
import shutil
import subprocess

import numpy as np
import pytest

import netgen

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
CSRC = os.path.join(ROOT, "paper_1511_04515_amd", "csrc")


def _write(net, path):
    with open(path, "wb") as f:
        def i32(*v):
            f.write(np.asarray(v, np.int32).tobytes())

        def csr(m):
            m = m.tocsr()
            m.sort_indices()
            i32(m.shape[0], m.shape[1], m.nnz)
            f.write(np.asarray(m.indptr, np.int32).tobytes())
            f.write(np.asarray(m.indices, np.int32).tobytes())
            f.write(np.asarray(m.data, np.float64).tobytes())

        d = net.mosfets
        i32(net.n, len(net.sources), int(d.shape[0]))
        csr(net.G)
        csr(net.C)
        csr(net.B)
        f.write(np.asarray(d["type"], np.int8).tobytes())
        for k in ("d", "g", "s"):
            f.write(np.asarray(d[k], np.int32).tobytes())
        for k in ("kp", "wl", "vth", "lam"):
            f.write(np.asarray(d[k], np.float64).tobytes())
        for s in net.sources:
            i32(len(s.t))
            f.write(np.asarray(s.t, np.float64).tobytes())
            f.write(np.asarray(s.v, np.float64).tobytes())
        f.write(np.asarray([net.vdd, net.T], np.float64).tobytes())


@pytest.fixture(scope="module")
def checker(tmp_path_factory):
    if shutil.which("g++") is None:
        pytest.skip("g++ is not available")
    out = str(tmp_path_factory.mktemp("asan") / "host_check")
    cmd = ["g++", "-std=c++17", "-g", "-O1", "-fno-omit-frame-pointer", "-fsanitize=address,undefined",
           "-fno-sanitize-recover=undefined", "-I", CSRC, os.path.join(HERE, "host_check.cpp"),
           os.path.join(CSRC, "symbolic.cpp"), os.path.join(CSRC, "frontal.cpp"),
           os.path.join(CSRC, "symbolic_capi.cpp"), "-o", out]
    r = subprocess.run(cmd, capture_output=True, text=True)
    if r.returncode != 0 and "asan" in (r.stderr or "").lower():
        pytest.skip("the sanitizer runtime is not available: " + r.stderr[-300:])
    assert r.returncode == 0, r.stderr[-2000:]
    return out


@pytest.mark.parametrize("name,build,mode", [
    ("mesh", lambda: netgen.config(1), "s"),
    ("chain", lambda: netgen.inverter_chain(seed=5, n_stages=40), "s"),
    ("grid", lambda: netgen.power_grid(seed=9003, side=24, T=0.05e-9, stim_seed=9004, n_drivers=12), "f"),
])
def test_host_analyses_run_clean_under_sanitizers(checker, tmp_path, name, build, mode):
    path = str(tmp_path / f"{name}.bin")
    _write(build(), path)
    env = dict(os.environ, ASAN_OPTIONS="detect_leaks=1:abort_on_error=1",
               UBSAN_OPTIONS="print_stacktrace=1:halt_on_error=1")
    r = subprocess.run([checker, path, mode], capture_output=True, text=True, env=env, timeout=600)
    assert r.returncode == 0 and r.stdout.startswith("ok"), (r.stdout + r.stderr)[-3000:]
    assert "runtime error" not in r.stderr, r.stderr[-3000:]
