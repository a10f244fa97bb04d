"""The C-ABI boundary without a GPU: libexpri.so loads, exports every function
include/expri.h declares (and nothing the binding uses is missing), the
host-only entry points behave as documented, and set-up errors are reported
as status codes rather than crashes."""
import ctypes as C
import os
import re

import numpy as np
import pytest

import netgen
import paper_1511_04515_amd as E

HEADER = os.path.join(os.path.dirname(os.path.dirname(os.path.abspath(__file__))), "include", "expri.h")


def header_functions():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"^[A-Za-z_][\w \*]*?\b(expri_\w+)\s*\(", text, flags=re.M)))


def test_header_declares_the_documented_entry_points():
    names = header_functions()
    for must in ("expri_setup", "expri_factor", "expri_step", "expri_run", "expri_mevp", "expri_solve",
                 "expri_dc", "expri_destroy", "expri_last_error"):
        assert must in names


def test_library_exports_every_declared_function():
    lib = E.load_library()
    missing = [n for n in header_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_binding_uses_only_declared_functions():
    assert set(E.binding.ENTRY_POINTS) <= set(header_functions())


def test_default_opts_are_the_documented_defaults():
    o = E.default_opts()
    assert o.E_rr == 1e-6 and o.eps_krylov == pytest.approx(1e-7)
    assert o.alpha == 0.5 and o.beta == 2.0 and o.grow_if_rejects_lt == 5
    assert o.h_init == 1e-13 and o.h_min == 1e-18 and o.m_max == 60


def test_null_arguments_are_rejected_without_a_gpu():
    lib = E.load_library()
    EINVAL = -1
    assert lib.expri_default_opts(None) == EINVAL
    assert lib.expri_workspace_size(None, None) == EINVAL
    assert lib.expri_symbolic_create(None, None) == EINVAL
    lib.expri_destroy(None)          # a no-op by contract
    lib.expri_symbolic_destroy(None)


def test_symbolic_entry_points_validate_input():
    net = netgen.inverter_chain(seed=1, n_stages=3)
    S = E.symbolic_analysis(net, block_size=256)
    assert S["perm"].size == net.n and sorted(S["perm"].tolist()) == list(range(net.n))
    # a block size outside {256, 512, 1024} is refused
    with pytest.raises(E.ExpriError):
        E.symbolic_analysis(net, block_size=128)
