"""The C-ABI library loads without a GPU and exports every entry point that
include/hsd.h declares (CPU only: no compute calls)."""

import ctypes
import os
import re
import subprocess

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "hsd.h")
LIB = os.path.join(ROOT, "paper_1311_4627_amd", "libhsd.so")


def declared_symbols():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(hsd_[a-z_A-Z0-9]+)\s*\(", text)))


def test_header_declares_the_binding_symbols():
    from paper_1311_4627_amd import hsd
    assert set(declared_symbols()) == set(hsd.SYMBOLS)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhsd.so not built (run __graft_entry__.build())")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    for name in declared_symbols():
        assert hasattr(lib, name), name
    out = subprocess.run(["nm", "-D", "--defined-only", LIB], capture_output=True, text=True).stdout
    exported = set(re.findall(r"\bT (hsd_\w+)", out))
    assert set(declared_symbols()) <= exported


@pytest.mark.skipif(not os.path.exists(LIB), reason="libhsd.so not built (run __graft_entry__.build())")
def test_binding_rejects_bad_arguments_without_a_gpu():
    from paper_1311_4627_amd import hsd
    lib = hsd.lib()
    out = ctypes.c_void_p()
    # null grid / too short grid are argument errors, reported before any device call
    assert lib.hsd_create(0, None, 400, ctypes.byref(out)) == -1
    import numpy as np
    lam = np.geomspace(1e-5, 1e-1, 8)
    assert lib.hsd_create(0, hsd._dptr(lam), 8, ctypes.byref(out)) == -1
    lam = np.linspace(1e-5, 1e-1, 64)                 # not log-uniform
    assert lib.hsd_create(0, hsd._dptr(lam), 64, ctypes.byref(out)) == -2
