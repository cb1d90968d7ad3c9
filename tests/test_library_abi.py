"""CPU checks of the C-ABI library: it loads and exports every entry point
declared in include/lmosem.h (no compute calls without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "lmosem.h")


def _declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(lmosem_[a-z_]+)\s*\(", text)))


@pytest.fixture(scope="module")
def lib_path():
    from paper_2002_12471_amd import LIB_PATH, build
    if not os.path.exists(LIB_PATH):
        build()
    return LIB_PATH


def test_header_declares_the_boundary():
    names = _declared()
    for n in ("lmosem_create", "lmosem_sensitivity", "lmosem_subset_update", "lmosem_reconstruct",
              "lmosem_destroy", "lmosem_last_error", "lmosem_abi_version", "lmosem_forward",
              "lmosem_backproject", "lmosem_events_load", "lmosem_iterate"):
        assert n in names


def test_library_exports_every_declared_symbol(lib_path):
    lib = ctypes.CDLL(lib_path)
    missing = [n for n in _declared() if not hasattr(lib, n)]
    assert not missing, missing


def test_abi_version_and_argument_checks_without_gpu(lib_path):
    lib = ctypes.CDLL(lib_path)
    lib.lmosem_abi_version.restype = ctypes.c_uint32
    assert lib.lmosem_abi_version() == 2
    # null arguments are rejected before any device call
    lib.lmosem_create.restype = ctypes.c_int
    out = ctypes.c_void_p()
    assert lib.lmosem_create(None, None, None, ctypes.byref(out)) == -1
    lib.lmosem_sensitivity.restype = ctypes.c_int
    assert lib.lmosem_sensitivity(None, 0, None) == -1
    lib.lmosem_destroy(None)


def test_binding_mirrors_the_header(lib_path):
    from paper_2002_12471_amd import lmosem as L
    for n in _declared():
        assert n in L.EXPORTED
        assert callable(getattr(L, n))
