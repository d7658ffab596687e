"""The C-ABI library loads and exports every entry point include/pamo.h
declares (no compute calls: this runs without a GPU)."""
import ctypes
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HEADER = os.path.join(ROOT, "include", "pamo.h")
LIB = os.path.join(ROOT, "paper_2509_05595_amd", "libpamo.so")


def declared():
    text = open(HEADER).read()
    text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
    return sorted(set(re.findall(r"\b(pamo_[a-z_0-9]+)\s*\(", text)))


def test_header_declares_the_method_entry_points():
    names = declared()
    for n in ["pamo_quadrics", "pamo_select", "pamo_check", "pamo_collapse", "pamo_simplify", "pamo_create",
              "pamo_destroy", "pamo_last_error", "pamo_self_intersections", "pamo_tri_pairs"]:
        assert n in names


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpamo.so not built")
def test_library_exports_every_declared_symbol():
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared() if not hasattr(lib, n)]
    assert not missing, missing


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpamo.so not built")
def test_binding_covers_the_header():
    import sys
    sys.path.insert(0, ROOT)
    from paper_2509_05595_amd import native
    assert set(declared()) <= set(native.EXPORTS)
    assert ctypes.sizeof(native.Options) == 8 + 8 + 4 * 8 + 8 + 4 + 4 + 4 + 4  # ..., key_mode, pair_capacity, pad
    assert ctypes.sizeof(native.Stats) == 8 * 18
    assert ctypes.sizeof(native.MLP) == 4 * (2048 + 64 + 4096 + 64 + 64 + 1 + 5 + 1)


@pytest.mark.skipif(not os.path.exists(LIB), reason="libpamo.so not built")
def test_workspace_size_query():
    """pamo_workspace_bytes is host-only: refused sizes give 0, and the bytes
    grow with the mesh (about a kilobyte per face)."""
    lib = ctypes.CDLL(LIB)
    f = lib.pamo_workspace_bytes
    f.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_void_p]
    f.restype = ctypes.c_size_t
    assert f(3, 100, None) == 0 and f(100, 3, None) == 0 and f(4, 2 ** 31, None) == 0
    a, b = f(2562, 5120, None), f(655362, 1310720, None)
    assert 0 < a < b < 2000 * 1310720
    assert a % 256 == 0 and b % 256 == 0
