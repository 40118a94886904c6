"""The C ABI library loads and exports every entry point declared in include/*.h (no GPU needed)."""

import ctypes
import glob
import os
import re

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
LIB = os.path.join(ROOT, "paper_2502_01157_amd", "librf.so")


def declared_functions():
    names = set()
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        for m in re.finditer(r"^\s*(?:const\s+)?[A-Za-z_][A-Za-z0-9_]*\s*\*?\s*(rf_[A-Za-z0-9_]+)\s*\(", text,
                             flags=re.M):
            names.add(m.group(1))
    return sorted(names)


def test_headers_declare_entry_points():
    names = declared_functions()
    for n in ("rf_render_forward", "rf_render_backward", "rf_pack_scene", "rf_raygen", "rf_last_error"):
        assert n in names


def test_library_exports_every_declared_symbol():
    if not os.path.exists(LIB):
        pytest.fail("librf.so is not built (run __graft_entry__.build())")
    lib = ctypes.CDLL(LIB)
    missing = [n for n in declared_functions() if not hasattr(lib, n)]
    assert not missing, missing


def test_host_side_errors_without_gpu():
    """Calls that fail argument checks return an error code before touching the device."""
    lib = ctypes.CDLL(LIB)
    lib.rf_last_error.restype = ctypes.c_char_p
    lib.rf_packed_bytes.argtypes = [ctypes.c_int64, ctypes.c_int64, ctypes.c_int32, ctypes.c_int32,
                                    ctypes.POINTER(ctypes.c_size_t)]
    n = ctypes.c_size_t()
    assert lib.rf_packed_bytes(1000, 15000, 3, 0, ctypes.byref(n)) == 0
    assert n.value >= 1000 * 256 + 15000 * 24
    n_bf = ctypes.c_size_t()
    assert lib.rf_packed_bytes(1000, 15000, 3, 1, ctypes.byref(n_bf)) == 0
    assert n_bf.value < n.value
    assert lib.rf_packed_bytes(1000, 15000, 4, 0, ctypes.byref(n)) == 1
    assert b"sh_degree" in lib.rf_last_error()
    assert lib.rf_packed_bytes(1 << 25, 15000, 3, 0, ctypes.byref(n)) == 4
    assert lib.rf_packed_bytes(0, 0, 3, 0, ctypes.byref(n)) == 1
    lib.rf_render_forward.argtypes = [ctypes.c_void_p] * 7
    assert lib.rf_render_forward(None, None, None, None, None, None, None) == 1
    assert lib.rf_last_error() != b""
