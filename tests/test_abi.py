"""The C-ABI library builds for gfx950, loads, and exports every declared entry point.

No compute call is made here (this runs without a GPU).
"""
import ctypes
import os
import re

from paper_2111_02912_amd import _lib

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def declared_symbols():
    inc = os.path.join(ROOT, "include")
    src = "".join(open(os.path.join(inc, f)).read() for f in sorted(os.listdir(inc)) if f.endswith(".h"))
    src = re.sub(r"/\*.*?\*/", "", src, flags=re.S)
    return sorted(set(re.findall(r"\b(kbn_[a-z_0-9]+)\s*\(", src)))


def test_header_and_binding_agree():
    assert declared_symbols() == sorted(_lib.EXPORTS)


def test_header_constants_match_binding():
    inc = os.path.join(ROOT, "include")
    src = "".join(open(os.path.join(inc, f)).read() for f in sorted(os.listdir(inc)) if f.endswith(".h"))
    consts = re.findall(r"#define\s+(KBN_[A-Z_0-9]+)\s+\(?(-?\d+)\)?", src)
    assert len(consts) >= 15
    for name, val in consts:
        assert getattr(_lib, name) == int(val), name


def test_library_exports_every_symbol():
    L = ctypes.CDLL(_lib.LIB_PATH)
    for name in declared_symbols():
        assert hasattr(L, name), name


def test_error_strings_without_gpu():
    L = _lib.lib()
    assert L.kbn_strerror(0) == b"success"
    assert L.kbn_strerror(_lib.KBN_ERR_NONFINITE) == b"non-finite sample location"
    # argument validation happens before any device call
    h = ctypes.c_void_p()
    N = (ctypes.c_int64 * 2)(64, 64)
    assert L.kbn_plan_create(ctypes.byref(h), 4, N, None) == _lib.KBN_ERR_INVALID_ARG
    o = _lib.KbnOpts()
    o.J = 9
    assert L.kbn_plan_create(ctypes.byref(h), 2, N, ctypes.byref(o)) == _lib.KBN_ERR_INVALID_ARG
    assert b"J" in L.kbn_last_error()
    o = _lib.KbnOpts()
    o.sigma = 0.5
    assert L.kbn_plan_create(ctypes.byref(h), 2, N, ctypes.byref(o)) == _lib.KBN_ERR_INVALID_ARG
    big = (ctypes.c_int64 * 2)(600, 64)  # K = 1200 > 1024
    assert L.kbn_plan_create(ctypes.byref(h), 2, big, None) == _lib.KBN_ERR_UNSUPPORTED
    small = (ctypes.c_int64 * 2)(3, 64)  # K = 6 < 2 J: the window does not fit the grid
    assert L.kbn_plan_create(ctypes.byref(h), 2, small, None) == _lib.KBN_ERR_UNSUPPORTED
    zero = (ctypes.c_int64 * 2)(0, 64)
    assert L.kbn_plan_create(ctypes.byref(h), 2, zero, None) == _lib.KBN_ERR_INVALID_ARG
    assert L.kbn_set_points(None, 1, None, None) == _lib.KBN_ERR_INVALID_ARG
    assert L.kbn_forward(None, 1, 1, None, None, None, None) == _lib.KBN_ERR_INVALID_ARG
