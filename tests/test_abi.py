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
    assert L.kbn_plan_create(ctypes.byref(h), 4, N, None, None, None) == _lib.KBN_ERR_INVALID_ARG
    o = _lib.KbnOpts()
    o.J = 9
    assert L.kbn_plan_create(ctypes.byref(h), 2, N, ctypes.byref(o), None, None) == _lib.KBN_ERR_INVALID_ARG
    assert b"J" in L.kbn_last_error()
    o = _lib.KbnOpts()
    o.sigma = 0.5
    assert L.kbn_plan_create(ctypes.byref(h), 2, N, ctypes.byref(o), None, None) == _lib.KBN_ERR_INVALID_ARG
    big = (ctypes.c_int64 * 2)(600, 64)  # K = 1200 > 1024
    assert L.kbn_plan_create(ctypes.byref(h), 2, big, None, None, None) == _lib.KBN_ERR_UNSUPPORTED
    small = (ctypes.c_int64 * 2)(3, 64)  # K = 6 < 2 J: the window does not fit the grid
    assert L.kbn_plan_create(ctypes.byref(h), 2, small, None, None, None) == _lib.KBN_ERR_UNSUPPORTED
    zero = (ctypes.c_int64 * 2)(0, 64)
    assert L.kbn_plan_create(ctypes.byref(h), 2, zero, None, None, None) == _lib.KBN_ERR_INVALID_ARG
    assert L.kbn_set_points(None, 1, None, None) == _lib.KBN_ERR_INVALID_ARG
    assert L.kbn_forward(None, 1, 1, None, None, None, None) == _lib.KBN_ERR_INVALID_ARG
    assert L.kbn_batch_fuse(None, 1) == _lib.KBN_ERR_INVALID_ARG
    assert L.kbn_batch_capture(None, None) == _lib.KBN_ERR_INVALID_ARG
    assert L.kbn_check_error(None, None) == _lib.KBN_ERR_INVALID_ARG
    assert L.kbn_timing_select(None, 1) == _lib.KBN_ERR_INVALID_ARG



def test_failing_allocator_gives_oom_and_no_plan():
    """Every device buffer of a plan comes from the caller's allocator: an
    allocator that refuses the first block makes creation fail with
    KBN_ERR_OOM before any device call, with no plan returned and nothing
    to release."""
    L = _lib.lib()
    calls = {"alloc": 0, "free": 0}

    def alloc(ctx, nbytes, stream):
        calls["alloc"] += 1
        assert nbytes > 0 and nbytes % 256 == 0
        return None

    def free(ctx, ptr, stream):
        calls["free"] += 1

    a_cb, f_cb = _lib.ALLOC_FN(alloc), _lib.FREE_FN(free)
    a = _lib.KbnAllocator(None, a_cb, f_cb)
    h = ctypes.c_void_p(1234)
    N = (ctypes.c_int64 * 2)(64, 48)
    assert L.kbn_plan_create(ctypes.byref(h), 2, N, None, ctypes.byref(a), None) == _lib.KBN_ERR_OOM
    assert h.value is None
    assert calls == {"alloc": 1, "free": 0}
    assert b"allocator" in L.kbn_last_error()
    # an allocator missing one of its functions is rejected
    half = _lib.KbnAllocator(None, a_cb, _lib.FREE_FN())
    assert L.kbn_plan_create(ctypes.byref(h), 2, N, None, ctypes.byref(half), None) == _lib.KBN_ERR_INVALID_ARG


def test_footprint_host_only():
    """kbn_plan_footprint sizes a plan without a GPU: it grows with the
    points, the batch and the Jacobian channels, follows sigma through the
    grid rule, and applies the workspace cap."""
    from paper_2111_02912_amd.nufft import footprint
    base = footprint((256, 256), 32768, B=1, C=1)
    assert base > 2 * 512 * 512 * 8  # at least the two grids of one channel
    assert footprint((256, 256), 65536) > base
    assert footprint((256, 256), 32768, B=4, C=8) > footprint((256, 256), 32768, B=1, C=8) > base
    assert footprint((256, 256), 32768, jac=True) > base
    # sigma 1.25 (grid 320) needs less than sigma 2 (grid 512)
    assert footprint((256, 256), 32768, accuracy="low") < base
    # a workspace cap chunks the batch
    capped = footprint((256, 256), 32768, B=64, C=8, max_workspace=64 << 20)
    assert capped < footprint((256, 256), 32768, B=64, C=8)
    L = _lib.lib()
    out = ctypes.c_int64()
    N = (ctypes.c_int64 * 3)(64, 64, 64)
    # the owner lists index M 2^D entries with int32 positions
    assert L.kbn_plan_footprint(3, N, None, 2 ** 28, 1, 1, 0, ctypes.byref(out)) == _lib.KBN_ERR_INVALID_ARG
    assert L.kbn_plan_footprint(3, N, None, 2 ** 28 - 1, 1, 1, 0, ctypes.byref(out)) == _lib.KBN_OK
