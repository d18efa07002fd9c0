"""ctypes binding of libkbnufft.so (argument marshalling only).

Every entry point of include/kbnufft.h is exposed under the same name.
Loading fails loudly when the library has not been built: there is no
fallback implementation.
"""
from __future__ import annotations

import ctypes
import os

LIB_PATH = os.path.join(os.path.dirname(os.path.abspath(__file__)), "libkbnufft.so")

KBN_OK = 0
KBN_ERR_INVALID_ARG = -1
KBN_ERR_UNSUPPORTED = -2
KBN_ERR_OOM = -3
KBN_ERR_HIP = -4
KBN_ERR_NONFINITE = -5
KBN_ERR_NO_POINTS = -6
KBN_OP_FORWARD = 0
KBN_OP_ADJOINT = 1
KBN_REG_IDENTITY = 0
KBN_REG_FINITE_DIFF = 1
KBN_TASK_FORWARD = 0
KBN_TASK_ADJOINT = 1
KBN_TASK_JAC_OMEGA_FWD = 2
KBN_TASK_JAC_OMEGA_ADJ = 3
KBN_TASK_JAC_X_FWD = 4
KBN_TASK_JAC_X_ADJ = 5
KBN_STATIC_WORKSPACE = 67108864

EXPORTS = (
    "kbn_plan_create", "kbn_plan_footprint", "kbn_set_points", "kbn_forward", "kbn_forward_static",
    "kbn_adjoint",
    "kbn_jac_omega_fwd", "kbn_forward_jac_omega", "kbn_jac_omega_adj", "kbn_jac_x", "kbn_plan_info",
    "kbn_get_points", "kbn_check_error", "kbn_plan_destroy", "kbn_strerror",
    "kbn_last_error", "kbn_timing", "kbn_timing_select", "kbn_timing_read", "kbn_timing_name",
    "kbn_batch_create", "kbn_batch_run", "kbn_batch_capture", "kbn_batch_fuse", "kbn_batch_launch",
    "kbn_batch_destroy", "kbn_cg_work_bytes", "kbn_cg_begin", "kbn_cg_step",
    "kbn_cg_begin_image", "kbn_field_forward", "kbn_field_adjoint", "kbn_field_jac_omega_fwd",
    "kbn_field_jac_omega_adj", "kbn_field_segments",
)


class KbnOpts(ctypes.Structure):
    _fields_ = [
        ("sigma", ctypes.c_double),
        ("J", ctypes.c_int),
        ("tile", ctypes.c_int * 3),
        ("max_workspace", ctypes.c_int64),
        ("spread_tile", ctypes.c_int),
    ]


# kbn_allocator: alloc(ctx, bytes, stream) -> ptr, free(ctx, ptr, stream)
ALLOC_FN = ctypes.CFUNCTYPE(ctypes.c_void_p, ctypes.c_void_p, ctypes.c_size_t, ctypes.c_void_p)
FREE_FN = ctypes.CFUNCTYPE(None, ctypes.c_void_p, ctypes.c_void_p, ctypes.c_void_p)


class KbnAllocator(ctypes.Structure):
    _fields_ = [
        ("ctx", ctypes.c_void_p),
        ("alloc", ALLOC_FN),
        ("free", FREE_FN),
    ]


class KbnTask(ctypes.Structure):
    _fields_ = [
        ("plan", ctypes.c_void_p),
        ("op", ctypes.c_int),
        ("B", ctypes.c_int),
        ("C", ctypes.c_int),
        ("a", ctypes.c_void_p),
        ("smaps", ctypes.c_void_p),
        ("g", ctypes.c_void_p),
        ("out", ctypes.c_void_p),
        ("accumulate", ctypes.c_int),
    ]


class KbnError(RuntimeError):
    def __init__(self, code: int, where: str, msg: str):
        super().__init__(f"{where}: {msg} (code {code})")
        self.code = code


_lib = None


def lib():
    """Load the HIP library (once).  Raises if it is missing."""
    global _lib
    if _lib is not None:
        return _lib
    if not os.path.exists(LIB_PATH):
        raise RuntimeError(
            f"{LIB_PATH} is missing: build it with `python -m paper_2111_02912_amd.build`")
    L = ctypes.CDLL(LIB_PATH)
    vp = ctypes.c_void_p
    i64 = ctypes.c_int64
    ci = ctypes.c_int
    L.kbn_plan_create.argtypes = [ctypes.POINTER(vp), ci, ctypes.POINTER(i64), ctypes.POINTER(KbnOpts),
                                  ctypes.POINTER(KbnAllocator), vp]
    L.kbn_plan_footprint.argtypes = [ci, ctypes.POINTER(i64), ctypes.POINTER(KbnOpts), i64, ci, ci, ci,
                                     ctypes.POINTER(i64)]
    L.kbn_set_points.argtypes = [vp, i64, vp, vp]
    L.kbn_forward.argtypes = [vp, ci, ci, vp, vp, vp, vp]
    L.kbn_forward_static.argtypes = [vp, ci, ci, vp, vp, vp, vp]
    L.kbn_adjoint.argtypes = [vp, ci, ci, vp, vp, vp, vp]
    L.kbn_jac_omega_fwd.argtypes = [vp, ci, ci, vp, vp, vp, vp, ci, vp]
    L.kbn_forward_jac_omega.argtypes = [vp, ci, ci, vp, vp, vp, vp, vp, ci, vp]
    L.kbn_jac_omega_adj.argtypes = [vp, ci, ci, vp, vp, vp, vp, ci, vp]
    L.kbn_jac_x.argtypes = [vp, ci, ci, ci, vp, vp, vp, vp]
    L.kbn_plan_info.argtypes = [vp, ctypes.POINTER(i64), ctypes.POINTER(ci), ctypes.POINTER(ci),
                                ctypes.POINTER(ctypes.c_double), ctypes.POINTER(i64),
                                ctypes.POINTER(i64), ctypes.POINTER(i64)]
    L.kbn_get_points.argtypes = [vp, vp, vp, vp, vp, vp]
    L.kbn_check_error.argtypes = [vp, vp]
    L.kbn_plan_destroy.argtypes = [vp, vp]
    L.kbn_strerror.argtypes = [ci]
    L.kbn_strerror.restype = ctypes.c_char_p
    L.kbn_last_error.argtypes = []
    L.kbn_last_error.restype = ctypes.c_char_p
    L.kbn_timing.argtypes = [vp, ci]
    L.kbn_timing_select.argtypes = [vp, ctypes.c_uint]
    L.kbn_timing_read.argtypes = [vp, ci, ctypes.POINTER(i64), ctypes.POINTER(ctypes.c_double)]
    L.kbn_timing_name.argtypes = [ci]
    L.kbn_timing_name.restype = ctypes.c_char_p
    L.kbn_batch_create.argtypes = [ctypes.POINTER(vp), ci, ctypes.POINTER(KbnTask), ci]
    L.kbn_batch_run.argtypes = [vp, vp]
    L.kbn_batch_capture.argtypes = [vp, vp]
    L.kbn_batch_fuse.argtypes = [vp, ci]
    L.kbn_batch_launch.argtypes = [vp, vp]
    L.kbn_batch_destroy.argtypes = [vp]
    L.kbn_cg_work_bytes.argtypes = [vp, ci, ci, ctypes.POINTER(i64)]
    L.kbn_cg_begin.argtypes = [vp, ci, ci, vp, vp, vp, vp, vp]
    L.kbn_cg_step.argtypes = [vp, ci, ci, vp, ctypes.c_double, ci, ci, vp, vp, vp]
    L.kbn_cg_begin_image.argtypes = [vp, ci, ci, vp, vp, vp, vp]
    L.kbn_field_forward.argtypes = [vp, ci, ci, ci, vp, vp, vp, vp, vp, vp]
    L.kbn_field_adjoint.argtypes = [vp, ci, ci, ci, vp, vp, vp, vp, vp, vp]
    L.kbn_field_jac_omega_fwd.argtypes = [vp, ci, ci, ci, vp, vp, vp, vp, vp, vp, ci, vp]
    L.kbn_field_jac_omega_adj.argtypes = [vp, ci, ci, ci, vp, vp, vp, vp, vp, vp, ci, vp]
    L.kbn_field_segments.argtypes = [ctypes.c_int64, vp, ctypes.c_double, ctypes.c_double,
                                     ctypes.c_int64, vp, ci, vp, vp, vp]
    for name in EXPORTS:
        if name not in ("kbn_strerror", "kbn_last_error", "kbn_timing_name"):
            getattr(L, name).restype = ci
    _lib = L
    return L


def check(code: int, where: str) -> int:
    if code != KBN_OK:
        L = lib()
        msg = L.kbn_last_error().decode() or L.kbn_strerror(code).decode()
        raise KbnError(code, where, msg)
    return code
