"""CG-SENSE and QPLS reconstruction on the GPU (kbn_cg_* of the C ABI).

Solves (E^H E + lambda T^H T) x = E^H y by plain conjugate gradients from
x = 0 (Sec. IV-B; T = I is CG-SENSE, T = first differences along each image
axis is QPLS), entirely in the HIP library, for a batch of independent
images that share the plan and coil maps: each iteration applies E^H E to
all of them at once while every image keeps its own CG scalars.  This module
allocates the solver's work buffer and the images with PyTorch and passes
pointers.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import torch

from . import _lib
from ._lib import check
from .nufft import KbNufft, _ptr, _stream

_SCAL = 32  # doubles of CG state per image at the start of the work buffer
REGS = {"identity": _lib.KBN_REG_IDENTITY, "finite_diff": _lib.KBN_REG_FINITE_DIFF}


def reg_code(reg) -> int:
    if reg not in REGS:
        raise ValueError(f"reg must be one of {sorted(REGS)}, got {reg!r}")
    return REGS[reg]


class CgSense:
    """One CG-SENSE solve in progress for `batch` images on a plan (points
    already set).  ``x`` is [batch, *N]."""

    def __init__(self, plan: KbNufft, coils: int = 1, batch: int = 1):
        plan._need_points()
        self.plan = plan
        self.C = int(coils)
        self.B = int(batch)
        nb = ctypes.c_int64()
        check(_lib.lib().kbn_cg_work_bytes(plan._h, self.B, self.C, ctypes.byref(nb)), "kbn_cg_work_bytes")
        self.work_bytes = int(nb.value)
        self.work = torch.empty(self.work_bytes, dtype=torch.uint8, device=plan.device)
        self.x = torch.empty((self.B,) + plan.N, dtype=torch.complex64, device=plan.device)

    def begin(self, y: torch.Tensor, smaps: Optional[torch.Tensor] = None):
        """x = 0, r = p = E^H y.  y: [B, C, M] (or [C, M] when B = 1) complex64."""
        p = self.plan
        s, C = p._maps(smaps)
        if C != self.C:
            raise ValueError(f"smaps has {C} coils, solver was made for {self.C}")
        yy = p._ksp(y, self.B, C, "y")
        self._keep = (yy, s)
        check(_lib.lib().kbn_cg_begin(p._h, self.B, C, _ptr(s), _ptr(yy), _ptr(self.x), _ptr(self.work),
                                      _stream(p.device)), "kbn_cg_begin")
        return self

    def begin_rhs(self, b: torch.Tensor, smaps: Optional[torch.Tensor] = None):
        """x = 0, r = p = b for image right-hand sides b [B, *N] (solving
        (E^H E + lam T^H T) x = b)."""
        p = self.plan
        s, C = p._maps(smaps)
        if C != self.C:
            raise ValueError(f"smaps has {C} coils, solver was made for {self.C}")
        bb = p._img(b, "b")
        if bb.shape[0] != self.B:
            raise ValueError(f"b holds {bb.shape[0]} images, solver was made for {self.B}")
        self._keep = (bb, s)
        check(_lib.lib().kbn_cg_begin_image(p._h, self.B, C, _ptr(bb), _ptr(self.x), _ptr(self.work),
                                            _stream(p.device)), "kbn_cg_begin_image")
        return self

    def step(self, iters: int, lam: float = 1e-3, reg: str = "identity"):
        """Run `iters` more iterations with F = E^H E + lam T^H T."""
        p = self.plan
        s = self._keep[1]
        check(_lib.lib().kbn_cg_step(p._h, self.B, self.C, _ptr(s), float(lam), reg_code(reg), int(iters),
                                     _ptr(self.x), _ptr(self.work), _stream(p.device)), "kbn_cg_step")
        return self

    def scalars(self) -> torch.Tensor:
        """Device view [B, 8] of [r'r, b'b, p'q, alpha, beta, ||r||/||b||, iterations, -]."""
        return self.work[: 8 * _SCAL * self.B].view(torch.float64).reshape(self.B, _SCAL)[:, :8]

    def residuals(self) -> torch.Tensor:
        """||r|| / ||b|| of every image after the iterations so far (synchronises)."""
        return self.scalars()[:, 5].cpu()

    def residual(self) -> float:
        """||r|| / ||b|| of the first image (synchronises)."""
        return float(self.scalars()[0, 5].item())


def cg_sense(plan: KbNufft, y: torch.Tensor, smaps: Optional[torch.Tensor] = None,
             lam: float = 1e-3, iters: int = 10, reg: str = "identity"):
    """Return (x, ||r||/||b||) after `iters` CG iterations: y [C, M] gives
    x [*N] and a float; y [B, C, M] gives x [B, *N] and a [B] tensor."""
    C = 1 if smaps is None else int(smaps.shape[0])
    if y.dim() == 2:
        s = CgSense(plan, C, 1).begin(y, smaps).step(iters, lam, reg)
        return s.x[0], s.residual()
    s = CgSense(plan, C, int(y.shape[0])).begin(y, smaps).step(iters, lam, reg)
    return s.x, s.residuals()
