"""CG-SENSE and QPLS reconstruction on the GPU (kbn_cg_* of the C ABI).

Solves (E^H E + lambda T^H T) x = E^H y by plain conjugate gradients from
x = 0 (Sec. IV-B; T = I is CG-SENSE, T = first differences along each image
axis is QPLS), entirely in the HIP library: this module allocates the
solver's work buffer and the image with PyTorch and passes pointers.
"""
from __future__ import annotations

import ctypes
from typing import Optional

import torch

from . import _lib
from ._lib import check
from .nufft import KbNufft, _ptr, _stream

_SCAL = 8  # leading doubles of the work buffer that hold the CG scalars
REGS = {"identity": _lib.KBN_REG_IDENTITY, "finite_diff": _lib.KBN_REG_FINITE_DIFF}


def reg_code(reg) -> int:
    if reg not in REGS:
        raise ValueError(f"reg must be one of {sorted(REGS)}, got {reg!r}")
    return REGS[reg]


class CgSense:
    """One CG-SENSE solve in progress on a plan (points already set)."""

    def __init__(self, plan: KbNufft, coils: int = 1):
        plan._need_points()
        self.plan = plan
        self.C = int(coils)
        nb = ctypes.c_int64()
        check(_lib.lib().kbn_cg_work_bytes(plan._h, self.C, ctypes.byref(nb)), "kbn_cg_work_bytes")
        self.work_bytes = int(nb.value)
        self.work = torch.empty(self.work_bytes, dtype=torch.uint8, device=plan.device)
        self.x = torch.empty(plan.N, dtype=torch.complex64, device=plan.device)

    def begin(self, y: torch.Tensor, smaps: Optional[torch.Tensor] = None):
        """x = 0, r = p = E^H y.  y: [C, M] (or [1, C, M]) complex64."""
        p = self.plan
        s, C = p._maps(smaps)
        if C != self.C:
            raise ValueError(f"smaps has {C} coils, solver was made for {self.C}")
        yy = p._ksp(y, 1, C, "y")
        self._keep = (yy, s)
        check(_lib.lib().kbn_cg_begin(p._h, C, _ptr(s), _ptr(yy), _ptr(self.x), _ptr(self.work),
                                      _stream(p.device)), "kbn_cg_begin")
        return self

    def begin_rhs(self, b: torch.Tensor, smaps: Optional[torch.Tensor] = None):
        """x = 0, r = p = b for an image right-hand side b [*N] (solving
        (E^H E + lam I) x = b)."""
        p = self.plan
        s, C = p._maps(smaps)
        if C != self.C:
            raise ValueError(f"smaps has {C} coils, solver was made for {self.C}")
        bb = p._img(b, "b").reshape(p.N)
        self._keep = (bb, s)
        check(_lib.lib().kbn_cg_begin_image(p._h, C, _ptr(bb), _ptr(self.x), _ptr(self.work),
                                            _stream(p.device)), "kbn_cg_begin_image")
        return self

    def step(self, iters: int, lam: float = 1e-3, reg: str = "identity"):
        """Run `iters` more iterations with F = E^H E + lam T^H T."""
        p = self.plan
        s = self._keep[1]
        check(_lib.lib().kbn_cg_step(p._h, self.C, _ptr(s), float(lam), reg_code(reg), int(iters),
                                     _ptr(self.x), _ptr(self.work), _stream(p.device)), "kbn_cg_step")
        return self

    def scalars(self) -> torch.Tensor:
        """Device view of [r'r, b'b, p'q, alpha, beta, ||r||/||b||, iterations, -]."""
        return self.work[: 8 * _SCAL].view(torch.float64)

    def residual(self) -> float:
        """||r|| / ||b|| after the iterations issued so far (synchronises)."""
        return float(self.scalars()[5].item())


def cg_sense(plan: KbNufft, y: torch.Tensor, smaps: Optional[torch.Tensor] = None,
             lam: float = 1e-3, iters: int = 10, reg: str = "identity"):
    """Return (x [*N] complex64, ||r||/||b||) after `iters` CG iterations."""
    C = 1 if smaps is None else int(smaps.shape[0])
    s = CgSense(plan, C).begin(y, smaps).step(iters, lam, reg)
    return s.x, s.residual()
