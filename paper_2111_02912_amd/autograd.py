"""Differentiable NUFFT layers: torch.autograd.Function pairs whose backward
passes are the omega-Jacobians of the paper.

Forward operator y = E(omega) x with E = (I_C kron A(omega)) S (Sec. II-G):
  * grad_x     = E^H g                               (Sec. II-C: dAx/dx = A)
  * grad_omega = sum_{b,c} Im{ A(s_c x_b r^[d]) conj(g_{b,c}) }
    (eq. (e,Ax) combined with the vector-Jacobian rule (e,jac,Ax,v))
Adjoint operator x = E(omega)^H y:
  * grad_y     = E g                                 (Sec. II-D)
  * grad_omega = sum_{b,c} Im{ A(s_c g_b r^[d]) conj(y_{b,c}) }   (eq. (e,A'y))

g is PyTorch's gradient of a real loss, dL/dRe + i dL/dIm; with that
convention the expressions above are the true real derivatives (the factor
of two between g and the conjugate Wirtinger derivative is already in g).
Every value is computed by the HIP library: the forward saves its inputs
and the backward calls kbn_jac_x and kbn_jac_omega_* on the same plan.
Coil maps are constants here: a map that requires a gradient is rejected.
The backward is not itself differentiable (no double backward).
"""
from __future__ import annotations

from typing import Optional, Sequence

import torch
from torch.autograd.function import once_differentiable

from . import _lib
from .nufft import KbNufft


def _no_map_grad(smaps):
    if smaps is not None and smaps.requires_grad:
        raise NotImplementedError("gradients with respect to coil maps are not provided")


class _ForwardOp(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, omega, smaps, plan):
        _no_map_grad(smaps)
        plan.ensure_points(omega)
        y = plan.forward(x, smaps)
        ctx.plan = plan
        ctx.xshape = x.shape
        ctx.save_for_backward(x, omega, smaps)
        return y

    @staticmethod
    @once_differentiable
    def backward(ctx, g):
        x, omega, smaps = ctx.saved_tensors
        plan = ctx.plan
        plan.ensure_points(omega)
        g = g.contiguous()
        gx = gom = None
        if ctx.needs_input_grad[0]:
            gx = plan.jac_x(_lib.KBN_OP_FORWARD, g, smaps).reshape(ctx.xshape)
        if ctx.needs_input_grad[1]:
            gom = plan.jac_omega_fwd(x, g, smaps)
        return gx, gom, None, None


class _AdjointOp(torch.autograd.Function):
    @staticmethod
    def forward(ctx, y, omega, smaps, plan):
        _no_map_grad(smaps)
        plan.ensure_points(omega)
        x = plan.adjoint(y, smaps)
        ctx.plan = plan
        ctx.yshape = y.shape
        ctx.save_for_backward(y, omega, smaps)
        return x

    @staticmethod
    @once_differentiable
    def backward(ctx, g):
        y, omega, smaps = ctx.saved_tensors
        plan = ctx.plan
        plan.ensure_points(omega)
        g = g.contiguous()
        gy = gom = None
        if ctx.needs_input_grad[0]:
            gy = plan.jac_x(_lib.KBN_OP_ADJOINT, g, smaps).reshape(ctx.yshape)
        if ctx.needs_input_grad[1]:
            gom = plan.jac_omega_adj(y, g, smaps)
        return gy, gom, None, None


def nufft(x: torch.Tensor, omega: torch.Tensor, plan: KbNufft,
          smaps: Optional[torch.Tensor] = None) -> torch.Tensor:
    """y = E(omega) x: x [B, *N] complex64, omega [M, D] float32 -> [B, C, M]."""
    return _ForwardOp.apply(x, omega, smaps, plan)


def nufft_adjoint(y: torch.Tensor, omega: torch.Tensor, plan: KbNufft,
                  smaps: Optional[torch.Tensor] = None) -> torch.Tensor:
    """x = E(omega)^H y: y [B, C, M] complex64, omega [M, D] float32 -> [B, *N]."""
    return _AdjointOp.apply(y, omega, smaps, plan)


class KbNufftLayer(torch.nn.Module):
    """Module form: one plan per image shape, created on first use.

    ``forward(x, omega, smaps=None)`` applies E(omega) and
    ``adjoint(y, omega, smaps=None)`` applies E(omega)^H; both are
    differentiable in their first argument and in omega.
    """

    def __init__(self, N: Sequence[int], sigma: float = 2.0, J: int = 6, tile=None,
                 accuracy: Optional[str] = None):
        super().__init__()
        self.N = tuple(int(n) for n in N)
        self._cfg = dict(sigma=sigma, J=J, tile=tile, accuracy=accuracy)
        self._plans = {}

    def plan(self, device) -> KbNufft:
        device = torch.device(device)
        key = (device.type, device.index)
        if key not in self._plans:
            self._plans[key] = KbNufft(self.N, device=device, **self._cfg)
        return self._plans[key]

    def forward(self, x, omega, smaps=None):
        return nufft(x, omega, self.plan(x.device), smaps)

    def adjoint(self, y, omega, smaps=None):
        return nufft_adjoint(y, omega, self.plan(y.device), smaps)


# ---------------------------------------------------------------------------
# Off-resonance model (Sec. II-H): E_f = sum_l diag(b_l) A diag(c_l) (with S)
# ---------------------------------------------------------------------------

class _FieldForwardOp(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, omega, smaps, b, c, plan):
        _no_map_grad(smaps)
        if b.requires_grad or c.requires_grad:
            raise NotImplementedError("gradients with respect to b and c are not provided")
        plan.ensure_points(omega)
        ctx.plan = plan
        ctx.xshape = x.shape
        ctx.save_for_backward(x, omega, smaps, b, c)
        return plan.field_forward(x, b, c, smaps)

    @staticmethod
    @once_differentiable
    def backward(ctx, g):
        x, omega, smaps, b, c = ctx.saved_tensors
        plan = ctx.plan
        plan.ensure_points(omega)
        g = g.contiguous()
        gx = gom = None
        if ctx.needs_input_grad[0]:
            gx = plan.field_adjoint(g, b, c, smaps).reshape(ctx.xshape)
        if ctx.needs_input_grad[1]:
            gom = plan.field_jac_omega_fwd(x, g, b, c, smaps)
        return gx, gom, None, None, None, None


class _FieldAdjointOp(torch.autograd.Function):
    @staticmethod
    def forward(ctx, y, omega, smaps, b, c, plan):
        _no_map_grad(smaps)
        if b.requires_grad or c.requires_grad:
            raise NotImplementedError("gradients with respect to b and c are not provided")
        plan.ensure_points(omega)
        ctx.plan = plan
        ctx.yshape = y.shape
        ctx.save_for_backward(y, omega, smaps, b, c)
        return plan.field_adjoint(y, b, c, smaps)

    @staticmethod
    @once_differentiable
    def backward(ctx, g):
        y, omega, smaps, b, c = ctx.saved_tensors
        plan = ctx.plan
        plan.ensure_points(omega)
        g = g.contiguous()
        gy = gom = None
        if ctx.needs_input_grad[0]:
            gy = plan.field_forward(g, b, c, smaps).reshape(ctx.yshape)
        if ctx.needs_input_grad[1]:
            gom = plan.field_jac_omega_adj(y, g, b, c, smaps)
        return gy, gom, None, None, None, None


def nufft_field(x: torch.Tensor, omega: torch.Tensor, plan: KbNufft, b: torch.Tensor, c: torch.Tensor,
                smaps: Optional[torch.Tensor] = None) -> torch.Tensor:
    """y = E_f(omega) x with E_f = sum_l diag(b_l) A diag(c_l) S; [B, C, M]."""
    return _FieldForwardOp.apply(x, omega, smaps, b, c, plan)


def nufft_field_adjoint(y: torch.Tensor, omega: torch.Tensor, plan: KbNufft, b: torch.Tensor,
                        c: torch.Tensor, smaps: Optional[torch.Tensor] = None) -> torch.Tensor:
    """x = E_f(omega)^H y; [B, *N]."""
    return _FieldAdjointOp.apply(y, omega, smaps, b, c, plan)


# ---------------------------------------------------------------------------
# Gram and regularised-inverse operators (Sec. II-E, II-F)
# ---------------------------------------------------------------------------

def _gram_vjp(plan: KbNufft, x, g, smaps, need_x: bool, need_om: bool):
    """(dx, domega) for z = E^H E x with upstream g: the omega-gradient has
    one term from each factor of the Gram operator,
    Im{E(g r) conj(E x)} + Im{E(x r) conj(E g)} summed over coils, and
    dx = E^H E g."""
    eg = plan.forward(g, smaps)
    gx = gom = None
    if need_x:
        gx = plan.adjoint(eg, smaps)
    if need_om:
        ex = plan.forward(x, smaps)
        gom = plan.jac_omega_fwd(g, ex, smaps)
        plan.jac_omega_fwd(x, eg, smaps, out=gom, accumulate=True)
    return gx, gom


class _GramOp(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, omega, smaps, plan):
        _no_map_grad(smaps)
        plan.ensure_points(omega)
        z = plan.adjoint(plan.forward(x, smaps), smaps).reshape(x.shape)
        ctx.plan = plan
        ctx.xshape = x.shape
        ctx.save_for_backward(x, omega, smaps)
        return z

    @staticmethod
    @once_differentiable
    def backward(ctx, g):
        x, omega, smaps = ctx.saved_tensors
        plan = ctx.plan
        plan.ensure_points(omega)
        gx, gom = _gram_vjp(plan, x, g.contiguous().reshape(ctx.xshape), smaps,
                            ctx.needs_input_grad[0], ctx.needs_input_grad[1])
        if gx is not None:
            gx = gx.reshape(ctx.xshape)
        return gx, gom, None, None


def _cg_solve(plan: KbNufft, x, smaps, lam: float, iters: int, reg: str):
    """F^{-1} x for all images at once with the library's batched CG
    (F = E^H E + lam T^H T), started from the image right-hand sides x."""
    from .cg import CgSense
    C = 1 if smaps is None else int(smaps.shape[0])
    s = CgSense(plan, C, int(x.shape[0]))
    s.begin_rhs(x, smaps).step(iters, lam, reg)
    return s.x


class _InverseOp(torch.autograd.Function):
    @staticmethod
    def forward(ctx, x, omega, smaps, plan, lam, iters, reg):
        _no_map_grad(smaps)
        plan.ensure_points(omega)
        xb = x.reshape((-1,) + plan.N).contiguous()
        z = _cg_solve(plan, xb, smaps, lam, iters, reg)
        ctx.plan = plan
        ctx.xshape = x.shape
        ctx.lam, ctx.iters, ctx.reg = lam, iters, reg
        ctx.save_for_backward(z, omega, smaps)
        return z.reshape(x.shape)

    @staticmethod
    @once_differentiable
    def backward(ctx, g):
        z, omega, smaps = ctx.saved_tensors
        plan = ctx.plan
        plan.ensure_points(omega)
        w = _cg_solve(plan, g.contiguous().reshape(z.shape), smaps, ctx.lam, ctx.iters, ctx.reg)
        gom = None
        if ctx.needs_input_grad[1]:
            _, gom = _gram_vjp(plan, z, w, smaps, False, True)
            gom = -gom
        gx = w.reshape(ctx.xshape) if ctx.needs_input_grad[0] else None
        return gx, gom, None, None, None, None, None


def gram(x: torch.Tensor, omega: torch.Tensor, plan: KbNufft,
         smaps: Optional[torch.Tensor] = None) -> torch.Tensor:
    """z = E(omega)^H E(omega) x: x [B, *N] complex64 -> [B, *N]."""
    return _GramOp.apply(x, omega, smaps, plan)


def inverse(x: torch.Tensor, omega: torch.Tensor, plan: KbNufft,
            smaps: Optional[torch.Tensor] = None, lam: float = 1e-3,
            iters: int = 20, reg: str = "identity") -> torch.Tensor:
    """z = (E^H E + lam T^H T)^{-1} x by `iters` CG iterations per image
    (T = I for reg "identity", first differences along each image axis for
    "finite_diff"); the backward solves with the same operator (the solve is
    treated as exact and the exact inverse is differentiated).  Memory does
    not grow with the number of iterations."""
    from .cg import reg_code
    reg_code(reg)
    return _InverseOp.apply(x, omega, smaps, plan, float(lam), int(iters), reg)
