"""Trajectory learning with the differentiable NUFFT layers (Sec. IV-B).

The training loss of the paper for a reconstruction x_K(omega) is
  L(omega) = ||x_K(omega) - x_true||^2
             + mu1 phi_{gamma dt gmax}(|D1 omega|) + mu2 phi_{gamma dt^2 smax}(|D2 omega|),
  phi_lam(|v|) = sum max(|v| - lam, 0),
with D1, D2 the first and second differences along each shot (soft limits
on gradient strength and slew rate), noiseless data y = E(omega) x_true, and
each shot parameterised by quadratic B-spline kernels (40 per shot in the
paper), initialised from an undersampled radial trajectory (16 spokes of
1280 samples, 5 ms each) and trained with Adam.

Readings where the paper is silent: |.| is taken per axis (each gradient
axis has its own limit); omega is in radians per voxel, so a k-space step
gamma g dt (cycles/cm) becomes 2 pi dx gamma g dt radians with the voxel
size dx = FOV / N (FOV 22 cm by default); gamma = 4257.6 Hz/G.  The
reconstruction here is CG-SENSE (or QPLS) through the regularised-inverse
layer, x_K = (E^H E + lam T^H T)^{-1} E^H y, so the gradient of the
reconstruction costs a fixed amount of memory whatever the CG count.

Every NUFFT, Jacobian and CG step runs in the HIP library; this module only
holds the loss, the spline basis (a fixed [samples, knots] matrix) and the
optimiser loop, in PyTorch.
"""
from __future__ import annotations

import math
from typing import Optional

import torch

from .autograd import inverse, nufft, nufft_adjoint
from .nufft import KbNufft

GAMMA_HZ_PER_G = 4257.6


def quadratic_bspline_basis(samples: int, knots: int) -> torch.Tensor:
    """[samples, knots] float64 basis of uniform quadratic B-splines whose
    centres are spaced h = (samples - 1) / (knots - 3) apart from -h, so that
    the kernels sum to one at every sample."""
    if knots < 4 or samples < 2:
        raise ValueError("need at least 4 knots and 2 samples")
    h = (samples - 1) / (knots - 3)
    s = torch.arange(samples, dtype=torch.float64)[:, None]
    centres = (torch.arange(knots, dtype=torch.float64)[None, :] - 1.0) * h
    t = (s - centres).abs() / h
    inner = 0.75 - t * t
    outer = 0.5 * (t - 1.5) ** 2
    return torch.where(t <= 0.5, inner, torch.where(t <= 1.5, outer, torch.zeros_like(t)))


def radial_init(shots: int, samples: int) -> torch.Tensor:
    """Undersampled radial start: `shots` spokes through the centre, angles
    uniform over pi, radius pi (2k - R) / R.  [shots, samples, 2] float64."""
    ang = torch.arange(shots, dtype=torch.float64) * math.pi / shots
    k = torch.arange(samples, dtype=torch.float64)
    rho = math.pi * (2.0 * k - samples) / samples
    return torch.stack([rho[None] * torch.cos(ang)[:, None], rho[None] * torch.sin(ang)[:, None]], -1)


def hardware_limits(dt: float, fov_cm: float, n: int, gmax: float = 5.0, smax: float = 15.0):
    """Per-sample limits on |D1 omega| and |D2 omega| in radians per voxel for
    gradient strength gmax (G/cm) and slew rate smax (G/cm/ms)."""
    dx = fov_cm / n
    k1 = GAMMA_HZ_PER_G * gmax * dt                  # cycles/cm per sample
    k2 = GAMMA_HZ_PER_G * (smax * 1e3) * dt * dt     # cycles/cm per sample^2
    return 2.0 * math.pi * dx * k1, 2.0 * math.pi * dx * k2


def soft_limit(v: torch.Tensor, lam: float) -> torch.Tensor:
    """phi_lam(|v|) = sum max(|v| - lam, 0)."""
    return torch.clamp(v.abs() - lam, min=0.0).sum()


def hardware_penalty(omega_shots: torch.Tensor, lim1: float, lim2: float, mu1: float = 10.0,
                     mu2: float = 10.0) -> torch.Tensor:
    """mu1 phi(|D1 omega|) + mu2 phi(|D2 omega|) over [shots, samples, D]."""
    d1 = omega_shots[:, 1:] - omega_shots[:, :-1]
    d2 = d1[:, 1:] - d1[:, :-1]
    return mu1 * soft_limit(d1, lim1) + mu2 * soft_limit(d2, lim2)


class TrajectoryLearner:
    """Adam on the spline coefficients of a multi-shot 2D trajectory."""

    def __init__(self, N, shots: int = 16, samples: int = 1280, knots: int = 40,
                 readout_s: float = 5e-3, fov_cm: float = 22.0, gmax: float = 5.0, smax: float = 15.0,
                 mu1: float = 10.0, mu2: float = 10.0, lam: float = 1e-3, cg_iters: int = 20,
                 reg: str = "identity", lr: float = 1e-4, accuracy: Optional[str] = None, device=None):
        self.N = tuple(int(n) for n in N)
        self.device = torch.device(device) if device is not None else torch.device("cuda", 0)
        self.shots, self.samples = shots, samples
        self.basis = quadratic_bspline_basis(samples, knots).to(torch.float32).to(self.device)
        init = radial_init(shots, samples)
        b64 = quadratic_bspline_basis(samples, knots)
        coef = torch.linalg.lstsq(b64[None].expand(shots, -1, -1), init).solution  # [shots, knots, 2]
        self.coef = coef.to(torch.float32).to(self.device).requires_grad_(True)
        self.lim1, self.lim2 = hardware_limits(readout_s / samples, fov_cm, max(self.N), gmax, smax)
        self.mu1, self.mu2 = mu1, mu2
        self.lam, self.cg_iters, self.reg = lam, cg_iters, reg
        self.plan = KbNufft(self.N, device=self.device, accuracy=accuracy)
        self.opt = torch.optim.Adam([self.coef], lr=lr)

    def omega_shots(self) -> torch.Tensor:
        return torch.matmul(self.basis, self.coef)  # [shots, samples, 2]

    def loss(self, x_true: torch.Tensor, smaps: torch.Tensor):
        """(total, reconstruction term, penalty) for images x_true [B, *N]."""
        om_s = self.omega_shots()
        om = om_s.reshape(-1, 2)
        y = nufft(x_true, om, self.plan, smaps)
        b = nufft_adjoint(y, om, self.plan, smaps)
        xk = inverse(b, om, self.plan, smaps, lam=self.lam, iters=self.cg_iters, reg=self.reg)
        rec = torch.view_as_real(xk - x_true).pow(2).sum()
        pen = hardware_penalty(om_s, self.lim1, self.lim2, self.mu1, self.mu2)
        return rec + pen, rec, pen

    def step(self, x_true: torch.Tensor, smaps: torch.Tensor):
        self.opt.zero_grad(set_to_none=False)
        total, rec, pen = self.loss(x_true, smaps)
        total.backward()
        self.opt.step()
        return float(total.detach()), float(rec.detach()), float(pen.detach())
