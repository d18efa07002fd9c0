"""FP64 Kaiser-Bessel NUFFT, written as the appendix's three steps.

Test infrastructure only (see the package docstring).

The appendix describes the NUFFT as (1) scaling the image by factors s_n,
(2) a zero-padded K-point FFT, and (3) a J-tap interpolation from the K
uniform frequencies to the M sample locations, with coefficients u_j(omega_m)
at offsets k_m + j.  The paper leaves the window to its NUFFT library; the
readings used here (and by the GPU path) are:

  window   psi(t) = I0(beta sqrt(1 - (2t/J)^2)) / I0(beta) for |t| <= J/2,
           beta from the Beatty et al. rule pi sqrt((J/sigma)^2 (sigma-1/2)^2
           - 0.8) (13.8551 for sigma = 2, J = 6);
  scaling  s_n = 1 / psi_hat(r_n / K) per axis, psi_hat the continuous
           Fourier transform of psi (closed form below);
  grid     K = smallest integer >= sigma N whose prime factors are 2, 3, 5, 7;
  taps     with u = omega K / (2 pi): k_start = floor(u - J/2) + 1, taps
           k_start + j for j = 0..J-1, weight psi(u - k_start - j); grid
           indices are taken modulo K (omega is periodic in 2 pi because the
           coordinates r are integers).

numpy's FFT serves as the FFT step.  Spreading (the adjoint's step 3) uses
numpy.add.at; the adjoint is the exact transpose of the forward.
"""
from __future__ import annotations

import itertools
import math

import numpy as np


def kb_beta(J: int, sigma: float) -> float:
    """Beatty et al. shape parameter for a width-J window on a sigma-oversampled grid."""
    return math.pi * math.sqrt((J / sigma) ** 2 * (sigma - 0.5) ** 2 - 0.8)


def grid_size(n: int, sigma: float) -> int:
    """Smallest 7-smooth integer >= sigma * n."""
    k = int(math.ceil(sigma * n - 1e-9))
    while True:
        r = k
        for p in (2, 3, 5, 7):
            while r % p == 0:
                r //= p
        if r == 1:
            return k
        k += 1


def kb_window(t, J: int, beta: float) -> np.ndarray:
    """psi(t), normalised so psi(0) = 1; zero outside |t| <= J/2."""
    t = np.asarray(t, dtype=np.float64)
    a = 1.0 - (2.0 * t / J) ** 2
    out = np.zeros_like(t)
    m = a >= 0.0
    out[m] = np.i0(beta * np.sqrt(a[m])) / np.i0(beta)
    return out


def kb_window_ft(f, J: int, beta: float) -> np.ndarray:
    """Continuous Fourier transform of psi: int psi(t) exp(-2 pi i f t) dt.

    J sinh(sqrt(beta^2 - (pi J f)^2)) / sqrt(beta^2 - (pi J f)^2) / I0(beta),
    continued analytically (sin branch) when pi J |f| > beta.
    """
    f = np.asarray(f, dtype=np.float64)
    z2 = beta * beta - (math.pi * J * f) ** 2
    out = np.empty_like(f)
    pos = z2 > 0
    z = np.sqrt(np.abs(z2))
    out[pos] = np.sinh(z[pos]) / z[pos]
    neg = z2 < 0
    out[neg] = np.sin(z[neg]) / z[neg]
    out[z2 == 0] = 1.0
    return J * out / np.i0(beta)


def scale_factors(n: int, K: int, J: int, beta: float) -> np.ndarray:
    """s_n = 1/psi_hat(r/K) for r = j - floor(n/2), j < n."""
    r = np.arange(n, dtype=np.float64) - (n // 2)
    return 1.0 / kb_window_ft(r / K, J, beta)


class Params:
    """Grid sizes, window and scaling of one NUFFT."""

    def __init__(self, N, sigma: float = 2.0, J: int = 6, K=None, beta=None):
        self.N = tuple(int(n) for n in N)
        self.D = len(self.N)
        self.sigma = float(sigma)
        self.J = int(J)
        self.K = tuple(int(k) for k in K) if K is not None else tuple(
            grid_size(n, sigma) for n in self.N)
        self.beta = float(beta) if beta is not None else kb_beta(self.J, self.sigma)
        self.s = [scale_factors(n, k, self.J, self.beta) for n, k in zip(self.N, self.K)]

    def scaling(self) -> np.ndarray:
        """Full separable scaling array s_n over the image."""
        out = np.ones(self.N)
        for d, sd in enumerate(self.s):
            shape = [1] * self.D
            shape[d] = -1
            out = out * sd.reshape(shape)
        return out


def _taps(p: Params, omega):
    """Per axis: integer tap indices [M, J] (mod K) and weights [M, J]."""
    om = np.asarray(omega, dtype=np.float64).reshape(-1, p.D)
    idx, wts = [], []
    for d in range(p.D):
        K = p.K[d]
        u = om[:, d] * (K / (2.0 * math.pi))
        k0 = np.floor(u - p.J / 2.0) + 1.0
        j = np.arange(p.J, dtype=np.float64)[None, :]
        k = k0[:, None] + j
        wts.append(kb_window(u[:, None] - k, p.J, p.beta))
        idx.append(np.mod(k, K).astype(np.int64))
    return idx, wts


def _pad_indices(p: Params):
    """Grid index of every image sample: r mod K per axis (an open mesh)."""
    out = []
    for d in range(p.D):
        r = np.arange(p.N[d]) - (p.N[d] // 2)
        out.append(np.mod(r, p.K[d]))
    return np.ix_(*out)


def forward(p: Params, omega, x) -> np.ndarray:
    """y ~ A(omega) x for every leading channel; x [..., *N] -> [..., M]."""
    x = np.asarray(x, dtype=np.complex128)
    lead = x.shape[: x.ndim - p.D]
    xs = x.reshape((-1,) + p.N)
    # step 1: scaling factors
    xs = xs * p.scaling()[None]
    # step 2: zero-pad to K and FFT
    grid = np.zeros((xs.shape[0],) + p.K, dtype=np.complex128)
    pad = _pad_indices(p)
    grid[(slice(None),) + pad] = xs
    G = np.fft.fftn(grid, axes=tuple(range(1, p.D + 1)))
    # step 3: J-tap interpolation at the sample locations
    idx, wts = _taps(p, omega)
    M = idx[0].shape[0]
    y = np.zeros((xs.shape[0], M), dtype=np.complex128)
    for js in itertools.product(range(p.J), repeat=p.D):
        w = np.ones(M)
        ind = []
        for d, j in enumerate(js):
            w = w * wts[d][:, j]
            ind.append(idx[d][:, j])
        y += w[None, :] * G[(slice(None),) + tuple(ind)]
    return y.reshape(lead + (M,))


def adjoint(p: Params, omega, y) -> np.ndarray:
    """x ~ A(omega)^H y for every leading channel; y [..., M] -> [..., *N]."""
    y = np.asarray(y, dtype=np.complex128)
    lead = y.shape[:-1]
    ys = y.reshape(-1, y.shape[-1])
    nch, M = ys.shape
    # step 3 transposed: spread onto the K grid
    idx, wts = _taps(p, omega)
    grid = np.zeros((nch,) + p.K, dtype=np.complex128)
    for js in itertools.product(range(p.J), repeat=p.D):
        w = np.ones(M)
        ind = []
        for d, j in enumerate(js):
            w = w * wts[d][:, j]
            ind.append(idx[d][:, j])
        for c in range(nch):
            np.add.at(grid[c], tuple(ind), w * ys[c])
    # step 2 transposed: unnormalised inverse FFT and crop
    H = np.fft.ifftn(grid, axes=tuple(range(1, p.D + 1))) * float(np.prod(p.K))
    pad = _pad_indices(p)
    xs = H[(slice(None),) + pad]
    # step 1 transposed: scaling factors
    xs = xs * p.scaling()[None]
    return xs.reshape(lead + p.N)


def coordinate_weighted(p: Params, x, d: int) -> np.ndarray:
    """x (.) r^[d], the operand of the omega-Jacobians (Sec. II-C, II-D)."""
    r = np.arange(p.N[d], dtype=np.float64) - (p.N[d] // 2)
    shape = [1] * p.D
    shape[d] = -1
    return np.asarray(x) * r.reshape(shape)
