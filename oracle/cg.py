"""FP64 CG-SENSE reconstruction with the exact NUDFT.

Test infrastructure only (see the package docstring).

Sec. IV-B reconstructs x_K = (E'E + lambda T'T)^{-1} E'y by conjugate
gradients; with T = I this is CG-SENSE.  E = (I_C kron A) S is the SENSE
model of Sec. II-F, applied here by the exact NUDFT of ``ndft``.  The solver
is the plain conjugate-gradient method of the reference the paper cites for
the residual norm (Shewchuk), started from x0 = 0 and run for a fixed
number of iterations; the reported residual is ||r|| / ||b|| with the
recursively updated residual r.
"""
from __future__ import annotations

import numpy as np

from . import ndft


def normal_op(omega, N, smaps, lam):
    """v -> (E^H E + lam I) v on one image [*N] (FP64)."""
    N = tuple(int(n) for n in N)

    def H(v):
        y = ndft.sense_forward(omega, v.reshape((1,) + N), N, smaps)
        return ndft.sense_adjoint(omega, y, N, smaps)[0] + lam * v
    return H


def cg_sense(omega, y, N, smaps=None, lam: float = 1e-3, iters: int = 10):
    """Solve (E^H E + lam I) x = E^H y by `iters` CG steps from x = 0.

    y: [C, M] k-space of one image; smaps [C, *N] or None (C = 1).
    Returns (x [*N] complex128, ||r|| / ||b||).
    """
    N = tuple(int(n) for n in N)
    y = np.asarray(y, dtype=np.complex128).reshape(1, -1, np.asarray(omega).shape[0])
    H = normal_op(omega, N, smaps, lam)
    b = ndft.sense_adjoint(omega, y, N, smaps)[0]
    x = np.zeros_like(b)
    r = b.copy()
    p = r.copy()
    rr = np.vdot(r, r).real
    bb = rr
    for _ in range(iters):
        q = H(p)
        pq = np.vdot(p, q).real
        alpha = rr / pq if (pq > 0 and rr > 0) else 0.0
        x = x + alpha * p
        r = r - alpha * q
        rr_new = np.vdot(r, r).real
        beta = rr_new / rr if rr > 0 else 0.0
        rr = rr_new
        p = r + beta * p
    rel = float(np.sqrt(rr / bb)) if bb > 0 else 0.0
    return x, rel
