"""FP64 CG-SENSE reconstruction with the exact NUDFT.

Test infrastructure only (see the package docstring).

Sec. IV-B reconstructs x_K = (E'E + lambda T'T)^{-1} E'y by conjugate
gradients; with T = I this is CG-SENSE, with T a finite-difference operator
it is QPLS.  The paper does not fix the finite differences' boundary; the
reading here is the non-circular first difference along each image axis,
(T_d x)_j = x_{j + e_d} - x_j for j_d < N_d - 1, stacked over d.  E = (I_C kron A) S is the SENSE
model of Sec. II-G, applied here by the exact NUDFT of ``ndft``.  The solver
is the plain conjugate-gradient method of the reference the paper cites for
the residual norm (Shewchuk), started from x0 = 0 and run for a fixed
number of iterations; the reported residual is ||r|| / ||b|| with the
recursively updated residual r.
"""
from __future__ import annotations

import numpy as np

from . import ndft


REGS = ("identity", "finite_diff")


def fd_forward(v, N):
    """T v: the first differences of the image v [*N] along each axis
    (list of D arrays, axis d one shorter)."""
    v = np.asarray(v).reshape(tuple(int(n) for n in N))
    return [np.diff(v, axis=d) for d in range(v.ndim)]


def fd_adjoint(us, N):
    """T^H u for u = [u_0, .., u_{D-1}] shaped like fd_forward's output:
    (D_d^T u)_j = u_{j - e_d} - u_j with u taken as zero outside its range."""
    N = tuple(int(n) for n in N)
    out = np.zeros(N, dtype=np.result_type(*[np.asarray(u) for u in us], np.complex128))
    for d, u in enumerate(us):
        pad = [(0, 0)] * len(N)
        pad[d] = (1, 1)
        out -= np.diff(np.pad(u, pad), axis=d)
    return out


def reg_normal(v, N, reg: str):
    """T^H T v for the regulariser `reg` ("identity" or "finite_diff")."""
    if reg == "identity":
        return np.asarray(v)
    if reg == "finite_diff":
        return fd_adjoint(fd_forward(v, N), N)
    raise ValueError(f"unknown regulariser {reg!r}")


def normal_op(omega, N, smaps, lam, reg: str = "identity"):
    """v -> (E^H E + lam T^H T) v on one image [*N] (FP64)."""
    N = tuple(int(n) for n in N)

    def H(v):
        y = ndft.sense_forward(omega, v.reshape((1,) + N), N, smaps)
        return ndft.sense_adjoint(omega, y, N, smaps)[0] + lam * reg_normal(v.reshape(N), N, reg)
    return H


def cg_sense(omega, y, N, smaps=None, lam: float = 1e-3, iters: int = 10, reg: str = "identity"):
    """Solve (E^H E + lam T^H T) x = E^H y by `iters` CG steps from x = 0.

    y: [C, M] k-space of one image; smaps [C, *N] or None (C = 1).
    Returns (x [*N] complex128, ||r|| / ||b||).
    """
    N = tuple(int(n) for n in N)
    y = np.asarray(y, dtype=np.complex128).reshape(1, -1, np.asarray(omega).shape[0])
    H = normal_op(omega, N, smaps, lam, reg)
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
