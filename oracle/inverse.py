"""Regularised inverse F^{-1} x, F = E^H E + lambda T^H T, and its gradients.

Test infrastructure only (see the package docstring).

T is the identity or the finite-difference operator of ``cg`` (T does not
depend on omega, so the gradient formulas are the same for both).
Sec. II-F treats the inverse as solved accurately (so that its Jacobian is
that of the exact inverse, evaluated approximately): with w = F^{-1} g,
  dL/dx     = w                            (F is Hermitian)
  dL/domega = - gram_vjp(x := F^{-1} x, g := w)
The solves here are dense FP64 solves of the normal matrix built from the
exact NUDFT, so this is for small problems only.
"""
from __future__ import annotations

import numpy as np

from . import cg, ndft


def normal_matrix(omega, N, smaps, lam, reg="identity"):
    """F = E^H E + lam T^H T as a dense [n, n] complex128 matrix (n = prod N)."""
    N = tuple(int(n) for n in N)
    n = int(np.prod(N))
    eye = np.eye(n, dtype=np.complex128).reshape((n,) + N)
    cols = ndft.gram(omega, eye, N, smaps).reshape(n, n)  # row k = E^H E e_k
    R = np.stack([cg.reg_normal(eye[k], N, reg).reshape(-1) for k in range(n)])
    return cols.T + lam * R.T


def solve(omega, x, N, smaps=None, lam=1e-3, reg="identity"):
    """z = F^{-1} x for x [B, *N]."""
    N = tuple(int(n) for n in N)
    F = normal_matrix(omega, N, smaps, lam, reg)
    xb = np.asarray(x, dtype=np.complex128).reshape(-1, F.shape[0])
    return np.linalg.solve(F, xb.T).T.reshape((-1,) + N)


def inverse_vjp(omega, x, g, N, smaps=None, lam=1e-3, reg="identity"):
    """(domega [M, D], dx [B, *N]) for z = F^{-1} x and upstream gradient g."""
    N = tuple(int(n) for n in N)
    F = normal_matrix(omega, N, smaps, lam, reg)
    n = F.shape[0]
    z = np.linalg.solve(F, np.asarray(x, dtype=np.complex128).reshape(-1, n).T).T.reshape((-1,) + N)
    w = np.linalg.solve(F, np.asarray(g, dtype=np.complex128).reshape(-1, n).T).T.reshape((-1,) + N)
    dom, _ = ndft.gram_vjp(omega, z, w, N, smaps)
    return -dom, w
