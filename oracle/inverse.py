"""Regularised inverse F^{-1} x, F = E^H E + lambda I, and its gradients.

Test infrastructure only (see the package docstring).

Sec. II-E treats the inverse as solved accurately (so that its Jacobian is
that of the exact inverse, evaluated approximately): with w = F^{-1} g,
  dL/dx     = w                            (F is Hermitian)
  dL/domega = - gram_vjp(x := F^{-1} x, g := w)
The solves here are dense FP64 solves of the normal matrix built from the
exact NUDFT, so this is for small problems only.
"""
from __future__ import annotations

import numpy as np

from . import ndft


def normal_matrix(omega, N, smaps, lam):
    """F = E^H E + lam I as a dense [n, n] complex128 matrix (n = prod N)."""
    N = tuple(int(n) for n in N)
    n = int(np.prod(N))
    eye = np.eye(n, dtype=np.complex128).reshape((n,) + N)
    cols = ndft.gram(omega, eye, N, smaps).reshape(n, n)  # row k = F e_k
    return cols.T + lam * np.eye(n)


def solve(omega, x, N, smaps=None, lam=1e-3):
    """z = F^{-1} x for x [B, *N]."""
    N = tuple(int(n) for n in N)
    F = normal_matrix(omega, N, smaps, lam)
    xb = np.asarray(x, dtype=np.complex128).reshape(-1, F.shape[0])
    return np.linalg.solve(F, xb.T).T.reshape((-1,) + N)


def inverse_vjp(omega, x, g, N, smaps=None, lam=1e-3):
    """(domega [M, D], dx [B, *N]) for z = F^{-1} x and upstream gradient g."""
    N = tuple(int(n) for n in N)
    F = normal_matrix(omega, N, smaps, lam)
    n = F.shape[0]
    z = np.linalg.solve(F, np.asarray(x, dtype=np.complex128).reshape(-1, n).T).T.reshape((-1,) + N)
    w = np.linalg.solve(F, np.asarray(g, dtype=np.complex128).reshape(-1, n).T).T.reshape((-1,) + N)
    dom, _ = ndft.gram_vjp(omega, z, w, N, smaps)
    return -dom, w
