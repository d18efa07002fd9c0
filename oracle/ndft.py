"""Exact FP64 NUDFT and its closed-form Jacobian-vector products.

Test infrastructure only (see the package docstring).

Operator (Sec. II-B, eq. (e,ndft)):  a_ij = exp(-i omega_i . r_j), with
r_j = j - floor(N/2) per axis.  The C library ``libndft.so`` evaluates the
sums; this module only marshals arrays and applies the closed forms:

  forward-op omega-gradient (Sec. II-C eq. (e,Ax) with the JVP rule
  (e,jac,Ax,v) of Sec. III):
      dL/domega[m, d] = sum_{b,c} Im{ [A(s_c x_b r^[d])]_m conj(g_{b,c,m}) }
  adjoint-op omega-gradient (Sec. II-D eq. (e,A'y)):
      dL/domega[m, d] = sum_{b,c} Im{ [A(s_c g_b r^[d])]_m conj(y_{b,c,m}) }
  x-gradients (linear part): A^H g (forward op), A g (adjoint op).

Gradient convention: ``g`` is PyTorch's gradient of a real loss with respect
to a complex tensor, dL/dRe + i dL/dIm, i.e. twice the Wirtinger derivative
dL/dz* of Sec. II-A.  With that reading the JVP rule (e,jac,Ax,v) returns the
true real derivative (a factor-2 reading of the paper's v, pinned by finite
differences in the tests).
"""
from __future__ import annotations

import ctypes

import numpy as np

from . import _build

_lib = None


def lib():
    global _lib
    if _lib is None:
        _lib = ctypes.CDLL(_build.build())
        i64p = ctypes.POINTER(ctypes.c_int64)
        dp = ctypes.POINTER(ctypes.c_double)
        for fn in (_lib.ndft_forward, _lib.ndft_adjoint):
            fn.restype = ctypes.c_int
            fn.argtypes = [ctypes.c_int, i64p, ctypes.c_int64, dp, ctypes.c_int, dp,
                           ctypes.c_int, i64p, ctypes.c_int64, dp]
        _lib.ndft_forward_sparse.restype = ctypes.c_int
        _lib.ndft_forward_sparse.argtypes = [ctypes.c_int, i64p, ctypes.c_int64, dp, ctypes.c_int,
                                             i64p, ctypes.c_int64, dp, dp]
        _lib.ndft_num_threads.restype = ctypes.c_int
    return _lib


def num_threads() -> int:
    return int(lib().ndft_num_threads())


def _c128(a) -> np.ndarray:
    return np.ascontiguousarray(np.asarray(a), dtype=np.complex128)


def _ptr(a, t):
    return a.ctypes.data_as(ctypes.POINTER(t))


def coords(N):
    """Per-axis voxel-centre coordinates r^[d] = j - floor(N_d/2)."""
    return [np.arange(n, dtype=np.float64) - (n // 2) for n in N]


def forward(omega, x, N, wdim: int = -1, rows=None) -> np.ndarray:
    """y = A(omega) (x (.) r^[wdim]) for every leading channel of x.

    x: [..., *N] complex; returns [..., M] (or [..., len(rows)]) complex128.
    """
    N = tuple(int(n) for n in N)
    D = len(N)
    om = np.ascontiguousarray(omega, dtype=np.float64).reshape(-1, D)
    M = om.shape[0]
    x = _c128(x)
    lead = x.shape[: x.ndim - D]
    nch = int(np.prod(lead)) if lead else 1
    xv = x.reshape(nch, -1)
    Na = np.array(N, dtype=np.int64)
    if rows is not None:
        rows = np.ascontiguousarray(rows, dtype=np.int64)
        R = rows.shape[0]
    else:
        R = M
    y = np.empty((nch, R), dtype=np.complex128)
    if nch and R:
        rc = lib().ndft_forward(D, _ptr(Na, ctypes.c_int64), M, _ptr(om, ctypes.c_double), nch,
                                _ptr(xv.view(np.float64), ctypes.c_double), wdim,
                                _ptr(rows, ctypes.c_int64) if rows is not None else None,
                                R, _ptr(y.view(np.float64), ctypes.c_double))
        assert rc == 0
    return y.reshape(lead + (R,))


def adjoint(omega, y, N, wdim: int = -1, pix=None) -> np.ndarray:
    """x = r^[wdim] (.) A(omega)^H y for every leading channel of y.

    y: [..., M] complex; returns [..., *N] (or [..., len(pix)]) complex128.
    """
    N = tuple(int(n) for n in N)
    D = len(N)
    om = np.ascontiguousarray(omega, dtype=np.float64).reshape(-1, D)
    M = om.shape[0]
    y = _c128(y)
    lead = y.shape[:-1]
    nch = int(np.prod(lead)) if lead else 1
    yv = y.reshape(nch, M)
    Na = np.array(N, dtype=np.int64)
    if pix is not None:
        pix = np.ascontiguousarray(pix, dtype=np.int64)
        P = pix.shape[0]
        oshape = lead + (P,)
    else:
        P = int(np.prod(N))
        oshape = lead + N
    x = np.empty((nch, P), dtype=np.complex128)
    if nch and P:
        rc = lib().ndft_adjoint(D, _ptr(Na, ctypes.c_int64), M, _ptr(om, ctypes.c_double), nch,
                                _ptr(yv.view(np.float64), ctypes.c_double), wdim,
                                _ptr(pix, ctypes.c_int64) if pix is not None else None,
                                P, _ptr(x.view(np.float64), ctypes.c_double))
        assert rc == 0
    return x.reshape(oshape)


def forward_sparse(omega, vals, pix, N) -> np.ndarray:
    """y = A(omega) x for an image x that is zero except x[pix[k]] = vals[..., k].

    The sum of eq. (e,ndft) over the listed voxels only (flat row-major
    indices, no repeats), for problems whose dense sum is too long.
    vals: [..., P] complex; returns [..., M] complex128.
    """
    N = tuple(int(n) for n in N)
    D = len(N)
    om = np.ascontiguousarray(omega, dtype=np.float64).reshape(-1, D)
    M = om.shape[0]
    vals = _c128(vals)
    lead = vals.shape[:-1]
    nch = int(np.prod(lead)) if lead else 1
    pix = np.ascontiguousarray(pix, dtype=np.int64)
    P = pix.shape[0]
    assert vals.shape[-1] == P and np.unique(pix).size == P
    vv = np.ascontiguousarray(vals.reshape(nch, P))
    Na = np.array(N, dtype=np.int64)
    y = np.empty((nch, M), dtype=np.complex128)
    if nch and M:
        rc = lib().ndft_forward_sparse(D, _ptr(Na, ctypes.c_int64), M, _ptr(om, ctypes.c_double), nch,
                                       _ptr(pix, ctypes.c_int64), P,
                                       _ptr(vv.view(np.float64), ctypes.c_double),
                                       _ptr(y.view(np.float64), ctypes.c_double))
        assert rc == 0
    return y.reshape(lead + (M,))


# ---------------------------------------------------------------------------
# SENSE model E = (I_C kron A) S (Sec. II-G)
# ---------------------------------------------------------------------------

def _coil_images(x, smaps, N):
    """[B, *N] images times [C, *N] maps -> [B, C, *N] (no maps: C = 1)."""
    x = _c128(x).reshape((-1,) + tuple(N))
    if smaps is None:
        return x[:, None]
    s = _c128(smaps).reshape((-1,) + tuple(N))
    return x[:, None] * s[None]


def sense_forward(omega, x, N, smaps=None, rows=None) -> np.ndarray:
    """y[b, c] = A (s_c (.) x_b); returns [B, C, M]."""
    return forward(omega, _coil_images(x, smaps, N), N, rows=rows)


def sense_adjoint(omega, y, N, smaps=None) -> np.ndarray:
    """x_b = sum_c conj(s_c) (.) A^H y[b, c]; y: [B, C, M]; returns [B, *N]."""
    y = _c128(y)
    B, C = y.shape[0], y.shape[1]
    xc = adjoint(omega, y, N)  # [B, C, *N]
    if smaps is None:
        return xc[:, 0]
    s = _c128(smaps).reshape((C,) + tuple(N))
    return np.sum(np.conj(s)[None] * xc, axis=1)


def jac_omega_fwd(omega, x, g, N, smaps=None, rows=None) -> np.ndarray:
    """Gradient of a real loss w.r.t. omega through y = E(omega) x.

    Implements eq. (e,Ax) with the JVP rule (e,jac,Ax,v):
    dL/domega^[d] = Re{ conj(-i A(s_c x_b (.) r^[d])) (.) g }, summed over
    images b and coils c.  x: [B, *N]; g: [B, C, M]; returns [M, D] (or
    [len(rows), D]).
    """
    N = tuple(int(n) for n in N)
    D = len(N)
    xs = _coil_images(x, smaps, N)
    g = _c128(g).reshape(xs.shape[0], xs.shape[1], -1)
    if rows is not None:
        g = g[:, :, np.asarray(rows)]
    out = []
    for d in range(D):
        z = forward(omega, xs, N, wdim=d, rows=rows)  # A(s_c x_b r^[d])
        jz = -1j * z                                    # diagonal of the Jacobian
        out.append(np.real(np.conj(jz) * g).sum(axis=(0, 1)))
    return np.stack(out, axis=-1)


def jac_omega_adj(omega, y, g, N, smaps=None, rows=None) -> np.ndarray:
    """Gradient of a real loss w.r.t. omega through x = E(omega)^H y.

    From eq. (e,A'y): d x_hat / d omega^[d] = i diag(r^[d]) A^H diag(y); its
    transpose applied to the upstream image gradient g gives
    dL/domega^[d]_l = sum_{b,c} Im{ [A(s_c g_b (.) r^[d])]_l conj(y_{b,c,l}) }.
    y: [B, C, M]; g: [B, *N]; returns [M, D].
    """
    N = tuple(int(n) for n in N)
    D = len(N)
    gs = _coil_images(g, smaps, N)
    y = _c128(y).reshape(gs.shape[0], gs.shape[1], -1)
    if rows is not None:
        y = y[:, :, np.asarray(rows)]
    out = []
    for d in range(D):
        w = forward(omega, gs, N, wdim=d, rows=rows)
        out.append(np.real(1j * y * np.conj(w)).sum(axis=(0, 1)))
    return np.stack(out, axis=-1)


def jac_x_fwd(omega, g, N, smaps=None) -> np.ndarray:
    """Gradient w.r.t. x through y = E x: E^H g (dA x / dx = A, Sec. II-C)."""
    return sense_adjoint(omega, g, N, smaps)


def jac_x_adj(omega, g, N, smaps=None) -> np.ndarray:
    """Gradient w.r.t. y through x = E^H y: E g (dA^H y / dy = A^H, Sec. II-D)."""
    return sense_forward(omega, g, N, smaps)


def rel_l2(a, b) -> float:
    """||a - b||_2 / ||b||_2 over the whole tensor."""
    a = np.asarray(a)
    b = np.asarray(b)
    nb = np.linalg.norm(b.ravel())
    return float(np.linalg.norm((a - b).ravel()) / (nb if nb > 0 else 1.0))


# ---------------------------------------------------------------------------
# Gram and regularised-inverse operators (Sec. II-E, II-F)
# ---------------------------------------------------------------------------

def gram_vjp(omega, x, g, N, smaps=None):
    """Gradients of a real loss through z = E^H E x (E = SENSE model).

    With the JVP rule (e,jac,Ax,v) applied to both factors of the Gram
    operator (Sec. II-E: the Jacobian of A'A x w.r.t. omega^[d] has one
    term from A and one from A'):
      dL/domega[m, d] = Im{ [E(g r^[d])]_m conj([E x]_m) }
                      + Im{ [E(x r^[d])]_m conj([E g]_m) }   (summed over coils)
      dL/dx           = E^H E g   (the Gram operator is Hermitian)
    x, g: [B, *N]; returns (domega [M, D], dx [B, *N]).
    """
    N = tuple(int(n) for n in N)
    ex = sense_forward(omega, x, N, smaps)
    eg = sense_forward(omega, g, N, smaps)
    dom = jac_omega_fwd(omega, g, ex, N, smaps) + jac_omega_fwd(omega, x, eg, N, smaps)
    dx = sense_adjoint(omega, eg, N, smaps)
    return dom, dx


def gram(omega, x, N, smaps=None):
    """z = E^H E x for images x [B, *N]."""
    N = tuple(int(n) for n in N)
    return sense_adjoint(omega, sense_forward(omega, x, N, smaps), N, smaps)


def gram_sparse(omega, vals, pix, N, smaps=None, out_pix=None) -> np.ndarray:
    """z = E^H E x at the voxels out_pix, for one image x that is zero except
    x[pix[k]] = vals[k] (vals: [P]).  Returns [len(out_pix)] complex128.

    E x = A(s_c (.) x) is summed over the listed voxels only; the adjoint is
    evaluated at the requested voxels only (Sec. II-E operator, SENSE form
    of Sec. II-G)."""
    N = tuple(int(n) for n in N)
    pix = np.asarray(pix, dtype=np.int64)
    out_pix = np.asarray(out_pix, dtype=np.int64)
    vals = _c128(vals).reshape(-1)
    if smaps is None:
        sv = vals[None]
    else:
        s = _c128(smaps).reshape(_c128(smaps).shape[0], -1)
        sv = s[:, pix] * vals[None]                   # [C, P]
    y = forward_sparse(omega, sv, pix, N)            # [C, M]
    xc = adjoint(omega, y, N, pix=out_pix)            # [C, Q]
    if smaps is None:
        return xc[0]
    return np.sum(np.conj(s[:, out_pix]) * xc, axis=0)
