"""Off-resonance (field inhomogeneity) model of Sec. II-H.

Test infrastructure only (see the package docstring).

Exact system matrix: a_ij = exp(-i omega_i . r_j) exp(-i w_j t_i), with w_j
the field map at voxel j (rad/s) and t_i the readout time of sample i (s).
The fast approximation the paper considers has the form
  E_f = sum_l diag(b_l) A(omega) diag(c_l),   b_l in C^M, c_l in C^N,
and its Jacobians follow by replacing A with E_f: b and c do not depend on
omega, so every omega-derivative of E_f is a sum over l of the NUFFT
Jacobian sandwiched between the same diagonals.  With coil maps the model is
E = sum_l diag(b_l) (I_C kron A) diag(c_l) S.

The paper does not fix how b and c are chosen (it cites time-segmentation
approximations); the reading used here is linear-interpolation time
segmentation: L segment times tau_l spread uniformly over [min t, max t],
c_lj = exp(-i w_j tau_l), and b_il the linear interpolation weights of t_i
between its two neighbouring tau_l (so sum_l b_il = 1).

Gradient conventions are those of ``ndft`` (upstream g = dL/dRe + i dL/dIm).
"""
from __future__ import annotations

import numpy as np

from . import ndft


def _flat_coords(N):
    N = tuple(int(n) for n in N)
    r = np.stack(np.meshgrid(*[np.arange(n) - n // 2 for n in N], indexing="ij"), -1)
    return r.reshape(-1, len(N)).astype(np.float64)


def exact_forward(omega, t, w, x, N, rows: int = 256):
    """y_i = sum_j x_j exp(-i (omega_i . r_j + w_j t_i)) for one image x [*N]
    (direct sum, FP64, in blocks of rows)."""
    om = np.asarray(omega, dtype=np.float64).reshape(-1, len(N))
    t = np.asarray(t, dtype=np.float64).reshape(-1)
    wf = np.asarray(w, dtype=np.float64).reshape(-1)
    xf = np.asarray(x, dtype=np.complex128).reshape(-1)
    r = _flat_coords(N)
    y = np.empty(om.shape[0], dtype=np.complex128)
    for i0 in range(0, om.shape[0], rows):
        ph = om[i0:i0 + rows] @ r.T + t[i0:i0 + rows, None] * wf[None, :]
        y[i0:i0 + rows] = np.exp(-1j * ph) @ xf
    return y


def exact_adjoint(omega, t, w, y, N, rows: int = 256):
    """x_j = sum_i y_i exp(+i (omega_i . r_j + w_j t_i)) (direct sum, FP64)."""
    om = np.asarray(omega, dtype=np.float64).reshape(-1, len(N))
    t = np.asarray(t, dtype=np.float64).reshape(-1)
    wf = np.asarray(w, dtype=np.float64).reshape(-1)
    yf = np.asarray(y, dtype=np.complex128).reshape(-1)
    r = _flat_coords(N)
    x = np.zeros(r.shape[0], dtype=np.complex128)
    for i0 in range(0, om.shape[0], rows):
        ph = om[i0:i0 + rows] @ r.T + t[i0:i0 + rows, None] * wf[None, :]
        x += yf[i0:i0 + rows] @ np.exp(1j * ph)
    return x.reshape(tuple(int(n) for n in N))


def time_segments(t, w, L: int):
    """Linear-interpolation time segmentation: (b [L, M], c [L, *N]) with
    E_f = sum_l diag(b_l) A diag(c_l) approximating the exact model."""
    t = np.asarray(t, dtype=np.float64).reshape(-1)
    w = np.asarray(w, dtype=np.float64)
    M = t.shape[0]
    t0, t1 = float(t.min()), float(t.max())
    if L == 1 or t1 == t0:
        tau = np.full(L, 0.5 * (t0 + t1))
        b = np.zeros((L, M), dtype=np.complex128)
        b[0] = 1.0
    else:
        tau = t0 + (t1 - t0) * np.arange(L) / (L - 1)
        b = np.zeros((L, M), dtype=np.complex128)
        for i in range(M):
            pos = (t[i] - t0) / (t1 - t0) * (L - 1)
            lo = min(int(np.floor(pos)), L - 2)
            frac = pos - lo
            b[lo, i] = 1.0 - frac
            b[lo + 1, i] = frac
    c = np.stack([np.exp(-1j * w * tau[l]) for l in range(L)])
    return b, c


def _maps(c, smaps, N):
    """Per (l, coil) image-domain factor c_l s_c, [L, C, *N]."""
    c = np.asarray(c, dtype=np.complex128)
    if smaps is None:
        return c[:, None]
    return c[:, None] * np.asarray(smaps, dtype=np.complex128)[None]


def seg_forward(omega, b, c, x, N, smaps=None):
    """y[b, k] = sum_l b_l (.) A(c_l s_k x_b); x [B, *N] -> [B, C, M]."""
    N = tuple(int(n) for n in N)
    x = np.asarray(x, dtype=np.complex128).reshape((-1,) + N)
    mp = _maps(c, smaps, N)
    L, C = mp.shape[:2]
    bb = np.asarray(b, dtype=np.complex128)
    out = np.zeros((x.shape[0], C, np.asarray(omega).shape[0]), dtype=np.complex128)
    for l in range(L):
        for k in range(C):
            out[:, k] += bb[l][None] * ndft.forward(omega, mp[l, k][None] * x, N)
    return out


def seg_adjoint(omega, b, c, y, N, smaps=None):
    """x_b = sum_{l,k} conj(c_l s_k) (.) A^H(conj(b_l) (.) y[b, k])."""
    N = tuple(int(n) for n in N)
    mp = _maps(c, smaps, N)
    L, C = mp.shape[:2]
    bb = np.asarray(b, dtype=np.complex128)
    y = np.asarray(y, dtype=np.complex128).reshape(-1, C, np.asarray(omega).shape[0])
    out = np.zeros((y.shape[0],) + N, dtype=np.complex128)
    for l in range(L):
        for k in range(C):
            out += np.conj(mp[l, k])[None] * ndft.adjoint(omega, np.conj(bb[l])[None] * y[:, k], N)
    return out


def seg_jac_omega_fwd(omega, b, c, x, g, N, smaps=None):
    """dL/domega for y = E_f x (with coil maps) and upstream g [B, C, M]:
    sum_{b,k,l} Im{ b_l (.) A(c_l s_k x_b (.) r^[d]) (.) conj(g_{b,k}) }."""
    N = tuple(int(n) for n in N)
    x = np.asarray(x, dtype=np.complex128).reshape((-1,) + N)
    mp = _maps(c, smaps, N)
    L, C = mp.shape[:2]
    bb = np.asarray(b, dtype=np.complex128)
    g = np.asarray(g, dtype=np.complex128).reshape(x.shape[0], C, -1)
    D = len(N)
    out = np.zeros((g.shape[2], D))
    for d in range(D):
        for l in range(L):
            for k in range(C):
                z = bb[l][None] * ndft.forward(omega, mp[l, k][None] * x, N, wdim=d)
                out[:, d] += np.sum(np.imag(z * np.conj(g[:, k])), axis=0)
    return out


def seg_jac_omega_adj(omega, b, c, y, g, N, smaps=None):
    """dL/domega for x = E_f^H y and upstream g [B, *N].  The term
    conj(c_l s_k) A^H(conj(b_l) y_k) has upstream c_l s_k g for its A^H
    output and data conj(b_l) y_k, so by the adjoint-operator rule
    (eq. (e,A'y)) it contributes Im{ A(c_l s_k g (.) r^[d]) (.) b_l conj(y_k) }."""
    N = tuple(int(n) for n in N)
    mp = _maps(c, smaps, N)
    L, C = mp.shape[:2]
    bb = np.asarray(b, dtype=np.complex128)
    g = np.asarray(g, dtype=np.complex128).reshape((-1,) + N)
    y = np.asarray(y, dtype=np.complex128).reshape(g.shape[0], C, -1)
    D = len(N)
    out = np.zeros((y.shape[2], D))
    for d in range(D):
        for l in range(L):
            for k in range(C):
                z = ndft.forward(omega, mp[l, k][None] * g, N, wdim=d)
                out[:, d] += np.sum(np.imag(z * bb[l][None] * np.conj(y[:, k])), axis=0)
    return out
