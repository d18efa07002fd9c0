"""Index pass reference: per-point grid cell, fraction, tile and tile order.

Test infrastructure only (see the package docstring).

The appendix places each sample between uniform frequencies via an offset
k_m and J taps k_m + j.  The GPU path derives those taps from the grid cell
that contains u = omega K / (2 pi) and the position inside that cell; this
module states that arithmetic exactly so that the GPU's integer results can
be compared bit for bit:

  s     = float64(K) * (1 / (2 pi))             (FP64, computed once per axis)
  u     = float64(omega) * s                    (one FP64 multiply, no FMA)
  fl    = floor(u)
  frac  = float32(u - fl)                       (u - fl is exact in FP64)
  cell  = fl mod K, in [0, K)                   (integer arithmetic)
  tile  = cell // T per axis; tile id row-major over ceil(K/T) tiles per axis
  order = stable sort of the points by tile id (ties keep input order)

Samples with a non-finite omega or |u| >= 2^40 are flagged, given cell 0,
frac 0 and the extra tile id ntiles, so they sort after all finite points.
"""
from __future__ import annotations

import math

import numpy as np

U_LIMIT = float(2 ** 40)


def axis_scale(K: int) -> float:
    return float(K) * (1.0 / (2.0 * math.pi))


def cells(omega, K):
    """Return (cell [M, D] int32, frac [M, D] float32, bad [M] bool)."""
    om = np.asarray(omega, dtype=np.float32)
    M, D = om.shape
    cell = np.zeros((M, D), dtype=np.int32)
    frac = np.zeros((M, D), dtype=np.float32)
    bad = np.zeros(M, dtype=bool)
    for d in range(D):
        s = axis_scale(K[d])
        u = om[:, d].astype(np.float64) * s
        ok = np.isfinite(u) & (np.abs(u) < U_LIMIT)
        bad |= ~ok
        uu = np.where(ok, u, 0.0)
        fl = np.floor(uu)
        frac[:, d] = (uu - fl).astype(np.float32)
        cell[:, d] = np.mod(fl.astype(np.int64), K[d]).astype(np.int32)
    cell[bad] = 0
    frac[bad] = 0.0
    return cell, frac, bad


def tiles(cell, K, T, bad=None):
    """Row-major tile id of every point; returns (tile [M] int32, ntiles).

    Flagged points (``bad``) get the id ntiles.
    """
    cell = np.asarray(cell)
    D = cell.shape[1]
    nt = [-(-int(K[d]) // int(T[d])) for d in range(D)]
    tid = np.zeros(cell.shape[0], dtype=np.int64)
    for d in range(D):
        tid = tid * nt[d] + cell[:, d] // int(T[d])
    ntiles = int(np.prod(nt))
    if bad is not None:
        tid[np.asarray(bad)] = ntiles
    return tid.astype(np.int32), ntiles


def tile_order(tid, ntiles):
    """Stable order of points by tile id, and offsets [ntiles + 2].

    off[t] is the first sorted position of tile t, off[ntiles] the end of
    the finite points and off[ntiles + 1] = M.
    """
    perm = np.argsort(tid, kind="stable").astype(np.int32)
    counts = np.bincount(tid, minlength=ntiles + 1)
    off = np.zeros(ntiles + 2, dtype=np.int32)
    off[1:] = np.cumsum(counts)
    return perm, off
