"""Per-problem choice of the tile sizes (host-side policy, no arithmetic).

Two tile sizes shape the interpolation kernels: the sorting tile (points are
bucketed by it and the gather stages one tile's grid region per
subproblem) and the spread owner tile (the grid block one spreading work
group accumulates).  Their best values depend on the trajectory's density
and the number of coils, so ``tune_plan`` times a few candidates on the
problem itself (forward + omega-Jacobian + adjoint, one image, all coils)
and keeps the fastest plan.  Results are cached per (shape, M bucket, coils,
trajectory fingerprint) for the life of the process.
"""
from __future__ import annotations

import hashlib
from typing import Dict, Optional, Sequence, Tuple

import torch

from ._lib import KBN_ERR_UNSUPPORTED, KbnError
from .nufft import KbNufft

CANDIDATES = {
    1: [dict(tile=(256,), spread_tile=128), dict(tile=(128,), spread_tile=64)],
    2: [dict(tile=(32, 32), spread_tile=12), dict(tile=(16, 16), spread_tile=12),
        dict(tile=(32, 32), spread_tile=8), dict(tile=(32, 32), spread_tile=16)],
    3: [dict(tile=(8, 8, 8), spread_tile=8), dict(tile=(16, 16, 16), spread_tile=8),
        dict(tile=(8, 8, 8), spread_tile=16)],
}

_cache: Dict[tuple, dict] = {}


def _key(N, omega: torch.Tensor, C: int) -> tuple:
    M = int(omega.shape[0])
    sample = omega[:: max(1, M // 256)].detach().float().cpu().numpy().tobytes()
    return (tuple(N), M.bit_length(), int(C), hashlib.sha1(sample).hexdigest()[:16])


def _time(plan: KbNufft, x, smaps, k, dom, reps: int) -> float:
    ev0 = torch.cuda.Event(enable_timing=True)
    ev1 = torch.cuda.Event(enable_timing=True)
    plan.forward(x, smaps)
    plan.jac_omega_fwd(x, k, smaps, out=dom)
    plan.adjoint(k, smaps)
    ev0.record()
    for _ in range(reps):
        plan.forward(x, smaps)
        plan.jac_omega_fwd(x, k, smaps, out=dom)
        plan.adjoint(k, smaps)
    ev1.record()
    ev1.synchronize()
    return ev0.elapsed_time(ev1) / reps


def tune_plan(N: Sequence[int], omega: torch.Tensor, C: int = 1, x=None, smaps=None, k=None,
              candidates: Optional[list] = None, reps: int = 2, sigma: float = 2.0, J: int = 6
              ) -> Tuple[KbNufft, dict]:
    """Return (plan with points set, {"choice", "ms"}) for the fastest candidate.

    x [1, *N], smaps [C, *N] (or None) and k [1, C, M] are timing inputs;
    random ones are drawn when absent.  Work runs on the current stream.
    """
    N = tuple(int(n) for n in N)
    dev = omega.device
    D = len(N)
    M = int(omega.shape[0])
    key = _key(N, omega, C)
    if key in _cache:
        c = _cache[key]["choice"]
        plan = KbNufft(N, sigma=sigma, J=J, tile=c["tile"], spread_tile=c["spread_tile"], device=dev)
        plan.set_points(omega)
        return plan, _cache[key]
    g = torch.Generator(device="cpu").manual_seed(12345)
    if x is None:
        x = torch.randn((1,) + N, generator=g, dtype=torch.complex64).to(dev)
    if k is None:
        k = torch.randn((1, C, M), generator=g, dtype=torch.complex64).to(dev)
    if smaps is None and C > 1:
        raise ValueError("C > 1 needs coil maps")
    dom = torch.empty((M, D), dtype=torch.float32, device=dev)
    best = None
    results = []
    for cand in (candidates or CANDIDATES[D]):
        try:
            plan = KbNufft(N, sigma=sigma, J=J, tile=cand["tile"], spread_tile=cand["spread_tile"],
                           device=dev)
        except KbnError as e:
            if e.code != KBN_ERR_UNSUPPORTED:  # e.g. too many tiles for this grid: skip
                raise
            continue
        plan.set_points(omega)
        ms = _time(plan, x, smaps, k, dom, reps)
        results.append((cand, ms))
        if best is None or ms < best[1]:
            if best is not None:
                best[2].close()
            best = (cand, ms, plan)
        else:
            plan.close()
    info = {"choice": best[0], "ms": best[1], "tried": results}
    _cache[key] = info
    return best[2], info
