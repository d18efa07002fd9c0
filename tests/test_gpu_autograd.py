"""Autograd layers on the GPU against the exact (FP64 NUDFT) gradients.

The loss is the training loss of the SENSE model, L = sum |E(omega) x - y|^2
(forward operator) or L = sum |E(omega)^H y - x|^2 (adjoint operator).
The oracle evaluates the exact gradients from eq. (e,Ax) / (e,A'y) with the
rule (e,jac,Ax,v) in FP64, with g computed exactly as well; tolerance 1e-4
(relative L2).  A finite-difference check of the GPU loss along a random
direction pins the sign and scale independently of the oracle.
"""
import sys

import numpy as np
import pytest
import torch

from oracle import ndft
from paper_2111_02912_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL_JAC = 1e-4


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda", 0)


def _c(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex64)).to(dev)


def _f(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)


def _np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _case(N, B, C, seed):
    D = len(N)
    if D == 2:
        om = W.radial_2d(24, 2 * max(N), jitter=np.pi / max(N), seed=seed)
    elif D == 1:
        om = W.uniform_random(700, 1, seed=seed)
    else:
        om = W.kooshball_3d(64, 2 * max(N))
    om = om.astype(np.float32)
    x = W.complex_normal((B,) + tuple(N), seed + 1).astype(np.complex64)
    smaps = W.sense_maps(C, N).astype(np.complex64) if C > 1 else None
    return om, x, smaps


CASES = [((48, 40), 2, 3), ((300,), 2, 1), ((12, 10, 14), 1, 2)]


@pytest.mark.parametrize("N,B,C", CASES)
def test_forward_op_gradients(N, B, C, dev):
    from paper_2111_02912_amd.autograd import nufft
    from paper_2111_02912_amd.nufft import KbNufft
    _say(f"forward-op autograd N={N} B={B} C={C}")
    om, x, smaps = _case(N, B, C, seed=4101)
    M = om.shape[0]
    yt = (0.5 * W.complex_normal((B, C, M), 4103) * np.sqrt(np.prod(N))).astype(np.complex64)
    plan = KbNufft(N, device=dev)
    xt = _c(x, dev).requires_grad_(True)
    omt = _f(om, dev).requires_grad_(True)
    st = _c(smaps, dev) if smaps is not None else None
    y = nufft(xt, omt, plan, st)
    loss = (y - _c(yt, dev)).abs().pow(2).sum()
    loss.backward()
    y_ex = ndft.sense_forward(om, x, N, smaps)
    g_ex = 2.0 * (y_ex - yt)
    dom_ex = ndft.jac_omega_fwd(om, x, g_ex, N, smaps)
    dx_ex = ndft.jac_x_fwd(om, g_ex, N, smaps)
    e_om = ndft.rel_l2(_np(omt.grad), dom_ex)
    e_x = ndft.rel_l2(_np(xt.grad), dx_ex)
    _say(f"  rel domega {e_om:.2e} dx {e_x:.2e}")
    assert e_om < TOL_JAC and e_x < TOL_JAC


@pytest.mark.parametrize("N,B,C", CASES)
def test_adjoint_op_gradients(N, B, C, dev):
    from paper_2111_02912_amd.autograd import nufft_adjoint
    from paper_2111_02912_amd.nufft import KbNufft
    _say(f"adjoint-op autograd N={N} B={B} C={C}")
    om, _, smaps = _case(N, B, C, seed=4201)
    M = om.shape[0]
    y = W.complex_normal((B, C, M), 4202).astype(np.complex64)
    xt_target = (W.complex_normal((B,) + tuple(N), 4203) * np.sqrt(M)).astype(np.complex64)
    plan = KbNufft(N, device=dev)
    yt = _c(y, dev).requires_grad_(True)
    omt = _f(om, dev).requires_grad_(True)
    st = _c(smaps, dev) if smaps is not None else None
    xh = nufft_adjoint(yt, omt, plan, st)
    loss = (xh - _c(xt_target, dev)).abs().pow(2).sum()
    loss.backward()
    x_ex = ndft.sense_adjoint(om, y, N, smaps)
    g_ex = 2.0 * (x_ex - xt_target)
    dom_ex = ndft.jac_omega_adj(om, y, g_ex, N, smaps)
    dy_ex = ndft.jac_x_adj(om, g_ex, N, smaps)
    e_om = ndft.rel_l2(_np(omt.grad), dom_ex)
    e_y = ndft.rel_l2(_np(yt.grad), dy_ex)
    _say(f"  rel domega {e_om:.2e} dy {e_y:.2e}")
    assert e_om < TOL_JAC and e_y < TOL_JAC


def test_finite_difference_direction(dev):
    """d/dt L(omega + t v) at t = 0 by central differences of the GPU loss
    (accumulated in FP64 on the host) against <grad_omega, v>."""
    from paper_2111_02912_amd.autograd import nufft
    from paper_2111_02912_amd.nufft import KbNufft
    N, B, C = (64, 64), 1, 2
    om, x, smaps = _case(N, B, C, seed=4301)
    M = om.shape[0]
    yt = (0.5 * W.complex_normal((B, C, M), 4302) * 64).astype(np.complex64)
    v = W.rng(4303).standard_normal(om.shape).astype(np.float32)
    plan = KbNufft(N, device=dev)
    st = _c(smaps, dev)
    xt = _c(x, dev)
    omt = _f(om, dev).requires_grad_(True)
    loss = (nufft(xt, omt, plan, st) - _c(yt, dev)).abs().pow(2).sum()
    loss.backward()
    grad = _np(omt.grad).astype(np.float64)
    h = 2e-4
    # the steps actually taken after rounding omega + t v to float32
    om_p = (om + np.float32(h) * v).astype(np.float32)
    om_m = (om - np.float32(h) * v).astype(np.float32)
    step = om_p.astype(np.float64) - om_m.astype(np.float64)
    dir_grad = float(np.sum(grad * step)) / (2 * h)

    def L(o):
        plan.set_points(_f(o, dev))
        y = _np(plan.forward(xt, st)).astype(np.complex128)
        return float(np.sum(np.abs(y - yt) ** 2))

    fd = (L(om_p) - L(om_m)) / (2 * h)
    rel = abs(fd - dir_grad) / abs(fd)
    _say(f"  fd {fd:.6e} autograd {dir_grad:.6e} rel {rel:.2e}")
    assert rel < 2e-3


def test_points_follow_inplace_update(dev):
    """An optimiser step on omega (in place) makes the next call re-sort."""
    from paper_2111_02912_amd.autograd import nufft
    from paper_2111_02912_amd.nufft import KbNufft
    N = (40, 48)
    om, x, _ = _case(N, 1, 1, seed=4401)
    plan = KbNufft(N, device=dev)
    omt = _f(om, dev).requires_grad_(True)
    xt = _c(x, dev)
    opt = torch.optim.SGD([omt], lr=1e-3)
    loss = nufft(xt, omt, plan).abs().pow(2).sum()
    loss.backward()
    opt.step()
    y1 = _np(nufft(xt, omt, plan))
    om1 = _np(omt)
    y_ex = ndft.sense_forward(om1, x, N)
    e = ndft.rel_l2(y1, y_ex)
    _say(f"  after step rel {e:.2e}")
    assert np.abs(om1 - om).max() > 0 and e < 2e-5


def test_map_gradient_rejected(dev):
    from paper_2111_02912_amd.autograd import nufft
    from paper_2111_02912_amd.nufft import KbNufft
    N = (16, 16)
    om, x, smaps = _case(N, 1, 2, seed=4501)
    plan = KbNufft(N, device=dev)
    st = _c(smaps, dev).requires_grad_(True)
    with pytest.raises(NotImplementedError):
        nufft(_c(x, dev), _f(om, dev), plan, st)


def test_sense_training_shape_sampled(dev):
    """320x320, 8 images x 8 coils, 16 x 1280 spiral (M = 20480), loss
    against a seeded random target: domega on a seeded subset of
    rows (each row's gradient depends only on its own residual)."""
    from paper_2111_02912_amd.autograd import nufft
    from paper_2111_02912_amd.nufft import KbNufft
    N, om, x, smaps = W.spiral_sense_case()
    _say(f"sense training shape N={N} M={om.shape[0]} B={x.shape[0]} C={smaps.shape[0]}")
    M = om.shape[0]
    B, C = x.shape[0], smaps.shape[0]
    yt = (0.3 * W.complex_normal((B, C, M), 3002) * 320).astype(np.complex64)
    plan = KbNufft(N, device=dev)
    xt = _c(x, dev).requires_grad_(True)
    omt = _f(om, dev).requires_grad_(True)
    st = _c(smaps, dev)
    loss = (nufft(xt, omt, plan, st) - _c(yt, dev)).abs().pow(2).sum()
    loss.backward()
    rows = np.sort(W.rng(3003).choice(M, 96, replace=False))
    y_ex = ndft.sense_forward(om, x, N, smaps, rows=rows)
    g_ex = np.zeros((B, C, M), dtype=np.complex128)  # only the sampled rows are read
    g_ex[:, :, rows] = 2.0 * (y_ex - yt[:, :, rows])
    dom_ex = ndft.jac_omega_fwd(om, x, g_ex, N, smaps, rows=rows)
    e = ndft.rel_l2(_np(omt.grad)[rows], dom_ex)
    _say(f"  sampled rel domega {e:.2e}")
    assert e < TOL_JAC
    assert np.isfinite(_np(xt.grad)).all()
