"""Off-resonance model (Sec. II-H) on the GPU against the FP64 oracle.

The segmented operator E_f = sum_l diag(b_l) A diag(c_l) (with coil maps)
is checked with random complex b and c against the oracle's definition at
the NUFFT tolerances (2e-5 forward/adjoint, 1e-4 omega-gradients): it is a
sum of L NUFFTs with weights of modulus ~1, so the errors of its terms add
without amplification.  The library's time segmentation is compared with
the oracle's (b to float rounding, c to 1e-6), and the GPU operator built
from it approximates the exact off-resonance operator as well as the FP64
segmented operator does (its error is the segmentation's, ~1e-2 at L = 8,
falling as 1/L^2).
"""
import sys

import numpy as np
import pytest
import torch

from oracle import field as fref
from oracle import ndft
from paper_2111_02912_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL = 2e-5
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


def _case(N, B, C, L, seed):
    D = len(N)
    if D == 2:
        om = W.radial_2d(24, 2 * max(N), jitter=np.pi / max(N), seed=seed)
    elif D == 1:
        om = W.uniform_random(500, 1, seed=seed)
    else:
        om = W.kooshball_3d(48, 2 * max(N))
    om = om.astype(np.float32)
    M = om.shape[0]
    g = W.rng(seed + 1)
    b = ((g.standard_normal((L, M)) + 1j * g.standard_normal((L, M))) / np.sqrt(2 * L)).astype(np.complex64)
    c = np.exp(1j * g.uniform(-np.pi, np.pi, (L,) + tuple(N))).astype(np.complex64)
    smaps = W.sense_maps(C, N).astype(np.complex64) if C > 1 else None
    x = W.complex_normal((B,) + tuple(N), seed + 2).astype(np.complex64)
    return om, b, c, smaps, x


CASES = [((48, 40), 2, 3, 4), ((300,), 2, 1, 3), ((12, 10, 14), 1, 2, 3), ((37, 29), 1, 1, 6)]


@pytest.mark.parametrize("N,B,C,L", CASES)
def test_segmented_operator_matches_oracle(N, B, C, L, dev):
    from paper_2111_02912_amd.nufft import KbNufft
    _say(f"field N={N} B={B} C={C} L={L}")
    om, b, c, smaps, x = _case(N, B, C, L, 7101)
    M = om.shape[0]
    plan = KbNufft(N, device=dev)
    plan.set_points(_f(om, dev))
    bt, ct = _c(b, dev), _c(c, dev)
    st = _c(smaps, dev) if smaps is not None else None
    y = plan.field_forward(_c(x, dev), bt, ct, st)
    v = W.complex_normal((B, C, M), 7103).astype(np.complex64)
    xa = plan.field_adjoint(_c(v, dev), bt, ct, st)
    dom = plan.field_jac_omega_fwd(_c(x, dev), _c(v, dev), bt, ct, st)
    h = W.complex_normal((B,) + tuple(N), 7104).astype(np.complex64)
    dom_a = plan.field_jac_omega_adj(_c(v, dev), _c(h, dev), bt, ct, st)
    ef = ndft.rel_l2(_np(y), fref.seg_forward(om, b, c, x, N, smaps))
    ea = ndft.rel_l2(_np(xa), fref.seg_adjoint(om, b, c, v, N, smaps))
    ej = ndft.rel_l2(_np(dom), fref.seg_jac_omega_fwd(om, b, c, x, v, N, smaps))
    eja = ndft.rel_l2(_np(dom_a), fref.seg_jac_omega_adj(om, b, c, v, h, N, smaps))
    _say(f"  fwd {ef:.2e} adj {ea:.2e} jac_fwd {ej:.2e} jac_adj {eja:.2e}")
    assert ef < TOL and ea < TOL and ej < TOL_JAC and eja < TOL_JAC


def test_one_flat_segment_equals_the_plain_calls(dev):
    """L = 1, b = 1, c = 1: the field calls reduce to the plain ones bit for bit."""
    from paper_2111_02912_amd.nufft import KbNufft
    N = (40, 36)
    om, _, _, smaps, x = _case(N, 2, 3, 1, 7201)
    M = om.shape[0]
    plan = KbNufft(N, device=dev)
    plan.set_points(_f(om, dev))
    st = _c(smaps, dev)
    b1 = torch.ones((1, M), dtype=torch.complex64, device=dev)
    c1 = torch.ones((1,) + N, dtype=torch.complex64, device=dev)
    xt = _c(x, dev)
    g = _c(W.complex_normal((2, 3, M), 7202), dev)
    assert torch.equal(plan.field_forward(xt, b1, c1, st), plan.forward(xt, st))
    assert torch.equal(plan.field_adjoint(g, b1, c1, st), plan.adjoint(g, st))
    assert torch.equal(plan.field_jac_omega_fwd(xt, g, b1, c1, st), plan.jac_omega_fwd(xt, g, st))


def test_image_chunks_under_a_small_workspace_cap(dev):
    """A cap that holds the expanded k-space of one image at a time gives the
    same results as one pass (forward bit for bit; sums to 1e-6)."""
    from paper_2111_02912_amd.nufft import KbNufft
    N, B, C, L = (32, 28), 3, 2, 4
    om, b, c, smaps, x = _case(N, B, C, L, 7301)
    M = om.shape[0]
    p1 = KbNufft(N, device=dev)
    p2 = KbNufft(N, device=dev, max_workspace=L * C * M * 8 + 1024)
    outs = []
    v = _c(W.complex_normal((B, C, M), 7302), dev)
    for p in (p1, p2):
        p.set_points(_f(om, dev))
        args = (_c(b, dev), _c(c, dev))
        outs.append((_np(p.field_forward(_c(x, dev), *args, _c(smaps, dev))),
                     _np(p.field_adjoint(v, *args, _c(smaps, dev))),
                     _np(p.field_jac_omega_fwd(_c(x, dev), v, *args, _c(smaps, dev)))))
    assert np.array_equal(outs[0][0], outs[1][0])
    assert ndft.rel_l2(outs[1][1], outs[0][1]) < 1e-6
    assert ndft.rel_l2(outs[1][2], outs[0][2]) < 1e-6


def test_time_segmentation_and_exact_model(dev):
    from paper_2111_02912_amd.nufft import KbNufft
    N = (40, 40)
    om = W.spiral_2d(4, 400).astype(np.float32)
    t = W.readout_times(4, 400, dwell=20e-6)   # 8 ms readouts
    w = W.field_map(N, peak_hz=60.0, seed=7401)
    x = W.complex_normal(N, 7402).astype(np.complex64)
    plan = KbNufft(N, device=dev)
    plan.set_points(_f(om, dev))
    exact = fref.exact_forward(om, t, w, x, N)
    errs = {}
    for L in (4, 8):
        b, c = plan.field_segments(_f(t, dev), _f(w, dev), L)
        b_ex, c_ex = fref.time_segments(t.astype(np.float64), w.astype(np.float64), L)
        assert np.abs(_np(b) - b_ex).max() < 1e-6
        assert np.abs(_np(c) - c_ex).max() < 1e-6
        y = _np(plan.field_forward(_c(x[None], dev), b, c))[0, 0]
        e_gpu = ndft.rel_l2(y, exact)
        e_ref = ndft.rel_l2(fref.seg_forward(om, b_ex, c_ex, x[None], N)[0, 0], exact)
        _say(f"  L={L}: segmented vs exact: gpu {e_gpu:.3e}, fp64 {e_ref:.3e}")
        assert abs(e_gpu - e_ref) <= 0.02 * e_ref + 2e-5
        errs[L] = e_gpu
    assert errs[8] < errs[4] / 3


def test_field_autograd_matches_oracle(dev):
    from paper_2111_02912_amd.autograd import nufft_field, nufft_field_adjoint
    from paper_2111_02912_amd.nufft import KbNufft
    N, B, C, L = (36, 32), 2, 2, 3
    om, b, c, smaps, x = _case(N, B, C, L, 7501)
    M = om.shape[0]
    yt = (0.5 * W.complex_normal((B, C, M), 7502) * np.sqrt(np.prod(N))).astype(np.complex64)
    plan = KbNufft(N, device=dev)
    xt = _c(x, dev).requires_grad_(True)
    omt = _f(om, dev).requires_grad_(True)
    bt, ct, st = _c(b, dev), _c(c, dev), _c(smaps, dev)
    loss = (nufft_field(xt, omt, plan, bt, ct, st) - _c(yt, dev)).abs().pow(2).sum()
    loss.backward()
    gk = 2.0 * (fref.seg_forward(om, b, c, x, N, smaps) - yt)
    ex = ndft.rel_l2(_np(xt.grad), fref.seg_adjoint(om, b, c, gk, N, smaps))
    eo = ndft.rel_l2(_np(omt.grad), fref.seg_jac_omega_fwd(om, b, c, x, gk, N, smaps))
    # adjoint operator: L = sum |E_f^H y - x|^2
    yv = _c(yt, dev).requires_grad_(True)
    om2 = _f(om, dev).requires_grad_(True)
    loss2 = (nufft_field_adjoint(yv, om2, plan, bt, ct, st) - _c(x, dev)).abs().pow(2).sum()
    loss2.backward()
    gi = 2.0 * (fref.seg_adjoint(om, b, c, yt, N, smaps) - x)
    ey = ndft.rel_l2(_np(yv.grad), fref.seg_forward(om, b, c, gi, N, smaps))
    eo2 = ndft.rel_l2(_np(om2.grad), fref.seg_jac_omega_adj(om, b, c, yt, gi, N, smaps))
    _say(f"  field autograd: dx {ex:.2e} domega {eo:.2e}; adjoint op: dy {ey:.2e} domega {eo2:.2e}")
    assert ex < TOL_JAC and eo < TOL_JAC and ey < TOL_JAC and eo2 < TOL_JAC


def test_bad_arguments_rejected(dev):
    from paper_2111_02912_amd import _lib
    from paper_2111_02912_amd.nufft import KbNufft, _ptr, _stream
    N = (16, 16)
    plan = KbNufft(N, device=dev)
    om = _f(W.uniform_random(100, 2, 7601), dev)
    plan.set_points(om)
    x = torch.zeros((1,) + N, dtype=torch.complex64, device=dev)
    y = torch.zeros((1, 1, 100), dtype=torch.complex64, device=dev)
    c = torch.ones((2,) + N, dtype=torch.complex64, device=dev)
    b = torch.ones((2, 100), dtype=torch.complex64, device=dev)
    L_ = _lib.lib()
    s = _stream(dev)
    assert L_.kbn_field_forward(plan._h, 1, 1, 0, _ptr(x), None, _ptr(b), _ptr(c), _ptr(y), s) == \
        _lib.KBN_ERR_INVALID_ARG
    assert L_.kbn_field_forward(plan._h, 1, 1, 2, _ptr(x), None, None, _ptr(c), _ptr(y), s) == \
        _lib.KBN_ERR_INVALID_ARG
    assert L_.kbn_field_segments(100, _ptr(om), 1.0, 0.0, 256, _ptr(om), 2, _ptr(b), _ptr(c), s) == \
        _lib.KBN_ERR_INVALID_ARG
    with pytest.raises(TypeError):
        plan.field_forward(x, b[:, :50], c)
