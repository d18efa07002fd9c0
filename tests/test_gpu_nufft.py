"""GPU parity: the HIP path through the C ABI against the FP64 oracle.

Tolerances (relative L2 over the whole output tensor):
  * forward / adjoint vs the exact NUDFT:            2e-5
  * omega-Jacobians / x-gradients vs the exact forms: 1e-4
  * forward / adjoint vs the FP64 three-step NUFFT with the same window,
    grid and taps (isolates GPU arithmetic from the NUFFT approximation):
    2e-6 (FP32 storage, FFT and accumulation give a few 1e-7)
  * index pass (cells, fractions, order, tile offsets): bit-exact.
"""
import math
import sys

import numpy as np
import pytest
import torch

from oracle import ndft, nufft_ref, points_ref
from paper_2111_02912_amd import workloads as W

pytestmark = pytest.mark.gpu

TOL_NUFFT = 2e-5
TOL_JAC = 1e-4
TOL_STEPS = 2e-6


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda", 0)


def _plan(N, dev, **kw):
    from paper_2111_02912_amd.nufft import KbNufft
    return KbNufft(N, device=dev, **kw)


def _c(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.complex64)).to(dev)


def _f(a, dev):
    return torch.from_numpy(np.ascontiguousarray(a, dtype=np.float32)).to(dev)


def _np(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


ADVERSARIAL_2D = np.array([
    [0.0, 0.0], [-np.pi, -np.pi], [np.pi, np.pi], [np.float32(np.pi) - 1e-6, -1e-30],
    [3.0 * np.pi, -5.0 * np.pi], [1e2, -7.5e1], [-0.0, 2 * np.pi / 128 * 5],
    [np.nextafter(np.float32(np.pi), np.float32(0)), np.nextafter(np.float32(-np.pi), np.float32(0))],
], dtype=np.float32)


@pytest.mark.parametrize("N,tile", [((64, 64), None), ((45, 37), (8, 12)), ((300,), None),
                                    ((12, 10, 14), (8, 8, 8))])
def test_index_pass_bit_exact(N, tile, dev):
    D = len(N)
    _say(f"index pass N={N} tile={tile}")
    parts = [W.uniform_random(3000, D, seed=101, lo=-4.0, hi=4.0)]
    if D == 2:
        parts += [W.radial_2d(32, 128), ADVERSARIAL_2D]
    om = np.concatenate(parts).astype(np.float32)
    p = _plan(N, dev, tile=tile)
    p.set_points(_f(om, dev))
    got = p.get_points()
    cell, frac, bad = points_ref.cells(om, p.K)
    assert not bad.any()
    tid, nt = points_ref.tiles(cell, p.K, p.tile, bad)
    assert nt == p.ntiles
    perm, off = points_ref.tile_order(tid, nt)
    assert np.array_equal(_np(got["order"]), perm)
    assert np.array_equal(_np(got["offsets"]), off)
    assert np.array_equal(_np(got["cell"]), cell[perm].T)
    assert np.array_equal(_np(got["frac"]).view(np.uint32), frac[perm].T.copy().view(np.uint32))
    assert p.check_error() == 0


def test_nonfinite_points_are_flagged(dev):
    _say("non-finite omega")
    N = (32, 32)
    om = W.uniform_random(200, 2, seed=7)
    om[[3, 50, 199]] = [[np.nan, 0.0], [0.0, np.inf], [1e30, 1.0]]
    p = _plan(N, dev)
    p.set_points(_f(om, dev))
    got = p.get_points()
    cell, frac, bad = points_ref.cells(om, p.K)
    tid, nt = points_ref.tiles(cell, p.K, p.tile, bad)
    perm, off = points_ref.tile_order(tid, nt)
    assert np.array_equal(_np(got["order"]), perm)
    assert np.array_equal(_np(got["offsets"]), off)
    x = W.complex_normal(N, 8)
    y = _np(p.forward(_c(x, dev)))[0, 0]
    assert np.isnan(y[[3, 50, 199]]).all()
    good = np.setdiff1d(np.arange(200), [3, 50, 199])
    assert np.isfinite(y[good]).all()
    assert p.check_error() == -5
    assert p.check_error() == 0  # the flag is cleared once reported


def test_index_pass_stream_ordering(dev):
    """The index pass runs on the plan's own stream: omega may be overwritten
    on the caller's stream right after kbn_set_points (the pass has read it
    by then), a forward call issued at once waits for the pass before its
    gather, and a second set_points that grows the point buffers waits for
    the first pass before freeing them."""
    _say("index pass on its own stream")
    N = (96, 80)
    x = _c(W.complex_normal((2,) + N, 31), dev)
    # above the size from which the pass runs on the plan's own stream
    om1 = W.uniform_random(12000, 2, seed=32)
    om2 = W.uniform_random(30000, 2, seed=33)
    ref = _plan(N, dev)
    ref.set_points(_f(om1, dev))
    y1 = ref.forward(x)
    ref.check_error()
    p = _plan(N, dev)
    for _ in range(3):
        t = _f(om1, dev)
        p.set_points(t)
        t.fill_(float("nan"))  # same stream, right after the call
        y = p.forward(x)
        assert torch.equal(y, y1)
        assert p.check_error() == 0
    # grow: the second pass's new buffers replace the first's while it may run
    p.set_points(_f(om1, dev))
    p.set_points(_f(om2, dev))
    # a small set on the caller's stream right after a large one on the plan's
    p.set_points(_f(om2[:500], dev))
    ref.set_points(_f(om2[:500], dev))
    assert torch.equal(p.forward(x), ref.forward(x))
    p.set_points(_f(om2, dev))
    y2 = p.forward(x)
    ref.set_points(_f(om2, dev))
    assert torch.equal(y2, ref.forward(x))
    got = p.get_points()
    cell, frac, bad = points_ref.cells(om2, p.K)
    tid, nt = points_ref.tiles(cell, p.K, p.tile, bad)
    perm, off = points_ref.tile_order(tid, nt)
    assert np.array_equal(_np(got["order"]), perm)


def test_timing_selected_classes(dev):
    """kbn_timing_select limits the timing events to the chosen classes."""
    _say("timing of selected kernel classes")
    N = (64, 48)
    p = _plan(N, dev)
    p.set_points(_f(W.uniform_random(3000, 2, seed=41), dev))
    x = _c(W.complex_normal((2,) + N, 42), dev)
    p.timing(True, classes=["fft_mid_fwd", "gather"])
    y = p.forward(x)
    p.adjoint(y)
    p.timing(False)
    got = {k: n for k, (n, ms) in p.timing_read().items() if n}
    assert set(got) == {"fft_mid_fwd", "gather"}
    p.timing(True)
    p.forward(x)
    p.adjoint(y)
    p.timing(False)
    got = {k for k, (n, ms) in p.timing_read().items() if n}
    assert {"fft_first", "fft_mid_fwd", "gather", "spread", "fft_mid_inv", "fft_last_adj"} <= got


def _case(N, M_kind, seed):
    D = len(N)
    if M_kind == "radial":
        om = W.radial_2d(32, 128)
    else:
        om = W.uniform_random(M_kind, D, seed=seed)
    return om


CASES = [
    ((64, 64), "radial"),        # the paper-shaped small case: 32 spokes x 128 samples
    ((45, 37), 1500),            # odd sizes, K = 90 x 75 (radices 2, 3, 5), ragged tiles
    ((96,), 700),                # 1D
    ((20, 18, 14), 900),         # 3D, K = 40 x 36 x 28 (radix 7)
]


@pytest.mark.parametrize("N,kind", CASES)
def test_forward_adjoint_parity(N, kind, dev):
    _say(f"forward/adjoint N={N} points={kind}")
    om = _case(N, kind, 11)
    M = om.shape[0]
    B = 2
    x = W.complex_normal((B,) + N, 12)
    y = W.complex_normal((B, 1, M), 13)
    p = _plan(N, dev)
    p.set_points(_f(om, dev))
    yg = _np(p.forward(_c(x, dev)))
    xg = _np(p.adjoint(_c(y, dev)))
    exact_f = ndft.forward(om, x, N)[:, None, :]
    exact_a = ndft.adjoint(om, y[:, 0], N)
    assert ndft.rel_l2(yg, exact_f) < TOL_NUFFT
    assert ndft.rel_l2(xg, exact_a) < TOL_NUFFT
    ref = nufft_ref.Params(N, 2.0, 6)
    assert ndft.rel_l2(yg[:, 0], nufft_ref.forward(ref, om, x)) < TOL_STEPS
    assert ndft.rel_l2(xg, nufft_ref.adjoint(ref, om, y[:, 0])) < TOL_STEPS


@pytest.mark.parametrize("N,kind", CASES[:2] + CASES[3:])
def test_sense_and_jacobians(N, kind, dev):
    _say(f"SENSE + Jacobians N={N} points={kind}")
    om = _case(N, kind, 21)
    M = om.shape[0]
    B, C = 2, 3
    x = W.complex_normal((B,) + N, 22)
    smaps = W.sense_maps(C, N)
    g = W.complex_normal((B, C, M), 23)
    gi = W.complex_normal((B,) + N, 24)
    p = _plan(N, dev)
    p.set_points(_f(om, dev))
    xs, ss, gs, gis = _c(x, dev), _c(smaps, dev), _c(g, dev), _c(gi, dev)
    y = _np(p.forward(xs, ss))
    assert ndft.rel_l2(y, ndft.sense_forward(om, x, N, smaps)) < TOL_NUFFT
    xa = _np(p.adjoint(gs, ss))
    assert ndft.rel_l2(xa, ndft.sense_adjoint(om, g, N, smaps)) < TOL_NUFFT
    dom = _np(p.jac_omega_fwd(xs, gs, ss))
    assert ndft.rel_l2(dom, ndft.jac_omega_fwd(om, x, g, N, smaps)) < TOL_JAC
    doma = _np(p.jac_omega_adj(gs, gis, ss))
    assert ndft.rel_l2(doma, ndft.jac_omega_adj(om, g, gi, N, smaps)) < TOL_JAC
    # accumulate adds onto the existing gradient (repeated: results must not vary)
    for rep in range(3):
        acc = p.jac_omega_fwd(xs, gs, ss)
        a1 = _np(acc)
        p.jac_omega_adj(gs, gis, ss, out=acc, accumulate=True)
        a2 = _np(acc)
        err = ndft.rel_l2(a2, dom + doma)
        if err >= 1e-6:
            bad = np.nonzero(np.abs(a2 - dom - doma).max(axis=1) > 1e-4 * np.abs(dom).max())[0]
            pts = p.get_points()
            order = _np(pts["order"])
            off = _np(pts["offsets"])
            pos = np.empty(M, np.int64)
            pos[order] = np.arange(M)
            _say(f"rep {rep}: fwd-part err {ndft.rel_l2(a1, dom):.3e}, adj-part err "
                 f"{ndft.rel_l2(a2 - a1, doma):.3e}; {len(bad)} bad rows, sorted positions "
                 f"{np.sort(pos[bad])[:16]}, tiles {np.unique(np.searchsorted(off, pos[bad], 'right') - 1)[:16]}")
        assert err < 1e-6
    # x-gradients: E^H g and E g
    from paper_2111_02912_amd._lib import KBN_OP_ADJOINT, KBN_OP_FORWARD
    assert ndft.rel_l2(_np(p.jac_x(KBN_OP_FORWARD, gs, ss)), ndft.jac_x_fwd(om, g, N, smaps)) < TOL_JAC
    assert ndft.rel_l2(_np(p.jac_x(KBN_OP_ADJOINT, gis, ss)), ndft.jac_x_adj(om, gi, N, smaps)) < TOL_JAC


def test_empty_points(dev):
    _say("empty point set")
    N = (32, 40)
    p = _plan(N, dev)
    p.set_points(torch.empty((0, 2), dtype=torch.float32, device=dev))
    x = _c(W.complex_normal((2,) + N, 5), dev)
    y = p.forward(x)
    assert y.shape == (2, 1, 0)
    xa = _np(p.adjoint(torch.empty((2, 1, 0), dtype=torch.complex64, device=dev)))
    assert xa.shape == (2,) + N and not np.any(xa)
    d = p.jac_omega_fwd(x, torch.empty((2, 1, 0), dtype=torch.complex64, device=dev))
    assert d.shape == (0, 2)


def test_chunked_batches_match_single_pass(dev):
    """A workspace cap forces channel chunks; results must not change."""
    _say("chunked batches")
    N = (48, 40)
    om = W.uniform_random(2000, 2, seed=31)
    x = W.complex_normal((5,) + N, 32)
    g = W.complex_normal((5, 1, 2000), 33)
    p1 = _plan(N, dev)
    gsz = p1.K[0] * p1.K[1] * 8
    p2 = _plan(N, dev, max_workspace=2 * gsz * 2 * 2)  # two images x two buffers x D weights
    for p in (p1, p2):
        p.set_points(_f(om, dev))
    a = [_np(p.forward(_c(x, dev))) for p in (p1, p2)]
    b = [_np(p.adjoint(_c(g, dev))) for p in (p1, p2)]
    c = [_np(p.jac_omega_fwd(_c(x, dev), _c(g, dev))) for p in (p1, p2)]
    assert np.array_equal(a[0], a[1])
    assert ndft.rel_l2(b[1], b[0]) < 1e-6
    assert ndft.rel_l2(c[1], c[0]) < 1e-6


FWD_JAC_CASES = [
    ((64, 64), "radial", True),      # K = 128 x 128: r^[0] channel derived in the axis-0 pass
    ((99, 80), 1700, True),          # odd N_0, K = 200 x 160, ragged tiles
    ((45, 37), 1500, False),         # K = 90 x 75: generic FFT lengths, two separate calls
    ((96,), 700, False),             # 1D
    ((20, 18, 14), 900, False),      # 3D
]


@pytest.mark.parametrize("N,kind,fused", FWD_JAC_CASES)
def test_forward_jac_omega(N, kind, fused, dev):
    """kbn_forward_jac_omega: y bit-equal to kbn_forward, domega equal to
    kbn_jac_omega_fwd up to float32 rounding where the r^[0] channel is
    derived (bit-equal where the call runs the two operations), both
    against the exact forms; accumulate adds; a workspace cap that splits
    the batch into chunks changes nothing."""
    _say(f"forward + omega-Jacobian N={N} points={kind} fused={fused}")
    om = _case(N, kind, 51)
    M = om.shape[0]
    B, C = 2, 3
    x = W.complex_normal((B,) + N, 52)
    smaps = W.sense_maps(C, N)
    g = W.complex_normal((B, C, M), 53)
    p = _plan(N, dev)
    p.set_points(_f(om, dev))
    xs, ss, gs = _c(x, dev), _c(smaps, dev), _c(g, dev)
    y_ref = _np(p.forward(xs, ss))
    d_ref = _np(p.jac_omega_fwd(xs, gs, ss))
    yt, dt = p.forward_jac_omega(xs, gs, ss)
    y, d = _np(yt), _np(dt)
    assert np.array_equal(y, y_ref)
    err = ndft.rel_l2(d, d_ref)
    _say(f"  domega vs kbn_jac_omega_fwd: {err:.2e}")
    if fused:
        assert err < TOL_STEPS
    else:
        assert np.array_equal(d, d_ref)
    assert ndft.rel_l2(y, ndft.sense_forward(om, x, N, smaps)) < TOL_NUFFT
    assert ndft.rel_l2(d, ndft.jac_omega_fwd(om, x, g, N, smaps)) < TOL_JAC
    _, acc = p.forward_jac_omega(xs, gs, ss, out=dt.clone(), accumulate=True)
    assert ndft.rel_l2(_np(acc), 2 * d) < 1e-6
    gsz = int(np.prod(p.K)) * 8
    pc = _plan(N, dev, max_workspace=2 * gsz * (len(N) + 1) * 2)  # two image-coil pairs per chunk
    pc.set_points(_f(om, dev))
    yc, dc = pc.forward_jac_omega(xs, gs, ss)
    assert np.array_equal(_np(yc), y)
    assert ndft.rel_l2(_np(dc), d) < 1e-6


def test_forward_jac_omega_persistent_twins(dev):
    """256 x 256 images (K = 512), 4 images x 3 coils: the persistent axis-0
    pass then meets each derived r^[0] tile right after its unweighted source
    in one full block of workgroup strides (values scaled in registers) and
    loads it again in the shorter last block.  y bit-equal to kbn_forward;
    domega against kbn_jac_omega_fwd and, on sampled rows, the exact
    gradient."""
    N = (256, 256)
    M = 3000
    B, C = 4, 3
    _say(f"forward + omega-Jacobian, persistent column pass N={N} M={M} B={B} C={C}")
    om = W.uniform_random(M, 2, seed=61)
    x = W.complex_normal((B,) + N, 62)
    smaps = W.sense_maps(C, N)
    g = W.complex_normal((B, C, M), 63)
    p = _plan(N, dev)
    p.set_points(_f(om, dev))
    xs, ss, gs = _c(x, dev), _c(smaps, dev), _c(g, dev)
    y_ref = _np(p.forward(xs, ss))
    d_ref = _np(p.jac_omega_fwd(xs, gs, ss))
    yt, dt = p.forward_jac_omega(xs, gs, ss)
    assert np.array_equal(_np(yt), y_ref)
    d = _np(dt)
    err = ndft.rel_l2(d, d_ref)
    _say(f"  domega vs kbn_jac_omega_fwd: {err:.2e}")
    assert err < TOL_STEPS
    rows = np.random.default_rng(64).choice(M, 48, replace=False)
    ex = ndft.jac_omega_fwd(om, x, g, N, smaps, rows=rows)
    assert ndft.rel_l2(d[rows], ex) < TOL_JAC


def test_chunked_jacobian_last_chunk_with_more_groups(dev):
    """omega-Jacobian in image chunks of 7 and 6 where the smaller last chunk
    splits into more channel groups than the first (about 2048 / blocks = 6
    groups at most): the per-group gradient buffer must hold the larger
    count.  Compared with the single-pass result and the exact gradient on
    sampled rows."""
    N = (48, 48)
    M = 85000
    _say(f"chunked jacobian N={N} M={M} B=13")
    om = W.uniform_random(M, 2, seed=41)
    x = W.complex_normal((13,) + N, 42)
    g = W.complex_normal((13, 1, M), 43)
    p1 = _plan(N, dev)
    per_img = p1.K[0] * p1.K[1] * 8 * 2 * 2  # two grids x D weight channels
    p2 = _plan(N, dev, max_workspace=7 * per_img + 1024)
    outs = []
    for p in (p1, p2):
        p.set_points(_f(om, dev))
        outs.append(_np(p.jac_omega_fwd(_c(x, dev), _c(g, dev))))
    assert ndft.rel_l2(outs[1], outs[0]) < 1e-6
    rows = np.sort(W.rng(44).choice(M, 64, replace=False))
    ex = ndft.jac_omega_fwd(om, x, g, N, rows=rows)
    assert ndft.rel_l2(outs[1][rows], ex) < 1e-4


def test_workspace_cap_splits_coils(dev):
    """When one image's coils do not fit under the workspace cap, the plan
    runs one image at a time in runs of coils (forward: runs of 2, 2, 1 of
    5 coils; Jacobian and adjoint: one coil at a time).  Forward values are
    per channel and must not change at all; the adjoint and the
    omega-gradient add the runs in a different order (1e-6).  Both are also
    compared with the exact NUDFT, and the workspace stays under the cap
    (plus the omega-gradient's per-group partials)."""
    N, B, C = (48, 40), 2, 5
    _say(f"coil-chunked plan N={N} B={B} C={C}")
    om = W.radial_2d(24, 96, jitter=np.pi / 48, seed=35).astype(np.float32)
    M = om.shape[0]
    x = W.complex_normal((B,) + N, 36)
    g = W.complex_normal((B, C, M), 37)
    smaps = _c(W.sense_maps(C, N), dev)
    p1 = _plan(N, dev)
    cap = 300_000
    p2 = _plan(N, dev, max_workspace=cap)
    for p in (p1, p2):
        p.set_points(_f(om, dev))
    a = [_np(p.forward(_c(x, dev), smaps)) for p in (p1, p2)]
    b = [_np(p.adjoint(_c(g, dev), smaps)) for p in (p1, p2)]
    c = [_np(p.jac_omega_fwd(_c(x, dev), _c(g, dev), smaps)) for p in (p1, p2)]
    assert np.array_equal(a[0], a[1])
    assert ndft.rel_l2(b[1], b[0]) < 1e-6
    assert ndft.rel_l2(c[1], c[0]) < 1e-6
    sm = W.sense_maps(C, N)
    assert ndft.rel_l2(a[1], ndft.sense_forward(om, x, N, sm)) < TOL_NUFFT
    assert ndft.rel_l2(b[1], ndft.sense_adjoint(om, g, N, sm)) < TOL_NUFFT
    assert ndft.rel_l2(c[1], ndft.jac_omega_fwd(om, x, g, N, sm)) < TOL_JAC
    ws = p2.info()["workspace_bytes"]
    _say(f"  workspace {ws} bytes under cap {cap}")
    assert ws <= cap + 64 * M * 2 * 4


def test_throughput_shape_sampled(dev):
    """256x256, 64 spokes x 512 samples + jitter, sigma 2, J 6: sampled rows/pixels."""
    _say("256x256 M=32768 sampled parity")
    N, om, x = W.throughput_case(batch=2)
    M = om.shape[0]
    p = _plan(N, dev)
    p.set_points(_f(om, dev))
    y = _np(p.forward(_c(x, dev)))[:, 0]
    rows = np.random.default_rng(5).choice(M, 400, replace=False)
    exact = ndft.forward(om, x, N, rows=rows)
    assert ndft.rel_l2(y[:, rows], exact) < TOL_NUFFT
    g = W.complex_normal((2, 1, M), 6)
    xa = _np(p.adjoint(_c(g, dev))).reshape(2, -1)
    pix = np.random.default_rng(6).choice(N[0] * N[1], 300, replace=False)
    exact_a = ndft.adjoint(om, g[:, 0], N, pix=pix)
    assert ndft.rel_l2(xa[:, pix], exact_a) < TOL_NUFFT
    dom = _np(p.jac_omega_fwd(_c(x, dev), _c(g, dev)))
    exact_j = ndft.jac_omega_fwd(om, x, g, N, rows=rows)
    assert ndft.rel_l2(dom[rows], exact_j) < TOL_JAC


def test_bench_configuration_sampled(dev):
    """The benchmarked step at its full size and launch shape: 256 images of
    256x256, M = 32768 (64 spokes x 512 samples with jitter): forward rows
    and adjoint pixels of images in different channel groups, and the
    omega-gradient (summed over all 256 images) on sampled rows."""
    B = 256
    _say(f"bench configuration B={B}")
    N, om, x = W.throughput_case(batch=B)
    M = om.shape[0]
    g = W.complex_normal((B, 1, M), 2101)
    p = _plan(N, dev)
    xt, gt = _c(x, dev), _c(g, dev)
    p.set_points(_f(om, dev))
    y = p.forward(xt)
    dom = p.jac_omega_fwd(xt, gt)
    xa = p.adjoint(gt)
    imgs = [0, 43, 130, 255]
    rows = np.sort(W.rng(2102).choice(M, 128, replace=False))
    pix = np.sort(W.rng(2103).choice(N[0] * N[1], 96, replace=False))
    y_ex = ndft.forward(om, x[imgs], N, rows=rows)
    e_f = ndft.rel_l2(_np(y)[imgs, 0][:, rows], y_ex)
    xa_ex = ndft.adjoint(om, g[imgs, 0], N, pix=pix)
    e_a = ndft.rel_l2(_np(xa).reshape(B, -1)[imgs][:, pix], xa_ex)
    dom_ex = ndft.jac_omega_fwd(om, x, g, N, rows=rows)
    e_j = ndft.rel_l2(_np(dom)[rows], dom_ex)
    _say(f"  fwd {e_f:.2e} adj {e_a:.2e} jac {e_j:.2e}")
    assert e_f < TOL_NUFFT and e_a < TOL_NUFFT and e_j < TOL_JAC


@pytest.mark.parametrize("N", [(64, 96), (160, 128), (48, 40, 64), (256, 130), (80, 200), (240, 160),
                               (200, 64), (40, 100, 80), (216, 225), (243, 250), (270, 288), (300, 324), (360, 375),
                               (225, 216), (375, 360), (216, 24, 250), (196, 224), (252, 294), (336, 343),
                               (378, 196), (100, 400), (400, 100), (135, 144), (150, 162), (180, 144),
                               (320, 384), (384, 320)])
def test_specialised_fft_matches_generic(N, dev, monkeypatch):
    """The compile-time specialised FFT passes and the generic ones agree, and
    both match the oracle (K = 128, 192, 320, 256, 96->generic, 160, 400,
    480, 200->generic ...; 432, 450, 486, 500, 540, 576, 600, 648, 720, 750
    on either axis, 432 x 48 x 500 in 3D; with radix 7: 392, 448, 504, 588,
    672, 686, 756; 200 and 800; 270, 288, 300, 324, 360; 640 and 768 with
    16 columns per column-pass workgroup)."""
    _say(f"specialised vs generic FFT N={N}")
    D = len(N)
    om = W.uniform_random(2500, D, seed=91)
    M = om.shape[0]
    x = W.complex_normal((2,) + N, 92)
    g = W.complex_normal((2, 1, M), 93)
    outs = []
    for generic in ("0", "1"):
        monkeypatch.setenv("KBN_GENERIC_FFT", generic)
        p = _plan(N, dev)
        p.set_points(_f(om, dev))
        outs.append((_np(p.forward(_c(x, dev))), _np(p.adjoint(_c(g, dev))),
                     _np(p.jac_omega_fwd(_c(x, dev), _c(g, dev)))))
    for a, b in zip(*outs):
        assert ndft.rel_l2(a, b) < 2e-6
    ref = nufft_ref.Params(N, 2.0, 6)
    assert ndft.rel_l2(outs[0][0][:, 0], nufft_ref.forward(ref, om, x)) < TOL_STEPS
    assert ndft.rel_l2(outs[0][1], nufft_ref.adjoint(ref, om, g[:, 0])) < TOL_STEPS


def test_grid_sizes_without_a_near_tile_divisor(dev):
    """N = 302 x 362 gives K = 625 x 729 (powers of 5 and 3): no tile edge
    near the preferred one divides K or leaves a last tile of at least J
    cells below it, so the tile search must also look upward."""
    N = (302, 362)
    _say(f"awkward grid N={N}")
    om = W.uniform_random(3000, 2, seed=9101)
    x = W.complex_normal((1,) + N, 9102)
    smaps = W.sense_maps(2, N).astype(np.complex64)
    p = _plan(N, dev)
    assert p.K == (625, 729)
    p.set_points(_f(om, dev))
    y = p.forward(_c(x, dev), _c(smaps, dev))
    g = W.complex_normal((1, 2, om.shape[0]), 9103)
    xa = p.adjoint(_c(g, dev), _c(smaps, dev))
    e_f = ndft.rel_l2(_np(y), ndft.sense_forward(om, x, N, smaps))
    e_a = ndft.rel_l2(_np(xa), ndft.sense_adjoint(om, g, N, smaps))
    _say(f"  fwd {e_f:.2e} adj {e_a:.2e}")
    assert e_f < TOL_NUFFT and e_a < TOL_NUFFT


def test_largest_grid_and_clustered_samples(dev):
    """The largest supported grid (512 x 512 images, K = 1024 per axis) with
    5000 samples at one location among uniform ones: hot tiles are split
    into many gather subproblems and spread work items."""
    N = (512, 512)
    _say(f"largest grid N={N} with clustered samples")
    hot = np.tile(np.array([[0.3, -1.1]], dtype=np.float32), (5000, 1))
    om = np.concatenate([W.uniform_random(3000, 2, seed=9301), hot]).astype(np.float32)
    x = W.complex_normal((1,) + N, 9302)
    g = W.complex_normal((1, 1, om.shape[0]), 9303)
    p = _plan(N, dev)
    assert p.K == (1024, 1024)
    p.set_points(_f(om, dev))
    y = _np(p.forward(_c(x, dev)))
    xa = _np(p.adjoint(_c(g, dev)))
    rows = np.concatenate([np.arange(0, 3000, 37), np.arange(3000, 8000, 500)])
    e_f = ndft.rel_l2(y[0, 0, rows], ndft.forward(om, x, N, rows=rows)[0])
    pix = np.sort(W.rng(9304).choice(N[0] * N[1], 200, replace=False))
    e_a = ndft.rel_l2(xa.reshape(-1)[pix], ndft.adjoint(om, g[0, 0], N, pix=pix))
    _say(f"  fwd {e_f:.2e} adj {e_a:.2e}")
    assert e_f < TOL_NUFFT and e_a < TOL_NUFFT


@pytest.mark.parametrize("N,kind,nch", [((256, 256), "radial", 96), ((135, 256), "clustered", 128),
                                         ((192, 192), "uniform", 160)])
def test_wide_channel_spread_matches_narrow_groups(N, kind, nch, dev):
    """2D adjoints of 64 or more channels on 8 x 8 owner tiles, with at least
    4096 (owner tile, 64-channel group) pairs, run the channel-per-lane
    spread; the same channels 32 at a time run the cell-per-lane spread.
    Both add the same weights in the same list order, so they agree bit for
    bit, and both match the NUDFT.  Cases: radial (hot centre tiles split
    into several work items), clustered samples on a grid whose last owner
    tile row is 6 cells tall (K = 270 x 512), and a channel count that
    leaves the last group of 64 half empty."""
    _say(f"wide-channel spread N={N} {kind} nch={nch}")
    if kind == "radial":
        om = W.radial_2d(32, 2 * max(N), jitter=np.pi / max(N), seed=9501)
    elif kind == "clustered":
        hot = W.uniform_random(1500, 2, seed=9502, lo=-0.2, hi=0.25)
        om = np.concatenate([W.uniform_random(1000, 2, seed=9503), hot])
    else:
        om = W.uniform_random(3000, 2, seed=9504)
    om = om.astype(np.float32)
    M = om.shape[0]
    g = W.complex_normal((nch, 1, M), 9505)
    p = _plan(N, dev, spread_tile=8)
    p.set_points(_f(om, dev))
    wide = _np(p.adjoint(_c(g, dev)))
    narrow = np.concatenate([_np(p.adjoint(_c(g[i:i + 32], dev))) for i in range(0, nch, 32)])
    assert np.array_equal(wide, narrow)
    idx = [0, 37, nch - 1]
    pix = np.sort(W.rng(9506).choice(N[0] * N[1], 300, replace=False))
    e_a = ndft.rel_l2(wide[idx].reshape(3, -1)[:, pix], ndft.adjoint(om, g[idx, 0], N, pix=pix))
    _say(f"  adj {e_a:.2e}")
    assert e_a < TOL_NUFFT


def _clusters(D, centres, each, seed, half=0.06):
    """Small square clusters of samples around the given centres, wrapped
    into [-pi, pi) (clusters at +-pi straddle the grid's wrap-around)."""
    parts = []
    for k, c in enumerate(centres):
        pts = np.asarray(c, np.float64) + W.uniform_random(each, D, seed=seed + k, lo=-half, hi=half)
        parts.append((pts + np.pi) % (2 * np.pi) - np.pi)
    return np.concatenate(parts).astype(np.float32)


@pytest.mark.parametrize("N,each", [((135, 150), 300), ((135, 150), 2600), ((300, 140), 300), ((20, 18, 14), 200)])
def test_sparse_support(N, each, dev):
    """Samples in a few small clusters (most of the oversampled grid outside
    every sample's taps): at the centre, across the +-pi wrap on every axis
    and off-centre; K = 270 x 300 (a partial last 8-row block), 600 x 280
    and 40 x 36 x 28.  A second point set on the same plan (other clusters,
    the grid workspace still holding the first set's values) must give the
    NUDFT as well.  10400 samples take the index pass on the plan's own
    stream, 1200 and 800 on the caller's."""
    D = len(N)
    _say(f"sparse support N={N} clusters of {each}")
    z = [0.0] * D
    sets = [
        [z, [np.pi - 0.02] * D, [-np.pi + 0.01] + [0.7] * (D - 1), [1.3] + [-np.pi + 0.005] * (D - 1)],
        [[-2.0] + [0.4] * (D - 1), [0.9] * D, [np.pi - 0.03] + [-1.1] * (D - 1)],
    ]
    p = _plan(N, dev)
    B = 2
    x = W.complex_normal((B,) + N, 9601)
    pix = np.sort(W.rng(9602).choice(int(np.prod(N)), 400, replace=False))
    for si, centres in enumerate(sets):
        om = _clusters(D, centres, each, 9610 + 10 * si)
        M = om.shape[0]
        g = W.complex_normal((B, 1, M), 9603 + si)
        p.set_points(_f(om, dev))
        xs, gs = _c(x, dev), _c(g, dev)
        yg = _np(p.forward(xs))
        xa = _np(p.adjoint(gs))
        sel = np.sort(W.rng(9604 + si).choice(M, min(M, 600), replace=False))
        e_f = ndft.rel_l2(yg[:, 0, sel], ndft.forward(om[sel], x, N))
        e_a = ndft.rel_l2(xa.reshape(B, -1)[:, pix], ndft.adjoint(om, g[:, 0], N, pix=pix))
        _say(f"  set {si}: M={M} forward {e_f:.2e} adjoint {e_a:.2e}")
        assert e_f < TOL_NUFFT and e_a < TOL_NUFFT
        if M <= 1200:
            gi = W.complex_normal((B,) + N, 9605 + si)
            dom = _np(p.jac_omega_fwd(xs, gs))
            doma = _np(p.jac_omega_adj(gs, _c(gi, dev)))
            e_j = ndft.rel_l2(dom, ndft.jac_omega_fwd(om, x, g, N))
            e_ja = ndft.rel_l2(doma, ndft.jac_omega_adj(om, g, gi, N))
            _say(f"  set {si}: omega-Jacobians {e_j:.2e} {e_ja:.2e}")
            assert e_j < TOL_JAC and e_ja < TOL_JAC


@pytest.mark.parametrize("N,st", [((60, 52), 24), ((20, 22, 18), 10)])
def test_scatter_spread_path(N, st, dev):
    """Owner tiles of more than 512 cells use the scatter spread kernel
    (lanes own (tap, channel) pairs; the path of 1D plans): adjoint and
    adjoint-operator Jacobian against the exact NUDFT, with coil maps."""
    D = len(N)
    _say(f"scatter spread N={N} spread_tile={st}")
    om = W.uniform_random(2500, D, seed=9401)
    C = 3
    smaps = W.sense_maps(C, N).astype(np.complex64)
    y = W.complex_normal((2, C, om.shape[0]), 9402)
    gi = W.complex_normal((2,) + N, 9403)
    p = _plan(N, dev, spread_tile=st)
    p.set_points(_f(om, dev))
    xa = _np(p.adjoint(_c(y, dev), _c(smaps, dev)))
    e_a = ndft.rel_l2(xa, ndft.sense_adjoint(om, y, N, smaps))
    dom = _np(p.jac_omega_adj(_c(y, dev), _c(gi, dev), _c(smaps, dev)))
    e_j = ndft.rel_l2(dom, ndft.jac_omega_adj(om, y, gi, N, smaps))
    _say(f"  adj {e_a:.2e} jac_adj {e_j:.2e}")
    assert e_a < TOL_NUFFT and e_j < TOL_JAC
