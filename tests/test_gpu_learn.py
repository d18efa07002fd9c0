"""The trajectory-learning loop (Sec. IV-B) on the GPU: every step runs the
forward NUFFT, the adjoint NUFFT and the CG-SENSE inverse layer with their
omega-gradients; a few Adam steps on a small problem must lower the
reconstruction error, keep the penalty zero while the trajectory stays
within the hardware limits, and cut the penalty when the limits are tight."""
import sys

import numpy as np
import pytest
import torch

from paper_2111_02912_amd import workloads as W

pytestmark = pytest.mark.gpu


def _say(msg):
    print(msg, flush=True)
    sys.stdout.flush()


@pytest.fixture(scope="module")
def dev():
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return torch.device("cuda", 0)


def _data(N, B, C, dev):
    x = torch.from_numpy(W.complex_normal((B,) + N, 8801)).to(dev)
    # smooth images: a low-pass copy of the noise (trajectories matter at low frequencies)
    k = torch.fft.fftshift(torch.fft.fft2(x), dim=(-2, -1))
    yy, xx = torch.meshgrid(torch.arange(N[0], device=dev) - N[0] // 2,
                            torch.arange(N[1], device=dev) - N[1] // 2, indexing="ij")
    k = k * (yy ** 2 + xx ** 2 < (N[0] // 6) ** 2)
    x = torch.fft.ifft2(torch.fft.ifftshift(k, dim=(-2, -1))).to(torch.complex64).contiguous()
    smaps = torch.from_numpy(W.sense_maps(C, N)).to(dev)
    return x, smaps


def test_learning_lowers_the_reconstruction_error(dev):
    from paper_2111_02912_amd.learn import TrajectoryLearner
    N, B, C = (48, 48), 2, 2
    x, smaps = _data(N, B, C, dev)
    tl = TrajectoryLearner(N, shots=6, samples=160, knots=10, lam=1e-2, cg_iters=8, lr=2e-3, device=dev)
    hist = [tl.step(x, smaps) for _ in range(12)]
    torch.cuda.synchronize()
    _say("  rec " + " ".join(f"{h[1]:.4g}" for h in hist) + f"  pen {hist[-1][2]:.3g}")
    assert all(np.isfinite(h[0]) for h in hist)
    # Adam at a small step: the error falls at every step, by more than 1% in all
    assert all(b[1] < a[1] for a, b in zip(hist, hist[1:]))
    assert hist[-1][1] < 0.99 * hist[0][1]
    assert tl.coef.grad is not None and torch.isfinite(tl.coef.grad).all()


def test_penalty_pulls_the_trajectory_inside_tight_limits(dev):
    from paper_2111_02912_amd.learn import TrajectoryLearner
    N, B, C = (32, 32), 1, 2
    x, smaps = _data(N, B, C, dev)
    # Adam moves each coefficient by about lr per step; the excess over the
    # limit is half the trajectory's extent (pi), so use a step of 0.05
    tl = TrajectoryLearner(N, shots=4, samples=128, knots=8, lam=1e-2, cg_iters=4, lr=5e-2, device=dev)
    # limits below the radial start's step (2 pi / 128 per sample): the penalty is active
    tl.lim1 = 0.5 * 2 * np.pi / 128
    pens = [tl.step(x, smaps)[2] for _ in range(10)]
    _say("  pen " + " ".join(f"{p:.4g}" for p in pens))
    assert pens[0] > 0 and pens[-1] < 0.8 * pens[0]


def _dense_E64(om, N, smaps):
    """E = (I_C kron A(omega)) S as a dense complex128 matrix [C*M, n] built
    from the definition a_mj = exp(-i omega_m . r_j) (Sec. II-B, II-G)."""
    r = np.stack(np.meshgrid(*[np.arange(n) - n // 2 for n in N], indexing="ij"), -1).reshape(-1, len(N))
    A = torch.exp(-1j * (om @ torch.from_numpy(r.astype(np.float64)).T).to(torch.complex128))
    s = torch.from_numpy(smaps.reshape(smaps.shape[0], -1).astype(np.complex128))
    return torch.cat([A * s[c][None, :] for c in range(s.shape[0])], 0)


def test_learning_gradient_matches_dense_fp64_route(dev):
    """dL/dcoef of one learning step (Sec. IV-B loss: CG-SENSE reconstruction
    error through the inverse layer, plus active gradient and slew
    penalties) against torch FP64 autograd through the dense E(omega) and
    torch.linalg.solve, with the same spline basis and coefficients.  The
    reconstruction term's gradient (forward, adjoint and inverse layers) is
    compared on its own and in the total.

    lam = 200 against a largest eigenvalue of E^H E of about 2.6e3 gives a
    condition number of about 14; 40 CG iterations take the Krylov error far
    below the FP32 floor, so what remains is the NUFFT error amplified by the
    condition number: 14 x 4e-5 (the Gram tolerance) = 5.6e-4, so 1e-3."""
    from paper_2111_02912_amd.learn import TrajectoryLearner, quadratic_bspline_basis
    N, B, C, shots, samples, knots, lam = (12, 10), 2, 4, 4, 40, 8, 200.0
    x_np = W.complex_normal((B,) + N, 8811)
    x = torch.from_numpy(x_np).to(dev)
    smaps_np = W.sense_maps(C, N)
    smaps = torch.from_numpy(smaps_np).to(dev)
    tl = TrajectoryLearner(N, shots=shots, samples=samples, knots=knots, lam=lam, cg_iters=40,
                           device=dev)
    # tight limits so that both penalty terms are active
    tl.lim1, tl.lim2 = 0.6 * 2 * np.pi / samples, 1e-3
    with torch.no_grad():  # move off the exact radial start (equal steps)
        tl.coef.add_(0.02 * torch.from_numpy(W.rng(8812).standard_normal(tuple(tl.coef.shape))).to(
            tl.coef.dtype).to(dev))
    grads = {}
    for part in ("rec", "total"):
        tl.coef.grad = None
        total, rec, pen = tl.loss(x, smaps)
        (rec if part == "rec" else total).backward()
        grads[part] = tl.coef.grad.detach().cpu().double()

    coef = tl.coef.detach().cpu().double().requires_grad_(True)
    om_s = torch.matmul(quadratic_bspline_basis(samples, knots), coef)
    E = _dense_E64(om_s.reshape(-1, 2), N, smaps_np)
    n = E.shape[1]
    xt = torch.from_numpy(x_np.astype(np.complex128)).reshape(B, n)
    Eh = E.conj().T
    F = Eh @ E + lam * torch.eye(n, dtype=torch.complex128)
    xk = torch.linalg.solve(F, (Eh @ (E @ xt.T))).T
    rec_ref = torch.view_as_real(xk - xt).pow(2).sum()
    d1 = om_s[:, 1:] - om_s[:, :-1]
    d2 = d1[:, 1:] - d1[:, :-1]
    pen_ref = tl.mu1 * torch.clamp(d1.abs() - tl.lim1, min=0).sum() + \
        tl.mu2 * torch.clamp(d2.abs() - tl.lim2, min=0).sum()
    rec_ref.backward(retain_graph=True)
    g_rec = coef.grad.clone()
    pen_ref.backward()
    g_tot = coef.grad
    rec, pen = rec.detach(), pen.detach()
    e_rec = abs(float(rec) - float(rec_ref)) / float(rec_ref)
    e_gr = float((grads["rec"] - g_rec).norm() / g_rec.norm())
    e_gt = float((grads["total"] - g_tot).norm() / g_tot.norm())
    _say(f"  rec {float(rec):.6g} vs {float(rec_ref):.6g} ({e_rec:.2e}); pen {float(pen):.4g} vs "
         f"{float(pen_ref):.4g}; dL/dcoef rec-only {e_gr:.2e}, total {e_gt:.2e}, "
         f"|g_rec| / |g_total| {float(g_rec.norm() / g_tot.norm()):.2f}")
    assert float(pen_ref) > 0
    assert e_rec < 1e-3
    assert e_gr < 1e-3
    assert e_gt < 1e-3
