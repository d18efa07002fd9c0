"""Pins of the off-resonance oracle (Sec. II-H).

Independent routes: dense matrices built from the definitions
(a_ij = exp(-i omega_i . r_j) exp(-i w_j t_i); E_f = sum_l diag(b_l) A
diag(c_l)) with torch FP64 autograd for the omega-gradients; special cases
that reduce to the plain NUDFT; the interpolation error of linear time
segmentation, which falls as 1/L^2.
"""
import numpy as np
import pytest
import torch

from oracle import field, ndft
from paper_2111_02912_amd import workloads as W


def _coords(N):
    return np.stack(np.meshgrid(*[np.arange(n) - n // 2 for n in N], indexing="ij"), -1).reshape(-1, len(N))


def _case(N=(6, 5), M=14, L=3, C=2, B=2, seed=9501):
    om = W.uniform_random(M, len(N), seed)
    rng = W.rng(seed + 1)
    b = rng.standard_normal((L, M)) + 1j * rng.standard_normal((L, M))
    c = rng.standard_normal((L,) + N) + 1j * rng.standard_normal((L,) + N)
    smaps = W.sense_maps(C, N) if C > 1 else None
    x = W.complex_normal((B,) + N, seed + 2).astype(np.complex128)
    return om, b, c, smaps, x


def _dense_Ef(om_t, b, c, smaps, N):
    """[C*M, n] torch matrix of sum_l diag(b_l) A diag(c_l s_k), coils stacked."""
    r = torch.from_numpy(_coords(N).astype(np.float64))
    A = torch.exp(-1j * (om_t @ r.T).to(torch.complex128))
    bt = torch.from_numpy(np.asarray(b, dtype=np.complex128))
    ct = torch.from_numpy(np.asarray(c, dtype=np.complex128).reshape(c.shape[0], -1))
    C = 1 if smaps is None else smaps.shape[0]
    st = torch.ones((1, ct.shape[1]), dtype=torch.complex128) if smaps is None else \
        torch.from_numpy(smaps.reshape(C, -1).astype(np.complex128))
    blocks = []
    for k in range(C):
        Ek = sum(bt[l][:, None] * A * (ct[l] * st[k])[None, :] for l in range(ct.shape[0]))
        blocks.append(Ek)
    return torch.cat(blocks, 0)


@pytest.mark.parametrize("C", [1, 2])
def test_segmented_operator_matches_dense_definition(C):
    N = (6, 5)
    om, b, c, smaps, x = _case(N, C=C)
    om_t = torch.from_numpy(om.astype(np.float64)).requires_grad_(True)
    Ef = _dense_Ef(om_t, b, c, smaps, N)
    M = om.shape[0]
    y = field.seg_forward(om, b, c, x, N, smaps)
    yd = (Ef @ torch.from_numpy(x.reshape(2, -1)).T).T.detach().numpy().reshape(2, C, M)
    assert np.allclose(y, yd, rtol=1e-11, atol=1e-11)
    yy = W.complex_normal((2, C, M), 9511).astype(np.complex128)
    xa = field.seg_adjoint(om, b, c, yy, N, smaps)
    xad = (Ef.conj().T @ torch.from_numpy(yy.reshape(2, -1)).T).T.detach().numpy().reshape(xa.shape)
    assert np.allclose(xa, xad, rtol=1e-11, atol=1e-11)


@pytest.mark.parametrize("C", [1, 2])
def test_segmented_gradients_match_dense_autograd(C):
    N = (5, 4)
    om, b, c, smaps, x = _case(N, M=11, C=C, seed=9601)
    M = om.shape[0]
    g = W.complex_normal((2, C, M), 9602).astype(np.complex128)
    # forward operator: L = Re<g, E_f x>
    om_t = torch.from_numpy(om.astype(np.float64)).requires_grad_(True)
    y = (_dense_Ef(om_t, b, c, smaps, N) @ torch.from_numpy(x.reshape(2, -1)).T).T
    (torch.from_numpy(g.reshape(2, -1)).conj() * y).real.sum().backward()
    dom = field.seg_jac_omega_fwd(om, b, c, x, g, N, smaps)
    assert np.allclose(dom, om_t.grad.numpy(), rtol=1e-9, atol=1e-9)
    # adjoint operator: L = Re<h, E_f^H v>
    v = W.complex_normal((2, C, M), 9603).astype(np.complex128)
    h = W.complex_normal((2,) + N, 9604).astype(np.complex128)
    om_t = torch.from_numpy(om.astype(np.float64)).requires_grad_(True)
    xa = (_dense_Ef(om_t, b, c, smaps, N).conj().T @ torch.from_numpy(v.reshape(2, -1)).T).T
    (torch.from_numpy(h.reshape(2, -1)).conj() * xa).real.sum().backward()
    dom_a = field.seg_jac_omega_adj(om, b, c, v, h, N, smaps)
    assert np.allclose(dom_a, om_t.grad.numpy(), rtol=1e-9, atol=1e-9)


def test_one_flat_segment_is_the_plain_nudft():
    N = (7, 6)
    om = W.uniform_random(30, 2, 9701)
    x = W.complex_normal((1,) + N, 9702)
    b = np.ones((1, 30), dtype=np.complex128)
    c = np.ones((1,) + N, dtype=np.complex128)
    assert np.allclose(field.seg_forward(om, b, c, x, N)[:, 0], ndft.forward(om, x, N), atol=1e-11)


def test_exact_model_special_cases_and_adjoint():
    N = (6, 7)
    M = 25
    om = W.uniform_random(M, 2, 9801)
    x = W.complex_normal(N, 9802).astype(np.complex128)
    w = W.rng(9803).uniform(-300, 300, N)
    t = np.linspace(0, 5e-3, M)
    # no field: the NUDFT
    assert np.allclose(field.exact_forward(om, t, np.zeros(N), x, N), ndft.forward(om, x[None], N)[0],
                       atol=1e-11)
    # one readout time t0: the NUDFT of x exp(-i w t0)
    t0 = np.full(M, 2e-3)
    assert np.allclose(field.exact_forward(om, t0, w, x, N),
                       ndft.forward(om, (x * np.exp(-1j * w * 2e-3))[None], N)[0], atol=1e-10)
    y = W.complex_normal((M,), 9804).astype(np.complex128)
    lhs = np.vdot(y, field.exact_forward(om, t, w, x, N))
    rhs = np.vdot(field.exact_adjoint(om, t, w, y, N), x)
    assert abs(lhs - rhs) <= 1e-12 * abs(lhs)


def test_linear_time_segmentation_converges_quadratically():
    N = (8, 8)
    M = 60
    om = W.uniform_random(M, 2, 9901)
    x = W.complex_normal(N, 9902).astype(np.complex128)
    w = 2 * np.pi * 60.0 * W.rng(9903).uniform(-1, 1, N)
    t = np.linspace(0, 8e-3, M)
    exact = field.exact_forward(om, t, w, x, N)
    errs = []
    for L in (4, 8, 16):
        b, c = field.time_segments(t, w, L)
        assert np.allclose(b.sum(0), 1.0) and np.all(b.real >= 0) and not np.any(b.imag)
        errs.append(ndft.rel_l2(field.seg_forward(om, b, c, x[None], N)[0, 0], exact))
    # interpolation error ~ (w dt)^2 / 8 with dt = T / (L - 1)
    assert errs[0] < 0.2 and errs[0] / errs[1] > 3.0 and errs[1] / errs[2] > 3.0
    # a sample exactly at a segment time has one-hot weights
    b, _ = field.time_segments(t, w, 4)
    assert np.isclose(b[0, 0], 1.0) and np.isclose(b[3, -1], 1.0)


def test_segmented_gradient_finite_difference():
    N = (5, 6)
    om, b, c, smaps, x = _case(N, M=9, C=2, B=1, seed=9951)
    g = W.complex_normal((1, 2, 9), 9952).astype(np.complex128)
    v = W.rng(9953).standard_normal(om.shape)

    def loss(o):
        return float(np.real(np.vdot(g, field.seg_forward(o, b, c, x, N, smaps))))

    h = 1e-6
    fd = (loss(om + h * v) - loss(om - h * v)) / (2 * h)
    dom = field.seg_jac_omega_fwd(om, b, c, x, g, N, smaps)
    assert abs(fd - np.sum(dom * v)) <= 1e-6 * max(1.0, abs(fd))
