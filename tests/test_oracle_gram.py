"""Pins of the Gram and regularised-inverse gradients (Sec. II-E, II-F).

The independent route is torch FP64 autograd through dense matrices built
from the definition a_mj = exp(-i omega_m . r_j) (Sec. II-B) and the SENSE
model E = (I_C kron A) S (Sec. II-G); the inverse goes through
torch.linalg.solve.  A central finite difference of the oracle's own Gram
operator ties the omega-gradient to the forward map as well.
"""
import numpy as np
import pytest
import torch

from oracle import inverse, ndft
from paper_2111_02912_amd import workloads as W


def _dense_E(om_t, N, smaps):
    r = np.stack(np.meshgrid(*[np.arange(n) - n // 2 for n in N], indexing="ij"), -1).reshape(-1, len(N))
    rt = torch.from_numpy(r.astype(np.float64))
    A = torch.exp(-1j * (om_t @ rt.T).to(torch.complex128))  # [M, n]
    if smaps is None:
        return A
    s = torch.from_numpy(smaps.reshape(smaps.shape[0], -1).astype(np.complex128))
    return torch.cat([A * s[c][None, :] for c in range(s.shape[0])], 0)


def _case(N=(5, 4), C=2, M=12, B=2, seed=7501):
    om = W.uniform_random(M, len(N), seed)
    smaps = W.sense_maps(C, N) if C > 1 else None
    x = W.complex_normal((B,) + N, seed + 1).astype(np.complex128)
    c = W.complex_normal((B,) + N, seed + 2).astype(np.complex128)
    return om, smaps, x, c


@pytest.mark.parametrize("C", [1, 2])
def test_gram_gradients_match_dense_autograd(C):
    N = (5, 4)
    om, smaps, x, c = _case(N, C=C)
    om_t = torch.from_numpy(om.astype(np.float64)).requires_grad_(True)
    x_t = torch.from_numpy(x.reshape(x.shape[0], -1)).requires_grad_(True)
    E = _dense_E(om_t, N, smaps)
    z = (E.conj().T @ (E @ x_t.T)).T
    loss = (torch.from_numpy(c.reshape(c.shape[0], -1)).conj() * z).real.sum()
    loss.backward()
    dom, dx = ndft.gram_vjp(om, x, c, N, smaps)
    assert np.allclose(dom, om_t.grad.numpy(), rtol=1e-9, atol=1e-9)
    assert np.allclose(dx.reshape(dx.shape[0], -1), x_t.grad.numpy(), rtol=1e-9, atol=1e-9)


@pytest.mark.parametrize("C", [1, 2])
def test_inverse_gradients_match_dense_autograd(C):
    N, lam = (5, 4), 1e-2
    om, smaps, x, c = _case(N, C=C, seed=7601)
    om_t = torch.from_numpy(om.astype(np.float64)).requires_grad_(True)
    x_t = torch.from_numpy(x.reshape(x.shape[0], -1)).requires_grad_(True)
    E = _dense_E(om_t, N, smaps)
    n = E.shape[1]
    F = E.conj().T @ E + lam * torch.eye(n, dtype=torch.complex128)
    z = torch.linalg.solve(F, x_t.T).T
    loss = (torch.from_numpy(c.reshape(c.shape[0], -1)).conj() * z).real.sum()
    loss.backward()
    dom, dx = inverse.inverse_vjp(om, x, c, N, smaps, lam)
    assert np.allclose(dom, om_t.grad.numpy(), rtol=1e-8, atol=1e-8)
    assert np.allclose(dx.reshape(dx.shape[0], -1), x_t.grad.numpy(), rtol=1e-8, atol=1e-8)
    zs = inverse.solve(om, x, N, smaps, lam)
    assert np.allclose(zs.reshape(zs.shape[0], -1), z.detach().numpy(), rtol=1e-9, atol=1e-9)


def test_gram_omega_gradient_finite_difference():
    N = (6, 5)
    om, smaps, x, c = _case(N, C=2, M=10, B=1, seed=7701)
    v = W.rng(7702).standard_normal(om.shape)

    def L(o):
        return float(np.real(np.sum(np.conj(c) * ndft.gram(o, x, N, smaps))))

    h = 1e-6
    fd = (L(om + h * v) - L(om - h * v)) / (2 * h)
    dom, _ = ndft.gram_vjp(om, x, c, N, smaps)
    assert abs(fd - np.sum(dom * v)) <= 1e-6 * max(1.0, abs(fd))
