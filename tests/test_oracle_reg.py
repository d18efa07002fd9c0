"""Pins of the finite-difference regulariser T (QPLS, Sec. IV-B) in the
oracle, and of CG / inverse gradients that use it.

T is formed densely here as a stack of Kronecker products of the 1D
first-difference matrix (rows e_{j+1} - e_j), an independent construction
from the oracle's np.diff / padding route.  T^H T in 1D is the path-graph
Laplacian, whose eigenvalues 2 - 2 cos(pi k / n) are known in closed form.
"""
import numpy as np
import pytest
import torch
from scipy.sparse.linalg import cg as scipy_cg

from oracle import cg as cg_ref
from oracle import inverse
from paper_2111_02912_amd import workloads as W


def _diff1(n):
    return np.eye(n - 1, n, 1) - np.eye(n - 1, n)


def _dense_T(N):
    blocks = []
    for d in range(len(N)):
        m = np.ones((1, 1))
        for e, n in enumerate(N):
            m = np.kron(m, _diff1(n) if e == d else np.eye(n))
        blocks.append(m)
    return np.concatenate(blocks, 0)


def _dense_E(omega, N, smaps):
    r = np.stack(np.meshgrid(*[np.arange(n) - n // 2 for n in N], indexing="ij"), -1).reshape(-1, len(N))
    A = np.exp(-1j * (omega.astype(np.float64) @ r.T.astype(np.float64)))
    if smaps is None:
        return A
    return np.concatenate([A * smaps[c].reshape(1, -1).astype(np.complex128)
                           for c in range(smaps.shape[0])], axis=0)


@pytest.mark.parametrize("N", [(7,), (5, 4), (3, 4, 5)])
def test_fd_matches_dense_kronecker_operator(N):
    T = _dense_T(N)
    x = W.complex_normal(N, 9001).astype(np.complex128)
    tx = np.concatenate([u.reshape(-1) for u in cg_ref.fd_forward(x, N)])
    assert np.allclose(tx, T @ x.reshape(-1), atol=1e-12)
    u = W.complex_normal((T.shape[0],), 9002).astype(np.complex128)
    parts, o = [], 0
    for d in range(len(N)):
        shp = tuple(n - 1 if e == d else n for e, n in enumerate(N))
        k = int(np.prod(shp))
        parts.append(u[o:o + k].reshape(shp))
        o += k
    assert np.allclose(cg_ref.fd_adjoint(parts, N).reshape(-1), T.conj().T @ u, atol=1e-12)
    assert np.allclose(cg_ref.reg_normal(x, N, "finite_diff").reshape(-1),
                       T.T @ (T @ x.reshape(-1)), atol=1e-12)


def test_fd_normal_is_path_laplacian():
    n = 6
    L = np.stack([cg_ref.reg_normal(np.eye(n)[k], (n,), "finite_diff") for k in range(n)])
    ref = 2 * np.eye(n) - np.eye(n, k=1) - np.eye(n, k=-1)
    ref[0, 0] = ref[-1, -1] = 1
    assert np.array_equal(L.real, ref) and not np.any(L.imag)
    ev = np.sort(np.linalg.eigvalsh(L.real))
    assert np.allclose(ev, np.sort(2 - 2 * np.cos(np.pi * np.arange(n) / n)), atol=1e-12)


def test_constants_are_the_null_space():
    N = (4, 5, 3)
    c = np.full(N, 0.7 - 0.2j)
    assert np.allclose(cg_ref.reg_normal(c, N, "finite_diff"), 0, atol=1e-15)
    imp = np.zeros(N, dtype=np.complex128)
    imp[1, 2, 1] = 1.0
    out = cg_ref.reg_normal(imp, N, "finite_diff")
    assert out[1, 2, 1] == 6.0 and out[0, 2, 1] == -1.0 and out[1, 2, 2] == -1.0
    assert np.isclose(out.sum(), 0.0)


def _case(N=(6, 5), C=2, M=40, seed=9101):
    om = W.uniform_random(M, len(N), seed)
    smaps = W.sense_maps(C, N) if C > 1 else None
    xt = W.complex_normal(N, seed + 1).astype(np.complex128)
    E = _dense_E(om, N, smaps)
    y = (E @ xt.reshape(-1)).reshape(C, M)
    return om, smaps, y, E


def test_qpls_cg_converges_to_direct_solve():
    N, lam = (6, 5), 0.5
    om, smaps, y, E = _case(N)
    T = _dense_T(N)
    H = E.conj().T @ E + lam * T.T @ T
    x_dir = np.linalg.solve(H, E.conj().T @ y.reshape(-1))
    x, rel = cg_ref.cg_sense(om, y, N, smaps, lam=lam, iters=200, reg="finite_diff")
    assert np.linalg.norm(x.reshape(-1) - x_dir) / np.linalg.norm(x_dir) < 1e-7
    assert rel < 1e-9


def test_qpls_ten_iterations_match_scipy_cg():
    N, lam = (6, 5), 0.3
    om, smaps, y, E = _case(N, seed=9201)
    T = _dense_T(N)
    H = E.conj().T @ E + lam * T.T @ T
    b = E.conj().T @ y.reshape(-1)
    x_sp, _ = scipy_cg(H, b, x0=np.zeros_like(b), rtol=1e-300, atol=0.0, maxiter=10)
    x, _ = cg_ref.cg_sense(om, y, N, smaps, lam=lam, iters=10, reg="finite_diff")
    assert np.linalg.norm(x.reshape(-1) - x_sp) / np.linalg.norm(x_sp) < 1e-9


@pytest.mark.parametrize("C", [1, 2])
def test_qpls_inverse_gradients_match_dense_autograd(C):
    N, lam = (5, 4), 0.2
    om = W.uniform_random(12, 2, 9301)
    smaps = W.sense_maps(C, N) if C > 1 else None
    x = W.complex_normal((2,) + N, 9302).astype(np.complex128)
    c = W.complex_normal((2,) + N, 9303).astype(np.complex128)
    r = np.stack(np.meshgrid(*[np.arange(n) - n // 2 for n in N], indexing="ij"), -1).reshape(-1, 2)
    om_t = torch.from_numpy(om.astype(np.float64)).requires_grad_(True)
    x_t = torch.from_numpy(x.reshape(2, -1)).requires_grad_(True)
    A = torch.exp(-1j * (om_t @ torch.from_numpy(r.T.astype(np.float64))).to(torch.complex128))
    if smaps is None:
        E = A
    else:
        s = torch.from_numpy(smaps.reshape(C, -1).astype(np.complex128))
        E = torch.cat([A * s[k][None, :] for k in range(C)], 0)
    T = torch.from_numpy(_dense_T(N)).to(torch.complex128)
    F = E.conj().T @ E + lam * (T.T @ T)
    z = torch.linalg.solve(F, x_t.T).T
    loss = (torch.from_numpy(c.reshape(2, -1)).conj() * z).real.sum()
    loss.backward()
    dom, dx = inverse.inverse_vjp(om, x, c, N, smaps, lam, reg="finite_diff")
    assert np.allclose(dom, om_t.grad.numpy(), rtol=1e-8, atol=1e-8)
    assert np.allclose(dx.reshape(2, -1), x_t.grad.numpy(), rtol=1e-8, atol=1e-8)
    zs = inverse.solve(om, x, N, smaps, lam, reg="finite_diff")
    assert np.allclose(zs.reshape(2, -1), z.detach().numpy(), rtol=1e-9, atol=1e-9)


def test_unknown_regulariser_rejected():
    with pytest.raises(ValueError):
        cg_ref.reg_normal(np.zeros((3, 3)), (3, 3), "tv")
    assert cg_ref.REGS == ("identity", "finite_diff")
