"""Pins of the FP64 CG-SENSE oracle against routines other than itself.

The SENSE matrix E is formed densely here straight from its definition
(a_mj = exp(-i omega_m . r_j), Sec. II-B; E = (I_C kron A) S, Sec. II-G), so
that the pins do not go through the oracle's NUDFT code.
"""
import numpy as np
import pytest
from scipy.sparse.linalg import cg as scipy_cg

from oracle import cg as cg_ref
from paper_2111_02912_amd import workloads as W


def _dense_E(omega, N, smaps):
    r = np.stack(np.meshgrid(*[np.arange(n) - n // 2 for n in N], indexing="ij"), -1).reshape(-1, len(N))
    A = np.exp(-1j * (omega.astype(np.float64) @ r.T.astype(np.float64)))  # [M, npix]
    if smaps is None:
        return A
    return np.concatenate([A * smaps[c].reshape(1, -1).astype(np.complex128)
                           for c in range(smaps.shape[0])], axis=0)  # [C*M, npix]


def _case(N=(6, 5), C=2, M=40, seed=7001):
    om = W.uniform_random(M, len(N), seed)
    smaps = W.sense_maps(C, N) if C > 1 else None
    xt = W.complex_normal(N, seed + 1).astype(np.complex128)
    E = _dense_E(om, N, smaps)
    y = (E @ xt.reshape(-1)).reshape(C, M)
    return om, smaps, y, E


def test_converges_to_direct_solve():
    N, lam = (6, 5), 1e-3
    om, smaps, y, E = _case(N)
    H = E.conj().T @ E + lam * np.eye(E.shape[1])
    x_dir = np.linalg.solve(H, E.conj().T @ y.reshape(-1))
    x, rel = cg_ref.cg_sense(om, y, N, smaps, lam=lam, iters=200)
    assert np.linalg.norm(x.reshape(-1) - x_dir) / np.linalg.norm(x_dir) < 1e-7
    assert rel < 1e-9


def test_ten_iterations_match_scipy_cg():
    N, lam = (6, 5), 1e-3
    om, smaps, y, E = _case(N, seed=7101)
    H = E.conj().T @ E + lam * np.eye(E.shape[1])
    b = E.conj().T @ y.reshape(-1)
    x_sp, _ = scipy_cg(H, b, x0=np.zeros_like(b), rtol=1e-300, atol=0.0, maxiter=10)
    x, _ = cg_ref.cg_sense(om, y, N, smaps, lam=lam, iters=10)
    assert np.linalg.norm(x.reshape(-1) - x_sp) / np.linalg.norm(x_sp) < 1e-9


@pytest.mark.parametrize("iters", [1, 3, 10])
def test_recursive_residual_is_true_residual(iters):
    N, lam = (6, 5), 1e-2
    om, smaps, y, E = _case(N, seed=7201)
    H = E.conj().T @ E + lam * np.eye(E.shape[1])
    b = E.conj().T @ y.reshape(-1)
    x, rel = cg_ref.cg_sense(om, y, N, smaps, lam=lam, iters=iters)
    true_rel = np.linalg.norm(b - H @ x.reshape(-1)) / np.linalg.norm(b)
    assert abs(rel - true_rel) < 1e-9 * max(1.0, true_rel) + 1e-12


def test_one_iteration_is_steepest_descent():
    """After one step x = (b'b / b'Hb) b."""
    N, lam = (5, 4), 1e-3
    om, smaps, y, E = _case(N, C=1, M=30, seed=7301)
    H = E.conj().T @ E + lam * np.eye(E.shape[1])
    b = E.conj().T @ y.reshape(-1)
    x1 = (np.vdot(b, b).real / np.vdot(b, H @ b).real) * b
    x, _ = cg_ref.cg_sense(om, y, N, None, lam=lam, iters=1)
    assert np.linalg.norm(x.reshape(-1) - x1) / np.linalg.norm(x1) < 1e-12


def test_zero_data_gives_zero():
    N = (4, 4)
    om, smaps, y, _ = _case(N, C=2, M=20, seed=7401)
    x, rel = cg_ref.cg_sense(om, np.zeros_like(y), N, smaps, iters=5)
    assert not np.any(x) and rel == 0.0
