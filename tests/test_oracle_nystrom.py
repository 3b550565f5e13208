"""Pins for the Nystrom approximation, preconditioner and PCG reference."""
import numpy as np
import pytest

from oracle import nystrom


def _psd(n, rank, seed, decay=True):
    rng = np.random.default_rng(seed)
    Q, _ = np.linalg.qr(rng.standard_normal((n, rank)))
    ev = np.logspace(2, -2, rank) if decay else rng.random(rank) + 0.5
    return (Q * ev) @ Q.T


def test_exact_when_rank_at_most_sketch():
    H = _psd(40, 6, 0)
    Om = np.random.default_rng(1).standard_normal((40, 8))
    Hh = nystrom.nystrom_dense(H, Om)
    assert np.allclose(Hh, H, atol=1e-9 * np.abs(H).max())
    U, lam = nystrom.nystrom(H, Om)
    assert np.allclose((U * lam) @ U.T, H, atol=1e-9 * np.abs(H).max())


def test_loewner_order_and_invariance():
    rng = np.random.default_rng(2)
    G = rng.standard_normal((30, 50))
    H = G.T @ G
    Om = rng.standard_normal((50, 10))
    Hh = nystrom.nystrom_dense(H, Om)
    assert np.linalg.eigvalsh(Hh).min() >= -1e-8 * np.abs(H).max()
    assert np.linalg.eigvalsh(H - Hh).min() >= -1e-8 * np.abs(H).max()
    R = rng.standard_normal((10, 10))
    Hh2 = nystrom.nystrom_dense(H, Om @ R)
    assert np.allclose(Hh, Hh2, atol=1e-7 * np.abs(H).max())


def test_two_routes_agree_and_u_orthonormal():
    rng = np.random.default_rng(3)
    G = rng.standard_normal((40, 60)) * np.arange(1, 61) ** -0.5
    H = G.T @ G
    Om = rng.standard_normal((60, 12))
    U, lam = nystrom.nystrom(H, Om)
    assert np.allclose(U.T @ U, np.eye(U.shape[1]), atol=1e-10)
    assert np.all(np.diff(lam) <= 1e-12)
    assert np.allclose((U * lam) @ U.T, nystrom.nystrom_dense(H, Om), atol=1e-9 * np.abs(H).max())


def test_preconditioner_spd_and_apply():
    rng = np.random.default_rng(4)
    G = rng.standard_normal((30, 45))
    H = G.T @ G
    U, lam = nystrom.nystrom(H, rng.standard_normal((45, 8)))
    for nu in (1e-3, 1.0, 100.0):
        P = nystrom.preconditioner(U, lam, nu)
        assert np.allclose(P, P.T)
        assert np.linalg.eigvalsh(P).min() > 0
        r = rng.standard_normal(45)
        assert np.allclose(P @ r, nystrom.apply_preconditioner(U, lam, nu, r))


def test_exact_low_rank_two_eigenvalues():
    H = _psd(50, 5, 5)
    Om = np.random.default_rng(6).standard_normal((50, 5))
    U, lam = nystrom.nystrom(H, Om)
    nu = 0.3
    P = nystrom.preconditioner(U, lam, nu)
    ev = np.sort(np.linalg.eigvals(P @ (H + nu * np.eye(50))).real)
    assert np.allclose(ev[:45], nu, rtol=1e-8)
    assert np.allclose(ev[45:], lam[-1] + nu, rtol=1e-8)


@pytest.mark.parametrize("nu", [1e-2, 1.0])
def test_condition_number_bound(nu):
    rng = np.random.default_rng(7)
    G = rng.standard_normal((60, 80)) * np.arange(1, 81) ** -1.0
    H = G.T @ G
    U, lam = nystrom.nystrom(H, rng.standard_normal((80, 10)))
    E = H - (U * lam) @ U.T
    Enorm = np.linalg.eigvalsh(E).max()
    P = nystrom.preconditioner(U, lam, nu)
    w, V = np.linalg.eigh(P)
    Ph = (V * np.sqrt(w)) @ V.T
    ev = np.linalg.eigvalsh(Ph @ (H + nu * np.eye(80)) @ Ph)
    kappa = ev.max() / ev.min()
    assert kappa <= nystrom.kappa_bound(lam, Enorm, nu) * (1 + 1e-8)
    assert kappa < np.linalg.cond(H + nu * np.eye(80))


def test_zero_matrix_gives_identity():
    U, lam = nystrom.nystrom(np.zeros((10, 10)), np.ones((10, 3)))
    assert U.shape[1] == 0
    assert np.allclose(nystrom.preconditioner(U, lam, 1.0), np.eye(10))


def test_solve_shifted():
    rng = np.random.default_rng(8)
    G = rng.standard_normal((20, 30))
    H = G.T @ G
    r = rng.standard_normal(30)
    x = nystrom.solve_shifted(H, 0.5, r)
    assert np.allclose(H @ x + 0.5 * x, r)
