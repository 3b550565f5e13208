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


def test_stabilised_at_zero_shift_is_the_plain_definition():
    # Cholesky + SVD route against the eigendecomposition route of the definition
    rng = np.random.default_rng(31)
    G = rng.standard_normal((25, 60)) * np.logspace(0, -2, 60)
    H = G.T @ G
    Om = rng.standard_normal((60, 12))
    U0, l0 = nystrom.nystrom(H, Om)
    U1, l1 = nystrom.nystrom_stabilised(H @ Om, Om, 0.0)
    assert np.allclose(l1, l0, rtol=1e-9, atol=1e-12 * l0[0])
    assert np.allclose((U1 * l1) @ U1.T, nystrom.nystrom_dense(H, Om), atol=1e-9 * np.abs(H).max())


@pytest.mark.parametrize("mu", [1e-3, 0.2])
def test_stabilised_is_the_definition_for_the_shifted_matrix(mu):
    # U diag(lam_hat + mu) U^T = (H + mu I)_hat, the dense pseudo-inverse formula
    # on H + mu I; Lam_hat is that minus mu (no clipping at these sizes)
    rng = np.random.default_rng(32)
    G = rng.standard_normal((20, 50)) * np.logspace(0, -1.5, 50)
    H = G.T @ G
    Om = rng.standard_normal((50, 10))
    U, lam = nystrom.nystrom_stabilised(H @ Om, Om, mu)
    Hs = H + mu * np.eye(50)
    ref = nystrom.nystrom_dense(Hs, Om)
    assert np.allclose((U * (lam + mu)) @ U.T, ref, atol=1e-9 * np.abs(Hs).max())
    ev = np.sort(np.linalg.eigvalsh(ref))[::-1][:10]
    assert np.allclose(lam, ev - mu, rtol=1e-9, atol=1e-12 * ev[0])
    assert np.allclose(U.T @ U, np.eye(10), atol=1e-10)
    # (H + mu I)_hat <= H + mu I in the Loewner order, i.e.
    # U Lam_hat U^T <= H + mu (I - U U^T)
    E = H + mu * (np.eye(50) - U @ U.T) - (U * lam) @ U.T
    assert np.linalg.eigvalsh(0.5 * (E + E.T)).min() >= -1e-9 * np.abs(H).max()


def test_stabilising_shift_is_unit_roundoff_times_frobenius_norm():
    Y = np.array([[3.0, 0.0], [0.0, 4.0]])
    assert nystrom.stabilising_shift(Y, 2.0 ** -24) == 5.0 * 2.0 ** -24


def _fp32_stabilised(G, Om, mu):
    """The stabilised core with the sketch and Omega^T Y_mu formed in FP32, as a
    single-precision device path forms them; returns lam_hat or None when the
    Cholesky factor does not exist."""
    Y32 = (G.T @ (G @ Om)).astype(np.float32)
    Ymu = (Y32 + np.float32(mu) * Om).astype(np.float32)
    M = (Om.T @ Ymu).astype(np.float32).astype(np.float64)
    try:
        C = np.linalg.cholesky(0.5 * (M + M.T))
    except np.linalg.LinAlgError:
        return None
    B = np.linalg.solve(C, Ymu.astype(np.float64).T).T
    sv = np.linalg.svd(B, compute_uv=False)
    return np.maximum(sv ** 2 - mu, 0.0)


@pytest.mark.parametrize("n,s,k", [(2000, 40, 20), (6000, 50, 20)])
def test_stabilising_shift_scale_is_bracketed(n, s, k):
    # The shift must be large enough that the s x s core of an exactly rank-k
    # operator (k < s) stays positive definite under FP32 rounding of the sketch,
    # and small enough that the recovered eigenvalues keep close to H's.  The
    # reading's u ||Y||_F meets both on every seed; a shift n times smaller (or
    # none) loses the factorisation, one sqrt(n) times larger (the orthonormal-
    # Omega formula applied unscaled to a Gaussian Omega) biases the eigenvalues.
    u = 2.0 ** -24
    for seed in range(6):
        rng = np.random.default_rng(seed)
        G = (rng.standard_normal((k, n)) * np.logspace(0, -1, n)).astype(np.float32)
        Om = rng.standard_normal((n, s)).astype(np.float32)
        G64 = G.astype(np.float64)
        ev = np.sort(np.linalg.eigvalsh(G64 @ G64.T))[::-1]   # the nonzero spectrum of G^T G
        mu = nystrom.stabilising_shift((G.T @ (G @ Om)).astype(np.float32), u)
        lam = _fp32_stabilised(G, Om, mu)
        assert lam is not None
        assert np.max(np.abs(lam[:k] - ev) / ev) <= 2e-3
        assert np.max(lam[k:]) <= 1e-6 * ev[0]              # the rank is recovered
        assert _fp32_stabilised(G, Om, 0.0) is None
        assert _fp32_stabilised(G, Om, mu / n) is None
        big = _fp32_stabilised(G, Om, mu * np.sqrt(n))
        assert np.max(np.abs(big[:k] - ev) / ev) > 1e-2
