"""Pins for the adaptive sketch size oracle (Sec. 2.2, adaptive sketch size)."""
import numpy as np
import pytest

from oracle import adaptive, nystrom, philox


def _decaying(n, m, p, seed):
    rng = np.random.default_rng(seed)
    G = rng.standard_normal((m, n)) * np.arange(1, n + 1) ** -p
    return G.T @ G


def test_power_estimate_is_a_lower_bound_that_converges():
    H = _decaying(120, 200, 0.8, 1)
    U, lam = adaptive.sketch_at(H, philox.gaussian_matrix(120, 8, 5).astype(np.float64), 2.0 ** -53, 1e-13)
    E = H - (U * lam) @ U.T
    exact = np.linalg.eigvalsh(E).max()
    v0 = np.random.default_rng(2).standard_normal(120)
    prev = -1.0
    for q in (1, 2, 5, 10, 200):
        est = adaptive.power_norm(lambda v: E @ v, v0, q)
        assert est <= exact * (1 + 1e-12)
        assert est >= prev - 1e-12 * exact  # Rayleigh quotients of PSD E rise
        prev = est
    assert abs(est - exact) <= 1e-8 * exact


@pytest.mark.parametrize("nu", [1e-2, 1.0])
def test_bound_holds_for_the_chosen_sketch(nu):
    H = _decaying(100, 150, 1.0, 3)
    out = adaptive.adaptive_sketch(H, nu, 4, 64, 10.0, 30, seed=11, unit_roundoff=2.0 ** -53,
                                   rel_thresh=1e-13)
    U, lam = out["U"], out["lam"]
    E = H - (U * lam) @ U.T
    exact = np.linalg.eigvalsh(E).max()
    P = nystrom.preconditioner(U, lam, nu)
    w, V = np.linalg.eigh(P)
    Ph = (V * np.sqrt(w)) @ V.T
    ev = np.linalg.eigvalsh(Ph @ (H + nu * np.eye(100)) @ Ph)
    assert ev.max() / ev.min() <= nystrom.kappa_bound(lam, exact, nu) * (1 + 1e-8)
    assert out["err"] <= exact * (1 + 1e-10)


def test_chosen_size_is_the_first_that_meets_the_target():
    H = _decaying(150, 200, 0.9, 4)
    nu, target, q = 0.5, 8.0, 20
    out = adaptive.adaptive_sketch(H, nu, 2, 128, target, q, seed=7)
    Om = philox.gaussian_matrix(150, 128, 7).astype(np.float64)
    v0 = philox.gaussian_matrix(150, 1, 7, adaptive.POWER_STREAM)[:, 0].astype(np.float64)
    sizes = [2, 4, 8, 16, 32, 64, 128]
    bounds = []
    for r in sizes:  # each size on its own
        U, lam = adaptive.sketch_at(H, Om[:, :r], 2.0 ** -24, 1e-6)
        err = adaptive.power_norm(lambda v: H @ v - U @ (lam * (U.T @ v)), v0, q)
        bounds.append(nystrom.kappa_bound(lam, err, nu))
    first = next((r for r, bd in zip(sizes, bounds) if bd <= target), sizes[-1])
    assert out["rank"] == first
    assert [h[0] for h in out["history"]] == sizes[:sizes.index(first) + 1]
    assert 2 < first < 128  # the case exercises growth and an early stop
    # the bound falls as the sketch grows (decaying spectrum)
    assert bounds[0] > bounds[sizes.index(first)]


def test_exact_low_rank_stops_at_the_first_size():
    rng = np.random.default_rng(5)
    G = rng.standard_normal((6, 80))
    H = G.T @ G  # rank 6
    out = adaptive.adaptive_sketch(H, 1.0, 8, 64, 1e6, 10, seed=3, unit_roundoff=2.0 ** -53,
                                   rel_thresh=1e-12)
    assert out["rank"] == 8 and out["lam"].size == 6
    assert out["err"] <= 1e-8 * np.linalg.eigvalsh(H).max()
