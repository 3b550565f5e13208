"""Pins for the Lasso oracle against closed forms, brute force and certificates."""
import numpy as np
import pytest

from oracle import lasso, prox, residuals


def _rand_lasso(m, n, seed, k=3, noise=0.05):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n)) / np.sqrt(m)
    x0 = np.zeros(n)
    x0[rng.choice(n, k, replace=False)] = rng.standard_normal(k)
    b = A @ x0 + noise * rng.standard_normal(m)
    return A, b


def test_soft_threshold_closed_form_and_ties():
    v = np.array([3.0, -3.0, 0.5, -0.5, 1.0, -1.0, 0.0])
    out = prox.soft_threshold(v, 1.0)
    assert np.array_equal(out, [2.0, -2.0, 0.0, 0.0, 0.0, 0.0, 0.0])


def test_soft_threshold_is_the_prox():
    # argmin_z kappa|z| + (1/2)(z - v)^2 by dense grid search, per element
    rng = np.random.default_rng(0)
    v = rng.standard_normal(25) * 2
    kappa = 0.7
    grid = np.linspace(-8, 8, 160001)
    for vi, zi in zip(v, prox.soft_threshold(v, kappa)):
        obj = kappa * np.abs(grid) + 0.5 * (grid - vi) ** 2
        assert abs(grid[np.argmin(obj)] - zi) <= 2e-4


def test_soft_threshold_float32_bitwise():
    rng = np.random.default_rng(1)
    v = rng.standard_normal(1000).astype(np.float32)
    k = np.float32(0.3)
    out = prox.soft_threshold(v, k)
    assert out.dtype == np.float32
    ref = np.where(v > k, v - k, np.where(v < -k, v + k, np.float32(0)))
    assert np.array_equal(out.view(np.uint32), ref.astype(np.float32).view(np.uint32))


def test_orthonormal_closed_form():
    rng = np.random.default_rng(2)
    Q, _ = np.linalg.qr(rng.standard_normal((40, 12)))
    b = rng.standard_normal(40)
    lam = 0.4
    sol = lasso.solve(Q, b, lam)
    expect = prox.soft_threshold(Q.T @ b, lam)
    assert np.allclose(sol["x"], expect, atol=1e-10)


@pytest.mark.parametrize("seed,n", [(3, 6), (4, 7), (5, 8)])
def test_brute_force_unique_kkt_point(seed, n):
    A, b = _rand_lasso(12, n, seed, k=2)
    lam = 0.2 * np.max(np.abs(A.T @ b))
    kkt, xbest, Fbest = lasso.brute_force(A, b, lam)
    assert len(kkt) == 1
    assert np.allclose(kkt[0], xbest, atol=1e-12)
    sol = lasso.solve(A, b, lam)
    assert np.allclose(sol["x"], xbest, atol=1e-9)
    assert abs(sol["F"] - Fbest) <= 1e-12 * Fbest


def test_brute_force_underdetermined():
    A, b = _rand_lasso(5, 8, 6, k=2)
    lam = 0.3 * np.max(np.abs(A.T @ b))
    kkt, xbest, Fbest = lasso.brute_force(A, b, lam)
    sol = lasso.solve(A, b, lam)
    assert abs(sol["F"] - Fbest) <= 1e-10 * Fbest
    assert np.allclose(sol["x"], xbest, atol=1e-8)


def test_lambda_max_gives_zero():
    A, b = _rand_lasso(30, 50, 7)
    lmax = np.max(np.abs(A.T @ b))
    assert np.all(lasso.solve(A, b, lmax * 1.0001)["x"] == 0)
    assert np.any(lasso.solve(A, b, lmax * 0.98)["x"] != 0)


def test_small_lambda_is_least_squares():
    A, b = _rand_lasso(60, 15, 8, k=15)
    sol = lasso.solve(A, b, 1e-10)
    ls = np.linalg.lstsq(A, b, rcond=None)[0]
    assert np.allclose(sol["x"], ls, atol=1e-8)


def test_duality_gap_bounds_suboptimality():
    A, b = _rand_lasso(40, 80, 9, k=5)
    lam = 0.1 * np.max(np.abs(A.T @ b))
    Fstar = lasso.solve(A, b, lam)["F"]
    rng = np.random.default_rng(10)
    for _ in range(20):
        x = rng.standard_normal(80) * rng.random()
        gap, F, d = lasso.duality_gap(A, b, lam, x)
        assert gap >= 0
        assert F - Fstar <= gap + 1e-12
        assert d <= Fstar + 1e-12
    sol = lasso.solve(A, b, lam)
    gap, F, _ = lasso.duality_gap(A, b, lam, sol["x"])
    assert gap <= 1e-11 * F
    assert lasso.kkt_violation(A, b, lam, sol["x"]) <= 1e-9


def test_genios_admm_fixed_point_matches_brute_force():
    # GeNIOS parameters (over-relaxation 1.6, sigma 1e-6, adaptive rho) must
    # converge to the same optimum as exhaustive enumeration.
    A, b = _rand_lasso(10, 7, 11, k=2)
    lam = 0.15 * np.max(np.abs(A.T @ b))
    _, xbest, Fbest = lasso.brute_force(A, b, lam)
    x, z, u, rho, hist = lasso.admm(A, b, lam, rho=1.0, alpha=1.6, sigma=1e-6,
                                    max_iter=3000, eps=1e-12, rho_update_every=25)
    assert np.allclose(z, xbest, atol=1e-8)
    assert hist[-1, 3] <= 1e-12


def test_admm_residual_history_and_rho_rule():
    A, b = _rand_lasso(20, 40, 12, k=4)
    lam = 0.05 * np.max(np.abs(A.T @ b))
    x, z, u, rho, hist = lasso.admm(A, b, lam, rho=50.0, alpha=1.6, sigma=1e-6,
                                    max_iter=200, rho_update_every=25, rho_update_until=100)
    # the penalty only changes at multiples of 25 up to 100, and by a factor tau
    for row in hist:
        k, rp, rd, rk, used, after = row
        if after != used:
            assert k % 25 == 0 and k <= 100
            assert after in (used * 2.0, used / 2.0)
            assert (after > used) == (rp > 10 * rd)
    assert hist[-1, 3] < hist[0, 3]


def test_r_kkt_matches_paper_test():
    rng = np.random.default_rng(13)
    for _ in range(200):
        n = 30
        x, z, u = (rng.standard_normal(n) for _ in range(3))
        z = x + rng.standard_normal(n) * 10 ** rng.uniform(-8, 0)
        g = -u + rng.standard_normal(n) * 10 ** rng.uniform(-8, 0)
        rho = 1.0
        rk, _, _ = residuals.r_kkt(x, z, u, rho, g)
        eps = 10 ** rng.uniform(-7, -1)
        assert (rk <= eps) == residuals.paper_stop_test(x, z, u, rho, g, eps, eps)


def test_hessian_vector_is_the_change_of_gradient():
    # f is quadratic: grad f(x + p) - grad f(x) = A^T A p exactly (up to rounding)
    A, b = _rand_lasso(40, 25, 11)
    rng = np.random.default_rng(12)
    x = rng.standard_normal(25)
    p = rng.standard_normal(25)
    hv = lasso.hessian_vector(A, p)
    ref = lasso.grad_f(A, b, x + p) - lasso.grad_f(A, b, x)
    assert np.allclose(hv, ref, rtol=1e-12, atol=1e-12)
    assert hv @ p > 0  # positive definite here (m > n)


def test_hessian_vector_with_logistic_weights_matches_gradient_differences():
    # H(x) p = A^T diag(s(1 - s)) A p: central differences of the logistic gradient
    from oracle import logreg
    rng = np.random.default_rng(13)
    A = rng.standard_normal((60, 15))
    y = np.where(rng.random(60) < 0.5, 1.0, -1.0)
    x = 0.3 * rng.standard_normal(15)
    p = rng.standard_normal(15)
    hv = lasso.hessian_vector(A, p, logreg.hess_diag(A, y, x))
    h = 1e-5
    fd = (logreg.grad_f(A, y, x + h * p) - logreg.grad_f(A, y, x - h * p)) / (2 * h)
    assert np.allclose(hv, fd, rtol=1e-7, atol=1e-8)


def test_working_set_solve_equals_the_plain_solve():
    import genios_data
    P = genios_data.config("lasso_200x1000")
    ref = lasso.solve(P["A"], P["b"], P["lam"])
    ws = lasso.solve_working_set(P["A"], P["b"], P["lam"], start=8, grow=8)
    assert ws["certified"] and ws["outer"] >= 2
    assert abs(ws["F"] - ref["F"]) <= 1e-12 * ref["F"]
    assert np.array_equal(ws["support"], ref["support"])
    assert np.allclose(ws["x"], ref["x"], rtol=1e-9, atol=1e-12)
    gap, F, _ = lasso.duality_gap(P["A"], P["b"], P["lam"], ws["x"])
    assert abs(gap - ws["gap"]) <= 1e-9 * F and gap <= 1e-11 * F
    assert np.allclose(lasso.rmatvec_rows(P["A"], P["b"], rows=7),
                       P["A"].astype(np.float64).T @ P["b"].astype(np.float64), rtol=1e-12)
