"""Pins for the l1-regularised Huber fitting oracle (Sec. 4.3, App. A)."""
import numpy as np
import pytest
from scipy.optimize import minimize

import genios_data
from oracle import huber, lasso


def test_loss_is_c1_with_the_stated_derivatives_and_conjugate():
    w = np.linspace(-3, 3, 61)
    for delta in (0.5, 1.0, 2.0):
        # continuity and slope match at |w| = delta
        for s in (-1.0, 1.0):
            a = huber.loss(np.array([s * delta * (1 - 1e-9)]), delta)[0]
            c = huber.loss(np.array([s * delta * (1 + 1e-9)]), delta)[0]
            assert abs(a - c) <= 1e-7
        h = 1e-6
        fd = (huber.loss(w + h, delta) - huber.loss(w - h, delta)) / (2 * h)
        assert np.allclose(fd, huber.dloss(w, delta), atol=1e-5)
        fd2 = (huber.dloss(w + h, delta) - huber.dloss(w - h, delta)) / (2 * h)
        away = np.abs(np.abs(w) - delta) > 1e-3
        assert np.allclose(fd2[away], huber.d2loss(w, delta)[away], atol=1e-4)
        # l*(v) = sup_w (v w - l(w)) = v^2 / 4 on [-2 delta, 2 delta]
        grid = np.linspace(-20, 20, 400001)
        for v in (-2 * delta, -delta, 0.3, 1.9 * delta):
            sup = float(np.max(v * grid - huber.loss(grid, delta)))
            assert abs(sup - v * v / 4) <= 1e-6


def test_large_delta_is_twice_the_lasso_at_half_lambda():
    # if every residual stays inside delta, l(w) = w^2 = 2 (w^2 / 2): the optimum is
    # the Lasso's at lam / 2
    rng = np.random.default_rng(1)
    A = rng.standard_normal((40, 25)) / np.sqrt(40)
    b = A @ np.where(rng.random(25) < 0.3, rng.standard_normal(25), 0.0) + 0.05 * rng.standard_normal(40)
    lam = 0.2 * np.max(np.abs(2 * A.T @ b))
    sol = huber.solve(A, b, lam, delta=1e6)
    ref = lasso.solve(A, b, lam / 2)
    assert np.allclose(sol["x"], ref["x"], atol=1e-8)
    assert abs(sol["F"] - 2 * ref["F"]) <= 1e-9 * sol["F"]


@pytest.mark.parametrize("lam2", [0.0, 0.3])
def test_optimum_kkt_gap_and_lbfgs(lam2):
    P = genios_data.huber_outliers(60, seed=3)
    A, b, lam = P["A"], P["b"], P["lam"]
    sol = huber.solve(A, b, lam, lam2=lam2)
    # with lam2 > 0 the gap with the unscaled nu is quadratic in the KKT residual,
    # so a 1e-12 relative gap certifies a KKT residual of about 1e-6 only
    assert huber.kkt_violation(A, b, lam, sol["x"], lam2=lam2) <= (1e-6 if lam2 == 0 else 1e-5)
    gap, pr, du = huber.duality_gap(A, b, lam, sol["x"], lam2=lam2)
    assert 0.0 <= gap <= 1e-8 * pr
    n = A.shape[1]
    A64, b64 = A.astype(np.float64), b.astype(np.float64)

    def fun(v):
        x = v[:n] - v[n:]
        r = A64 @ x - b64
        g = A64.T @ huber.dloss(r) + lam2 * x
        f = float(np.sum(huber.loss(r))) + lam * float(np.sum(v)) + 0.5 * lam2 * float(x @ x)
        return f, np.concatenate([g + lam, -g + lam])
    res = minimize(fun, np.zeros(2 * n), jac=True, method="L-BFGS-B",
                   bounds=[(0, None)] * (2 * n), options=dict(maxiter=20000, ftol=1e-15, gtol=1e-12))
    x_lb = res.x[:n] - res.x[n:]
    F_lb = huber.objective(A, b, lam, x_lb, lam2=lam2)
    assert F_lb >= sol["F"] - 1e-9 * sol["F"]
    assert abs(F_lb - sol["F"]) <= 1e-6 * sol["F"]
    # weak duality away from the optimum
    x = sol["x"] + 0.05 * np.random.default_rng(2).standard_normal(n)
    gap, pr, du = huber.duality_gap(A, b, lam, x, lam2=lam2)
    assert gap >= huber.objective(A, b, lam, x, lam2=lam2) - sol["F"] - 1e-12


def test_admm_fixed_point_is_the_optimum():
    P = genios_data.huber_outliers(60, seed=4)
    A, b, lam = P["A"], P["b"], P["lam"]
    sol = huber.solve(A, b, lam)
    x, z, u, rho, hist = huber.admm(A, b, lam, rho=1.0, alpha=1.6, sigma=1e-6, max_iter=5000,
                                    eps=1e-11)
    assert np.allclose(z, sol["x"], atol=1e-7)


def test_generator_follows_the_recipe():
    P = genios_data.huber_outliers(400, seed=5)
    A, b = P["A"].astype(np.float64), P["b"].astype(np.float64)
    assert A.shape == (200, 400) and P["s"] == 0 and P["delta"] == 1.0
    assert np.allclose(A.mean(axis=0), 0.0, atol=1e-6)
    assert np.allclose(np.linalg.norm(A, axis=0), 1.0, atol=1e-5)
    assert np.count_nonzero(P["x0"]) == 40
    big = np.abs(b - A @ P["x0"]) > 5.0
    assert big.sum() == 10
    assert abs(P["lam"] - 0.1 * np.max(np.abs(A.T @ b))) <= 1e-6 * P["lam"]


def test_subdifferential_distance_brute_force_and_optimum():
    from oracle import residuals
    rng = np.random.default_rng(9)
    g = rng.standard_normal(12)
    z = np.where(rng.random(12) < 0.5, rng.standard_normal(12), 0.0)
    lam = 0.7
    # brute force: every v in d||z||_1 on a fine grid of [-1, 1] for the zero entries
    grid = np.linspace(-1, 1, 200001)
    best = np.where(z != 0, np.abs(g + lam * np.sign(z)),
                    np.array([np.min(np.abs(gi + lam * grid)) for gi in g]))
    assert abs(residuals.subdifferential_distance(g, z, lam) - np.linalg.norm(best)) <= 1e-5
    P = genios_data.huber_outliers(60, seed=3)
    sol = huber.solve(P["A"], P["b"], P["lam"])
    d = residuals.subdifferential_distance(huber.grad_f(P["A"], P["b"], sol["x"]), sol["x"], P["lam"])
    assert d <= 1e-6 * P["lam"]
