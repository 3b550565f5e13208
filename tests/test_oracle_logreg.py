"""Pins for the logistic-regression oracle."""
import numpy as np
import pytest
from scipy.optimize import minimize

import genios_data
from oracle import logreg


def _data(m, n, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n))
    x0 = np.zeros(n)
    x0[: max(1, n // 5)] = rng.standard_normal(max(1, n // 5))
    p = 1 / (1 + np.exp(-A @ x0))
    y = np.where(rng.random(m) < p, 1.0, -1.0)
    return A, y


def test_gradient_and_hessian_by_finite_differences():
    A, y = _data(30, 6, 0)
    rng = np.random.default_rng(1)
    x = rng.standard_normal(6) * 0.3
    f = lambda v: logreg.objective(A, y, 0.0, v)
    g = logreg.grad_f(A, y, x)
    h = 1e-6
    for i in range(6):
        e = np.zeros(6)
        e[i] = h
        assert abs((f(x + e) - f(x - e)) / (2 * h) - g[i]) <= 1e-6 * max(1, abs(g[i]))
    d = logreg.hess_diag(A, y, x)
    H = A.T @ (d[:, None] * A)
    for i in range(6):
        e = np.zeros(6)
        e[i] = h
        col = (logreg.grad_f(A, y, x + e) - logreg.grad_f(A, y, x - e)) / (2 * h)
        assert np.allclose(col, H[:, i], atol=1e-6)


def test_zero_solution_threshold():
    A, y = _data(40, 8, 2)
    lmax = np.max(np.abs(A.T @ y)) / 2
    assert np.all(logreg.solve(A, y, lmax * 1.001)["x"] == 0)
    assert np.any(logreg.solve(A, y, lmax * 0.9)["x"] != 0)


def _lbfgs_split(A, y, lam):
    n = A.shape[1]

    def fun(w):
        x = w[:n] - w[n:]
        marg = -y * (A @ x)
        val = np.sum(np.logaddexp(0, marg)) + lam * np.sum(w)
        s = 1 / (1 + np.exp(-marg))
        g = A.T @ (-y * s)
        return val, np.concatenate([g + lam, -g + lam])

    res = minimize(fun, np.zeros(2 * n), jac=True, method="L-BFGS-B",
                   bounds=[(0, None)] * (2 * n),
                   options=dict(maxiter=20000, ftol=1e-15, gtol=1e-12))
    return res.fun


@pytest.mark.parametrize("seed", [3, 4])
def test_matches_lbfgsb_split_reformulation(seed):
    A, y = _data(60, 10, seed)
    lam = 0.2 * np.max(np.abs(A.T @ y)) / 2
    sol = logreg.solve(A, y, lam)
    Fl = _lbfgs_split(A, y, lam)
    assert sol["F"] <= Fl + 1e-9 * abs(Fl)
    assert abs(sol["F"] - Fl) <= 1e-7 * abs(Fl)
    assert sol["gap"] <= 1e-11 * sol["F"]
    assert logreg.kkt_violation(A, y, lam, sol["x"]) <= 1e-6


def test_gap_bounds_suboptimality():
    A, y = _data(50, 12, 5)
    lam = 0.1 * np.max(np.abs(A.T @ y)) / 2
    Fstar = logreg.solve(A, y, lam)["F"]
    rng = np.random.default_rng(6)
    for _ in range(20):
        x = rng.standard_normal(12) * rng.random()
        gap, F, d = logreg.duality_gap(A, y, lam, x)
        assert gap >= 0 and F - Fstar <= gap + 1e-10 and d <= Fstar + 1e-10


def test_genios_second_order_admm_reaches_optimum():
    A, y = _data(80, 10, 7)
    lam = 0.1 * np.max(np.abs(A.T @ y)) / 2
    sol = logreg.solve(A, y, lam)
    x, z, u, rho, hist = logreg.admm(A, y, lam, rho=1.0, alpha=1.6, sigma=1e-6,
                                     max_iter=2000, eps=1e-11, xstep="approx")
    assert abs(logreg.objective(A, y, lam, z) - sol["F"]) <= 1e-9 * sol["F"]
    assert np.allclose(z, sol["x"], atol=1e-6)


def test_relative_gap_bounds_relative_suboptimality():
    # (l(x) - g(nu)) / min(l(x), |g(nu)|) >= (l(x) - l*) / min(l(x), |g(nu)|) >= 0
    P = genios_data.logreg_factor(300, 30, nnz_frac=0.1, seed=3, s=5)
    sol = logreg.solve(P["A"], P["y"], P["lam"])
    rng = np.random.default_rng(4)
    for scale in (0.0, 1e-3, 1e-1):
        x = sol["x"] + scale * rng.standard_normal(sol["x"].size)
        gap, pr, du = logreg.duality_gap(P["A"], P["y"], P["lam"], x)
        rel = logreg.relative_gap(P["A"], P["y"], P["lam"], x)
        assert rel == gap / min(pr, abs(du))
        assert rel >= (logreg.objective(P["A"], P["y"], P["lam"], x) - sol["F"]) / min(pr, abs(du)) - 1e-12
        assert rel >= -1e-12


def test_l2_term_optimum_satisfies_kkt_and_matches_lbfgs():
    # lam2 > 0: the certified optimum satisfies App. A's conditions and agrees with
    # L-BFGS-B on the split (x+, x-) >= 0 form with the l2 term
    P = genios_data.logreg_factor(300, 30, nnz_frac=0.1, seed=3, s=5)
    A, y, lam, lam2 = P["A"], P["y"], P["lam"], 0.5
    sol = logreg.solve(A, y, lam, lam2=lam2)
    assert logreg.kkt_violation(A, y, lam, sol["x"], lam2) <= 1e-5
    gap, pr, du = logreg.duality_gap(A, y, lam, sol["x"], lam2)
    assert 0.0 <= gap <= 1e-8 * pr
    n = A.shape[1]

    def fun(v):
        xp, xm = v[:n], v[n:]
        x = xp - xm
        w = logreg.margins(A, y, x)
        g = logreg.grad_f(A, y, x, lam2)
        f = float(np.sum(np.logaddexp(0.0, w))) + lam * float(np.sum(v)) + 0.5 * lam2 * float(x @ x)
        return f, np.concatenate([g + lam, -g + lam])
    res = minimize(fun, np.zeros(2 * n), jac=True, method="L-BFGS-B",
                   bounds=[(0, None)] * (2 * n), options=dict(maxiter=5000, ftol=1e-15, gtol=1e-12))
    x_lb = res.x[:n] - res.x[n:]
    assert logreg.objective(A, y, lam, x_lb, lam2) >= sol["F"] - 1e-9
    assert abs(logreg.objective(A, y, lam, x_lb, lam2) - sol["F"]) <= 1e-6 * sol["F"]
    # weak duality away from the optimum
    x = sol["x"] + 0.1 * np.random.default_rng(1).standard_normal(n)
    gap, pr, du = logreg.duality_gap(A, y, lam, x, lam2)
    assert gap >= logreg.objective(A, y, lam, x, lam2) - sol["F"] - 1e-12
