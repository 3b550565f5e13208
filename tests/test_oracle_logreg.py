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


def test_newton_prox_converges_under_large_curvature():
    # the shared factor gives curvature of 1e4 and more: the gradient norm of the
    # prox objective bottoms out near 1e-12 in FP64, so the decrement criterion
    # has to end the Newton loop; the result is still the prox point
    P = genios_data.logreg_factor(1500, 120, nnz_frac=0.05, seed=11, s=8)
    A, y = P["A"].astype(np.float64), P["y"].astype(np.float64)
    rho = P["rho"]
    v = np.random.default_rng(1).standard_normal(A.shape[1]) * 0.1
    x = logreg._newton_prox(A, y, rho, v, np.zeros(A.shape[1]))
    g = logreg.grad_f(A, y, x) + rho * (x - v)
    g0 = logreg.grad_f(A, y, np.zeros(A.shape[1])) + rho * (0 - v)
    assert np.linalg.norm(g) <= 1e-12 * np.linalg.norm(g0)


def test_working_set_solve_equals_the_plain_solve():
    P = genios_data.logreg_factor(600, 200, nnz_frac=0.05, seed=12, s=8)
    ref = logreg.solve(P["A"], P["y"], P["lam"], rho=P["rho"])
    ws = logreg.solve_working_set(P["A"], P["y"], P["lam"], start=16, grow=8)
    assert ws["certified"] and ws["outer"] >= 2          # the working set had to grow
    assert abs(ws["F"] - ref["F"]) <= 1e-12 * ref["F"]
    assert np.max(np.abs(ws["x"] - ref["x"])) <= 1e-8 * np.max(np.abs(ref["x"]))
    assert np.array_equal(np.flatnonzero(ws["x"]), np.flatnonzero(ref["x"]))
    gap, F, _ = logreg.duality_gap(P["A"], P["y"], P["lam"], ws["x"])
    assert gap <= 1e-11 * F and logreg.kkt_violation(P["A"], P["y"], P["lam"], ws["x"]) <= 1e-8


def test_polish_on_the_right_support_is_certified_and_on_a_wrong_one_rejected():
    P = genios_data.logreg_factor(600, 200, nnz_frac=0.05, seed=12, s=8)
    A, y, lam = P["A"], P["y"], P["lam"]
    ref = logreg.solve(A, y, lam, rho=P["rho"])
    # an inexact point with the optimum's support and signs
    z = ref["x"] * (1.0 + 0.01 * np.random.default_rng(2).standard_normal(200))
    xp = logreg.polish(A, y, lam, z)
    gap, F, _ = logreg.duality_gap(A, y, lam, xp)
    assert gap <= 1e-11 * F and abs(F - ref["F"]) <= 1e-12 * ref["F"]
    # dropping the largest coefficient leaves a support whose polished point the gap rejects
    zw = ref["x"].copy()
    zw[np.argmax(np.abs(zw))] = 0.0
    xw = logreg.polish(A, y, lam, zw)
    assert xw is None or logreg.duality_gap(A, y, lam, xw)[0] > 1e-6 * F


def test_penalty_at_the_mean_curvature_converges_where_rho_one_stalls():
    # The workload's reading of the initial penalty: rho = ||A||_F^2 / (4 n), the
    # mean eigenvalue of A^T D A at x = 0.  With the shared factor the whole
    # Hessian spectrum lies far above 1; at rho = 1 the residual-balancing rule
    # of Sec. 2.5 never fires (the residuals stay within a factor mu of each
    # other) and GeNIOS's ADMM creeps; at the mean curvature it converges.
    P = genios_data.logreg_factor(2000, 500, nnz_frac=0.02, seed=4, s=20)
    A, y, lam = P["A"].astype(np.float64), P["y"].astype(np.float64), P["lam"]
    d0 = logreg.hess_diag(A, y, np.zeros(500))
    ev = np.linalg.eigvalsh(A.T @ (d0[:, None] * A))
    assert ev[0] > 50.0 and abs(P["rho"] - ev.mean()) <= 1e-9 * ev.mean()
    kw = dict(alpha=1.6, sigma=1e-6, rho_update_every=25, eps=1e-4)
    _, _, _, rho1, h1 = logreg.admm(A, y, lam, rho=1.0, max_iter=150, **kw)
    assert h1[-1, 3] > 1e-3 and rho1 == 1.0                   # stalled, rule silent
    at = h1[h1[:, 0] % 25 == 0]                                # the rule's iterations
    assert np.all(np.maximum(at[:, 1] / at[:, 2], at[:, 2] / at[:, 1]) < 10.0)
    _, z, _, _, h = logreg.admm(A, y, lam, rho=P["rho"], max_iter=150, **kw)
    assert h[-1, 3] <= 1e-4 and len(h) <= 60
    ref = logreg.solve(A, y, lam, rho=P["rho"])
    assert abs(logreg.objective(A, y, lam, z) - ref["F"]) <= 1e-5 * ref["F"]
