"""Pins for the elastic-net extension of the Lasso oracle (lam2 > 0).

The problem is (1/2)||Ax - b||^2 + lam ||x||_1 + (lam2/2)||x||^2 (Sec. 4.1;
App. A with lam2 > 0)."""
import numpy as np
import pytest

from oracle import lasso
from oracle.prox import soft_threshold


def _data(m, n, seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n)) / np.sqrt(m)
    x0 = np.zeros(n)
    x0[rng.choice(n, max(1, n // 5), replace=False)] = rng.standard_normal(max(1, n // 5))
    b = A @ x0 + 0.05 * rng.standard_normal(m)
    return A, b


def test_orthonormal_design_closed_form():
    # A^T A = I: the objective separates, x* = S_lam(A^T b) / (1 + lam2)
    rng = np.random.default_rng(1)
    Q, _ = np.linalg.qr(rng.standard_normal((30, 12)))
    b = rng.standard_normal(30)
    lam, lam2 = 0.3, 0.7
    sol = lasso.solve(Q, b, lam, lam2=lam2)
    ref = soft_threshold(Q.T @ b, lam) / (1.0 + lam2)
    assert np.allclose(sol["x"], ref, atol=1e-10)


@pytest.mark.parametrize("seed", [2, 3])
def test_brute_force_agrees_with_solve(seed):
    A, b = _data(9, 6, seed)
    lam = 0.2 * np.max(np.abs(A.T @ b))
    lam2 = 0.4
    kkt, xb, Fb = lasso.brute_force(A, b, lam, lam2)
    assert len(kkt) == 1  # strictly convex: one KKT point
    sol = lasso.solve(A, b, lam, lam2=lam2)
    assert np.allclose(sol["x"], xb, atol=1e-9)
    assert abs(sol["F"] - Fb) <= 1e-12 * abs(Fb)


def test_gap_is_a_certificate():
    A, b = _data(40, 25, 4)
    lam = 0.1 * np.max(np.abs(A.T @ b))
    lam2 = 0.2
    sol = lasso.solve(A, b, lam, lam2=lam2)
    gap, p, d = lasso.duality_gap(A, b, lam, sol["x"], lam2)
    assert abs(gap) <= 1e-10 * p
    rng = np.random.default_rng(5)
    for scale in (1e-3, 1e-1, 1.0):
        x = sol["x"] + scale * rng.standard_normal(25)
        gap, p, d = lasso.duality_gap(A, b, lam, x, lam2)
        F = lasso.objective(A, b, lam, x, lam2)
        assert p == F
        assert gap >= F - sol["F"] - 1e-12 >= -1e-12  # weak duality: g(nu) <= F*


def test_admm_fixed_point_is_the_optimum():
    A, b = _data(30, 50, 6)
    lam = 0.1 * np.max(np.abs(A.T @ b))
    lam2 = 0.3
    sol = lasso.solve(A, b, lam, lam2=lam2)
    x, z, u, rho, hist = lasso.admm(A, b, lam, rho=1.0, alpha=1.6, sigma=1e-6, max_iter=3000,
                                    eps=1e-12, lam2=lam2)
    assert np.allclose(z, sol["x"], atol=1e-8)


def test_lam2_zero_is_the_lasso():
    A, b = _data(20, 15, 7)
    lam = 0.1 * np.max(np.abs(A.T @ b))
    x = np.random.default_rng(8).standard_normal(15)
    assert lasso.objective(A, b, lam, x, 0.0) == lasso.objective(A, b, lam, x)
    assert lasso.duality_gap(A, b, lam, x, 0.0) == lasso.duality_gap(A, b, lam, x)


def test_adjoint_with_l2_matches_central_differences():
    # L = ||x* - x0||^2: x* is affine in (b, lam) on a fixed support, so central
    # differences of the certified solution map are exact up to solver error
    from oracle import adjoint
    A, b = _data(30, 12, 9)
    lam = 0.15 * np.max(np.abs(A.T @ b))
    lam2 = 0.25
    x0 = np.random.default_rng(10).standard_normal(12)
    sol = lasso.solve(A, b, lam, lam2=lam2)
    assert adjoint.strict_complementarity_margin(A, b, lam, sol["x"]) > 1e-3
    gb, gl, _ = adjoint.lasso_adjoint(A, sol["x"], 2.0 * (sol["x"] - x0), lam2)
    L = lambda bb, ll: float(np.sum((lasso.solve(A, bb, ll, lam2=lam2)["x"] - x0) ** 2))
    h = 1e-4
    for i in (0, 5, 17):
        e = np.zeros(30)
        e[i] = h
        fd = (L(b + e, lam) - L(b - e, lam)) / (2 * h)
        assert abs(fd - gb[i]) <= 1e-6 * (1 + abs(gb[i]))
    fdl = (L(b, lam + h) - L(b, lam - h)) / (2 * h)
    assert abs(fdl - gl) <= 1e-6 * (1 + abs(gl))
