"""Pins for the box-constrained least squares oracle (Sec. 4.5, Sec. 3.2)."""
import numpy as np
import pytest
from scipy.optimize import lsq_linear

import genios_data
from oracle import boxls


def test_orthonormal_columns_clip_the_unconstrained_solution():
    rng = np.random.default_rng(1)
    Q, _ = np.linalg.qr(rng.standard_normal((40, 12)))
    b = 2.0 * rng.standard_normal(40)
    sol = boxls.solve(Q, b, 0.0, 1.0)
    assert np.allclose(sol["x"], np.clip(Q.T @ b, 0.0, 1.0), atol=1e-10)


def test_infinite_bounds_give_lstsq():
    rng = np.random.default_rng(2)
    A = rng.standard_normal((30, 10))
    b = rng.standard_normal(30)
    sol = boxls.solve(A, b, None, None)
    assert np.allclose(sol["x"], np.linalg.lstsq(A, b, rcond=None)[0], atol=1e-9)


@pytest.mark.parametrize("seed", [3, 4, 5])
def test_brute_force_small(seed):
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((12, 6))
    b = 3.0 * rng.standard_normal(12)
    lo = np.array([0.0, -1.0, -np.inf, 0.0, -0.5, 0.0])
    hi = np.array([1.0, 1.0, 0.5, np.inf, 0.5, 0.2])
    sol = boxls.solve(A, b, lo, hi)
    x_bf, F_bf = boxls.brute_force(A, b, lo, hi)
    assert np.allclose(sol["x"], x_bf, atol=1e-9)
    assert abs(sol["F"] - F_bf) <= 1e-10 * max(1.0, F_bf)


def test_matches_bvls_and_certificates():
    P = genios_data.boxls_decay(240, 120, seed=3)
    A, b = P["A"].astype(np.float64), P["b"].astype(np.float64)
    sol = boxls.solve(A, b, 0.0, 1.0)
    ref = lsq_linear(A, b, bounds=(0.0, 1.0), method="bvls", tol=1e-14)
    assert np.allclose(sol["x"], ref.x, atol=1e-8)
    gap, pr, du = boxls.duality_gap(A, b, 0.0, 1.0, sol["x"])
    assert 0.0 <= gap <= 1e-10 * pr
    g = boxls.grad_f(A, b, sol["x"])
    assert boxls.normal_cone_distance(g, sol["x"], np.zeros(120), np.ones(120)) <= 1e-8
    # a real mix of active and free coordinates
    assert 10 < np.sum((sol["x"] == 0) | (sol["x"] == 1)) < 110
    # weak duality at feasible points away from the optimum
    x = np.clip(sol["x"] + 0.1 * np.random.default_rng(0).standard_normal(120), 0, 1)
    gap, pr, du = boxls.duality_gap(A, b, 0.0, 1.0, x)
    assert gap >= pr - sol["F"] - 1e-12


def test_admm_fixed_point_is_the_optimum():
    P = genios_data.boxls_decay(120, 60, seed=4)
    A, b = P["A"], P["b"]
    sol = boxls.solve(A, b, 0.0, 1.0)
    x, z, u, rho, hist = boxls.admm(A, b, 0.0, 1.0, rho=1.0, alpha=1.6, sigma=1e-6,
                                    max_iter=20000, eps=1e-12)
    assert np.allclose(z, sol["x"], atol=1e-7)


def test_generator_recipe():
    P = genios_data.boxls_decay(400, 200, seed=5)
    assert P["A"].shape == (400, 200) and P["kind"] == "boxls"
    assert np.all(P["lo"] == 0.0) and np.all(P["hi"] == 1.0)
