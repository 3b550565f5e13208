"""Implicit differentiation of the Lasso solution (test infrastructure).

Not in the paper; derived from its optimality conditions (App. A, with
f'(w) = w and the l2 weight lam2 >= 0): on the support S of x* with signs s,
    A_S^T (A_S x*_S - b) + lam2 x*_S + lam s = 0
        =>   x*_S = G^-1 (A_S^T b - lam s),  G = A_S^T A_S + lam2 I,
and x* = 0 off S.  If S and s are locally constant (strict complementarity),
x* is affine in (b, lam) and for a loss L(x*) with gradient g = dL/dx*,
    dL/db   = A_S G^-1 g_S,
    dL/dlam = -s^T G^-1 g_S.
Pinned by central finite differences of L through ``oracle.lasso.solve``:
for L = ||x* - x0||^2 (quadratic in an affine map) the central difference is
exact up to solver error, so agreement is tight (tests/test_oracle_adjoint.py).
"""
import numpy as np
import scipy.linalg as sla


def lasso_adjoint(A, x_star, g, lam2=0.0):
    """Return (dL/db, dL/dlam, w) for the Lasso (elastic-net) solution x_star and g = dL/dx*."""
    A = np.asarray(A, np.float64)
    x_star = np.asarray(x_star, np.float64)
    g = np.asarray(g, np.float64)
    S = np.flatnonzero(x_star != 0)
    m = A.shape[0]
    if S.size == 0:
        return np.zeros(m), 0.0, np.zeros(0)
    s = np.sign(x_star[S])
    AS = A[:, S]
    G = AS.T @ AS + lam2 * np.eye(S.size)
    w = sla.cho_solve(sla.cho_factor(G, lower=True), g[S])
    return AS @ w, -float(s @ w), w


def strict_complementarity_margin(A, b, lam, x_star, lam2=0.0):
    """min over the off-support set of (lam - |A_i^T (A x* - b)|) / lam (>0 means strict);
    off the support x* = 0, so the l2 term does not enter."""
    A = np.asarray(A, np.float64)
    x_star = np.asarray(x_star, np.float64)
    g = A.T @ (A @ x_star - np.asarray(b, np.float64))
    off = x_star == 0
    if not off.any():
        return 1.0
    return float(np.min(lam - np.abs(g[off]))) / lam
