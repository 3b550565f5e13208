"""Box-constrained least squares oracle (test infrastructure).

Problem (Sec. 4.5, bounded least squares; the QP form of Sec. 3.2 with
P = A^T A, q = -A^T b, M = I, c = 0):
    minimize (1/2)||A x - b||^2   subject to  lo <= x <= hi
(entries of lo may be -inf and of hi +inf).  Reading: the printed q = A^T b
is the sign of a typo; (1/2) x^T P x + q^T x equals the objective up to a
constant only with q = -A^T b.

What is here
------------
* ``admm``: the ADMM of Sec. 2 for this split, f(x) = (1/2)||Ax - b||^2,
  g(z) = indicator of the box: x-system (P + (rho + sigma) I) x =
  sigma x^k - q + rho (z - u) (Sec. 3.2, solved exactly), over-relaxation,
  z = projection of x_hat + u onto the box (Sec. 3.2), u update, the penalty
  rule of Sec. 2.5.
* ``duality_gap``: Lagrange dual of the split with the residual nu = A x - b:
  g(nu) = -||nu||^2/2 - b^T nu - sum_j s_j(-(A^T nu)_j), s_j(w) = max(lo_j w, hi_j w)
  the support function of the box (+inf where an infinite bound meets a wrong
  sign).  gap = (1/2)||Ax - b||^2 - g(nu) >= F(x) - F* for feasible x.
* ``normal_cone_distance``: ||dist(0, grad f(x) + N_box(x))||_2, the box
  analogue of the subdifferential distance.
* ``solve``: classic ADMM with exact x-steps, then an active-set polish (free
  coordinates solved exactly by least squares with the active bounds fixed,
  accepted when feasible and the KKT signs hold), certified by the gap.
* ``brute_force``: every assignment of {free, at lo, at hi} (n <= 8).

Pins (tests/test_oracle_boxls.py): orthonormal columns give x* = clip(A^T b);
infinite bounds give numpy.linalg.lstsq; brute force; scipy.optimize.lsq_linear
(BVLS); the gap is >= F(x) - F* and ~0 at the optimum; KKT signs; the exact-step
ADMM fixed point.
"""
import itertools

import numpy as np

from .lasso import ShiftedGramSolve
from .residuals import r_kkt


def _f64(a):
    return np.asarray(a, dtype=np.float64)


def _bounds(lo, hi, n):
    lo = np.full(n, -np.inf) if lo is None else np.broadcast_to(_f64(lo), (n,)).copy()
    hi = np.full(n, np.inf) if hi is None else np.broadcast_to(_f64(hi), (n,)).copy()
    return lo, hi


def objective(A, b, x):
    r = _f64(A) @ _f64(x) - _f64(b)
    return 0.5 * float(r @ r)


def grad_f(A, b, x):
    A = _f64(A)
    return A.T @ (A @ _f64(x) - _f64(b))


def project(v, lo, hi):
    return np.minimum(np.maximum(_f64(v), lo), hi)


def admm(A, b, lo, hi, rho=1.0, alpha=1.0, sigma=0.0, max_iter=500, eps=None,
         rho_update_every=0, rho_update_until=500, tau=2.0, mu=10.0):
    A = _f64(A)
    b = _f64(b)
    n = A.shape[1]
    lo, hi = _bounds(lo, hi, n)
    c = A.T @ b  # -q
    x = np.zeros(n)
    z = np.zeros(n)
    u = np.zeros(n)
    hist = []
    solver = ShiftedGramSolve(A, rho + sigma)
    for k in range(1, max_iter + 1):
        x = solver.solve(sigma * x + c + rho * (z - u))
        xh = alpha * x + (1.0 - alpha) * z
        z = project(xh + u, lo, hi)
        u = u + xh - z
        rk, rp, rd = r_kkt(x, z, u, rho, grad_f(A, b, x))
        rho_used = rho
        if rho_update_every > 0 and k % rho_update_every == 0 and k <= rho_update_until:
            new = rho
            if rp > mu * rd:
                new = tau * rho
            elif rd > mu * rp:
                new = rho / tau
            if new != rho:
                u = u * (rho / new)
                rho = new
                solver = ShiftedGramSolve(A, rho + sigma)
        hist.append((k, rp, rd, rk, rho_used, rho))
        if eps is not None and rk <= eps:
            break
    return x, z, u, rho, np.array(hist)


def support_term(w, lo, hi):
    """sum_j max(lo_j w_j, hi_j w_j) (0 * inf = 0: a zero w_j adds nothing)."""
    w = _f64(w)
    with np.errstate(invalid="ignore"):
        a = np.where(w == 0, 0.0, lo * w)
        c = np.where(w == 0, 0.0, hi * w)
    return float(np.sum(np.maximum(a, c)))


def duality_gap(A, b, lo, hi, x):
    """(gap, primal, dual) with nu = A x - b."""
    A = _f64(A)
    b = _f64(b)
    x = _f64(x)
    lo, hi = _bounds(lo, hi, x.size)
    nu = A @ x - b
    primal = 0.5 * float(nu @ nu)
    dual = -0.5 * float(nu @ nu) - float(b @ nu) - support_term(-(A.T @ nu), lo, hi)
    return primal - dual, primal, dual


def relative_gap(A, b, lo, hi, x):
    gap, p, d = duality_gap(A, b, lo, hi, x)
    return gap / min(p, abs(d))


def normal_cone_distance(g, x, lo, hi):
    """||dist(0, g + N_box(x))||_2 for x in the box (g = grad f(x))."""
    g = _f64(g)
    x = _f64(x)
    lo, hi = _bounds(lo, hi, x.size)
    at_lo = x <= lo
    at_hi = x >= hi
    d = np.where(at_lo & at_hi, 0.0,
                 np.where(at_lo, np.maximum(-g, 0.0), np.where(at_hi, np.maximum(g, 0.0), np.abs(g))))
    return float(np.linalg.norm(d))


def _polish(A, b, lo, hi, z, tol):
    """Fix the coordinates at their bounds, solve the rest exactly; None if it fails."""
    n = z.size
    flo, fhi = np.isfinite(lo), np.isfinite(hi)
    with np.errstate(invalid="ignore"):
        return _polish_masked(A, b, lo, hi, z, tol, flo, fhi)


def _polish_masked(A, b, lo, hi, z, tol, flo, fhi):
    at_lo = flo & (z <= np.where(flo, lo + tol * np.maximum(1.0, np.abs(lo)), 0.0))
    at_hi = fhi & (z >= np.where(fhi, hi - tol * np.maximum(1.0, np.abs(hi)), 0.0)) & ~at_lo
    free = ~(at_lo | at_hi)
    x = np.where(at_lo, lo, np.where(at_hi, hi, 0.0))
    if free.any():
        rhs = b - A[:, ~free] @ x[~free]
        x[free] = np.linalg.lstsq(A[:, free], rhs, rcond=None)[0]
    if np.any(flo & (x < np.where(flo, lo - 1e-12 * np.maximum(1.0, np.abs(lo)), 0.0))) or \
            np.any(fhi & (x > np.where(fhi, hi + 1e-12 * np.maximum(1.0, np.abs(hi)), 0.0))):
        return None
    x = project(x, lo, hi)
    g = grad_f(A, b, x)
    scale = max(1.0, float(np.max(np.abs(A.T @ b))))
    if np.any(g[at_lo] < -1e-9 * scale) or np.any(g[at_hi] > 1e-9 * scale):
        return None
    return x


def solve(A, b, lo, hi, rho=1.0, max_iter=20000, gap_rel=1e-13, check_every=25):
    """Certified optimum: classic ADMM with exact steps, polished when it can be."""
    A = _f64(A)
    b = _f64(b)
    n = A.shape[1]
    lo, hi = _bounds(lo, hi, n)
    c = A.T @ b
    x = np.zeros(n)
    z = np.zeros(n)
    u = np.zeros(n)
    solver = ShiftedGramSolve(A, rho)
    best = None
    for k in range(1, max_iter + 1):
        x = solver.solve(c + rho * (z - u))
        z = project(x + u, lo, hi)
        u = u + x - z
        if k % check_every == 0:
            for cand in (_polish(A, b, lo, hi, z, 1e-9), z):
                if cand is None:
                    continue
                gap, F, _ = duality_gap(A, b, lo, hi, cand)
                if best is None or F < best[1]:
                    best = (cand, F, gap, k)
                if gap <= gap_rel * max(F, 1e-300):
                    return dict(x=cand, F=F, gap=gap, iters=k)
    x, F, gap, k = best
    return dict(x=x, F=F, gap=gap, iters=k)


def brute_force(A, b, lo, hi):
    A = _f64(A)
    b = _f64(b)
    n = A.shape[1]
    assert n <= 8
    lo, hi = _bounds(lo, hi, n)
    best = None
    for pat in itertools.product((0, 1, 2), repeat=n):
        pat = np.array(pat)
        if np.any((pat == 1) & ~np.isfinite(lo)) or np.any((pat == 2) & ~np.isfinite(hi)):
            continue
        x = np.where(pat == 1, lo, np.where(pat == 2, hi, 0.0))
        free = pat == 0
        if free.any():
            x[free] = np.linalg.lstsq(A[:, free], b - A[:, ~free] @ x[~free], rcond=None)[0]
        if np.any(x < lo - 1e-12) or np.any(x > hi + 1e-12):
            continue
        F = objective(A, b, x)
        if best is None or F < best[1]:
            best = (x, F)
    return best
