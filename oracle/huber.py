"""l1-regularised Huber fitting oracle (test infrastructure).

Problem (Sec. 4.3, Huber fitting, in the ML form of Sec. 3.3):
    minimize sum_i l(a_i^T x - b_i) + lam ||x||_1 + (lam2/2)||x||^2,
    l(w) = w^2 for |w| <= delta,  2 delta |w| - delta^2 otherwise
(delta = 1 is the paper's loss), so that
    l'(w)  = 2 clip(w, -delta, delta),   l''(w) = 2 [|w| <= delta],
    l*(v)  = v^2 / 4 on |v| <= 2 delta (+inf outside)  (App. A's conjugate).

What is here
------------
* ``loss``, ``dloss``, ``d2loss``: the loss and its derivatives, elementwise.
* ``objective``, ``grad_f``, ``hess_diag``.
* ``admm``: GeNIOS's ADMM for ML problems (Sec. 3.3): the x-system
  (A^T D_k A + (rho + sigma + lam2) I) x = (A^T D_k A + sigma I) x^k - grad f(x^k)
  + rho (z - u) + lam2 x^k - lam2 x^k, D_k = l''(A x^k - b), solved exactly;
  z, u, over-relaxation and residuals as for the Lasso.
* ``duality_gap``: App. A with l*; lam2 = 0: nu = l'(r) min(1, lam / ||A^T l'(r)||_inf)
  (|nu_i| <= 2 delta stays in the conjugate's domain); lam2 > 0: nu = l'(r) and
  the dual gains -(1/(2 lam2)) ||(|A^T nu| - lam)_+||^2.
* ``solve``: classic ADMM with the exact x-prox (damped Newton on the
  piecewise-quadratic objective), certified by the duality gap.

Pins (tests/test_oracle_huber.py): the loss is C^1 with the stated
derivatives (finite differences) and conjugate (grid supremum); for a delta
above every residual the problem is twice the Lasso at lam / 2 (lasso.solve);
KKT at the optimum; agreement with L-BFGS-B on the split form; the gap
certifies suboptimality.
"""
import numpy as np

from .lasso import ShiftedGramSolve
from .prox import soft_threshold
from .residuals import r_kkt


def _f64(a):
    return np.asarray(a, dtype=np.float64)


def loss(w, delta=1.0):
    w = _f64(w)
    a = np.abs(w)
    return np.where(a <= delta, w * w, 2.0 * delta * a - delta * delta)


def dloss(w, delta=1.0):
    return 2.0 * np.clip(_f64(w), -delta, delta)


def d2loss(w, delta=1.0):
    return np.where(np.abs(_f64(w)) <= delta, 2.0, 0.0)


def objective(A, b, lam, x, delta=1.0, lam2=0.0):
    x = _f64(x)
    r = _f64(A) @ x - _f64(b)
    return (float(np.sum(loss(r, delta))) + lam * float(np.sum(np.abs(x))) +
            0.5 * lam2 * float(x @ x))


def grad_f(A, b, x, delta=1.0, lam2=0.0):
    A = _f64(A)
    x = _f64(x)
    return A.T @ dloss(A @ x - _f64(b), delta) + lam2 * x


def hess_diag(A, b, x, delta=1.0):
    return d2loss(_f64(A) @ _f64(x) - _f64(b), delta)


def _newton_prox(A, b, rho, v, x0, delta=1.0, lam2=0.0, tol=1e-13, max_newton=200):
    """argmin_x f(x) + (rho/2)||x - v||^2 by damped Newton with Armijo backtracking."""
    A = _f64(A)
    x = _f64(x0).copy()

    def phi(xx):
        return (float(np.sum(loss(A @ xx - b, delta))) + 0.5 * lam2 * float(xx @ xx) +
                0.5 * rho * float((xx - v) @ (xx - v)))

    for _ in range(max_newton):
        g = grad_f(A, b, x, delta, lam2) + rho * (x - v)
        if np.linalg.norm(g) <= tol * max(1.0, np.linalg.norm(x)):
            break
        d = hess_diag(A, b, x, delta)
        step = -ShiftedGramSolve(A, rho + lam2, d).solve(g)
        t, f0, slope = 1.0, phi(x), float(g @ step)
        while phi(x + t * step) > f0 + 1e-4 * t * slope and t > 1e-12:
            t *= 0.5
        x = x + t * step
    return x


def admm(A, b, lam, rho=1.0, alpha=1.0, sigma=0.0, max_iter=500, eps=None, delta=1.0,
         lam2=0.0, rho_update_every=0, rho_update_until=500, tau=2.0, mu=10.0):
    """ADMM of Sec. 2 / Sec. 3.3 (one Newton-type x-step per iteration)."""
    A = _f64(A)
    b = _f64(b)
    n = A.shape[1]
    x = np.zeros(n)
    z = np.zeros(n)
    u = np.zeros(n)
    hist = []
    for k in range(1, max_iter + 1):
        d = hess_diag(A, b, x, delta)
        g = grad_f(A, b, x, delta, lam2)
        Hx = A.T @ (d * (A @ x)) + lam2 * x
        rhs = Hx + sigma * x - g + rho * (z - u)
        x = ShiftedGramSolve(A, rho + sigma + lam2, d).solve(rhs)
        xh = alpha * x + (1.0 - alpha) * z
        z = soft_threshold(xh + u, lam / rho)
        u = u + xh - z
        rk, rp, rd = r_kkt(x, z, u, rho, grad_f(A, b, x, delta, lam2))
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
        hist.append((k, rp, rd, rk, rho_used, rho))
        if eps is not None and rk <= eps:
            break
    return x, z, u, rho, np.array(hist)


def duality_gap(A, b, lam, x, delta=1.0, lam2=0.0):
    """(gap, primal, dual) per App. A with l*(v) = v^2 / 4 on [-2 delta, 2 delta]."""
    A = _f64(A)
    b = _f64(b)
    x = _f64(x)
    r = A @ x - b
    f1 = dloss(r, delta)
    primal = objective(A, b, lam, x, delta, lam2)
    if lam2 > 0.0:
        nu = f1
        excess = np.maximum(np.abs(A.T @ nu) - lam, 0.0)
        dual = -0.25 * float(nu @ nu) - float(b @ nu) - float(excess @ excess) / (2.0 * lam2)
        return primal - dual, primal, dual
    g = A.T @ f1
    ginf = float(np.max(np.abs(g))) if g.size else 0.0
    nu = (1.0 if ginf <= lam else lam / ginf) * f1
    dual = -0.25 * float(nu @ nu) - float(b @ nu)
    return primal - dual, primal, dual


def relative_gap(A, b, lam, x, delta=1.0, lam2=0.0):
    gap, p, d = duality_gap(A, b, lam, x, delta, lam2)
    return gap / min(p, abs(d))


def kkt_violation(A, b, lam, x, delta=1.0, lam2=0.0):
    x = _f64(x)
    g = grad_f(A, b, x, delta, lam2)
    on = x != 0
    v = np.where(on, np.abs(g + lam * np.sign(x)), np.maximum(np.abs(g) - lam, 0.0))
    return float(np.max(v)) / lam


def solve(A, b, lam, delta=1.0, lam2=0.0, rho=1.0, max_iter=20000, gap_rel=1e-12,
          check_every=5):
    """Certified optimum by classic ADMM with the exact x-prox."""
    A = _f64(A)
    b = _f64(b)
    n = A.shape[1]
    x = np.zeros(n)
    z = np.zeros(n)
    u = np.zeros(n)
    out = None
    for k in range(1, max_iter + 1):
        x = _newton_prox(A, b, rho, z - u, x, delta, lam2)
        z = soft_threshold(x + u, lam / rho)
        u = u + x - z
        if k % check_every == 0:
            gap, F, _ = duality_gap(A, b, lam, z, delta, lam2)
            if gap <= gap_rel * F:
                out = (z, F, gap, k)
                break
    if out is None:
        gap, F, _ = duality_gap(A, b, lam, z, delta, lam2)
        out = (z, F, gap, max_iter)
    z, F, gap, k = out
    return dict(x=z, F=F, gap=gap, iters=k)
