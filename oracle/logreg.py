"""l1-logistic regression oracle (test infrastructure).

Problem (Sec. 4.2, in the machine-learning form of Sec. 3.3):
    minimize sum_i l(w_i) + lam ||x||_1,   l(w) = log(1 + e^w),   w_i = -y_i a_i^T x,
with labels y_i in {-1, +1}.  Reading: the data are generated with
P(y = +1 | a) = sigmoid(a^T x0), so the per-sample margin is w_i = -y_i a_i^T x
(the paper's form with x replaced by -x); y is folded into the vectors.

With rows a~_i = -y_i a_i (the paper's a_i = b_i a_i), f(x) = sum l(a~_i^T x),
    grad f(x)   = A^T (-y o l'(w)),          l'(w)  = sigmoid(w)
    Hess f(x)   = A^T diag(l''(w)) A,        l''(w) = sigmoid(w)(1 - sigmoid(w))
(Sec. 3.3, gradient and Hessian of the ML objective).

What is here
------------
* ``admm``: GeNIOS's ADMM for ML problems (Sec. 3.3): the x-system
  (A^T D_k A + (rho + sigma) I) x = (A^T D_k A + sigma I) x^k - grad f(x^k) + rho (z^k - u^k)
  (eq. x-update-lin-sys; reading: the sign of the rho-term follows the general
  form, the ML display has a sign typo), solved exactly (Cholesky / Woodbury);
  or, with ``xstep='exact'``, the classic ADMM x-step minimised by damped
  Newton.  z- and u-updates, over-relaxation and residuals as for the Lasso.
* ``duality_gap``: App. A with f*(v) = v log v + (1 - v) log(1 - v) on [0, 1]
  and the dual point nu = sigmoid(w) min(1, lam / ||A^T (y o sigmoid(w))||_inf).
* ``solve``: classic exact-x-step ADMM certified by the duality gap.

Pins (tests/test_oracle_logreg.py): lam >= ||A^T y||_inf / 2 gives x* = 0
(App. A with f'(0) = 1/2); KKT with f' = sigmoid; gap >= 0 and -> 0;
agreement with scipy's L-BFGS-B on the split (x+, x-) >= 0 reformulation.
"""
import numpy as np
import scipy.linalg as sla
from scipy.special import expit, xlogy

from .lasso import ShiftedGramSolve
from .prox import soft_threshold
from .residuals import r_kkt


def _f64(a):
    return np.asarray(a, dtype=np.float64)


def margins(A, y, x):
    return -_f64(y) * (_f64(A) @ _f64(x))


def objective(A, y, lam, x, lam2=0.0):
    """sum_i l(w_i) + lam ||x||_1 + (lam2/2)||x||^2 (Sec. 3.3 with the l2 term)."""
    x = _f64(x)
    w = margins(A, y, x)
    return (float(np.sum(np.logaddexp(0.0, w))) + lam * float(np.sum(np.abs(x))) +
            0.5 * lam2 * float(x @ x))


def grad_f(A, y, x, lam2=0.0):
    x = _f64(x)
    w = margins(A, y, x)
    return _f64(A).T @ (-_f64(y) * expit(w)) + lam2 * x


def hess_diag(A, y, x):
    s = expit(margins(A, y, x))
    return s * (1.0 - s)


def _newton_prox(A, y, rho, v, x0, tol=1e-12, max_newton=100, lam2=0.0, dec_rel=1e-20):
    """argmin_x f(x) + (rho/2)||x - v||^2 by damped Newton with Armijo backtracking.

    Stops when ||grad|| <= tol max(1, ||x||) or when the Newton decrement
    g^T H^-1 g / 2 falls to dec_rel max(1, |phi(x)|) (the textbook criterion,
    Boyd and Vandenberghe, Sec. 9.5): with curvature of 1e3 and more the gradient
    norm bottoms out near 1e-12 in FP64, above an absolute tolerance, while the
    decrement keeps measuring the distance to the minimiser in objective terms."""
    A = _f64(A)
    x = _f64(x0).copy()

    def phi(xx):
        w = margins(A, y, xx)
        return (float(np.sum(np.logaddexp(0.0, w))) + 0.5 * lam2 * float(xx @ xx) +
                0.5 * rho * float((xx - v) @ (xx - v)))

    for _ in range(max_newton):
        g = grad_f(A, y, x, lam2) + rho * (x - v)
        if np.linalg.norm(g) <= tol * max(1.0, np.linalg.norm(x)):
            break
        d = hess_diag(A, y, x)
        step = -ShiftedGramSolve(A, rho + lam2, d).solve(g)
        t, f0, slope = 1.0, phi(x), float(g @ step)
        if -0.5 * slope <= dec_rel * max(1.0, abs(f0)):
            x = x + step
            break
        while phi(x + t * step) > f0 + 1e-4 * t * slope and t > 1e-12:
            t *= 0.5
        x = x + t * step
    return x


def admm(A, y, lam, rho=1.0, alpha=1.0, sigma=0.0, max_iter=500, eps=None,
         xstep="approx", rho_update_every=0, rho_update_until=500, tau=2.0, mu=10.0,
         lam2=0.0):
    """ADMM of Sec. 2 / Sec. 3.3 for l1-logistic; returns (x, z, u, rho, hist)."""
    A = _f64(A)
    y = _f64(y)
    m, n = A.shape
    x = np.zeros(n)
    z = np.zeros(n)
    u = np.zeros(n)
    hist = []
    for k in range(1, max_iter + 1):
        if xstep == "approx":
            d = hess_diag(A, y, x)
            g = grad_f(A, y, x, lam2)
            Hx = A.T @ (d * (A @ x)) + lam2 * x
            rhs = Hx + sigma * x - g + rho * (z - u)
            x = ShiftedGramSolve(A, rho + sigma + lam2, d).solve(rhs)
        else:
            x = _newton_prox(A, y, rho, z - u, x, lam2=lam2)
        xh = alpha * x + (1.0 - alpha) * z
        z = soft_threshold(xh + u, lam / rho)
        u = u + xh - z
        rk, rp, rd = r_kkt(x, z, u, rho, grad_f(A, y, x, lam2))
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


def duality_gap(A, y, lam, x, lam2=0.0):
    """(gap, primal, dual): App. A with the logistic conjugate h(v) = v log v +
    (1 - v) log(1 - v).  lam2 = 0: nu = s min(1, lam / ||A^T (y o s)||_inf);
    lam2 > 0: nu = s and g(nu) = -sum h(nu_i) - (1/(2 lam2)) ||(|A^T (y o nu)| - lam)_+||^2
    (s = sigmoid of the margins; the folded rows -y_i a_i make A~^T nu = -A^T (y o nu))."""
    A = _f64(A)
    y = _f64(y)
    w = margins(A, y, x)
    s = expit(w)
    primal = objective(A, y, lam, x, lam2)
    if lam2 > 0.0:
        nu = s
        excess = np.maximum(np.abs(A.T @ (y * nu)) - lam, 0.0)
        dual = (-float(np.sum(xlogy(nu, nu) + xlogy(1.0 - nu, 1.0 - nu))) -
                float(excess @ excess) / (2.0 * lam2))
        return primal - dual, primal, dual
    g = A.T @ (y * s)
    ginf = float(np.max(np.abs(g)))
    scale = 1.0 if ginf <= lam else lam / ginf
    nu = scale * s
    dual = -float(np.sum(xlogy(nu, nu) + xlogy(1.0 - nu, 1.0 - nu)))
    return primal - dual, primal, dual


def relative_gap(A, y, lam, x, lam2=0.0):
    """The relative duality gap of Sec. 3.3: (l(x) - g(nu)) / min(l(x), |g(nu)|)."""
    gap, p, d = duality_gap(A, y, lam, x, lam2)
    return gap / min(p, abs(d))


def kkt_violation(A, y, lam, x, lam2=0.0):
    x = _f64(x)
    g = grad_f(A, y, x, lam2)
    on = x != 0
    v = np.where(on, np.abs(g + lam * np.sign(x)), np.maximum(np.abs(g) - lam, 0.0))
    return float(np.max(v)) / lam


def polish(A, y, lam, z, lam2=0.0, max_newton=50):
    """Newton on the support S of z with the signs s = sign(z_S) held fixed.

    On the right support the optimality conditions of App. A (with f' = sigmoid)
    read A_S^T (-y o sigmoid(w)) + lam s + lam2 x_S = 0, the stationarity of the
    smooth, strictly convex function sum_i l(w_i) + lam s^T x_S + (lam2/2)||x_S||^2
    of x_S alone, so its minimiser is x*_S.  Returns the full vector (zeros off
    S) or None when the signs do not survive; the caller certifies it by the gap."""
    A = _f64(A)
    y = _f64(y)
    S = np.flatnonzero(_f64(z))
    if S.size == 0:
        return None
    s = np.sign(_f64(z)[S])
    AS = A[:, S]
    xs = _f64(z)[S].copy()

    def phi(v):
        w = -y * (AS @ v)
        return float(np.sum(np.logaddexp(0.0, w))) + lam * float(s @ v) + 0.5 * lam2 * float(v @ v)

    for _ in range(max_newton):
        w = -y * (AS @ xs)
        sg = expit(w)
        g = AS.T @ (-y * sg) + lam * s + lam2 * xs
        Hs = AS.T @ ((sg * (1.0 - sg))[:, None] * AS)
        Hs[np.diag_indices(S.size)] += lam2
        step = -sla.cho_solve(sla.cho_factor(Hs, lower=True), g)
        t, f0, slope = 1.0, phi(xs), float(g @ step)
        if -0.5 * slope <= 1e-20 * max(1.0, abs(f0)):
            xs = xs + step
            break
        while phi(xs + t * step) > f0 + 1e-4 * t * slope and t > 1e-12:
            t *= 0.5
        xs = xs + t * step
    if np.any(np.sign(xs) != s):
        return None
    x = np.zeros(A.shape[1])
    x[S] = xs
    return x


def solve(A, y, lam, rho=1.0, max_iter=5000, gap_rel=1e-12, check_every=5, lam2=0.0,
          polish_below=1e-2):
    """Certified optimum: classic ADMM (exact Newton x-step, fixed rho) and, once
    the relative gap is below polish_below, a support polish (``polish``) that is
    kept only if its own duality gap meets gap_rel; the ADMM continues otherwise.
    Returns x, F, gap, iters and whether the certified point came from the polish."""
    A = _f64(A)
    y = _f64(y)
    n = A.shape[1]
    x = np.zeros(n)
    z = np.zeros(n)
    u = np.zeros(n)
    out = None
    for k in range(1, max_iter + 1):
        x = _newton_prox(A, y, rho, z - u, x, lam2=lam2)
        z = soft_threshold(x + u, lam / rho)
        u = u + x - z
        if k % check_every == 0:
            gap, F, _ = duality_gap(A, y, lam, z, lam2)
            if gap <= gap_rel * F:
                out = (z, F, gap, k, False)
                break
            if gap <= polish_below * F:
                xp = polish(A, y, lam, z, lam2)
                if xp is not None:
                    gp, Fp, _ = duality_gap(A, y, lam, xp, lam2)
                    if gp <= gap_rel * Fp:
                        out = (xp, Fp, gp, k, True)
                        break
    if out is None:
        gap, F, _ = duality_gap(A, y, lam, z, lam2)
        out = (z, F, gap, max_iter, False)
    z, F, gap, k, pol = out
    return dict(x=z, F=F, gap=gap, iters=k, polished=pol)


def _rmatvec_rows(A, r, rows=2048):
    """A^T r in FP64 over row blocks (A may be FP32; each block upcast exactly)."""
    r = _f64(r)
    out = np.zeros(A.shape[1])
    for i in range(0, A.shape[0], rows):
        out += _f64(A[i:i + rows]).T @ r[i:i + rows]
    return out


def solve_working_set(A, y, lam, gap_rel=1e-12, start=256, grow=256, max_outer=50, lam2=0.0):
    """Certified optimum of a large problem through a working set W of columns.

    The problem restricted to W is solved by ``solve`` (its own penalty set to the
    mean eigenvalue of the restricted Hessian at 0, ||A_W||_F^2 / (4 |W|): the
    optimum does not depend on it), x is that solution padded with zeros and the
    full gradient g = A^T (-y o sigmoid(w)) + lam2 x is formed once.  On W the
    restricted optimality conditions are the full ones; off W they ask
    |g_j| <= lam (App. A with f' = sigmoid).  Violators (up to ``grow``, worst
    first) join W and the loop repeats; otherwise the duality gap of the full
    problem (App. A, entropy conjugate) certifies x.  W starts as the ``start``
    largest |A^T y|."""
    y = _f64(y)
    n = A.shape[1]
    g0 = _rmatvec_rows(A, y)
    W = np.sort(np.argsort(-np.abs(g0))[:min(n, start)])
    for outer in range(1, max_outer + 1):
        AW = _f64(A[:, W])
        rho = float(np.sum(AW * AW)) / (4.0 * W.size)
        sub = solve(AW, y, lam, rho=rho, gap_rel=min(gap_rel, 1e-13), lam2=lam2)
        x = np.zeros(n)
        x[W] = sub["x"]
        w = -y * (AW @ sub["x"])
        sg = expit(w)
        g = _rmatvec_rows(A, -y * sg) + lam2 * x
        viol = np.abs(g) - lam * (1.0 + 1e-12)
        viol[W] = -np.inf
        if np.max(viol) > 0.0:
            add = np.argsort(-viol)[:grow]
            add = add[viol[add] > 0.0]
            W = np.union1d(W, add)
            continue
        primal = (float(np.sum(np.logaddexp(0.0, w))) + lam * float(np.sum(np.abs(x))) +
                  0.5 * lam2 * float(x @ x))
        aty = -(g - lam2 * x)          # A^T (y o sigmoid(w))
        if lam2 > 0.0:
            excess = np.maximum(np.abs(aty) - lam, 0.0)
            dual = (-float(np.sum(xlogy(sg, sg) + xlogy(1.0 - sg, 1.0 - sg))) -
                    float(excess @ excess) / (2.0 * lam2))
        else:
            ginf = float(np.max(np.abs(aty)))
            nu = sg * (1.0 if ginf <= lam else lam / ginf)
            dual = -float(np.sum(xlogy(nu, nu) + xlogy(1.0 - nu, 1.0 - nu)))
        gap = primal - dual
        return dict(x=x, F=primal, gap=gap, iters=sub["iters"], polished=sub["polished"],
                    working_set=int(W.size), outer=outer, certified=bool(gap <= gap_rel * primal))
    raise RuntimeError("working set did not settle")
