"""Lasso oracle: plain FP64 ADMM with exact x-steps, polish and certificates.

Test infrastructure only (never imported by the product library).

Problem (Sec. 3.1, Lasso example; Sec. 4.1 elastic net with lam2 >= 0, the
ML problem of Sec. 3.3 with the squared loss):
    minimize (1/2)||A x - b||_2^2 + lam ||x||_1 + (lam2/2)||x||_2^2,
split as f(x) = (1/2)||Ax - b||^2 + (lam2/2)||x||^2, g(z) = lam ||z||_1,
M = I, c = 0.  Every function takes lam2 (default 0: the Lasso).

What is here
------------
* ``admm``: the scaled ADMM of Sec. 2 (eqs. x-, z-, u-update) with the
  second-order x-subproblem of eq. x-update-nysadmm, whose linear system is
  eq. x-update-lin-sys.  The right-hand side is formed exactly as printed,
  (H + sigma I) x^k - grad f(x^k) + rho (z^k - u^k) with H = A^T A, and the
  system (H + (rho + sigma) I) x = rhs is solved EXACTLY by Cholesky
  (Woodbury identity when m < n).  Over-relaxation (Sec. 2.5) with parameter
  alpha; the penalty update rule of Sec. 2.5 (tau, mu, every k iterations,
  stopping after a fixed iteration) with u rescaled by rho_old / rho_new.
  With alpha = 1, sigma = 0 this is classic ADMM.
* ``duality_gap``: App. A with loss f(w) = w^2/2, conjugate f*(v) = v^2/2.
  lam2 = 0: the dual point nu = (Ax - b) min(1, lam / ||A^T (Ax - b)||_inf)
  (reading: App. A scales by lam/||.||_inf; scaling by the min keeps the point
  feasible and equals it whenever ||.||_inf >= lam).  lam2 > 0: nu = Ax - b
  and g(nu) = -||nu||^2/2 - b^T nu - (1/(2 lam2)) sum_i ((|A^T nu|_i - lam)_+)^2.
* ``polish``: on the support S of z with signs s, the optimality conditions
  of App. A with f'(w) = w give A_S^T (A_S x_S - b) + lam s = 0; accept if the
  signs agree and |A_i^T (A x - b)| <= lam off S.
* ``brute_force``: enumerates all 3^n sign patterns (n <= 10).
* ``solve``: classic ADMM + polish, certified by the duality gap.

Pins (tests/test_oracle_lasso.py, tests/test_oracle_elastic_net.py):
orthonormal A gives x* = S_lam(A^T b) / (1 + lam2);
brute force at n <= 8; lam >= ||A^T b||_inf gives x* = 0 (App. A); lam -> 0
with m >= n gives numpy.linalg.lstsq; duality gap >= 0 and -> 0; KKT; the
exact-solve ADMM fixed point equals the brute-force optimum.
"""
import itertools

import numpy as np
import scipy.linalg as sla

from .prox import soft_threshold
from .residuals import r_kkt


def _f64(a):
    return np.asarray(a, dtype=np.float64)


def objective(A, b, lam, x, lam2=0.0):
    A = _f64(A)
    x = _f64(x)
    r = A @ x - _f64(b)
    return 0.5 * float(r @ r) + lam * float(np.sum(np.abs(x))) + 0.5 * lam2 * float(x @ x)


def grad_f(A, b, x, lam2=0.0):
    """grad f(x) = A^T (A x - b) + lam2 x  (Sec. 3.1; Sec. 3.3 with lam2)."""
    A = _f64(A)
    x = _f64(x)
    return A.T @ (A @ x - _f64(b)) + lam2 * x


def hessian_vector(A, p, d=None):
    """H p with H = A^T diag(d) A: the Lasso Hessian A^T A (d = None, Sec. 3.1
    HVP example) or the logistic one with curvature weights d (Sec. 3.3).
    Written as two products, A p then A^T (d o A p)."""
    A = _f64(A)
    t = A @ _f64(p)
    if d is not None:
        t = _f64(d) * t
    return A.T @ t


class ShiftedGramSolve:
    """Exact solves with (A^T diag(d) A + nu I); d = None means d = 1.

    m >= n: Cholesky of the n x n matrix.  m < n: Woodbury identity
    (A^T D A + nu I)^-1 v = (v - A^T D^1/2 (nu I + D^1/2 A A^T D^1/2)^-1 D^1/2 A v) / nu.
    """

    def __init__(self, A, nu, d=None):
        A = _f64(A)
        self.A, self.nu = A, float(nu)
        m, n = A.shape
        self.sq = None if d is None else np.sqrt(_f64(d))
        self.wood = m < n
        if self.wood:
            As = A if self.sq is None else self.sq[:, None] * A
            K = As @ As.T
            K[np.diag_indices(m)] += self.nu
            self.c = sla.cho_factor(K, lower=True)
            self.As = As
        else:
            As = A if self.sq is None else self.sq[:, None] * A
            K = As.T @ As
            K[np.diag_indices(n)] += self.nu
            self.c = sla.cho_factor(K, lower=True)

    def solve(self, v):
        v = _f64(v)
        if self.wood:
            y = sla.cho_solve(self.c, self.As @ v)
            return (v - self.As.T @ y) / self.nu
        return sla.cho_solve(self.c, v)


def admm(A, b, lam, rho=1.0, alpha=1.0, sigma=0.0, max_iter=1000, eps=None,
         rho_update_every=0, rho_update_until=500, tau=2.0, mu=10.0,
         x0=None, z0=None, u0=None, record=True, lam2=0.0, clock=None):
    """Scaled ADMM of Sec. 2 with exact x-steps.  Returns (x, z, u, rho, hist).

    hist has one row per iteration k = 1..K:
        (k, ||r_p||, ||r_d||, r_kkt, rho_used, rho_after)
    where r_p = x - z and r_d = grad f(x) + rho u are evaluated at (x^k, z^k, u^k)
    with the rho of that iteration (Sec. 2.3).  If ``eps`` is given the loop
    stops at the first k with r_kkt <= eps.  ``clock`` (a list) receives
    time.perf_counter() stamps: at entry, after the factorisation, after every
    iteration (timing only; the arithmetic is the same).
    """
    import time
    if clock is not None:
        clock.append(time.perf_counter())
    A = _f64(A)
    b = _f64(b)
    m, n = A.shape
    x = np.zeros(n) if x0 is None else _f64(x0).copy()
    z = np.zeros(n) if z0 is None else _f64(z0).copy()
    u = np.zeros(n) if u0 is None else _f64(u0).copy()
    solver = ShiftedGramSolve(A, rho + sigma + lam2)
    if clock is not None:
        clock.append(time.perf_counter())
    hist = []
    for k in range(1, max_iter + 1):
        # eq. x-update-lin-sys with H = A^T A + lam2 I, M = I, c = 0
        Hx = A.T @ (A @ x) + lam2 * x
        g = grad_f(A, b, x, lam2)
        rhs = Hx + sigma * x - g + rho * (z - u)
        x = solver.solve(rhs)
        # over-relaxation (Sec. 2.5), z-update (prox), u-update
        xh = alpha * x + (1.0 - alpha) * z
        z = soft_threshold(xh + u, lam / rho)
        u = u + xh - z
        gx = grad_f(A, b, x, lam2)
        rk, rp, rd = r_kkt(x, z, u, rho, gx)
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
                solver = ShiftedGramSolve(A, rho + sigma + lam2)
        if record:
            hist.append((k, rp, rd, rk, rho_used, rho))
        if clock is not None:
            clock.append(time.perf_counter())
        if eps is not None and rk <= eps:
            break
    return x, z, u, rho, np.array(hist)


def duality_gap(A, b, lam, x, lam2=0.0):
    """(gap, primal, dual) per App. A with f(w) = w^2/2, f*(v) = v^2/2."""
    A = _f64(A)
    b = _f64(b)
    x = _f64(x)
    r = A @ x - b
    primal = objective(A, b, lam, x, lam2)
    if lam2 > 0.0:
        nu = r
        excess = np.maximum(np.abs(A.T @ nu) - lam, 0.0)
        dual = -0.5 * float(nu @ nu) - float(b @ nu) - float(excess @ excess) / (2.0 * lam2)
        return primal - dual, primal, dual
    g = A.T @ r
    ginf = float(np.max(np.abs(g))) if g.size else 0.0
    scale = 1.0 if ginf <= lam else lam / ginf
    nu = scale * r
    dual = -0.5 * float(nu @ nu) - float(b @ nu)
    return primal - dual, primal, dual


def relative_gap(A, b, lam, x, lam2=0.0):
    """The relative duality gap of Sec. 3.3: (l(x) - g(nu)) / min(l(x), |g(nu)|)."""
    gap, p, d = duality_gap(A, b, lam, x, lam2)
    return gap / min(p, abs(d))


def kkt_violation(A, b, lam, x, lam2=0.0):
    """max_i violation of the optimality conditions of App. A, relative to lam."""
    x = _f64(x)
    g = grad_f(A, b, x, lam2)
    on = x != 0
    v = np.where(on, np.abs(g + lam * np.sign(x)), np.maximum(np.abs(g) - lam, 0.0))
    return float(np.max(v)) / lam if v.size else 0.0


def polish(A, b, lam, z, tol=1e-12, lam2=0.0):
    """Solve the KKT system on the support of z; returns x or None if not optimal."""
    A = _f64(A)
    b = _f64(b)
    n = A.shape[1]
    S = np.flatnonzero(np.asarray(z) != 0)
    x = np.zeros(n)
    if S.size == 0:
        g = A.T @ b
        return x if np.max(np.abs(g)) <= lam * (1 + tol) else None
    s = np.sign(np.asarray(z, np.float64)[S])
    AS = A[:, S]
    G = AS.T @ AS + lam2 * np.eye(S.size)
    try:
        c = sla.cho_factor(G, lower=True)
    except np.linalg.LinAlgError:
        return None
    xs = sla.cho_solve(c, AS.T @ b - lam * s)
    if not np.all(np.sign(xs) == s):
        return None
    x[S] = xs
    g = A.T @ (A @ x - b)
    off = np.ones(n, bool)
    off[S] = False
    if off.any() and np.max(np.abs(g[off])) > lam * (1 + 1e-9):
        return None
    return x


def solve(A, b, lam, rhos=(1.0, 0.1, 0.01), iters_per_rho=1500, gap_rel=1e-12,
          check_every=10, lam2=0.0):
    """Certified Lasso optimum: classic ADMM (alpha = 1, sigma = 0), then polish.

    The optimum does not depend on the penalty, so the penalty is lowered
    along ``rhos`` (warm start, u rescaled by rho_old / rho_new) whenever
    ``iters_per_rho`` iterations pass without a certificate; the last penalty
    runs for 10 * iters_per_rho.  A point is accepted when its duality gap is
    at most ``gap_rel`` times its objective.
    Returns dict(x, F, gap, support, signs, iters, polished).
    """
    A = _f64(A)
    b = _f64(b)
    m, n = A.shape
    z = np.zeros(n)
    u = np.zeros(n)
    Atb = A.T @ b
    best = None
    total = 0
    prev = None
    for i, rho in enumerate(rhos):
        if prev is not None:
            u = u * (prev / rho)
        prev = rho
        solver = ShiftedGramSolve(A, rho + lam2)
        budget = iters_per_rho * (10 if i == len(rhos) - 1 else 1)
        for k in range(1, budget + 1):
            total += 1
            x = solver.solve(Atb + rho * (z - u))
            z = soft_threshold(x + u, lam / rho)
            u = u + x - z
            if k % check_every == 0:
                xp = polish(A, b, lam, z, lam2=lam2)
                cand = xp if xp is not None else z
                gap, F, _ = duality_gap(A, b, lam, cand, lam2)
                if gap <= gap_rel * max(F, 1e-300):
                    best = (cand, F, gap, xp is not None, total)
                    break
        if best is not None:
            break
    if best is None:
        gap, F, _ = duality_gap(A, b, lam, z, lam2)
        best = (z, F, gap, False, total)
    cand, F, gap, pol, k = best
    S = np.flatnonzero(cand != 0)
    return dict(x=cand, F=F, gap=gap, support=S, signs=np.sign(cand[S]), iters=k,
                polished=pol)


def rmatvec_rows(A, r, rows=2048):
    """A^T r in FP64 over row blocks of A (A may be FP32; each block is upcast
    exactly), so a matrix of several GB is never copied whole."""
    r = _f64(r)
    out = np.zeros(A.shape[1])
    for i in range(0, A.shape[0], rows):
        out += _f64(A[i:i + rows]).T @ r[i:i + rows]
    return out


def solve_working_set(A, b, lam, gap_rel=1e-12, start=256, grow=256, max_outer=50, lam2=0.0):
    """Certified Lasso optimum of a large problem through a working set W.

    The restricted problem on the columns W is solved by ``solve`` (certified on
    its own), x is that solution padded with zeros, and the full gradient
    g = A^T (A x - b) + lam2 x is formed once.  On W the restricted optimality
    conditions are the full ones; off W they ask |g_j| <= lam (App. A with
    f'(w) = w).  If some j outside W violates that, up to ``grow`` of the worst
    violators join W and the loop repeats; otherwise x is optimal, and the
    duality gap of the full problem (App. A) certifies it.  W starts as the
    ``start`` largest |A^T b|.  Returns the fields of ``solve`` plus the
    working-set size and the number of outer rounds."""
    b = _f64(b)
    n = A.shape[1]
    g0 = rmatvec_rows(A, -b)
    W = np.sort(np.argsort(-np.abs(g0))[:min(n, start)])
    for outer in range(1, max_outer + 1):
        AW = _f64(A[:, W])
        sub = solve(AW, b, lam, gap_rel=min(gap_rel, 1e-13), lam2=lam2)
        x = np.zeros(n)
        x[W] = sub["x"]
        r = AW @ sub["x"] - b
        g = rmatvec_rows(A, r) + lam2 * x
        viol = np.abs(g) - lam * (1.0 + 1e-12)
        viol[W] = -np.inf
        if np.max(viol) > 0.0:
            add = np.argsort(-viol)[:grow]
            add = add[viol[add] > 0.0]
            W = np.union1d(W, add)
            continue
        primal = 0.5 * float(r @ r) + lam * float(np.sum(np.abs(x))) + 0.5 * lam2 * float(x @ x)
        if lam2 > 0.0:
            excess = np.maximum(np.abs(g - lam2 * x) - lam, 0.0)
            dual = -0.5 * float(r @ r) - float(b @ r) - float(excess @ excess) / (2.0 * lam2)
        else:
            ginf = float(np.max(np.abs(g)))
            scale = 1.0 if ginf <= lam else lam / ginf
            nu = scale * r
            dual = -0.5 * float(nu @ nu) - float(b @ nu)
        gap = primal - dual
        S = np.flatnonzero(x != 0)
        return dict(x=x, F=primal, gap=gap, support=S, signs=np.sign(x[S]),
                    iters=sub["iters"], polished=sub["polished"], working_set=int(W.size),
                    outer=outer, certified=bool(gap <= gap_rel * primal))
    raise RuntimeError("working set did not settle")


def brute_force(A, b, lam, lam2=0.0):
    """Enumerate all 3^n sign patterns; returns (x_kkt_list, x_minF, F_min).

    For each pattern s in {-1, 0, +1}^n with support S, solve
    (A_S^T A_S + lam2 I) x_S = A_S^T b - lam s_S; keep sign-consistent candidates.
    """
    A = _f64(A)
    b = _f64(b)
    n = A.shape[1]
    kkt = []
    bestF, bestx = np.inf, None
    for pat in itertools.product((-1.0, 0.0, 1.0), repeat=n):
        s = np.array(pat)
        S = np.flatnonzero(s != 0)
        x = np.zeros(n)
        if S.size:
            AS = A[:, S]
            G = AS.T @ AS + lam2 * np.eye(S.size)
            if np.linalg.matrix_rank(G) < S.size:
                continue
            xs = np.linalg.solve(G, AS.T @ b - lam * s[S])
            if not np.all(np.sign(xs) == s[S]):
                continue
            x[S] = xs
        F = objective(A, b, lam, x, lam2)
        if F < bestF:
            bestF, bestx = F, x
        if kkt_violation(A, b, lam, x, lam2) <= 1e-9:
            kkt.append(x)
    return kkt, bestx, bestF
