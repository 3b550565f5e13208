"""KKT residual used as the accuracy metric (test infrastructure).

Sec. 2.3 (termination criteria) defines, with M = I and c = 0,
    r_p = x - z,      r_d = grad f(x) + rho*u,
and stops when ||r_p|| <= sqrt(n) eps_abs + eps_rel max(||x||, ||z||) and
||r_d|| <= sqrt(n) eps_abs + eps_rel ||rho u||.  With eps_abs = eps_rel = eps
both tests pass iff
    r_kkt = max( ||r_p|| / (sqrt(n) + max(||x||, ||z||)),
                 ||r_d|| / (sqrt(n) + ||rho u||) )  <=  eps.
Reading: the paper's sqrt(m) is the dimension of z, which is n here (M = I).
``grad`` must be the gradient of the smooth part with the true (FP32 or FP64)
data.  Pinned by the identity r_kkt <= eps <=> both tests pass (tested).
"""
import numpy as np


def r_kkt(x, z, u, rho, grad):
    x = np.asarray(x, np.float64)
    z = np.asarray(z, np.float64)
    u = np.asarray(u, np.float64)
    grad = np.asarray(grad, np.float64)
    n = x.size
    rp = np.linalg.norm(x - z)
    rd = np.linalg.norm(grad + rho * u)
    a = rp / (np.sqrt(n) + max(np.linalg.norm(x), np.linalg.norm(z)))
    b = rd / (np.sqrt(n) + np.linalg.norm(rho * u))
    return max(a, b), rp, rd


def paper_stop_test(x, z, u, rho, grad, eps_abs, eps_rel):
    """The two inequalities of Sec. 2.3 written out as stated (M = I, c = 0)."""
    x = np.asarray(x, np.float64)
    z = np.asarray(z, np.float64)
    u = np.asarray(u, np.float64)
    n = x.size
    rp = np.linalg.norm(x - z)
    rd = np.linalg.norm(np.asarray(grad, np.float64) + rho * u)
    ok_p = rp <= np.sqrt(n) * eps_abs + eps_rel * max(np.linalg.norm(x), np.linalg.norm(z), 0.0)
    ok_d = rd <= np.sqrt(n) * eps_abs + eps_rel * np.linalg.norm(rho * u)
    return bool(ok_p and ok_d)


def subgradient_residual(g, z, lam):
    """Iterate-free optimality residual of an l1 problem at z, relative to lam.

    v_i = g_i + lam*sign(z_i) on the support, max(|g_i| - lam, 0) off it, where
    g is the gradient of the smooth part at z; returns ||v||_inf / lam.
    """
    g = np.asarray(g, np.float64)
    z = np.asarray(z, np.float64)
    on = z != 0
    v = np.where(on, g + lam * np.sign(z), np.maximum(np.abs(g) - lam, 0.0))
    return float(np.max(np.abs(v))) / lam


def subdifferential_distance(g, z, lam):
    """dist(0, g + lam d||z||_1) in the l2 norm: the stopping criterion of the Huber
    comparison (Sec. 4.3), with g the gradient of the smooth part at z.  Per entry
    the closest point of g_i + lam [-1, 1] (z_i = 0) or g_i + lam sign(z_i) to 0."""
    g = np.asarray(g, np.float64)
    z = np.asarray(z, np.float64)
    on = z != 0
    v = np.where(on, g + lam * np.sign(z), np.maximum(np.abs(g) - lam, 0.0))
    return float(np.linalg.norm(v))
