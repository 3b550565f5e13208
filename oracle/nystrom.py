"""Randomized Nystrom approximation and preconditioner (test infrastructure).

Sec. 2.2: for a PSD matrix H (the paper's "A" in that section; here
H = A^T A for the Lasso or A^T D A for logistic regression) and a test matrix
Omega in R^{n x r},
    H_hat = (H Omega)(Omega^T H Omega)^+ (H Omega)^T = U Lam_hat U^T,
with U orthonormal and Lam_hat diagonal.  The preconditioner for H + nu I is
(eq. preconditioner)
    P^-1 = (Lam_hat_rr + nu) U (Lam_hat + nu I)^-1 U^T + I - U U^T,
and Prop. 5.3 of the cited preconditioning paper (quoted in Sec. 2.2) bounds
    kappa(P^-1/2 (H + nu I) P^-1/2) <= 1 + (Lam_hat_rr + ||E||) / nu,  E = H - H_hat.

Reading (pseudo-inverse): eigenvalues of Omega^T H Omega below
``rel_thresh`` times the largest are treated as zero.  Lam_hat_rr is the
smallest retained eigenvalue (Lam_hat sorted descending).

Pins (tests/test_oracle_nystrom.py): H_hat = H when rank(H) <= r;
0 <= H_hat <= H (Loewner order); H_hat invariant under Omega -> Omega R;
P^-1 SPD; for rank(H) <= r, P^-1 (H + nu I) has eigenvalues {Lam_rr + nu, nu};
the condition-number bound holds (numpy.linalg.eigvalsh).
"""
import numpy as np


def nystrom(H, Omega, rel_thresh=1e-12):
    """Return (U, lam_hat) with H_hat = U diag(lam_hat) U^T, lam_hat descending."""
    H = np.asarray(H, np.float64)
    return nystrom_from_sketch(H @ np.asarray(Omega, np.float64), Omega, rel_thresh)


def nystrom_from_sketch(Y, Omega, rel_thresh=1e-12):
    """The same (U, lam_hat) from the sketch Y = H Omega alone (H never formed)."""
    Y = np.asarray(Y, np.float64)
    Omega = np.asarray(Omega, np.float64)
    Mm = Omega.T @ Y
    Mm = 0.5 * (Mm + Mm.T)
    ev, V = np.linalg.eigh(Mm)
    keep = ev > rel_thresh * max(ev.max(), 0.0) if ev.max() > 0 else np.zeros_like(ev, bool)
    if not keep.any():
        return np.zeros((Y.shape[0], 0)), np.zeros(0)
    # H_hat = Y V_k diag(1/ev_k) V_k^T Y^T = B B^T with B = Y V_k diag(ev_k^-1/2)
    B = (Y @ V[:, keep]) / np.sqrt(ev[keep])
    Ub, sv, _ = np.linalg.svd(B, full_matrices=False)
    return Ub, sv ** 2


def nystrom_dense(H, Omega, rel_thresh=1e-12):
    """H_hat as a dense n x n matrix, written as the definition Y (Omega^T Y)^+ Y^T."""
    H = np.asarray(H, np.float64)
    Omega = np.asarray(Omega, np.float64)
    Y = H @ Omega
    Mm = Omega.T @ Y
    Mm = 0.5 * (Mm + Mm.T)
    ev, V = np.linalg.eigh(Mm)
    inv = np.zeros_like(ev)
    pos = ev > rel_thresh * max(ev.max(), 0.0)
    inv[pos] = 1.0 / ev[pos]
    return Y @ (V * inv) @ V.T @ Y.T


def preconditioner(U, lam_hat, nu):
    """Dense P^-1 of eq. preconditioner (identity when the sketch is empty)."""
    U = np.asarray(U, np.float64)
    n = U.shape[0]
    if U.shape[1] == 0:
        return np.eye(n)
    lam_hat = np.asarray(lam_hat, np.float64)
    lrr = lam_hat[-1]
    return (lrr + nu) * (U / (lam_hat + nu)) @ U.T + np.eye(n) - U @ U.T


def apply_preconditioner(U, lam_hat, nu, r):
    """P^-1 r without forming P^-1: (lrr+nu) U (Lam+nu)^-1 U^T r + r - U U^T r."""
    U = np.asarray(U, np.float64)
    r = np.asarray(r, np.float64)
    if U.shape[1] == 0:
        return r.copy()
    lam_hat = np.asarray(lam_hat, np.float64)
    w = U.T @ r
    return (lam_hat[-1] + nu) * (U @ (w / (lam_hat + nu))) + r - U @ w


def kappa_bound(lam_hat, E_norm, nu):
    """1 + (Lam_rr + ||E||)/nu (Sec. 2.2, adaptive sketch size paragraph)."""
    lrr = lam_hat[-1] if len(lam_hat) else 0.0
    return 1.0 + (lrr + E_norm) / nu


def solve_shifted(H, nu, r):
    """Reference solution of (H + nu I) x = r (numpy.linalg.solve)."""
    H = np.asarray(H, np.float64)
    return np.linalg.solve(H + nu * np.eye(H.shape[0]), np.asarray(r, np.float64))
