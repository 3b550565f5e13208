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

Stabilised form (the randomized Nystrom algorithm that Sec. 2.2 cites): with
a shift mu >= 0 and Y_mu = H Omega + mu Omega,
    C = chol(sym(Omega^T Y_mu)),  B = Y_mu C^-T = U Sigma V^T (thin SVD),
    Lam_hat = max(Sigma^2 - mu, 0),
i.e. the Nystrom approximation of H + mu I with mu taken back off its
eigenvalues.  Reading (shift size): mu = u ||Y||_F, u the unit roundoff of
the arithmetic that formed Y, the equivalent for a Gaussian Omega of the
published sqrt(n) u ||Y|| for an orthonormal one.  mu = 0 is the plain
definition above when Omega^T H Omega is nonsingular.

Pins (tests/test_oracle_nystrom.py): H_hat = H when rank(H) <= r;
0 <= H_hat <= H (Loewner order); H_hat invariant under Omega -> Omega R;
P^-1 SPD; for rank(H) <= r, P^-1 (H + nu I) has eigenvalues {Lam_rr + nu, nu};
the condition-number bound holds (numpy.linalg.eigvalsh); the stabilised form
at mu = 0 equals the plain one, and at mu > 0 U diag(Lam_hat + mu) U^T is the
dense definition applied to H + mu I.
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


def stabilising_shift(Y, unit_roundoff):
    """mu = u ||Y||_F (reading of the shift size for a Gaussian test matrix)."""
    return float(unit_roundoff) * float(np.linalg.norm(np.asarray(Y, np.float64)))


def nystrom_stabilised(Y, Omega, mu):
    """(U, lam_hat) of the shifted algorithm from the sketch Y = H Omega:
    the Nystrom approximation of H + mu I through a Cholesky factor of
    Omega^T Y_mu and a thin SVD, eigenvalues reduced by mu and clipped at 0."""
    Y = np.asarray(Y, np.float64)
    Omega = np.asarray(Omega, np.float64)
    Ymu = Y + mu * Omega
    M = Omega.T @ Ymu
    M = 0.5 * (M + M.T)
    C = np.linalg.cholesky(M)                  # M = C C^T, C lower triangular
    B = np.linalg.solve(C, Ymu.T).T            # B = Y_mu C^-T
    U, sv, _ = np.linalg.svd(B, full_matrices=False)
    return U, np.maximum(sv ** 2 - mu, 0.0)


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
