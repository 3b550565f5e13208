"""Adaptive sketch size for the Nystrom preconditioner (test infrastructure).

Sec. 2.2, adaptive sketch size selection: the preconditioned x-system has
    kappa <= 1 + (Lam_hat_rr + ||E||) / nu,   E = H - H_hat,
so the sketch is grown from a small size until that bound is small enough or the
size reaches its cap.  Lam_hat_rr comes with the sketch; ||E|| is estimated by
a few steps of the randomized power method (the method the paper cites from the
randomized linear algebra survey): from a Gaussian start v, repeat
w = E v, theta = v^T w, v = w / ||w||, and report the last theta.  E is
positive semidefinite (H_hat <= H), so theta is a lower estimate of ||E|| that
converges to it.

Readings (the paper gives no numbers): the sizes double, r0, 2 r0, 4 r0, ...
capped at r_max; the target is kappa_target (bound <= target stops); the
test matrix of size r is the first r columns of the Philox matrix of size
r_max (column-major draw order), so a larger sketch extends the smaller one;
the power method starts from the Philox vector with stream id
POWER_STREAM + problem.  The Nystrom step is the stabilised form of
oracle.nystrom with the shift u ||Y||_F, eigenpairs with Lam_hat_j <=
rel_thresh Lam_hat_1 dropped (Lam_hat_rr is the smallest one kept).

Pins (tests/test_oracle_adaptive.py): the power estimate is <= the exact
||E|| (numpy.linalg.eigvalsh) and converges to it; the bound with the exact
||E|| holds for the chosen sketch (eigvalsh of the preconditioned matrix);
the chosen size is the first size of the schedule whose bound meets the target
(each size evaluated on its own); an exactly rank-k H with k <= r0 stops at r0
with ||E|| ~ 0.
"""
import numpy as np

from . import nystrom, philox

POWER_STREAM = 0x706F776572  # stream id of the power method's start vectors


def power_norm(apply_E, v0, q):
    """Randomized power method: q products with E from v0; the last Rayleigh quotient."""
    v = np.asarray(v0, np.float64)
    nv = np.linalg.norm(v)
    if nv == 0.0:
        return 0.0
    v = v / nv
    theta = 0.0
    for _ in range(q):
        w = apply_E(v)
        theta = float(v @ w)
        nw = np.linalg.norm(w)
        if nw == 0.0:
            return 0.0
        v = w / nw
    return theta


def sketch_at(H, Omega, unit_roundoff, rel_thresh):
    """Stabilised Nystrom of H from the test matrix Omega, small eigenpairs dropped."""
    Y = np.asarray(H, np.float64) @ Omega
    mu = nystrom.stabilising_shift(Y, unit_roundoff)
    U, lam = nystrom.nystrom_stabilised(Y, Omega, mu)
    keep = lam > rel_thresh * lam[0] if lam.size and lam[0] > 0 else np.zeros(lam.size, bool)
    return U[:, keep], lam[keep]


def adaptive_sketch(H, nu, r0, r_max, kappa_target, q, seed, problem=0,
                    unit_roundoff=2.0 ** -24, rel_thresh=1e-6):
    """Doubling rule of Sec. 2.2.  Returns dict(rank, U, lam, err, bound, history)."""
    H = np.asarray(H, np.float64)
    n = H.shape[0]
    Om_full = philox.gaussian_matrix(n, r_max, seed, problem).astype(np.float64)
    v0 = philox.gaussian_matrix(n, 1, seed, POWER_STREAM + problem)[:, 0].astype(np.float64)
    r = min(r0, r_max)
    hist = []
    while True:
        U, lam = sketch_at(H, Om_full[:, :r], unit_roundoff, rel_thresh)
        err = power_norm(lambda v: H @ v - U @ (lam * (U.T @ v)), v0, q)
        bound = nystrom.kappa_bound(lam, err, nu)
        hist.append((r, lam.size, lam[-1] if lam.size else 0.0, err, bound))
        if bound <= kappa_target or r >= r_max:
            return dict(rank=r, U=U, lam=lam, err=err, bound=bound, history=hist)
        r = min(2 * r, r_max)
