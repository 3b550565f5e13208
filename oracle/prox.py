"""Soft-thresholding: the proximal operator of g(z) = lam*||z||_1 (test infrastructure).

Sec. 3.1 (Lasso example) gives prox_{g/rho}(v)_i elementwise:
    v_i - lam/rho   if v_i >  lam/rho
    0               if |v_i| <= lam/rho
    v_i + lam/rho   if v_i < -lam/rho
Pinned by: the closed form itself on hand-chosen points, the tie |v| = kappa
mapping to zero, and the prox optimality condition (v - z) in kappa*d|z|.
"""
import numpy as np


def soft_threshold(v, kappa):
    """Elementwise S_kappa(v) in the dtype of ``v`` (kappa cast to that dtype)."""
    v = np.asarray(v)
    k = v.dtype.type(kappa)
    out = np.zeros_like(v)
    hi = v > k
    lo = v < -k
    out[hi] = v[hi] - k
    out[lo] = v[lo] + k
    return out
