"""Seeded synthetic problem generators shared by the oracle tests and the GPU path.

This module holds data generation only: it draws matrices, sparse ground-truth
vectors, noise and labels, and evaluates the regularisation level that the
workload recipe asks for.  It contains none of the solver's arithmetic (no ADMM,
no conjugate gradient, no sketch, no proximal step).

Every array is drawn with numpy's PCG64 ``default_rng`` in a fixed order:
base matrix (in row chunks, each chunk with its own child stream so large
matrices can be drawn by several threads), support indices, values, noise,
labels.  The FP32 matrix is the master copy that every precision solves; FP64
consumers use its exact upcast.  ``b`` is formed in FP64 from the FP32 matrix
and rounded once to FP32; ``lam`` is formed in FP64 from the rounded ``b``.

Workload recipes (the paper's datasets are not available; these synthetic
problems stand in for their shapes):

* ``lasso_small``   - Lasso, A m x n iid N(0, 1/m), k nonzeros of +-1,
                      noise 0.01, lam = 0.1 ||A^T b||_inf   (200 x 1000, s = 20).
* ``lasso_decay``   - Lasso, A = G diag(j^-1/2), G iid N(0, 1/m), k nonzeros
                      N(0,1), noise 0.1, lam = 0.05 ||A^T b||_inf.
                      (1000 x 10000, s = 50; 20000 x 40000, s = 100;
                      2000 x 8000 per problem for the batched adjoint workload.)
* ``logreg_factor`` - l1-logistic regression, A = Z + F G^T / sqrt(20) with
                      Z, F, G iid N(0,1) (a rank-20 shared factor), x0 with
                      2 % nonzeros N(0, 1/k), y_i = +1 with probability
                      sigmoid(a_i^T x0), lam = 0.05 ||A^T y||_inf / 2, and
                      the initial penalty rho = ||A||_F^2 / (4 n), the mean
                      eigenvalue of the logistic Hessian A^T D A at x = 0
                      (D = 1/4).  The paper runs its logistic experiment at
                      rho = 1 on rows of unit norm, where this mean is about 1;
                      these rows have squared norm about 2n, and at rho = 1 the
                      penalty sits three orders of magnitude below the whole
                      Hessian spectrum.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor

import numpy as np

CHUNK_ROWS = 1000

# Stream identifiers inside one seed.
_STREAM_MISC = 0
_STREAM_MATRIX = 1
_STREAM_FACTOR = 2


def _threads() -> int:
    n = os.cpu_count() or 1
    return max(1, min(16, n))


def _gaussian_rows(seed: int, stream: int, m: int, n: int) -> np.ndarray:
    """m x n iid N(0,1) float32, drawn in CHUNK_ROWS-row chunks (thread parallel)."""
    out = np.empty((m, n), dtype=np.float32)
    nchunks = (m + CHUNK_ROWS - 1) // CHUNK_ROWS

    def fill(c: int) -> None:
        r0 = c * CHUNK_ROWS
        r1 = min(m, r0 + CHUNK_ROWS)
        rng = np.random.default_rng([seed, stream, c])
        rng.standard_normal((r1 - r0, n), dtype=np.float32, out=out[r0:r1])

    if nchunks == 1:
        fill(0)
    else:
        with ThreadPoolExecutor(_threads()) as ex:
            list(ex.map(fill, range(nchunks)))
    return out


def _scale_columns_inplace(G: np.ndarray, col_scale: np.ndarray) -> np.ndarray:
    """A = float32(float64(G) * col_scale), row chunk by row chunk (thread parallel)."""
    m = G.shape[0]
    nchunks = (m + CHUNK_ROWS - 1) // CHUNK_ROWS

    def work(c: int) -> None:
        r0 = c * CHUNK_ROWS
        r1 = min(m, r0 + CHUNK_ROWS)
        G[r0:r1] = (G[r0:r1].astype(np.float64) * col_scale[None, :]).astype(np.float32)

    if nchunks == 1:
        work(0)
    else:
        with ThreadPoolExecutor(_threads()) as ex:
            list(ex.map(work, range(nchunks)))
    return G


def matvec_f64(A: np.ndarray, v: np.ndarray) -> np.ndarray:
    """A @ v in FP64 for an FP32 (or FP64) A, chunked so the FP64 copy stays small."""
    m = A.shape[0]
    v = np.asarray(v, dtype=np.float64)
    out = np.empty(m, dtype=np.float64)
    step = 2048
    for r0 in range(0, m, step):
        out[r0:r0 + step] = A[r0:r0 + step].astype(np.float64) @ v
    return out


def rmatvec_f64(A: np.ndarray, w: np.ndarray) -> np.ndarray:
    """A^T @ w in FP64 for an FP32 (or FP64) A, chunked over rows."""
    m, n = A.shape
    w = np.asarray(w, dtype=np.float64)
    out = np.zeros(n, dtype=np.float64)
    step = 2048
    for r0 in range(0, m, step):
        out += A[r0:r0 + step].astype(np.float64).T @ w[r0:r0 + step]
    return out


def lasso_small(m: int = 200, n: int = 1000, k: int = 20, noise: float = 0.01,
                lam_frac: float = 0.1, seed: int = 1, s: int = 20) -> dict:
    """Lasso with iid N(0, 1/m) features and a +-1 sparse ground truth."""
    G = _gaussian_rows(seed, _STREAM_MATRIX, m, n)
    A = _scale_columns_inplace(G, np.full(n, 1.0 / math.sqrt(m)))
    rng = np.random.default_rng([seed, _STREAM_MISC])
    supp = np.sort(rng.choice(n, size=min(k, n), replace=False))
    x0 = np.zeros(n)
    x0[supp] = rng.choice(np.array([-1.0, 1.0]), size=supp.size)
    e = rng.standard_normal(m)
    b64 = A[:, supp].astype(np.float64) @ x0[supp] + noise * e
    b = b64.astype(np.float32)
    lam = lam_frac * float(np.max(np.abs(rmatvec_f64(A, b))))
    return dict(kind="lasso", A=A, b=b, lam=lam, x0=x0, s=s, rho=1.0,
                name=f"lasso_small_{m}x{n}")


def lasso_decay(m: int, n: int, k: int, noise: float = 0.1, lam_frac: float = 0.05,
                seed: int = 2, s: int = 50) -> dict:
    """Lasso with A = G diag(j^-1/2), G iid N(0, 1/m): decaying spectrum of A^T A."""
    G = _gaussian_rows(seed, _STREAM_MATRIX, m, n)
    j = np.arange(1, n + 1, dtype=np.float64)
    A = _scale_columns_inplace(G, j ** -0.5 / math.sqrt(m))
    rng = np.random.default_rng([seed, _STREAM_MISC])
    supp = np.sort(rng.choice(n, size=min(k, n), replace=False))
    x0 = np.zeros(n)
    x0[supp] = rng.standard_normal(supp.size)
    e = rng.standard_normal(m)
    b64 = A[:, supp].astype(np.float64) @ x0[supp] + noise * e
    b = b64.astype(np.float32)
    lam = lam_frac * float(np.max(np.abs(rmatvec_f64(A, b))))
    return dict(kind="lasso", A=A, b=b, lam=lam, x0=x0, s=s, rho=1.0,
                name=f"lasso_decay_{m}x{n}")


def logreg_factor(m: int = 20000, n: int = 5000, nnz_frac: float = 0.02, rank: int = 20,
                  lam_frac: float = 0.05, seed: int = 4, s: int = 50) -> dict:
    """l1-logistic data: iid N(0,1) features plus a rank-`rank` shared factor."""
    Z = _gaussian_rows(seed, _STREAM_MATRIX, m, n)
    F = _gaussian_rows(seed, _STREAM_FACTOR, m, rank).astype(np.float64)
    rngf = np.random.default_rng([seed, _STREAM_FACTOR, 10 ** 6])
    Gf = rngf.standard_normal((n, rank))
    A = np.empty((m, n), dtype=np.float32)
    for r0 in range(0, m, CHUNK_ROWS):
        r1 = min(m, r0 + CHUNK_ROWS)
        A[r0:r1] = (Z[r0:r1].astype(np.float64) + F[r0:r1] @ Gf.T / math.sqrt(rank)).astype(np.float32)
    del Z
    rng = np.random.default_rng([seed, _STREAM_MISC])
    k = max(1, int(round(nnz_frac * n)))
    supp = np.sort(rng.choice(n, size=k, replace=False))
    x0 = np.zeros(n)
    x0[supp] = rng.standard_normal(k) / math.sqrt(k)
    margin = A[:, supp].astype(np.float64) @ x0[supp]
    p = 1.0 / (1.0 + np.exp(-margin))
    y = np.where(rng.random(m) < p, 1.0, -1.0).astype(np.float32)
    lam = lam_frac * float(np.max(np.abs(rmatvec_f64(A, y)))) / 2.0
    fro2 = 0.0
    for r0 in range(0, m, CHUNK_ROWS):
        blk = A[r0:r0 + CHUNK_ROWS].astype(np.float64)
        fro2 += float(np.sum(blk * blk))
    rho = fro2 / (4.0 * n)
    return dict(kind="logreg", A=A, y=y, lam=lam, x0=x0, s=s, rho=rho,
                name=f"logreg_factor_{m}x{n}")


def huber_outliers(n: int = 2000, seed: int = 6, s: int = 0) -> dict:
    """Huber-fitting data (the paper's recipe): N = n/2 samples of n iid N(0, 1)
    features, columns centred and scaled to unit l2 norm; x0 with 10 % N(0, 1)
    nonzeros; b = A x0 + 0.1 v, then 5 % of the entries shifted by +-10;
    lam = 0.1 ||A^T b||_inf.  s = 0: the paper runs this problem unpreconditioned."""
    m = n // 2
    G = _gaussian_rows(seed, _STREAM_MATRIX, m, n).astype(np.float64)
    G -= G.mean(axis=0, keepdims=True)
    G /= np.linalg.norm(G, axis=0, keepdims=True)
    A = G.astype(np.float32)
    del G
    rng = np.random.default_rng([seed, _STREAM_MISC])
    k = max(1, n // 10)
    supp = np.sort(rng.choice(n, size=k, replace=False))
    x0 = np.zeros(n)
    x0[supp] = rng.standard_normal(k)
    b64 = A[:, supp].astype(np.float64) @ x0[supp] + 0.1 * rng.standard_normal(m)
    out = np.sort(rng.choice(m, size=max(1, m // 20), replace=False))
    b64[out] += rng.choice(np.array([-10.0, 10.0]), size=out.size)
    b = b64.astype(np.float32)
    lam = 0.1 * float(np.max(np.abs(rmatvec_f64(A, b))))
    return dict(kind="huber", A=A, b=b, lam=lam, x0=x0, s=s, rho=1.0, delta=1.0,
                name=f"huber_{m}x{n}")


def boxls_decay(m: int = 20000, n: int = 10000, seed: int = 8, s: int = 50,
                noise: float = 0.01, scale: float = 10.0) -> dict:
    """Bounded least squares data: A = scale G diag(j^-1/2) / sqrt(m) with G iid N(0, 1)
    (a dense matrix with a decaying spectrum, top eigenvalue of A^T A ~ scale^2, N = m
    samples and n = N/2 features in the paper's runs), x0 ~ U(-0.5, 1.5)^n,
    b = A x0 + noise N(0, 1); bounds 0 <= x <= 1."""
    G = _gaussian_rows(seed, _STREAM_MATRIX, m, n)
    j = np.arange(1, n + 1, dtype=np.float64)
    A = _scale_columns_inplace(G, scale * j ** -0.5 / math.sqrt(m))
    rng = np.random.default_rng([seed, _STREAM_MISC])
    x0 = rng.uniform(-0.5, 1.5, size=n)
    b = (matvec_f64(A, x0) + noise * rng.standard_normal(m)).astype(np.float32)
    return dict(kind="boxls", A=A, b=b, lo=np.zeros(n), hi=np.ones(n), x0=x0, s=s, rho=1.0,
                lam=0.0, name=f"boxls_{m}x{n}")


def lasso_batch(batch: int = 64, m: int = 2000, n: int = 8000, k: int = 80,
                seed0: int = 5000, s: int = 50) -> dict:
    """`batch` independent decaying-spectrum Lasso problems, problem j seeded seed0 + j."""
    probs = [lasso_decay(m, n, k, noise=0.1, lam_frac=0.05, seed=seed0 + j, s=s)
             for j in range(batch)]
    A = np.stack([p["A"] for p in probs])
    b = np.stack([p["b"] for p in probs])
    lam = np.array([p["lam"] for p in probs])
    x0 = np.stack([p["x0"] for p in probs])
    return dict(kind="lasso_batch", A=A, b=b, lam=lam, x0=x0, s=s, rho=1.0,
                name=f"lasso_batch_{batch}x{m}x{n}")


# The five workloads, by name.
def config(name: str) -> dict:
    if name == "lasso_200x1000":
        return lasso_small(200, 1000, 20, 0.01, 0.1, seed=1, s=20)
    if name == "lasso_1000x10000":
        return lasso_decay(1000, 10000, 100, 0.1, 0.05, seed=2, s=50)
    if name == "lasso_20000x40000":
        return lasso_decay(20000, 40000, 400, 0.1, 0.05, seed=3, s=100)
    if name == "logreg_20000x5000":
        return logreg_factor(20000, 5000, 0.02, 20, 0.05, seed=4, s=50)
    if name == "lasso_batch_64x2000x8000":
        return lasso_batch(64, 2000, 8000, 80, 5000, s=50)
    raise KeyError(name)


WORKLOADS = ("lasso_200x1000", "lasso_1000x10000", "lasso_20000x40000",
             "logreg_20000x5000", "lasso_batch_64x2000x8000")


def gaussian_test_matrix(n: int, s: int, seed: int) -> np.ndarray:
    """A seeded n x s standard-normal FP32 test matrix, for callers that pass Omega in."""
    rng = np.random.default_rng([seed, 7])
    return rng.standard_normal((n, s)).astype(np.float32)
