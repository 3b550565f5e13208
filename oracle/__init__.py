"""CPU FP64 oracle for the GeNIOS inexact-ADMM hot path (test infrastructure).

This package is test infrastructure only.  It is a plain, slow, obviously
correct NumPy/SciPy FP64 restatement of what the GPU library computes, written
from the paper (Diamandis, Frangella, Zhao, Stellato, Udell, "GeNIOS: an
(almost) second-order operator-splitting solver for large-scale convex
optimization", 2023).  Only the test-suite, the smoke check and the
benchmark's CPU-baseline leg may import it; the product library never does,
and this package imports nothing from the product library.

Modules
-------
prox       soft-thresholding, the prox of lam*||.||_1 (Sec. 3.1, Lasso example)
lasso      Lasso objective, ADMM (Sec. 2, eqs. x/z/u-update, over-relaxation,
           penalty update), termination residuals (Sec. 2.3), duality gap
           (App. A), support polish, KKT check, brute-force enumeration
logreg     l1-logistic objective (Sec. 4.2), ADMM with the second-order
           x-subproblem (eq. x-update-lin-sys, Sec. 3.3) or an exact Newton
           x-step, entropy-conjugate duality gap (App. A)
nystrom    randomized Nystrom approximation and the preconditioner
           (Sec. 2.2, eq. preconditioner), condition-number bound
adjoint    implicit differentiation of the Lasso solution on its support
           (derived from the optimality conditions of App. A)
philox     Philox4x64-10 counter-based generator and Box-Muller normals
           (Salmon et al., SC'11), used to reproduce the sketch test matrix
bf16       round-to-nearest-even FP32 -> BF16 conversion
residuals  the KKT residual r_kkt used as the accuracy metric (Sec. 2.3)

Parity status of each function is stated in its module header.
"""
