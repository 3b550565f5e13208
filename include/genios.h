/*
 * genios.h - C ABI of the MI355X (gfx950) GeNIOS hot-path library.
 *
 * The library solves the x-subproblem of GeNIOS's inexact ADMM,
 *     (H + (rho + sigma) I) x = rhs,     H = A^T A (Lasso) or A^T D A (l1-logistic),
 * by conjugate gradient with a randomized Nystrom preconditioner, and runs the
 * surrounding ADMM iteration (prox, dual update, residuals, penalty update) on
 * the GPU.  Paper: Diamandis, Frangella, Zhao, Stellato, Udell, "GeNIOS: an
 * (almost) second-order operator-splitting solver for large-scale convex
 * optimization" (2023).  Section numbers below refer to that paper.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * Memory.  Pointers are DEVICE pointers unless a parameter says "(host)".  The
 *   caller owns every input, output and workspace buffer; the library never
 *   allocates device memory during a call.  Pointers must stay valid until the
 *   call returns.  A is row-major (element (i, j) at A[i * lda + j]).
 * Vector dtype.  Vectors (b, y, x, z, u, d, U, Omega, r, ...) are float when
 *   A.hi_dtype == GENIOS_DT_F32 and double when A.hi_dtype == GENIOS_DT_F64.
 * Batches.  A call may carry `batch` independent problems.  Problem p uses
 *   A_hi + p * stride_A (and A_bf16 + p * stride_A); m-vectors at offset p * m,
 *   n-vectors at offset p * n, n x s matrices at offset p * n * s, s-vectors at
 *   p * s, host arrays (lambda, info, grad_lambda) at index p.  stride_A == 0
 *   shares one matrix across the batch.
 * Streams.  All device work is enqueued on opts->stream (a hipStream_t; NULL
 *   is the null stream).  Solves block the host because they read a few
 *   convergence scalars every ADMM iteration; the other calls synchronise the
 *   stream before returning.  The library never calls hipDeviceSynchronize.
 * Errors.  Negative return values are errors, positive ones are warnings with
 *   valid outputs.  Argument and shape errors are detected on the host before
 *   any HIP call and leave outputs untouched.  No exception or abort crosses
 *   the ABI; genios_last_error() returns a thread-local description.
 * Determinism.  Reductions are two-stage with a fixed order and no floating
 *   point atomics: a fixed seed gives bitwise-identical results on one GPU.
 * Reentrancy.  Calls are reentrant given distinct workspaces.  The only
 *   process-wide state is a lazily created per-thread pinned host staging block
 *   and the per-GPU static scratch buffer of genios_hvp_noalloc.
 */
#ifndef GENIOS_H
#define GENIOS_H

#include <stddef.h>
#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

#define GENIOS_ABI_VERSION 1

/* Return codes. */
#define GENIOS_OK 0
#define GENIOS_MAX_ITER 1           /* iteration cap reached; outputs are the last iterate */
#define GENIOS_WARN_PRECOND 2       /* sketch core failed; identity preconditioner used */
#define GENIOS_ERR_ARG (-1)         /* invalid scalar argument or option */
#define GENIOS_ERR_SHAPE (-2)       /* inconsistent sizes or strides */
#define GENIOS_ERR_NUMERIC (-3)     /* NaN/Inf in a residual, or CG breakdown (p^T q <= 0) */
#define GENIOS_ERR_FACTOR (-4)      /* factorisation failure that could not be recovered */
#define GENIOS_ERR_DEVICE (-5)      /* a HIP runtime call failed */
#define GENIOS_ERR_WORKSPACE (-6)   /* workspace missing, misaligned or too small */
#define GENIOS_ERR_UNSUPPORTED (-7) /* valid request the library does not implement */

/* Element types of the data matrix. */
typedef enum { GENIOS_DT_F32 = 0, GENIOS_DT_BF16 = 1, GENIOS_DT_F64 = 2 } genios_dtype;

/* Arithmetic of the matrix-vector products inside CG.
 *   F64          A and all vectors FP64 (requires hi_dtype F64).
 *   F32          A FP32, vectors FP32, dot products FP64.
 *   BF16_REFINE  A in BF16 (FP32 accumulation) until the KKT residual of the
 *                BF16 problem reaches switch_tol (or stalls), then FP32 A,
 *                warm-started, until the FP32 KKT residual reaches eps.
 *   BF16_ONLY    BF16 A throughout; certification uses the BF16 operator. */
typedef enum {
  GENIOS_PREC_F64 = 0,
  GENIOS_PREC_F32 = 1,
  GENIOS_PREC_BF16_REFINE = 2,
  GENIOS_PREC_BF16_ONLY = 3
} genios_precision;

/* Operation ids for genios_workspace_size. */
typedef enum {
  GENIOS_OP_LASSO = 0,
  GENIOS_OP_LOGREG = 1,
  GENIOS_OP_NYSTROM = 2,
  GENIOS_OP_BACKWARD = 3,
  GENIOS_OP_MATVEC = 4,
  GENIOS_OP_HVP = 5,
  GENIOS_OP_HUBER = 6,
  GENIOS_OP_BOXLS = 7
} genios_op;

/* Dense data matrix (or a batch of them).  m rows (samples) by n columns
 * (features), row-major with leading dimension lda >= n. */
typedef struct {
  int64_t m, n, lda;
  int64_t batch;          /* number of independent problems, >= 1 */
  int64_t stride_A;       /* elements between consecutive problems' matrices; 0 = shared */
  int32_t hi_dtype;       /* GENIOS_DT_F32 or GENIOS_DT_F64: the master copy */
  int32_t reserved;
  const void* A_hi;       /* required master copy */
  const uint16_t* A_bf16; /* optional BF16 bit patterns, same layout; when NULL and the
                             precision needs BF16, the library rounds A_hi into the workspace */
} genios_matrix;

/* Solver options.  genios_default_opts fills the paper's defaults (Table of
 * default parameters, Sec. 4): sigma 1e-6, gamma 1.2, sketch size min(50, n/20),
 * re-sketch every 20 iterations, l2 residuals, eps_abs = eps_rel = 1e-4,
 * alpha 1.6, tau 2, mu 10. */
typedef struct {
  uint32_t struct_size;        /* sizeof(genios_opts), for ABI versioning */
  int32_t precision;           /* genios_precision; default BF16_REFINE (F64 for F64 data) */
  double sigma;                /* x-subproblem proximal offset (Sec. 2.1), default 1e-6 */
  double alpha;                /* over-relaxation (Sec. 2.5), default 1.6 */
  double gamma;                /* CG tolerance exponent (Sec. 2.1), default 1.2 */
  double eps_abs, eps_rel;     /* termination (Sec. 2.3), default 1e-4 each */
  double tau, mu;              /* penalty update factor / threshold (Sec. 2.5), 2 and 10 */
  int32_t rho_update_every;    /* iterations between penalty updates, default 25; 0 = fixed */
  int32_t rho_update_until;    /* no penalty update after this iteration, default 500 */
  int32_t max_iter;            /* ADMM iteration cap, default 5000 */
  int32_t max_cg_iter;         /* CG iteration cap per x-solve, default 100 */
  double cg_tol_floor;         /* lower bound on the CG relative tolerance, default 1e-7
                                  (1e-13 for FP64); also the tolerance of exact solves */
  int32_t sketch_rank;         /* Nystrom rank s (<= 128); 0 = min(50, floor(n/20)) */
  int32_t resketch_every;      /* logistic and Huber (D changes with x): re-sketch period in
                                  ADMM iterations, default 20 */
  int32_t precondition;        /* 1 = Nystrom preconditioner, 0 = plain CG; default 1 */
  int32_t inexact;             /* 1 = tolerance schedule of Sec. 2.1, 0 = exact (cg_tol_floor) */
  double switch_tol;           /* BF16 -> FP32 switch when the BF16 problem's r_kkt <= switch_tol;
                                  0 = max(eps_abs, eps_rel) */
  int32_t stall_window;        /* ... or when r_kkt fell < 10% over this many iterations; 10 */
  int32_t rhs_relative;        /* CG stops at ||r|| <= rtol ||r_0||, r_0 the residual of the
                                  solve warm-started at x^k (0, default: the relative tolerance
                                  of Sec. 2.1 taken against the initial residual), or at
                                  ||r|| <= rtol ||rhs|| of the x-system (1: looser, still a
                                  summable error sequence) */
  uint64_t seed;               /* key of the counter-based Gaussian test matrix */
  int32_t warm_start;          /* 1 = start from the caller's x, z, u and the rho argument */
  int32_t profile_kernels;     /* 1 = time every matrix-vector product with HIP events on
                                  `stream` (adds one event pair per product) */
  void* workspace;             /* device workspace, >= genios_workspace_size bytes, 256-B aligned */
  size_t workspace_bytes;
  void* stream;                /* hipStream_t */
  double* history;             /* (host, optional) per-iteration log, see GENIOS_HIST_* */
  int32_t history_cap;         /* rows per problem in `history` */
  int32_t termination;         /* 0 (default): the residual tests of Sec. 2.3;
                                  1: the relative duality gap of Sec. 3.3 / App. A at z,
                                  (l(z) - g(nu)) / min(l(z), |g(nu)|) <= eps_gap, evaluated
                                  with the master copy (BF16_REFINE: in the FP32 phase;
                                  BF16_ONLY: with the BF16 copy) every gap_every iterations;
                                  2: the same pass's distance from 0 to the subdifferential
                                  of the objective at z, ||grad f(z) + lambda v||_2 for the
                                  best v in d||z||_1 (genios_boxls_solve: in the box's normal
                                  cone at z), <= eps_gap (the criterion of the Huber
                                  comparison in Sec. 4.3) */
  int32_t gap_every;           /* iterations between gap evaluations, default 1 */
  double eps_gap;              /* tolerance of termination 1 (relative) or 2 (absolute),
                                  default 1e-4 */
  double lambda2;              /* (lambda2 / 2) ||x||^2 added to the loss (elastic net, Sec. 4.1,
                                  App. A), >= 0, default 0; the x-system shift becomes
                                  rho + sigma + lambda2, the adjoint's lambda2 */
  double huber_delta;          /* genios_huber_solve: the loss is quadratic for |r| <= delta and
                                  linear beyond, l(r) = r^2 or 2 delta |r| - delta^2 (Sec. 4.3
                                  uses delta = 1, the default); > 0 */
  int32_t adaptive_sketch;     /* 1: choose the Nystrom size at each build by the doubling rule of
                                  Sec. 2.2 (adaptive sketch size): sizes sketch_rank_init,
                                  2 sketch_rank_init, ... capped at the sketch size s above,
                                  until 1 + (lam_hat_rr + ||E||) / nu <= sketch_kappa for every
                                  problem, ||E|| = ||H - H_hat|| estimated by power_iters steps
                                  of the randomized power method (start vector: Philox with key
                                  (seed, 0x706F776572 + problem)); 0 (default): fixed size s */
  int32_t sketch_rank_init;    /* first size of the doubling rule, default 8, >= 1 */
  double sketch_kappa;         /* target of the condition-number bound, default 10, > 1 */
  int32_t power_iters;         /* power-method steps per size, default 10, >= 1 */
  int32_t batch_mfma;          /* a batch sharing one matrix (stride_A = 0) forms the H p of
                                  all problems at once on the matrix cores: T = A [p_1 .. p_B],
                                  each column weighted by its problem's curvature D (logistic,
                                  Huber), then A^T T: two streams of A instead of B.  BF16 operand: p and T carried as
                                  BF16 hi + lo parts (~16 bits); FP32 operand: FP32 products
                                  and accumulation throughout.  0 = off, 1 (default) = for
                                  batches of 5 to 128 problems while at least 3 (FP32
                                  operand) or 4 (BF16) of them still run (fewer: one fused
                                  pass per running problem), 2 = for 2 to 128 while at least
                                  2 run */
  int32_t refine_cg_bf16;      /* BF16_REFINE, after the switch to the master copy: 0 = CG
                                  products with the master copy; 1 = CG keeps the BF16 copy
                                  (the x-system's Hessian model) while the master copy forms
                                  grad f(x) (for the squared loss H x, one fused pass) once
                                  per ADMM iteration, so the right-hand side, r_d and the
                                  stopping test are the master copy's and the fixed point is
                                  the FP32 problem's (the approximate-Hessian x-step of
                                  Sec. 2.1); -1 (default) = 1 when one problem's master copy
                                  holds at least GENIOS_REFINE_CG_BF16_MIN_BYTES (its
                                  products are bandwidth-bound, and the BF16 ones take half
                                  the time) in the iterations whose predicted CG count is 3
                                  or more (fewer products do not pay for the extra master
                                  pass), else 0 (measured: on the 20000 x 40000 Lasso 1
                                  saves 3 % of the time to 1e-4, on the 1000 x 10000 one it
                                  costs 19 %: the extra pass per iteration is launch-bound
                                  there).  The logistic and Huber losses take 0 whatever the
                                  value */
} genios_opts;

/* Master-copy bytes of one problem (m n element size) from which refine_cg_bf16 = -1
 * keeps the BF16 copy inside CG after the switch. */
#define GENIOS_REFINE_CG_BF16_MIN_BYTES ((int64_t)256 << 20)

/* Per-iteration history row layout (doubles); problem p, iteration k (1-based)
 * at history[(p * history_cap + k - 1) * GENIOS_HIST_FIELDS + field]. */
#define GENIOS_HIST_FIELDS 10
#define GENIOS_HIST_K 0        /* ADMM iteration k */
#define GENIOS_HIST_RP 1       /* ||x^k - z^k||_2 */
#define GENIOS_HIST_RD 2       /* ||grad f(x^k) + rho u^k||_2 (operator of the phase) */
#define GENIOS_HIST_RKKT 3     /* KKT residual (Sec. 2.3 tests with eps_abs = eps_rel) */
#define GENIOS_HIST_RHO 4      /* rho used in iteration k */
#define GENIOS_HIST_CG 5       /* CG iterations spent in iteration k */
#define GENIOS_HIST_RTOL 6     /* CG relative tolerance used in iteration k */
#define GENIOS_HIST_PHASE 7    /* 0 = BF16 operator, 1 = FP32/FP64 operator */
#define GENIOS_HIST_TIME 8     /* seconds since the call's entry, at the end of iteration k */
#define GENIOS_HIST_XNORM 9    /* ||x^k||_2 */

/* Per-problem results (host). */
typedef struct {
  int32_t status;            /* per-problem return code */
  int32_t iters;             /* ADMM iterations */
  int32_t cg_iters;          /* total CG iterations */
  int32_t phase_switch_iter; /* first FP32-operator iteration (BF16_REFINE), else -1 */
  int32_t resketches;        /* Nystrom builds performed */
  int32_t precond_rank;      /* retained sketch rank of the last build (eigenpairs kept) */
  double obj;                /* objective at z with the master-copy data (FP64 reduction; the
                                duality-gap pass's primal value, gap_primal) */
  double r_p, r_d, r_kkt;    /* final residuals (r_d with the master-copy operator) */
  double rho;                /* final penalty */
  double t_setup;            /* seconds: casting, A^T b, first sketch */
  double t_precond;          /* seconds spent in Nystrom builds */
  double t_solve;            /* seconds in the ADMM loop */
  double t_linsys;           /* seconds in CG (x-subproblem) */
  double t_prox;             /* seconds in the fused prox / dual update kernel */
  double t_total;            /* seconds from entry to return */
  double t_to_target;        /* seconds from entry to the first certified r_kkt <= eps, or -1 */
  double t_matvec_n;         /* with profile_kernels: summed duration of the A v products */
  double t_matvec_t;         /* with profile_kernels: summed duration of the A^T w products */
  int32_t n_matvec_n;        /* number of A v launches (counted with or without profiling) */
  int32_t n_matvec_t;        /* number of A^T w launches */
  int64_t bytes_matvec_n;    /* matrix bytes streamed by the A v products (BF16 or master copy) */
  int64_t bytes_matvec_t;    /* matrix bytes streamed by the A^T w products */
  double t_hvp;              /* with profile_kernels: summed duration of the fused H p products
                                (A^T D A p in one pass over A) on the BF16 copy */
  int32_t n_hvp;             /* number of those launches */
  int32_t n_hvp_hi;          /* number of fused H p launches on the master copy */
  int64_t bytes_hvp;         /* bytes they must move: A once, p in, H p out (BF16 copy) */
  double t_hvp_hi;           /* the same for the fused products on the master copy */
  int64_t bytes_hvp_hi;
  double t_sketch_mc;        /* with profile_kernels: summed duration of the sketch products
                                W = A Omega, Y = A^T D W on the matrix cores (BF16 operand) */
  int64_t flops_sketch_mc;   /* their algorithmic flops, 4 m n s per problem and sketch */
  int32_t n_sketch_mc;       /* sketches whose products ran on the matrix cores */
  int32_t n_sketch_fma;      /* sketches whose products ran on the vector units */
  double t_sketch_fma;       /* the same for the vector-unit products */
  int64_t flops_sketch_fma;
  double rel_gap;            /* relative duality gap (Sec. 3.3, App. A) at the returned z with the
                                master copy: (l(z) - g(nu)) / min(l(z), |g(nu)|) */
  double gap_primal;         /* l(z) */
  double gap_dual;           /* g(nu), nu = min(1, lambda / ||A^T f'(A z - b)||_inf) f'(A z - b)
                                (lambda2 > 0 or the box: nu = f'(A z - b); the box dual is
                                -inf where an infinite bound meets a wrong sign of A^T nu) */
  int32_t gap_checks;        /* gap evaluations during the solve (termination = 1 or 2) */
  int32_t n_hvp_tail;        /* batch: fused H p launches made over the whole chip for one
                                running problem each (at most 8 problems still running) */
  double subgrad_dist;       /* at the returned z with the master copy: the distance from 0 to
                                grad f(z) + lambda d||z||_1 (box: + the normal cone; l2 norm) */
  double sketch_err;         /* adaptive_sketch: power-method estimate of ||H - H_hat|| for the
                                last Nystrom build, else 0 */
  double kappa_bound;        /* adaptive_sketch: 1 + (lam_hat_rr + sketch_err) / nu of that build */
  int32_t sketch_rounds;     /* sizes tried in the last build (1 without adaptive_sketch) */
  int32_t n_hvp_mrhs;        /* batch_mfma: H p launches that served the whole batch */
  double t_hvp_mrhs;         /* with profile_kernels: their summed duration */
  int64_t bytes_hvp_mrhs;    /* bytes they must move: A twice, every problem's p in and H p out */
  int32_t n_hvp_resized;     /* batch of matrices of 256 MB or more: fused H p launches whose grid
                                was sized for the running problems (more than 8, fewer than all) */
  int32_t reserved3;
  double bf16_bound;         /* GENIOS_PREC_BF16_ONLY: a-posteriori bound on F(z) - F* from the
                                rounding of A to BF16 alone (no FP32 pass): with E = A - A~,
                                |E| <= u |A~|, u = 2^-8 / (1 - 2^-8), twice the perturbation
                                bound at z, u ||A~ z - b|| || |A~| |z| || + u^2 || |A~| |z| ||^2 / 2
                                (square loss), u sum_i |y_i| (|A~| |z|)_i (logistic),
                                2 delta u sum_i (|A~| |z|)_i (Huber); the bound's second term
                                evaluates the perturbation at z in place of the unknown
                                optimum.  rel_gap (FP32 master) certifies F(z) - F* itself.
                                0 for the other precisions */
} genios_info;

/* Fill *o with the defaults listed above.  Returns GENIOS_OK. */
int genios_default_opts(genios_opts* o);

/* Bytes of workspace an operation needs for matrix *A and options *o
 * (o may be NULL for defaults).  Returns 0 on invalid arguments. */
size_t genios_workspace_size(int op, const genios_matrix* A, const genios_opts* o);

/* Lasso, minimize (1/2)||A x - b||^2 + lambda ||x||_1 (Sec. 3.1 example, Sec. 4.1
 * with lambda_2 = 0), by the inexact ADMM of Sec. 2 with M = I, c = 0.
 *   b        m per problem.
 *   lambda   (host) batch values, >= 0.
 *   rho      initial penalty (> 0); the paper's experiments use 1.
 *   x, z, u  n per problem, written on return (read too when opts->warm_start).
 *            z is the exactly sparse solution; ||x - z|| is reported as r_p.
 *   info     (host) batch entries, written.
 * Returns the worst per-problem status (errors < warnings < OK ordering). */
int genios_lasso_solve(const genios_matrix* A, const void* b, const double* lambda, double rho,
                       const genios_opts* o, void* x, void* z, void* u, genios_info* info);

/* l1-regularised logistic regression (Sec. 4.2 with the machine-learning
 * interface of Sec. 3.3):
 *   minimize sum_i log(1 + exp(-y_i a_i^T x)) + lambda ||x||_1,
 * labels y in {-1, +1} (m per problem).  The Hessian A^T D A, D = l''(w), is
 * applied at every iteration; the Nystrom sketch of it is refreshed every
 * opts->resketch_every iterations (Sec. 3.3, Table of defaults).  Other
 * arguments as genios_lasso_solve. */
int genios_logreg_solve(const genios_matrix* A, const void* y, const double* lambda, double rho,
                        const genios_opts* o, void* x, void* z, void* u, genios_info* info);

/* l1-regularised Huber fitting (Sec. 4.3, Huber fitting, with the machine-learning
 * interface of Sec. 3.3):
 *   minimize sum_i l(a_i^T x - b_i) + lambda ||x||_1 (+ (lambda2 / 2) ||x||^2),
 *   l(r) = r^2 for |r| <= delta, 2 delta |r| - delta^2 otherwise, delta = opts->huber_delta.
 * The x-system uses H = A^T D A with D = l''(A x^k - b) = 2 [|r_i| <= delta]; the
 * Nystrom sketch of it (opts->precondition, off in the paper's Huber runs) is refreshed
 * every opts->resketch_every iterations.  The duality gap uses l*(v) = v^2 / 4 on
 * |v| <= 2 delta (App. A).  b m per problem; other arguments as genios_lasso_solve. */
int genios_huber_solve(const genios_matrix* A, const void* b, const double* lambda, double rho,
                       const genios_opts* o, void* x, void* z, void* u, genios_info* info);

/* Box-constrained least squares (Sec. 4.5, bounded least squares, through the QP
 * form of Sec. 3.2 with P = A^T A, q = -A^T b, M = I):
 *   minimize (1/2)||A x - b||^2  subject to  lo <= x <= hi.
 * The x-system is the Lasso's ((A^T A + (rho + sigma) I) x = rhs, Nystrom-preconditioned
 * CG); the z-step projects onto the box.
 *   lo, hi   (device) n per problem in the vector dtype, or NULL for -inf / +inf;
 *            lo <= hi is the caller's to ensure (where lo > hi, z takes hi).
 * opts->lambda2 must be 0.  The duality gap and the termination rules use the dual of
 * this split (the box's support function, App. A's construction) and, for
 * termination = 2, the distance from 0 to grad f(z) + the box's normal cone at z.
 * z is the feasible solution; other arguments as genios_lasso_solve. */
int genios_boxls_solve(const genios_matrix* A, const void* b, const void* lo, const void* hi,
                       double rho, const genios_opts* o, void* x, void* z, void* u,
                       genios_info* info);

/* Randomized Nystrom approximation (Sec. 2.2) of H = A^T diag(d) A (d == NULL:
 * H = A^T A) with an n x s test matrix Omega:
 *   H_hat = (H Omega)(Omega^T H Omega)^+ (H Omega)^T = U diag(lambda_hat) U^T.
 *   d          m per problem or NULL.
 *   s          sketch rank, 1 <= s <= min(128, n).
 *   omega      n x s column-major per problem, or NULL to draw the standard
 *              normal matrix on the device (Philox4x64-10, key (opts->seed, p) for
 *              problem p, see genios_gaussian_matrix).
 *   precision  opts->precision selects the operator: BF16 modes sketch the BF16
 *              matrix, F32/F64 the master copy.
 *   U          n x s column-major per problem, orthonormal columns (written).
 *   lambda_hat (device) s doubles per problem, descending, >= 0 (written).
 *   info       (host) precond_rank and status per problem (written).
 * Stabilised as in the randomized Nystrom method the paper cites: a shift
 * mu = eps * ||Y||_F (eps = unit roundoff of Y; equal to the published
 * sqrt(n) eps ||Y|| for an orthonormal test matrix of the same range) is added
 * as Y + mu Omega before the Cholesky factor and removed
 * from the eigenvalues.  If the s x s core cannot be factored after three
 * tenfold shift increases, U = 0, lambda_hat = 0 (identity preconditioner)
 * and the status is GENIOS_WARN_PRECOND. */
int genios_nystrom_build(const genios_matrix* A, const void* d, int32_t s, const void* omega,
                         const genios_opts* o, void* U, double* lambda_hat, genios_info* info);

/* Apply the Nystrom preconditioner of eq. preconditioner,
 *   z = (lambda_hat_s + nu) U (diag(lambda_hat) + nu I)^-1 U^T r + r - U U^T r,
 * to r (n per problem).  dtype is GENIOS_DT_F32 or GENIOS_DT_F64 for U, r, z;
 * lambda_hat (device) s doubles per problem, descending.  nu > 0. */
int genios_nystrom_apply(int64_t n, int32_t s, int64_t batch, int32_t dtype, const void* U,
                         const double* lambda_hat, double nu, const void* r, void* z,
                         const genios_opts* o);

/* Adjoint of the Lasso (elastic-net) solution map (implicit differentiation on
 * the active set, from the optimality conditions of App. A with f'(w) = w): with
 * S the support of z_star, s its signs and G = A_S^T A_S + opts->lambda2 I,
 *   grad_b      = A_S G^-1 grad_z_S                     (m per problem, written)
 *   grad_lambda = -s^T G^-1 grad_z_S                     (host, batch, written)
 * Without the l2 term |S| must not exceed min(m, n) (else G is singular:
 * GENIOS_ERR_NUMERIC).
 * The active columns of the FP32 (or FP64) master copy are gathered, in order,
 * into an m x |S| block in the workspace (padded to a multiple of 8 with
 * identity columns), and the system is solved there by Nystrom-preconditioned
 * CG (sketch of A_S^T A_S) to relative residual opts->cg_tol_floor (default 1e-7
 * here as well); info->iters reports |S|, info->cg_iters the CG iterations.  The
 * sketch size is the solver's s capped at a quarter of the compact system's size,
 * max(8, ceil(|S| / 4) rounded up to 8) with |S| the largest support of the batch:
 * past that the s x s core costs more than the CG iterations it saves.
 *   z_star, grad_z  n per problem.  lambda (host) is accepted for symmetry with
 *   the forward call and checked to be >= 0. */
int genios_lasso_backward(const genios_matrix* A, const void* z_star, const void* grad_z,
                          const double* lambda, const genios_opts* o, void* grad_b,
                          double* grad_lambda, genios_info* info);

/* Dense matrix-vector products with the library's kernels (parity and
 * bandwidth measurement).  trans = 0: out = A v (v n, out m per problem);
 * trans = 1: out = A^T v (v m, out n).  use_bf16 selects the BF16 copy (which
 * must be given).  Vectors follow the vector dtype convention. */
int genios_matvec(const genios_matrix* A, int32_t trans, int32_t use_bf16, const void* v,
                  void* out, const genios_opts* o);

/* The Hessian-vector product of the x-subproblem, out = A^T diag(d) A p
 * (Sec. 3.1 HVP example; Sec. 3.3 ML Hessian with D = diag(d); d NULL: D = I),
 * with the kernels the CG loop uses: one pass over A when the matrix qualifies
 * (FP32 vectors, n % 8 == 0 and lda % 8 == 0 for BF16 or % 4 for FP32, n <= 40704),
 * else A p then A^T (d o A p).  use_bf16 selects the BF16 copy (which must be
 * given).  p, out: n per problem; d: m per problem.  Synchronises o->stream. */
int genios_hvp(const genios_matrix* A, int32_t use_bf16, const void* d, const void* p, void* out,
               const genios_opts* o);

/* For callers that cannot allocate device memory (code recorded under HIP graph
 * capture, tight serving loops, harnesses that forbid allocation): genios_hvp
 * without a workspace.  The product's partial sums live in a library-owned
 * static device buffer of GENIOS_HVP_NOALLOC_SCRATCH_BYTES per GPU, resolved
 * once per device on the first call there and held until the process ends;
 * o->workspace and o->workspace_bytes are ignored.  The call allocates nothing
 * (no hipMalloc, hipFree, pinned host memory or allocating library routine).
 * Errors: GENIOS_ERR_WORKSPACE, detected before any HIP call, when
 * genios_workspace_size(GENIOS_OP_HVP, A, o) exceeds the buffer (one fused
 * product of a 20000 x 40000 matrix needs about 80 MiB); otherwise as
 * genios_hvp.  Every call on one GPU shares that GPU's buffer and the buffer
 * keeps the last call's contents (the kernels write every partial they read):
 * calls that overlap on one GPU (several streams or threads) race, so the caller
 * serialises them.  Arguments, results and the stream synchronisation are those
 * of genios_hvp, and the kernels and launch shapes are the same, so the output
 * is bitwise equal to genios_hvp's. */
#define GENIOS_HVP_NOALLOC_SCRATCH_BYTES ((size_t)128 << 20)
int genios_hvp_noalloc(const genios_matrix* A, int32_t use_bf16, const void* d, const void* p,
                       void* out, const genios_opts* o);

/* Round `count` FP32 values to BF16, nearest-even, NaN -> 0x7FC0 (device). */
int genios_cast_bf16(const float* src, uint16_t* dst, int64_t count, const genios_opts* o);

/* Measurement reference, not part of the method: the HBM read rate a kernel
 * that only streams reaches.  Reads `bytes` (a positive multiple of 16) at the
 * 16-byte aligned device address p once per repetition with a plain streaming
 * kernel, after one untimed warm-up, and stores in *seconds (host) the HIP-event
 * time of the `reps` timed reads on o->stream (synchronised).  scratch: device,
 * GENIOS_STREAM_READ_SCRATCH words, receives one XOR checksum per block. */
#define GENIOS_STREAM_READ_SCRATCH 4096
int genios_stream_read(const void* p, int64_t bytes, int32_t reps, uint32_t* scratch,
                       double* seconds, const genios_opts* o);

/* Draw the n x s (column-major) standard normal test matrix the sketch uses,
 * for key (seed, stream_id): Philox4x64-10 + Box-Muller, rounded to FP32. */
int genios_gaussian_matrix(int64_t n, int32_t s, uint64_t seed, uint64_t stream_id, float* out,
                           const genios_opts* o);

/* One fused ADMM update (Sec. 2, z- and u-update with over-relaxation of
 * Sec. 2.5 and the prox of Sec. 3.1) on n-vectors, for testing:
 *   xh = alpha x + (1 - alpha) z;  z <- S_kappa(xh + u);  u <- u + xh - z;
 * and norms[0..3] (host) = ||x - z_new||^2, ||x||^2, ||z_new||^2, ||u_new||^2
 * accumulated in FP64.  dtype GENIOS_DT_F32 or GENIOS_DT_F64. */
int genios_admm_update(int64_t n, int32_t dtype, double alpha, double kappa, const void* x,
                       void* z, void* u, double* norms, const genios_opts* o);

const char* genios_status_string(int status);
const char* genios_last_error(void);

/* sizeof(genios_matrix), sizeof(genios_opts), sizeof(genios_info) as compiled
 * into the library (host), so bindings can verify their struct layouts. */
void genios_abi_struct_sizes(size_t* matrix_bytes, size_t* opts_bytes, size_t* info_bytes);

#ifdef __cplusplus
}
#endif
#endif /* GENIOS_H */
