// Internal declarations shared by the HIP kernels, the host engine and the C ABI.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include <string>

#include "genios.h"

namespace genios {

// Vector element type of a call: float when the master copy is FP32, double for FP64.
enum VType { VT_F32 = 0, VT_F64 = 1 };
// Element type of the matrix a product reads.
enum MType { MT_BF16 = 0, MT_F32 = 1, MT_F64 = 2 };

constexpr int kMaxS = 128;            // largest supported sketch rank
constexpr int kVecBlock = 256;        // threads per block of the vector kernels
constexpr int kVecChunk = 1024;       // elements per block of the vector kernels
constexpr int kMaxVecBlocks = 128;    // blocks per problem of the vector kernels
constexpr int kPartW = kMaxS + 16;    // doubles per block partial (U^T r + scalars)
constexpr int kNumCounters = 16;      // last-block counters per problem

// Rows per block of the CG/ADMM vector kernels: one row per thread, growing in
// whole block widths only when a problem would otherwise need more than 1024
// blocks (the last-block reductions scale with the block count).
inline int64_t vec_chunk(int64_t n) {
  const int64_t blocks = (n + kVecBlock - 1) / kVecBlock;
  const int64_t q = blocks > 1024 ? (blocks + 1023) / 1024 : 1;
  const int64_t c = (int64_t)kVecBlock * q;
  return c < 4 * kVecChunk ? c : 4 * kVecChunk;
}
// The finer grid of k_cg_alpha (sum of the H p block partials): 64 elements per
// block (the four waves split the partial slots) until a problem has 1024 blocks,
// then wider chunks in steps of 64, at most 4 kVecChunk.
inline int64_t vec_chunk_fine(int64_t n) {
  const int64_t per = (n + 1023) / 1024;
  const int64_t c = per <= 64 ? 64 : (per + 63) / 64 * 64;
  return c < 4 * kVecChunk ? c : 4 * kVecChunk;
}
// Largest block count either grid gives for any length up to n (partial-slot capacity).
inline int64_t vec_blocks_max(int64_t n) {
  const int64_t cf = vec_chunk_fine(n), cc = vec_chunk(n);
  const int64_t nf = (n + cf - 1) / cf, nc = (n + cc - 1) / cc;
  const int64_t small = (n + 63) / 64 < 1024 ? (n + 63) / 64 : 1024;
  const int64_t m1 = nf > nc ? nf : nc;
  return m1 > small ? m1 : small;
}

// Host-written parameters of one problem, uploaded before each ADMM iteration.
struct alignas(128) ProbParams {
  double nu;         // CG shift rho + sigma
  double rho;
  double sigma;
  double kappa;      // lambda / rho, the soft-threshold level
  double alpha;      // over-relaxation
  double u_scale;    // u <- u * u_scale at the start of the iteration (penalty change)
  double rtol;       // CG relative tolerance of this iteration
  double tol_floor;  // CG tolerance floor, relative to ||rhs||
  double lambda;
  double lambda2;    // (lambda2 / 2) ||x||^2 in the loss: grad f gains lambda2 x
  int32_t run;       // problem takes part in this iteration
  int32_t max_cg;
  int32_t rhs_rel;   // 1: tolerance relative to ||rhs||, 0: relative to ||r_0||
  int32_t use_c;     // 1: gradient is h - c (Lasso); 0: gradient vector given
  int32_t prox;      // z-step: kProxL1 (soft-threshold at kappa) or kProxBox (clamp to [lo, hi])
};
enum : int32_t { kProxL1 = 0, kProxBox = 1 };

// Device-written state of one problem (read back by the host after each sync).
struct alignas(128) ProbState {
  double rz2[2];     // r^T P^-1 r, ping-pong by CG iteration parity (rz2[t & 1] at iteration t)
  double pq;         // p^T (H + nu I) p
  double rr;         // ||r||^2
  double tol2;       // squared absolute CG tolerance
  double alpha_cg, beta_cg;
  double rhs2;       // ||rhs||^2
  double r02;        // ||r_0||^2
  int32_t cg_active; // CG running for this problem
  int32_t cg_iters;  // CG iterations in the current x-solve
  int32_t admm_done; // the fused z/u update ran this iteration
  int32_t breakdown; // p^T q <= 0 or non-finite
  double red[8];     // reductions of the fused update (see kRed*)
};

// Indices into ProbState::red written by the fused ADMM update.
enum {
  kRedRp2 = 0,   // ||x - z||^2
  kRedX2 = 1,    // ||x||^2
  kRedZ2 = 2,    // ||z||^2
  kRedU2 = 3,    // ||u||^2 (scaled dual)
  kRedRd2 = 4,   // ||grad + rho u||^2 (Lasso: grad = h - c)
  kRedZ1 = 5,    // ||z||_1
  kRedNnz = 6,   // nonzeros of z
  kRedAux = 7    // unused
};

// Slots of the block-partial array (slot-major: spart[b][slot][block]).  A kernel
// writes one partial per block; the kernel that consumes the sum reduces the
// partials itself, every block in the same fixed order, so no kernel waits on
// another block of its own grid.
enum {
  kSlRhs2 = 0,   // ||rhs||^2 of the x-system
  kSlRr,         // ||r||^2 (r_0 at admm_begin, r_{t+1} at cg_update)
  kSlRz,         // r^T P^-1 r
  kSlPq,         // p^T (H + nu I) p
  kSlEnd0,       // the 7 reductions of admm_end (kRedRp2 .. kRedNnz order)
  kSlDual = kSlEnd0 + 7,  // ||grad + rho u||^2
  kSlPp,         // ||p||^2 where the operator is H + nu I (every coordinate unless masked)
  kSlPpOff,      // ||p||^2 where it is the identity (masked-off coordinates)
  kNumSlots
};

// Counter slots for the last-block reductions.
enum {
  kCntBegin = 0, kCntPrecond, kCntAlpha, kCntUpdate, kCntEnd, kCntAux0, kCntAux1, kCntAux2,
  kCntObj /* unused */, kCntMasked
};

// Pointers to the per-problem control arrays in the workspace.
struct Ctrl {
  ProbParams* params;   // [batch]
  ProbState* state;     // [batch]
  double* part;         // [batch][part_stride] block partials (kPartW doubles per block)
  int64_t part_stride;  // doubles per problem in `part`
  double* spart;        // [batch][kNumSlots][pstride] scalar block partials
  double* upart;        // [batch][kMaxS][pstride] U^T r block partials (column-major)
  int64_t pstride;      // blocks reserved per slot (>= blocks of any vector kernel)
  unsigned* counters;   // [batch][kNumCounters]
  double* coef;         // [batch][2 kMaxS] preconditioner coefficients c_j of the current r,
                        // then their terms c_j (U^T r)_j of r^T P^-1 r
  int32_t* s_eff;       // [batch] retained sketch rank
  double* lamhat;       // [batch][s] (s = sketch stride)
  int32_t s_stride;     // lamhat stride per problem
};

// A matrix operand as the kernels see it.
struct MatArg {
  const void* ptr;
  MType mt;
  int64_t m, n, lda, strideA;
};

// ---- launchers (kernels.hip) ------------------------------------------------
// All launchers enqueue on `st` and return hipSuccess or the launch error.

// Partials of t = A v over `nsplit` column splits: out[b][split][m].
hipError_t launch_gemv_n(const MatArg& A, int64_t batch, VType vt, const void* v, int64_t v_stride,
                         void* out, int64_t out_split_stride, int64_t out_prob_stride, int nsplit,
                         const int32_t* gate, int gate_stride_ints, hipStream_t st);
// |A| |v| with elementwise absolute values (same partial layout as launch_gemv_n).
hipError_t launch_gemv_n_abs(const MatArg& A, int64_t batch, VType vt, const void* v,
                             int64_t v_stride, void* out, int64_t oss, int64_t ops, int nsplit,
                             hipStream_t st);
// Per problem (4 doubles each) of the split-summed rows y: mode 0 writes sum y^2 at [0],
// sum |y| at [1] and sum |c| |y| at [3]; mode 1 writes sum (y - c)^2 at [2].
hipError_t launch_bound_terms(VType vt, int64_t m, int64_t batch, const void* parts, int nsplit,
                              int64_t split_stride, int64_t prob_stride, const void* c,
                              int64_t c_stride, int mode, double* out, hipStream_t st);
// Partials of y = A^T (d o sum_s tin_s) over `ksplit` row splits, for nrhs columns:
// ypart[b][ks][k][npad].  tin[k] column at tin + k * tin_col_stride.
hipError_t launch_gemv_t(const MatArg& A, int64_t batch, VType vt, const void* tin, int nsplit_in,
                         int64_t tin_split_stride, int64_t tin_prob_stride, int64_t tin_col_stride,
                         int nrhs, const void* dscale, int64_t d_stride, void* ypart, int ksplit,
                         int64_t ypart_ks_stride, int64_t ypart_col_stride, int64_t ypart_prob_stride,
                         const int32_t* gate, int gate_stride_ints, hipStream_t st);
// Fused H p = A^T (d o (A p)) in one pass over A (FP32 vectors; A in BF16 or FP32).
// One partial of hp per block: ypart[b][block][ks_stride].
constexpr int kHvpMaxBlocks = 512;  // partials reserved across a batch
struct HvpGeom {
  int threads = 0;         // 0: A does not qualify (use gemv_n + gemv_t)
  int ept = 0;             // owned columns per thread
  int rows = 0;            // rows per group
  int blocks = 0;          // blocks (partials) per problem; block g owns rows g, g + blocks, ...
  int rows_per_block = 0;  // the most rows a block owns
};
HvpGeom hvp_geometry(const MatArg& A, int64_t batch, bool query_device);
// the fused product reads p in 16-byte pieces
bool hvp_p_aligned(const void* p, int64_t p_stride, int64_t batch);
// pq (nullable): per block, the sum over its rows of d_i (a_i^T p)^2 (= p^T H p of the
// block's rows), at pq[b * pq_stride + block].
hipError_t launch_hvp_fused(const MatArg& A, const HvpGeom& g, int64_t batch, const float* p,
                            int64_t p_stride, const float* d, int64_t d_stride, float* ypart,
                            int64_t ks_stride, int64_t prob_stride, const int32_t* gate,
                            int gate_stride, hipStream_t st, double* pq = nullptr,
                            int64_t pq_stride = 0);
int gemv_n_splits(const MatArg& A, int64_t batch);
int gemv_t_splits(const MatArg& A, int64_t batch);
int gemv_t_rows_per_split(const MatArg& A, int ksplit);

// out[b][i] = sum_{k<nsplit} in[b][k][i] for problems whose gate is nonzero (gate may be NULL).
hipError_t launch_sum_splits(VType vt, int64_t batch, int64_t len, const void* in, int nsplit,
                             int64_t split_stride, int64_t prob_stride_in, void* out,
                             int64_t prob_stride_out, hipStream_t st,
                             const int32_t* gate = nullptr, int gate_stride = 0);

hipError_t launch_cast_bf16(const float* src, uint16_t* dst, int64_t count, hipStream_t st);
// Streaming-read reference (stream.hip): blocks for `bytes` on `cus` CUs, at most max_blocks.
int stream_read_blocks(int64_t bytes, int cus, int max_blocks);
hipError_t launch_stream_read(const void* p, int64_t bytes, uint32_t* out, int blocks,
                              hipStream_t st);
hipError_t launch_fill(void* p, size_t bytes, hipStream_t st);  // zero fill (no memset nodes)
hipError_t launch_copy(VType vt, const void* src, void* dst, int64_t count, hipStream_t st);

// ---- CG / ADMM vector kernels ------------------------------------------------
struct VecArgs {
  VType vt;
  int64_t n, batch;
  int nb;                 // blocks per problem
  int64_t chunk;          // elements per block
  int nbf;                // k_cg_alpha's blocks per problem (finer grid)
  int64_t chunkf;         // and its elements per block
  Ctrl ctrl;
  // n-vectors (per problem stride n)
  void *x, *z, *u, *h, *g, *c, *r, *p, *hp, *w;  // w: preconditioned residual
  const void* U;          // n x s_stride column-major per problem (nullable)
  int s_stride;
  const void* ypart;      // gemv_t partials feeding hp (prob stride, ks stride)
  int ksplit;
  int64_t ypart_ks_stride, ypart_prob_stride;
  const uint8_t* mask;    // masked operator (adjoint): 1 = in the active set
  const void *lo, *hi;    // box bounds of kProxBox, n per problem (nullable: unbounded side)
  // the fused product's per-block p^T H p partials (cg_step): hpq[b * hpq_stride + k],
  // k < nhpq
  const double* hpq;
  int64_t hpq_stride;
  int nhpq;
};
// One x-solve: admm_begin; precond_coef, precond_p(init); then per CG iteration
// t = 0, 1, ...: after the fused product cg_step(t), after the others cg_alpha and
// cg_update(t); then precond_coef, precond_p(t); then admm_end, admm_finish.  np:
// the partial blocks of the kernel that wrote ||r||^2 and U^T r (nb: cg_update;
// nbf: admm_begin, cg_step).  Every kernel is gated on the problem's flags, so
// surplus iterations are no-ops.
hipError_t launch_admm_begin(const VecArgs& a, hipStream_t st);
hipError_t launch_precond_coef(const VecArgs& a, int np, hipStream_t st);
hipError_t launch_precond_p(const VecArgs& a, int t, int init, int np, hipStream_t st);
hipError_t launch_cg_alpha(const VecArgs& a, hipStream_t st);
hipError_t launch_cg_update(const VecArgs& a, int t, hipStream_t st);
hipError_t launch_cg_step(const VecArgs& a, int t, hipStream_t st);
hipError_t launch_admm_end(const VecArgs& a, hipStream_t st);
hipError_t launch_admm_finish(const VecArgs& a, hipStream_t st);
// ||g + rho u||^2 into state.red[kRedRd2] with g = h - c or the given g (two kernels).
hipError_t launch_dual_residual(const VecArgs& a, hipStream_t st);
// Smooth losses of the ML interface (Sec. 3.3), per sample with t = a_i^T x:
//   square    (t - b)^2 / 2 (the Lasso),
//   logistic  log(1 + exp(-y t)) (Sec. 4.2),
//   Huber     l(t - b), l(r) = r^2 (|r| <= delta), 2 delta |r| - delta^2 (Sec. 4.3).
enum LossKind : int { kLossSquare = 0, kLossLogistic = 1, kLossHuber = 2 };
// Elementwise terms of the ML x-system from the t = A x partials: the curvature
// d = f''(t) and the two right-hand columns col0 = d o t (for H x) and
// col1 = f'(t) (for grad f).  Logistic: d = s (1 - s), f' = -y s with s = sigmoid(-y t);
// Huber: d = 2 [|t - b| <= delta], f' = 2 clip(t - b, -delta, delta).
hipError_t launch_loss_elem(VType vt, int loss, double delta, int64_t m, int64_t batch,
                            const void* tparts, int nsplit, int64_t split_stride,
                            int64_t prob_stride, const void* bvec, void* d, void* cols,
                            int64_t col_stride, const int32_t* gate, int gate_stride,
                            hipStream_t st);
// ---- relative duality gap (App. A), gap.hip ----
struct GapState {
  double loss;      // sum_i f(t_i)
  double grad_inf;  // ||A^T f'(t)||_inf
  double l1;        // ||v||_1
  double x2;        // ||v||^2
  double excess2;   // ||(|A^T f'(t)| - lambda)_+||^2; box: the support function sum
                    // sum_j max(lo_j w_j, hi_j w_j), w = -A^T f'(t)
  double kappa;     // lambda2 = 0: min(1, lambda / grad_inf); lambda2 > 0: 1
  double reg;       // lambda2 > 0: -excess2 / (2 lambda2), the dual's l2 part; else 0
  double primal;    // l(v) = loss + lambda ||v||_1 + (lambda2 / 2) ||v||^2
  double dual;      // g(nu)
  double gap;       // primal - dual
  double rel_gap;   // gap / min(primal, |dual|)
  double subgrad;   // ||.||_2 of the least-norm element of grad f(v) + lambda d||v||_1
                    // (box: of grad f(v) + the normal cone of the box at v)
};
constexpr int kGapPStride = 256;  // block partials per reduction and problem
constexpr int kGapSlots = 7;      // loss, inf, l1, conjugate sum, x2, excess2, subgrad^2
struct GapArgs {
  VType vt;
  int64_t m, n, batch;
  const void* tparts;  // t = A v column-split partials
  int nsplit;
  int64_t split_stride, prob_stride;
  const void* bvec;    // b (Lasso, Huber) or the labels y (logistic), m per problem
  int loss;            // LossKind
  double delta;        // Huber threshold
  void* fprime;        // [batch][m] f'(t), the input of A^T
  void* sfold;         // [batch][m] f'(t) (Lasso, Huber) or sigmoid(w) (logistic)
  const void* ypart;   // A^T f'(t) row-split partials
  int ks;
  int64_t ks_stride, yprob;
  const void* v;       // the point, n per problem
  const ProbParams* params;  // lambda, lambda2, prox
  const void *lo, *hi; // box bounds (prox = kProxBox), n per problem, nullable
  double* part;        // [batch][kGapSlots][kGapPStride]
  GapState* state;     // [batch]
};
int gap_blocks(int64_t len);
// ---- set-up pass of a BF16-A solve, setup.hip ----
// Row splits of the fused pass (at most max_splits).
int cast_atb_splits(int64_t m, int64_t n, int64_t batch, int max_splits);
bool cast_atb_eligible(const void* A, int64_t lda, int64_t strideA, int64_t n, const void* A16,
                       const void* ypart, int64_t ks_stride);
// A16 = bf16(A) and the per-split partials of A^T b (slots [0, ksplit)) and
// bf16(A)^T b (slots lo_offset / ks_stride + [0, ksplit)), FP32 b.
hipError_t launch_cast_atb(const float* A, int64_t lda, int64_t strideA, uint16_t* A16,
                           int64_t m, int64_t n, int64_t batch, const float* b, float* ypart,
                           int ksplit, int64_t ks_stride, int64_t lo_offset,
                           int64_t prob_stride, hipStream_t st);
// ---- power method on E = H - U diag(lam_hat) U^T (Sec. 2.2 adaptive sketch), adaptive.hip ----
struct PowerArgs {
  VType vt;
  int64_t n, batch;
  const void* U;             // n x s_stride column-major per problem
  int s_stride;              // also the lam_hat stride
  const double* lamhat;
  const int32_t* s_eff;      // retained columns per problem
  const void* h;             // H v, n per problem
  void* v;                   // the unit vector (updated in place by a step)
  void* ev;                  // E v (the start vector before launch_power_start)
  double* ut_part;           // [batch][kMaxS][pstride]
  double* part2;             // [batch][2][pstride]
  int pstride, nb;           // nb = power_blocks(n, pstride)
  double* est;               // [batch] v^T E v of the last step
};
int power_blocks(int64_t n, int pstride);
// Philox stream id of the power method's start vectors (key (seed, kPowerStream + problem)).
constexpr uint64_t kPowerStream = 0x706F776572ull;
// v = ev / ||ev|| (the start vector drawn into ev).
hipError_t launch_power_start(const PowerArgs& a, hipStream_t st);
// With h = H v: est = v^T E v, v <- E v / ||E v||.
hipError_t launch_power_step(const PowerArgs& a, hipStream_t st);
// f'(t), the folded s and the loss partials from the t partials.
hipError_t launch_gap_elem(const GapArgs& a, hipStream_t st);
// After A^T f'(t) is in ypart: ||.||_inf, ||v||_1, kappa, primal, dual, gap.
hipError_t launch_gap_after_t(const GapArgs& a, hipStream_t st);

// Stand-alone fused ADMM update test hook.
hipError_t launch_admm_update_hook(VType vt, int64_t n, double alpha, double kappa, const void* x,
                                   void* z, void* u, double* part, unsigned* counter,
                                   double* out4, hipStream_t st);
// Stand-alone preconditioner apply.
hipError_t launch_precond_apply(VType vt, int64_t n, int s, int64_t batch, const void* U,
                                const double* lamhat, const int32_t* s_eff, double nu,
                                const void* r, void* z, double* part, int64_t part_stride,
                                unsigned* counters, double* coef, hipStream_t st);
// Adjoint helpers.
hipError_t launch_build_mask(VType vt, int64_t n, int64_t batch, const void* zstar,
                             const void* gz, uint8_t* mask, void* sgn, void* neg_rhs,
                             hipStream_t st);
hipError_t launch_masked_dot(VType vt, int64_t n, int64_t batch, const void* a, const void* b,
                             double* part, int64_t part_stride, unsigned* counters, double* out,
                             hipStream_t st);

// ---- sketch (sketch.hip) ------------------------------------------------------
hipError_t launch_gaussian(VType vt, int64_t n, int s, int s_stride, int64_t batch, uint64_t seed,
                           uint64_t stream_id, const uint8_t* mask, void* out, hipStream_t st);
struct SketchWs {
  void* omega;      // n x sp per problem (vt)
  void* W;          // m x sp per problem (float or double)
  void* Wpart;      // ksW x m x sp per problem
  void* Ypart;      // ksY x n x sp per problem
  void* Y;          // n x sp per problem
  double* gpart;    // Gram partials
  double* gram;     // 3 x s x s per problem
  double* core;     // core scratch per problem (C, X, V, T, ...)
  uint16_t* o16;    // BF16 Omega [c][kpad(n)] per problem (matrix-core path), or NULL
  uint16_t* w16;    // BF16 hi then lo parts of d o W [c][kpad(m)] (matrix-core path), or NULL
  int ksW, ksY, nbG;
  hipEvent_t ev_gemm[2];  // recorded before and after the sketch products when non-null
};
// The sketch products on the matrix cores (BF16 operand, FP32 vectors).
bool sketch_mfma_eligible(const MatArg& A, VType vt, const SketchWs& ws);
hipError_t launch_sketch_mfma(const MatArg& A, int64_t batch, int sp, const float* d,
                              int64_t d_stride, const SketchWs& ws, hipStream_t st);
int sketch_pad(int s);
// The s x s core for s <= kCoreLdsMaxS (core.hip): one workgroup per problem for the
// Cholesky, the triangular solves and block Jacobi, then the eigenvector columns T.
constexpr int kCoreLdsMaxS = 100;
hipError_t launch_nystrom_core_lds(int64_t batch, int s, int SPg, double eps, double rel_floor,
                                   double jac_tol, const double* gram, double* core,
                                   double* lamhat, int32_t* s_eff, int32_t* status, double* shift,
                                   hipStream_t st);
// ---- H p of a batch sharing A on the matrix cores (sketch_mfma.hip) ----
struct MrhsWs {
  uint16_t* p16 = nullptr;  // BF16 hi then lo parts of the p block [c][kpad(n)] (FP32
                            // operand: the p block in FP32, same bytes)
  uint16_t* w16 = nullptr;  // BF16 hi then lo parts of T = A P [c][kpad(m)] (FP32: T)
  float* wpart = nullptr;   // ksW x SP x m partials of T
  int sp = 0, ksW = 1, ksY = 1;  // ksY: row splits of A^T T with the BF16 operand
  int ksYf = 1;                  // ... and with the FP32 operand (256 columns per block)
};
int mrhs_pad(int B);
bool mrhs_eligible(const MatArg& A, VType vt, int64_t B, const MrhsWs& ws);
// ypart[ks][c][j] (column stride ldy, split stride sp ldy) for ks < ws.ksY; every kernel
// exits at once when no problem's flag (gate, gstride) is set.
// With d, problem c's product is A^T diag(d + c d_stride) A p_c.
hipError_t launch_mrhs_hvp(const MatArg& A, int B, const float* P, int64_t pstride,
                           const float* d, int64_t d_stride, const MrhsWs& ws, float* ypart,
                           int64_t ldy, const int32_t* gate, int gstride, hipStream_t st);
size_t sketch_ws_bytes(int64_t m, int64_t n, int s, int64_t batch, VType vt, int* ksW, int* ksY,
                       int* nbG);
// Y = H Omega (H = A^T diag(d) A) then the stabilised s x s core and U.
// Writes U (n x s col-major, vt), lamhat (s doubles, descending), s_eff, status.
hipError_t run_nystrom(const MatArg& A, int64_t batch, VType vt, const void* d, int64_t d_stride,
                       int s, const void* omega_in, uint64_t seed, uint64_t stream_id,
                       const uint8_t* mask, const SketchWs& ws, void* U, double* lamhat,
                       int32_t* s_eff, int32_t* core_status, double* shift_out, hipStream_t st);

// ---- errors -----------------------------------------------------------------
void set_error(const std::string& s);
const char* last_error();

}  // namespace genios

namespace genios {
// Active-set compaction (adjoint): ordered indices of the mask, column gather of
// A (zero padding up to ldS), gather of two n-vectors plus the padding mask.
hipError_t launch_compact_index(int64_t n, int64_t batch, const uint8_t* mask, int32_t* idx,
                                int32_t* cnt, hipStream_t st);
hipError_t launch_gather_cols(MType mt, const void* A, int64_t lda, int64_t strideA, int64_t m,
                              int64_t n, int64_t batch, const int32_t* idx, const int32_t* cnt,
                              int ldS, void* out, hipStream_t st);
hipError_t launch_gather_vec(VType vt, int64_t n, int64_t batch, const int32_t* idx,
                             const int32_t* cnt, int ldS, const void* in0, void* out0,
                             const void* in1, void* out1, uint8_t* mask_out, hipStream_t st);
}  // namespace genios
