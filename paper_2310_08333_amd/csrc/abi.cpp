// C ABI of the library: host-side validation, defaults and dispatch.
// Every argument check happens before the first HIP call, so an invalid call
// never touches the device and leaves the outputs untouched.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <mutex>
#include <string>
#include <vector>

#include "engine.hpp"
#include "genios.h"
#include "internal.hpp"

using namespace genios;

namespace {

#define FAIL(code, msg)  \
  do {                   \
    set_error(msg);      \
    return (code);       \
  } while (0)

int check_opts(const genios_opts* o) {
  if (o == nullptr) FAIL(GENIOS_ERR_ARG, "opts is NULL (use genios_default_opts)");
  if (o->struct_size != sizeof(genios_opts))
    FAIL(GENIOS_ERR_ARG, "opts->struct_size does not match this library's genios_opts");
  if (o->precision < GENIOS_PREC_F64 || o->precision > GENIOS_PREC_BF16_ONLY)
    FAIL(GENIOS_ERR_ARG, "opts->precision out of range");
  if (!(o->sigma >= 0.0) || !std::isfinite(o->sigma)) FAIL(GENIOS_ERR_ARG, "sigma must be >= 0");
  if (!(o->alpha > 0.0 && o->alpha < 2.0)) FAIL(GENIOS_ERR_ARG, "alpha must lie in (0, 2)");
  if (!(o->gamma > 0.0) || !std::isfinite(o->gamma)) FAIL(GENIOS_ERR_ARG, "gamma must be > 0");
  if (!(o->eps_abs >= 0.0) || !(o->eps_rel >= 0.0) || !(o->eps_abs + o->eps_rel > 0.0))
    FAIL(GENIOS_ERR_ARG, "eps_abs, eps_rel must be >= 0 and not both zero");
  if (!(o->tau > 1.0) || !(o->mu > 1.0)) FAIL(GENIOS_ERR_ARG, "tau and mu must be > 1");
  if (o->rho_update_every < 0) FAIL(GENIOS_ERR_ARG, "rho_update_every must be >= 0");
  if (o->max_iter < 1 || o->max_cg_iter < 1) FAIL(GENIOS_ERR_ARG, "max_iter, max_cg_iter >= 1");
  if (!(o->cg_tol_floor > 0.0 && o->cg_tol_floor < 1.0))
    FAIL(GENIOS_ERR_ARG, "cg_tol_floor must lie in (0, 1)");
  if (o->sketch_rank < 0 || o->sketch_rank > kMaxS)
    FAIL(GENIOS_ERR_ARG, "sketch_rank must lie in [0, 128]");
  if (o->resketch_every < 1) FAIL(GENIOS_ERR_ARG, "resketch_every must be >= 1");
  if (!(o->switch_tol >= 0.0)) FAIL(GENIOS_ERR_ARG, "switch_tol must be >= 0");
  if (o->history != nullptr && o->history_cap < 1)
    FAIL(GENIOS_ERR_ARG, "history_cap must be >= 1 when history is given");
  if (o->termination < 0 || o->termination > 2)
    FAIL(GENIOS_ERR_ARG, "termination must be 0, 1 or 2");
  if (o->gap_every < 1) FAIL(GENIOS_ERR_ARG, "gap_every must be >= 1");
  if (!(o->eps_gap > 0.0) || !std::isfinite(o->eps_gap)) FAIL(GENIOS_ERR_ARG, "eps_gap must be > 0");
  if (!(o->lambda2 >= 0.0) || !std::isfinite(o->lambda2))
    FAIL(GENIOS_ERR_ARG, "lambda2 must be finite and >= 0");
  if (!(o->huber_delta > 0.0) || !std::isfinite(o->huber_delta))
    FAIL(GENIOS_ERR_ARG, "huber_delta must be finite and > 0");
  if (o->adaptive_sketch < 0 || o->adaptive_sketch > 1)
    FAIL(GENIOS_ERR_ARG, "adaptive_sketch must be 0 or 1");
  if (o->sketch_rank_init < 1) FAIL(GENIOS_ERR_ARG, "sketch_rank_init must be >= 1");
  if (!(o->sketch_kappa > 1.0) || !std::isfinite(o->sketch_kappa))
    FAIL(GENIOS_ERR_ARG, "sketch_kappa must be finite and > 1");
  if (o->power_iters < 1 || o->power_iters > 1000)
    FAIL(GENIOS_ERR_ARG, "power_iters must lie in [1, 1000]");
  if (o->batch_mfma < 0 || o->batch_mfma > 2) FAIL(GENIOS_ERR_ARG, "batch_mfma must be 0, 1 or 2");
  if (o->refine_cg_bf16 < -1 || o->refine_cg_bf16 > 1)
    FAIL(GENIOS_ERR_ARG, "refine_cg_bf16 must be -1, 0 or 1");
  return GENIOS_OK;
}

int check_matrix(const genios_matrix* A) {
  if (A == nullptr) FAIL(GENIOS_ERR_ARG, "matrix descriptor is NULL");
  if (A->A_hi == nullptr) FAIL(GENIOS_ERR_ARG, "A_hi is NULL");
  if (A->m < 1 || A->n < 1) FAIL(GENIOS_ERR_SHAPE, "m and n must be >= 1");
  if (A->m > (int64_t)INT32_MAX || A->n > (int64_t)INT32_MAX)
    FAIL(GENIOS_ERR_SHAPE, "m and n must be < 2^31");
  if (A->lda < A->n) FAIL(GENIOS_ERR_SHAPE, "lda must be >= n");
  if (A->batch < 1 || A->batch > 65535) FAIL(GENIOS_ERR_SHAPE, "batch must lie in [1, 65535]");
  if (A->stride_A != 0 && A->stride_A < A->m * A->lda)
    FAIL(GENIOS_ERR_SHAPE, "stride_A must be 0 or >= m * lda");
  if (A->hi_dtype != GENIOS_DT_F32 && A->hi_dtype != GENIOS_DT_F64)
    FAIL(GENIOS_ERR_ARG, "hi_dtype must be GENIOS_DT_F32 or GENIOS_DT_F64");
  if (A->A_bf16 != nullptr && A->hi_dtype != GENIOS_DT_F32)
    FAIL(GENIOS_ERR_ARG, "a BF16 copy requires an FP32 master copy");
  return GENIOS_OK;
}

int check_precision_vs_dtype(const genios_matrix* A, const genios_opts* o) {
  if (o->precision == GENIOS_PREC_F64 && A->hi_dtype != GENIOS_DT_F64)
    FAIL(GENIOS_ERR_ARG, "precision F64 requires FP64 data");
  if (o->precision != GENIOS_PREC_F64 && A->hi_dtype == GENIOS_DT_F64)
    FAIL(GENIOS_ERR_UNSUPPORTED, "FP64 data is solved with precision F64 only");
  return GENIOS_OK;
}

int check_ws(int op, const genios_matrix* A, const genios_opts* o) {
  const size_t need = genios_workspace_size(op, A, o);
  if (need == 0) FAIL(GENIOS_ERR_ARG, "cannot size the workspace for these arguments");
  if (o->workspace == nullptr || reinterpret_cast<uintptr_t>(o->workspace) % 256 != 0 ||
      o->workspace_bytes < need)
    FAIL(GENIOS_ERR_WORKSPACE, "workspace missing, not 256-byte aligned, or smaller than " +
                                   std::to_string(need) + " bytes");
  return GENIOS_OK;
}

int check_lambda(const double* lambda, int64_t batch) {
  if (lambda == nullptr) FAIL(GENIOS_ERR_ARG, "lambda is NULL");
  for (int64_t b = 0; b < batch; ++b)
    if (!(lambda[b] >= 0.0) || !std::isfinite(lambda[b]))
      FAIL(GENIOS_ERR_ARG, "lambda must be finite and >= 0");
  return GENIOS_OK;
}

// Library-owned device buffer of genios_hvp_noalloc (one copy per GPU, each at its
// own address).  The host never passes the array's name to a kernel: its device
// address is looked up per device with hipGetSymbolAddress and kept below.
static __device__ __align__(256) unsigned char scratch[GENIOS_HVP_NOALLOC_SCRATCH_BYTES];

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};

// Device address of the current device's copy of `scratch` (resolved on the first
// call on that device, with that device current), or an error code.
int noalloc_scratch(void** ptr) {
  int dev = -1;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) FAIL(GENIOS_ERR_DEVICE, std::string("HIP error: ") + hipGetErrorString(e));
  if (dev < 0 || dev >= kMaxDevices) FAIL(GENIOS_ERR_UNSUPPORTED, "device index beyond 63");
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch_ptr[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess || p == nullptr)
      FAIL(GENIOS_ERR_DEVICE, std::string("hipGetSymbolAddress(scratch): ") + hipGetErrorString(e));
    g_scratch_ptr[dev] = p;
  }
  *ptr = g_scratch_ptr[dev];
  return GENIOS_OK;
}

size_t small_ws_bytes(int64_t n, int64_t batch) {
  const int64_t nb = (n + kVecChunk - 1) / kVecChunk;
  size_t b = 0;
  auto add = [&](size_t x) { b += (x + 255) / 256 * 256; };
  add(batch * nb * kPartW * sizeof(double));  // partials
  add(batch * kNumCounters * sizeof(unsigned));
  add(batch * kMaxS * sizeof(double));        // coefficients
  add(batch * 8 * sizeof(double));            // outputs
  return b + 256;
}

}  // namespace

extern "C" {

int genios_default_opts(genios_opts* o) {
  if (o == nullptr) FAIL(GENIOS_ERR_ARG, "opts is NULL");
  std::memset(o, 0, sizeof(*o));
  o->struct_size = sizeof(genios_opts);
  o->precision = GENIOS_PREC_BF16_REFINE;
  o->sigma = 1e-6;
  o->alpha = 1.6;
  o->gamma = 1.2;
  o->eps_abs = 1e-4;
  o->eps_rel = 1e-4;
  o->tau = 2.0;
  o->mu = 10.0;
  o->rho_update_every = 25;
  o->rho_update_until = 500;
  o->max_iter = 5000;
  o->max_cg_iter = 100;
  o->cg_tol_floor = 1e-7;
  o->sketch_rank = 0;
  o->resketch_every = 20;
  o->precondition = 1;
  o->inexact = 1;
  o->switch_tol = 0.0;
  o->stall_window = 10;
  o->rhs_relative = 0;
  o->seed = 0x5eed2310ull;
  o->termination = 0;
  o->gap_every = 1;
  o->eps_gap = 1e-4;
  o->lambda2 = 0.0;
  o->huber_delta = 1.0;
  o->adaptive_sketch = 0;
  o->sketch_rank_init = 8;
  o->sketch_kappa = 10.0;
  o->power_iters = 10;
  o->batch_mfma = 1;
  o->refine_cg_bf16 = -1;
  return GENIOS_OK;
}

size_t genios_workspace_size(int op, const genios_matrix* A, const genios_opts* o) {
  genios_opts d;
  if (o == nullptr) {
    genios_default_opts(&d);
    o = &d;
  }
  if (A == nullptr || A->m < 1 || A->n < 1 || A->batch < 1) return 0;
  Layout L;
  int s = 0;
  switch (op) {
    case GENIOS_OP_LASSO:
    case GENIOS_OP_LOGREG:
    case GENIOS_OP_HUBER:
    case GENIOS_OP_BOXLS:
    case GENIOS_OP_BACKWARD:
      s = o->precondition ? effective_rank(o, A->n, A->m) : 0;
      break;
    case GENIOS_OP_NYSTROM:
      s = o->sketch_rank > 0 ? std::min<int>(o->sketch_rank, kMaxS) : effective_rank(o, A->n, A->m);
      break;
    case GENIOS_OP_MATVEC:
    case GENIOS_OP_HVP:
      s = 0;
      break;
    default:
      return 0;
  }
  L.setup(op, A, o, s);
  return L.total;
}

int genios_lasso_solve(const genios_matrix* A, const void* b, const double* lambda, double rho,
                       const genios_opts* o, void* x, void* z, void* u, genios_info* info) {
  int rc;
  if ((rc = check_matrix(A)) || (rc = check_opts(o)) || (rc = check_precision_vs_dtype(A, o)))
    return rc;
  if (b == nullptr || x == nullptr || z == nullptr || u == nullptr || info == nullptr)
    FAIL(GENIOS_ERR_ARG, "b, x, z, u and info must be non-NULL");
  if ((rc = check_lambda(lambda, A->batch))) return rc;
  if (!(rho > 0.0) || !std::isfinite(rho)) FAIL(GENIOS_ERR_ARG, "rho must be finite and > 0");
  if ((rc = check_ws(GENIOS_OP_LASSO, A, o))) return rc;
  return run_admm(A, b, lambda, rho, o, x, z, u, info, kLossSquare);
}

int genios_logreg_solve(const genios_matrix* A, const void* y, const double* lambda, double rho,
                        const genios_opts* o, void* x, void* z, void* u, genios_info* info) {
  int rc;
  if ((rc = check_matrix(A)) || (rc = check_opts(o)) || (rc = check_precision_vs_dtype(A, o)))
    return rc;
  if (y == nullptr || x == nullptr || z == nullptr || u == nullptr || info == nullptr)
    FAIL(GENIOS_ERR_ARG, "y, x, z, u and info must be non-NULL");
  if ((rc = check_lambda(lambda, A->batch))) return rc;
  if (!(rho > 0.0) || !std::isfinite(rho)) FAIL(GENIOS_ERR_ARG, "rho must be finite and > 0");
  if ((rc = check_ws(GENIOS_OP_LOGREG, A, o))) return rc;
  return run_admm(A, y, lambda, rho, o, x, z, u, info, kLossLogistic);
}

int genios_huber_solve(const genios_matrix* A, const void* b, const double* lambda, double rho,
                       const genios_opts* o, void* x, void* z, void* u, genios_info* info) {
  int rc;
  if ((rc = check_matrix(A)) || (rc = check_opts(o)) || (rc = check_precision_vs_dtype(A, o)))
    return rc;
  if (b == nullptr || x == nullptr || z == nullptr || u == nullptr || info == nullptr)
    FAIL(GENIOS_ERR_ARG, "b, x, z, u and info must be non-NULL");
  if ((rc = check_lambda(lambda, A->batch))) return rc;
  if (!(rho > 0.0) || !std::isfinite(rho)) FAIL(GENIOS_ERR_ARG, "rho must be finite and > 0");
  if ((rc = check_ws(GENIOS_OP_HUBER, A, o))) return rc;
  return run_admm(A, b, lambda, rho, o, x, z, u, info, kLossHuber);
}

int genios_boxls_solve(const genios_matrix* A, const void* b, const void* lo, const void* hi,
                       double rho, const genios_opts* o, void* x, void* z, void* u,
                       genios_info* info) {
  int rc;
  if ((rc = check_matrix(A)) || (rc = check_opts(o)) || (rc = check_precision_vs_dtype(A, o)))
    return rc;
  if (b == nullptr || x == nullptr || z == nullptr || u == nullptr || info == nullptr)
    FAIL(GENIOS_ERR_ARG, "b, x, z, u and info must be non-NULL");
  if (o->lambda2 != 0.0) FAIL(GENIOS_ERR_UNSUPPORTED, "the box path takes no l2 term (lambda2 = 0)");
  if (!(rho > 0.0) || !std::isfinite(rho)) FAIL(GENIOS_ERR_ARG, "rho must be finite and > 0");
  if ((rc = check_ws(GENIOS_OP_BOXLS, A, o))) return rc;
  std::vector<double> zero((size_t)A->batch, 0.0);
  ProxSpec box;
  box.kind = kProxBox;
  box.lo = lo;
  box.hi = hi;
  return run_admm(A, b, zero.data(), rho, o, x, z, u, info, kLossSquare, box);
}

int genios_nystrom_build(const genios_matrix* A, const void* d, int32_t s, const void* omega,
                         const genios_opts* o, void* U, double* lambda_hat, genios_info* info) {
  int rc;
  if ((rc = check_matrix(A)) || (rc = check_opts(o)) || (rc = check_precision_vs_dtype(A, o)))
    return rc;
  if (U == nullptr || lambda_hat == nullptr) FAIL(GENIOS_ERR_ARG, "U and lambda_hat must be non-NULL");
  if (s < 1 || s > kMaxS || s > A->n) FAIL(GENIOS_ERR_ARG, "s must lie in [1, min(128, n)]");
  genios_opts oo = *o;
  oo.sketch_rank = s;
  if ((rc = check_ws(GENIOS_OP_NYSTROM, A, &oo))) return rc;
  return run_nystrom_build(A, d, s, omega, &oo, U, lambda_hat, info);
}

int genios_nystrom_apply(int64_t n, int32_t s, int64_t batch, int32_t dtype, const void* U,
                         const double* lambda_hat, double nu, const void* r, void* z,
                         const genios_opts* o) {
  int rc;
  if ((rc = check_opts(o))) return rc;
  if (n < 1 || s < 1 || s > kMaxS || s > n || batch < 1 || batch > 65535)
    FAIL(GENIOS_ERR_SHAPE, "need n >= 1, 1 <= s <= min(128, n), 1 <= batch <= 65535");
  if (dtype != GENIOS_DT_F32 && dtype != GENIOS_DT_F64) FAIL(GENIOS_ERR_ARG, "dtype must be F32 or F64");
  if (U == nullptr || lambda_hat == nullptr || r == nullptr || z == nullptr)
    FAIL(GENIOS_ERR_ARG, "U, lambda_hat, r, z must be non-NULL");
  if (!(nu > 0.0) || !std::isfinite(nu)) FAIL(GENIOS_ERR_ARG, "nu must be finite and > 0");
  const size_t need = small_ws_bytes(n, batch);
  if (o->workspace == nullptr || reinterpret_cast<uintptr_t>(o->workspace) % 256 != 0 ||
      o->workspace_bytes < need)
    FAIL(GENIOS_ERR_WORKSPACE, "nystrom_apply needs " + std::to_string(need) + " workspace bytes");
  hipStream_t st = static_cast<hipStream_t>(o->stream);
  char* base = static_cast<char*>(o->workspace);
  const int64_t nb = (n + kVecChunk - 1) / kVecChunk;
  size_t off = 0;
  auto take = [&](size_t x) {
    char* p = base + off;
    off += (x + 255) / 256 * 256;
    return p;
  };
  double* part = reinterpret_cast<double*>(take(batch * nb * kPartW * sizeof(double)));
  unsigned* counters = reinterpret_cast<unsigned*>(take(batch * kNumCounters * sizeof(unsigned)));
  double* coef = reinterpret_cast<double*>(take(batch * kMaxS * sizeof(double)));
  hipError_t e = launch_fill(counters, batch * kNumCounters * sizeof(unsigned), st);
  if (e == hipSuccess)
    e = launch_precond_apply(dtype == GENIOS_DT_F32 ? VT_F32 : VT_F64, n, s, batch, U, lambda_hat,
                             nullptr, nu, r, z, part, nb * kPartW, counters, coef, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) FAIL(GENIOS_ERR_DEVICE, std::string("HIP error: ") + hipGetErrorString(e));
  return GENIOS_OK;
}

int genios_lasso_backward(const genios_matrix* A, const void* z_star, const void* grad_z,
                          const double* lambda, const genios_opts* o, void* grad_b,
                          double* grad_lambda, genios_info* info) {
  int rc;
  if ((rc = check_matrix(A)) || (rc = check_opts(o))) return rc;
  if (o->precision == GENIOS_PREC_F64 && A->hi_dtype != GENIOS_DT_F64)
    FAIL(GENIOS_ERR_ARG, "precision F64 requires FP64 data");
  if (z_star == nullptr || grad_z == nullptr || grad_b == nullptr || grad_lambda == nullptr)
    FAIL(GENIOS_ERR_ARG, "z_star, grad_z, grad_b, grad_lambda must be non-NULL");
  if ((rc = check_lambda(lambda, A->batch))) return rc;
  if ((rc = check_ws(GENIOS_OP_BACKWARD, A, o))) return rc;
  return run_backward(A, z_star, grad_z, o, grad_b, grad_lambda, info);
}

int genios_matvec(const genios_matrix* A, int32_t trans, int32_t use_bf16, const void* v,
                  void* out, const genios_opts* o) {
  int rc;
  if ((rc = check_matrix(A)) || (rc = check_opts(o))) return rc;
  if (v == nullptr || out == nullptr) FAIL(GENIOS_ERR_ARG, "v and out must be non-NULL");
  if (trans != 0 && trans != 1) FAIL(GENIOS_ERR_ARG, "trans must be 0 or 1");
  if (use_bf16 && A->A_bf16 == nullptr) FAIL(GENIOS_ERR_ARG, "use_bf16 needs A_bf16");
  if ((rc = check_ws(GENIOS_OP_MATVEC, A, o))) return rc;
  return run_matvec(A, trans, use_bf16, v, out, o);
}

int genios_hvp(const genios_matrix* A, int32_t use_bf16, const void* d, const void* p, void* out,
               const genios_opts* o) {
  int rc;
  if ((rc = check_matrix(A)) || (rc = check_opts(o))) return rc;
  if (p == nullptr || out == nullptr) FAIL(GENIOS_ERR_ARG, "p and out must be non-NULL");
  if (use_bf16 && A->A_bf16 == nullptr) FAIL(GENIOS_ERR_ARG, "use_bf16 needs A_bf16");
  if ((rc = check_ws(GENIOS_OP_HVP, A, o))) return rc;
  return run_hvp(A, use_bf16, d, p, out, o);
}

int genios_hvp_noalloc(const genios_matrix* A, int32_t use_bf16, const void* d, const void* p,
                       void* out, const genios_opts* o) {
  int rc;
  if ((rc = check_matrix(A)) || (rc = check_opts(o))) return rc;
  if (p == nullptr || out == nullptr) FAIL(GENIOS_ERR_ARG, "p and out must be non-NULL");
  if (use_bf16 && A->A_bf16 == nullptr) FAIL(GENIOS_ERR_ARG, "use_bf16 needs A_bf16");
  const size_t need = genios_workspace_size(GENIOS_OP_HVP, A, o);
  if (need == 0) FAIL(GENIOS_ERR_ARG, "cannot size the workspace for these arguments");
  if (need > GENIOS_HVP_NOALLOC_SCRATCH_BYTES)
    FAIL(GENIOS_ERR_WORKSPACE, "genios_hvp_noalloc: this product needs " + std::to_string(need) +
                                   " bytes of scratch, more than the library's " +
                                   std::to_string(GENIOS_HVP_NOALLOC_SCRATCH_BYTES) +
                                   "; use genios_hvp with a workspace");
  void* ptr = nullptr;
  if ((rc = noalloc_scratch(&ptr))) return rc;
  genios_opts oo = *o;
  oo.workspace = ptr;
  oo.workspace_bytes = GENIOS_HVP_NOALLOC_SCRATCH_BYTES;
  return run_hvp(A, use_bf16, d, p, out, &oo);
}

int genios_cast_bf16(const float* src, uint16_t* dst, int64_t count, const genios_opts* o) {
  if (o == nullptr || o->struct_size != sizeof(genios_opts)) FAIL(GENIOS_ERR_ARG, "bad opts");
  if (count < 0) FAIL(GENIOS_ERR_SHAPE, "count must be >= 0");
  if (count > 0 && (src == nullptr || dst == nullptr)) FAIL(GENIOS_ERR_ARG, "NULL pointer");
  hipStream_t st = static_cast<hipStream_t>(o->stream);
  hipError_t e = launch_cast_bf16(src, dst, count, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) FAIL(GENIOS_ERR_DEVICE, std::string("HIP error: ") + hipGetErrorString(e));
  return GENIOS_OK;
}

constexpr int64_t kStreamReadMaxBlocks = GENIOS_STREAM_READ_SCRATCH;

int genios_stream_read(const void* p, int64_t bytes, int32_t reps, uint32_t* scratch,
                       double* seconds, const genios_opts* o) {
  if (o == nullptr || o->struct_size != sizeof(genios_opts)) FAIL(GENIOS_ERR_ARG, "bad opts");
  if (p == nullptr || scratch == nullptr || seconds == nullptr) FAIL(GENIOS_ERR_ARG, "NULL pointer");
  if (bytes < 16 || bytes % 16 || reinterpret_cast<uintptr_t>(p) % 16)
    FAIL(GENIOS_ERR_SHAPE, "bytes must be a positive multiple of 16 at a 16-byte aligned address");
  if (reps < 1) FAIL(GENIOS_ERR_ARG, "reps must be >= 1");
  hipStream_t st = static_cast<hipStream_t>(o->stream);
  int dev = 0, cus = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  const int blocks = stream_read_blocks(bytes, cus, (int)kStreamReadMaxBlocks);
  hipEvent_t ev[2] = {nullptr, nullptr};
  if (e == hipSuccess) e = hipEventCreate(&ev[0]);
  if (e == hipSuccess) e = hipEventCreate(&ev[1]);
  if (e == hipSuccess) e = launch_stream_read(p, bytes, scratch, blocks, st);  // warm-up
  if (e == hipSuccess) e = hipEventRecord(ev[0], st);
  for (int r = 0; r < reps && e == hipSuccess; ++r) e = launch_stream_read(p, bytes, scratch, blocks, st);
  if (e == hipSuccess) e = hipEventRecord(ev[1], st);
  if (e == hipSuccess) e = hipEventSynchronize(ev[1]);
  float ms = 0.f;
  if (e == hipSuccess) e = hipEventElapsedTime(&ms, ev[0], ev[1]);
  for (hipEvent_t x : ev)
    if (x) (void)hipEventDestroy(x);
  if (e != hipSuccess) FAIL(GENIOS_ERR_DEVICE, std::string("HIP error: ") + hipGetErrorString(e));
  *seconds = ms * 1e-3;
  return GENIOS_OK;
}

int genios_gaussian_matrix(int64_t n, int32_t s, uint64_t seed, uint64_t stream_id, float* out,
                           const genios_opts* o) {
  if (o == nullptr || o->struct_size != sizeof(genios_opts)) FAIL(GENIOS_ERR_ARG, "bad opts");
  if (n < 1 || s < 1 || n * (int64_t)s > ((int64_t)1 << 40)) FAIL(GENIOS_ERR_SHAPE, "bad n, s");
  if (out == nullptr) FAIL(GENIOS_ERR_ARG, "out is NULL");
  hipStream_t st = static_cast<hipStream_t>(o->stream);
  hipError_t e = launch_gaussian(VT_F32, n, s, s, 1, seed, stream_id, nullptr, out, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) FAIL(GENIOS_ERR_DEVICE, std::string("HIP error: ") + hipGetErrorString(e));
  return GENIOS_OK;
}

int genios_admm_update(int64_t n, int32_t dtype, double alpha, double kappa, const void* x,
                       void* z, void* u, double* norms, const genios_opts* o) {
  if (o == nullptr || o->struct_size != sizeof(genios_opts)) FAIL(GENIOS_ERR_ARG, "bad opts");
  if (n < 1) FAIL(GENIOS_ERR_SHAPE, "n must be >= 1");
  if (dtype != GENIOS_DT_F32 && dtype != GENIOS_DT_F64) FAIL(GENIOS_ERR_ARG, "dtype must be F32 or F64");
  if (x == nullptr || z == nullptr || u == nullptr || norms == nullptr)
    FAIL(GENIOS_ERR_ARG, "NULL pointer");
  if (!(alpha > 0.0 && alpha < 2.0) || !(kappa >= 0.0)) FAIL(GENIOS_ERR_ARG, "bad alpha or kappa");
  const size_t need = small_ws_bytes(n, 1);
  if (o->workspace == nullptr || reinterpret_cast<uintptr_t>(o->workspace) % 256 != 0 ||
      o->workspace_bytes < need)
    FAIL(GENIOS_ERR_WORKSPACE, "admm_update needs " + std::to_string(need) + " workspace bytes");
  hipStream_t st = static_cast<hipStream_t>(o->stream);
  char* base = static_cast<char*>(o->workspace);
  const int64_t nb = (n + kVecChunk - 1) / kVecChunk;
  double* part = reinterpret_cast<double*>(base);
  const size_t off1 = ((size_t)nb * kPartW * sizeof(double) + 255) / 256 * 256;
  unsigned* counter = reinterpret_cast<unsigned*>(base + off1);
  double* out4 = reinterpret_cast<double*>(base + off1 + 256);
  double h4[4];
  hipError_t e = launch_fill(counter, 256, st);
  if (e == hipSuccess)
    e = launch_admm_update_hook(dtype == GENIOS_DT_F32 ? VT_F32 : VT_F64, n, alpha, kappa, x, z, u,
                                part, counter, out4, st);
  if (e == hipSuccess) e = hipMemcpyAsync(h4, out4, sizeof(h4), hipMemcpyDeviceToHost, st);
  if (e == hipSuccess) e = hipStreamSynchronize(st);
  if (e != hipSuccess) FAIL(GENIOS_ERR_DEVICE, std::string("HIP error: ") + hipGetErrorString(e));
  for (int k = 0; k < 4; ++k) norms[k] = h4[k];
  return GENIOS_OK;
}

const char* genios_status_string(int status) {
  switch (status) {
    case GENIOS_OK: return "ok";
    case GENIOS_MAX_ITER: return "iteration limit reached";
    case GENIOS_WARN_PRECOND: return "sketch core failed; identity preconditioner used";
    case GENIOS_ERR_ARG: return "invalid argument";
    case GENIOS_ERR_SHAPE: return "inconsistent shape";
    case GENIOS_ERR_NUMERIC: return "non-finite residual or CG breakdown";
    case GENIOS_ERR_FACTOR: return "factorisation failure";
    case GENIOS_ERR_DEVICE: return "HIP runtime error";
    case GENIOS_ERR_WORKSPACE: return "workspace missing or too small";
    case GENIOS_ERR_UNSUPPORTED: return "unsupported request";
    default: return "unknown status";
  }
}

const char* genios_last_error(void) { return last_error(); }

void genios_abi_struct_sizes(size_t* matrix_bytes, size_t* opts_bytes, size_t* info_bytes) {
  if (matrix_bytes) *matrix_bytes = sizeof(genios_matrix);
  if (opts_bytes) *opts_bytes = sizeof(genios_opts);
  if (info_bytes) *info_bytes = sizeof(genios_info);
}

}  // extern "C"
