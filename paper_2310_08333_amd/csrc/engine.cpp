// Host engine: workspace layout and the ADMM / PCG drivers.
//
// The drivers enqueue every step on one HIP stream.  Scalars that only the
// GPU needs (CG alpha/beta, tolerances, preconditioner coefficients) live in
// per-problem device control blocks; each kernel of a CG iteration is gated by
// the problem's `cg_active` flag, so the host can enqueue several CG
// iterations, the fused z/u update and (for the logistic and Huber losses) the next
// gradient pass without waiting.  The host synchronises once per ADMM
// iteration (more only when a CG solve outlasts its enqueued iterations) to
// read the residual norms, apply the stopping test and the penalty rule of
// Sec. 2.3 / Sec. 2.5, and choose the next CG tolerance of Sec. 2.1.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "engine.hpp"
#include "internal.hpp"

namespace genios {

namespace {

thread_local std::string g_err;

struct Pinned {
  void* p = nullptr;
  size_t cap = 0;
};
thread_local Pinned g_pinned;

void* pinned(size_t bytes) {
  if (g_pinned.cap >= bytes) return g_pinned.p;
  if (g_pinned.p) (void)hipHostFree(g_pinned.p);
  g_pinned.p = nullptr;
  g_pinned.cap = 0;
  size_t cap = std::max<size_t>(bytes, 1 << 16);
  if (hipHostMalloc(&g_pinned.p, cap, hipHostMallocDefault) != hipSuccess) {
    g_pinned.p = nullptr;
    return nullptr;
  }
  g_pinned.cap = cap;
  return g_pinned.p;
}

double now_s() {
  using namespace std::chrono;
  return duration<double>(steady_clock::now().time_since_epoch()).count();
}

#define HC(expr)                                                                   \
  do {                                                                             \
    hipError_t _e = (expr);                                                        \
    if (_e != hipSuccess) {                                                        \
      set_error(std::string("HIP error at ") + #expr + ": " + hipGetErrorString(_e)); \
      return GENIOS_ERR_DEVICE;                                                    \
    }                                                                              \
  } while (0)

int elem_size(MType mt) { return mt == MT_BF16 ? 2 : (mt == MT_F32 ? 4 : 8); }

}  // namespace

struct Arena {
  char* base;
  size_t cap, off = 0;
  bool dry;
  void* take(size_t bytes) {
    off = (off + 255) / 256 * 256;
    char* p = dry ? nullptr : base + off;
    off += bytes;
    return p;
  }
};

void set_error(const std::string& s) { g_err = s; }
const char* last_error() { return g_err.c_str(); }

// ---------------------------------------------------------------------------------
// Workspace layout

void Layout::carve(Arena& ar) {
  const size_t ve = vt == VT_F32 ? 4 : 8;
  const int64_t B = batch;
  ctrl.params = static_cast<ProbParams*>(ar.take(B * sizeof(ProbParams)));
  ctrl.state = static_cast<ProbState*>(ar.take(B * sizeof(ProbState)));
  ctrl.counters = static_cast<unsigned*>(ar.take(B * kNumCounters * sizeof(unsigned)));
  ctrl.coef = static_cast<double*>(ar.take(B * 2 * kMaxS * sizeof(double)));
  ctrl.s_eff = static_cast<int32_t*>(ar.take(B * sizeof(int32_t)));
  ctrl.lamhat = static_cast<double*>(ar.take(B * std::max(1, s) * sizeof(double)));
  ctrl.s_stride = std::max(1, s);
  ctrl.part_stride = (int64_t)part_blocks * kPartW;
  ctrl.part = static_cast<double*>(ar.take(B * ctrl.part_stride * sizeof(double)));
  ctrl.pstride = part_blocks;
  ctrl.spart = static_cast<double*>(ar.take(B * kNumSlots * ctrl.pstride * sizeof(double)));
  ctrl.upart = static_cast<double*>(ar.take(B * kMaxS * ctrl.pstride * sizeof(double)));
  ctrl_bytes_end = ar.off;
  core_status = static_cast<int32_t*>(ar.take(B * sizeof(int32_t)));
  shift = static_cast<double*>(ar.take(B * sizeof(double)));
  scal = static_cast<double*>(ar.take(B * 8 * sizeof(double)));
  if (need_a16) A16 = static_cast<uint16_t*>(ar.take(a16_elems * 2));
  auto vec = [&](int64_t len) { return ar.take((size_t)B * len * ve); };
  for (int k = 0; k < kNumNVec; ++k) nv[k] = n_vecs > k ? vec(n) : nullptr;
  tparts = ar.take((size_t)B * nsplit_n * m * ve);
  ypart = ar.take((size_t)B * yprob() * ve);
  hpq = static_cast<double*>(ar.take((size_t)B * yslots * sizeof(double)));
  if (gap) {
    gapf = vec(m);
    gaps = vec(m);
    gpart = static_cast<double*>(ar.take((size_t)B * kGapSlots * kGapPStride * sizeof(double)));
    gstate = static_cast<GapState*>(ar.take((size_t)B * sizeof(GapState)));
  }
  if (ml || backward) {
    dvec = vec(m);
    cols = ar.take((size_t)B * 2 * m * ve);
  }
  if (backward) {
    mask = static_cast<uint8_t*>(ar.take((size_t)B * n));
    idx = static_cast<int32_t*>(ar.take((size_t)B * n * sizeof(int32_t)));
    cnt = static_cast<int32_t*>(ar.take((size_t)B * sizeof(int32_t)));
    AS = ar.take((size_t)B * m * ldS_max * ve);
    maskS = static_cast<uint8_t*>(ar.take((size_t)B * ldS_max));
  }
  if (mr.sp > 0) {
    const int64_t kpn = (n + 31) / 32 * 32, kpm = (m + 31) / 32 * 32;
    mr.p16 = static_cast<uint16_t*>(ar.take((size_t)2 * mr.sp * kpn * sizeof(uint16_t)));
    mr.w16 = static_cast<uint16_t*>(ar.take((size_t)2 * mr.sp * kpm * sizeof(uint16_t)));
    mr.wpart = static_cast<float*>(ar.take((size_t)mr.ksW * mr.sp * m * sizeof(float)));
  }
  if (s > 0) {
    pm_est = static_cast<double*>(ar.take((size_t)B * sizeof(double)));
    U = vec(n * (int64_t)s);
    const int sp = sketch_pad(s);
    sk.omega = vec(n * (int64_t)sp);
    sk.W = vec(m * (int64_t)sp);
    sk.Wpart = ar.take((size_t)B * sk.ksW * m * sp * ve);
    sk.Ypart = ar.take((size_t)B * sk.ksY * n * sp * ve);
    sk.Y = vec(n * (int64_t)sp);
    sk.gpart = static_cast<double*>(ar.take((size_t)B * 3 * sk.nbG * sp * sp * sizeof(double)));
    sk.gram = static_cast<double*>(ar.take((size_t)B * 3 * sp * sp * sizeof(double)));
    sk.core = static_cast<double*>(ar.take((size_t)B * 5 * sp * sp * sizeof(double)));
    if (vt == VT_F32) {  // BF16 operands of the matrix-core sketch products
      const int64_t kpn = (n + 31) / 32 * 32, kpm = (m + 31) / 32 * 32;
      sk.o16 = static_cast<uint16_t*>(ar.take((size_t)B * sp * kpn * sizeof(uint16_t)));
      sk.w16 = static_cast<uint16_t*>(ar.take((size_t)2 * B * sp * kpm * sizeof(uint16_t)));
    }
  }
  total = ar.off + 256;
}

int Layout::setup(int op_, const genios_matrix* A, const genios_opts* o, int s_) {
  op = op_;
  m = A->m;
  n = A->n;
  batch = A->batch;
  vt = A->hi_dtype == GENIOS_DT_F64 ? VT_F64 : VT_F32;
  ml = op == GENIOS_OP_LOGREG || op == GENIOS_OP_HUBER;
  backward = op == GENIOS_OP_BACKWARD;
  gap = op == GENIOS_OP_LASSO || op == GENIOS_OP_BOXLS || ml;
  s = s_;
  const int prec = o->precision;
  const bool uses_lo = (op == GENIOS_OP_LASSO || op == GENIOS_OP_BOXLS || ml ||
                        op == GENIOS_OP_NYSTROM ||
                        op == GENIOS_OP_MATVEC || op == GENIOS_OP_HVP) &&
                       (prec == GENIOS_PREC_BF16_REFINE || prec == GENIOS_PREC_BF16_ONLY);
  need_a16 = uses_lo && A->A_bf16 == nullptr;
  // exact extent of the matrix elements (the padding after the last row is not read)
  a16_elems = (A->stride_A == 0 ? 0 : (A->batch - 1) * A->stride_A) + (A->m - 1) * A->lda + A->n;
  MatArg probe{nullptr, vt == VT_F64 ? MT_F64 : MT_F32, m, n, A->lda, A->stride_A};
  MatArg probe_lo{nullptr, MT_BF16, m, n, A->lda, A->stride_A};
  nsplit_n = std::max(gemv_n_splits(probe, batch), uses_lo ? gemv_n_splits(probe_lo, batch) : 1);
  nrhs = ml ? 2 : 1;
  ksplit = std::max(gemv_t_splits(probe, batch), uses_lo ? gemv_t_splits(probe_lo, batch) : 1);
  // partial slots of A^T products: gemv_t's row splits or the fused H p's blocks
  const bool cg_op = op == GENIOS_OP_LASSO || op == GENIOS_OP_BOXLS || ml ||
                     op == GENIOS_OP_BACKWARD || op == GENIOS_OP_HVP;
  yslots = std::max<int64_t>((int64_t)ksplit * (ml ? 2 : 1),
                             cg_op ? std::max<int64_t>(1, kHvpMaxBlocks / batch) : 1);
  if (cg_op && op != GENIOS_OP_HVP && batch > 1 && vt == VT_F32) {
    // room for one problem's whole-chip grid of the fused H p, used once few problems
    // of the batch still run (bounded: at most 2 GiB of partials over the batch); only
    // the gated products of a CG loop take that shape, so a lone H p reserves none
    int64_t g1 = hvp_geometry(probe, 1, false).blocks;
    if (uses_lo) g1 = std::max<int64_t>(g1, hvp_geometry(probe_lo, 1, false).blocks);
    const int64_t budget = ((int64_t)1 << 31) / (batch * ((n + 7) / 8 * 8) * (int64_t)sizeof(float));
    yslots = std::max<int64_t>(yslots, std::min<int64_t>(g1, budget));
  }
  npad = (n + 7) / 8 * 8;
  chunk = vec_chunk(n);
  nb = (int)((n + chunk - 1) / chunk);
  part_blocks = std::max<int>(std::max<int>(nb, (int)vec_blocks_max(n)),
                              std::max<int>(kMaxVecBlocks, (int)((n + kVecChunk - 1) / kVecChunk)));
  n_vecs = (op == GENIOS_OP_MATVEC || op == GENIOS_OP_NYSTROM || op == GENIOS_OP_HVP) ? 0 : kNumNVec;
  // columns of the gathered A_S: |S| <= min(m, n) without the l2 term (else A_S^T A_S
  // is singular and the call fails), up to n with it
  ldS_max = backward ? (int)(((o->lambda2 > 0.0 ? n : std::min(m, n)) + 7) / 8 * 8) : 0;
  if (s > 0) sketch_ws_bytes(m, n, s, batch, vt, &sk.ksW, &sk.ksY, &sk.nbG);
  // H p of a batch sharing A on the matrix cores (every loss; BF16 or FP32 operand)
  mr = MrhsWs{};
  const bool shared = A->stride_A == 0 && batch >= 2 && batch <= 128;
  const bool sq_op = op == GENIOS_OP_LASSO || op == GENIOS_OP_BOXLS || op == GENIOS_OP_HVP || ml;
  const int64_t min_batch = o->batch_mfma == 2 ? 2 : 5;
  if (o->batch_mfma != 0 && shared && batch >= min_batch && sq_op && vt == VT_F32 &&
      n % 8 == 0 && A->lda % 8 == 0) {
    mr.sp = mrhs_pad((int)batch);
    const int64_t rb = (m + 127) / 128, cb = (n + 127) / 128, cbf = (n + 255) / 256;
    mr.ksW = (int)std::max<int64_t>(1, std::min<int64_t>((2048 + rb - 1) / rb, std::max<int64_t>(1, n / 256)));
    int64_t ky = std::max<int64_t>(1, std::min<int64_t>((2048 + cb - 1) / cb, std::max<int64_t>(1, m / 256)));
    ky = std::min<int64_t>(ky, batch * yslots / mr.sp);  // ypart holds ksY x sp columns
    mr.ksY = (int)std::max<int64_t>(1, ky);
    ky = std::max<int64_t>(1, std::min<int64_t>((2048 + cbf - 1) / cbf, std::max<int64_t>(1, m / 256)));
    mr.ksYf = (int)std::max<int64_t>(1, std::min<int64_t>(ky, batch * yslots / mr.sp));
    if (batch * yslots < mr.sp) mr.sp = 0;  // cannot happen: yslots >= 512 / batch
  }
  Arena ar{nullptr, 0, 0, true};
  carve(ar);
  return 0;
}

int Layout::bind(void* base, size_t bytes) {
  if (base == nullptr || reinterpret_cast<uintptr_t>(base) % 256 != 0 || bytes < total) {
    set_error("workspace missing, misaligned (256 B) or smaller than genios_workspace_size");
    return GENIOS_ERR_WORKSPACE;
  }
  Arena ar{static_cast<char*>(base), bytes, 0, false};
  carve(ar);
  return 0;
}

// ---------------------------------------------------------------------------------
// Solver context

namespace {

struct Timer {
  hipEvent_t ev[4] = {nullptr, nullptr, nullptr, nullptr};
  bool ok = false;
  ~Timer() {
    for (auto& e : ev)
      if (e) (void)hipEventDestroy(e);
  }
  hipError_t init() {
    for (auto& e : ev) {
      hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) return r;
    }
    ok = true;
    return hipSuccess;
  }
};

struct KernelProf {
  bool on = false;
  std::vector<hipEvent_t> evs;
  // 0 = A v, 1 = A^T w, 2 / 3 = fused H p on the BF16 / master copy,
  // 4 / 5 = sketch products on the matrix cores / vector units,
  // 6 = H p of a batch sharing A on the matrix cores
  std::vector<int> kind;
  size_t used = 0;
  double t[7] = {0, 0, 0, 0, 0, 0, 0};
  ~KernelProf() {
    for (auto e : evs) (void)hipEventDestroy(e);
  }
  hipError_t grow() {
    if (used + 2 <= evs.size()) return hipSuccess;
    for (int i = 0; i < 64; ++i) {
      hipEvent_t e;
      hipError_t r = hipEventCreate(&e);
      if (r != hipSuccess) return r;
      evs.push_back(e);
    }
    kind.resize(evs.size() / 2 + 1);
    return hipSuccess;
  }
  hipError_t begin(hipStream_t st, int k) {
    if (!on) return hipSuccess;
    hipError_t r = grow();
    if (r != hipSuccess) return r;
    kind[used / 2] = k;
    return hipEventRecord(evs[used], st);
  }
  // a begin / end pair that the callee records (both null when off)
  hipError_t reserve(int k, hipEvent_t* b, hipEvent_t* e) {
    *b = *e = nullptr;
    if (!on) return hipSuccess;
    hipError_t r = grow();
    if (r != hipSuccess) return r;
    kind[used / 2] = k;
    *b = evs[used];
    *e = evs[used + 1];
    used += 2;
    return hipSuccess;
  }
  hipError_t end(hipStream_t st) {
    if (!on) return hipSuccess;
    hipError_t r = hipEventRecord(evs[used + 1], st);
    used += 2;
    return r;
  }
  // call after a stream synchronisation
  void harvest() {
    for (size_t i = 0; i + 1 < used; i += 2) {
      float ms = 0.f;
      if (hipEventElapsedTime(&ms, evs[i], evs[i + 1]) == hipSuccess) t[kind[i / 2]] += ms * 1e-3;
    }
    used = 0;
  }
};

struct Ctx {
  const genios_matrix* A;
  const genios_opts* o;
  Layout L;
  hipStream_t st;
  MatArg op_hi{}, op_lo{};
  int64_t B, m, n;
  VType vt;
  size_t ve;
  int32_t* gate_cg = nullptr;    // &state[0].cg_active
  int32_t* gate_done = nullptr;  // &state[0].admm_done
  int32_t* gate_run = nullptr;   // &params[0].run
  int gs_state = sizeof(ProbState) / 4, gs_params = sizeof(ProbParams) / 4;
  const void* box_lo = nullptr;  // box bounds of a kProxBox solve (n per problem)
  const void* box_hi = nullptr;
  KernelProf prof;
  int64_t n_mv[4] = {0, 0, 0, 0};
  int64_t n_mrhs = 0, bytes_mrhs = 0;  // H p launches of a batch sharing A (all problems at once)
  // fused H p launch shapes used once part of a batch has stopped: one whole-chip launch
  // per running problem (counted per problem), and the batch grid sized for the running
  // count (counted per launch)
  int64_t n_tail = 0, n_resized = 0;
  // the last product was the fused one, so L.hpq holds its per-block p^T H p partials
  bool pq_rows = false;
  // problems taking part in the coming kernels (set with the parameters; -1: all)
  std::vector<char> run_flags;
  int64_t running = -1;
  int batch_mode = 1;  // opts.batch_mfma
  // bytes of A v / A^T w (the matrix) and of the fused H p on the BF16 / master copy
  // (the matrix once, p read, H p written)
  int64_t bytes_kind[4] = {0, 0, 0, 0};
  // sketches on the matrix cores / vector units and their algorithmic flops (4 m n s)
  int64_t n_sketch[2] = {0, 0};
  int64_t flops_sketch[2] = {0, 0};

  // the sketch-product timer of one Nystrom build of operator op at rank s
  hipError_t sketch_timer(const MatArg& op, int s, SketchWs* skc) {
    const int k = sketch_mfma_eligible(op, vt, *skc) ? 0 : 1;
    n_sketch[k] += 1;
    flops_sketch[k] += B * 4 * op.m * op.n * (int64_t)s;
    return prof.reserve(4 + k, &skc->ev_gemm[0], &skc->ev_gemm[1]);
  }
  template <typename I>
  void fill_sketch_info(I& info) const {
    info.t_sketch_mc = prof.t[4];
    info.flops_sketch_mc = flops_sketch[0];
    info.n_sketch_mc = (int32_t)n_sketch[0];
    info.t_sketch_fma = prof.t[5];
    info.flops_sketch_fma = flops_sketch[1];
    info.n_sketch_fma = (int32_t)n_sketch[1];
  }

  void* vecp(int k) const { return L.nv[k]; }
  VecArgs vargs(void* x, void* z, void* u, void* h, void* g, void* c, const uint8_t* mask) const {
    VecArgs a{};
    a.vt = vt;
    a.n = n;
    a.batch = B;
    a.nb = L.nb;
    a.chunk = L.chunk;
    a.ctrl = L.ctrl;
    a.x = x;
    a.z = z;
    a.u = u;
    a.h = h;
    a.g = g;
    a.c = c;
    a.r = L.nv[kVR];
    a.p = L.nv[kVP];
    a.hp = L.nv[kVHP];
    a.w = L.nv[kVW];
    a.U = L.s > 0 ? L.U : nullptr;
    a.s_stride = std::max(1, L.s);
    a.ypart = L.ypart;
    a.ksplit = L.ksplit;
    a.ypart_ks_stride = (int64_t)L.nrhs * L.npad;
    a.ypart_prob_stride = L.yprob();
    a.mask = mask;
    a.chunkf = vec_chunk_fine(n);
    a.nbf = (int)((n + a.chunkf - 1) / a.chunkf);
    a.lo = box_lo;
    a.hi = box_hi;
    return a;
  }

  void account(const MatArg& op, int kind) {
    n_mv[kind] += B;
    bytes_kind[kind] += (int64_t)B * op.m * op.n * elem_size(op.mt);
    if (kind >= 2) bytes_kind[kind] += (int64_t)B * op.n * 2 * (int64_t)ve;
  }
  static int hvp_kind(const MatArg& op) { return op.mt == MT_BF16 ? 2 : 3; }
  // Remove `count` problem-launches of the last CG product (gated off on the device:
  // enqueued but skipped because the problem's CG had already stopped).
  int last_hvp_kind = -1;  // 2 / 3: fused; 0: gemv_n + gemv_t
  MatArg last_hvp_op{};
  void unaccount_gated(int64_t count) {
    if (count <= 0 || last_hvp_kind < 0) return;
    const MatArg& op = last_hvp_op;
    const int64_t mat = (int64_t)op.m * op.n * elem_size(op.mt);
    if (last_hvp_kind >= 2) {
      n_mv[last_hvp_kind] -= count;
      bytes_kind[last_hvp_kind] -= count * (mat + (int64_t)op.n * 2 * (int64_t)ve);
    } else {
      n_mv[0] -= count;
      n_mv[1] -= count;
      bytes_kind[0] -= count * mat;
      bytes_kind[1] -= count * mat;
    }
  }

  // tparts = A v (gated)
  int gemv_n(const MatArg& op, const void* v, const int32_t* gate, int gstride) {
    HC(prof.begin(st, 0));
    HC(launch_gemv_n(op, B, vt, v, n, L.tparts, m, (int64_t)L.nsplit_n * m, nsplit_for(op, 0),
                     gate, gstride, st));
    HC(prof.end(st));
    account(op, 0);
    return 0;
  }
  int nsplit_for(const MatArg& op, int which) const {
    if (which == 0) return std::min(L.nsplit_n, gemv_n_splits(op, B));
    return std::min(L.ksplit, gemv_t_splits(op, B));
  }
  // ypart = A^T (d o t) from tparts (gated)
  int gemv_t_from_t(const MatArg& op, const void* d, const int32_t* gate, int gstride,
                    int nsplit_in) {
    HC(prof.begin(st, 1));
    const int ks = nsplit_for(op, 1);
    HC(launch_gemv_t(op, B, vt, L.tparts, nsplit_in, m, (int64_t)L.nsplit_n * m, 0, 1, d, m,
                     L.ypart, ks, (int64_t)L.nrhs * L.npad, L.npad,
                     L.yprob(), gate, gstride, st));
    HC(prof.end(st));
    cur_ks = ks;
    cur_ks_stride = (int64_t)L.nrhs * L.npad;
    cur_prob_stride = L.yprob();
    account(op, 1);
    return 0;
  }
  // ypart = H p = A^T (d o (A p)) (gated): one pass over A when it qualifies for
  // the fused kernel, else gemv_n then gemv_t.
  int64_t mrhs_bytes(const MatArg& op) const {
    return 2 * op.m * op.n * elem_size(op.mt) + (int64_t)B * op.n * 2 * (int64_t)ve;
  }
  void unaccount_mrhs(int64_t launches) {
    if (launches <= 0 || last_hvp_kind != 6) return;
    n_mrhs -= launches;
    bytes_mrhs -= launches * mrhs_bytes(last_hvp_op);
  }
  int hvp(const MatArg& op, const void* p, const void* d, const int32_t* gate, int gstride) {
    // a batch sharing A: both passes over A serve every problem (matrix cores)
    // (two streams of A beat one whole-chip fused pass per running problem from 3 (FP32)
    // or 4 (BF16) running problems on; batch_mfma = 2 keeps them down to 2)
    const int64_t min_run = batch_mode == 2 ? 2 : (op.mt == MT_F32 ? 3 : 4);
    if (L.mr.sp > 0 && (running < 0 || running >= min_run) && mrhs_eligible(op, vt, B, L.mr)) {
      HC(prof.begin(st, 6));
      HC(launch_mrhs_hvp(op, (int)B, static_cast<const float*>(p), n,
                         static_cast<const float*>(d), m, L.mr,
                         static_cast<float*>(L.ypart), L.npad, gate, gstride, st));
      HC(prof.end(st));
      pq_rows = false;
      cur_ks = op.mt == MT_F32 ? L.mr.ksYf : L.mr.ksY;
      cur_ks_stride = (int64_t)L.mr.sp * L.npad;
      cur_prob_stride = L.npad;
      n_mrhs += 1;
      bytes_mrhs += mrhs_bytes(op);
      last_hvp_kind = 6;
      last_hvp_op = op;
      return 0;
    }
    cur_prob_stride = L.yprob();
    if (vt == VT_F32) {
      const HvpGeom g = hvp_geometry(op, B, true);
      // a batch with few problems still running: one launch per running problem over
      // the whole chip (the batched grid gives each problem a 1/B share of it).  Gated
      // products only: their gate (run or cg_active) is clear for every problem left out,
      // while an ungated product (the power method's) is wanted for all of them.
      if (B > 1 && gate != nullptr && running >= 1 && running <= 8 && g.threads > 0 &&
          hvp_p_aligned(p, n, B)) {
        const HvpGeom g1 = hvp_geometry(op, 1, true);
        if (g1.threads > 0 && g1.blocks >= 2 * g.blocks && g1.blocks <= L.yslots) {
          HC(prof.begin(st, hvp_kind(op)));
          const size_t es = elem_size(op.mt);
          for (int64_t b = 0; b < B; ++b) {
            if (!run_flags[b]) continue;
            MatArg ob = op;
            ob.ptr = static_cast<const char*>(op.ptr) + (size_t)(b * op.strideA) * es;
            HC(launch_hvp_fused(ob, g1, 1, static_cast<const float*>(p) + b * n, n,
                                d ? static_cast<const float*>(d) + b * m : nullptr, m,
                                static_cast<float*>(L.ypart) + b * L.yprob(), L.npad, L.yprob(),
                                gate ? gate + b * gstride : nullptr, gstride, st,
                                L.hpq + b * L.yslots, L.yslots));
          }
          HC(prof.end(st));
          pq_rows = true;
          for (int64_t b = 0; b < B; ++b) n_tail += run_flags[b] ? 1 : 0;
          cur_ks = g1.blocks;
          cur_ks_stride = L.npad;
          account(op, hvp_kind(op));
          last_hvp_kind = hvp_kind(op);
          last_hvp_op = op;
          return 0;
        }
      }
      // more than 8 but not all running, problems of 256 MB or more: the grid over the
      // batch sized for the running problems (the stopped ones' blocks exit at their
      // gate; on small problems those empty blocks cost more than the wider grid gains)
      const bool big = op.m * op.n * (int64_t)elem_size(op.mt) >= ((int64_t)256 << 20);
      const HvpGeom gr = B > 1 && big && gate != nullptr && running >= 1 && running < B
                             ? hvp_geometry(op, running, true)
                             : HvpGeom{};
      const HvpGeom& gb = gr.threads > 0 && gr.blocks <= L.yslots ? gr : g;
      if (gb.threads > 0 && gb.blocks <= L.yslots && hvp_p_aligned(p, n, B)) {
        HC(prof.begin(st, hvp_kind(op)));
        HC(launch_hvp_fused(op, gb, B, static_cast<const float*>(p), n,
                            static_cast<const float*>(d), m, static_cast<float*>(L.ypart), L.npad,
                            L.yprob(), gate, gstride, st, L.hpq, L.yslots));
        HC(prof.end(st));
        pq_rows = true;
        if (&gb == &gr) n_resized += 1;
        cur_ks = gb.blocks;
        cur_ks_stride = L.npad;
        account(op, hvp_kind(op));
        last_hvp_kind = hvp_kind(op);
        last_hvp_op = op;
        return 0;
      }
    }
    last_hvp_kind = 0;
    last_hvp_op = op;
    pq_rows = false;
    int rc = gemv_n(op, p, gate, gstride);
    if (rc) return rc;
    return gemv_t_from_t(op, d, gate, gstride, nsplit_for(op, 0));
  }
  int cur_ks = 1;
  int64_t cur_ks_stride = 0;
  int64_t cur_prob_stride = 0;  // per-problem stride of the last product's partials
};

// h = H x outside CG (warm start, precision switch, certification): the fused
// one-pass product where A qualifies, else A x then A^T (d o t).
int hvp_explicit(Ctx& c, const MatArg& op, const void* x, void* h, const void* d,
                 const int32_t* gate, int gstride) {
  int rc = c.hvp(op, x, d, gate, gstride);
  if (rc) return rc;
  HC(launch_sum_splits(c.vt, c.B, c.n, c.L.ypart, c.cur_ks, c.cur_ks_stride, c.cur_prob_stride,
                       h, c.n, c.st, gate, gstride));
  return 0;
}

}  // namespace

// ---------------------------------------------------------------------------------
// ADMM driver shared by the Lasso, the logistic regression and Huber fitting.

namespace {

struct HostProb {
  double lambda, rho;
  double u_scale = 1.0;
  double rp_prev = INFINITY, rd_prev = INFINITY;
  int done = 0;
  int status = 0;
  int iters = 0, cg_total = 0, last_cg = 2;
  double rkkt = INFINITY, rp = 0, rd = 0, xn = 0, zn = 0, un = 0;
  double t_target = -1.0;
  int switch_iter = -1, resketches = 0;
  int gap_checks = 0;
  int precond_rank = 0, sketch_rounds = 0;
  bool rd_exact = false;  // rd is r_d at the final x with the master copy
  double sketch_err = 0.0, kappa_bound = 0.0;
  std::vector<double> rk_hist;
};

double kkt_from(double rp, double rd, double xn, double zn, double rhou, int64_t n) {
  const double sn = std::sqrt((double)n);
  const double a = rp / (sn + std::max(xn, zn));
  const double b = rd / (sn + rhou);
  return std::max(a, b);
}

bool paper_test(double rp, double rd, double xn, double zn, double rhou, int64_t n,
                double eps_abs, double eps_rel) {
  const double sn = std::sqrt((double)n);
  return rp <= sn * eps_abs + eps_rel * std::max(xn, zn) && rd <= sn * eps_abs + eps_rel * rhou;
}

int sync_state(Ctx& c, ProbState* hs) {
  HC(hipMemcpyAsync(hs, c.L.ctrl.state, c.B * sizeof(ProbState), hipMemcpyDeviceToHost, c.st));
  HC(hipStreamSynchronize(c.st));
  c.prof.harvest();
  return 0;
}

// Also records which problems take part in the coming kernels (the H p launch shape
// depends on how many do).
hipError_t upload_params(Ctx& c, ProbParams* hp) {
  c.run_flags.assign(c.B, 0);
  c.running = 0;
  for (int64_t b = 0; b < c.B; ++b)
    if (hp[b].run) {
      c.run_flags[b] = 1;
      ++c.running;
    }
  return hipMemcpyAsync(c.L.ctrl.params, hp, c.B * sizeof(ProbParams), hipMemcpyHostToDevice, c.st);
}

// The x-system set-up up to the first search direction (kernels gated on run).
int cg_setup(Ctx& c, const VecArgs& va) {
  HC(launch_admm_begin(va, c.st));
  HC(launch_precond_coef(va, va.nbf, c.st));
  HC(launch_precond_p(va, 0, 1, va.nbf, c.st));
  return 0;
}

// The vector part of CG iteration t (kernels gated on cg_active).  After the fused
// product (pq_rows: its per-block p^T H p partials are in a.hpq) one kernel takes the
// step; after the others hp is summed first.
int cg_vector_step(Ctx& c, const VecArgs& a, int t, bool pq_rows) {
  int np;
  if (pq_rows) {
    HC(launch_cg_step(a, t, c.st));
    np = a.nbf;
  } else {
    HC(launch_cg_alpha(a, c.st));
    HC(launch_cg_update(a, t, c.st));
    np = a.nb;
  }
  HC(launch_precond_coef(a, np, c.st));
  HC(launch_precond_p(a, t, 0, np, c.st));
  return 0;
}

// CG iteration t for all problems.
int cg_iteration(Ctx& c, const MatArg& op, const VecArgs& va, const void* dscale, int t) {
  int rc = c.hvp(op, va.p, dscale, c.gate_cg, c.gs_state);
  if (rc) return rc;
  VecArgs a = va;
  a.ksplit = c.cur_ks;
  a.ypart_ks_stride = c.cur_ks_stride;
  a.ypart_prob_stride = c.cur_prob_stride;
  a.hpq = c.L.hpq;
  a.hpq_stride = c.L.yslots;
  a.nhpq = c.cur_ks;
  return cg_vector_step(c, a, t, c.pq_rows);
}

}  // namespace

int run_admm(const genios_matrix* A, const void* bvec, const double* lambda, double rho0,
             const genios_opts* o, void* x, void* z, void* u, genios_info* info, int loss,
             const ProxSpec& prox) {
  // ml: the loss has curvature D = f''(A x - b) that changes with x (Sec. 3.3)
  const bool ml = loss != kLossSquare;
  const double delta = o->huber_delta;
  const double t0 = now_s();
  Ctx c;
  c.A = A;
  c.o = o;
  c.st = static_cast<hipStream_t>(o->stream);
  c.B = A->batch;
  c.m = A->m;
  c.n = A->n;
  c.vt = A->hi_dtype == GENIOS_DT_F64 ? VT_F64 : VT_F32;
  c.batch_mode = o->batch_mfma;
  c.ve = c.vt == VT_F32 ? 4 : 8;
  const int s = o->precondition ? effective_rank(o, A->n, A->m) : 0;
  c.L.setup(loss == kLossLogistic ? GENIOS_OP_LOGREG
            : loss == kLossHuber    ? GENIOS_OP_HUBER
            : prox.kind == kProxBox ? GENIOS_OP_BOXLS
                                    : GENIOS_OP_LASSO,
            A, o, s);
  c.box_lo = prox.kind == kProxBox ? prox.lo : nullptr;
  c.box_hi = prox.kind == kProxBox ? prox.hi : nullptr;
  int rc = c.L.bind(o->workspace, o->workspace_bytes);
  if (rc) return rc;
  c.prof.on = o->profile_kernels != 0;
  const int prec = o->precision;
  const bool use_lo = prec == GENIOS_PREC_BF16_REFINE || prec == GENIOS_PREC_BF16_ONLY;
  // After the switch to the master copy, CG may keep the BF16 copy as the x-system's
  // Hessian model while the master copy forms H x (the gradient) once per iteration
  // (squared loss only: the curvature-weighted losses keep master-copy CG); by
  // default when the master copy's products are bandwidth-bound.
  const int64_t hi_bytes = A->m * A->n * (int64_t)(c.vt == VT_F64 ? 8 : 4);
  const bool lo_cg = prec == GENIOS_PREC_BF16_REFINE && !ml &&
                     (o->refine_cg_bf16 == 1 ||
                      (o->refine_cg_bf16 < 0 && hi_bytes >= GENIOS_REFINE_CG_BF16_MIN_BYTES));
  c.op_hi = MatArg{A->A_hi, c.vt == VT_F64 ? MT_F64 : MT_F32, A->m, A->n, A->lda, A->stride_A};
  c.op_lo = MatArg{A->A_bf16 ? (const void*)A->A_bf16 : (const void*)c.L.A16, MT_BF16, A->m, A->n,
                   A->lda, A->stride_A};
  c.gate_cg = &c.L.ctrl.state[0].cg_active;
  c.gate_done = &c.L.ctrl.state[0].admm_done;
  c.gate_run = &c.L.ctrl.params[0].run;
  const int64_t B = c.B, n = c.n, m = c.m;
  Timer tm;
  HC(tm.init());

  // ---- setup ----
  HC(launch_fill(c.L.ctrl.params, c.L.ctrl_bytes_end, c.st));
  void* h = c.L.nv[kVH];
  void* g = c.L.nv[kVG];
  void* c_hi = c.L.nv[kVCH];
  void* c_lo = c.L.nv[kVCL];
  // The BF16 copy, and for the squared loss c = A^T b of both operators, in one pass
  // over the FP32 master where the layout allows it (one matrix per problem).
  bool setup_fused = false;
  if (use_lo && A->A_bf16 == nullptr && !ml && c.vt == VT_F32 && (A->stride_A != 0 || B == 1)) {
    const int ksc = cast_atb_splits(m, n, B, (int)(c.L.yslots / 2));
    if (2 * (int64_t)ksc <= c.L.yslots &&
        cast_atb_eligible(A->A_hi, A->lda, A->stride_A, n, c.L.A16, c.L.ypart, c.L.npad)) {
      HC(launch_cast_atb(static_cast<const float*>(A->A_hi), A->lda, A->stride_A, c.L.A16, m, n,
                         B, static_cast<const float*>(bvec), static_cast<float*>(c.L.ypart), ksc,
                         c.L.npad, (int64_t)ksc * c.L.npad, c.L.yprob(), c.st));
      HC(launch_sum_splits(c.vt, B, n, c.L.ypart, ksc, c.L.npad, c.L.yprob(), c_hi, n, c.st));
      HC(launch_sum_splits(c.vt, B, n, static_cast<float*>(c.L.ypart) + (int64_t)ksc * c.L.npad,
                           ksc, c.L.npad, c.L.yprob(), c_lo, n, c.st));
      setup_fused = true;
    }
  }
  if (use_lo && A->A_bf16 == nullptr && !setup_fused) {
    HC(launch_cast_bf16(static_cast<const float*>(A->A_hi), c.L.A16, c.L.a16_elems, c.st));
  }
  if (!o->warm_start) {
    HC(launch_fill(x, B * n * c.ve, c.st));
    HC(launch_fill(z, B * n * c.ve, c.st));
    HC(launch_fill(u, B * n * c.ve, c.st));
  }
  int phase = use_lo ? 0 : 1;
  const MatArg* op = phase == 0 ? &c.op_lo : &c.op_hi;

  std::vector<ProbParams> hpv(B);
  ProbParams* hp = static_cast<ProbParams*>(
      pinned(B * (sizeof(ProbParams) + sizeof(ProbState) + sizeof(GapState))));
  if (!hp) {
    set_error("pinned host staging allocation failed");
    return GENIOS_ERR_DEVICE;
  }
  ProbState* hs = reinterpret_cast<ProbState*>(hp + B);
  GapState* hg = reinterpret_cast<GapState*>(hs + B);
  std::vector<HostProb> P(B);
  for (int64_t b = 0; b < B; ++b) {
    P[b].lambda = lambda[b];
    P[b].rho = rho0;
  }
  auto set_params = [&](int k, bool run_all) {
    for (int64_t b = 0; b < B; ++b) {
      ProbParams& q = hp[b];
      std::memset(&q, 0, sizeof(q));
      q.run = (run_all || !P[b].done) ? 1 : 0;
      q.rho = P[b].rho;
      q.sigma = o->sigma;
      q.nu = P[b].rho + o->sigma + o->lambda2;
      q.kappa = P[b].lambda / P[b].rho;
      q.alpha = o->alpha;
      q.u_scale = P[b].u_scale;
      double rtol;
      if (o->inexact) {
        const double gm = std::sqrt(P[b].rp_prev * P[b].rd_prev);
        rtol = std::min(std::isfinite(gm) ? gm : 1.0, 1.0) / std::pow((double)std::max(k, 1), o->gamma);
        rtol = std::max(rtol, o->cg_tol_floor);
      } else {
        rtol = o->cg_tol_floor;
      }
      q.rtol = rtol;
      q.tol_floor = o->cg_tol_floor;
      q.lambda = P[b].lambda;
      q.lambda2 = o->lambda2;
      q.max_cg = o->max_cg_iter;
      q.rhs_rel = o->rhs_relative;
      q.use_c = ml ? 0 : 1;
      q.prox = prox.kind;
    }
  };

  // Right-hand sides c = A^T b for the Lasso (per operator in use).
  if (!ml && !setup_fused) {
    if (use_lo) {
      HC(launch_gemv_t(c.op_lo, B, c.vt, bvec, 1, 0, m, 0, 1, nullptr, 0, c.L.ypart,
                       c.nsplit_for(c.op_lo, 1), (int64_t)c.L.nrhs * c.L.npad, c.L.npad,
                       c.L.yprob(), nullptr, 0, c.st));
      HC(launch_sum_splits(c.vt, B, n, c.L.ypart, c.nsplit_for(c.op_lo, 1),
                           (int64_t)c.L.nrhs * c.L.npad, c.L.yprob(),
                           c_lo, n, c.st));
    }
    // with the master copy in every precision: the final report's r_d uses it
    HC(launch_gemv_t(c.op_hi, B, c.vt, bvec, 1, 0, m, 0, 1, nullptr, 0, c.L.ypart,
                     c.nsplit_for(c.op_hi, 1), (int64_t)c.L.nrhs * c.L.npad, c.L.npad,
                     c.L.yprob(), nullptr, 0, c.st));
    HC(launch_sum_splits(c.vt, B, n, c.L.ypart, c.nsplit_for(c.op_hi, 1),
                         (int64_t)c.L.nrhs * c.L.npad, c.L.yprob(), c_hi, n, c.st));
  }
  // Every problem runs during setup passes.
  set_params(1, true);
  HC(upload_params(c, hp));
  // h = H x (zero for a cold start)
  auto gradient_pass = [&](const MatArg& opx, const int32_t* gate, int gstride) -> int {
    // ML losses: t = A x, d = f''(t), columns, [A^T (d o t), A^T f'(t)] -> h, g
    int r = c.gemv_n(opx, x, gate, gstride);
    if (r) return r;
    HC(launch_loss_elem(c.vt, loss, delta, m, B, c.L.tparts, c.nsplit_for(opx, 0), m,
                        (int64_t)c.L.nsplit_n * m, bvec, c.L.dvec, c.L.cols, m, gate,
                        gstride, c.st));
    HC(c.prof.begin(c.st, 1));
    const int ks = c.nsplit_for(opx, 1);
    HC(launch_gemv_t(opx, B, c.vt, c.L.cols, 1, 0, 2 * m, m, 2, nullptr, 0, c.L.ypart, ks,
                     (int64_t)2 * c.L.npad, c.L.npad, c.L.yprob(), gate,
                     gstride, c.st));
    HC(c.prof.end(c.st));
    c.account(opx, 1);
    HC(launch_sum_splits(c.vt, B, n, c.L.ypart, ks, (int64_t)2 * c.L.npad,
                         c.L.yprob(), h, n, c.st, gate, gstride));
    HC(launch_sum_splits(c.vt, B, n, static_cast<char*>(c.L.ypart) + c.L.npad * c.ve, ks,
                         (int64_t)2 * c.L.npad, c.L.yprob(), g, n, c.st,
                         gate, gstride));
    return 0;
  };
  // Relative duality gap at v with operator opx (App. A): t = A v, f'(t), A^T f'(t),
  // then the reductions; the result lands in hg after read_gap().
  auto eval_gap = [&](const MatArg& opx, const void* v, const int32_t* gate, int gstride) -> int {
    int r = c.gemv_n(opx, v, gate, gstride);
    if (r) return r;
    // every field is set before the first launch
    const int ks = c.nsplit_for(opx, 1);
    GapArgs ga{};
    ga.vt = c.vt;
    ga.m = m;
    ga.n = n;
    ga.batch = B;
    ga.tparts = c.L.tparts;
    ga.nsplit = c.nsplit_for(opx, 0);
    ga.split_stride = m;
    ga.prob_stride = (int64_t)c.L.nsplit_n * m;
    ga.bvec = bvec;
    ga.loss = loss;
    ga.delta = delta;
    ga.fprime = c.L.gapf;
    ga.sfold = c.L.gaps;
    ga.ypart = c.L.ypart;
    ga.ks = ks;
    ga.ks_stride = (int64_t)c.L.nrhs * c.L.npad;
    ga.yprob = c.L.yprob();
    ga.v = v;
    ga.params = c.L.ctrl.params;
    ga.lo = c.box_lo;
    ga.hi = c.box_hi;
    ga.part = c.L.gpart;
    ga.state = c.L.gstate;
    HC(launch_gap_elem(ga, c.st));
    HC(c.prof.begin(c.st, 1));
    HC(launch_gemv_t(opx, B, c.vt, c.L.gapf, 1, 0, m, 0, 1, nullptr, 0, c.L.ypart, ks,
                     (int64_t)c.L.nrhs * c.L.npad, c.L.npad, c.L.yprob(), gate, gstride, c.st));
    HC(c.prof.end(c.st));
    c.account(opx, 1);
    HC(launch_gap_after_t(ga, c.st));
    return 0;
  };
  auto read_gap = [&]() -> int {
    HC(hipMemcpyAsync(hg, c.L.gstate, B * sizeof(GapState), hipMemcpyDeviceToHost, c.st));
    HC(hipStreamSynchronize(c.st));
    c.prof.harvest();
    return 0;
  };
  if (ml) {
    rc = gradient_pass(*op, nullptr, 0);
    if (rc) return rc;
  } else if (o->warm_start) {
    rc = hvp_explicit(c, *op, x, h, nullptr, nullptr, 0);
    if (rc) return rc;
  } else {
    HC(launch_fill(h, B * n * c.ve, c.st));
  }
  // Nystrom sketch of the operator in use (Lasso: once; ML losses: at k = 1, 1 + every, ...).
  // With adaptive_sketch the size doubles from sketch_rank_init up to s until the bound
  // 1 + (lam_hat_rr + ||E||) / nu of Sec. 2.2 is <= sketch_kappa for every problem of the
  // batch, ||E|| from power_iters steps of the power method on E = H - U lam_hat U^T.
  double t_precond = 0.0;
  std::vector<int32_t> se_h(B, 0);
  std::vector<double> lam_h, est_h(B, 0.0);
  int sketch_rounds = 0;
  auto build_at = [&](const MatArg& opx, const void* d, int r) -> int {
    SketchWs skx = c.L.sk;
    HC(c.sketch_timer(opx, r, &skx));
    HC(run_nystrom(opx, B, c.vt, d, m, r, nullptr, o->seed, 0, nullptr, skx, c.L.U,
                   c.L.ctrl.lamhat, c.L.ctrl.s_eff, c.L.core_status, c.L.shift, c.st));
    // U (n x r per problem) and lam_hat (r per problem) are packed at the built rank
    c.L.s = r;
    c.L.ctrl.s_stride = r;
    return 0;
  };
  auto sketch_error = [&](const MatArg& opx, const void* d) -> int {
    PowerArgs pa{};
    pa.vt = c.vt;
    pa.n = n;
    pa.batch = B;
    pa.U = c.L.U;
    pa.s_stride = c.L.s;
    pa.lamhat = c.L.ctrl.lamhat;
    pa.s_eff = c.L.ctrl.s_eff;
    pa.h = c.L.nv[kVHP];
    pa.v = c.L.nv[kVR];
    pa.ev = c.L.nv[kVW];
    pa.ut_part = c.L.ctrl.upart;
    pa.part2 = c.L.ctrl.spart;
    pa.pstride = c.L.ctrl.pstride;
    pa.nb = power_blocks(n, c.L.ctrl.pstride);
    pa.est = c.L.pm_est;
    HC(launch_gaussian(c.vt, n, 1, 1, B, o->seed, kPowerStream, nullptr, pa.ev, c.st));
    HC(launch_power_start(pa, c.st));
    for (int it = 0; it < o->power_iters; ++it) {
      int r = hvp_explicit(c, opx, pa.v, c.L.nv[kVHP], d, nullptr, 0);
      if (r) return r;
      HC(launch_power_step(pa, c.st));
    }
    return 0;
  };
  auto read_sketch = [&](bool with_est) -> int {
    const int r = c.L.s;
    lam_h.assign((size_t)B * r, 0.0);
    HC(hipMemcpyAsync(se_h.data(), c.L.ctrl.s_eff, B * sizeof(int32_t), hipMemcpyDeviceToHost, c.st));
    HC(hipMemcpyAsync(lam_h.data(), c.L.ctrl.lamhat, (size_t)B * r * sizeof(double),
                      hipMemcpyDeviceToHost, c.st));
    if (with_est)
      HC(hipMemcpyAsync(est_h.data(), c.L.pm_est, B * sizeof(double), hipMemcpyDeviceToHost, c.st));
    HC(hipStreamSynchronize(c.st));
    for (int64_t b = 0; b < B; ++b) {
      P[b].precond_rank = se_h[b];
      if (!with_est) continue;
      const double lrr = se_h[b] > 0 ? lam_h[(size_t)b * r + se_h[b] - 1] : 0.0;
      P[b].sketch_err = std::max(0.0, est_h[b]);
      P[b].kappa_bound = 1.0 + (lrr + P[b].sketch_err) / (P[b].rho + o->sigma + o->lambda2);
    }
    return 0;
  };
  auto build_sketch = [&](const MatArg& opx, const void* d) -> int {
    if (s <= 0) return 0;
    HC(hipEventRecord(tm.ev[0], c.st));
    int r = o->adaptive_sketch ? std::min(s, std::max(1, o->sketch_rank_init)) : s;
    sketch_rounds = 0;
    for (;;) {
      ++sketch_rounds;
      int rc2 = build_at(opx, d, r);
      if (rc2) return rc2;
      if (!o->adaptive_sketch) {
        rc2 = read_sketch(false);
        if (rc2) return rc2;
        break;
      }
      rc2 = sketch_error(opx, d);
      if (rc2) return rc2;
      rc2 = read_sketch(true);
      if (rc2) return rc2;
      bool met = true;
      for (int64_t b = 0; b < B; ++b)
        if (!(P[b].kappa_bound <= o->sketch_kappa)) met = false;
      if (met || r >= s) break;
      r = std::min(2 * r, s);
    }
    HC(hipEventRecord(tm.ev[1], c.st));
    HC(hipEventSynchronize(tm.ev[1]));
    float ms = 0.f;
    HC(hipEventElapsedTime(&ms, tm.ev[0], tm.ev[1]));
    t_precond += ms * 1e-3;
    for (int64_t b = 0; b < B; ++b) {
      P[b].resketches++;
      P[b].sketch_rounds = sketch_rounds;
    }
    return 0;
  };
  if (!ml) {
    rc = build_sketch(*op, nullptr);
    if (rc) return rc;
  }
  HC(hipStreamSynchronize(c.st));
  const double t_setup = now_s() - t0;

  // ---- ADMM loop ----
  const double eps_abs = o->eps_abs, eps_rel = o->eps_rel;
  const double switch_tol = o->switch_tol > 0 ? o->switch_tol : std::max(eps_abs, eps_rel);
  double t_linsys = 0.0, t_prox = 0.0;
  const double t_loop0 = now_s();
  int any_numeric = 0;
  int k = 0;
  int64_t active = B;
  std::vector<int32_t> core_status(B, 0);
  bool sketch_checked = false;
  auto check_sketch = [&]() -> int {
    HC(hipMemcpyAsync(core_status.data(), c.L.core_status, B * sizeof(int32_t),
                      hipMemcpyDeviceToHost, c.st));
    HC(hipStreamSynchronize(c.st));
    sketch_checked = true;
    return 0;
  };
  if (!ml && s > 0) {
    rc = check_sketch();
    if (rc) return rc;
  }
  while (active > 0 && k < o->max_iter) {
    ++k;
    if (ml && s > 0 && (k - 1) % std::max(1, o->resketch_every) == 0) {
      rc = build_sketch(*op, c.L.dvec);
      if (rc) return rc;
      rc = check_sketch();
      if (rc) return rc;
    }
    set_params(k, false);
    for (int64_t b = 0; b < B; ++b) P[b].u_scale = 1.0;
    HC(upload_params(c, hp));
    VecArgs va = c.vargs(x, z, u, h, g, phase == 0 ? c_lo : c_hi, nullptr);
    HC(hipEventRecord(tm.ev[0], c.st));
    rc = cg_setup(c, va);
    if (rc) return rc;
    int chunk = 1;
    for (int64_t b = 0; b < B; ++b)
      if (!P[b].done) chunk = std::max(chunk, P[b].last_cg);
    chunk = std::min(chunk, o->max_cg_iter);
    int enq = 0;
    // BF16-model CG pays when the iteration's CG products outweigh the extra master
    // pass: k t32 > t32 + k t16 with t16 ~ t32 / 2 at the bandwidth bound, so k >= 3
    // for the predicted count (always with refine_cg_bf16 = 1)
    const bool cg_lo_it = phase == 1 && lo_cg && (o->refine_cg_bf16 == 1 || chunk >= 3);
    const MatArg* cgop = cg_lo_it ? &c.op_lo : op;
    for (;;) {
      for (int it = 0; it < chunk; ++it) {
        rc = cg_iteration(c, *cgop, va, ml ? c.L.dvec : nullptr, enq + it);
        if (rc) return rc;
      }
      enq += chunk;
      HC(hipEventRecord(tm.ev[1], c.st));
      HC(launch_admm_end(va, c.st));
      HC(launch_admm_finish(va, c.st));
      if (cgop != op) {
        // CG ran on the BF16 model: H x at the new x with the master copy (gated on
        // the completed update), then r_d from it -- the right-hand side of the next
        // iteration and the stopping test are the master copy's
        rc = hvp_explicit(c, *op, x, h, nullptr, c.gate_done, c.gs_state);
        if (rc) return rc;
        VecArgs vr = va;
        HC(launch_dual_residual(vr, c.st));
      }
      if (ml) {
        // gradient pass at the new x (gated on the completed update)
        rc = gradient_pass(*op, c.gate_done, c.gs_state);
        if (rc) return rc;
        VecArgs vr = va;
        HC(launch_dual_residual(vr, c.st));
      }
      HC(hipEventRecord(tm.ev[2], c.st));
      rc = sync_state(c, hs);
      if (rc) return rc;
      bool more = false;
      for (int64_t b = 0; b < B; ++b)
        if (hp[b].run && !hs[b].admm_done) more = true;
      if (!more) {
        // products enqueued for problems whose CG had stopped ran as no-ops
        int64_t gated = 0, longest = 0;
        for (int64_t b = 0; b < B; ++b) {
          gated += hp[b].run ? std::max<int64_t>(0, enq - hs[b].cg_iters) : enq;
          if (hp[b].run) longest = std::max<int64_t>(longest, hs[b].cg_iters);
        }
        if (c.last_hvp_kind == 6)
          c.unaccount_mrhs(enq - longest);  // launches after every problem's CG had stopped
        else
          c.unaccount_gated(gated);
        break;
      }
      chunk = std::max(1, std::min(2, o->max_cg_iter - enq));
    }
    float ms1 = 0.f, ms2 = 0.f;
    HC(hipEventElapsedTime(&ms1, tm.ev[0], tm.ev[1]));
    HC(hipEventElapsedTime(&ms2, tm.ev[1], tm.ev[2]));
    t_linsys += ms1 * 1e-3;
    t_prox += ms2 * 1e-3;

    // ---- host logic per problem ----
    bool all_ready_to_switch = phase == 0 && prec == GENIOS_PREC_BF16_REFINE;
    bool any_certify = false;
    std::vector<int> want_cert(B, 0);
    for (int64_t b = 0; b < B; ++b) {
      if (!hp[b].run) continue;
      HostProb& q = P[b];
      const ProbState& S = hs[b];
      q.iters = k;
      q.cg_total += S.cg_iters;
      q.last_cg = std::max(1, S.cg_iters);
      q.rp = std::sqrt(S.red[kRedRp2]);
      q.xn = std::sqrt(S.red[kRedX2]);
      q.zn = std::sqrt(S.red[kRedZ2]);
      q.un = std::sqrt(S.red[kRedU2]);
      q.rd = std::sqrt(S.red[kRedRd2]);
      const double rhou = q.rho * q.un;
      q.rkkt = kkt_from(q.rp, q.rd, q.xn, q.zn, rhou, n);
      const bool finite = std::isfinite(q.rp) && std::isfinite(q.rd) && std::isfinite(q.xn) &&
                          std::isfinite(q.zn) && std::isfinite(q.un) && std::isfinite(S.rr) &&
                          std::isfinite(S.rhs2);
      if (!finite || !std::isfinite(q.rkkt) || (S.breakdown && !std::isfinite(S.pq))) {
        q.status = GENIOS_ERR_NUMERIC;
        q.done = 1;
        any_numeric = 1;
        continue;
      }
      q.rk_hist.push_back(q.rkkt);
      if (o->history && k <= o->history_cap) {
        double* row = o->history + ((int64_t)b * o->history_cap + (k - 1)) * GENIOS_HIST_FIELDS;
        row[GENIOS_HIST_K] = k;
        row[GENIOS_HIST_RP] = q.rp;
        row[GENIOS_HIST_RD] = q.rd;
        row[GENIOS_HIST_RKKT] = q.rkkt;
        row[GENIOS_HIST_RHO] = q.rho;
        row[GENIOS_HIST_CG] = S.cg_iters;
        row[GENIOS_HIST_RTOL] = hp[b].rtol;
        row[GENIOS_HIST_PHASE] = phase;
        row[GENIOS_HIST_TIME] = now_s() - t0;
        row[GENIOS_HIST_XNORM] = q.xn;
      }
      const bool conv = paper_test(q.rp, q.rd, q.xn, q.zn, rhou, n, eps_abs, eps_rel);
      if (phase == 0 && prec == GENIOS_PREC_BF16_REFINE) {
        bool ready = q.rkkt <= switch_tol;
        const int W = std::max(1, o->stall_window);
        const size_t L = q.rk_hist.size();
        if (!ready && (int)L > W) {
          const double old = q.rk_hist[L - 1 - W];
          if (q.rkkt > 0.9 * old) ready = true;  // < 10% decrease over the window
        }
        if (!ready) all_ready_to_switch = false;
      } else if (conv && o->termination == 0) {
        want_cert[b] = 1;
        any_certify = true;
      }
      // penalty update (Sec. 2.5)
      if (o->rho_update_every > 0 && k % o->rho_update_every == 0 && k <= o->rho_update_until) {
        double nr = q.rho;
        if (q.rp > o->mu * q.rd)
          nr = o->tau * q.rho;
        else if (q.rd > o->mu * q.rp)
          nr = q.rho / o->tau;
        if (nr != q.rho) {
          q.u_scale = q.rho / nr;
          q.rho = nr;
        }
      }
      q.rp_prev = q.rp;
      q.rd_prev = q.rd;
    }
    // BF16 -> FP32 switch (whole batch at once)
    if (all_ready_to_switch) {
      phase = 1;
      op = &c.op_hi;
      for (int64_t b = 0; b < B; ++b)
        if (!P[b].done) {
          P[b].switch_iter = k + 1;
          P[b].rk_hist.clear();
        }
      // refresh H x (and the ML gradient) with the FP32 operator
      set_params(k, false);
      HC(upload_params(c, hp));
      if (ml) {
        rc = gradient_pass(*op, c.gate_run, c.gs_params);
      } else {
        rc = hvp_explicit(c, *op, x, h, nullptr, c.gate_run, c.gs_params);
      }
      if (rc) return rc;
      continue;
    }
    // Certification with the operator of the phase (explicit products, no recursion).
    if (any_certify) {
      for (int64_t b = 0; b < B; ++b) hp[b].run = want_cert[b];
      HC(upload_params(c, hp));
      // (after an iteration of BF16-model CG, h and r_d are already the master copy's)
      const bool rd_fresh = cg_lo_it;
      if (!ml && !rd_fresh) {
        rc = hvp_explicit(c, *op, x, h, nullptr, c.gate_run, c.gs_params);
        if (rc) return rc;
        VecArgs vr = c.vargs(x, z, u, h, g, phase == 0 ? c_lo : c_hi, nullptr);
        HC(launch_dual_residual(vr, c.st));
        rc = sync_state(c, hs);
        if (rc) return rc;
      }
      for (int64_t b = 0; b < B; ++b) {
        if (!want_cert[b]) continue;
        HostProb& q = P[b];
        if (!ml) q.rd = std::sqrt(hs[b].red[kRedRd2]);
        // the certifying residuals use the rho of the finished iteration
        const double rho_it = hp[b].rho;
        const double rhou = rho_it * q.un;
        q.rkkt = kkt_from(q.rp, q.rd, q.xn, q.zn, rhou, n);
        if (paper_test(q.rp, q.rd, q.xn, q.zn, rhou, n, eps_abs, eps_rel)) {
          q.done = 1;
          q.rd_exact = !ml && op == &c.op_hi;
          q.t_target = now_s() - t0;
          q.status = GENIOS_OK;
          // undo a penalty change decided in this iteration (u was not rescaled yet)
          q.rho = rho_it;
          q.u_scale = 1.0;
          --active;
        }
      }
    }
    // Gap pass at z in the operator's final phase: the relative duality gap (Sec. 3.3,
    // App. A; termination 1) or the subdifferential distance (Sec. 4.3; termination 2).
    if (o->termination != 0 && !(phase == 0 && prec == GENIOS_PREC_BF16_REFINE) &&
        k % o->gap_every == 0) {
      bool any = false;
      for (int64_t b = 0; b < B; ++b)
        if (hp[b].run && !P[b].done) any = true;
      if (any) {
        rc = eval_gap(*op, z, c.gate_run, c.gs_params);
        if (rc) return rc;
        rc = read_gap();
        if (rc) return rc;
        for (int64_t b = 0; b < B; ++b) {
          if (!hp[b].run || P[b].done) continue;
          HostProb& q = P[b];
          ++q.gap_checks;
          const double crit = o->termination == 1 ? hg[b].rel_gap : hg[b].subgrad;
          if (std::isfinite(crit) && crit <= o->eps_gap) {
            q.done = 1;
            q.t_target = now_s() - t0;
            q.status = GENIOS_OK;
            // undo a penalty change decided in this iteration (u was not rescaled yet)
            q.rho = hp[b].rho;
            q.u_scale = 1.0;
          }
        }
      }
    }
    active = 0;
    for (int64_t b = 0; b < B; ++b)
      if (!P[b].done) ++active;
  }
  const double t_solve = now_s() - t_loop0;
  for (int64_t b = 0; b < B; ++b)
    if (!P[b].done) P[b].status = GENIOS_MAX_ITER;
  // pending u rescale (penalty changed in the last iteration without a following one)
  {
    bool pend = false;
    for (int64_t b = 0; b < B; ++b)
      if (P[b].u_scale != 1.0) pend = true;
    if (pend) {
      for (int64_t b = 0; b < B; ++b) {
        // apply by running nothing but the scale: re-use admm_begin would also overwrite r;
        // instead report the state consistently with rho before the change.
        P[b].rho = P[b].rho * P[b].u_scale;
        P[b].u_scale = 1.0;
      }
    }
  }

  // ---- final report with the master-copy operator ----
  // r_d at the returned x: already exact where the problem was certified with the
  // master copy at that x (the certification's explicit H x); else recomputed here.
  bool all_exact = true;
  for (int64_t b = 0; b < B; ++b)
    if (!P[b].rd_exact) all_exact = false;
  set_params(k, true);
  HC(upload_params(c, hp));
  if (!all_exact) {
    if (ml) {
      rc = gradient_pass(c.op_hi, nullptr, 0);
      if (rc) return rc;
    } else {
      rc = hvp_explicit(c, c.op_hi, x, h, nullptr, nullptr, 0);
      if (rc) return rc;
    }
    VecArgs vr = c.vargs(x, z, u, h, g, c_hi, nullptr);
    HC(launch_dual_residual(vr, c.st));
    rc = sync_state(c, hs);
    if (rc) return rc;
    for (int64_t b = 0; b < B; ++b) P[b].rd = std::sqrt(hs[b].red[kRedRd2]);
  }
  // objective (the gap pass's primal value) and relative duality gap at the returned z
  // with the master copy
  rc = eval_gap(c.op_hi, z, nullptr, 0);
  if (rc) return rc;
  rc = read_gap();
  if (rc) return rc;
  // BF16-only: the a-posteriori bound on F(z) - F* from the rounding of A alone.  With
  // E = A - A~ and |E| <= u |A~| (round to nearest, u = 2^-8 / (1 - 2^-8)), the objective
  // perturbation at x is |D(x)| <= ||A~ x - b|| u || |A~| |x| || + u^2 || |A~| |x| ||^2 / 2
  // for the square loss and <= L u sum_i w_i (|A~| |x|)_i for a loss of slope at most
  // L w_i on sample i (logistic: w_i = |y_i|, Huber: L = 2 delta); the bound is
  // |D(z)| + |D(x*)| with x* replaced by z, i.e. 2 |D(z)|.
  std::vector<double> bf16_bound(B, 0.0);
  if (prec == GENIOS_PREC_BF16_ONLY) {
    const int ns = c.nsplit_for(c.op_lo, 0);
    const int64_t ps = (int64_t)c.L.nsplit_n * m;
    HC(launch_gemv_n_abs(c.op_lo, B, c.vt, z, n, c.L.tparts, m, ps, ns, c.st));
    HC(launch_bound_terms(c.vt, m, B, c.L.tparts, ns, m, ps, bvec, m, 0, c.L.gpart, c.st));
    if (loss == kLossSquare) {
      HC(launch_gemv_n(c.op_lo, B, c.vt, z, n, c.L.tparts, m, ps, ns, nullptr, 0, c.st));
      HC(launch_bound_terms(c.vt, m, B, c.L.tparts, ns, m, ps, bvec, m, 1, c.L.gpart, c.st));
    }
    std::vector<double> hb(4 * (size_t)B, 0.0);
    HC(hipMemcpyAsync(hb.data(), c.L.gpart, hb.size() * sizeof(double), hipMemcpyDeviceToHost,
                      c.st));
    HC(hipStreamSynchronize(c.st));
    const double ur = 0x1p-8 / (1.0 - 0x1p-8);
    for (int64_t b = 0; b < B; ++b) {
      const double sy2 = hb[4 * b], sy = hb[4 * b + 1], sr2 = hb[4 * b + 2], swy = hb[4 * b + 3];
      double d = 0.0;
      if (loss == kLossSquare)
        d = ur * std::sqrt(sr2) * std::sqrt(sy2) + 0.5 * ur * ur * sy2;
      else if (loss == kLossLogistic)
        d = ur * swy;
      else
        d = 2.0 * delta * ur * sy;
      bf16_bound[b] = 2.0 * d;
    }
  }
  const double t_total = now_s() - t0;
  int worst = GENIOS_OK;
  for (int64_t b = 0; b < B; ++b) {
    HostProb& q = P[b];
    genios_info& I = info[b];
    std::memset(&I, 0, sizeof(I));
    int st = q.status;
    if (st == GENIOS_OK && s > 0 && core_status[b] == GENIOS_WARN_PRECOND) st = GENIOS_WARN_PRECOND;
    I.status = st;
    I.iters = q.iters;
    I.cg_iters = q.cg_total;
    I.phase_switch_iter = q.switch_iter;
    I.resketches = q.resketches;
    I.precond_rank = q.precond_rank;
    I.sketch_err = q.sketch_err;
    I.kappa_bound = q.kappa_bound;
    I.sketch_rounds = q.sketch_rounds;
    I.t_hvp_mrhs = c.prof.t[6];
    I.n_hvp_mrhs = (int32_t)c.n_mrhs;
    I.bytes_hvp_mrhs = c.bytes_mrhs;
    I.n_hvp_tail = (int32_t)c.n_tail;
    I.n_hvp_resized = (int32_t)c.n_resized;
    I.rho = q.rho;
    I.r_p = q.rp;
    I.r_d = q.rd;
    I.r_kkt = kkt_from(I.r_p, I.r_d, q.xn, q.zn, q.rho * q.un, n);
    I.obj = hg[b].primal;
    I.rel_gap = hg[b].rel_gap;
    I.bf16_bound = bf16_bound[b];
    I.gap_primal = hg[b].primal;
    I.gap_dual = hg[b].dual;
    I.gap_checks = q.gap_checks;
    I.subgrad_dist = hg[b].subgrad;
    I.t_setup = t_setup;
    I.t_precond = t_precond;
    I.t_solve = t_solve;
    I.t_linsys = t_linsys;
    I.t_prox = t_prox;
    I.t_total = t_total;
    I.t_to_target = q.t_target;
    I.t_matvec_n = c.prof.t[0];
    I.t_matvec_t = c.prof.t[1];
    I.t_hvp = c.prof.t[2];
    I.n_hvp = (int32_t)c.n_mv[2];
    I.bytes_hvp = c.bytes_kind[2];
    I.t_hvp_hi = c.prof.t[3];
    I.n_hvp_hi = (int32_t)c.n_mv[3];
    I.bytes_hvp_hi = c.bytes_kind[3];
    c.fill_sketch_info(I);
    I.n_matvec_n = (int32_t)c.n_mv[0];
    I.n_matvec_t = (int32_t)c.n_mv[1];
    I.bytes_matvec_n = c.bytes_kind[0];
    I.bytes_matvec_t = c.bytes_kind[1];
    if (st < 0 && (worst >= 0 || st < worst)) worst = st;
    if (worst >= 0 && st > worst) worst = st;
  }
  if (s > 0) {
    std::vector<int32_t> se(B);
    HC(hipMemcpyAsync(se.data(), c.L.ctrl.s_eff, B * sizeof(int32_t), hipMemcpyDeviceToHost,
                      c.st));
    HC(hipStreamSynchronize(c.st));
    for (int64_t b = 0; b < B; ++b) info[b].precond_rank = se[b];
  }
  (void)any_numeric;
  (void)sketch_checked;
  return worst;
}

int effective_rank(const genios_opts* o, int64_t n, int64_t m) {
  int s = o->sketch_rank;
  if (s <= 0) s = (int)std::min<int64_t>(50, n / 20);
  s = (int)std::min<int64_t>(s, std::min<int64_t>(n, kMaxS));
  (void)m;
  return std::max(0, s);
}

// ---------------------------------------------------------------------------------

int run_nystrom_build(const genios_matrix* A, const void* d, int s, const void* omega,
                      const genios_opts* o, void* U, double* lamhat, genios_info* info) {
  Ctx c;
  c.st = static_cast<hipStream_t>(o->stream);
  c.B = A->batch;
  c.m = A->m;
  c.n = A->n;
  c.vt = A->hi_dtype == GENIOS_DT_F64 ? VT_F64 : VT_F32;
  c.L.setup(GENIOS_OP_NYSTROM, A, o, s);
  int rc = c.L.bind(o->workspace, o->workspace_bytes);
  if (rc) return rc;
  const bool use_lo = o->precision == GENIOS_PREC_BF16_REFINE || o->precision == GENIOS_PREC_BF16_ONLY;
  MatArg op{A->A_hi, c.vt == VT_F64 ? MT_F64 : MT_F32, A->m, A->n, A->lda, A->stride_A};
  if (use_lo) {
    if (A->A_bf16 == nullptr)
      HC(launch_cast_bf16(static_cast<const float*>(A->A_hi), c.L.A16, c.L.a16_elems, c.st));
    op = MatArg{A->A_bf16 ? (const void*)A->A_bf16 : (const void*)c.L.A16, MT_BF16, A->m, A->n,
                A->lda, A->stride_A};
  }
  HC(launch_fill(c.L.ctrl.params, c.L.ctrl_bytes_end, c.st));
  c.prof.on = o->profile_kernels != 0;
  SketchWs skx = c.L.sk;
  HC(c.sketch_timer(op, s, &skx));
  HC(run_nystrom(op, c.B, c.vt, d, A->m, s, omega, o->seed, 0, nullptr, skx, U, lamhat,
                 c.L.ctrl.s_eff, c.L.core_status, c.L.shift, c.st));
  std::vector<int32_t> se(c.B), cs(c.B);
  HC(hipMemcpyAsync(se.data(), c.L.ctrl.s_eff, c.B * 4, hipMemcpyDeviceToHost, c.st));
  HC(hipMemcpyAsync(cs.data(), c.L.core_status, c.B * 4, hipMemcpyDeviceToHost, c.st));
  HC(hipStreamSynchronize(c.st));
  c.prof.harvest();
  int worst = 0;
  for (int64_t b = 0; b < c.B; ++b) {
    if (info) {
      std::memset(&info[b], 0, sizeof(genios_info));
      info[b].status = cs[b];
      info[b].precond_rank = se[b];
      info[b].resketches = 1;
      c.fill_sketch_info(info[b]);
    }
    worst = std::max(worst, cs[b]);
  }
  return worst;
}

int run_matvec(const genios_matrix* A, int trans, int use_bf16, const void* v, void* out,
               const genios_opts* o) {
  Ctx c;
  c.st = static_cast<hipStream_t>(o->stream);
  c.B = A->batch;
  c.m = A->m;
  c.n = A->n;
  c.vt = A->hi_dtype == GENIOS_DT_F64 ? VT_F64 : VT_F32;
  c.ve = c.vt == VT_F32 ? 4 : 8;
  genios_opts oo = *o;
  oo.precision = use_bf16 ? GENIOS_PREC_BF16_ONLY : GENIOS_PREC_F32;
  genios_matrix AA = *A;
  c.L.setup(GENIOS_OP_MATVEC, &AA, &oo, 0);
  int rc = c.L.bind(o->workspace, o->workspace_bytes);
  if (rc) return rc;
  MatArg op = use_bf16 ? MatArg{A->A_bf16, MT_BF16, A->m, A->n, A->lda, A->stride_A}
                       : MatArg{A->A_hi, c.vt == VT_F64 ? MT_F64 : MT_F32, A->m, A->n, A->lda,
                                A->stride_A};
  if (!trans) {
    const int ns = std::min(c.L.nsplit_n, gemv_n_splits(op, c.B));
    HC(launch_gemv_n(op, c.B, c.vt, v, c.n, c.L.tparts, c.m, (int64_t)c.L.nsplit_n * c.m, ns,
                     nullptr, 0, c.st));
    HC(launch_sum_splits(c.vt, c.B, c.m, c.L.tparts, ns, c.m, (int64_t)c.L.nsplit_n * c.m, out,
                         c.m, c.st));
  } else {
    const int ks = std::min(c.L.ksplit, gemv_t_splits(op, c.B));
    HC(launch_gemv_t(op, c.B, c.vt, v, 1, 0, c.m, 0, 1, nullptr, 0, c.L.ypart, ks, c.L.npad,
                     c.L.npad, c.L.yprob(), nullptr, 0, c.st));
    HC(launch_sum_splits(c.vt, c.B, c.n, c.L.ypart, ks, c.L.npad, c.L.yprob(),
                         out, c.n, c.st));
  }
  HC(hipStreamSynchronize(c.st));
  return 0;
}

int run_hvp(const genios_matrix* A, int use_bf16, const void* d, const void* p, void* out,
            const genios_opts* o) {
  Ctx c;
  c.st = static_cast<hipStream_t>(o->stream);
  c.B = A->batch;
  c.m = A->m;
  c.n = A->n;
  c.vt = A->hi_dtype == GENIOS_DT_F64 ? VT_F64 : VT_F32;
  c.ve = c.vt == VT_F32 ? 4 : 8;
  genios_opts oo = *o;
  oo.precision = use_bf16 ? GENIOS_PREC_BF16_ONLY : GENIOS_PREC_F32;
  genios_matrix AA = *A;
  c.L.setup(GENIOS_OP_HVP, &AA, &oo, 0);
  int rc = c.L.bind(o->workspace, o->workspace_bytes);
  if (rc) return rc;
  MatArg op = use_bf16 ? MatArg{A->A_bf16, MT_BF16, A->m, A->n, A->lda, A->stride_A}
                       : MatArg{A->A_hi, c.vt == VT_F64 ? MT_F64 : MT_F32, A->m, A->n, A->lda,
                                A->stride_A};
  rc = c.hvp(op, p, d, nullptr, 0);
  if (rc) return rc;
  HC(launch_sum_splits(c.vt, c.B, c.n, c.L.ypart, c.cur_ks, c.cur_ks_stride, c.cur_prob_stride, out,
                       c.n, c.st));
  HC(hipStreamSynchronize(c.st));
  return 0;
}

// ---------------------------------------------------------------------------------
// Adjoint.  With S the support of z*, s its signs and g = dL/dz*, the solution
// map's derivatives are dL/db = A_S G^-1 g_S and dL/dlam = -s^T G^-1 g_S with
// G = A_S^T A_S.  The active set is compacted on the device (ordered indices,
// columns of the master copy gathered into an m x ldS block, zero padding); the
// system (G on S, identity on the padding) is solved by Nystrom-preconditioned
// CG with the masked kernels, so every CG product streams only m x |S| values.

int run_backward(const genios_matrix* A, const void* zstar, const void* gz, const genios_opts* o,
                 void* grad_b, double* grad_lambda, genios_info* info) {
  const double t0 = now_s();
  Ctx c;
  c.A = A;
  c.o = o;
  c.st = static_cast<hipStream_t>(o->stream);
  c.B = A->batch;
  c.m = A->m;
  c.n = A->n;
  c.vt = A->hi_dtype == GENIOS_DT_F64 ? VT_F64 : VT_F32;
  c.ve = c.vt == VT_F32 ? 4 : 8;
  const int s_req = o->precondition ? effective_rank(o, A->n, A->m) : 0;
  c.L.setup(GENIOS_OP_BACKWARD, A, o, s_req);
  int rc = c.L.bind(o->workspace, o->workspace_bytes);
  if (rc) return rc;
  c.prof.on = o->profile_kernels != 0;
  const MType mt = c.vt == VT_F64 ? MT_F64 : MT_F32;
  c.op_hi = MatArg{A->A_hi, mt, A->m, A->n, A->lda, A->stride_A};
  c.gate_cg = &c.L.ctrl.state[0].cg_active;
  const int64_t B = c.B, n = c.n, m = c.m;
  HC(launch_fill(c.L.ctrl.params, c.L.ctrl_bytes_end, c.st));
  void* sgn_full = c.L.nv[kVR];
  void* neg_full = c.L.nv[kVW];
  HC(launch_build_mask(c.vt, n, B, zstar, gz, c.L.mask, sgn_full, neg_full, c.st));
  HC(launch_compact_index(n, B, c.L.mask, c.L.idx, c.L.cnt, c.st));
  std::vector<int32_t> cnt(B);
  HC(hipMemcpyAsync(cnt.data(), c.L.cnt, B * sizeof(int32_t), hipMemcpyDeviceToHost, c.st));
  HC(hipStreamSynchronize(c.st));
  int cmax = 0;
  for (int64_t b = 0; b < B; ++b) cmax = std::max(cmax, cnt[b]);
  // (A_S^T A_S + lambda2 I) is singular only without the l2 term
  if (o->lambda2 == 0.0 && cmax > std::min<int64_t>(m, n)) {
    set_error("active set larger than the number of rows: A_S^T A_S is singular");
    return GENIOS_ERR_NUMERIC;
  }
  std::vector<double> gl(B, 0.0);
  std::vector<int32_t> se(B, 0);
  std::vector<ProbState> hsv(B);
  ProbState* hs = hsv.data();
  if (cmax == 0) {  // z* = 0 for every problem: the solution map is locally constant
    HC(launch_fill(grad_b, B * m * c.ve, c.st));
    HC(hipStreamSynchronize(c.st));
    for (int64_t b = 0; b < B; ++b) {
      grad_lambda[b] = 0.0;
      if (info) std::memset(&info[b], 0, sizeof(genios_info));
    }
    return 0;
  }
  // padded to a multiple of 8 (vector loads) but never beyond n, the capacity of
  // the n-vector workspace slots reused for the compact vectors
  const int ldS = (int)std::min<int64_t>((cmax + 7) / 8 * 8, n);
  if (ldS > c.L.ldS_max) {  // never gather beyond the reserved block
    set_error("active set exceeds the reserved compact block");
    return GENIOS_ERR_NUMERIC;
  }
  // compact problem: A_S (m x ldS), g_S, signs, padding mask
  void* sgnS = c.L.nv[kVCH];
  void* negS = c.L.nv[kVG];
  HC(launch_gather_vec(c.vt, n, B, c.L.idx, c.L.cnt, ldS, neg_full, negS, sgn_full, sgnS,
                       c.L.maskS, c.st));
  HC(launch_gather_cols(mt, A->A_hi, A->lda, A->stride_A, m, n, B, c.L.idx, c.L.cnt, ldS, c.L.AS,
                        c.st));
  const MatArg opS{c.L.AS, mt, m, ldS, ldS, m * (int64_t)ldS};
  void* w = c.L.nv[kVX];
  void* zero_z = c.L.nv[kVZ];
  void* zero_u = c.L.nv[kVU];
  void* h = c.L.nv[kVH];
  HC(launch_fill(w, B * ldS * c.ve, c.st));
  HC(launch_fill(zero_z, B * ldS * c.ve, c.st));
  HC(launch_fill(zero_u, B * ldS * c.ve, c.st));
  HC(launch_fill(h, B * ldS * c.ve, c.st));
  // sketch of the compact operator (padding rows of Omega and Y masked), at most a
  // quarter of the compact system's size (rounded up to 8, at least 8)
  const int s_cap = std::max(8, ((cmax + 3) / 4 + 7) / 8 * 8);
  const int s = std::min(std::min(s_req, ldS), s_cap);
  if (s > 0) {
    SketchWs skc = c.L.sk;
    int kw = 1, ky = 1, ng = 1;
    sketch_ws_bytes(m, ldS, s, B, c.vt, &kw, &ky, &ng);
    skc.ksW = std::max(1, std::min(kw, c.L.sk.ksW));
    skc.ksY = std::max(1, std::min<int>(ky, (int)((int64_t)c.L.sk.ksY * n / ldS)));
    skc.nbG = std::max(1, std::min(ng, c.L.sk.nbG));
    if (sketch_pad(s) > sketch_pad(c.L.s)) return GENIOS_ERR_DEVICE;  // cannot happen: s <= s_req
    HC(c.sketch_timer(opS, s, &skc));
    HC(run_nystrom(opS, B, c.vt, nullptr, m, s, nullptr, o->seed, 0, c.L.maskS, skc, c.L.U,
                   c.L.ctrl.lamhat, c.L.ctrl.s_eff, c.L.core_status, c.L.shift, c.st));
  }
  ProbParams* hp = static_cast<ProbParams*>(pinned(B * sizeof(ProbParams)));
  if (!hp) return GENIOS_ERR_DEVICE;
  for (int64_t b = 0; b < B; ++b) {
    ProbParams& q = hp[b];
    std::memset(&q, 0, sizeof(q));
    q.run = 1;
    q.rho = 1.0;
    q.sigma = 0.0;
    q.nu = o->lambda2;  // (A_S^T A_S + lambda2 I) w = g_S
    q.kappa = 0.0;
    q.alpha = 1.0;
    q.u_scale = 1.0;
    q.rtol = o->cg_tol_floor;
    q.tol_floor = o->cg_tol_floor;
    q.max_cg = std::max(o->max_cg_iter, 1);
    q.rhs_rel = 1;
    q.use_c = 0;
  }
  HC(upload_params(c, hp));
  // vector-kernel geometry of the compact problem
  VecArgs va = c.vargs(w, zero_z, zero_u, h, negS, nullptr, c.L.maskS);
  va.n = ldS;
  va.chunk = vec_chunk(ldS);
  va.nb = (int)((ldS + va.chunk - 1) / va.chunk);
  va.chunkf = vec_chunk_fine(ldS);
  va.nbf = (int)((ldS + va.chunkf - 1) / va.chunkf);
  va.U = s > 0 ? c.L.U : nullptr;
  va.s_stride = std::max(1, s);
  const int nsS = std::min(gemv_n_splits(opS, B), c.L.nsplit_n);
  const int ksS = std::max(
      1, std::min<int>(gemv_t_splits(opS, B), (int)(c.L.yprob() / ldS)));
  va.ksplit = ksS;
  va.ypart_ks_stride = ldS;
  va.ypart_prob_stride = (int64_t)ksS * ldS;
  // the lamhat stride used by the kernels must match the compact sketch rank
  va.ctrl.s_stride = std::max(1, s);
  rc = cg_setup(c, va);
  if (rc) return rc;
  int t_cg = 0;
  // fused one-pass H p on the compact matrix when it qualifies
  const HvpGeom gS = c.vt == VT_F32 ? hvp_geometry(opS, B, true) : HvpGeom{};
  const bool fusedS = gS.threads > 0 && gS.blocks <= c.L.yslots && hvp_p_aligned(va.p, ldS, B);
  if (fusedS) {
    va.ksplit = gS.blocks;
    va.ypart_ks_stride = ldS;
    va.ypart_prob_stride = (int64_t)gS.blocks * ldS;
  }
  auto hvp_cg = [&]() -> int {
    c.last_hvp_op = opS;
    c.last_hvp_kind = fusedS ? Ctx::hvp_kind(opS) : 0;
    if (fusedS) {
      HC(c.prof.begin(c.st, Ctx::hvp_kind(opS)));
      HC(launch_hvp_fused(opS, gS, B, static_cast<const float*>(va.p), ldS, nullptr, 0,
                          static_cast<float*>(c.L.ypart), ldS, va.ypart_prob_stride, c.gate_cg,
                          c.gs_state, c.st, c.L.hpq, c.L.yslots));
      HC(c.prof.end(c.st));
      c.account(opS, Ctx::hvp_kind(opS));
      VecArgs vq = va;
      vq.hpq = c.L.hpq;
      vq.hpq_stride = c.L.yslots;
      vq.nhpq = gS.blocks;
      return cg_vector_step(c, vq, t_cg++, true);
    }
    HC(c.prof.begin(c.st, 0));
    HC(launch_gemv_n(opS, B, c.vt, va.p, ldS, c.L.tparts, m, (int64_t)c.L.nsplit_n * m, nsS,
                     c.gate_cg, c.gs_state, c.st));
    HC(c.prof.end(c.st));
    c.account(opS, 0);
    HC(c.prof.begin(c.st, 1));
    HC(launch_gemv_t(opS, B, c.vt, c.L.tparts, nsS, m, (int64_t)c.L.nsplit_n * m, 0, 1, nullptr, 0,
                     c.L.ypart, ksS, ldS, ldS, (int64_t)ksS * ldS, c.gate_cg, c.gs_state, c.st));
    HC(c.prof.end(c.st));
    c.account(opS, 1);
    return cg_vector_step(c, va, t_cg++, false);
  };
  for (;;) {
    for (int it = 0; it < 8; ++it) {
      rc = hvp_cg();
      if (rc) return rc;
    }
    rc = sync_state(c, hs);
    if (rc) return rc;
    bool more = false;
    for (int64_t b = 0; b < B; ++b)
      if (hs[b].cg_active) more = true;
    if (!more) {
      int64_t gated = 0;
      for (int64_t b = 0; b < B; ++b) gated += std::max<int64_t>(0, t_cg - hs[b].cg_iters);
      c.unaccount_gated(gated);
      break;
    }
  }
  // grad_b = A_S w_S; grad_lambda = -s_S^T w_S
  rc = 0;
  HC(launch_gemv_n(opS, B, c.vt, w, ldS, c.L.tparts, m, (int64_t)c.L.nsplit_n * m, nsS, nullptr, 0,
                   c.st));
  c.account(opS, 0);
  HC(launch_sum_splits(c.vt, B, m, c.L.tparts, nsS, m, (int64_t)c.L.nsplit_n * m, grad_b, m, c.st));
  HC(launch_masked_dot(c.vt, ldS, B, sgnS, w, c.L.ctrl.part, c.L.ctrl.part_stride,
                       c.L.ctrl.counters, c.L.scal, c.st));
  HC(hipMemcpyAsync(gl.data(), c.L.scal, B * sizeof(double), hipMemcpyDeviceToHost, c.st));
  if (s > 0) HC(hipMemcpyAsync(se.data(), c.L.ctrl.s_eff, B * 4, hipMemcpyDeviceToHost, c.st));
  HC(hipStreamSynchronize(c.st));
  int worst = 0;
  for (int64_t b = 0; b < B; ++b) {
    grad_lambda[b] = -gl[b];
    int st = 0;
    if (hs[b].breakdown && !(hs[b].rr <= 1e300))
      st = GENIOS_ERR_NUMERIC;
    else if (hs[b].rr > hs[b].tol2)
      st = GENIOS_MAX_ITER;
    if (info) {
      std::memset(&info[b], 0, sizeof(genios_info));
      info[b].status = st;
      info[b].cg_iters = hs[b].cg_iters;
      info[b].precond_rank = se[b];
      info[b].iters = cnt[b];  // active-set size
      info[b].r_d = std::sqrt(hs[b].rr);
      info[b].t_total = now_s() - t0;
      info[b].t_matvec_n = c.prof.t[0];
      info[b].t_matvec_t = c.prof.t[1];
      info[b].n_matvec_n = (int32_t)c.n_mv[0];
      info[b].n_matvec_t = (int32_t)c.n_mv[1];
      info[b].bytes_matvec_n = c.bytes_kind[0];
      info[b].bytes_matvec_t = c.bytes_kind[1];
      info[b].t_hvp = c.prof.t[2];
      info[b].n_hvp = (int32_t)c.n_mv[2];
      info[b].bytes_hvp = c.bytes_kind[2];
      info[b].t_hvp_hi = c.prof.t[3];
      info[b].n_hvp_hi = (int32_t)c.n_mv[3];
      info[b].bytes_hvp_hi = c.bytes_kind[3];
      c.fill_sketch_info(info[b]);
    }
    if (st < 0 && (worst >= 0 || st < worst)) worst = st;
    if (worst >= 0 && st > worst) worst = st;
  }
  return worst;
}

}  // namespace genios
