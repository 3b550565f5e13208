// Host engine interface: workspace layout and the drivers behind the C ABI.
#pragma once

#include <stddef.h>
#include <stdint.h>

#include "genios.h"
#include "internal.hpp"

namespace genios {

// Internal n-vector slots of the workspace.
enum {
  kVH = 0,   // h = H x (tracked through CG)
  kVG,       // gradient of the smooth part (logistic, Huber) / -rhs (adjoint)
  kVCH,      // c = A^T b with the master copy (adjoint: signs of z*)
  kVCL,      // c = A^T b with the BF16 copy
  kVR,       // CG residual
  kVP,       // CG direction
  kVHP,      // H p
  kVW,       // preconditioned residual
  kVX,       // adjoint solution
  kVZ,       // adjoint zero vector
  kVU,       // adjoint zero vector
  kNumNVec
};

struct Arena;

struct Layout {
  int op = 0;
  int64_t m = 0, n = 0, batch = 1;
  VType vt = VT_F32;
  bool ml = false, backward = false;  // ml: the logistic or Huber loss (Sec. 3.3)
  int s = 0;
  bool need_a16 = false;
  int64_t a16_elems = 0;
  int nsplit_n = 1, nrhs = 1, ksplit = 1;
  int64_t npad = 0, chunk = 256;
  int64_t yslots = 1;  // n-vector partial slots per problem in `ypart`
  int64_t yprob() const { return yslots * npad; }
  int nb = 1, part_blocks = 1, n_vecs = 0;
  SketchWs sk{};
  Ctrl ctrl{};
  size_t ctrl_bytes_end = 0;
  int32_t* core_status = nullptr;
  double* shift = nullptr;
  double* scal = nullptr;
  uint16_t* A16 = nullptr;
  void* nv[kNumNVec] = {};
  void* tparts = nullptr;
  void* ypart = nullptr;
  double* hpq = nullptr;  // [batch][yslots] per-block p^T H p partials of the fused product
  void* dvec = nullptr;
  void* cols = nullptr;
  uint8_t* mask = nullptr;
  void* U = nullptr;
  // adjoint: active-set compaction
  int ldS_max = 0;          // columns reserved for the compacted A_S (multiple of 8)
  int32_t* idx = nullptr;   // [batch][n] ordered active indices
  int32_t* cnt = nullptr;   // [batch] active-set sizes
  void* AS = nullptr;       // [batch][m][ldS] gathered columns of the master copy
  uint8_t* maskS = nullptr; // [batch][ldS] 1 for real columns, 0 for padding
  // relative duality gap (solves)
  bool gap = false;
  void* gapf = nullptr;       // [batch][m] f'(t)
  void* gaps = nullptr;       // [batch][m] r or sigmoid(w)
  double* gpart = nullptr;    // [batch][kGapSlots][kGapPStride]
  GapState* gstate = nullptr; // [batch]
  double* pm_est = nullptr;   // [batch] power-method estimate of ||H - H_hat|| (adaptive sketch)
  MrhsWs mr{};                // H p of a batch sharing A on the matrix cores (sp = 0: off)
  size_t total = 0;

  int setup(int op, const genios_matrix* A, const genios_opts* o, int s);
  int bind(void* base, size_t bytes);
  void carve(Arena& ar);
};

int effective_rank(const genios_opts* o, int64_t n, int64_t m);
// z-step of the solve: soft-threshold (l1) or projection onto [lo, hi] (device
// n-vectors per problem, nullable for an unbounded side).
struct ProxSpec {
  int kind = kProxL1;
  const void* lo = nullptr;
  const void* hi = nullptr;
};
int run_admm(const genios_matrix* A, const void* bvec, const double* lambda, double rho0,
             const genios_opts* o, void* x, void* z, void* u, genios_info* info, int loss,
             const ProxSpec& prox = ProxSpec{});
int run_nystrom_build(const genios_matrix* A, const void* d, int s, const void* omega,
                      const genios_opts* o, void* U, double* lamhat, genios_info* info);
int run_matvec(const genios_matrix* A, int trans, int use_bf16, const void* v, void* out,
               const genios_opts* o);
int run_hvp(const genios_matrix* A, int use_bf16, const void* d, const void* p, void* out,
            const genios_opts* o);
int run_backward(const genios_matrix* A, const void* zstar, const void* gz, const genios_opts* o,
                 void* grad_b, double* grad_lambda, genios_info* info);

}  // namespace genios
