// Vector kernels of the inexact ADMM / preconditioned CG loop.
//
// Per ADMM iteration (Sec. 2, M = I, c = 0):
//   admm_begin    u <- u * scale (penalty change, Sec. 2.5); the x-system of
//                 eq. x-update-lin-sys, (H + nu I) x = rhs with
//                 rhs = (H + sigma I) x^k - grad f(x^k) + rho (z^k - u^k),
//                 warm-started at x^k, so r_0 = rho (z - u - x) - grad f(x^k).
//   precond_coef  coefficients c_j of P^-1 = I + U diag(d) U^T (eq. preconditioner),
//                 c = d o (U^T r), and the terms c_j (U^T r)_j of r^T P^-1 r.
//   precond_p     stopping decision for the current residual (CG tolerance of
//                 the schedule, iteration limit), then r^T P^-1 r = ||r||^2 +
//                 sum_j c_j (U^T r)_j, beta, and p = P^-1 r + beta p = r + U c + beta p
//                 in one pass (P^-1 r is never stored).
//   cg_alpha      hp = H p (sum of gemv_t partials), q = hp + nu p.
//   cg_update     alpha = r^T w / p^T q; x += alpha p, h += alpha hp (h tracks
//                 H x), r -= alpha q.
//   admm_end      over-relaxed z- and u-updates with the soft-threshold prox
//                 (Sec. 2.5, Sec. 3.1) and the residual norms of Sec. 2.3.
//   admm_finish   the residual sums into the problem state.
// Reductions accumulate in FP64.  A kernel writes one partial per block; the
// kernel that needs the sum reduces the partials itself, every block in the
// same fixed order (bit-identical in every block), so no block of a grid waits
// on another and no result depends on timing.
#include <algorithm>

#include "device.hpp"

namespace genios {

namespace {

struct Chunk {
  int64_t lo, hi;
};

__device__ __forceinline__ Chunk my_chunk(int64_t n, int64_t chunk) {
  const int64_t lo = (int64_t)blockIdx.x * chunk;
  return Chunk{lo, min(n, lo + chunk)};
}

template <typename VT>
__device__ __forceinline__ VT soft_threshold(VT v, VT k) {
  return v > k ? v - k : (v < -k ? v + k : VT(0));
}

// U^T r partials of this block: r values of the chunk are in LDS (rs).
// Wave w owns columns w, w+4, ...; lane l rows l, l+64, ...  Columns go in
// groups of G whose loads are all issued before the multiply-adds, so a block
// pays the memory latency once per group rather than once per row.  Loads are
// unconditional: rows past the chunk read its last row with weight 0 and
// columns past s_eff re-read column `wave` (their sums are never stored).
template <typename VT, int T = 4>  // T: row loads per lane per column (a 64 T-row slab)
__device__ __forceinline__ void ut_r_partial(const VT* __restrict__ Ub, int64_t ldu, int s_eff,
                                             const Chunk& ch, const VT* rs, double* part_out,
                                             int64_t ostride = 1) {
  constexpr int G = sizeof(VT) == 4 ? 16 : 8;  // columns in flight per lane
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int len = (int)(ch.hi - ch.lo);
  const VT* base = Ub + ch.lo;
  const int ncol = s_eff > wave ? (s_eff - wave + 3) / 4 : 0;
  for (int g0 = 0; g0 < ncol; g0 += G) {
    double acc[G];
#pragma unroll
    for (int jj = 0; jj < G; ++jj) acc[jj] = 0.0;
#pragma unroll 1
    for (int i0 = 0; i0 < len; i0 += 64 * T) {
      double rv[T];
      int ii[T];
#pragma unroll
      for (int t = 0; t < T; ++t) {
        const int i = i0 + lane + 64 * t;
        ii[t] = i < len ? i : len - 1;
        rv[t] = i < len ? double(rs[ii[t]]) : 0.0;
      }
      VT uv[G][T];
#pragma unroll
      for (int jj = 0; jj < G; ++jj) {
        const int j = g0 + jj < ncol ? wave + 4 * (g0 + jj) : wave;
        const VT* col = base + (int64_t)j * ldu;
#pragma unroll
        for (int t = 0; t < T; ++t) uv[jj][t] = col[ii[t]];
      }
#pragma unroll
      for (int jj = 0; jj < G; ++jj)
#pragma unroll
        for (int t = 0; t < T; ++t) acc[jj] += double(uv[jj][t]) * rv[t];
    }
#pragma unroll
    for (int jj = 0; jj < G; ++jj) {
      const double v = wave_sum(acc[jj]);
      if (g0 + jj < ncol && lane == 0) part_out[(int64_t)(wave + 4 * (g0 + jj)) * ostride] = v;
    }
  }
}

// U^T r over 64 rows [lo, lo + 64) of a chunk, in two parts: ut_r64_load issues the
// U values ahead of the step's other work (they do not depend on it) -- thread t takes
// column j = t / 2 (column 0, never summed, past the allocated width) and the 32 rows
// lo + 32 (t % 2) + [0, 32), all 32 loads in flight, rows past `hi` re-reading row
// hi - 1 -- and ut_r64_use weights them by r from LDS (rs[0..63], zero past the
// chunk) into `acc`.  No cross-lane reduction: ut_r64_store combines the two halves.
template <typename VT>
__device__ __forceinline__ void ut_r64_load(const VT* __restrict__ Ub, int64_t ldu, int s_width,
                                            int64_t lo, int64_t hi, VT (&uv)[32]) {
  const int j = threadIdx.x >> 1, half = threadIdx.x & 1;
  const VT* col = Ub + (int64_t)(j < s_width ? j : 0) * ldu;
#pragma unroll
  for (int q = 0; q < 32; ++q) {
    const int64_t i = lo + 32 * half + q;
    uv[q] = col[i < hi ? i : hi - 1];
  }
}
template <typename VT>
__device__ __forceinline__ void ut_r64_use(int s_eff, const VT (&uv)[32], const VT* rs, double& acc) {
  const int j = threadIdx.x >> 1, half = threadIdx.x & 1;
  if (j >= s_eff) return;
#pragma unroll
  for (int q = 0; q < 32; ++q) acc += double(uv[q]) * double(rs[32 * half + q]);
}
// Partial of column j = threadIdx.x / 2: the two halves' sums added in lane order.
__device__ __forceinline__ void ut_r64_store(int s_eff, double acc, double* part_out,
                                             int64_t ostride) {
  const double other = __shfl_xor(acc, 1, 64);
  const int j = threadIdx.x >> 1;
  if ((threadIdx.x & 1) == 0 && j < s_eff) part_out[(int64_t)j * ostride] = acc + other;
}

// Last block: w_j = sum over the nb block partials, then
// coef_j = ((lam_rr + nu)/(lam_j + nu) - 1) w_j.  Wave q sums the q-th quarter
// of the partials for columns lane and lane + 64; the quarters are combined in
// order.  Called by every thread of the block (s_eff is uniform).
__device__ __forceinline__ void finish_coef(const double* part_b, int nb, int s_eff, const double* lamhat_b,
                            double nu, double* coef_b) {
  __shared__ double qs[4 * kMaxS];
  if (s_eff <= 0) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int q = (nb + 3) / 4;
  const int k0 = min(nb, wave * q), k1 = min(nb, k0 + q);
  for (int j = lane; j < s_eff; j += 64) {
    double w = 0.0;
    int k = k0;
    for (; k + 4 <= k1; k += 4) {
      const double a0 = load_partial(part_b + (int64_t)(k + 0) * kPartW + j);
      const double a1 = load_partial(part_b + (int64_t)(k + 1) * kPartW + j);
      const double a2 = load_partial(part_b + (int64_t)(k + 2) * kPartW + j);
      const double a3 = load_partial(part_b + (int64_t)(k + 3) * kPartW + j);
      w += a0;
      w += a1;
      w += a2;
      w += a3;
    }
    for (; k < k1; ++k) w += load_partial(part_b + (int64_t)k * kPartW + j);
    qs[wave * kMaxS + j] = w;
  }
  __syncthreads();
  const double lrr = lamhat_b[s_eff - 1];
  for (int j = threadIdx.x; j < s_eff; j += blockDim.x) {
    const double w = ((qs[j] + qs[kMaxS + j]) + qs[2 * kMaxS + j]) + qs[3 * kMaxS + j];
    coef_b[j] = ((lrr + nu) / (lamhat_b[j] + nu) - 1.0) * w;
  }
}

// v[q] += load(q, k) for k = threadIdx.x, threadIdx.x + blockDim.x, ... < nb, in
// increasing k (the order of a plain strided loop), with four loads per list in
// flight: indices past nb re-read index k0 and are not added.  One memory round
// trip per 4 blockDim.x partials instead of one per blockDim.x.
template <int NV, typename L>
__device__ __forceinline__ void strided_sum4(int nb, const L& load, double (&v)[NV]) {
  const int bd = (int)blockDim.x;
  for (int k0 = threadIdx.x; k0 < nb; k0 += 4 * bd) {
    double e[NV][4];
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int k = k0 + q * bd;
#pragma unroll
      for (int i = 0; i < NV; ++i) e[i][q] = load(i, k < nb ? k : k0);
    }
#pragma unroll
    for (int q = 0; q < 4; ++q)
      if (k0 + q * bd < nb)
#pragma unroll
        for (int i = 0; i < NV; ++i) v[i] += e[i][q];
  }
}

// Fixed-order parallel sum of NV scalar slots over the nb block partials of one
// problem.  Called by every thread of the last block; the result is valid in
// thread 0.
template <int NV>
__device__ void sum_slots(const double* part_b, int nb, int slot0, double (&v)[NV],
                          double* smem) {
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = 0.0;
  for (int k = threadIdx.x; k < nb; k += blockDim.x)
#pragma unroll
    for (int q = 0; q < NV; ++q) v[q] += load_partial(part_b + (int64_t)k * kPartW + kMaxS + slot0 + q);
  block_sum<NV>(v, smem);
}

// Fixed-order sum of NV slot partials over the nb blocks of problem b.  Every
// thread of the calling block gets the result; every block that calls it with
// the same arguments gets the same bits (same loads, same tree).
template <int NV>
__device__ __forceinline__ void reduce_slots(const Ctrl& ctrl, int b, int nb, const int (&slot)[NV],
                                             double (&out)[NV]) {
  __shared__ double sm[4 * NV];
  __shared__ double bc[NV];
  const double* sp = ctrl.spart + (int64_t)b * kNumSlots * ctrl.pstride;
  double v[NV];
#pragma unroll
  for (int q = 0; q < NV; ++q) v[q] = 0.0;
  strided_sum4<NV>(nb, [&](int q, int k) { return sp[(int64_t)slot[q] * ctrl.pstride + k]; }, v);
  block_sum<NV>(v, sm);
  if (threadIdx.x == 0)
#pragma unroll
    for (int q = 0; q < NV; ++q) bc[q] = v[q];
  __syncthreads();
#pragma unroll
  for (int q = 0; q < NV; ++q) out[q] = bc[q];
}

// Block-uniform read of the CG gate: thread 0 reads the flags and the block
// follows its value, so a flag that block 0 of the same kernel clears can never
// split a block between waves that saw it set and waves that saw it cleared.
__device__ __forceinline__ bool block_gate_cg(const ProbParams& P, const ProbState* S) {
  __shared__ int g;
  if (threadIdx.x == 0) g = (P.run && S->cg_active) ? 1 : 0;
  __syncthreads();
  return g != 0;
}

__device__ __forceinline__ double* slot_ptr(const Ctrl& ctrl, int b, int slot) {
  return ctrl.spart + ((int64_t)b * kNumSlots + slot) * ctrl.pstride;
}

// x-system set-up: u <- u * scale, r_0 = rho (z - u - x) - grad f(x^k) and the
// partials of ||rhs||^2, ||r_0||^2 and U^T r_0.  Block 0 re-arms the problem's
// flags (none of them is read by this kernel).
template <typename VT>
__global__ __launch_bounds__(256) void k_admm_begin(VecArgs a) {
  const int b = blockIdx.y;
  const ProbParams P = a.ctrl.params[b];
  ProbState* S = a.ctrl.state + b;
  if (!P.run) {
    // a problem left out of this iteration: its update flag must not open the
    // products gated on a completed update (they would redo its last one)
    if (blockIdx.x == 0 && threadIdx.x == 0) S->admm_done = 0;
    return;
  }
  if (blockIdx.x == 0 && threadIdx.x == 0) {
    S->admm_done = 0;
    S->breakdown = 0;
    S->cg_iters = 0;
    S->cg_active = 1;
  }
  const int64_t n = a.n;
  const Chunk ch = my_chunk(n, a.chunkf);  // the finer grid: 64 rows per step
  const int64_t off = (int64_t)b * n;
  VT* x = static_cast<VT*>(a.x) + off;
  VT* z = static_cast<VT*>(a.z) + off;
  VT* u = static_cast<VT*>(a.u) + off;
  const VT* h = static_cast<const VT*>(a.h) + off;
  const VT* g = P.use_c ? nullptr : static_cast<const VT*>(a.g) + off;
  const VT* c = P.use_c ? static_cast<const VT*>(a.c) + off : nullptr;
  VT* r = static_cast<VT*>(a.r) + off;
  const uint8_t* mask = a.mask ? a.mask + off : nullptr;
  const int s_eff = a.U ? a.ctrl.s_eff[b] : 0;
  const VT* Ub = a.U ? static_cast<const VT*>(a.U) + (int64_t)b * n * a.s_stride : nullptr;
  __shared__ VT rs[64];
  __shared__ double red[16];
  const VT rho = VT(P.rho), sig = VT(P.sigma), usc = VT(P.u_scale), l2 = VT(P.lambda2);
  const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
  double ur = 0.0;  // this thread's share of (U^T r_0)_j, j = threadIdx.x / 2
  double rhs2 = 0.0, rr = 0.0;
  for (int64_t base = ch.lo; base < ch.hi; base += 64) {
    const int64_t i = base + lane;
    const bool ok = i < ch.hi;
    if (grp == 0) {
      VT ri = VT(0);
      if (ok) {
        // all loads before the first store (the vectors are distinct)
        VT ui = u[i];
        const VT xi = x[i], zi = z[i], hi = h[i];
        // grad f(x^k) with the l2 term; (H + sigma I) x^k with H's lambda2 I
        const VT gi = (c ? hi - c[i] : g[i]) + l2 * xi;
        if (P.u_scale != 1.0) {
          ui *= usc;
          u[i] = ui;
        }
        VT rhs = hi + l2 * xi + sig * xi - gi + rho * (zi - ui);
        ri = rho * (zi - ui - xi) - gi;
        if (mask && !mask[i]) {
          rhs = VT(0);
          ri = VT(0);
        }
        r[i] = ri;
        rhs2 += double(rhs) * double(rhs);
        rr += double(ri) * double(ri);
      }
      rs[lane] = ri;  // zero past the chunk
    }
    __syncthreads();
    // (the U rows after r_0: issued first, they held up the first wave's vectors)
    if ((int)(threadIdx.x >> 1) < s_eff) {
      VT uv[32];
      ut_r64_load<VT>(Ub, n, a.s_stride, base, ch.hi, uv);
      ut_r64_use<VT>(s_eff, uv, rs, ur);
    }
    __syncthreads();
  }
  if (s_eff > 0)
    ut_r64_store(s_eff, ur, a.ctrl.upart + (int64_t)b * kMaxS * a.ctrl.pstride + blockIdx.x,
                 a.ctrl.pstride);
  double v[2] = {rhs2, rr};
  block_sum<2>(v, red);
  if (threadIdx.x == 0) {
    slot_ptr(a.ctrl, b, kSlRhs2)[blockIdx.x] = v[0];
    slot_ptr(a.ctrl, b, kSlRr)[blockIdx.x] = v[1];
  }
}

// coef_j = ((lam_rr + nu)/(lam_j + nu) - 1) (U^T r)_j, one block per column j:
// the block sums the column's block partials in a fixed order.
__global__ __launch_bounds__(256) void k_precond_coef(Ctrl ctrl, int nb) {
  const int b = blockIdx.y, j = blockIdx.x;
  const ProbParams P = ctrl.params[b];
  if (!P.run || !ctrl.state[b].cg_active) return;
  const int s_eff = ctrl.s_eff[b];
  if (j >= s_eff) return;
  __shared__ double sm[4];
  const double* up = ctrl.upart + ((int64_t)b * kMaxS + j) * ctrl.pstride;
  double v[1] = {0.0};
  strided_sum4<1>(nb, [&](int, int k) { return up[k]; }, v);
  block_sum<1>(v, sm);
  if (threadIdx.x == 0) {
    const double* lam = ctrl.lamhat + (int64_t)b * ctrl.s_stride;
    const double lrr = lam[s_eff - 1];
    const double cj = ((lrr + P.nu) / (lam[j] + P.nu) - 1.0) * v[0];
    ctrl.coef[(int64_t)b * 2 * kMaxS + j] = cj;
    ctrl.coef[(int64_t)b * 2 * kMaxS + kMaxS + j] = cj * v[0];  // its share of r^T P^-1 r
  }
}

// The stopping decision for the residual it is given -- init: the x-system's set-up
// (tolerance of the CG schedule, empty or non-finite right-hand side); else the
// residual of CG iteration t (tolerance reached or iteration limit) -- then, with
// P^-1 = I + U diag(d) U^T (eq. preconditioner) and c = d o (U^T r) from
// precond_coef, r^T P^-1 r = ||r||^2 + sum_j c_j (U^T r)_j (every block sums the
// same terms in the same order), beta = (r^T P^-1 r) / (the previous one) and
// p = r + U c + beta p (init: beta = 0).  The new r^T P^-1 r goes to the parity
// slot of the next iteration.
template <typename VT>
__global__ __launch_bounds__(256) void k_precond_p(VecArgs a, int t, int init, int np) {
  const int b = blockIdx.y;
  const ProbParams P = a.ctrl.params[b];
  ProbState* S = a.ctrl.state + b;
  if (!block_gate_cg(P, S)) return;
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  bool stop;
  double rr;
  if (init) {
    const int sl[2] = {kSlRhs2, kSlRr};
    double tv[2];
    reduce_slots<2>(a.ctrl, b, np, sl, tv);
    const double trhs2 = tv[0], tr2 = tv[1];
    const bool bad = !(trhs2 <= 1.0e300) || !(tr2 <= 1.0e300);  // NaN or Inf
    stop = bad || !(tr2 > 0.0) || P.max_cg <= 0;
    rr = tr2;
    if (lead) {
      double tol2 = P.rtol * P.rtol * (P.rhs_rel ? trhs2 : tr2);
      tol2 = fmax(tol2, P.tol_floor * P.tol_floor * trhs2);
      S->rhs2 = trhs2;
      S->r02 = tr2;
      S->rr = tr2;
      S->tol2 = tol2;
      if (bad) S->breakdown = 1;
      if (stop) S->cg_active = 0;
    }
  } else {
    const int sl[1] = {kSlRr};
    double tv[1];
    reduce_slots<1>(a.ctrl, b, np, sl, tv);  // written by the CG update in use
    rr = tv[0];
    const bool bad = !(rr <= 1.0e300);
    stop = bad || rr <= S->tol2 || t + 1 >= P.max_cg;
    if (lead) {
      S->rr = rr;
      S->cg_iters = t + 1;
      if (bad) S->breakdown = 1;
      if (stop) S->cg_active = 0;
    }
  }
  if (stop) return;
  const int64_t n = a.n;
  const Chunk ch = my_chunk(n, a.chunkf);  // the finer grid: 64 rows per step
  const int64_t off = (int64_t)b * n;
  const VT* r = static_cast<const VT*>(a.r) + off;
  VT* p = static_cast<VT*>(a.p) + off;
  __shared__ double cf[kMaxS];  // c_j, zero past s_eff
  __shared__ double s_rz;
  __shared__ double uc[4][64];
  const int s_eff = a.U ? a.ctrl.s_eff[b] : 0;
  const double* cb = a.ctrl.coef + (int64_t)b * 2 * kMaxS;
  __shared__ double tm[kMaxS];
  for (int j = threadIdx.x; j < kMaxS; j += blockDim.x) {
    cf[j] = j < s_eff ? cb[j] : 0.0;
    tm[j] = j < s_eff ? cb[kMaxS + j] : 0.0;
  }
  __syncthreads();
  if (threadIdx.x < 64) {  // fixed order: lane l adds terms l and l + 64, then the wave sum
    const double w = wave_sum(tm[threadIdx.x] + tm[threadIdx.x + 64]);
    if (threadIdx.x == 0) s_rz = rr + w;
  }
  __syncthreads();
  const double rz_new = s_rz;
  double beta = 0.0;
  if (!init) {
    const double rz_old = S->rz2[t & 1];
    beta = rz_old != 0.0 ? rz_new / rz_old : 0.0;
  }
  if (lead) {
    S->rz2[init ? 0 : ((t + 1) & 1)] = rz_new;
    S->beta_cg = beta;
  }
  const VT* Ub = a.U ? static_cast<const VT*>(a.U) + (int64_t)b * n * a.s_stride : nullptr;
  const uint8_t* mask = a.mask ? a.mask + off : nullptr;
  const VT be = VT(beta);
  const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
  __shared__ double red[16];
  double pp_on = 0.0, pp_off = 0.0;  // ||p||^2 on and off the mask (for p^T q)
  for (int64_t base = ch.lo; base < ch.hi; base += 64) {
    const int64_t i = base + lane;
    const bool ok = i < ch.hi;
    const int64_t ic = ok ? i : ch.hi - 1;
    // (U c)_i: wave grp takes columns grp, grp + 4, ..., all its loads in flight at once
    // (columns past s_eff re-read the last one with weight 0)
    if (s_eff > 0) {
      constexpr int NJ = kMaxS / 4;
      VT uv[NJ];
#pragma unroll
      for (int jj = 0; jj < NJ; ++jj) {
        const int j = min(grp + 4 * jj, s_eff - 1);
        uv[jj] = Ub[(int64_t)j * n + ic];
      }
      double acc = 0.0;
#pragma unroll
      for (int jj = 0; jj < NJ; ++jj) acc += double(uv[jj]) * cf[grp + 4 * jj];
      uc[grp][lane] = acc;
    }
    __syncthreads();
    if (grp == 0 && ok) {
      double acc = double(r[i]);
      if (s_eff > 0) acc += ((uc[0][lane] + uc[1][lane]) + uc[2][lane]) + uc[3][lane];
      const VT wi = VT(acc);
      const VT pi = init ? wi : wi + be * p[i];
      p[i] = pi;
      const double p2 = double(pi) * double(pi);
      if (mask && !mask[i])
        pp_off += p2;
      else
        pp_on += p2;
    }
    __syncthreads();
  }
  double v[2] = {pp_on, pp_off};
  block_sum<2>(v, red);
  if (threadIdx.x == 0) {
    slot_ptr(a.ctrl, b, kSlPp)[blockIdx.x] = v[0];
    slot_ptr(a.ctrl, b, kSlPpOff)[blockIdx.x] = v[1];
  }
}

// hp = H p (sum of the gemv_t split partials) and the partials of p^T q,
// q = hp + nu p (masked coordinates: q = p).
template <typename VT>
__global__ __launch_bounds__(256) void k_cg_alpha(VecArgs a) {
  const int b = blockIdx.y;
  const ProbParams P = a.ctrl.params[b];
  const ProbState* S = a.ctrl.state + b;
  if (!P.run || !S->cg_active) return;
  const int64_t n = a.n;
  const Chunk ch = my_chunk(n, a.chunkf);
  const int64_t off = (int64_t)b * n;
  const VT* p = static_cast<const VT*>(a.p) + off;
  VT* hp = static_cast<VT*>(a.hp) + off;
  const VT* yp = static_cast<const VT*>(a.ypart) + (int64_t)b * a.ypart_prob_stride;
  const uint8_t* mask = a.mask ? a.mask + off : nullptr;
  __shared__ double red[16];
  __shared__ VT sums[4][64];
  const VT nu = VT(P.nu);
  const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int64_t kst = a.ypart_ks_stride;
  double pq = 0.0;
  // 64 elements per step; wave grp sums the partial slots grp, grp + 4, ... (8 loads
  // in flight), then wave 0 adds the four sums in a fixed order
  for (int64_t base = ch.lo; base < ch.hi; base += 64) {
    const int64_t i = base + lane;
    const bool ok = i < ch.hi;
    const int64_t ic = ok ? i : ch.hi - 1;
    VT s = VT(0);
    int k = grp;
    for (; k + 28 < a.ksplit; k += 32) {
      VT tq[8];
#pragma unroll
      for (int q = 0; q < 8; ++q) tq[q] = yp[(int64_t)(k + 4 * q) * kst + ic];
#pragma unroll
      for (int q = 0; q < 8; ++q) s += tq[q];
    }
    for (; k < a.ksplit; k += 4) s += yp[(int64_t)k * kst + ic];
    sums[grp][lane] = s;
    __syncthreads();
    if (grp == 0 && ok) {
      VT t = ((sums[0][lane] + sums[1][lane]) + sums[2][lane]) + sums[3][lane];
      const VT pi = p[i];
      VT q;
      if (mask && !mask[i]) {
        t = VT(0);
        q = pi;
      } else {
        q = t + nu * pi;
      }
      hp[i] = t;
      pq += double(pi) * double(q);
    }
    __syncthreads();
  }
  double v[1] = {pq};
  block_sum<1>(v, red);
  if (threadIdx.x == 0) slot_ptr(a.ctrl, b, kSlPq)[blockIdx.x] = v[0];
}

// alpha = (r^T w)_t / p^T q, then x += alpha p, h += alpha hp (h tracks H x),
// r -= alpha q, and the partials of ||r||^2 and U^T r.
template <typename VT>
__global__ __launch_bounds__(256) void k_cg_update(VecArgs a, int t) {
  const int b = blockIdx.y;
  const ProbParams P = a.ctrl.params[b];
  ProbState* S = a.ctrl.state + b;
  if (!block_gate_cg(P, S)) return;
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  const int sl[1] = {kSlPq};
  double tv[1];
  reduce_slots<1>(a.ctrl, b, a.nbf, sl, tv);  // written by k_cg_alpha's finer grid
  const double pq = tv[0];
  if (!(pq > 0.0) || !(pq <= 1.0e300)) {  // not positive definite along p, or non-finite
    if (lead) {
      S->pq = pq;
      S->alpha_cg = 0.0;
      S->breakdown = 1;
      S->cg_active = 0;
    }
    return;
  }
  const double alpha = S->rz2[t & 1] / pq;
  if (lead) {
    S->pq = pq;
    S->alpha_cg = alpha;
  }
  const int64_t n = a.n;
  const Chunk ch = my_chunk(n, a.chunk);
  const int64_t off = (int64_t)b * n;
  VT* x = static_cast<VT*>(a.x) + off;
  VT* h = static_cast<VT*>(a.h) + off;
  VT* r = static_cast<VT*>(a.r) + off;
  const VT* p = static_cast<const VT*>(a.p) + off;
  const VT* hp = static_cast<const VT*>(a.hp) + off;
  const uint8_t* mask = a.mask ? a.mask + off : nullptr;
  __shared__ VT rs[kVecChunk * 4];
  __shared__ double red[16];
  const VT al = VT(alpha), nu = VT(P.nu);
  double rr = 0.0;
  for (int64_t i = ch.lo + threadIdx.x; i < ch.hi; i += blockDim.x) {
    // all loads before the first store (the vectors are distinct)
    const VT pi = p[i], hpi = hp[i], xi = x[i], hi = h[i], r0 = r[i];
    const VT q = (mask && !mask[i]) ? pi : hpi + nu * pi;
    x[i] = xi + al * pi;
    h[i] = hi + al * hpi;
    const VT ri = r0 - al * q;
    r[i] = ri;
    rs[i - ch.lo] = ri;
    rr += double(ri) * double(ri);
  }
  __syncthreads();
  const int s_eff = a.U ? a.ctrl.s_eff[b] : 0;
  if (s_eff > 0)
    ut_r_partial<VT>(static_cast<const VT*>(a.U) + (int64_t)b * n * a.s_stride, n, s_eff, ch, rs,
                     a.ctrl.upart + (int64_t)b * kMaxS * a.ctrl.pstride + blockIdx.x,
                     a.ctrl.pstride);
  double v[1] = {rr};
  block_sum<1>(v, red);
  if (threadIdx.x == 0) slot_ptr(a.ctrl, b, kSlRr)[blockIdx.x] = v[0];
}

// CG iteration t after the fused product (one pass over A, which also left per block
// the sum over its rows of d_i (a_i^T p)^2): p^T q = p^T H p + nu ||p||^2 (masked
// coordinates: q = p) from those partials and precond_p's ||p||^2 partials, every
// block summing them in the same order; alpha = (r^T P^-1 r)_t / p^T q; then, 64
// elements per step with the four waves splitting the product's block partials,
// hp = H p, x += alpha p, h += alpha hp (h tracks H x), r -= alpha q, and the
// partials of ||r||^2 and U^T r over the block's chunk.  It replaces cg_alpha and
// cg_update (hp is never stored) on the finer grid.
template <typename VT>
__global__ __launch_bounds__(256) void k_cg_step(VecArgs a, int t) {
  const int b = blockIdx.y;
  const ProbParams P = a.ctrl.params[b];
  ProbState* S = a.ctrl.state + b;
  if (!block_gate_cg(P, S)) return;
  const bool lead = blockIdx.x == 0 && threadIdx.x == 0;
  const int64_t n = a.n;
  const Chunk ch = my_chunk(n, a.chunkf);
  const VT* Ub = a.U ? static_cast<const VT*>(a.U) + (int64_t)b * a.n * a.s_stride : nullptr;
  VT uv[32];  // the first step's U rows, in flight during the alpha and H p sums
  if (Ub && ch.lo < ch.hi) ut_r64_load<VT>(Ub, n, a.s_stride, ch.lo, ch.hi, uv);
  __shared__ double red[16];
  __shared__ double bc[3];
  {
    double v[3] = {0.0, 0.0, 0.0};
    const double* hq = a.hpq + (int64_t)b * a.hpq_stride;
    double vh[1] = {0.0};
    strided_sum4<1>(a.nhpq, [&](int, int k) { return hq[k]; }, vh);
    v[0] = vh[0];
    const double* s_on = slot_ptr(a.ctrl, b, kSlPp);  // written by precond_p
    const double* s_off = slot_ptr(a.ctrl, b, kSlPpOff);
    double vp[2] = {0.0, 0.0};
    strided_sum4<2>(a.nbf, [&](int q, int k) { return q == 0 ? s_on[k] : s_off[k]; }, vp);
    v[1] = vp[0];
    v[2] = vp[1];
    block_sum<3>(v, red);
    if (threadIdx.x == 0) {
      bc[0] = v[0];
      bc[1] = v[1];
      bc[2] = v[2];
    }
    __syncthreads();
  }
  const double pq = (bc[0] + P.nu * bc[1]) + bc[2];
  if (!(pq > 0.0) || !(pq <= 1.0e300)) {  // not positive definite along p, or non-finite
    if (lead) {
      S->pq = pq;
      S->alpha_cg = 0.0;
      S->breakdown = 1;
      S->cg_active = 0;
    }
    return;
  }
  const double alpha = S->rz2[t & 1] / pq;
  if (lead) {
    S->pq = pq;
    S->alpha_cg = alpha;
  }
  const int64_t off = (int64_t)b * n;
  VT* x = static_cast<VT*>(a.x) + off;
  VT* h = static_cast<VT*>(a.h) + off;
  VT* r = static_cast<VT*>(a.r) + off;
  const VT* p = static_cast<const VT*>(a.p) + off;
  const VT* yp = static_cast<const VT*>(a.ypart) + (int64_t)b * a.ypart_prob_stride;
  const uint8_t* mask = a.mask ? a.mask + off : nullptr;
  const int s_eff = a.U ? a.ctrl.s_eff[b] : 0;
  __shared__ VT sums[4][64];
  __shared__ VT rs[64];
  const VT al = VT(alpha), nu = VT(P.nu);
  const int lane = threadIdx.x & 63, grp = threadIdx.x >> 6;
  const int64_t kst = a.ypart_ks_stride;
  constexpr int KB = 32;  // partial slots in flight per lane
  double ur = 0.0;        // this thread's share of (U^T r)_j, j = threadIdx.x / 2
  double rr = 0.0;
  for (int64_t base = ch.lo; base < ch.hi; base += 64) {
    if (Ub && base != ch.lo) ut_r64_load<VT>(Ub, n, a.s_stride, base, ch.hi, uv);
    const int64_t i = base + lane;
    const bool ok = i < ch.hi;
    const int64_t ic = ok ? i : ch.hi - 1;
    // hp_i: wave grp sums the partial slots grp, grp + 4, ..., KB loads in flight
    VT sacc = VT(0);
    for (int k0 = grp; k0 < a.ksplit; k0 += 4 * KB) {
      VT tq[KB];
#pragma unroll
      for (int q = 0; q < KB; ++q) {
        const int k = k0 + 4 * q;
        tq[q] = yp[(int64_t)(k < a.ksplit ? k : grp) * kst + ic];
      }
#pragma unroll
      for (int q = 0; q < KB; ++q)
        if (k0 + 4 * q < a.ksplit) sacc += tq[q];
    }
    sums[grp][lane] = sacc;
    __syncthreads();
    if (grp == 0) {
      VT ri = VT(0);
      if (ok) {
        const VT hpi = ((sums[0][lane] + sums[1][lane]) + sums[2][lane]) + sums[3][lane];
        const VT pi = p[i], xi = x[i], hi = h[i], r0 = r[i];
        const bool on = !(mask && !mask[i]);
        const VT q = on ? hpi + nu * pi : pi;
        x[i] = xi + al * pi;
        if (on) h[i] = hi + al * hpi;
        ri = r0 - al * q;
        r[i] = ri;
        rr += double(ri) * double(ri);
      }
      rs[lane] = ri;  // zero past the chunk
    }
    __syncthreads();
    if (s_eff > 0) ut_r64_use<VT>(s_eff, uv, rs, ur);
    __syncthreads();
  }
  if (s_eff > 0)
    ut_r64_store(s_eff, ur, a.ctrl.upart + (int64_t)b * kMaxS * a.ctrl.pstride + blockIdx.x,
                 a.ctrl.pstride);
  double v[1] = {rr};
  block_sum<1>(v, red);
  if (threadIdx.x == 0) slot_ptr(a.ctrl, b, kSlRr)[blockIdx.x] = v[0];
}

// Over-relaxed z- and u-updates with the soft-threshold prox (Sec. 2.5, Sec. 3.1)
// and the partials of the residual norms of Sec. 2.3; runs once the x-solve of
// the iteration has finished.
template <typename VT>
__global__ __launch_bounds__(256) void k_admm_end(VecArgs a) {
  const int b = blockIdx.y;
  const ProbParams P = a.ctrl.params[b];
  const ProbState* S = a.ctrl.state + b;
  if (!P.run || S->cg_active || S->admm_done) return;
  const int64_t n = a.n;
  const Chunk ch = my_chunk(n, a.chunk);
  const int64_t off = (int64_t)b * n;
  const VT* x = static_cast<const VT*>(a.x) + off;
  VT* z = static_cast<VT*>(a.z) + off;
  VT* u = static_cast<VT*>(a.u) + off;
  const VT* h = static_cast<const VT*>(a.h) + off;
  const VT* c = P.use_c ? static_cast<const VT*>(a.c) + off : nullptr;
  const bool box = P.prox == kProxBox;
  const VT* lo = box && a.lo ? static_cast<const VT*>(a.lo) + off : nullptr;
  const VT* hi_b = box && a.hi ? static_cast<const VT*>(a.hi) + off : nullptr;
  __shared__ double red[7 * 4];
  const VT al = VT(P.alpha), one_m = VT(1.0 - P.alpha), kap = VT(P.kappa), rho = VT(P.rho);
  double s_rp = 0, s_x = 0, s_z = 0, s_u = 0, s_rd = 0, s_z1 = 0, s_nnz = 0;
  for (int64_t i = ch.lo + threadIdx.x; i < ch.hi; i += blockDim.x) {
    const VT xi = x[i], zi = z[i], ui = u[i];
    const VT hi = c ? h[i] : VT(0), ci = c ? c[i] : VT(0);
    const VT xh = al * xi + one_m * zi;
    VT zn;
    if (box) {  // projection onto the box (Sec. 3.2)
      zn = xh + ui;
      if (lo) zn = zn < lo[i] ? lo[i] : zn;
      if (hi_b) zn = zn > hi_b[i] ? hi_b[i] : zn;
    } else {
      zn = soft_threshold<VT>(xh + ui, kap);
    }
    const VT un = ui + xh - zn;
    z[i] = zn;
    u[i] = un;
    const double d = double(xi) - double(zn);
    s_rp += d * d;
    s_x += double(xi) * double(xi);
    s_z += double(zn) * double(zn);
    s_u += double(un) * double(un);
    if (c) {
      const double rd = double(hi - ci) + P.lambda2 * double(xi) + double(rho) * double(un);
      s_rd += rd * rd;
    }
    s_z1 += fabs(double(zn));
    s_nnz += (zn != VT(0)) ? 1.0 : 0.0;
  }
  double v[7] = {s_rp, s_x, s_z, s_u, s_rd, s_z1, s_nnz};
  block_sum<7>(v, red);
  if (threadIdx.x == 0)
#pragma unroll
    for (int k = 0; k < 7; ++k) slot_ptr(a.ctrl, b, kSlEnd0 + k)[blockIdx.x] = v[k];
}

// One block per problem: the 7 sums of admm_end into the state, then admm_done.
__global__ __launch_bounds__(256) void k_admm_finish(Ctrl ctrl, int nb) {
  const int b = blockIdx.y;
  const ProbParams P = ctrl.params[b];
  ProbState* S = ctrl.state + b;
  if (!P.run || S->cg_active || S->admm_done) return;
  const int sl[7] = {kSlEnd0, kSlEnd0 + 1, kSlEnd0 + 2, kSlEnd0 + 3,
                     kSlEnd0 + 4, kSlEnd0 + 5, kSlEnd0 + 6};
  double tv[7];
  reduce_slots<7>(ctrl, b, nb, sl, tv);
  if (threadIdx.x == 0) {
    for (int k = 0; k < 7; ++k) S->red[k] = tv[k];
    S->admm_done = 1;
  }
}

template <typename VT>
__global__ __launch_bounds__(256) void k_dual_residual(VecArgs a) {
  const int b = blockIdx.y;
  const ProbParams P = a.ctrl.params[b];
  if (!P.run) return;
  const int64_t n = a.n;
  const Chunk ch = my_chunk(n, a.chunk);
  const int64_t off = (int64_t)b * n;
  const VT* u = static_cast<const VT*>(a.u) + off;
  const VT* x = static_cast<const VT*>(a.x) + off;
  const VT* h = static_cast<const VT*>(a.h) + off;
  const VT* c = P.use_c ? static_cast<const VT*>(a.c) + off : nullptr;
  const VT* g = P.use_c ? nullptr : static_cast<const VT*>(a.g) + off;
  __shared__ double red[4];
  double s = 0.0;
  for (int64_t i = ch.lo + threadIdx.x; i < ch.hi; i += blockDim.x) {
    const double gi = (c ? double(h[i] - c[i]) : double(g[i])) + P.lambda2 * double(x[i]);
    const double rd = gi + P.rho * double(u[i]);
    s += rd * rd;
  }
  double v[1] = {s};
  block_sum<1>(v, red);
  if (threadIdx.x == 0) slot_ptr(a.ctrl, b, kSlDual)[blockIdx.x] = v[0];
}

__global__ __launch_bounds__(256) void k_dual_finish(Ctrl ctrl, int nb) {
  const int b = blockIdx.y;
  if (!ctrl.params[b].run) return;
  const int sl[1] = {kSlDual};
  double tv[1];
  reduce_slots<1>(ctrl, b, nb, sl, tv);
  if (threadIdx.x == 0) ctrl.state[b].red[kRedRd2] = tv[0];
}

// Elementwise terms of the ML x-system: d = f''(t), col0 = d o t (for H x),
// col1 = f'(t) (for grad f).  Logistic (LOSS = kLossLogistic): w = -y t,
// s = sigmoid(w), d = s (1 - s), f' = -y s.  Huber: r = t - b, d = 2 [|r| <= delta],
// f' = 2 clip(r, -delta, delta).
template <typename VT, int LOSS>
__global__ __launch_bounds__(256) void k_loss_elem(int64_t m, const VT* __restrict__ tparts,
                                                   int nsplit, int64_t split_stride,
                                                   int64_t prob_stride,
                                                   const VT* __restrict__ bv, VT delta,
                                                   VT* __restrict__ d, VT* __restrict__ cols,
                                                   int64_t col_stride,
                                                   const int32_t* __restrict__ gate,
                                                   int gate_stride) {
  const int b = blockIdx.y;
  if (gate != nullptr && gate[(int64_t)b * gate_stride] == 0) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * blockDim.x) {
    VT t = VT(0);
    for (int k = 0; k < nsplit; ++k) t += tparts[(int64_t)b * prob_stride + (int64_t)k * split_stride + i];
    const VT bi = bv[(int64_t)b * m + i];
    VT di, fi;
    if constexpr (LOSS == kLossLogistic) {
      const VT w = -bi * t;
      VT s;
      if constexpr (sizeof(VT) == 4)
        s = 1.0f / (1.0f + expf(-w));
      else
        s = 1.0 / (1.0 + exp(-w));
      di = s * (VT(1) - s);
      fi = -bi * s;
    } else {
      const VT r = t - bi;
      di = fabs(r) <= delta ? VT(2) : VT(0);
      fi = VT(2) * fmin(fmax(r, -delta), delta);
    }
    d[(int64_t)b * m + i] = di;
    VT* cb = cols + (int64_t)b * 2 * col_stride;
    cb[i] = di * t;
    cb[col_stride + i] = fi;
  }
}

template <typename VT>
__global__ __launch_bounds__(256) void k_admm_update_hook(int64_t n, double alpha, double kappa,
                                                          const VT* __restrict__ x,
                                                          VT* __restrict__ z, VT* __restrict__ u,
                                                          double* part, unsigned* counter,
                                                          double* out4, int nb) {
  const int64_t chunk = (n + nb - 1) / nb;
  const int64_t lo = (int64_t)blockIdx.x * chunk, hi = min(n, lo + chunk);
  __shared__ double red[16];
  const VT al = VT(alpha), one_m = VT(1.0 - alpha), kap = VT(kappa);
  double s0 = 0, s1 = 0, s2 = 0, s3 = 0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x) {
    const VT xi = x[i], zi = z[i], ui = u[i];
    const VT xh = al * xi + one_m * zi;
    const VT zn = soft_threshold<VT>(xh + ui, kap);
    const VT un = ui + xh - zn;
    z[i] = zn;
    u[i] = un;
    const double d = double(xi) - double(zn);
    s0 += d * d;
    s1 += double(xi) * double(xi);
    s2 += double(zn) * double(zn);
    s3 += double(un) * double(un);
  }
  double v[4] = {s0, s1, s2, s3};
  block_sum<4>(v, red);
  if (threadIdx.x == 0)
    for (int k = 0; k < 4; ++k) part[(int64_t)blockIdx.x * 4 + k] = v[k];
  if (!last_block_arrive(counter, nb)) return;
  if (threadIdx.x == 0)
    for (int k = 0; k < 4; ++k) {
      double s = 0.0;
      for (int j = 0; j < nb; ++j) s += load_partial(part + (int64_t)j * 4 + k);
      out4[k] = s;
    }
}

// Stand-alone preconditioner apply: z = r + U (((lam_rr + nu)/(lam + nu) - 1) o U^T r).
template <typename VT>
__global__ __launch_bounds__(256) void k_precond_utr(int64_t n, int s, const VT* __restrict__ U,
                                                     const double* __restrict__ lamhat,
                                                     const int32_t* __restrict__ s_eff_arr,
                                                     double nu, const VT* __restrict__ r,
                                                     double* part, int64_t part_stride,
                                                     unsigned* counters, double* coef, int nb,
                                                     int64_t chunk) {
  const int b = blockIdx.y;
  const Chunk ch = my_chunk(n, chunk);
  const int s_eff = s_eff_arr ? s_eff_arr[b] : s;
  __shared__ VT rs[kVecChunk * 4];
  const VT* rb = r + (int64_t)b * n;
  for (int64_t i = ch.lo + threadIdx.x; i < ch.hi; i += blockDim.x) rs[i - ch.lo] = rb[i];
  __syncthreads();
  double* part_b = part + (int64_t)b * part_stride;
  ut_r_partial<VT>(U + (int64_t)b * n * s, n, s_eff, ch, rs, part_b + (int64_t)blockIdx.x * kPartW);
  if (!last_block_arrive(counters + (int64_t)b * kNumCounters + kCntAux1, nb)) return;
  finish_coef(part_b, nb, s_eff, lamhat + (int64_t)b * s, nu, coef + (int64_t)b * kMaxS);
}

template <typename VT>
__global__ __launch_bounds__(256) void k_precond_out(int64_t n, int s, const VT* __restrict__ U,
                                                     const int32_t* __restrict__ s_eff_arr,
                                                     const VT* __restrict__ r,
                                                     const double* __restrict__ coef,
                                                     VT* __restrict__ z) {
  const int b = blockIdx.y;
  const int s_eff = s_eff_arr ? s_eff_arr[b] : s;
  __shared__ double cf[kMaxS];
  for (int j = threadIdx.x; j < s_eff; j += blockDim.x) cf[j] = coef[(int64_t)b * kMaxS + j];
  __syncthreads();
  const VT* Ub = U + (int64_t)b * n * s;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    double acc = double(r[(int64_t)b * n + i]);
    for (int j = 0; j < s_eff; ++j) acc += double(Ub[(int64_t)j * n + i]) * cf[j];
    z[(int64_t)b * n + i] = VT(acc);
  }
}

template <typename VT>
__global__ __launch_bounds__(256) void k_build_mask(int64_t n, const VT* __restrict__ zs,
                                                    const VT* __restrict__ gz,
                                                    uint8_t* __restrict__ mask,
                                                    VT* __restrict__ sgn, VT* __restrict__ rhs) {
  const int b = blockIdx.y;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n;
       i += (int64_t)gridDim.x * blockDim.x) {
    const int64_t k = (int64_t)b * n + i;
    const VT zi = zs[k];
    const bool on = zi != VT(0);
    mask[k] = on ? 1 : 0;
    sgn[k] = zi > VT(0) ? VT(1) : (zi < VT(0) ? VT(-1) : VT(0));
    rhs[k] = on ? -gz[k] : VT(0);  // the CG start uses g = -rhs
  }
}

template <typename VT>
__global__ __launch_bounds__(256) void k_masked_dot(int64_t n, const VT* __restrict__ a,
                                                    const VT* __restrict__ bv, double* part,
                                                    int64_t part_stride, unsigned* counters,
                                                    double* out, int nb) {
  const int b = blockIdx.y;
  const int64_t chunk = (n + nb - 1) / nb;
  const int64_t lo = (int64_t)blockIdx.x * chunk, hi = min(n, lo + chunk);
  __shared__ double red[4];
  double s = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += blockDim.x)
    s += double(a[(int64_t)b * n + i]) * double(bv[(int64_t)b * n + i]);
  double v[1] = {s};
  block_sum<1>(v, red);
  double* pb = part + (int64_t)b * part_stride;
  if (threadIdx.x == 0) pb[(int64_t)blockIdx.x * kPartW + kMaxS + 14] = v[0];
  if (!last_block_arrive(counters + (int64_t)b * kNumCounters + kCntMasked, nb)) return;
  double tv[1];
  sum_slots<1>(pb, nb, 14, tv, red);
  if (threadIdx.x == 0) out[b] = tv[0];
}

}  // namespace

#define GENIOS_VEC_LAUNCH(kern, ...)                                                   \
  do {                                                                                 \
    dim3 grid((unsigned)a.nb, (unsigned)a.batch);                                      \
    if (a.vt == VT_F32)                                                                \
      hipLaunchKernelGGL(kern<float>, grid, dim3(kVecBlock), 0, st, a, ##__VA_ARGS__); \
    else                                                                               \
      hipLaunchKernelGGL(kern<double>, grid, dim3(kVecBlock), 0, st, a, ##__VA_ARGS__); \
    return hipGetLastError();                                                          \
  } while (0)

static bool vec_geometry_ok(const VecArgs& a) {
  // every vector kernel writes one partial per block into pstride-sized slots
  return a.nb >= 1 && a.nb <= a.ctrl.pstride && a.chunk >= 1 && a.chunk <= 4 * kVecChunk &&
         (int64_t)a.nb * a.chunk >= a.n && a.nbf >= 1 && a.nbf <= a.ctrl.pstride &&
         a.chunkf >= 1 && a.chunkf <= 4 * kVecChunk && (int64_t)a.nbf * a.chunkf >= a.n;
}

#define GENIOS_VEC_CHECK() \
  do {                     \
    if (!vec_geometry_ok(a)) return hipErrorInvalidValue; \
  } while (0)

hipError_t launch_admm_begin(const VecArgs& a, hipStream_t st) {
  GENIOS_VEC_CHECK();
  dim3 grid((unsigned)a.nbf, (unsigned)a.batch);  // the finer grid
  if (a.vt == VT_F32)
    hipLaunchKernelGGL(k_admm_begin<float>, grid, dim3(kVecBlock), 0, st, a);
  else
    hipLaunchKernelGGL(k_admm_begin<double>, grid, dim3(kVecBlock), 0, st, a);
  return hipGetLastError();
}
hipError_t launch_precond_coef(const VecArgs& a, int np, hipStream_t st) {
  GENIOS_VEC_CHECK();
  if (np < 1 || np > a.ctrl.pstride) return hipErrorInvalidValue;
  if (a.U == nullptr) return hipSuccess;
  hipLaunchKernelGGL(k_precond_coef, dim3((unsigned)kMaxS, (unsigned)a.batch), dim3(256), 0, st,
                     a.ctrl, np);
  return hipGetLastError();
}
hipError_t launch_precond_p(const VecArgs& a, int t, int init, int np, hipStream_t st) {
  GENIOS_VEC_CHECK();
  if (np < 1 || np > a.ctrl.pstride) return hipErrorInvalidValue;
  dim3 grid((unsigned)a.nbf, (unsigned)a.batch);  // the finer grid
  if (a.vt == VT_F32)
    hipLaunchKernelGGL(k_precond_p<float>, grid, dim3(kVecBlock), 0, st, a, t, init, np);
  else
    hipLaunchKernelGGL(k_precond_p<double>, grid, dim3(kVecBlock), 0, st, a, t, init, np);
  return hipGetLastError();
}
hipError_t launch_cg_step(const VecArgs& a, int t, hipStream_t st) {
  GENIOS_VEC_CHECK();
  if (a.hpq == nullptr || a.nhpq < 1 || a.nhpq > a.hpq_stride) return hipErrorInvalidValue;
  dim3 grid((unsigned)a.nbf, (unsigned)a.batch);  // the finer grid
  if (a.vt == VT_F32)
    hipLaunchKernelGGL(k_cg_step<float>, grid, dim3(kVecBlock), 0, st, a, t);
  else
    hipLaunchKernelGGL(k_cg_step<double>, grid, dim3(kVecBlock), 0, st, a, t);
  return hipGetLastError();
}
hipError_t launch_cg_alpha(const VecArgs& a, hipStream_t st) {
  GENIOS_VEC_CHECK();
  dim3 grid((unsigned)a.nbf, (unsigned)a.batch);  // the finer grid
  if (a.vt == VT_F32)
    hipLaunchKernelGGL(k_cg_alpha<float>, grid, dim3(kVecBlock), 0, st, a);
  else
    hipLaunchKernelGGL(k_cg_alpha<double>, grid, dim3(kVecBlock), 0, st, a);
  return hipGetLastError();
}
hipError_t launch_cg_update(const VecArgs& a, int t, hipStream_t st) {
  GENIOS_VEC_CHECK();
  GENIOS_VEC_LAUNCH(k_cg_update, t);
}
hipError_t launch_admm_end(const VecArgs& a, hipStream_t st) {
  GENIOS_VEC_CHECK();
  GENIOS_VEC_LAUNCH(k_admm_end);
}
hipError_t launch_admm_finish(const VecArgs& a, hipStream_t st) {
  GENIOS_VEC_CHECK();
  hipLaunchKernelGGL(k_admm_finish, dim3(1, (unsigned)a.batch), dim3(256), 0, st, a.ctrl, a.nb);
  return hipGetLastError();
}
hipError_t launch_dual_residual(const VecArgs& a, hipStream_t st) {
  GENIOS_VEC_CHECK();
  dim3 grid((unsigned)a.nb, (unsigned)a.batch);
  if (a.vt == VT_F32)
    hipLaunchKernelGGL(k_dual_residual<float>, grid, dim3(kVecBlock), 0, st, a);
  else
    hipLaunchKernelGGL(k_dual_residual<double>, grid, dim3(kVecBlock), 0, st, a);
  hipLaunchKernelGGL(k_dual_finish, dim3(1, (unsigned)a.batch), dim3(256), 0, st, a.ctrl, a.nb);
  return hipGetLastError();
}

static int m_blocks(int64_t m) {
  return (int)std::max<int64_t>(1, std::min<int64_t>((m + kVecChunk - 1) / kVecChunk, kMaxVecBlocks));
}

template <typename VT, int LOSS>
static void loss_elem_vt(dim3 grid, int64_t m, const void* tparts, int nsplit,
                         int64_t split_stride, int64_t prob_stride, const void* bvec, double delta,
                         void* d, void* cols, int64_t col_stride, const int32_t* gate,
                         int gate_stride, hipStream_t st) {
  hipLaunchKernelGGL((k_loss_elem<VT, LOSS>), grid, dim3(256), 0, st, m,
                     static_cast<const VT*>(tparts), nsplit, split_stride, prob_stride,
                     static_cast<const VT*>(bvec), VT(delta), static_cast<VT*>(d),
                     static_cast<VT*>(cols), col_stride, gate, gate_stride);
}

hipError_t launch_loss_elem(VType vt, int loss, double delta, int64_t m, int64_t batch,
                            const void* tparts, int nsplit, int64_t split_stride,
                            int64_t prob_stride, const void* bvec, void* d, void* cols,
                            int64_t col_stride, const int32_t* gate, int gate_stride,
                            hipStream_t st) {
  if (loss != kLossLogistic && loss != kLossHuber) return hipErrorInvalidValue;
  const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((m + 255) / 256, 512));
  dim3 grid(nb, (unsigned)batch);
  if (vt == VT_F32) {
    if (loss == kLossLogistic)
      loss_elem_vt<float, kLossLogistic>(grid, m, tparts, nsplit, split_stride, prob_stride, bvec,
                                         delta, d, cols, col_stride, gate, gate_stride, st);
    else
      loss_elem_vt<float, kLossHuber>(grid, m, tparts, nsplit, split_stride, prob_stride, bvec,
                                      delta, d, cols, col_stride, gate, gate_stride, st);
  } else {
    if (loss == kLossLogistic)
      loss_elem_vt<double, kLossLogistic>(grid, m, tparts, nsplit, split_stride, prob_stride,
                                          bvec, delta, d, cols, col_stride, gate, gate_stride, st);
    else
      loss_elem_vt<double, kLossHuber>(grid, m, tparts, nsplit, split_stride, prob_stride, bvec,
                                       delta, d, cols, col_stride, gate, gate_stride, st);
  }
  return hipGetLastError();
}

hipError_t launch_admm_update_hook(VType vt, int64_t n, double alpha, double kappa, const void* x,
                                   void* z, void* u, double* part, unsigned* counter,
                                   double* out4, hipStream_t st) {
  const int nb = m_blocks(n);
  if (vt == VT_F32)
    hipLaunchKernelGGL(k_admm_update_hook<float>, dim3(nb), dim3(256), 0, st, n, alpha, kappa,
                       static_cast<const float*>(x), static_cast<float*>(z),
                       static_cast<float*>(u), part, counter, out4, nb);
  else
    hipLaunchKernelGGL(k_admm_update_hook<double>, dim3(nb), dim3(256), 0, st, n, alpha, kappa,
                       static_cast<const double*>(x), static_cast<double*>(z),
                       static_cast<double*>(u), part, counter, out4, nb);
  return hipGetLastError();
}

hipError_t launch_precond_apply(VType vt, int64_t n, int s, int64_t batch, const void* U,
                                const double* lamhat, const int32_t* s_eff, double nu,
                                const void* r, void* z, double* part, int64_t part_stride,
                                unsigned* counters, double* coef, hipStream_t st) {
  const int64_t chunk = kVecChunk;
  const int nb = (int)((n + chunk - 1) / chunk);
  if ((int64_t)nb * kPartW > part_stride) return hipErrorInvalidValue;
  dim3 g1((unsigned)nb, (unsigned)batch);
  const unsigned nb2 = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 1024));
  dim3 g2(nb2, (unsigned)batch);
  if (vt == VT_F32) {
    hipLaunchKernelGGL(k_precond_utr<float>, g1, dim3(256), 0, st, n, s,
                       static_cast<const float*>(U), lamhat, s_eff, nu,
                       static_cast<const float*>(r), part, part_stride, counters, coef, nb,
                       chunk);
    hipLaunchKernelGGL(k_precond_out<float>, g2, dim3(256), 0, st, n, s,
                       static_cast<const float*>(U), s_eff, static_cast<const float*>(r), coef,
                       static_cast<float*>(z));
  } else {
    hipLaunchKernelGGL(k_precond_utr<double>, g1, dim3(256), 0, st, n, s,
                       static_cast<const double*>(U), lamhat, s_eff, nu,
                       static_cast<const double*>(r), part, part_stride, counters, coef, nb,
                       chunk);
    hipLaunchKernelGGL(k_precond_out<double>, g2, dim3(256), 0, st, n, s,
                       static_cast<const double*>(U), s_eff, static_cast<const double*>(r), coef,
                       static_cast<double*>(z));
  }
  return hipGetLastError();
}

hipError_t launch_build_mask(VType vt, int64_t n, int64_t batch, const void* zstar,
                             const void* gz, uint8_t* mask, void* sgn, void* rhs,
                             hipStream_t st) {
  const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, 512));
  dim3 grid(nb, (unsigned)batch);
  if (vt == VT_F32)
    hipLaunchKernelGGL(k_build_mask<float>, grid, dim3(256), 0, st, n,
                       static_cast<const float*>(zstar), static_cast<const float*>(gz), mask,
                       static_cast<float*>(sgn), static_cast<float*>(rhs));
  else
    hipLaunchKernelGGL(k_build_mask<double>, grid, dim3(256), 0, st, n,
                       static_cast<const double*>(zstar), static_cast<const double*>(gz), mask,
                       static_cast<double*>(sgn), static_cast<double*>(rhs));
  return hipGetLastError();
}

hipError_t launch_masked_dot(VType vt, int64_t n, int64_t batch, const void* a, const void* b,
                             double* part, int64_t part_stride, unsigned* counters, double* out,
                             hipStream_t st) {
  const int nb = m_blocks(n);
  dim3 grid((unsigned)nb, (unsigned)batch);
  if (vt == VT_F32)
    hipLaunchKernelGGL(k_masked_dot<float>, grid, dim3(256), 0, st, n,
                       static_cast<const float*>(a), static_cast<const float*>(b), part, part_stride,
                       counters, out, nb);
  else
    hipLaunchKernelGGL(k_masked_dot<double>, grid, dim3(256), 0, st, n,
                       static_cast<const double*>(a), static_cast<const double*>(b), part,
                       part_stride, counters, out, nb);
  return hipGetLastError();
}

}  // namespace genios

// ---- active-set compaction for the adjoint ---------------------------------------
namespace genios {

namespace {

// idx[b][0..cnt) = positions of the nonzero mask entries of problem b, in order.
// One 1024-thread block per problem: per-thread counts, a block scan in LDS,
// then ordered writes (deterministic).
__global__ __launch_bounds__(1024) void k_compact_index(int64_t n, const uint8_t* __restrict__ mask,
                                                        int32_t* __restrict__ idx,
                                                        int32_t* __restrict__ cnt) {
  __shared__ int32_t sc[1024];
  const int b = blockIdx.x, t = threadIdx.x, nt = blockDim.x;
  const int64_t per = (n + nt - 1) / nt;
  const int64_t lo = min(n, (int64_t)t * per), hi = min(n, lo + per);
  const uint8_t* mb = mask + (int64_t)b * n;
  int32_t c = 0;
  for (int64_t i = lo; i < hi; ++i) c += mb[i] ? 1 : 0;
  sc[t] = c;
  __syncthreads();
  for (int off = 1; off < nt; off <<= 1) {  // inclusive Hillis-Steele scan
    const int32_t v = t >= off ? sc[t - off] : 0;
    __syncthreads();
    sc[t] += v;
    __syncthreads();
  }
  int32_t pos = sc[t] - c;
  int32_t* ib = idx + (int64_t)b * n;
  for (int64_t i = lo; i < hi; ++i)
    if (mb[i]) ib[pos++] = (int32_t)i;
  if (t == nt - 1) cnt[b] = sc[t];
}

// out[b] (m x ldS, row-major) = columns idx[b][0..cnt) of A[b], zero padding.
template <typename T>
__global__ __launch_bounds__(256) void k_gather_cols(const T* __restrict__ A, int64_t lda,
                                                     int64_t strideA, int64_t m, int64_t n,
                                                     const int32_t* __restrict__ idx,
                                                     const int32_t* __restrict__ cnt, int ldS,
                                                     T* __restrict__ out) {
  const int b = blockIdx.y;
  const int c = cnt[b];
  const T* Ab = A + (int64_t)b * strideA;
  const int32_t* ib = idx + (int64_t)b * n;
  T* ob = out + (int64_t)b * m * ldS;
  const int64_t total = m * (int64_t)ldS;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t r = e / ldS;
    const int k = (int)(e - r * ldS);
    ob[e] = k < c ? Ab[r * lda + ib[k]] : T(0);
  }
}

// out[b][k] = in[b][idx[b][k]] for k < cnt[b], 0 after (length ldS); mask_out[b][k] = k < cnt[b].
template <typename VT>
__global__ __launch_bounds__(256) void k_gather_vec(int64_t n, const int32_t* __restrict__ idx,
                                                    const int32_t* __restrict__ cnt, int ldS,
                                                    const VT* __restrict__ in0, VT* __restrict__ out0,
                                                    const VT* __restrict__ in1, VT* __restrict__ out1,
                                                    uint8_t* __restrict__ mask_out) {
  const int b = blockIdx.y;
  const int c = cnt[b];
  const int32_t* ib = idx + (int64_t)b * n;
  for (int k = blockIdx.x * blockDim.x + threadIdx.x; k < ldS; k += gridDim.x * blockDim.x) {
    const bool on = k < c;
    const int64_t src = on ? ib[k] : 0;
    out0[(int64_t)b * ldS + k] = on ? in0[(int64_t)b * n + src] : VT(0);
    out1[(int64_t)b * ldS + k] = on ? in1[(int64_t)b * n + src] : VT(0);
    mask_out[(int64_t)b * ldS + k] = on ? 1 : 0;
  }
}

}  // namespace

hipError_t launch_compact_index(int64_t n, int64_t batch, const uint8_t* mask, int32_t* idx,
                                int32_t* cnt, hipStream_t st) {
  hipLaunchKernelGGL(k_compact_index, dim3((unsigned)batch), dim3(1024), 0, st, n, mask, idx, cnt);
  return hipGetLastError();
}

hipError_t launch_gather_cols(MType mt, const void* A, int64_t lda, int64_t strideA, int64_t m,
                              int64_t n, int64_t batch, const int32_t* idx, const int32_t* cnt,
                              int ldS, void* out, hipStream_t st) {
  const int64_t total = m * (int64_t)ldS;
  const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((total + 255) / 256, 8192));
  dim3 grid(nb, (unsigned)batch);
  if (mt == MT_F32)
    hipLaunchKernelGGL(k_gather_cols<float>, grid, dim3(256), 0, st, static_cast<const float*>(A),
                       lda, strideA, m, n, idx, cnt, ldS, static_cast<float*>(out));
  else if (mt == MT_F64)
    hipLaunchKernelGGL(k_gather_cols<double>, grid, dim3(256), 0, st,
                       static_cast<const double*>(A), lda, strideA, m, n, idx, cnt, ldS,
                       static_cast<double*>(out));
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_gather_vec(VType vt, int64_t n, int64_t batch, const int32_t* idx,
                             const int32_t* cnt, int ldS, const void* in0, void* out0,
                             const void* in1, void* out1, uint8_t* mask_out, hipStream_t st) {
  const unsigned nb = (unsigned)std::max(1, std::min((ldS + 255) / 256, 1024));
  dim3 grid(nb, (unsigned)batch);
  if (vt == VT_F32)
    hipLaunchKernelGGL(k_gather_vec<float>, grid, dim3(256), 0, st, n, idx, cnt, ldS,
                       static_cast<const float*>(in0), static_cast<float*>(out0),
                       static_cast<const float*>(in1), static_cast<float*>(out1), mask_out);
  else
    hipLaunchKernelGGL(k_gather_vec<double>, grid, dim3(256), 0, st, n, idx, cnt, ldS,
                       static_cast<const double*>(in0), static_cast<double*>(out0),
                       static_cast<const double*>(in1), static_cast<double*>(out1), mask_out);
  return hipGetLastError();
}

}  // namespace genios
