// The s x s core of the stabilised Nystrom approximation (Sec. 2.2), for s <= 100, in
// two kernels:
//
//   k_nystrom_core_lds (one 1024-thread workgroup per problem, G in LDS)
//     M = sym(Omega^T Y) + mu Omega^T Omega = C C^T   blocked right-looking Cholesky
//                                                     (shift x10 on failure, <= 3 times)
//     G = C^-1 (Y_mu^T Y_mu) C^-T                     two blocked forward substitutions
//     G = V Sigma^2 V^T                               block Jacobi (below), V in global
//                                                     memory (core scratch)
//     sigma^2 sorted descending, the kept count, lambda_hat = max(sigma^2 - mu, 0)
//   k_core_vt (16 eigenvector columns per workgroup)
//     T = C^-T V(:, perm) Sigma^-1 by back substitution
//
// Block Jacobi.  The indices are cut into blocks of 8 (an even number of blocks, the
// padding rows and columns of G are zero and never rotate).  A sweep is the round-robin
// (circle method) over the blocks: in every round the blocks form disjoint pairs, each
// pair is a 16 x 16 subproblem, and one wavefront rotates it in place by one cyclic
// Jacobi pass over its index pairs, accumulating the 16 x 16 product R of its 2 x 2
// rotations.  The pass takes the pairs (i, i xor k) of the 16 indices for k = 1..15 in
// the first round of the sweep (every block meets its own pairs once per sweep) and for
// k = 8..15 afterwards (the pairs across the two blocks only), so that every index pair
// of G is rotated once per sweep, as in scalar cyclic Jacobi.  The rest of G then
// becomes R_A^T G[A, B] R_B, block by block, on the FP64 matrix cores.  A pair is
// rotated only while g_pq^2 > tol^2 |g_pp g_qq| (the threshold form for positive
// semidefinite matrices) and g_pq is then set to zero; the iteration ends after a sweep
// without a rotation or once every off-diagonal entry meets the threshold.  V <- V R
// for the previous round runs on the wavefronts that have no pair, while the others
// rotate their subproblems.
#include <algorithm>
#include <cmath>
#include <type_traits>

#include "device.hpp"

namespace genios {

namespace {

constexpr int kCoreThreads = 1024;
constexpr int kCoreWaves = kCoreThreads / 64;
constexpr int kChol = 16;  // block width of the Cholesky and of the triangular solves
constexpr int kJacMaxBlocks = 2 * ((kCoreLdsMaxS + 15) / 16);
constexpr int kJacMaxPairs = kJacMaxBlocks / 2;
constexpr int kJacMaxN = 8 * kJacMaxBlocks;
constexpr int kRs = 17;  // row stride of a 16 x 16 block in LDS
constexpr int kJacMaxSweeps = 16;
typedef double v4d __attribute__((ext_vector_type(4)));
static_assert(2 * kJacMaxPairs <= kCoreWaves, "one wavefront per block pair for the passes and for V");

__host__ __device__ inline int jac_blocks(int s) { return 2 * ((s + 15) / 16); }

// Pairs of the circle method: round r, pair t of nb (even) blocks, as (low, high).
__device__ __forceinline__ int2 circle_pair(int nb, int r, int t) {
  const int a0 = t, a1 = nb - 1 - t;
  int t0 = a0 - 1 + r, t1 = a1 - 1 + r;
  t0 %= (nb - 1);
  t1 %= (nb - 1);
  const int p = a0 == 0 ? 0 : 1 + t0;
  const int q = a1 == 0 ? 0 : 1 + t1;
  return make_int2(min(p, q), max(p, q));
}

// Workgroup barrier that orders LDS traffic only: the wavefront's LDS operations are
// complete (lgkmcnt 0) before s_barrier, while its global loads and stores stay in
// flight (a full __syncthreads also waits for those).  The empty asm statements keep
// the compiler from moving memory operations across it.
__device__ __forceinline__ void lds_barrier() {
  asm volatile("" ::: "memory");
  __builtin_amdgcn_s_waitcnt(0xc07f);  // vmcnt and expcnt at their maximum, lgkmcnt(0)
  __builtin_amdgcn_s_barrier();
  asm volatile("" ::: "memory");
}

// for (e = tid; e < n; e += nt) f(e), with the loads of kBatch consecutive iterations
// issued before their uses: load(e) returns what store(e, value) consumes.
template <int kBatch, typename Load, typename Store>
__device__ __forceinline__ void staged_for(int n, int tid, int nt, Load load, Store store) {
  for (int e0 = tid; e0 < n; e0 += kBatch * nt) {
    decltype(load(0)) v[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int e = e0 + u * nt;
      if (e < n) v[u] = load(e);
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int e = e0 + u * nt;
      if (e < n) store(e, v[u]);
    }
  }
}

__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// 1 / sqrt(x) for finite x > 0: the hardware estimate (relative error about 2^-24) and
// two Newton steps y <- y + y (1/2 - (x/2) y^2), each squaring the error.
__device__ __forceinline__ double rsqrt_nr(double x) {
  double y = __builtin_amdgcn_rsq(x);
  const double hx = 0.5 * x;
  y = fma(y, fma(-hx * y, y, 0.5), y);
  y = fma(y, fma(-hx * y, y, 0.5), y);
  return y;
}

// Rotation that zeroes the (p, q) entry of [[app, apq], [apq, aqq]] through J^T B J with
// J = [[c, s], [-s, c]]: h = aqq - app, g = 2 apq, r = sqrt(h^2 + g^2), d = |h| + r,
// c = d / sqrt(2 r d), s = sign(h) g / sqrt(2 r d) (then d^2 + g^2 = 2 r d, so
// c^2 + s^2 = 1 to the accuracy of the reciprocal square root).  Returns false
// (identity) below the threshold; above it g != 0, so r and d are positive.
__device__ __forceinline__ bool jac_rotation(double app, double aqq, double apq, double tol2,
                                             double& c, double& sn) {
  c = 1.0;
  sn = 0.0;
  if (!(apq * apq > tol2 * fabs(app * aqq))) return false;
  const double h = aqq - app, g2 = 2.0 * apq;
  const double r2 = fma(h, h, g2 * g2);
  double r, d, inv;
  if (r2 > 1.0e-280 && r2 < 1.0e280) {  // no denormal or overflow on the way
    r = r2 * rsqrt_nr(r2);
    d = fabs(h) + r;
    inv = rsqrt_nr(2.0 * r * d);
  } else {
    r = hypot(h, g2);
    d = fabs(h) + r;
    inv = 1.0 / (sqrt(2.0 * r) * sqrt(d));
  }
  c = d * inv;
  sn = (h >= 0.0 ? g2 : -g2) * inv;
  return true;
}

// One wavefront rotates the 16 x 16 subproblem of blocks (I, J) of G (ld ldg) in place
// and leaves the product of its rotations in R (16 x 16, ld kRs).  Index i < 8 of the
// subproblem is row I * 8 + i of G, index i >= 8 is row J * 8 + i - 8.
__device__ __forceinline__ bool jac_pair_pass(double* __restrict__ G, int ldg, int I, int J, double* __restrict__ R,
                              double2* __restrict__ cs, int kfirst, double tol2, int lane) {
  auto gi = [&](int i) { return i < 8 ? I * 8 + i : J * 8 + i - 8; };
  for (int e = lane; e < 256; e += 64) R[(e >> 4) * kRs + (e & 15)] = (e >> 4) == (e & 15) ? 1.0 : 0.0;
  wave_sync();
  bool any = false;
  const int P = lane >> 3, Q = lane & 7;
  for (int k = kfirst; k < 16; ++k) {
    const int hbit = 31 - __builtin_clz(k);
    const int lowm = (1 << hbit) - 1;
    // pair t of this pass: p has bit hbit clear, q = p xor k
    auto pair_p = [&](int t) { return ((t >> hbit) << (hbit + 1)) | (t & lowm); };
    int rot = 0;
    if (lane < 8) {
      const int p = pair_p(lane), q = p ^ k;
      const int gp = gi(p), gq = gi(q);
      double c, sn;
      rot = jac_rotation(G[gp * ldg + gp], G[gq * ldg + gq], G[gp * ldg + gq], tol2, c, sn) ? 1 : 0;
      cs[lane] = make_double2(c, sn);
    }
    wave_sync();
    if (__ballot(rot) == 0) continue;
    any = true;
    const double2 rp = cs[P], rq = cs[Q];
    const int pP = pair_p(P), qP = pP ^ k, pQ = pair_p(Q), qQ = pQ ^ k;
    // two-sided update of the 2 x 2 block (pair P rows, pair Q columns), P <= Q; the
    // transpose is written by the same lane
    if (P <= Q && (rp.y != 0.0 || rq.y != 0.0)) {
      const int a0 = gi(pP), a1 = gi(qP), b0 = gi(pQ), b1 = gi(qQ);
      const double g00 = G[a0 * ldg + b0], g01 = G[a0 * ldg + b1];
      const double g10 = G[a1 * ldg + b0], g11 = G[a1 * ldg + b1];
      const double r00 = rp.x * g00 - rp.y * g10, r01 = rp.x * g01 - rp.y * g11;
      const double r10 = rp.y * g00 + rp.x * g10, r11 = rp.y * g01 + rp.x * g11;
      double o00 = rq.x * r00 - rq.y * r01, o01 = rq.y * r00 + rq.x * r01;
      double o10 = rq.x * r10 - rq.y * r11, o11 = rq.y * r10 + rq.x * r11;
      if (P == Q) {  // the rotated pair itself (reached only when it rotated)
        o01 = 0.0;
        o10 = 0.0;
      }
      G[a0 * ldg + b0] = o00;
      G[a0 * ldg + b1] = o01;
      G[a1 * ldg + b0] = o10;
      G[a1 * ldg + b1] = o11;
      if (P != Q) {
        G[b0 * ldg + a0] = o00;
        G[b1 * ldg + a0] = o01;
        G[b0 * ldg + a1] = o10;
        G[b1 * ldg + a1] = o11;
      }
    }
    // R <- R J_Q on columns (pQ, qQ), rows P and P + 8
    if (rq.y != 0.0) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const int r = P + 8 * h;
        const double a = R[r * kRs + pQ], b = R[r * kRs + qQ];
        R[r * kRs + pQ] = rq.x * a - rq.y * b;
        R[r * kRs + qQ] = rq.y * a + rq.x * b;
      }
    }
    wave_sync();
  }
  return any;
}

// The cross pass (the pairs (i, 8 + (i xor kap)), kap = 0..7) of blocks (I, J) with
// the subproblem in registers.  For the current kap, lane L = 8 a + b holds the 2 x 2
// block of row pair (a, 8 + (a xor kap)) and column pair (b, 8 + (b xor kap)):
//   x = S[a][b], y = S[a][8 + (b ^ kap)], z = S[8 + (a ^ kap)][b], w = S[8 + (a ^ kap)][8 + (b ^ kap)]
// and the same entries of R, so a two-sided rotation step is local to the lane.  Pair
// a's rotation comes from lane 9 a (whose block is the pair's own 2 x 2 block) and is
// broadcast across lanes.  kap runs in Gray-code order; going from kap to kap ^ d moves
// y by lane xor d, z by 8 d and w by 9 d.  Same rotations as jac_pair_pass with
// k = 8 + kap, in another order.
__device__ __forceinline__ bool jac_cross_pass_reg(double* __restrict__ G, int ldg, int I, int J,
                                                   double* __restrict__ R, double tol2, int lane) {
  const int a = lane >> 3, b = lane & 7;
  const int gIa = I * 8 + a, gIb = I * 8 + b, gJa = J * 8 + a, gJb = J * 8 + b;
  double x = G[gIa * ldg + gIb], y = G[gIa * ldg + gJb];
  double z = G[gJa * ldg + gIb], w = G[gJa * ldg + gJb];
  double rx = a == b ? 1.0 : 0.0, ry = 0.0, rz = 0.0, rw = rx;
  bool any = false;
  int kap = 0;
#pragma unroll
  for (int st = 0; st < 8; ++st) {
    double c = 1.0, sn = 0.0;
    const bool rot = a == b && jac_rotation(x, w, y, tol2, c, sn);
    if (__ballot(rot) != 0) {
      any = true;
      const double ca = __shfl(c, 9 * a), sa = __shfl(sn, 9 * a);
      const double cb = __shfl(c, 9 * b), sb = __shfl(sn, 9 * b);
      const double r00 = ca * x - sa * z, r01 = ca * y - sa * w;
      const double r10 = sa * x + ca * z, r11 = sa * y + ca * w;
      x = cb * r00 - sb * r01;
      y = sb * r00 + cb * r01;
      z = cb * r10 - sb * r11;
      w = sb * r10 + cb * r11;
      if (rot) {  // the rotated pair's own off-diagonal entry
        y = 0.0;
        z = 0.0;
      }
      const double tx = cb * rx - sb * ry, ty = sb * rx + cb * ry;
      const double tz = cb * rz - sb * rw, tw = sb * rz + cb * rw;
      rx = tx;
      ry = ty;
      rz = tz;
      rw = tw;
    }
    if (st < 7) {
      const int d = (st & 1) ? ((st & 2) ? 4 : 2) : 1;  // Gray code: 1 2 1 4 1 2 1
      y = __shfl_xor(y, d);
      z = __shfl_xor(z, 8 * d);
      w = __shfl_xor(w, 9 * d);
      ry = __shfl_xor(ry, d);
      rz = __shfl_xor(rz, 8 * d);
      rw = __shfl_xor(rw, 9 * d);
      kap ^= d;
    }
  }
  // write back (kap = 4 now); G stays exactly symmetric: the I x I and J x J blocks
  // from the lanes with a <= b, the I x J block from y, each with its transpose
  const int bk = b ^ kap, ak = a ^ kap;
  if (a <= b) {
    G[gIa * ldg + gIb] = x;
    G[gIb * ldg + gIa] = x;
  }
  if (ak <= bk) {
    G[(J * 8 + ak) * ldg + J * 8 + bk] = w;
    G[(J * 8 + bk) * ldg + J * 8 + ak] = w;
  }
  G[gIa * ldg + J * 8 + bk] = y;
  G[(J * 8 + bk) * ldg + gIa] = y;
  R[a * kRs + b] = rx;
  R[a * kRs + 8 + bk] = ry;
  R[(8 + ak) * kRs + b] = rz;
  R[(8 + ak) * kRs + 8 + bk] = rw;
  return any;
}

// Blocked forward substitution with the lower factor L (LDS, ld ld, 1 / L_ii at column s
// of row i): X <- L^-1 X for the s x s right-hand side in B (element (r, j) at
// B[r * ld + j], or at B[j * ld + r] when kTrans).  Every thread of the workgroup calls it.
template <bool kTrans>
__device__ __forceinline__ void fwd_blocked(const double* __restrict__ L, double* __restrict__ B,
                                            int s, int ld, int tid, int nt) {
  auto at = [&](int r, int j) -> double& { return kTrans ? B[j * ld + r] : B[r * ld + j]; };
  for (int k0 = 0; k0 < s; k0 += kChol) {
    const int kb = min(kChol, s - k0);
    // diagonal block rows: column j solved by thread j
    for (int j = tid; j < s; j += nt) {
      double x[kChol];
#pragma unroll
      for (int r = 0; r < kChol; ++r) {
        if (r < kb) {
          double v = at(k0 + r, j);
#pragma unroll
          for (int l = 0; l < r; ++l) v -= L[(k0 + r) * ld + k0 + l] * x[l];
          x[r] = v * L[(k0 + r) * ld + s];
        }
      }
#pragma unroll
      for (int r = 0; r < kChol; ++r)
        if (r < kb) at(k0 + r, j) = x[r];
    }
    __syncthreads();
    // rows below: 4 x 4 tiles of (rows k0+kb.., all columns)
    const int rem = s - k0 - kb;
    if (rem > 0) {
      const int tr = (rem + 3) / 4, tc = (s + 3) / 4;
      for (int t = tid; t < tr * tc; t += nt) {
        const int i0 = k0 + kb + 4 * (t / tc), j0 = 4 * (t % tc);
        double acc[4][4] = {};
        int ia[4], jb[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          ia[u] = min(i0 + u, s - 1);  // clamped rows and columns are computed, not stored
          jb[u] = min(j0 + u, s - 1);
        }
#pragma unroll 2
        for (int l = 0; l < kb; ++l) {
          double a[4], b[4];
#pragma unroll
          for (int u = 0; u < 4; ++u) {
            a[u] = L[ia[u] * ld + k0 + l];
            b[u] = at(k0 + l, jb[u]);
          }
#pragma unroll
          for (int u = 0; u < 4; ++u)
#pragma unroll
            for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v)
            if (i0 + u < s && j0 + v < s) at(i0 + u, j0 + v) -= acc[u][v];
      }
    }
    __syncthreads();
  }
}

// Blocked right-looking Cholesky of the lower triangle of A (LDS, ld ld); writes 1 / L_ii
// at column s of row i.  Returns false (every thread) when a pivot is not positive and
// finite.
__device__ __forceinline__ bool chol_blocked(double* __restrict__ A, int s, int ld, int tid, int nt, int* s_flag) {
  const int wave = tid >> 6, lane = tid & 63;
  if (tid == 0) *s_flag = 0;
  __syncthreads();
  for (int k0 = 0; k0 < s; k0 += kChol) {
    const int kb = min(kChol, s - k0);
    if (wave == 0) {  // the diagonal block, unblocked, in one wavefront
      for (int kk = 0; kk < kb; ++kk) {
        const int c = k0 + kk;
        const double d = A[c * ld + c];
        if (!(d > 0.0) || !(d < 1.0e300)) {
          if (lane == 0) *s_flag = 1;
          break;
        }
        const double piv = sqrt(d), inv = 1.0 / piv;
        if (lane < kb - kk - 1) A[(c + 1 + lane) * ld + c] *= inv;
        if (lane == 0) {
          A[c * ld + c] = piv;
          A[c * ld + s] = inv;
        }
        wave_sync();
        const int rem = kb - kk - 1;
        for (int e = lane; e < rem * rem; e += 64) {
          const int a = e / rem, b = e - a * rem;
          if (b <= a) A[(c + 1 + a) * ld + c + 1 + b] -= A[(c + 1 + a) * ld + c] * A[(c + 1 + b) * ld + c];
        }
        wave_sync();
      }
    }
    __syncthreads();
    if (*s_flag) return false;
    const int rem = s - k0 - kb;
    if (rem == 0) break;
    // panel: row i of L21 solves x L11^T = a_i
    for (int t = tid; t < rem; t += nt) {
      const int i = k0 + kb + t;
      double x[kChol];
#pragma unroll
      for (int j = 0; j < kChol; ++j) {
        if (j < kb) {
          double v = A[i * ld + k0 + j];
#pragma unroll
          for (int l = 0; l < j; ++l) v -= x[l] * A[(k0 + j) * ld + k0 + l];
          x[j] = v * A[(k0 + j) * ld + s];
        }
      }
#pragma unroll
      for (int j = 0; j < kChol; ++j)
        if (j < kb) A[i * ld + k0 + j] = x[j];
    }
    __syncthreads();
    // trailing lower triangle -= L21 L21^T in 4 x 4 tiles
    const int nt4 = (rem + 3) / 4;
    for (int t = tid; t < nt4 * nt4; t += nt) {
      const int ti = t / nt4, tj = t - ti * nt4;
      if (tj > ti) continue;
      const int i0 = k0 + kb + 4 * ti, j0 = k0 + kb + 4 * tj;
      double acc[4][4] = {};
      int ia[4], jb[4];
#pragma unroll
      for (int u = 0; u < 4; ++u) {
        ia[u] = min(i0 + u, s - 1);  // clamped rows and columns are computed, not stored
        jb[u] = min(j0 + u, s - 1);
      }
#pragma unroll 2
      for (int l = 0; l < kb; ++l) {
        double a[4], b[4];
#pragma unroll
        for (int u = 0; u < 4; ++u) {
          a[u] = A[ia[u] * ld + k0 + l];
          b[u] = A[jb[u] * ld + k0 + l];
        }
#pragma unroll
        for (int u = 0; u < 4; ++u)
#pragma unroll
          for (int v = 0; v < 4; ++v) acc[u][v] = fma(a[u], b[v], acc[u][v]);
      }
#pragma unroll
      for (int u = 0; u < 4; ++u)
#pragma unroll
        for (int v = 0; v < 4; ++v)
          if (i0 + u < s && j0 + v <= i0 + u) A[(i0 + u) * ld + j0 + v] -= acc[u][v];
    }
    __syncthreads();
  }
  return true;
}

// Core scratch of problem b (core + b * 5 SP^2): C (SP x SP, row-major, zero above the
// diagonal) at 0, sigma^2 sorted descending at SP^2, their indices (as doubles) at
// SP^2 + SP, V (SJ x SJ, row-major, SJ = 16 ceil(s / 16) <= SP) at 2 SP^2, T (column j
// at 4 SP^2 + j SP) written by k_core_vt.
__global__ __launch_bounds__(kCoreThreads) void k_nystrom_core_lds(
    int s, double eps, double rel_floor, double jac_tol, const double* __restrict__ gram, int SPg,
    double* __restrict__ core,
    double* __restrict__ lamhat, int lam_stride, int32_t* __restrict__ s_eff_out,
    int32_t* __restrict__ status_out, double* __restrict__ shift_out) {
  extern __shared__ double lds[];
  __shared__ int16_t perm[kCoreLdsMaxS];
  __shared__ double evals[kCoreLdsMaxS];
  __shared__ double s_red;
  __shared__ double s_shift;
  __shared__ int s_flag;
  __shared__ int s_rot[2], s_bad[2];
  __shared__ int s_pair_rot[2][kJacMaxPairs];
  const int b = blockIdx.x, tid = threadIdx.x, nt = blockDim.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int LG = s + 1;
  double* R2 = lds;           // s x LG: M, then C (1 / C_ii at column s)
  double* R1 = lds + s * LG;  // s x LG: Q, X = C^-1 Q, G^T = C^-1 X^T
  const int sp2 = SPg * SPg;
  const double* G1 = gram + ((int64_t)b * 3 + 0) * sp2;
  const double* G2 = gram + ((int64_t)b * 3 + 1) * sp2;
  const double* G3 = gram + ((int64_t)b * 3 + 2) * sp2;
  double* Cg = core + (int64_t)b * 5 * sp2;
  double* lam_b = lamhat + (int64_t)b * lam_stride;

  if (wave == 0) {  // trace of Y^T Y: lane sums, then a fixed butterfly
    double tr = 0.0;
    for (int k = lane; k < s; k += 64) tr += G3[k * SPg + k];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) tr += __shfl_xor(tr, off);
    if (lane == 0) s_red = tr;
  }
  __syncthreads();
  const double trace3 = s_red;
  if (!(trace3 > 0.0) || !(trace3 < 1.0e300)) {
    for (int j = tid; j < s; j += nt) lam_b[j] = 0.0;
    if (tid == 0) {
      s_eff_out[b] = 0;
      status_out[b] = (trace3 == 0.0) ? 0 : GENIOS_WARN_PRECOND;
      shift_out[b] = 0.0;
    }
    return;
  }
  if (tid == 0) s_shift = eps * sqrt(trace3);
  __syncthreads();

  // ---- Cholesky of M = sym(Omega^T Y) + mu Omega^T Omega (retry with 10 mu) ----
  bool ok = false;
  for (int attempt = 0; attempt < 4 && !ok; ++attempt) {
    const double mu = s_shift;
    staged_for<4>(
        s * s, tid, nt,
        [&](int e) {
          const int i = e / s, j = e - i * s;
          return 0.5 * (G1[i * SPg + j] + G1[j * SPg + i]) + mu * G2[i * SPg + j];
        },
        [&](int e, double v) { R2[(e / s) * LG + e % s] = v; });
    __syncthreads();
    ok = chol_blocked(R2, s, LG, tid, nt, &s_flag);
    if (!ok) {
      __syncthreads();
      if (tid == 0) s_shift = 10.0 * s_shift;
      __syncthreads();
    }
  }
  if (!ok) {
    for (int j = tid; j < s; j += nt) lam_b[j] = 0.0;
    if (tid == 0) {
      s_eff_out[b] = 0;
      status_out[b] = GENIOS_WARN_PRECOND;
      shift_out[b] = s_shift;
    }
    return;
  }
  const double mu = s_shift;
  // C (lower, zero above) to global; Q = Y_mu^T Y_mu into R1
  for (int e = tid; e < s * s; e += nt) {
    const int i = e / s, j = e % s;
    Cg[i * SPg + j] = (j <= i) ? R2[i * LG + j] : 0.0;
  }
  staged_for<4>(
      s * s, tid, nt,
      [&](int e) {
        const int i = e / s, j = e - i * s;
        return G3[i * SPg + j] + mu * (G1[i * SPg + j] + G1[j * SPg + i]) + mu * mu * G2[i * SPg + j];
      },
      [&](int e, double v) { R1[(e / s) * LG + e % s] = v; });
  __syncthreads();
  fwd_blocked<false>(R2, R1, s, LG, tid, nt);  // X = C^-1 Q
  fwd_blocked<true>(R2, R1, s, LG, tid, nt);   // G = C^-1 X^T, stored transposed

  // ---- G (symmetrised, zero padded) into the Jacobi layout; V = I in global memory ----
  const int nbk = jac_blocks(s), SJ = 8 * nbk, npair = nbk / 2;
  const int LDJ = SJ + 1;
  double* GJ = lds;                                // SJ x LDJ
  double* Rb = GJ + SJ * LDJ;                      // two rounds of npair blocks 16 x kRs
  double2* csb = reinterpret_cast<double2*>(Rb + 2 * kJacMaxPairs * 16 * kRs);  // 8 per pair
  double* Vg = Cg + 2 * sp2;                       // SJ x SJ, row-major
  {
    constexpr int kPer = (kJacMaxN * kJacMaxN + kCoreThreads - 1) / kCoreThreads;
    double g[kPer];
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = tid + u * nt;
      const int i = e / SJ, j = e - i * SJ;
      g[u] = (e < SJ * SJ && i < s && j < s) ? 0.5 * (R1[i * LG + j] + R1[j * LG + i]) : 0.0;
      if (e < SJ * SJ) Vg[e] = i == j ? 1.0 : 0.0;
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < kPer; ++u) {
      const int e = tid + u * nt;
      const int i = e / SJ, j = e - i * SJ;
      if (e < SJ * SJ) GJ[i * LDJ + j] = g[u];
    }
  }
  if (tid == 0) {
    s_rot[0] = 0;
    s_bad[0] = 0;
  }
  __syncthreads();

  // V[:, pair p] <- V[:, pair p] R_p on the matrix cores, for pair p of circle round rr
  // (block in Rpar): the SJ rows in kT = SJ / 16 tiles of 16.  Fully unrolled with the
  // loads two tiles ahead of the products (a ring of three tiles in registers), so that
  // each product waits for its own loads only and few registers are live.
  const int li = lane & 15, lk = lane >> 4;
  auto v_update_pair = [&](auto kTc, int rr, const double* Rpar, int p) __attribute__((always_inline)) {
    constexpr int kT = decltype(kTc)::value;
    const int2 IJ = circle_pair(nbk, rr, p);
    const double* R = Rpar + p * 16 * kRs;
    const uint32_t tstep = 16u * (uint32_t)SJ;  // a tile is 16 SJ elements further
    uint32_t lo[4];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) {
      const int c = 4 * ks + lk;
      lo[ks] = (uint32_t)(li * SJ + (c < 8 ? IJ.x * 8 + c : IJ.y * 8 + c - 8));
    }
    const uint32_t so = (uint32_t)(lk * SJ + (li < 8 ? IJ.x * 8 + li : IJ.y * 8 + li - 8));
    double rb[4];
#pragma unroll
    for (int ks = 0; ks < 4; ++ks) rb[ks] = R[(4 * ks + lk) * kRs + li];
    double av[3][4];
    auto load = [&](int t) __attribute__((always_inline)) {
#pragma unroll
      for (int ks = 0; ks < 4; ++ks) av[t % 3][ks] = Vg[lo[ks] + t * tstep];
    };
    load(0);
    if (kT > 1) load(1);
#pragma unroll
    for (int t = 0; t < kT; ++t) {
      if (t + 2 < kT) load(t + 2);
      v4d d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
      for (int ks = 0; ks < 4; ++ks)
        d = __builtin_amdgcn_mfma_f64_16x16x4f64(av[t % 3][ks], rb[ks], d, 0, 0, 0);
#pragma unroll
      for (int v = 0; v < 4; ++v) Vg[so + t * tstep + 4u * v * (uint32_t)SJ] = d[v];
    }
  };
  auto v_update = [&](int rr, const double* Rpar, int p) __attribute__((always_inline)) {
    switch (npair) {  // SJ / 16 tiles = npair
      case 1: v_update_pair(std::integral_constant<int, 1>{}, rr, Rpar, p); break;
      case 2: v_update_pair(std::integral_constant<int, 2>{}, rr, Rpar, p); break;
      case 3: v_update_pair(std::integral_constant<int, 3>{}, rr, Rpar, p); break;
      case 4: v_update_pair(std::integral_constant<int, 4>{}, rr, Rpar, p); break;
      case 5: v_update_pair(std::integral_constant<int, 5>{}, rr, Rpar, p); break;
      case 6: v_update_pair(std::integral_constant<int, 6>{}, rr, Rpar, p); break;
      default: v_update_pair(std::integral_constant<int, 7>{}, rr, Rpar, p); break;
    }
  };

  // ---- block Jacobi ----
  const double tol2 = jac_tol * jac_tol;
  int round = 0, prev_r = -1;
  for (int sweep = 0; sweep < kJacMaxSweeps; ++sweep) {
    for (int r = 0; r < nbk - 1; ++r, ++round) {
      const int par = round & 1;
      double* Rcur = Rb + par * kJacMaxPairs * 16 * kRs;
      if (wave < npair) {  // inner passes, one wavefront per block pair
        const int2 IJ = circle_pair(nbk, r, wave);
        double* R = Rcur + wave * 16 * kRs;
        const bool any = r == 0 ? jac_pair_pass(GJ, LDJ, IJ.x, IJ.y, R, csb + wave * 8, 1, tol2, lane)
                                : jac_cross_pass_reg(GJ, LDJ, IJ.x, IJ.y, R, tol2, lane);
        if (lane == 0) {
          s_pair_rot[par][wave] = any ? 1 : 0;
          if (any) s_rot[sweep & 1] = 1;
        }
      } else if (prev_r >= 0 && wave < 2 * npair && s_pair_rot[1 - par][wave - npair]) {
        // the previous round's V update meanwhile, one wavefront per rotated pair
        v_update(prev_r, Rb + (1 - par) * kJacMaxPairs * 16 * kRs, wave - npair);
      }
      __syncthreads();  // also orders the V stores before the next round's V loads
      if (r == 0 && tid == 0) {
        s_rot[(sweep + 1) & 1] = 0;
        s_bad[(sweep + 1) & 1] = 0;
      }
      // G[A, B] <- R_A^T G[A, B] R_B for the block pairs A < B (and the transpose), on
      // the FP64 matrix cores: v_mfma_f64_16x16x4 reads A[i][k] from lane 16 k + i and
      // B[k][j] from lane 16 k + j, and leaves D[4 v + L / 16][L % 16] in register v of
      // lane L.  With R_B, the first product is T^T = G[B, A] R_A, whose result layout is
      // the A-operand layout of T in the second product O = T R_B.
      const int* rot = s_pair_rot[par];
      const int nunit = npair * (npair - 1) / 2;
      for (int u = wave; u < nunit; u += kCoreWaves) {
        int A = 0, rest = u;
        while (rest >= npair - 1 - A) {
          rest -= npair - 1 - A;
          ++A;
        }
        const int B = A + 1 + rest;
        const bool ra = rot[A] != 0, rb = rot[B] != 0;
        if (!ra && !rb) continue;
        const int2 pa = circle_pair(nbk, r, A), pb = circle_pair(nbk, r, B);
        auto ga = [&](int i) { return i < 8 ? pa.x * 8 + i : pa.y * 8 + i - 8; };
        auto gb = [&](int i) { return i < 8 ? pb.x * 8 + i : pb.y * 8 + i - 8; };
        const double* RA = Rcur + A * 16 * kRs;
        const double* RB = Rcur + B * 16 * kRs;
        v4d o = {0.0, 0.0, 0.0, 0.0};
        if (rb) {
          double ta[4];  // A operand of T: T[li][4 ks + lk]
          if (ra) {
            v4d tt = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) {
              const int k = 4 * ks + lk;
              tt = __builtin_amdgcn_mfma_f64_16x16x4f64(GJ[gb(li) * LDJ + ga(k)],
                                                         RA[k * kRs + li], tt, 0, 0, 0);
            }
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) ta[ks] = tt[ks];
          } else {
#pragma unroll
            for (int ks = 0; ks < 4; ++ks) ta[ks] = GJ[ga(li) * LDJ + gb(4 * ks + lk)];
          }
#pragma unroll
          for (int ks = 0; ks < 4; ++ks)
            o = __builtin_amdgcn_mfma_f64_16x16x4f64(ta[ks], RB[(4 * ks + lk) * kRs + li], o, 0,
                                                      0, 0);
        } else {  // O = R_A^T G[A, B]
#pragma unroll
          for (int ks = 0; ks < 4; ++ks) {
            const int k = 4 * ks + lk;
            o = __builtin_amdgcn_mfma_f64_16x16x4f64(RA[k * kRs + li], GJ[ga(k) * LDJ + gb(li)], o,
                                                      0, 0, 0);
          }
        }
        // every lane's reads of G[A, B] and G[B, A] are done before any lane writes
        wave_sync();
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          GJ[ga(4 * v + lk) * LDJ + gb(li)] = o[v];
          GJ[gb(li) * LDJ + ga(4 * v + lk)] = o[v];
        }
      }
      prev_r = r;
      lds_barrier();
    }
    // converged when no pair rotated in the sweep, or every off-diagonal entry now
    // meets the threshold
    for (int e = tid; e < s * s; e += nt) {
      const int i = e / s, j = e - i * s;
      if (i < j) {
        const double g = GJ[i * LDJ + j];
        if (g * g > tol2 * fabs(GJ[i * LDJ + i] * GJ[j * LDJ + j])) s_bad[sweep & 1] = 1;
      }
    }
    lds_barrier();
    if (s_rot[sweep & 1] == 0 || s_bad[sweep & 1] == 0) break;
  }
  // the last round's V update
  if (prev_r >= 0 && wave < npair && s_pair_rot[(round - 1) & 1][wave])
    v_update(prev_r, Rb + ((round - 1) & 1) * kJacMaxPairs * 16 * kRs, wave);

  // ---- eigenvalues sorted descending: rank of g_jj under (value desc, index asc), NaN
  // as -inf, a total order, so perm is a permutation ----
  for (int j = tid; j < s; j += nt) {
    const double vj = GJ[j * LDJ + j];
    const double kj = vj == vj ? vj : -INFINITY;
    int rank = 0;
    for (int i = 0; i < s; ++i) {
      const double vi = GJ[i * LDJ + i];
      const double ki = vi == vi ? vi : -INFINITY;
      rank += (ki > kj || (ki == kj && i < j)) ? 1 : 0;
    }
    perm[rank] = (int16_t)j;
    evals[rank] = vj;
  }
  __syncthreads();
  if (tid == 0) {
    const double top = evals[0] - mu;
    int keep = 0;
    for (int j = 0; j < s; ++j) {
      if (top > 0.0 && evals[j] - mu > rel_floor * top)
        keep = j + 1;
      else
        break;
    }
    s_flag = keep;
  }
  __syncthreads();
  const int keep = s_flag;
  for (int j = tid; j < s; j += nt) {
    lam_b[j] = (j < keep) ? fmax(evals[j] - mu, 0.0) : 0.0;
    Cg[sp2 + j] = evals[j];
    Cg[sp2 + SPg + j] = (double)perm[j];
  }
  if (tid == 0) {
    s_eff_out[b] = keep;
    status_out[b] = 0;
    shift_out[b] = mu;
  }
}

// T(:, j) = C^-T V(:, perm[j]) / sigma_j for j < keep, zero for the other columns.  A
// workgroup takes 16 columns and solves C^T t = v by right-looking back substitution
// with C in LDS, two columns per wavefront, the rows of a column over 32 lanes.
constexpr int kVtCols = 16;
constexpr int kVtThreads = 512;
static_assert(kVtThreads / 64 * 2 == kVtCols, "two columns per wavefront");
__global__ __launch_bounds__(kVtThreads) void k_core_vt(int s, int SPg, double* __restrict__ core,
                                                        const int32_t* __restrict__ s_eff) {
  extern __shared__ double vl[];
  const int b = blockIdx.y, tid = threadIdx.x, nt = blockDim.x;
  const int wave = tid >> 6, lane = tid & 63;
  const int sp2 = SPg * SPg;
  double* Cg = core + (int64_t)b * 5 * sp2;
  const double* Vg = Cg + 2 * sp2;
  double* Tg = Cg + 4 * sp2;
  const int keep = s_eff[b];
  const int c0 = blockIdx.x * kVtCols;
  if (c0 >= keep) {
    for (int e = tid; e < kVtCols * SPg; e += nt) {
      const int col = c0 + e / SPg;
      if (col < SPg) Tg[(int64_t)col * SPg + e % SPg] = 0.0;
    }
    return;
  }
  const int SJ = 8 * jac_blocks(s);
  const int LC = s + 1;
  double* Vt = vl;                        // s x kVtCols
  double* Cl = vl + kCoreLdsMaxS * kVtCols;  // s x LC, 1 / C_ii at column s
  __shared__ int s_perm[kVtCols];
  if (tid < kVtCols) s_perm[tid] = c0 + tid < keep ? (int)Cg[sp2 + SPg + c0 + tid] : -1;
  __syncthreads();
  staged_for<4>(
      s * kVtCols, tid, nt,
      [&](int e) {
        const int q = s_perm[e % kVtCols];
        return q >= 0 ? Vg[(e / kVtCols) * SJ + q] : 0.0;
      },
      [&](int e, double v) { Vt[e] = v; });
  staged_for<8>(
      s * s, tid, nt, [&](int e) { return Cg[(e / s) * SPg + e % s]; },
      [&](int e, double v) {
        const int i = e / s, j = e - i * s;
        Cl[i * LC + j] = j <= i ? v : 0.0;
        if (j == i) Cl[i * LC + s] = 1.0 / v;
      });
  __syncthreads();
  {
    const int c = 2 * wave + (lane >> 5), g = lane & 31;
    for (int i = s - 1; i >= 0; --i) {
      const double ti = Vt[i * kVtCols + c] * Cl[i * LC + s];
      wave_sync();
      if (g == 0) Vt[i * kVtCols + c] = ti;
      for (int l = g; l < i; l += 32) Vt[l * kVtCols + c] -= Cl[i * LC + l] * ti;
      wave_sync();
    }
  }
  __syncthreads();
  for (int e = tid; e < kVtCols * SPg; e += nt) {
    const int cc = e / SPg, i = e - cc * SPg, col = c0 + cc;
    if (col >= SPg) continue;
    double v = 0.0;
    if (col < keep && i < s) v = Vt[i * kVtCols + cc] / sqrt(Cg[sp2 + col]);
    Tg[(int64_t)col * SPg + i] = v;
  }
}

}  // namespace

size_t core_lds_bytes(int s) {
  const int nbk = jac_blocks(s), SJ = 8 * nbk;
  const size_t pre = (size_t)2 * s * (s + 1);
  const size_t jac = (size_t)SJ * (SJ + 1) + (size_t)2 * kJacMaxPairs * 16 * kRs +
                     (size_t)kJacMaxPairs * 8 * 2;
  return std::max(pre, jac) * sizeof(double);
}

hipError_t launch_nystrom_core_lds(int64_t batch, int s, int SPg, double eps, double rel_floor,
                                   double jac_tol, const double* gram, double* core,
                                   double* lamhat, int32_t* s_eff, int32_t* status, double* shift,
                                   hipStream_t st) {
  if (s < 1 || s > kCoreLdsMaxS || 8 * jac_blocks(s) > SPg) return hipErrorInvalidValue;
  const size_t lds = core_lds_bytes(s);
  hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_nystrom_core_lds),
                                     hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_nystrom_core_lds, dim3((unsigned)batch), dim3(kCoreThreads), lds, st, s,
                     eps, rel_floor, jac_tol, gram, SPg, core, lamhat, s, s_eff, status, shift);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  const size_t lds2 = ((size_t)kCoreLdsMaxS * kVtCols + (size_t)s * (s + 1)) * sizeof(double);
  e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_core_vt),
                          hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds2);
  if (e != hipSuccess) return e;
  dim3 grid((unsigned)((SPg + kVtCols - 1) / kVtCols), (unsigned)batch);
  hipLaunchKernelGGL(k_core_vt, grid, dim3(kVtThreads), lds2, st, s, SPg, core, s_eff);
  return hipGetLastError();
}

}  // namespace genios
