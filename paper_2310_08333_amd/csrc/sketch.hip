// Randomized Nystrom approximation of H = A^T diag(d) A (Sec. 2.2).
//
//   1. Omega (n x s) standard normal: Philox4x64-10 counters + Box-Muller.
//   2. W = A Omega            (m x s)   tiled GEMM, split over n
//   3. Y = A^T (d o W)        (n x s)   tiled GEMM, split over m      => Y = H Omega
//   4. FP64 Grams  Omega^T Y, Omega^T Omega, Y^T Y (s x s)
//   5. s x s core in one workgroup (FP64): with the stabilising shift
//      mu = eps ||Y||_F and Y_mu = Y + mu Omega (the published shift
//      sqrt(n) eps ||Y|| of the stabilised Nystrom method assumes an
//      orthonormal test matrix; a Gaussian Omega with the same range has
//      columns of norm ~sqrt(n), and the equivalent shift is eps ||Y||_F),
//        M = Omega^T Y_mu = C C^T (Cholesky; shift x10 on failure, <= 3 times),
//        G = C^-1 (Y_mu^T Y_mu) C^-T = V Sigma^2 V^T (block Jacobi in core.hip for
//        s <= 100, cyclic Jacobi below for larger s),
//        lambda_hat = max(Sigma^2 - mu, 0), T = C^-T V Sigma^-1,
//      so that B = Y_mu C^-T = U Sigma V^T and H_hat = Y_mu M^-1 Y_mu^T = B B^T.
//   6. U = Y_mu T             (n x s)   orthonormal columns.
// Steps 2-3 stream A twice, the cost the paper quotes for the sketch
// ("about a matrix-vector product with A" per column block).
#include <algorithm>
#include <type_traits>
#include <cmath>

#include "device.hpp"

namespace genios {

namespace {

// ---- Philox4x64-10 and Box-Muller ---------------------------------------------

__device__ __forceinline__ void philox4x64_10(uint64_t (&c)[4], uint64_t k0, uint64_t k1) {
  const uint64_t M0 = 0xD2E7470EE14C6C93ull, M1 = 0xCA5A826395121157ull;
  const uint64_t W0 = 0x9E3779B97F4A7C15ull, W1 = 0xBB67AE8584CAA73Bull;
#pragma unroll
  for (int r = 0; r < 10; ++r) {
    const uint64_t lo0 = M0 * c[0], hi0 = __umul64hi(M0, c[0]);
    const uint64_t lo1 = M1 * c[2], hi1 = __umul64hi(M1, c[2]);
    const uint64_t n0 = hi1 ^ c[1] ^ k0, n1 = lo1, n2 = hi0 ^ c[3] ^ k1, n3 = lo0;
    c[0] = n0;
    c[1] = n1;
    c[2] = n2;
    c[3] = n3;
    k0 += W0;
    k1 += W1;
  }
}

__device__ __forceinline__ void box_muller(uint64_t a, uint64_t b, double& z0, double& z1) {
  const double u1 = ((double)(a >> 11) + 0.5) * 0x1p-53;
  const double u2 = (double)(b >> 11) * 0x1p-53;
  const double r = sqrt(-2.0 * log(u1));
  const double t = 2.0 * M_PI * u2;
  z0 = r * cos(t);
  z1 = r * sin(t);
}

// out[b] is n x ld (column-major, ld columns >= s); element e = j n + i of the
// first s columns comes from block e/4, lane e%4, key (seed, stream_id + b).
template <typename VT>
__global__ __launch_bounds__(256) void k_gaussian(int64_t n, int s, int ld_cols, uint64_t seed,
                                                  uint64_t stream_id,
                                                  const uint8_t* __restrict__ mask,
                                                  VT* __restrict__ out) {
  const int b = blockIdx.y;
  const int64_t total = n * (int64_t)s;
  const int64_t nblk = (total + 3) / 4;
  VT* ob = out + (int64_t)b * n * ld_cols;
  for (int64_t c = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; c < nblk;
       c += (int64_t)gridDim.x * blockDim.x) {
    uint64_t ctr[4] = {(uint64_t)c, 0ull, 0ull, 0ull};
    philox4x64_10(ctr, seed, stream_id + (uint64_t)b);
    double z[4];
    box_muller(ctr[0], ctr[1], z[0], z[1]);
    box_muller(ctr[2], ctr[3], z[2], z[3]);
#pragma unroll
    for (int l = 0; l < 4; ++l) {
      const int64_t e = 4 * c + l;
      if (e < total) {
        const int64_t j = e / n, i = e - j * n;
        const bool keep = mask == nullptr || mask[(int64_t)b * n + i] != 0;
        ob[j * n + i] = keep ? VT((float)z[l]) : VT(0);
      }
    }
  }
}

template <typename VT>
__global__ __launch_bounds__(256) void k_copy_omega(int64_t n, int s, int ld_cols,
                                                    const VT* __restrict__ in,
                                                    const uint8_t* __restrict__ mask,
                                                    VT* __restrict__ out) {
  const int b = blockIdx.y;
  const int64_t total = n * (int64_t)s;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t j = e / n, i = e - j * n;
    const bool keep = mask == nullptr || mask[(int64_t)b * n + i] != 0;
    out[(int64_t)b * n * ld_cols + j * n + i] = keep ? in[(int64_t)b * n * s + e] : VT(0);
  }
}

// ---- skinny GEMMs ----------------------------------------------------------------
// Output tile 64 x SP per block, K chunks of 32, 256 threads, each thread 4 x SP/16.

constexpr int kBM = 64;
constexpr int kBK = 32;

template <typename Acc, int SP>
__device__ __forceinline__ void micro_tile(const Acc (*As)[kBM + 4], const Acc (*Bs)[SP + 4],
                                           Acc (&acc)[4][SP / 16], int tr, int tc) {
  constexpr int CT = SP / 16;
#pragma unroll 4
  for (int kk = 0; kk < kBK; ++kk) {
    Acc a[4], bb[CT];
#pragma unroll
    for (int i = 0; i < 4; ++i) a[i] = As[kk][tr * 4 + i];
#pragma unroll
    for (int j = 0; j < CT; ++j) bb[j] = Bs[kk][tc * CT + j];
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < CT; ++j) acc[i][j] += a[i] * bb[j];
  }
}

// Wpart[b][ks] (m x SP, col-major) = A[:, k-range] Omega[k-range, :]
template <typename T, typename VT, int SP>
__global__ __launch_bounds__(256) void k_sketch_w(const T* __restrict__ A, int64_t lda,
                                                  int64_t strideA, int m, int n,
                                                  const VT* __restrict__ omega,
                                                  VT* __restrict__ wpart, int kchunk,
                                                  int64_t wpart_ks_stride,
                                                  int64_t wpart_prob_stride) {
  using Acc = typename Elem<T>::Acc;
  constexpr int CT = SP / 16;
  __shared__ Acc As[kBK][kBM + 4];
  __shared__ Acc Bs[kBK][SP + 4];
  const int b = blockIdx.z, ks = blockIdx.y;
  const int row0 = blockIdx.x * kBM;
  const int k0 = ks * kchunk, k1 = min(n, k0 + kchunk);
  const T* Ab = A + (int64_t)b * strideA;
  const VT* Ob = omega + (int64_t)b * n * SP;
  const int tid = threadIdx.x, tr = tid % 16, tc = tid / 16;
  Acc acc[4][CT];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < CT; ++j) acc[i][j] = Acc(0);
  const int lr = tid / 4, lk = (tid % 4) * 8;  // A tile load: one row, 8 consecutive k
  for (int kb = k0; kb < k1; kb += kBK) {
    {
      const int row = row0 + lr;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int k = kb + lk + q;
        As[lk + q][lr] = (row < m && k < k1) ? Acc(Elem<T>::cvt(Ab[(int64_t)row * lda + k])) : Acc(0);
      }
    }
    for (int e = tid; e < kBK * SP; e += 256) {
      const int j = e / kBK, kk = e % kBK;
      const int k = kb + kk;
      Bs[kk][j] = (k < k1) ? Acc(Ob[(int64_t)j * n + k]) : Acc(0);
    }
    __syncthreads();
    micro_tile<Acc, SP>(As, Bs, acc, tr, tc);
    __syncthreads();
  }
  VT* Wb = wpart + (int64_t)b * wpart_prob_stride + (int64_t)ks * wpart_ks_stride;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int row = row0 + tr * 4 + i;
    if (row < m)
#pragma unroll
      for (int j = 0; j < CT; ++j) Wb[(int64_t)(tc * CT + j) * m + row] = VT(acc[i][j]);
  }
}

// Ypart[b][ks] (n x SP) = A[r-range, :]^T (d o W)[r-range, :]
template <typename T, typename VT, int SP>
__global__ __launch_bounds__(256) void k_sketch_y(const T* __restrict__ A, int64_t lda,
                                                  int64_t strideA, int m, int n,
                                                  const VT* __restrict__ W,
                                                  const VT* __restrict__ d, int64_t d_stride,
                                                  VT* __restrict__ ypart, int rchunk,
                                                  int64_t ypart_ks_stride,
                                                  int64_t ypart_prob_stride) {
  using Acc = typename Elem<T>::Acc;
  constexpr int CT = SP / 16;
  __shared__ Acc As[kBK][kBM + 4];
  __shared__ Acc Bs[kBK][SP + 4];
  const int b = blockIdx.z, ks = blockIdx.y;
  const int col0 = blockIdx.x * kBM;
  const int r0 = ks * rchunk, r1 = min(m, r0 + rchunk);
  const T* Ab = A + (int64_t)b * strideA;
  const VT* Wb = W + (int64_t)b * m * SP;
  const VT* db = d ? d + (int64_t)b * d_stride : nullptr;
  const int tid = threadIdx.x, tr = tid % 16, tc = tid / 16;
  Acc acc[4][CT];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < CT; ++j) acc[i][j] = Acc(0);
  const int lr = tid / 8, lc = (tid % 8) * 8;  // A tile load: one row, 8 consecutive columns
  for (int rb = r0; rb < r1; rb += kBK) {
    {
      const int r = rb + lr;
#pragma unroll
      for (int q = 0; q < 8; ++q) {
        const int c = col0 + lc + q;
        As[lr][lc + q] = (r < r1 && c < n) ? Acc(Elem<T>::cvt(Ab[(int64_t)r * lda + c])) : Acc(0);
      }
    }
    for (int e = tid; e < kBK * SP; e += 256) {
      const int j = e / kBK, kk = e % kBK;
      const int r = rb + kk;
      Acc v = Acc(0);
      if (r < r1) {
        v = Acc(Wb[(int64_t)j * m + r]);
        if (db) v *= Acc(db[r]);
      }
      Bs[kk][j] = v;
    }
    __syncthreads();
    micro_tile<Acc, SP>(As, Bs, acc, tr, tc);
    __syncthreads();
  }
  VT* Yb = ypart + (int64_t)b * ypart_prob_stride + (int64_t)ks * ypart_ks_stride;
#pragma unroll
  for (int i = 0; i < 4; ++i) {
    const int c = col0 + tr * 4 + i;
    if (c < n)
#pragma unroll
      for (int j = 0; j < CT; ++j) Yb[(int64_t)(tc * CT + j) * n + c] = VT(acc[i][j]);
  }
}

// ---- Grams ----------------------------------------------------------------------
// Y = sum of the split partials, rows outside the mask zero.
template <typename VT, int SP>
__global__ __launch_bounds__(256) void k_y_sum(int64_t n, const VT* __restrict__ ypart, int ksY,
                                               int64_t ks_stride, int64_t prob_stride,
                                               const uint8_t* __restrict__ mask,
                                               VT* __restrict__ Y) {
  const int b = blockIdx.y;
  const VT* Yp = ypart + (int64_t)b * prob_stride;
  const uint8_t* mb = mask ? mask + (int64_t)b * n : nullptr;
  VT* Yb = Y + (int64_t)b * n * SP;
  const int64_t total = n * SP;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    VT acc = VT(0);
    for (int k = 0; k < ksY; ++k) acc += Yp[(int64_t)k * ks_stride + e];
    if (mb && !mb[e % n]) acc = VT(0);
    Yb[e] = acc;
  }
}

// which = 0: Omega^T Y, 1: Omega^T Omega, 2: Y^T Y (FP64 accumulation); block g
// covers a row range.  Tiles of RT rows x SP columns are staged in LDS as
// doubles; the loads of the next tile are issued before the current tile is
// used (unconditional, rows clamped, values past the range or past s zeroed).
template <typename VT, int SP>
__global__ __launch_bounds__(256) void k_gram(int64_t n, int s, const VT* __restrict__ omega,
                                              const VT* __restrict__ Y,
                                              double* __restrict__ gpart, int nbG) {
  constexpr int SB = SP / 16;
  constexpr int RT = 16;              // rows per LDS tile
  constexpr int LP = SP + 2;          // LDS pitch in doubles (rows 16-byte aligned)
  constexpr int EPT = RT * SP / 256;  // staged elements per thread per matrix
  __shared__ __align__(16) double L1[RT][LP];
  __shared__ __align__(16) double L2[RT][LP];
  const int b = blockIdx.z, which = blockIdx.y, g = blockIdx.x;
  const int64_t rows_per = (n + nbG - 1) / nbG;
  const int64_t lo = min(n, (int64_t)g * rows_per), hi = min(n, lo + rows_per);
  const VT* M1 = (which == 2 ? Y : omega) + (int64_t)b * n * SP;
  const VT* M2 = (which == 1 ? omega : Y) + (int64_t)b * n * SP;
  const bool same = which != 0;
  const int tid = threadIdx.x, ti = tid % 16, tj = tid / 16;
  double acc[SB][SB];
#pragma unroll
  for (int i = 0; i < SB; ++i)
#pragma unroll
    for (int j = 0; j < SB; ++j) acc[i][j] = 0.0;
  VT r1[EPT], r2[EPT];
  auto load = [&](int64_t r0) {
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int e = tid + 256 * q, c = e / RT, rr = e % RT;
      const int64_t r = min(r0 + rr, hi - 1);
      r1[q] = M1[(int64_t)c * n + r];
      r2[q] = same ? r1[q] : M2[(int64_t)c * n + r];
    }
  };
  if (lo < hi) load(lo);
  for (int64_t r0 = lo; r0 < hi; r0 += RT) {
#pragma unroll
    for (int q = 0; q < EPT; ++q) {
      const int e = tid + 256 * q, c = e / RT, rr = e % RT;
      const bool ok = r0 + rr < hi && c < s;
      L1[rr][c] = ok ? double(r1[q]) : 0.0;
      L2[rr][c] = ok ? double(r2[q]) : 0.0;
    }
    __syncthreads();
    if (r0 + RT < hi) load(r0 + RT);
#pragma unroll 2
    for (int rr = 0; rr < RT; ++rr) {
      double a[SB], bb[SB];
#pragma unroll
      for (int i = 0; i < SB; ++i) a[i] = L1[rr][ti * SB + i];
#pragma unroll
      for (int j = 0; j < SB; ++j) bb[j] = L2[rr][tj * SB + j];
#pragma unroll
      for (int i = 0; i < SB; ++i)
#pragma unroll
        for (int j = 0; j < SB; ++j) acc[i][j] += a[i] * bb[j];
    }
    __syncthreads();
  }
  double* gp = gpart + (((int64_t)b * 3 + which) * nbG + g) * SP * SP;
#pragma unroll
  for (int i = 0; i < SB; ++i)
#pragma unroll
    for (int j = 0; j < SB; ++j) gp[(int64_t)(ti * SB + i) * SP + tj * SB + j] = acc[i][j];
}

__global__ __launch_bounds__(256) void k_gram_reduce(int sp2, const double* __restrict__ gpart,
                                                     int nbG, double* __restrict__ gram) {
  const int b = blockIdx.z, which = blockIdx.y;
  const double* gp = gpart + ((int64_t)b * 3 + which) * nbG * sp2;
  double* out = gram + ((int64_t)b * 3 + which) * sp2;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < sp2; e += gridDim.x * blockDim.x) {
    double s = 0.0;
    for (int g = 0; g < nbG; ++g) s += gp[(int64_t)g * sp2 + e];
    out[e] = s;
  }
}

// ---- s x s core -------------------------------------------------------------------
// Scratch per problem (doubles, each SP*SP): C (lower), X, G, V, T.

template <int SP>
__global__ __launch_bounds__(256) void k_nystrom_core(int s, int64_t n, double eps,
                                                      double rel_floor,
                                                      const double* __restrict__ gram,
                                                      double* __restrict__ core,
                                                      double* __restrict__ lamhat, int lam_stride,
                                                      int32_t* __restrict__ s_eff_out,
                                                      int32_t* __restrict__ status_out,
                                                      double* __restrict__ shift_out) {
  constexpr int LD = SP + 1;
  extern __shared__ double lds[];  // SP * LD doubles
  __shared__ int s_fail;
  __shared__ double s_shift;
  __shared__ double s_red[4];
  __shared__ int perm[SP];
  __shared__ double evals[SP];
  __shared__ double cs_c[SP / 2], cs_s[SP / 2];
  __shared__ int pr_p[SP / 2], pr_q[SP / 2];
  const int b = blockIdx.x;
  const int tid = threadIdx.x, nt = blockDim.x;
  const int sp2 = SP * SP;
  const double* G1 = gram + ((int64_t)b * 3 + 0) * sp2;
  const double* G2 = gram + ((int64_t)b * 3 + 1) * sp2;
  const double* G3 = gram + ((int64_t)b * 3 + 2) * sp2;
  double* Cg = core + (int64_t)b * 5 * sp2;
  double* Xg = Cg + sp2;
  double* Gg = Xg + sp2;
  double* Vg = Gg + sp2;
  double* Tg = Vg + sp2;
  double* lam_b = lamhat + (int64_t)b * lam_stride;
  double* M = lds;

  // ||Y||_F^2 = trace(Y^T Y)
  if (tid == 0) {
    double tr = 0.0;
    for (int k = 0; k < s; ++k) tr += G3[k * SP + k];
    s_red[0] = tr;
  }
  __syncthreads();
  const double trace3 = s_red[0];
  if (!(trace3 > 0.0) || !(trace3 < 1.0e300)) {
    // H Omega = 0 (H = 0 on the sketch) or non-finite: identity preconditioner.
    for (int j = tid; j < s; j += nt) lam_b[j] = 0.0;
    if (tid == 0) {
      s_eff_out[b] = 0;
      status_out[b] = (trace3 == 0.0) ? 0 : GENIOS_WARN_PRECOND;
      shift_out[b] = 0.0;
    }
    return;
  }
  if (tid == 0) s_shift = eps * sqrt(trace3);
  (void)n;
  __syncthreads();

  bool ok = false;
  for (int attempt = 0; attempt < 4 && !ok; ++attempt) {
    const double mu = s_shift;
    for (int e = tid; e < s * s; e += nt) {
      const int i = e / s, j = e % s;
      M[i * LD + j] = 0.5 * (G1[i * SP + j] + G1[j * SP + i]) + mu * G2[i * SP + j];
    }
    if (tid == 0) s_fail = 0;
    __syncthreads();
    for (int k = 0; k < s; ++k) {
      if (tid == 0) {
        const double dkk = M[k * LD + k];
        if (!(dkk > 0.0) || !(dkk < 1.0e300))
          s_fail = 1;
        else
          M[k * LD + k] = sqrt(dkk);
      }
      __syncthreads();
      if (s_fail) break;
      const double piv = M[k * LD + k];
      for (int i = k + 1 + tid; i < s; i += nt) M[i * LD + k] /= piv;
      __syncthreads();
      const int rem = s - k - 1;
      for (int e = tid; e < rem * rem; e += nt) {
        const int i = k + 1 + e / rem, j = k + 1 + e % rem;
        if (j <= i) M[i * LD + j] -= M[i * LD + k] * M[j * LD + k];
      }
      __syncthreads();
    }
    if (!s_fail) {
      ok = true;
    } else {
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
  // Save C (lower triangle, zeros above) and form Q = Y_mu^T Y_mu in Xg (col-major).
  for (int e = tid; e < s * s; e += nt) {
    const int i = e / s, j = e % s;
    Cg[i * SP + j] = (j <= i) ? M[i * LD + j] : 0.0;
    Xg[j * SP + i] = G3[i * SP + j] + mu * (G1[i * SP + j] + G1[j * SP + i]) + mu * mu * G2[i * SP + j];
  }
  __syncthreads();
  // X = C^-1 Q: thread j solves for column j (C from LDS).
  for (int j = tid; j < s; j += nt) {
    double* xc = Xg + (int64_t)j * SP;
    for (int i = 0; i < s; ++i) {
      double v = xc[i];
      for (int l = 0; l < i; ++l) v -= M[i * LD + l] * xc[l];
      xc[i] = v / M[i * LD + i];
    }
  }
  __syncthreads();
  // G = C^-1 X^T: column j of G solves C g = (row j of X)^T.
  for (int j = tid; j < s; j += nt) {
    double* gc = Gg + (int64_t)j * SP;
    for (int i = 0; i < s; ++i) {
      double v = Xg[(int64_t)i * SP + j];  // X[j][i] stored col-major at (i, j) -> X(j, i)
      for (int l = 0; l < i; ++l) v -= M[i * LD + l] * gc[l];
      gc[i] = v / M[i * LD + i];
    }
  }
  __syncthreads();
  // G into LDS, symmetrised; V = I.
  for (int e = tid; e < s * s; e += nt) {
    const int i = e / s, j = e % s;
    M[i * LD + j] = 0.5 * (Gg[(int64_t)j * SP + i] + Gg[(int64_t)i * SP + j]);
    Vg[(int64_t)j * SP + i] = (i == j) ? 1.0 : 0.0;
  }
  __shared__ int s_rot[2];  // a rotation happened in the sweep of this parity
  if (tid == 0) s_rot[0] = 0;
  __syncthreads();

  // Cyclic Jacobi with round-robin pairing; S players (s rounded up to even).
  // A pair is rotated only while |g_pq| > tol sqrt(g_pp g_qq), and g_pq is
  // then set to zero; the iteration ends after a sweep without a rotation.
  constexpr double tol = 1.0e-14;
  const int S = (s + 1) & ~1;
  const int npairs = S / 2;
  for (int sweep = 0; sweep < 40; ++sweep) {
    for (int round = 0; round < S - 1; ++round) {
      if (tid < npairs) {
        auto player = [&](int pos) { return pos == 0 ? 0 : 1 + ((pos - 1 + round) % (S - 1)); };
        int p = player(tid), q = player(S - 1 - tid);
        if (p > q) {
          const int t = p;
          p = q;
          q = t;
        }
        double c = 1.0, sn = 0.0;
        if (q < s) {
          const double apq = M[p * LD + q];
          const double app = M[p * LD + p], aqq = M[q * LD + q];
          if (fabs(apq) > tol * sqrt(fabs(app * aqq))) {
            const double theta = (aqq - app) / (2.0 * apq);
            const double t = (theta >= 0.0 ? 1.0 : -1.0) / (fabs(theta) + sqrt(theta * theta + 1.0));
            c = 1.0 / sqrt(t * t + 1.0);
            sn = t * c;
            s_rot[sweep & 1] = 1;
          }
        }
        pr_p[tid] = p;
        pr_q[tid] = q;
        cs_c[tid] = c;
        cs_s[tid] = sn;
      }
      __syncthreads();
      if (round == 0 && tid == 0) s_rot[(sweep + 1) & 1] = 0;
      // rows: (M_pk, M_qk) <- (c M_pk - s M_qk, s M_pk + c M_qk)
      for (int e = tid; e < npairs * s; e += nt) {
        const int pi = e / s, k = e % s;
        const int p = pr_p[pi], q = pr_q[pi];
        if (q >= s || cs_s[pi] == 0.0) continue;
        const double c = cs_c[pi], sn = cs_s[pi];
        const double a = M[p * LD + k], bq = M[q * LD + k];
        M[p * LD + k] = c * a - sn * bq;
        M[q * LD + k] = sn * a + c * bq;
      }
      __syncthreads();
      // columns, and V <- V P
      for (int e = tid; e < npairs * s; e += nt) {
        const int pi = e / s, k = e % s;
        const int p = pr_p[pi], q = pr_q[pi];
        if (q >= s || cs_s[pi] == 0.0) continue;
        const double c = cs_c[pi], sn = cs_s[pi];
        const double a = M[k * LD + p], bq = M[k * LD + q];
        M[k * LD + p] = k == q ? 0.0 : c * a - sn * bq;
        M[k * LD + q] = k == p ? 0.0 : sn * a + c * bq;
        const double va = Vg[(int64_t)p * SP + k], vb = Vg[(int64_t)q * SP + k];
        Vg[(int64_t)p * SP + k] = c * va - sn * vb;
        Vg[(int64_t)q * SP + k] = sn * va + c * vb;
      }
      __syncthreads();
    }
    if (s_rot[sweep & 1] == 0) break;
  }
  // Sort eigenvalues descending.
  if (tid == 0) {
    for (int j = 0; j < s; ++j) {
      perm[j] = j;
      evals[j] = M[j * LD + j];
    }
    for (int i = 1; i < s; ++i) {
      const double ev = evals[i];
      const int pv = perm[i];
      int k = i - 1;
      while (k >= 0 && evals[k] < ev) {
        evals[k + 1] = evals[k];
        perm[k + 1] = perm[k];
        --k;
      }
      evals[k + 1] = ev;
      perm[k + 1] = pv;
    }
    // keep the leading eigenpairs whose shifted value is resolvable at the
    // precision of Y: lambda_hat_j = sigma_j^2 - mu > rel_floor * lambda_hat_0
    const double top = evals[0] - mu;
    int keep = 0;
    for (int j = 0; j < s; ++j) {
      if (top > 0.0 && evals[j] - mu > rel_floor * top)
        keep = j + 1;
      else
        break;
    }
    s_fail = keep;
  }
  __syncthreads();
  const int keep = s_fail;
  for (int j = tid; j < s; j += nt) lam_b[j] = (j < keep) ? fmax(evals[j] - mu, 0.0) : 0.0;
  // Reload C into LDS, then T(:, j) = C^-T V(:, perm[j]) / sigma_j.
  __syncthreads();
  for (int e = tid; e < s * s; e += nt) {
    const int i = e / s, j = e % s;
    M[i * LD + j] = Cg[i * SP + j];
  }
  __syncthreads();
  for (int j = tid; j < SP; j += nt) {
    double* tcol = Tg + (int64_t)j * SP;
    if (j >= keep) {
      for (int i = 0; i < SP; ++i) tcol[i] = 0.0;
      continue;
    }
    const double* vcol = Vg + (int64_t)perm[j] * SP;
    const double inv_sig = 1.0 / sqrt(evals[j]);
    for (int i = s - 1; i >= 0; --i) {
      double v = vcol[i];
      for (int l = i + 1; l < s; ++l) v -= M[l * LD + i] * tcol[l];
      tcol[i] = v / M[i * LD + i];
    }
    for (int i = 0; i < s; ++i) tcol[i] *= inv_sig;
    for (int i = s; i < SP; ++i) tcol[i] = 0.0;
  }
  if (tid == 0) {
    s_eff_out[b] = keep;
    status_out[b] = 0;
    shift_out[b] = mu;
  }
}

// U[b] (n x s, col-major, ld n) = (Y + mu Omega) T  for the first s_eff columns, 0 after
// (T is zero there).  FP64 products on the matrix cores (v_mfma_f64_16x16x4: A[i][k] from
// lane 16 k + i, B[k][j] from lane 16 k + j, D[4 v + L / 16][L % 16] in register v).  A
// block of kFuRows rows stages T (s x sc, sc = s rounded up to 16) in LDS once;
// wavefront w owns rows 16 w .. 16 w + 15 and holds their A operands (Y + mu Omega in
// FP64) for every K step; each 16-column tile of U is staged in LDS and written a
// column at a time.
constexpr int kFuWaves = 8, kFuRows = 16 * kFuWaves;
template <typename VT, int SP>
__global__ __launch_bounds__(64 * kFuWaves) void k_form_u(int64_t n, int s,
                                                          const VT* __restrict__ Y,
                                                          const VT* __restrict__ omega,
                                                          const double* __restrict__ core,
                                                          const double* __restrict__ shift,
                                                          VT* __restrict__ U) {
  typedef double v4d __attribute__((ext_vector_type(4)));
  constexpr int KS = SP / 4;
  extern __shared__ double Tl[];  // s rows (k) x (sc + 1), T[k][j]
  __shared__ VT Ut[16][kFuRows + 4];
  const int b = blockIdx.y, tid = threadIdx.x, nt = blockDim.x;
  const double mu = shift[b];
  const int64_t row0 = (int64_t)blockIdx.x * kFuRows;
  const int wave = tid >> 6, lane = tid & 63;
  const int li = lane & 15, lk = lane >> 4;
  const VT* Yb = Y + (int64_t)b * n * SP;
  const VT* Ob = omega + (int64_t)b * n * SP;
  const double* Tg = core + (int64_t)b * 5 * SP * SP + 4 * SP * SP;
  VT* Ub = U + (int64_t)b * n * s;
  const int sc = (s + 15) / 16 * 16, lt = sc + 1;
  // T into LDS (eight loads in flight per thread)
  for (int e0 = tid; e0 < s * sc; e0 += 8 * nt) {
    double v[8];
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * nt;
      v[u] = e < s * sc ? Tg[(int64_t)(e / s) * SP + e % s] : 0.0;  // column e / s, row e % s
    }
#pragma unroll
    for (int u = 0; u < 8; ++u) {
      const int e = e0 + u * nt;
      if (e < s * sc) Tl[(e % s) * lt + e / s] = v[u];
    }
  }
  const int nks = (s + 3) / 4;
  const int64_t r = row0 + 16 * wave + li;
  const int64_t rc = r < n ? r : n - 1;  // clamped: every load is issued unconditionally
  VT ya[KS], oa[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const int kc = min(4 * ks + lk, s - 1);
    ya[ks] = Yb[(int64_t)kc * n + rc];
    oa[ks] = Ob[(int64_t)kc * n + rc];
  }
  __syncthreads();
  double a[KS];
#pragma unroll
  for (int ks = 0; ks < KS; ++ks) {
    const bool ok = r < n && 4 * ks + lk < s;
    a[ks] = ok ? double(ya[ks]) + mu * double(oa[ks]) : 0.0;
  }
  for (int j0 = 0; j0 < s; j0 += 16) {
    v4d d = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
    for (int ks = 0; ks < KS; ++ks) {
      const int k = 4 * ks + lk;
      if (ks < nks) d = __builtin_amdgcn_mfma_f64_16x16x4f64(a[ks], k < s ? Tl[k * lt + j0 + li] : 0.0,
                                                             d, 0, 0, 0);
    }
    // D[4 v + lk][li]: row 16 wave + 4 v + lk of the block, column j0 + li
#pragma unroll
    for (int v = 0; v < 4; ++v) Ut[li][16 * wave + 4 * v + lk] = VT(d[v]);
    __syncthreads();
    for (int e = tid; e < 16 * kFuRows; e += nt) {
      const int c = e / kFuRows, q = e - c * kFuRows;
      const int j = j0 + c;
      const int64_t i = row0 + q;
      if (j < s && i < n) Ub[(int64_t)j * n + i] = Ut[c][q];
    }
    __syncthreads();
  }
}

int pad_rank(int s) { return s <= 16 ? 16 : (s <= 32 ? 32 : (s <= 64 ? 64 : 128)); }

template <typename T, typename VT, int SP>
hipError_t sketch_gemms_impl(const MatArg& A, int64_t batch, const VT* d, int64_t d_stride,
                        const SketchWs& ws, hipStream_t st) {
  if constexpr (std::is_same<T, uint16_t>::value && std::is_same<VT, float>::value) {
    if (sketch_mfma_eligible(A, VT_F32, ws))
      return launch_sketch_mfma(A, batch, SP, d, d_stride, ws, st);
  }
  const int m = (int)A.m, n = (int)A.n;
  const T* Ap = static_cast<const T*>(A.ptr);
  // W = A Omega, split over n
  {
    int kchunk = (int)((A.n + ws.ksW - 1) / ws.ksW);
    kchunk = ((kchunk + kBK - 1) / kBK) * kBK;
    dim3 grid((unsigned)((m + kBM - 1) / kBM), (unsigned)ws.ksW, (unsigned)batch);
    hipLaunchKernelGGL((k_sketch_w<T, VT, SP>), grid, dim3(256), 0, st, Ap, A.lda, A.strideA, m,
                       n, static_cast<const VT*>(ws.omega), static_cast<VT*>(ws.Wpart), kchunk,
                       (int64_t)m * SP, (int64_t)ws.ksW * m * SP);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    e = launch_sum_splits(sizeof(VT) == 4 ? VT_F32 : VT_F64, batch, (int64_t)m * SP, ws.Wpart,
                          ws.ksW, (int64_t)m * SP, (int64_t)ws.ksW * m * SP, ws.W,
                          (int64_t)m * SP, st);
    if (e != hipSuccess) return e;
  }
  // Y = A^T (d o W), split over m
  {
    int rchunk = (int)((A.m + ws.ksY - 1) / ws.ksY);
    rchunk = ((rchunk + kBK - 1) / kBK) * kBK;
    dim3 grid((unsigned)((n + kBM - 1) / kBM), (unsigned)ws.ksY, (unsigned)batch);
    hipLaunchKernelGGL((k_sketch_y<T, VT, SP>), grid, dim3(256), 0, st, Ap, A.lda, A.strideA, m,
                       n, static_cast<const VT*>(ws.W), d, d_stride, static_cast<VT*>(ws.Ypart),
                       rchunk, (int64_t)n * SP, (int64_t)ws.ksY * n * SP);
    return hipGetLastError();
  }
}

template <typename T, typename VT, int SP>
hipError_t sketch_gemms(const MatArg& A, int64_t batch, const VT* d, int64_t d_stride,
                        const SketchWs& ws, hipStream_t st) {
  hipError_t e = hipSuccess;
  if (ws.ev_gemm[0] != nullptr && (e = hipEventRecord(ws.ev_gemm[0], st)) != hipSuccess) return e;
  e = sketch_gemms_impl<T, VT, SP>(A, batch, d, d_stride, ws, st);
  if (e != hipSuccess) return e;
  if (ws.ev_gemm[1] != nullptr) e = hipEventRecord(ws.ev_gemm[1], st);
  return e;
}

template <typename VT, int SP>
hipError_t run_core(const MatArg& A, int64_t batch, int s, const uint8_t* mask, const SketchWs& ws,
                    void* U, double* lamhat, int32_t* s_eff, int32_t* status, double* shift,
                    hipStream_t st) {
  const int64_t n = A.n;
  {
    const unsigned nby = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n * SP + 255) / 256, 2048));
    hipLaunchKernelGGL((k_y_sum<VT, SP>), dim3(nby, (unsigned)batch), dim3(256), 0, st, n,
                       static_cast<const VT*>(ws.Ypart), ws.ksY, (int64_t)n * SP,
                       (int64_t)ws.ksY * n * SP, mask, static_cast<VT*>(ws.Y));
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
    dim3 grid((unsigned)ws.nbG, 3u, (unsigned)batch);
    hipLaunchKernelGGL((k_gram<VT, SP>), grid, dim3(256), 0, st, n, s,
                       static_cast<const VT*>(ws.omega), static_cast<const VT*>(ws.Y), ws.gpart,
                       ws.nbG);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
    dim3 g2((unsigned)((SP * SP + 255) / 256), 3u, (unsigned)batch);
    hipLaunchKernelGGL(k_gram_reduce, g2, dim3(256), 0, st, SP * SP, ws.gpart, ws.nbG, ws.gram);
    e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  const double eps = sizeof(VT) == 4 ? 0x1p-24 : 0x1p-53;
  const double rel_floor = sizeof(VT) == 4 ? 1.0e-6 : 1.0e-13;
  // Jacobi stops once every |g_pq| <= tol sqrt(g_pp g_qq); the columns of U then are
  // orthonormal to about tol, far below the FP32 rounding of U for tol = 1e-9
  const double jac_tol = sizeof(VT) == 4 ? 1.0e-9 : 1.0e-14;
  hipError_t e = hipSuccess;
  if (s <= kCoreLdsMaxS) {
    e = launch_nystrom_core_lds(batch, s, SP, eps, rel_floor, jac_tol, ws.gram, ws.core, lamhat,
                                s_eff, status, shift, st);
    if (e != hipSuccess) return e;
  } else {
    const size_t lds = (size_t)SP * (SP + 1) * sizeof(double);
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_nystrom_core<SP>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    hipLaunchKernelGGL((k_nystrom_core<SP>), dim3((unsigned)batch), dim3(256), lds, st, s, n, eps,
                       rel_floor, ws.gram, ws.core, lamhat, s, s_eff, status, shift);
  }
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  {
    const int sc = (s + 15) / 16 * 16;
    const size_t lds = (size_t)s * (sc + 1) * sizeof(double);
    e = hipFuncSetAttribute(reinterpret_cast<const void*>(&k_form_u<VT, SP>),
                            hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    dim3 g3((unsigned)((n + kFuRows - 1) / kFuRows), (unsigned)batch);
    hipLaunchKernelGGL((k_form_u<VT, SP>), g3, dim3(64 * kFuWaves), lds, st, n, s,
                       static_cast<const VT*>(ws.Y), static_cast<const VT*>(ws.omega), ws.core,
                       shift, static_cast<VT*>(U));
  }
  return hipGetLastError();
}

template <typename VT>
hipError_t dispatch_rank(const MatArg& A, int64_t batch, const VT* d, int64_t d_stride, int s,
                         const uint8_t* mask, const SketchWs& ws, void* U, double* lamhat,
                         int32_t* s_eff, int32_t* status, double* shift, hipStream_t st) {
  const int sp = pad_rank(s);
  hipError_t e = hipSuccess;
#define GENIOS_SK(SPV)                                                                     \
  if (sp == SPV) {                                                                         \
    if constexpr (sizeof(VT) == 4) {                                                       \
      if (A.mt == MT_BF16)                                                                 \
        e = sketch_gemms<uint16_t, VT, SPV>(A, batch, d, d_stride, ws, st);                \
      else                                                                                 \
        e = sketch_gemms<float, VT, SPV>(A, batch, d, d_stride, ws, st);                   \
    } else {                                                                               \
      e = sketch_gemms<double, VT, SPV>(A, batch, d, d_stride, ws, st);                    \
    }                                                                                      \
    if (e != hipSuccess) return e;                                                         \
    return run_core<VT, SPV>(A, batch, s, mask, ws, U, lamhat, s_eff, status, shift, st); \
  }
  GENIOS_SK(16)
  GENIOS_SK(32)
  GENIOS_SK(64)
  GENIOS_SK(128)
#undef GENIOS_SK
  return hipErrorInvalidValue;
}

}  // namespace

int sketch_pad(int s) { return pad_rank(s); }

size_t sketch_ws_bytes(int64_t m, int64_t n, int s, int64_t batch, VType vt, int* ksW, int* ksY,
                       int* nbG) {
  const int sp = pad_rank(s);
  const size_t e = vt == VT_F32 ? 4 : 8;
  const int64_t rb = ((m + kBM - 1) / kBM) * batch;
  int64_t kw = (1024 + rb - 1) / rb;
  kw = std::max<int64_t>(1, std::min<int64_t>(kw, std::max<int64_t>(1, n / 256)));
  const int64_t cb = ((n + kBM - 1) / kBM) * batch;
  int64_t ky = (1024 + cb - 1) / cb;
  ky = std::max<int64_t>(1, std::min<int64_t>(ky, std::max<int64_t>(1, m / 256)));
  int64_t ng = std::max<int64_t>(1, std::min<int64_t>((n + 255) / 256, std::max<int64_t>(1, 256 / batch)));
  if (ksW) *ksW = (int)kw;
  if (ksY) *ksY = (int)ky;
  if (nbG) *nbG = (int)ng;
  size_t bytes = 0;
  auto add = [&](size_t b) { bytes += (b + 255) / 256 * 256; };
  add(batch * n * sp * e);               // omega
  add(batch * m * sp * e);               // W
  add(batch * kw * m * sp * e);          // Wpart
  add(batch * ky * n * sp * e);          // Ypart
  add(batch * n * sp * e);               // Y
  add(batch * 3 * ng * sp * sp * 8);     // gpart
  add(batch * 3 * sp * sp * 8);          // gram
  add(batch * 5 * sp * sp * 8);          // core
  return bytes;
}

hipError_t launch_gaussian(VType vt, int64_t n, int s, int s_stride, int64_t batch, uint64_t seed,
                           uint64_t stream_id, const uint8_t* mask, void* out, hipStream_t st) {
  const int64_t nblk = (n * s + 3) / 4;
  const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((nblk + 255) / 256, 2048));
  dim3 grid(nb, (unsigned)batch);
  if (vt == VT_F32)
    hipLaunchKernelGGL(k_gaussian<float>, grid, dim3(256), 0, st, n, s, s_stride, seed, stream_id,
                       mask, static_cast<float*>(out));
  else
    hipLaunchKernelGGL(k_gaussian<double>, grid, dim3(256), 0, st, n, s, s_stride, seed,
                       stream_id, mask, static_cast<double*>(out));
  return hipGetLastError();
}

hipError_t run_nystrom(const MatArg& A, int64_t batch, VType vt, const void* d, int64_t d_stride,
                       int s, const void* omega_in, uint64_t seed, uint64_t stream_id,
                       const uint8_t* mask, const SketchWs& ws, void* U, double* lamhat,
                       int32_t* s_eff, int32_t* core_status, double* shift_out, hipStream_t st) {
  const int sp = pad_rank(s);
  const int64_t n = A.n;
  const size_t e = vt == VT_F32 ? 4 : 8;
  hipError_t err = launch_fill(ws.omega, (size_t)batch * n * sp * e, st);
  if (err != hipSuccess) return err;
  if (omega_in) {
    const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((n * s + 255) / 256, 2048));
    dim3 grid(nb, (unsigned)batch);
    if (vt == VT_F32)
      hipLaunchKernelGGL(k_copy_omega<float>, grid, dim3(256), 0, st, n, s, sp,
                         static_cast<const float*>(omega_in), mask, static_cast<float*>(ws.omega));
    else
      hipLaunchKernelGGL(k_copy_omega<double>, grid, dim3(256), 0, st, n, s, sp,
                         static_cast<const double*>(omega_in), mask,
                         static_cast<double*>(ws.omega));
    err = hipGetLastError();
  } else {
    err = launch_gaussian(vt, n, s, sp, batch, seed, stream_id, mask, ws.omega, st);
  }
  if (err != hipSuccess) return err;
  if (vt == VT_F32)
    return dispatch_rank<float>(A, batch, static_cast<const float*>(d), d_stride, s, mask, ws, U,
                                lamhat, s_eff, core_status, shift_out, st);
  return dispatch_rank<double>(A, batch, static_cast<const double*>(d), d_stride, s, mask, ws, U,
                               lamhat, s_eff, core_status, shift_out, st);
}

}  // namespace genios
