// Error of the Nystrom approximation for the adaptive sketch size (Sec. 2.2):
// the randomized power method on E = H - U diag(lam_hat) U^T, which is positive
// semidefinite.  One step, per problem, after h = H v is formed by the matrix
// products:
//   k_pm_ut     y = U^T v as column partials over row chunks,
//   k_pm_apply  E v = h - U (lam_hat o y) and the partials of ||E v||^2, v^T E v,
//   k_pm_norm   theta = v^T E v (the estimate) and v <- E v / ||E v||.
// The start vector is normalised by k_pm_sq + k_pm_norm.  Partials are summed in a
// fixed order by the consumer (the same bits in every block), no atomics.
#include <algorithm>
#include <cmath>

#include "device.hpp"

namespace genios {

namespace {

constexpr int kPmThreads = 256;

__device__ __forceinline__ double pm_block_sum(double v, double* sm) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = v;
  __syncthreads();
  const double r = ((sm[0] + sm[1]) + sm[2]) + sm[3];
  __syncthreads();
  return r;
}

__device__ __forceinline__ void pm_rows(int64_t n, int nb, int64_t& lo, int64_t& hi) {
  const int64_t chunk = (n + nb - 1) / nb;
  lo = (int64_t)blockIdx.x * chunk;
  hi = lo + chunk < n ? lo + chunk : n;
}

// grid (nb * s_stride, batch): block x = j * nb + chunk.
template <typename VT>
__global__ __launch_bounds__(kPmThreads) void k_pm_ut(int64_t n, int s_stride,
                                                      const VT* __restrict__ U,
                                                      const VT* __restrict__ v,
                                                      const int32_t* __restrict__ s_eff,
                                                      double* __restrict__ part, int pstride,
                                                      int nb) {
  __shared__ double sm[4];
  const int b = blockIdx.y;
  const int j = blockIdx.x / nb, blk = blockIdx.x - j * nb;
  if (j >= s_eff[b]) return;  // partials of dropped columns are never read
  const int64_t chunk = (n + nb - 1) / nb;
  const int64_t lo = (int64_t)blk * chunk, hi = lo + chunk < n ? lo + chunk : n;
  const VT* Uj = U + ((int64_t)b * s_stride + j) * n;
  const VT* vb = v + (int64_t)b * n;
  double acc = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kPmThreads) acc += (double)Uj[i] * (double)vb[i];
  acc = pm_block_sum(acc, sm);
  if (threadIdx.x == 0) part[((int64_t)b * kMaxS + j) * pstride + blk] = acc;
}

// grid (nb, batch)
template <typename VT>
__global__ __launch_bounds__(kPmThreads) void k_pm_apply(
    int64_t n, int s_stride, const VT* __restrict__ U, const double* __restrict__ lamhat,
    const int32_t* __restrict__ s_eff, const double* __restrict__ ut_part, int pstride,
    const VT* __restrict__ h, const VT* __restrict__ v, VT* __restrict__ ev,
    double* __restrict__ part2, int nb) {
  __shared__ double coef[kMaxS];
  __shared__ double sm[4];
  const int b = blockIdx.y;
  const int se = s_eff[b];
  for (int j = threadIdx.x; j < se; j += kPmThreads) {
    const double* pj = ut_part + ((int64_t)b * kMaxS + j) * pstride;
    double y = 0.0;
    for (int k = 0; k < nb; ++k) y += pj[k];
    coef[j] = lamhat[(int64_t)b * s_stride + j] * y;
  }
  __syncthreads();
  int64_t lo, hi;
  pm_rows(n, nb, lo, hi);
  const VT* Ub = U + (int64_t)b * s_stride * n;
  const VT* hb = h + (int64_t)b * n;
  const VT* vb = v + (int64_t)b * n;
  VT* eb = ev + (int64_t)b * n;
  double n2 = 0.0, vt = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kPmThreads) {
    double s = 0.0;
    for (int j = 0; j < se; ++j) s += (double)Ub[(int64_t)j * n + i] * coef[j];
    const double e = (double)hb[i] - s;
    const VT ei = VT(e);
    eb[i] = ei;
    n2 += (double)ei * (double)ei;
    vt += (double)vb[i] * (double)ei;
  }
  n2 = pm_block_sum(n2, sm);
  vt = pm_block_sum(vt, sm);
  if (threadIdx.x == 0) {
    part2[((int64_t)b * 2 + 0) * pstride + blockIdx.x] = n2;
    part2[((int64_t)b * 2 + 1) * pstride + blockIdx.x] = vt;
  }
}

// ||w||^2 partials of the start vector (slot 1 = 0: no estimate).  grid (nb, batch)
template <typename VT>
__global__ __launch_bounds__(kPmThreads) void k_pm_sq(int64_t n, const VT* __restrict__ w,
                                                      double* __restrict__ part2, int pstride,
                                                      int nb) {
  __shared__ double sm[4];
  const int b = blockIdx.y;
  int64_t lo, hi;
  pm_rows(n, nb, lo, hi);
  const VT* wb = w + (int64_t)b * n;
  double n2 = 0.0;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kPmThreads) n2 += (double)wb[i] * (double)wb[i];
  n2 = pm_block_sum(n2, sm);
  if (threadIdx.x == 0) {
    part2[((int64_t)b * 2 + 0) * pstride + blockIdx.x] = n2;
    part2[((int64_t)b * 2 + 1) * pstride + blockIdx.x] = 0.0;
  }
}

// v <- w / ||w||, est[b] <- the v^T E v partial sum (when est != nullptr).  grid (nb, batch)
template <typename VT>
__global__ __launch_bounds__(kPmThreads) void k_pm_norm(int64_t n, const VT* __restrict__ w,
                                                        VT* __restrict__ v,
                                                        const double* __restrict__ part2,
                                                        int pstride, int nb,
                                                        double* __restrict__ est) {
  __shared__ double tot[2];
  const int b = blockIdx.y;
  if (threadIdx.x < 2) {
    const double* p = part2 + ((int64_t)b * 2 + threadIdx.x) * pstride;
    double s = 0.0;
    for (int k = 0; k < nb; ++k) s += p[k];
    tot[threadIdx.x] = s;
  }
  __syncthreads();
  const double nrm = sqrt(tot[0]);
  if (est != nullptr && blockIdx.x == 0 && threadIdx.x == 0) est[b] = nrm > 0.0 ? tot[1] : 0.0;
  const double inv = nrm > 0.0 ? 1.0 / nrm : 0.0;
  int64_t lo, hi;
  pm_rows(n, nb, lo, hi);
  const VT* wb = w + (int64_t)b * n;
  VT* vb = v + (int64_t)b * n;
  for (int64_t i = lo + threadIdx.x; i < hi; i += kPmThreads) vb[i] = VT((double)wb[i] * inv);
}

template <typename VT>
hipError_t pm_start_vt(const PowerArgs& a, hipStream_t st) {
  dim3 grid((unsigned)a.nb, (unsigned)a.batch);
  hipLaunchKernelGGL((k_pm_sq<VT>), grid, dim3(kPmThreads), 0, st, a.n,
                     static_cast<const VT*>(a.ev), a.part2, a.pstride, a.nb);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_pm_norm<VT>), grid, dim3(kPmThreads), 0, st, a.n,
                     static_cast<const VT*>(a.ev), static_cast<VT*>(a.v), a.part2, a.pstride, a.nb,
                     (double*)nullptr);
  return hipGetLastError();
}

template <typename VT>
hipError_t pm_step_vt(const PowerArgs& a, hipStream_t st) {
  hipLaunchKernelGGL((k_pm_ut<VT>), dim3((unsigned)(a.nb * a.s_stride), (unsigned)a.batch),
                     dim3(kPmThreads), 0, st, a.n, a.s_stride, static_cast<const VT*>(a.U),
                     static_cast<const VT*>(a.v), a.s_eff, a.ut_part, a.pstride, a.nb);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  dim3 grid((unsigned)a.nb, (unsigned)a.batch);
  hipLaunchKernelGGL((k_pm_apply<VT>), grid, dim3(kPmThreads), 0, st, a.n, a.s_stride,
                     static_cast<const VT*>(a.U), a.lamhat, a.s_eff, a.ut_part, a.pstride,
                     static_cast<const VT*>(a.h), static_cast<const VT*>(a.v),
                     static_cast<VT*>(a.ev), a.part2, a.nb);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_pm_norm<VT>), grid, dim3(kPmThreads), 0, st, a.n,
                     static_cast<const VT*>(a.ev), static_cast<VT*>(a.v), a.part2, a.pstride, a.nb,
                     a.est);
  return hipGetLastError();
}

bool power_args_ok(const PowerArgs& a) {
  return a.n >= 1 && a.batch >= 1 && a.nb >= 1 && a.nb <= a.pstride && a.s_stride >= 1 &&
         a.s_stride <= kMaxS && a.v && a.ev && a.part2;
}

}  // namespace

int power_blocks(int64_t n, int pstride) {
  const int64_t nb = (n + kPmThreads - 1) / kPmThreads;
  return (int)std::max<int64_t>(1, std::min<int64_t>(nb, pstride));
}

hipError_t launch_power_start(const PowerArgs& a, hipStream_t st) {
  if (!power_args_ok(a)) return hipErrorInvalidValue;
  return a.vt == VT_F32 ? pm_start_vt<float>(a, st) : pm_start_vt<double>(a, st);
}

hipError_t launch_power_step(const PowerArgs& a, hipStream_t st) {
  if (!power_args_ok(a) || !a.U || !a.lamhat || !a.s_eff || !a.ut_part || !a.h || !a.est)
    return hipErrorInvalidValue;
  return a.vt == VT_F32 ? pm_step_vt<float>(a, st) : pm_step_vt<double>(a, st);
}

}  // namespace genios
