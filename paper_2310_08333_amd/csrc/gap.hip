// Relative duality gap of the l1-regularised ML problems (App. A).
//
// For  l(x) = sum_i f(t_i) + lam ||x||_1,  t = A x,
//   Lasso:     f(t_i) = (t_i - b_i)^2 / 2,        f'(t_i) = t_i - b_i,
//   logistic:  f(t_i) = log(1 + e^{w_i}), w_i = -y_i t_i,  f'(t_i) = -y_i sigmoid(w_i)
//   (the logistic labels folded into the rows, so b = 0 there),
//   Huber:     f(t_i) = l(t_i - b_i),  f'(t_i) = 2 clip(t_i - b_i, -delta, delta),
// the dual point is
// nu = kappa f'(t) with kappa = min(1, lam / ||A^T f'(t)||_inf), which makes
// ||A^T nu||_inf <= lam, and the dual function is
//   Lasso:     g(nu) = -||nu||^2 / 2 - b^T nu,
//   logistic:  g(nu) = -sum_i h(kappa s_i),  h(v) = v log v + (1 - v) log(1 - v),
//              with s_i = sigmoid(w_i) (the folded rows' nu);
//   Huber:     g(nu) = -||nu||^2 / 4 - b^T nu  (l*(v) = v^2 / 4 on |v| <= 2 delta,
//              where every kappa f'(t_i) lies);
// with the l2 term (lambda2 > 0) the dual is finite for every nu: kappa = 1
// and g gains -(1 / (2 lambda2)) ||(|A^T nu| - lam)_+||^2, while l(x) gains
// (lambda2 / 2) ||x||^2,
// with a box instead of the l1 term (box-constrained least squares, the QP of
// Sec. 3.2 with M = I), nu = t - b unscaled and g(nu) = -||nu||^2 / 2 - b^T nu -
// sum_j max(lo_j w_j, hi_j w_j), w = -A^T nu (the box's support function),
// so l(x) - g(nu) >= l(x) - l(x*) and the relative gap is
// (l(x) - g(nu)) / min(l(x), |g(nu)|) (Sec. 3.3).
//
// Passes: t = A v (gemv_n partials), the elementwise step below (f'(t) into an
// m-vector, loss partials), A^T f'(t) (gemv_t partials), ||.||_inf and ||v||_1
// partials, kappa and l(x) (one block per problem), sum of the conjugate terms
// at kappa (second m-pass), g(nu) and the relative gap (one block per problem).
// Every reduction writes one partial per block; the finishing blocks reduce
// them in a fixed order.
#include <algorithm>
#include <cmath>

#include "device.hpp"

namespace genios {

namespace {

constexpr int kGapThreads = 256;

// v <- sum over the first `count` entries of p (stride `step`), fixed order:
// lane l sums entries l, l + 64, ..., then the wavefront sums the lanes.
__device__ __forceinline__ double wave_fixed_sum(const double* p, int count, int step) {
  const int lane = threadIdx.x & 63;
  double s = 0.0;
  for (int i = lane; i < count; i += 64) s += p[(int64_t)i * step];
  return wave_sum(s);
}
__device__ __forceinline__ double wave_fixed_max(const double* p, int count, int step) {
  const int lane = threadIdx.x & 63;
  double s = 0.0;
  for (int i = lane; i < count; i += 64) s = fmax(s, p[(int64_t)i * step]);
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) s = fmax(s, __shfl_xor(s, o, 64));
  return s;
}

// Block sum of one double per thread (256 threads), valid in thread 0.
__device__ __forceinline__ double block_sum1(double v, double* sm) {
  v = wave_sum(v);
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = v;
  __syncthreads();
  const double r = ((sm[0] + sm[1]) + sm[2]) + sm[3];
  __syncthreads();
  return r;
}
__device__ __forceinline__ double block_max1(double v, double* sm) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  if ((threadIdx.x & 63) == 0) sm[threadIdx.x >> 6] = v;
  __syncthreads();
  const double r = fmax(fmax(sm[0], sm[1]), fmax(sm[2], sm[3]));
  __syncthreads();
  return r;
}

__device__ __forceinline__ double sigmoid_d(double w) {
  return w >= 0.0 ? 1.0 / (1.0 + exp(-w)) : exp(w) / (1.0 + exp(w));
}
// log(1 + e^w) without overflow
__device__ __forceinline__ double softplus_d(double w) {
  return w > 0.0 ? w + log1p(exp(-w)) : log1p(exp(w));
}
// v log v + (1 - v) log(1 - v) on [0, 1] (0 log 0 = 0)
__device__ __forceinline__ double neg_entropy(double v) {
  const double a = v > 0.0 ? v * log(v) : 0.0;
  const double b = v < 1.0 ? (1.0 - v) * log1p(-v) : 0.0;
  return a + b;
}

// t from its column-split partials; nu_i = f'(t_i) (Lasso: t - b; Huber:
// 2 clip(t - b, -delta, delta); logistic: the folded s_i = sigmoid(-y_i t_i), with
// f'(t_i) = -y_i s_i formed for A^T); partial sums of the loss.
template <typename VT>
__global__ __launch_bounds__(kGapThreads) void k_gap_elem(
    int64_t m, const VT* __restrict__ tparts, int nsplit, int64_t split_stride,
    int64_t prob_stride, const VT* __restrict__ bvec, int lossk, double delta,
    VT* __restrict__ fprime,
    VT* __restrict__ sfold, double* __restrict__ part, int pstride) {
  __shared__ double sm[4];
  const int b = blockIdx.y;
  const VT* tp = tparts + (int64_t)b * prob_stride;
  const VT* bb = bvec + (int64_t)b * m;
  VT* fp = fprime + (int64_t)b * m;
  VT* sf = sfold + (int64_t)b * m;
  double loss = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kGapThreads + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * kGapThreads) {
    double t = 0.0;
    for (int k = 0; k < nsplit; ++k) t += (double)tp[(int64_t)k * split_stride + i];
    const double bi = (double)bb[i];
    if (lossk == kLossLogistic) {
      const double w = -bi * t;
      const double s = sigmoid_d(w);
      loss += softplus_d(w);
      fp[i] = VT(-bi * s);
      sf[i] = VT(s);
    } else if (lossk == kLossHuber) {
      const double r = t - bi, a = fabs(r);
      loss += a <= delta ? r * r : 2.0 * delta * a - delta * delta;
      const double f1 = 2.0 * fmin(fmax(r, -delta), delta);
      fp[i] = VT(f1);
      sf[i] = VT(f1);
    } else {
      const double r = t - bi;
      loss += 0.5 * r * r;
      fp[i] = VT(r);
      sf[i] = VT(r);
    }
  }
  loss = block_sum1(loss, sm);
  if (threadIdx.x == 0) part[((int64_t)b * kGapSlots + 0) * pstride + blockIdx.x] = loss;
}

// ||A^T f'(t)||_inf and ||(|A^T f'(t)| - lambda)_+||^2 from the row-split
// partials, ||v||_1, ||v||^2, and the squared distance from 0 to
// grad f(v) + lambda d||v||_1 (grad f = A^T f'(t) + lambda2 v): per entry
// grad_j + lambda sign(v_j) where v_j != 0, (|grad_j| - lambda)_+ where v_j = 0.
// Box: the support-function terms instead of the excess, and the distance from 0
// to grad f(v) + the box's normal cone at v.
template <typename VT>
__global__ __launch_bounds__(kGapThreads) void k_gap_inf(
    int64_t n, const VT* __restrict__ ypart, int ks, int64_t ks_stride, int64_t prob_stride,
    const VT* __restrict__ v, const ProbParams* __restrict__ params, const VT* __restrict__ lo_all,
    const VT* __restrict__ hi_all, double* __restrict__ part, int pstride) {
  __shared__ double sm[4];
  const int b = blockIdx.y;
  const double lam = params[b].lambda, lam2 = params[b].lambda2;
  const bool box = params[b].prox == kProxBox;
  const VT* lo = box && lo_all ? lo_all + (int64_t)b * n : nullptr;
  const VT* hi = box && hi_all ? hi_all + (int64_t)b * n : nullptr;
  const VT* yp = ypart + (int64_t)b * prob_stride;
  const VT* vb = v + (int64_t)b * n;
  double gmax = 0.0, l1 = 0.0, x2 = 0.0, ex2 = 0.0, sd2 = 0.0;
  for (int64_t j = (int64_t)blockIdx.x * kGapThreads + threadIdx.x; j < n;
       j += (int64_t)gridDim.x * kGapThreads) {
    double g = 0.0;
    for (int k = 0; k < ks; ++k) g += (double)yp[(int64_t)k * ks_stride + j];
    gmax = fmax(gmax, fabs(g));
    const double vj = (double)vb[j];
    l1 += fabs(vj);
    x2 += vj * vj;
    const double gf = g + lam2 * vj;
    if (box) {
      // support function of the box at w = -g, and the normal-cone distance at v
      const double w = -g;
      const double lj = lo ? (double)lo[j] : -INFINITY, hj = hi ? (double)hi[j] : INFINITY;
      if (w > 0.0) ex2 += hj * w;
      else if (w < 0.0) ex2 += lj * w;
      const bool at_lo = lo && vj <= lj, at_hi = hi && vj >= hj;
      const double sd = (at_lo && at_hi) ? 0.0
                        : at_lo ? fmax(-gf, 0.0) : (at_hi ? fmax(gf, 0.0) : fabs(gf));
      sd2 += sd * sd;
    } else {
      const double e = fmax(fabs(g) - lam, 0.0);
      ex2 += e * e;
      const double sd = vj != 0.0 ? gf + copysign(lam, vj) : fmax(fabs(gf) - lam, 0.0);
      sd2 += sd * sd;
    }
  }
  gmax = block_max1(gmax, sm);
  l1 = block_sum1(l1, sm);
  x2 = block_sum1(x2, sm);
  ex2 = block_sum1(ex2, sm);
  sd2 = block_sum1(sd2, sm);
  if (threadIdx.x == 0) {
    double* pb = part + (int64_t)b * kGapSlots * pstride + blockIdx.x;
    pb[1 * pstride] = gmax;
    pb[2 * pstride] = l1;
    pb[4 * pstride] = x2;
    pb[5 * pstride] = ex2;
    pb[6 * pstride] = sd2;
  }
}

// kappa, the primal value and the dual's l2 part (one 64-thread block per problem).
__global__ __launch_bounds__(64) void k_gap_kappa(const double* __restrict__ part, int pstride,
                                                  int nb_m, int nb_n,
                                                  const ProbParams* __restrict__ params,
                                                  GapState* __restrict__ gs) {
  const int b = blockIdx.x;
  const double* pb = part + (int64_t)b * kGapSlots * pstride;
  const double loss = wave_fixed_sum(pb, nb_m, 1);
  const double ginf = wave_fixed_max(pb + pstride, nb_n, 1);
  const double l1 = wave_fixed_sum(pb + 2 * pstride, nb_n, 1);
  const double x2 = wave_fixed_sum(pb + 4 * pstride, nb_n, 1);
  const double ex2 = wave_fixed_sum(pb + 5 * pstride, nb_n, 1);
  const double sd2 = wave_fixed_sum(pb + 6 * pstride, nb_n, 1);
  if (threadIdx.x == 0) {
    const double lam = params[b].lambda, lam2 = params[b].lambda2;
    GapState& G = gs[b];
    G.loss = loss;
    G.grad_inf = ginf;
    G.l1 = l1;
    G.x2 = x2;
    G.excess2 = ex2;
    G.subgrad = sqrt(sd2);
    // lambda2 > 0: g is finite for every nu, nu = f'(t) unscaled (App. A); box: the
    // dual of the split is finite wherever the support function is, nu = f'(t)
    const bool box = params[b].prox == kProxBox;
    G.kappa = (lam2 > 0.0 || box) ? 1.0 : (ginf > lam ? lam / ginf : 1.0);
    G.reg = box ? -ex2 : (lam2 > 0.0 ? -ex2 / (2.0 * lam2) : 0.0);
    G.primal = loss + lam * l1 + 0.5 * lam2 * x2;
  }
}

// Conjugate terms at kappa: Lasso v^2 / 2 + b_i v, Huber v^2 / 4 + b_i v with
// v = kappa f'(t_i); logistic h(kappa s_i).  Their sum is -g(nu).
template <typename VT>
__global__ __launch_bounds__(kGapThreads) void k_gap_dual(
    int64_t m, const VT* __restrict__ sfold, const VT* __restrict__ bvec, int lossk,
    const GapState* __restrict__ gs, double* __restrict__ part, int pstride) {
  __shared__ double sm[4];
  const int b = blockIdx.y;
  const double kap = gs[b].kappa;
  const VT* sf = sfold + (int64_t)b * m;
  const VT* bb = bvec + (int64_t)b * m;
  double acc = 0.0;
  for (int64_t i = (int64_t)blockIdx.x * kGapThreads + threadIdx.x; i < m;
       i += (int64_t)gridDim.x * kGapThreads) {
    const double v = kap * (double)sf[i];
    acc += lossk == kLossLogistic ? neg_entropy(v)
           : (lossk == kLossHuber ? 0.25 : 0.5) * v * v + (double)bb[i] * v;
  }
  acc = block_sum1(acc, sm);
  if (threadIdx.x == 0) part[((int64_t)b * kGapSlots + 3) * pstride + blockIdx.x] = acc;
}

__global__ __launch_bounds__(64) void k_gap_final(const double* __restrict__ part, int pstride,
                                                  int nb_m, GapState* __restrict__ gs) {
  const int b = blockIdx.x;
  const double conj = wave_fixed_sum(part + ((int64_t)b * kGapSlots + 3) * pstride, nb_m, 1);
  if (threadIdx.x == 0) {
    GapState& G = gs[b];
    G.dual = -conj + G.reg;
    const double den = fmin(G.primal, fabs(G.dual));
    G.gap = G.primal - G.dual;
    G.rel_gap = den > 0.0 ? G.gap / den : (G.gap == 0.0 ? 0.0 : INFINITY);
  }
}

template <typename VT>
hipError_t gap_elem_vt(const GapArgs& a, hipStream_t st) {
  const int nb = gap_blocks(a.m);
  hipLaunchKernelGGL((k_gap_elem<VT>), dim3(nb, (unsigned)a.batch), dim3(kGapThreads), 0, st,
                     a.m, static_cast<const VT*>(a.tparts), a.nsplit, a.split_stride,
                     a.prob_stride, static_cast<const VT*>(a.bvec), a.loss, a.delta,
                     static_cast<VT*>(a.fprime), static_cast<VT*>(a.sfold), a.part, kGapPStride);
  return hipGetLastError();
}

template <typename VT>
hipError_t gap_after_t_vt(const GapArgs& a, hipStream_t st) {
  const int nbm = gap_blocks(a.m), nbn = gap_blocks(a.n);
  hipLaunchKernelGGL((k_gap_inf<VT>), dim3(nbn, (unsigned)a.batch), dim3(kGapThreads), 0, st,
                     a.n, static_cast<const VT*>(a.ypart), a.ks, a.ks_stride, a.yprob,
                     static_cast<const VT*>(a.v), a.params, static_cast<const VT*>(a.lo),
                     static_cast<const VT*>(a.hi), a.part, kGapPStride);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gap_kappa, dim3((unsigned)a.batch), dim3(64), 0, st, a.part, kGapPStride,
                     nbm, nbn, a.params, a.state);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL((k_gap_dual<VT>), dim3(nbm, (unsigned)a.batch), dim3(kGapThreads), 0, st,
                     a.m, static_cast<const VT*>(a.sfold), static_cast<const VT*>(a.bvec),
                     a.loss, a.state, a.part, kGapPStride);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(k_gap_final, dim3((unsigned)a.batch), dim3(64), 0, st, a.part, kGapPStride,
                     nbm, a.state);
  return hipGetLastError();
}

}  // namespace

int gap_blocks(int64_t len) {
  const int64_t nb = (len + kGapThreads - 1) / kGapThreads;
  return (int)std::max<int64_t>(1, std::min<int64_t>(nb, kGapPStride));
}

// Every buffer the kernels touch must be given (checked on the host).
static bool gap_args_complete(const GapArgs& a) {
  return a.m >= 1 && a.n >= 1 && a.batch >= 1 && a.tparts && a.nsplit >= 1 && a.bvec &&
         a.loss >= kLossSquare && a.loss <= kLossHuber && (a.loss != kLossHuber || a.delta > 0.0) &&
         a.fprime && a.sfold && a.ypart && a.ks >= 1 && a.ks_stride >= a.n && a.v && a.params &&
         a.part && a.state;
}

hipError_t launch_gap_elem(const GapArgs& a, hipStream_t st) {
  if (!gap_args_complete(a)) return hipErrorInvalidValue;
  return a.vt == VT_F32 ? gap_elem_vt<float>(a, st) : gap_elem_vt<double>(a, st);
}

hipError_t launch_gap_after_t(const GapArgs& a, hipStream_t st) {
  if (!gap_args_complete(a)) return hipErrorInvalidValue;
  return a.vt == VT_F32 ? gap_after_t_vt<float>(a, st) : gap_after_t_vt<double>(a, st);
}

}  // namespace genios
