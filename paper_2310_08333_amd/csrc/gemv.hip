// Dense matrix-vector products for the Hessian-vector product of the CG loop.
//
// The x-subproblem operator is applied as two matrix-vector products,
// H v = A^T (D (A v)) (Sec. 3.1 HVP example, Sec. 3.3 ML Hessian), both
// HBM-bandwidth bound: every element of A is read once per product.
//
//   gemv_n   t = A v         one wavefront owns ROWS rows of a column split;
//                            lanes stride the row with 16-byte loads, the
//                            partial sums are reduced with cross-lane shuffles.
//   gemv_t   y = A^T (d o t) a lane owns V consecutive columns (16 bytes of
//                            each row); a block's four wavefronts cover the
//                            same 64*V columns over interleaved rows of a row
//                            split and combine in LDS; the split's t values
//                            (optionally scaled by d and summed over gemv_n's
//                            column splits) are staged in LDS; results are
//                            per-split partials reduced later in a fixed order.
// No floating-point atomics: results are bitwise reproducible.
#include <algorithm>

#include "device.hpp"

namespace genios {

namespace {

constexpr int kMaxRowsPerSplit = 2048;

// Rows per wavefront in gemv_n: 8 for BF16 (the FP32 vector chunk is then read
// once per 8 rows of 16-byte matrix loads), 4 otherwise.
template <typename T>
constexpr int gemv_n_rows() {
  return sizeof(T) == 2 ? 8 : 4;
}

template <typename T, typename VT, int ROWS, bool VEC, bool ABS = false>
__global__ __launch_bounds__(256) void k_gemv_n(const T* __restrict__ A, int64_t lda,
                                                int64_t strideA, int m, int n,
                                                const VT* __restrict__ v, int64_t v_stride,
                                                VT* __restrict__ out, int64_t out_split_stride,
                                                int64_t out_prob_stride, int cols_per_split,
                                                const int32_t* __restrict__ gate, int gate_stride) {
  using Acc = typename Elem<T>::Acc;
  constexpr int V = Elem<T>::V;
  const int b = blockIdx.z;
  if (gate != nullptr && gate[(int64_t)b * gate_stride] == 0) return;
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int row0 = (blockIdx.x * 4 + wave) * ROWS;
  if (row0 >= m) return;
  const int split = blockIdx.y;
  const int c0 = split * cols_per_split;
  const int c1 = min(n, c0 + cols_per_split);
  const T* Ab = A + (int64_t)b * strideA;
  const VT* vb = v + (int64_t)b * v_stride;
  const T* rowp[ROWS];
#pragma unroll
  for (int r = 0; r < ROWS; ++r) rowp[r] = Ab + (int64_t)min(row0 + r, m - 1) * lda;
  Acc acc[ROWS];
#pragma unroll
  for (int r = 0; r < ROWS; ++r) acc[r] = Acc(0);
  if constexpr (VEC) {
    int c = c0 + lane * V;
#pragma unroll 2
    for (; c + V <= c1; c += 64 * V) {
      Acc av[ROWS][V];
#pragma unroll
      for (int r = 0; r < ROWS; ++r) Elem<T>::load(rowp[r] + c, av[r]);
      Acc vv[V];
      load_vec<VT, Acc, V>(vb + c, vv);
      if constexpr (ABS) {
#pragma unroll
        for (int j = 0; j < V; ++j) vv[j] = fabs(vv[j]);
#pragma unroll
        for (int r = 0; r < ROWS; ++r)
#pragma unroll
          for (int j = 0; j < V; ++j) av[r][j] = fabs(av[r][j]);
      }
#pragma unroll
      for (int r = 0; r < ROWS; ++r)
#pragma unroll
        for (int j = 0; j < V; ++j) acc[r] += av[r][j] * vv[j];
    }
    for (int cc = c; cc < c1 && cc < c + V; ++cc) {
      const Acc vv = ABS ? fabs(Acc(vb[cc])) : Acc(vb[cc]);
#pragma unroll
      for (int r = 0; r < ROWS; ++r) {
        const Acc a = Elem<T>::cvt(rowp[r][cc]);
        acc[r] += (ABS ? fabs(a) : a) * vv;
      }
    }
  } else {
    for (int cc = c0 + lane; cc < c1; cc += 64) {
      const Acc vv = ABS ? fabs(Acc(vb[cc])) : Acc(vb[cc]);
#pragma unroll
      for (int r = 0; r < ROWS; ++r) {
        const Acc a = Elem<T>::cvt(rowp[r][cc]);
        acc[r] += (ABS ? fabs(a) : a) * vv;
      }
    }
  }
#pragma unroll
  for (int r = 0; r < ROWS; ++r) acc[r] = wave_sum(acc[r]);
  if (lane < ROWS && row0 + lane < m) {
    Acc mine = acc[0];
#pragma unroll
    for (int r = 1; r < ROWS; ++r)
      if (lane == r) mine = acc[r];
    out[(int64_t)b * out_prob_stride + (int64_t)split * out_split_stride + row0 + lane] = VT(mine);
  }
}

// Block = 4 wavefronts sharing one 64*V-column tile of a row split: wave w takes
// rows w, w+4, ...; the four partial sums are combined in LDS in a fixed order.
template <typename T, typename VT, int NR, bool VEC>
__global__ __launch_bounds__(256) void k_gemv_t(
    const T* __restrict__ A, int64_t lda, int64_t strideA, int m, int n,
    const VT* __restrict__ tin, int nsplit_in, int64_t tin_split_stride, int64_t tin_prob_stride,
    int64_t tin_col_stride, const VT* __restrict__ dscale, int64_t d_stride,
    VT* __restrict__ ypart, int64_t ypart_ks_stride, int64_t ypart_col_stride,
    int64_t ypart_prob_stride, int rows_per_split, const int32_t* __restrict__ gate,
    int gate_stride) {
  using Acc = typename Elem<T>::Acc;
  constexpr int V = VEC ? Elem<T>::V : 1;
  __shared__ Acc ts[NR][kMaxRowsPerSplit];
  __shared__ Acc red[3][NR][64 * V];
  const int b = blockIdx.z;
  if (gate != nullptr && gate[(int64_t)b * gate_stride] == 0) return;
  const int ks = blockIdx.y;
  const int r0 = ks * rows_per_split;
  const int r1 = min(m, r0 + rows_per_split);
  const int nr = r1 - r0;
  const VT* tb = tin + (int64_t)b * tin_prob_stride;
  for (int i = threadIdx.x; i < nr; i += blockDim.x) {
#pragma unroll
    for (int k = 0; k < NR; ++k) {
      Acc s = Acc(0);
      for (int sp = 0; sp < nsplit_in; ++sp)
        s += Acc(tb[(int64_t)k * tin_col_stride + (int64_t)sp * tin_split_stride + r0 + i]);
      if (dscale != nullptr) s *= Acc(dscale[(int64_t)b * d_stride + r0 + i]);
      ts[k][i] = s;
    }
  }
  __syncthreads();
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
  const int c = (blockIdx.x * 64 + lane) * V;
  const T* Ab = A + (int64_t)b * strideA + (int64_t)r0 * lda;
  Acc acc[NR][V];
#pragma unroll
  for (int k = 0; k < NR; ++k)
#pragma unroll
    for (int j = 0; j < V; ++j) acc[k][j] = Acc(0);
  if (c < n) {
    if (VEC && c + V <= n) {
      if constexpr (VEC) {
        constexpr int U = 8;
        int i = wave;
        for (; i + 4 * (U - 1) < nr; i += 4 * U) {
          Acc av[U][V];
#pragma unroll
          for (int u = 0; u < U; ++u) Elem<T>::load(Ab + (int64_t)(i + 4 * u) * lda + c, av[u]);
#pragma unroll
          for (int u = 0; u < U; ++u)
#pragma unroll
            for (int k = 0; k < NR; ++k) {
              const Acc t = ts[k][i + 4 * u];
#pragma unroll
              for (int j = 0; j < V; ++j) acc[k][j] += av[u][j] * t;
            }
        }
        for (; i < nr; i += 4) {
          Acc av[V];
          Elem<T>::load(Ab + (int64_t)i * lda + c, av);
#pragma unroll
          for (int k = 0; k < NR; ++k) {
            const Acc t = ts[k][i];
#pragma unroll
            for (int j = 0; j < V; ++j) acc[k][j] += av[j] * t;
          }
        }
      }
    } else {
      const int ce = min(n, c + V);
      for (int i = wave; i < nr; i += 4) {
        for (int cc = c; cc < ce; ++cc) {
          const Acc a = Elem<T>::cvt(Ab[(int64_t)i * lda + cc]);
#pragma unroll
          for (int k = 0; k < NR; ++k) acc[k][cc - c] += a * ts[k][i];
        }
      }
    }
  }
  if (wave > 0) {
#pragma unroll
    for (int k = 0; k < NR; ++k)
#pragma unroll
      for (int j = 0; j < V; ++j) red[wave - 1][k][lane * V + j] = acc[k][j];
  }
  __syncthreads();
  if (wave != 0 || c >= n) return;
#pragma unroll
  for (int w = 0; w < 3; ++w)
#pragma unroll
    for (int k = 0; k < NR; ++k)
#pragma unroll
      for (int j = 0; j < V; ++j) acc[k][j] += red[w][k][lane * V + j];
  VT* yb = ypart + (int64_t)b * ypart_prob_stride + (int64_t)ks * ypart_ks_stride;
  const int ce = min(n, c + V);
#pragma unroll
  for (int k = 0; k < NR; ++k)
#pragma unroll
    for (int j = 0; j < V; ++j)
      if (c + j < ce) yb[(int64_t)k * ypart_col_stride + c + j] = VT(acc[k][j]);
}

int elem_v(MType mt) { return mt == MT_BF16 ? 8 : (mt == MT_F32 ? 4 : 2); }
int elem_bytes(MType mt) { return mt == MT_BF16 ? 2 : (mt == MT_F32 ? 4 : 8); }
int rows_n(MType mt) { return mt == MT_BF16 ? 8 : 4; }

bool vec_ok(const MatArg& A) {
  const int V = elem_v(A.mt);
  const uintptr_t pa = reinterpret_cast<uintptr_t>(A.ptr);
  return pa % 16 == 0 && A.lda % V == 0 && A.strideA % V == 0;
}

}  // namespace

int gemv_n_splits(const MatArg& A, int64_t batch) {
  const int R = rows_n(A.mt);
  const int64_t rb = (A.m + 4 * R - 1) / (4 * R);
  const int V = elem_v(A.mt);
  const int64_t want = (2048 + rb * batch - 1) / (rb * batch);
  const int64_t maxs = std::max<int64_t>(1, A.n / (64 * V * 8));
  return (int)std::max<int64_t>(1, std::min<int64_t>(want, std::min<int64_t>(maxs, 64)));
}

int gemv_t_splits(const MatArg& A, int64_t batch) {
  const int V = elem_v(A.mt);
  const int64_t cb = (A.n + 64 * V - 1) / (64 * V);
  int64_t ks = (2048 + cb * batch - 1) / (cb * batch);
  // keep the partial traffic at <= ~2% of the matrix traffic
  const int64_t cap = std::max<int64_t>(1, (A.m * elem_bytes(A.mt)) / (50 * 4));
  ks = std::min(ks, cap);
  ks = std::min<int64_t>(ks, (A.m + 31) / 32);
  ks = std::max<int64_t>(ks, (A.m + kMaxRowsPerSplit - 1) / kMaxRowsPerSplit);
  return (int)std::max<int64_t>(1, ks);
}

int gemv_t_rows_per_split(const MatArg& A, int ksplit) {
  return (int)((A.m + ksplit - 1) / ksplit);
}

template <typename T, typename VT, bool ABS = false>
static hipError_t gemv_n_t(const MatArg& A, int64_t batch, const VT* v, int64_t v_stride, VT* out,
                           int64_t oss, int64_t ops, int nsplit, const int32_t* gate, int gs,
                           hipStream_t st) {
  constexpr int V = Elem<T>::V;
  constexpr int R = gemv_n_rows<T>();
  const int64_t rb = (A.m + 4 * R - 1) / (4 * R);
  int cps = (int)((A.n + nsplit - 1) / nsplit);
  cps = ((cps + V - 1) / V) * V;
  dim3 grid((unsigned)rb, (unsigned)nsplit, (unsigned)batch);
  const bool vec = vec_ok(A) && (reinterpret_cast<uintptr_t>(v) % 16 == 0) && (v_stride % V == 0);
  const T* Ap = static_cast<const T*>(A.ptr);
  if (vec)
    hipLaunchKernelGGL((k_gemv_n<T, VT, R, true, ABS>), grid, dim3(256), 0, st, Ap, A.lda,
                       A.strideA, (int)A.m, (int)A.n, v, v_stride, out, oss, ops, cps, gate, gs);
  else
    hipLaunchKernelGGL((k_gemv_n<T, VT, R, false, ABS>), grid, dim3(256), 0, st, Ap, A.lda,
                       A.strideA, (int)A.m, (int)A.n, v, v_stride, out, oss, ops, cps, gate, gs);
  return hipGetLastError();
}

hipError_t launch_gemv_n(const MatArg& A, int64_t batch, VType vt, const void* v, int64_t v_stride,
                         void* out, int64_t oss, int64_t ops, int nsplit, const int32_t* gate,
                         int gs, hipStream_t st) {
  if (vt == VT_F32) {
    const float* vv = static_cast<const float*>(v);
    float* o = static_cast<float*>(out);
    if (A.mt == MT_BF16)
      return gemv_n_t<uint16_t, float>(A, batch, vv, v_stride, o, oss, ops, nsplit, gate, gs, st);
    if (A.mt == MT_F32)
      return gemv_n_t<float, float>(A, batch, vv, v_stride, o, oss, ops, nsplit, gate, gs, st);
    return hipErrorInvalidValue;
  }
  if (A.mt != MT_F64) return hipErrorInvalidValue;
  return gemv_n_t<double, double>(A, batch, static_cast<const double*>(v), v_stride,
                                  static_cast<double*>(out), oss, ops, nsplit, gate, gs, st);
}

// |A| |v| (elementwise absolute values of both), the same split partials as launch_gemv_n.
hipError_t launch_gemv_n_abs(const MatArg& A, int64_t batch, VType vt, const void* v,
                             int64_t v_stride, void* out, int64_t oss, int64_t ops, int nsplit,
                             hipStream_t st) {
  if (vt == VT_F32) {
    const float* vv = static_cast<const float*>(v);
    float* o = static_cast<float*>(out);
    if (A.mt == MT_BF16)
      return gemv_n_t<uint16_t, float, true>(A, batch, vv, v_stride, o, oss, ops, nsplit, nullptr,
                                             0, st);
    if (A.mt == MT_F32)
      return gemv_n_t<float, float, true>(A, batch, vv, v_stride, o, oss, ops, nsplit, nullptr, 0,
                                          st);
    return hipErrorInvalidValue;
  }
  if (A.mt != MT_F64) return hipErrorInvalidValue;
  return gemv_n_t<double, double, true>(A, batch, static_cast<const double*>(v), v_stride,
                                        static_cast<double*>(out), oss, ops, nsplit, nullptr, 0,
                                        st);
}

namespace {
// One block per problem: y_i = sum over the nsplit partials (fixed order) of row i, then
// out[4 b + 0] = sum y_i^2, out[4 b + 1] = sum |y_i| and out[4 b + 3] = sum |c_i| |y_i|
// (mode 0), or out[4 b + 2] = sum (y_i - c_i)^2 (mode 1, c the right-hand side).
// Fixed-order sums.
template <typename VT>
__global__ __launch_bounds__(256) void k_bound_terms(int64_t m, const VT* __restrict__ parts,
                                                     int nsplit, int64_t split_stride,
                                                     int64_t prob_stride,
                                                     const VT* __restrict__ c, int64_t c_stride,
                                                     int mode, double* __restrict__ out) {
  __shared__ double red[3][256];
  const int b = blockIdx.x, tid = threadIdx.x;
  const VT* pb = parts + (int64_t)b * prob_stride;
  double s0 = 0.0, s1 = 0.0, s2 = 0.0;
  for (int64_t i = tid; i < m; i += 256) {
    double y = 0.0;
    for (int k = 0; k < nsplit; ++k) y += double(pb[(int64_t)k * split_stride + i]);
    const double ci = double(c[(int64_t)b * c_stride + i]);
    if (mode == 0) {
      s0 += y * y;
      s1 += fabs(y);
      s2 += fabs(ci) * fabs(y);
    } else {
      s0 += (y - ci) * (y - ci);
    }
  }
  red[0][tid] = s0;
  red[1][tid] = s1;
  red[2][tid] = s2;
  __syncthreads();
  for (int h = 128; h > 0; h >>= 1) {
    if (tid < h) {
#pragma unroll
      for (int q = 0; q < 3; ++q) red[q][tid] += red[q][tid + h];
    }
    __syncthreads();
  }
  if (tid == 0) {
    if (mode == 0) {
      out[4 * b + 0] = red[0][0];
      out[4 * b + 1] = red[1][0];
      out[4 * b + 3] = red[2][0];
    } else {
      out[4 * b + 2] = red[0][0];
    }
  }
}
}  // namespace

hipError_t launch_bound_terms(VType vt, int64_t m, int64_t batch, const void* parts, int nsplit,
                              int64_t split_stride, int64_t prob_stride, const void* c,
                              int64_t c_stride, int mode, double* out, hipStream_t st) {
  if (vt == VT_F32)
    hipLaunchKernelGGL(k_bound_terms<float>, dim3((unsigned)batch), dim3(256), 0, st, m,
                       static_cast<const float*>(parts), nsplit, split_stride, prob_stride,
                       static_cast<const float*>(c), c_stride, mode, out);
  else
    hipLaunchKernelGGL(k_bound_terms<double>, dim3((unsigned)batch), dim3(256), 0, st, m,
                       static_cast<const double*>(parts), nsplit, split_stride, prob_stride,
                       static_cast<const double*>(c), c_stride, mode, out);
  return hipGetLastError();
}

template <typename T, typename VT, int NR>
static hipError_t gemv_t_t(const MatArg& A, int64_t batch, const VT* tin, int nsplit_in,
                           int64_t tss, int64_t tps, int64_t tcs, const VT* d, int64_t ds,
                           VT* yp, int ksplit, int64_t yks, int64_t ycs, int64_t yps,
                           const int32_t* gate, int gs, hipStream_t st) {
  constexpr int V = Elem<T>::V;
  const int rps = gemv_t_rows_per_split(A, ksplit);
  if (rps > kMaxRowsPerSplit) return hipErrorInvalidValue;
  const bool vec = vec_ok(A);
  const T* Ap = static_cast<const T*>(A.ptr);
  if (vec) {
    dim3 grid((unsigned)((A.n + 64 * V - 1) / (64 * V)), (unsigned)ksplit, (unsigned)batch);
    hipLaunchKernelGGL((k_gemv_t<T, VT, NR, true>), grid, dim3(256), 0, st, Ap, A.lda, A.strideA,
                       (int)A.m, (int)A.n, tin, nsplit_in, tss, tps, tcs, d, ds, yp, yks, ycs, yps,
                       rps, gate, gs);
  } else {
    dim3 grid((unsigned)((A.n + 63) / 64), (unsigned)ksplit, (unsigned)batch);
    hipLaunchKernelGGL((k_gemv_t<T, VT, NR, false>), grid, dim3(256), 0, st, Ap, A.lda,
                       A.strideA, (int)A.m, (int)A.n, tin, nsplit_in, tss, tps, tcs, d, ds, yp,
                       yks, ycs, yps, rps, gate, gs);
  }
  return hipGetLastError();
}

template <typename VT>
static hipError_t gemv_t_vt(const MatArg& A, int64_t batch, const VT* tin, int nsplit_in,
                            int64_t tss, int64_t tps, int64_t tcs, int nrhs, const VT* d,
                            int64_t ds, VT* yp, int ksplit, int64_t yks, int64_t ycs, int64_t yps,
                            const int32_t* gate, int gs, hipStream_t st) {
  if constexpr (sizeof(VT) == 4) {
    if (A.mt == MT_BF16) {
      if (nrhs == 1)
        return gemv_t_t<uint16_t, VT, 1>(A, batch, tin, nsplit_in, tss, tps, tcs, d, ds, yp,
                                         ksplit, yks, ycs, yps, gate, gs, st);
      return gemv_t_t<uint16_t, VT, 2>(A, batch, tin, nsplit_in, tss, tps, tcs, d, ds, yp, ksplit,
                                       yks, ycs, yps, gate, gs, st);
    }
    if (A.mt == MT_F32) {
      if (nrhs == 1)
        return gemv_t_t<float, VT, 1>(A, batch, tin, nsplit_in, tss, tps, tcs, d, ds, yp, ksplit,
                                      yks, ycs, yps, gate, gs, st);
      return gemv_t_t<float, VT, 2>(A, batch, tin, nsplit_in, tss, tps, tcs, d, ds, yp, ksplit,
                                    yks, ycs, yps, gate, gs, st);
    }
    return hipErrorInvalidValue;
  } else {
    if (A.mt != MT_F64) return hipErrorInvalidValue;
    if (nrhs == 1)
      return gemv_t_t<double, VT, 1>(A, batch, tin, nsplit_in, tss, tps, tcs, d, ds, yp, ksplit,
                                     yks, ycs, yps, gate, gs, st);
    return gemv_t_t<double, VT, 2>(A, batch, tin, nsplit_in, tss, tps, tcs, d, ds, yp, ksplit, yks,
                                   ycs, yps, gate, gs, st);
  }
}

hipError_t launch_gemv_t(const MatArg& A, int64_t batch, VType vt, const void* tin, int nsplit_in,
                         int64_t tss, int64_t tps, int64_t tcs, int nrhs, const void* d,
                         int64_t ds, void* yp, int ksplit, int64_t yks, int64_t ycs, int64_t yps,
                         const int32_t* gate, int gs, hipStream_t st) {
  if (nrhs < 1 || nrhs > 2) return hipErrorInvalidValue;
  if (vt == VT_F32)
    return gemv_t_vt<float>(A, batch, static_cast<const float*>(tin), nsplit_in, tss, tps, tcs,
                            nrhs, static_cast<const float*>(d), ds, static_cast<float*>(yp),
                            ksplit, yks, ycs, yps, gate, gs, st);
  return gemv_t_vt<double>(A, batch, static_cast<const double*>(tin), nsplit_in, tss, tps, tcs,
                           nrhs, static_cast<const double*>(d), ds, static_cast<double*>(yp),
                           ksplit, yks, ycs, yps, gate, gs, st);
}

// ---- small utility kernels ---------------------------------------------------

// ---- fused Hessian-vector product ---------------------------------------------
// hp = A^T (d o (A p)) in one pass over A (Sec. 3.1 HVP example, Sec. 3.3 ML
// Hessian with D = diag(d)).  Of the G blocks of a problem, block g owns the
// rows g, g + G, g + 2G, ..., so the grid reads A as one band moving down the
// matrix (measured faster than G separate row ranges), with non-temporal loads.
// p sits in LDS (FP32); thread t owns the 16-byte column chunks
// c = V (t + THREADS k) and keeps their share of the result in registers.  Each row's chunks are loaded
// once (packed; the next row's loads are in flight while a row is processed),
// the row's dot product is reduced over the block (shuffles, then one LDS
// exchange and one barrier), scaled by d, and the same registers update the
// owned result columns.  Each block writes one partial of hp; the partials are
// summed in a fixed order by the consumer.
// Requires n % V == 0, lda % V == 0, 16-byte aligned rows and a 16-byte
// aligned p (with p_stride % 4 == 0 between problems).

template <typename T>
struct Raw;
template <>
struct Raw<uint16_t> {
  using type = u32x4_t;  // 8 BF16
  __device__ static __forceinline__ float get(const u32x4_t& q, int e) {
    const uint32_t w = e < 2 ? q.x : (e < 4 ? q.y : (e < 6 ? q.z : q.w));
    return __uint_as_float((e & 1) ? (w & 0xffff0000u) : (w << 16));
  }
  // The same value through a byte permute: a second, differently written unpack,
  // so the compiler recomputes it instead of keeping the first one's results live.
  __device__ static __forceinline__ float get2(const u32x4_t& q, int e) {
    const uint32_t w = e < 2 ? q.x : (e < 4 ? q.y : (e < 6 ? q.z : q.w));
    return __uint_as_float(__builtin_amdgcn_perm(w, w, (e & 1) ? 0x07060c0cu : 0x05040c0cu));
  }
};
template <>
struct Raw<float> {
  using type = f32x4_t;
  __device__ static __forceinline__ float get(const f32x4_t& q, int e) {
    return e == 0 ? q.x : (e == 1 ? q.y : (e == 2 ? q.z : q.w));
  }
  __device__ static __forceinline__ float get2(const f32x4_t& q, int e) { return get(q, e); }
};

// Fixed-order wavefront sum without LDS traffic: DPP butterflies inside each
// 16-lane row (pairs, quads, then row rotations by 4 and 8), then the four row
// sums read from lanes 0, 16, 32, 48 and added in that order.  Every lane gets
// the total.  All 64 lanes must be active.
template <int CTRL>
__device__ __forceinline__ float dpp_mov(float v) {
  return __int_as_float(__builtin_amdgcn_update_dpp(0, __float_as_int(v), CTRL, 0xf, 0xf, false));
}
__device__ __forceinline__ float wave_sum_dpp(float v) {
  v += dpp_mov<0xB1>(v);   // quad_perm [1,0,3,2]
  v += dpp_mov<0x4E>(v);   // quad_perm [2,3,0,1]
  v += dpp_mov<0x124>(v);  // row_ror 4
  v += dpp_mov<0x128>(v);  // row_ror 8
  const int b = __float_as_int(v);
  const float r0 = __int_as_float(__builtin_amdgcn_readlane(b, 0));
  const float r1 = __int_as_float(__builtin_amdgcn_readlane(b, 16));
  const float r2 = __int_as_float(__builtin_amdgcn_readlane(b, 32));
  const float r3 = __int_as_float(__builtin_amdgcn_readlane(b, 48));
  return ((r0 + r1) + r2) + r3;
}

constexpr int kCpolNT = 2;  // cache-policy operand of a buffer load: non-temporal

template <typename T, int THREADS, int EPT, int D>
__global__ __launch_bounds__(THREADS) void k_hvp_fused(
    const T* __restrict__ A, int64_t lda, int64_t strideA, int m, int n,
    const float* __restrict__ p, int64_t p_stride, const float* __restrict__ d, int64_t d_stride,
    float* __restrict__ ypart, int64_t ks_stride, int64_t prob_stride,
    const int32_t* __restrict__ gate, int gate_stride, double* __restrict__ pqpart,
    int64_t pq_stride) {
  static_assert(D >= 0 && D <= 2, "prefetch depth 0..2");
  constexpr int V = Elem<T>::V;
  constexpr int NC = EPT / V;
  constexpr int W = THREADS / 64;
  using RT = typename Raw<T>::type;
  extern __shared__ float ps[];  // n floats
  __shared__ float red[2][W];
  const int b = blockIdx.y;
  if (gate != nullptr && gate[(int64_t)b * gate_stride] == 0) return;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  // the block's rows by local index i in [r0, r1): row blockIdx.x + i * gridDim.x
  const int G = (int)gridDim.x;
  const int r0 = 0, r1 = (m - (int)blockIdx.x + G - 1) / G;
  // p in LDS, owner-major: the first NC - 1 chunks of thread t at t (NC - 1) V,
  // the (possibly partial) last chunk row after them, so a thread reads its
  // values from one base with small immediate offsets.  Exactly n floats.
  constexpr int HEAD = (NC - 1) * V;  // floats per thread in the first NC - 1 chunks
  const T* Ab = A + (int64_t)b * strideA;
  const float* db = d ? d + (int64_t)b * d_stride : nullptr;
  // Chunks k < NC - 1 always lie inside the row (EPT is the least multiple of V
  // with EPT * THREADS >= n); only the last one may fall past n (n % V == 0: a
  // chunk is wholly inside or outside), and is then read from column 0.
  const bool last_ok = V * (tid + THREADS * (NC - 1)) < n;
  auto col = [&](int k) { return (k < NC - 1 || last_ok) ? V * (tid + THREADS * k) : 0; };
  // (owner slices start at multiples of V floats: 16-byte aligned for float4 reads)
  const float4* pmine = reinterpret_cast<const float4*>(ps + tid * HEAD);
  const float4* plast = reinterpret_cast<const float4*>(ps + (last_ok ? THREADS * HEAD + tid * V : 0));
  const float lmask = last_ok ? 1.f : 0.f;  // the last chunk's p, zeroed past n (no branch)
  // A row's loads stay together and in chunk order (the scheduler may not move
  // other work across them), so a buffer's first chunk is the first to arrive
  // and the wait before each use covers only the loads issued before it.  The
  // row's d_i goes out first, as a buffer load: a vector load, retired in order
  // with the row's chunks.  (A scalar load, issued as late as its use, would
  // put its latency on every row: consecutive rows of a block are G apart in d.)
  // Raw buffer over the problem's m values of d (word 3: 32-bit data format).
  // The load is unconditional (a load under a branch gets a full wait at the
  // join): without d the buffer has no records, so the load at offset 0 is out
  // of range, touches no memory and returns 0 (its value is not used).
  // The row itself is read through a raw buffer over its n e_A bytes, with
  // non-temporal loads (A is streamed once per product).  The loads are
  // unconditional for the same reason; what must not be read is kept out by
  // the buffer's range check, which returns 0 without touching memory: a ring
  // slot past the block's last row (never processed) gets a buffer with no
  // records, and a last chunk past n (its p is zero and its result is never
  // stored) lies past the row's records.
  const __amdgpu_buffer_rsrc_t drs = __builtin_amdgcn_make_buffer_rsrc(
      const_cast<float*>(db ? db : p), 0, db ? m * 4 : 0, 0x00020000);
  auto load_row = [&](int i, RT (&dst)[NC], float& dv) {
    const bool live = i < r1;
    const int row = live ? (int)blockIdx.x + i * G : 0;
    const __amdgpu_buffer_rsrc_t ars = __builtin_amdgcn_make_buffer_rsrc(
        const_cast<T*>(Ab + (int64_t)row * lda), 0, live ? n * (int)sizeof(T) : 0, 0x00020000);
    __builtin_amdgcn_sched_barrier(0);
    dv = __uint_as_float(__builtin_amdgcn_raw_buffer_load_b32(drs, db ? row * 4 : 0, 0, 0));
#pragma unroll
    for (int k = 0; k < NC; ++k)
      dst[k] = __builtin_bit_cast(
          RT, __builtin_amdgcn_raw_buffer_load_b128(ars, 16 * (tid + THREADS * k), 0, kCpolNT));
    __builtin_amdgcn_sched_barrier(0);
  };
  float y[NC][V];
#pragma unroll
  for (int k = 0; k < NC; ++k)
#pragma unroll
    for (int e = 0; e < V; ++e) y[k][e] = 0.f;
  int par = 0;
  // p^T H p of the block's rows, sum of d_i (a_i^T p)^2 (the same value in every thread)
  double pq = 0.0;
  // one row: dot with p, block reduction, scale, rank-one update of the owned columns
  auto process = [&](RT (&cur)[NC], float dv) {
    float s = 0.f;
#pragma unroll
    for (int k = 0; k < NC; ++k) {
#pragma unroll
      for (int e4 = 0; e4 < V / 4; ++e4) {
        float4 q = k < NC - 1 ? pmine[k * (V / 4) + e4] : plast[e4];
        if (k == NC - 1) q = make_float4(q.x * lmask, q.y * lmask, q.z * lmask, q.w * lmask);
        s = fmaf(Raw<T>::get(cur[k], 4 * e4 + 0), q.x, s);
        s = fmaf(Raw<T>::get(cur[k], 4 * e4 + 1), q.y, s);
        s = fmaf(Raw<T>::get(cur[k], 4 * e4 + 2), q.z, s);
        s = fmaf(Raw<T>::get(cur[k], 4 * e4 + 3), q.w, s);
      }
    }
    s = wave_sum_dpp(s);
    if (lane == 0) red[par][wave] = s;
    __syncthreads();
    float t = 0.f;
#pragma unroll
    for (int w = 0; w < W; ++w) t += red[par][w];
    const float traw = t;
    if (db) t *= dv;
    pq = fma(double(traw), double(t), pq);
    par ^= 1;
#pragma unroll
    for (int k = 0; k < NC; ++k)
#pragma unroll
      for (int e = 0; e < V; ++e) y[k][e] = fmaf(Raw<T>::get2(cur[k], e), t, y[k][e]);
  };
  // Ring of D + 1 row buffers, loop rotated: each step first issues the row D
  // ahead into the free buffer, then processes the oldest one, so rows r + 1 ..
  // r + D are in flight while row r is processed and the wait before a buffer's
  // use covers only it (the newer D rows stay in flight).  Loads are
  // unconditional -- past the block's last row they are out of range and read
  // nothing (above) -- so every path reaches the loop head with the same loads
  // outstanding.  The prologue's rows are kept apart by a wavefront-scope fence
  // (a compiler barrier only).
  // (Every block owns at least one row: r0 < r1.)
  RT b0[NC], b1[NC], b2[NC];
  float d0 = 1.f, d1 = 1.f, d2 = 1.f;
  // Prologue: each thread loads the p values of the chunks it owns (16-byte
  // loads, all independent), then the first row's loads go out, then p is
  // written to LDS.  Loads retire in issue order, so the wait for p leaves
  // the row loads in flight.
  {
    const float* pb = p + (int64_t)b * p_stride;
    float4 pv[NC][V / 4];
#pragma unroll
    for (int k = 0; k < NC; ++k)
#pragma unroll
      for (int e4 = 0; e4 < V / 4; ++e4)
        pv[k][e4] = *reinterpret_cast<const float4*>(pb + col(k) + 4 * e4);
    load_row(r0, b0, d0);
#pragma unroll
    for (int k = 0; k < NC - 1; ++k)
#pragma unroll
      for (int e4 = 0; e4 < V / 4; ++e4)
        *reinterpret_cast<float4*>(ps + tid * HEAD + k * V + 4 * e4) = pv[k][e4];
    if (last_ok) {
#pragma unroll
      for (int e4 = 0; e4 < V / 4; ++e4)
        *reinterpret_cast<float4*>(ps + THREADS * HEAD + tid * V + 4 * e4) = pv[NC - 1][e4];
    }
  }
  if constexpr (D >= 2) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
    load_row(r0 + 1, b1, d1);
  }
  __syncthreads();  // p in LDS
  if constexpr (D == 0) {
    for (int r = r0; r < r1; ++r) {
      process(b0, d0);
      load_row(r + 1, b0, d0);
    }
  } else if constexpr (D == 1) {
    for (int r = r0; r < r1; r += 2) {
      load_row(r + 1, b1, d1);
      process(b0, d0);
      load_row(r + 2, b0, d0);
      if (r + 1 < r1) process(b1, d1);
    }
  } else {
    for (int r = r0; r < r1; r += 3) {
      load_row(r + 2, b2, d2);
      process(b0, d0);
      load_row(r + 3, b0, d0);
      if (r + 1 < r1) process(b1, d1);
      load_row(r + 4, b1, d1);
      if (r + 2 < r1) process(b2, d2);
    }
  }
  if (pqpart != nullptr && tid == 0) pqpart[(int64_t)b * pq_stride + blockIdx.x] = pq;
  float* yb = ypart + (int64_t)b * prob_stride + (int64_t)blockIdx.x * ks_stride;
#pragma unroll
  for (int k = 0; k < NC; ++k) {
    if (k < NC - 1 || last_ok) {
#pragma unroll
      for (int e = 0; e < V; e += 4)
        *reinterpret_cast<float4*>(yb + col(k) + e) =
            make_float4(y[k][e], y[k][e + 1], y[k][e + 2], y[k][e + 3]);
    }
  }
}

template <typename VT>
__global__ __launch_bounds__(256) void k_sum_splits(int64_t len, const VT* __restrict__ in,
                                                    int nsplit, int64_t split_stride,
                                                    int64_t psi, VT* __restrict__ out,
                                                    int64_t pso, const int32_t* __restrict__ gate,
                                                    int gate_stride) {
  const int b = blockIdx.y;
  if (gate != nullptr && gate[(int64_t)b * gate_stride] == 0) return;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < len;
       i += (int64_t)gridDim.x * blockDim.x) {
    const VT* src = in + (int64_t)b * psi + i;
    VT s = VT(0);
    int k = 0;
    for (; k + 16 <= nsplit; k += 16) {  // 16 loads in flight, then the adds in order
      VT tq[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) tq[q] = src[(int64_t)(k + q) * split_stride];
#pragma unroll
      for (int q = 0; q < 16; ++q) s += tq[q];
    }
    for (; k < nsplit; ++k) s += src[(int64_t)k * split_stride];
    out[(int64_t)b * pso + i] = s;
  }
}

hipError_t launch_sum_splits(VType vt, int64_t batch, int64_t len, const void* in, int nsplit,
                             int64_t split_stride, int64_t psi, void* out, int64_t pso,
                             hipStream_t st, const int32_t* gate, int gate_stride) {
  const unsigned nb = (unsigned)std::min<int64_t>((len + 255) / 256, 1024);
  dim3 grid(std::max(1u, nb), (unsigned)batch);
  if (vt == VT_F32)
    hipLaunchKernelGGL(k_sum_splits<float>, grid, dim3(256), 0, st, len,
                       static_cast<const float*>(in), nsplit, split_stride, psi,
                       static_cast<float*>(out), pso, gate, gate_stride);
  else
    hipLaunchKernelGGL(k_sum_splits<double>, grid, dim3(256), 0, st, len,
                       static_cast<const double*>(in), nsplit, split_stride, psi,
                       static_cast<double*>(out), pso, gate, gate_stride);
  return hipGetLastError();
}

// FP32 -> BF16, round to nearest even; NaN -> canonical quiet NaN 0x7FC0.
__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  const uint32_t x = __float_as_uint(f);
  if ((x & 0x7fffffffu) > 0x7f800000u) return 0x7fc0u;
  const uint32_t lsb = (x >> 16) & 1u;
  return static_cast<uint16_t>((x + 0x7fffu + lsb) >> 16);
}

__global__ __launch_bounds__(256) void k_cast_bf16(const float* __restrict__ src,
                                                   uint16_t* __restrict__ dst, int64_t count) {
  const int64_t stride = (int64_t)gridDim.x * blockDim.x * 8;
  for (int64_t i = ((int64_t)blockIdx.x * blockDim.x + threadIdx.x) * 8; i < count; i += stride) {
    if (i + 8 <= count && (reinterpret_cast<uintptr_t>(src + i) % 16 == 0) &&
        (reinterpret_cast<uintptr_t>(dst + i) % 16 == 0)) {
      const float4 a = *reinterpret_cast<const float4*>(src + i);
      const float4 b = *reinterpret_cast<const float4*>(src + i + 4);
      uint4 o;
      o.x = f32_to_bf16_rne(a.x) | (uint32_t(f32_to_bf16_rne(a.y)) << 16);
      o.y = f32_to_bf16_rne(a.z) | (uint32_t(f32_to_bf16_rne(a.w)) << 16);
      o.z = f32_to_bf16_rne(b.x) | (uint32_t(f32_to_bf16_rne(b.y)) << 16);
      o.w = f32_to_bf16_rne(b.z) | (uint32_t(f32_to_bf16_rne(b.w)) << 16);
      *reinterpret_cast<uint4*>(dst + i) = o;
    } else {
      for (int64_t k = i; k < count && k < i + 8; ++k) dst[k] = f32_to_bf16_rne(src[k]);
    }
  }
}

hipError_t launch_cast_bf16(const float* src, uint16_t* dst, int64_t count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const int64_t groups = (count + 7) / 8;
  const unsigned nb = (unsigned)std::min<int64_t>((groups + 255) / 256, 8192);
  hipLaunchKernelGGL(k_cast_bf16, dim3(nb), dim3(256), 0, st, src, dst, count);
  return hipGetLastError();
}

__global__ __launch_bounds__(256) void k_fill_zero(uint32_t* __restrict__ p, int64_t words) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < words;
       i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0u;
}

hipError_t launch_fill(void* p, size_t bytes, hipStream_t st) {
  if (bytes == 0) return hipSuccess;
  if (bytes % 4 != 0 || reinterpret_cast<uintptr_t>(p) % 4 != 0) return hipErrorInvalidValue;
  const int64_t words = (int64_t)(bytes / 4);
  const unsigned nb = (unsigned)std::min<int64_t>((words + 255) / 256, 4096);
  hipLaunchKernelGGL(k_fill_zero, dim3(nb), dim3(256), 0, st, static_cast<uint32_t*>(p), words);
  return hipGetLastError();
}

template <typename VT>
__global__ __launch_bounds__(256) void k_copy(const VT* __restrict__ s, VT* __restrict__ d,
                                              int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count;
       i += (int64_t)gridDim.x * blockDim.x)
    d[i] = s[i];
}

hipError_t launch_copy(VType vt, const void* src, void* dst, int64_t count, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  const unsigned nb = (unsigned)std::min<int64_t>((count + 255) / 256, 4096);
  if (vt == VT_F32)
    hipLaunchKernelGGL(k_copy<float>, dim3(nb), dim3(256), 0, st, static_cast<const float*>(src),
                       static_cast<float*>(dst), count);
  else
    hipLaunchKernelGGL(k_copy<double>, dim3(nb), dim3(256), 0, st,
                       static_cast<const double*>(src), static_cast<double*>(dst), count);
  return hipGetLastError();
}

// ---- fused Hessian-vector product: geometry and dispatch ----------------------

namespace {

constexpr int kHvpLdsBytes = 160 * 1024 - 1024;  // dynamic LDS for p; 1 KB for statics

template <typename T, int THREADS, int EPT, int D>
hipError_t hvp_launch_one(const MatArg& A, const HvpGeom& g, int64_t batch, const float* p,
                          int64_t p_stride, const float* d, int64_t d_stride, float* ypart,
                          int64_t ks_stride, int64_t prob_stride, const int32_t* gate,
                          int gate_stride, double* pq, int64_t pq_stride, hipStream_t st) {
  auto* fn = &k_hvp_fused<T, THREADS, EPT, D>;
  const size_t lds = (size_t)A.n * sizeof(float);
  static bool big_lds = false;  // the attribute is set once per instantiation
  if (lds > 64 * 1024 && !big_lds) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, kHvpLdsBytes);
    if (e != hipSuccess) return e;
    big_lds = true;
  }
  hipLaunchKernelGGL(fn, dim3((unsigned)g.blocks, (unsigned)batch), dim3(THREADS), lds, st,
                     static_cast<const T*>(A.ptr), A.lda, A.strideA, (int)A.m, (int)A.n, p,
                     p_stride, d, d_stride, ypart, ks_stride, prob_stride, gate, gate_stride, pq,
                     pq_stride);
  return hipGetLastError();
}

// Prefetch depth (rows in flight while one is processed): one row when every
// row the shape serves (n > THREADS (EPT - V)) is at least 24 KB, else two
// (measured, non-temporal loads: 20000 x 40000 BF16 6.17 against 5.96 TB/s with
// two rows ahead, 32000 x 16000 BF16 6.85 against 6.67; 20000 x 5000 FP32 with
// 1024 threads 6.38 with two), within the register budget of the block size:
// D + 1 packed row buffers plus the EPT owned results.
template <typename T, int THREADS, int EPT>
constexpr int hvp_depth() {
  constexpr int row_regs = EPT * (int)sizeof(T) / 4;
  constexpr int budget = THREADS >= 1024 ? 80 : 210;
  constexpr int min_row = THREADS * (EPT - Elem<T>::V) * (int)sizeof(T);
  constexpr int max_depth = min_row >= 24576 ? 1 : 2;
  return (max_depth >= 2 && 3 * row_regs + EPT <= budget)
             ? 2
             : ((2 * row_regs + EPT <= budget) ? 1 : 0);
}

template <typename T, int THREADS, int... E>
hipError_t hvp_dispatch(int ept, const MatArg& A, const HvpGeom& g, int64_t batch, const float* p,
                        int64_t p_stride, const float* d, int64_t d_stride, float* ypart,
                        int64_t ks_stride, int64_t prob_stride, const int32_t* gate,
                        int gate_stride, double* pq, int64_t pq_stride, hipStream_t st) {
  hipError_t r = hipErrorInvalidValue;
  bool hit = false;
  ((ept == E && !hit
        ? (hit = true,
           r = hvp_launch_one<T, THREADS, E, hvp_depth<T, THREADS, E>()>(
               A, g, batch, p, p_stride, d, d_stride, ypart, ks_stride, prob_stride, gate,
               gate_stride, pq, pq_stride, st))
        : r),
   ...);
  return r;
}

int num_cus() {
  static int cus = 0;
  if (cus == 0) {
    int dev = 0, v = 0;
    if (hipGetDevice(&dev) == hipSuccess &&
        hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) == hipSuccess && v > 0)
      cus = v;
    else
      cus = 256;
  }
  return cus;
}

}  // namespace

bool hvp_p_aligned(const void* p, int64_t p_stride, int64_t batch) {
  return reinterpret_cast<uintptr_t>(p) % 16 == 0 && (batch == 1 || p_stride % 4 == 0);
}

HvpGeom hvp_geometry(const MatArg& A, int64_t batch, bool query_device) {
  HvpGeom g{};
  if (A.mt == MT_F64 || A.m < 1 || A.n < 1) return g;
  const int V = A.mt == MT_BF16 ? 8 : 4;
  if (A.n % V || A.lda % V || (batch > 1 && A.strideA % V)) return g;
  if (reinterpret_cast<uintptr_t>(A.ptr) % 16) return g;
  if (A.n * (int64_t)sizeof(float) > kHvpLdsBytes) return g;
  // 256 threads (up to two blocks per CU) for short rows; 1024 threads while 8
  // owned columns per thread suffice (FP32 only: BF16 rows that short take the
  // 256-thread shape); beyond, one block of 512 threads per CU with up to 80 owned
  // columns.  Measured with non-temporal loads: 512 threads against 1024 at
  // 20000 x 40000 FP32 6.72 / 6.54 TB/s, at 32000 x 16000 BF16 6.85 / 6.77 and
  // FP32 6.75 / 6.67; at 20000 x 5000 BF16 two 256-thread blocks per CU 5.77
  // against four 4.82 (the block partials of H p grow with the grid), FP32 one
  // 1024-thread block 6.38 against four 256-thread blocks 5.50.
  const int e_small = A.mt == MT_BF16 ? 32 : 16;
  if (A.n <= 256 * e_small)
    g.threads = 256;
  else if (A.n <= 1024 * 8)
    g.threads = 1024;
  else
    g.threads = 512;
  g.ept = (int)(V * ((A.n + (int64_t)V * g.threads - 1) / ((int64_t)V * g.threads)));
  if (g.ept > 80) {
    g.threads = 0;
    return g;
  }
  g.rows = 1;
  int per_cu = 1;
  if (g.threads == 256)
    per_cu = (int)std::max<int64_t>(1, std::min<int64_t>(2, (160 * 1024) / (A.n * 4 + 1024)));
  const int cus = query_device ? num_cus() : 256;
  const int64_t cap = std::max<int64_t>(1, kHvpMaxBlocks / batch);
  const int64_t groups = (A.m + g.rows - 1) / g.rows;
  int64_t G = std::max<int64_t>(1, (int64_t)per_cu * cus / batch);
  G = std::min<int64_t>(G, std::min<int64_t>(cap, groups));
  // block g owns rows g, g + G, ... (G <= m: none is empty); the most any owns:
  g.rows_per_block = (int)((A.m + G - 1) / G);
  g.blocks = (int)G;
  return g;
}

hipError_t launch_hvp_fused(const MatArg& A, const HvpGeom& g, int64_t batch, const float* p,
                            int64_t p_stride, const float* d, int64_t d_stride, float* ypart,
                            int64_t ks_stride, int64_t prob_stride, const int32_t* gate,
                            int gate_stride, hipStream_t st, double* pq, int64_t pq_stride) {
  if (g.threads == 0 || g.blocks < 1 || g.blocks > kHvpMaxBlocks ||
      g.blocks > A.m || ks_stride < A.n ||  // every block owns a row
      !hvp_p_aligned(p, p_stride, batch))
    return hipErrorInvalidValue;
  if (A.mt == MT_BF16) {
    if (g.threads == 256)
      return hvp_dispatch<uint16_t, 256, 8, 16, 24, 32>(g.ept, A, g, batch, p, p_stride, d,
                                                           d_stride, ypart, ks_stride, prob_stride,
                                                           gate, gate_stride, pq, pq_stride, st);
    if (g.threads == 512)
      return hvp_dispatch<uint16_t, 512, 24, 32, 40, 48, 56, 64, 72, 80>(
          g.ept, A, g, batch, p, p_stride, d, d_stride, ypart, ks_stride, prob_stride, gate,
          gate_stride, pq, pq_stride, st);
    return hipErrorInvalidValue;
  }
  if (A.mt == MT_F32) {
    if (g.threads == 256)
      return hvp_dispatch<float, 256, 4, 8, 12, 16>(g.ept, A, g, batch, p, p_stride, d,
                                                       d_stride, ypart, ks_stride, prob_stride,
                                                       gate, gate_stride, pq, pq_stride, st);
    if (g.threads == 1024)
      return hvp_dispatch<float, 1024, 8>(g.ept, A, g, batch, p, p_stride, d, d_stride, ypart,
                                          ks_stride, prob_stride, gate, gate_stride, pq, pq_stride,
                                          st);
    return hvp_dispatch<float, 512, 20, 24, 28, 32, 36, 40, 44, 48, 52, 56, 60, 64, 68, 72, 76, 80>(
        g.ept, A, g, batch, p, p_stride, d, d_stride, ypart, ks_stride, prob_stride, gate,
        gate_stride, pq, pq_stride, st);
  }
  return hipErrorInvalidValue;
}

}  // namespace genios

