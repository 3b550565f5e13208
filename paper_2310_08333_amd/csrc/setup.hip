// Set-up pass of a BF16-A solve in one stream of the FP32 master: the BF16 copy of
// A (round to nearest even) and the right-hand side c = A^T b of both operators
// (Sec. 3.1: grad f = A^T A x - A^T b), c_hi with A and c_lo with the rounded copy.
// A block owns 1024 columns (4 per thread, one 16-byte load per row) and a range of
// rows; it writes its rows of the copy and one FP32 partial of each column's sums
// per row split, summed afterwards in a fixed order.
#include <algorithm>

#include "device.hpp"

namespace genios {

namespace {

constexpr int kCastCols = 1024;  // columns per block (256 threads x 4)
constexpr int kCastUnroll = 4;   // rows in flight per thread

__device__ __forceinline__ uint32_t bf16_rne_bits(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return 0x7fc0u;  // NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return u >> 16;
}

// grid (column blocks, row splits, batch)
__global__ __launch_bounds__(256) void k_cast_atb(const float* __restrict__ A, int64_t lda,
                                                  int64_t strideA, uint16_t* __restrict__ A16,
                                                  int m, int n, int rchunk,
                                                  const float* __restrict__ bvec,
                                                  float* __restrict__ ypart, int64_t ks_stride,
                                                  int64_t lo_offset, int64_t prob_stride) {
  const int b = blockIdx.z, ks = blockIdx.y;
  const int j = blockIdx.x * kCastCols + 4 * threadIdx.x;
  const int r0 = ks * rchunk, r1 = min(m, r0 + rchunk);
  const bool col_ok = j < n;  // n is a multiple of 4: the whole float4 is in range
  const float* Ab = A + (int64_t)b * strideA;
  uint16_t* Db = A16 + (int64_t)b * strideA;
  const float* bb = bvec + (int64_t)b * m;
  float hi[4] = {0.f, 0.f, 0.f, 0.f}, lo[4] = {0.f, 0.f, 0.f, 0.f};
  const int jc = col_ok ? j : 0;
  for (int r = r0; r < r1; r += kCastUnroll) {
    float4 a[kCastUnroll];
    float br[kCastUnroll];
#pragma unroll
    for (int u = 0; u < kCastUnroll; ++u) {  // clamped rows are read, not used
      const int rr = min(r + u, r1 - 1);
      a[u] = load_stream_f4(Ab + (int64_t)rr * lda + jc);
      br[u] = bb[rr];
    }
#pragma unroll
    for (int u = 0; u < kCastUnroll; ++u) {
      if (r + u >= r1) break;
      const uint32_t h0 = bf16_rne_bits(a[u].x), h1 = bf16_rne_bits(a[u].y);
      const uint32_t h2 = bf16_rne_bits(a[u].z), h3 = bf16_rne_bits(a[u].w);
      if (col_ok) {
        uint2 o;
        o.x = h0 | (h1 << 16);
        o.y = h2 | (h3 << 16);
        *reinterpret_cast<uint2*>(Db + (int64_t)(r + u) * lda + j) = o;
      }
      const float bv = br[u];
      hi[0] += bv * a[u].x;
      hi[1] += bv * a[u].y;
      hi[2] += bv * a[u].z;
      hi[3] += bv * a[u].w;
      lo[0] += bv * __uint_as_float(h0 << 16);
      lo[1] += bv * __uint_as_float(h1 << 16);
      lo[2] += bv * __uint_as_float(h2 << 16);
      lo[3] += bv * __uint_as_float(h3 << 16);
    }
  }
  if (!col_ok) return;
  float* yb = ypart + (int64_t)b * prob_stride + (int64_t)ks * ks_stride + j;
  *reinterpret_cast<float4*>(yb) = make_float4(hi[0], hi[1], hi[2], hi[3]);
  *reinterpret_cast<float4*>(yb + lo_offset) = make_float4(lo[0], lo[1], lo[2], lo[3]);
}

}  // namespace

int cast_atb_splits(int64_t m, int64_t n, int64_t batch, int max_splits) {
  const int64_t cb = ((n + kCastCols - 1) / kCastCols) * batch;
  int64_t ks = (2048 + cb - 1) / cb;
  ks = std::min<int64_t>(ks, std::max<int64_t>(1, m / 64));
  return (int)std::max<int64_t>(1, std::min<int64_t>(ks, max_splits));
}

bool cast_atb_eligible(const void* A, int64_t lda, int64_t strideA, int64_t n, const void* A16,
                       const void* ypart, int64_t ks_stride) {
  return n % 4 == 0 && lda % 4 == 0 && strideA % 4 == 0 && ks_stride % 4 == 0 &&
         reinterpret_cast<uintptr_t>(A) % 16 == 0 && reinterpret_cast<uintptr_t>(A16) % 8 == 0 &&
         reinterpret_cast<uintptr_t>(ypart) % 16 == 0;
}

hipError_t launch_cast_atb(const float* A, int64_t lda, int64_t strideA, uint16_t* A16,
                           int64_t m, int64_t n, int64_t batch, const float* b, float* ypart,
                           int ksplit, int64_t ks_stride, int64_t lo_offset,
                           int64_t prob_stride, hipStream_t st) {
  if (ksplit < 1 || m < 1 || n < 1) return hipErrorInvalidValue;
  int rchunk = (int)((m + ksplit - 1) / ksplit);
  rchunk = (rchunk + kCastUnroll - 1) / kCastUnroll * kCastUnroll;
  dim3 grid((unsigned)((n + kCastCols - 1) / kCastCols), (unsigned)ksplit, (unsigned)batch);
  hipLaunchKernelGGL(k_cast_atb, grid, dim3(256), 0, st, A, lda, strideA, A16, (int)m, (int)n,
                     rchunk, b, ypart, ks_stride, lo_offset, prob_stride);
  return hipGetLastError();
}

}  // namespace genios
