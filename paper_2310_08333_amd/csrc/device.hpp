// Device-side helpers: element conversion, 16-byte vector loads, wave and block
// reductions, and the deterministic last-block reduction pattern.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "internal.hpp"

namespace genios {

__device__ __forceinline__ float bf16_bits_to_float(uint16_t h) {
  return __uint_as_float(static_cast<uint32_t>(h) << 16);
}

// 16-byte loads of the matrix, which every product streams once: non-temporal,
// so that A passes through the caches at the eviction end and leaves the
// vectors, partials and U resident (measured: a plain read of a 1.6 GB buffer
// runs at 6.2 TB/s, the same read non-temporal at 7.0 TB/s).
typedef uint32_t u32x4_t __attribute__((ext_vector_type(4)));
typedef float f32x4_t __attribute__((ext_vector_type(4)));
typedef double f64x2_t __attribute__((ext_vector_type(2)));
template <typename VEC>
__device__ __forceinline__ VEC load_stream(const void* p) {
  return __builtin_nontemporal_load(reinterpret_cast<const VEC*>(p));
}
__device__ __forceinline__ uint4 load_stream_u4(const void* p) {
  const u32x4_t q = load_stream<u32x4_t>(p);
  return make_uint4(q.x, q.y, q.z, q.w);
}
__device__ __forceinline__ float4 load_stream_f4(const void* p) {
  const f32x4_t q = load_stream<f32x4_t>(p);
  return make_float4(q.x, q.y, q.z, q.w);
}

template <typename T>
struct Elem;
template <>
struct Elem<uint16_t> {
  using Acc = float;
  static constexpr int V = 8;  // elements per 16-byte load
  __device__ static __forceinline__ float cvt(uint16_t x) { return bf16_bits_to_float(x); }
  __device__ static __forceinline__ void load(const uint16_t* p, float (&o)[8]) {
    const u32x4_t q = load_stream<u32x4_t>(p);
    o[0] = __uint_as_float(q.x << 16);
    o[1] = __uint_as_float(q.x & 0xffff0000u);
    o[2] = __uint_as_float(q.y << 16);
    o[3] = __uint_as_float(q.y & 0xffff0000u);
    o[4] = __uint_as_float(q.z << 16);
    o[5] = __uint_as_float(q.z & 0xffff0000u);
    o[6] = __uint_as_float(q.w << 16);
    o[7] = __uint_as_float(q.w & 0xffff0000u);
  }
};
template <>
struct Elem<float> {
  using Acc = float;
  static constexpr int V = 4;
  __device__ static __forceinline__ float cvt(float x) { return x; }
  __device__ static __forceinline__ void load(const float* p, float (&o)[4]) {
    const f32x4_t q = load_stream<f32x4_t>(p);
    o[0] = q.x;
    o[1] = q.y;
    o[2] = q.z;
    o[3] = q.w;
  }
};
template <>
struct Elem<double> {
  using Acc = double;
  static constexpr int V = 2;
  __device__ static __forceinline__ double cvt(double x) { return x; }
  __device__ static __forceinline__ void load(const double* p, double (&o)[2]) {
    const f64x2_t q = load_stream<f64x2_t>(p);
    o[0] = q.x;
    o[1] = q.y;
  }
};

// Load V consecutive vector entries (float or double) as Acc.
template <typename VT, typename Acc, int V>
__device__ __forceinline__ void load_vec(const VT* p, Acc (&o)[V]) {
  if constexpr (sizeof(VT) == 4 && V % 4 == 0) {
#pragma unroll
    for (int k = 0; k < V / 4; ++k) {
      const float4 q = reinterpret_cast<const float4*>(p)[k];
      o[4 * k + 0] = q.x;
      o[4 * k + 1] = q.y;
      o[4 * k + 2] = q.z;
      o[4 * k + 3] = q.w;
    }
  } else if constexpr (sizeof(VT) == 8 && V % 2 == 0) {
#pragma unroll
    for (int k = 0; k < V / 2; ++k) {
      const double2 q = reinterpret_cast<const double2*>(p)[k];
      o[2 * k + 0] = q.x;
      o[2 * k + 1] = q.y;
    }
  } else {
#pragma unroll
    for (int k = 0; k < V; ++k) o[k] = p[k];
  }
}

// The value of v in lane l (l uniform), as a wave-uniform scalar.
__device__ __forceinline__ double readlane_f64(double v, int l) {
  const unsigned long long b = (unsigned long long)__double_as_longlong(v);
  const unsigned lo = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b & 0xffffffffull), l);
  const unsigned hi = (unsigned)__builtin_amdgcn_readlane((int)(unsigned)(b >> 32), l);
  return __longlong_as_double((long long)(((unsigned long long)hi << 32) | lo));
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

// Sum NV doubles over a 256-thread block; the result is valid in thread 0.
template <int NV>
__device__ __forceinline__ void block_sum(double (&v)[NV], double* smem /* >= 4*NV */) {
  const int lane = threadIdx.x & 63, wave = threadIdx.x >> 6;
#pragma unroll
  for (int k = 0; k < NV; ++k) v[k] = wave_sum(v[k]);
  if (lane == 0) {
#pragma unroll
    for (int k = 0; k < NV; ++k) smem[wave * NV + k] = v[k];
  }
  __syncthreads();
  if (threadIdx.x == 0) {
    const int nw = blockDim.x >> 6;
#pragma unroll
    for (int k = 0; k < NV; ++k) {
      double s = 0.0;
      for (int w = 0; w < nw; ++w) s += smem[w * NV + k];
      v[k] = s;
    }
  }
  __syncthreads();
}

// Deterministic grid reduction: every block stores its partial, then the last
// block to arrive (integer atomic counter) sees all partials in a fixed order.
// Returns true in every thread of the last block, which also resets the counter.
__device__ __forceinline__ bool last_block_arrive(unsigned* counter, unsigned nblocks) {
  __shared__ int s_last;
  // every wave may have written partials: release them at agent scope first
  __threadfence();
  __syncthreads();
  if (threadIdx.x == 0) {
    __threadfence();
    const unsigned prev = atomicAdd(counter, 1u);
    s_last = (prev == nblocks - 1) ? 1 : 0;
  }
  __syncthreads();
  const bool last = s_last != 0;
  if (last) {
    __threadfence();
    if (threadIdx.x == 0) atomicExch(counter, 0u);
  }
  return last;
}

// Load of a partial written by another block of the same kernel.  Only used by
// the last block after last_block_arrive(), whose agent-scope acquire fence
// invalidates this CU's vector L1, so a plain (pipelined) load is coherent.
__device__ __forceinline__ double load_partial(const double* p) { return *p; }

}  // namespace genios
