// Streaming read: the measurement reference for the HBM-bound kernels (not part
// of the method).  A block reads contiguous tiles of 256 threads x 8 16-byte
// words (32 KB) with non-temporal loads (as the products read A), all eight
// loads of a thread in flight before any is used, and steps through the buffer
// by the grid's tile stride; the XOR of the words a block read goes to
// out[block], so no load is dead.
#include "device.hpp"

namespace genios {

namespace {

constexpr int kStreamThreads = 256;
constexpr int kStreamUnroll = 8;

__global__ __launch_bounds__(kStreamThreads) void k_stream_read(const uint4* __restrict__ p,
                                                                int64_t words,
                                                                uint32_t* __restrict__ out) {
  constexpr int64_t tile = (int64_t)kStreamThreads * kStreamUnroll;
  uint32_t acc = 0;
  for (int64_t base = (int64_t)blockIdx.x * tile; base < words; base += (int64_t)gridDim.x * tile) {
    if (base + tile <= words) {
      uint4 v[kStreamUnroll];
#pragma unroll
      for (int k = 0; k < kStreamUnroll; ++k) v[k] = load_stream_u4(p + base + k * kStreamThreads + threadIdx.x);
#pragma unroll
      for (int k = 0; k < kStreamUnroll; ++k) acc ^= (v[k].x ^ v[k].y) ^ (v[k].z ^ v[k].w);
    } else {
      for (int k = 0; k < kStreamUnroll; ++k) {
        const int64_t i = base + k * kStreamThreads + threadIdx.x;
        if (i < words) {
          const uint4 a = load_stream_u4(p + i);
          acc ^= (a.x ^ a.y) ^ (a.z ^ a.w);
        }
      }
    }
  }
  __shared__ uint32_t red[kStreamThreads / 64];
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) acc ^= (uint32_t)__shfl_xor((int)acc, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
  __syncthreads();
  if (threadIdx.x == 0) out[blockIdx.x] = red[0] ^ red[1] ^ red[2] ^ red[3];
}

}  // namespace

int stream_read_blocks(int64_t bytes, int cus, int max_blocks) {
  const int64_t tiles = (bytes / 16 + (int64_t)kStreamThreads * kStreamUnroll - 1) /
                        ((int64_t)kStreamThreads * kStreamUnroll);
  const int64_t resident = 8 * (int64_t)(cus > 0 ? cus : 1);  // 8 blocks of 4 waves per CU
  return (int)std::max<int64_t>(1, std::min<int64_t>(tiles, std::min<int64_t>(resident, max_blocks)));
}

hipError_t launch_stream_read(const void* p, int64_t bytes, uint32_t* out, int blocks,
                              hipStream_t st) {
  hipLaunchKernelGGL(k_stream_read, dim3((unsigned)blocks), dim3(kStreamThreads), 0, st,
                     static_cast<const uint4*>(p), bytes / 16, out);
  return hipGetLastError();
}

}  // namespace genios
