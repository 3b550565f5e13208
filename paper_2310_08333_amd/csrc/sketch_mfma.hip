// Sketch products on the matrix cores (BF16 operand, FP32 accumulation).
//
// The Nystrom sketch Y = A^T diag(d) A Omega (Sec. 2.2, Sec. 3.3 for the
// logistic D) is two skinny products with s right-hand columns:
//   W = A Omega      (m x s, K = n)   k_sketch_w_mfma
//   Y = A^T (d o W)  (n x s, K = m)   k_sketch_y_mfma
// Each is bandwidth-bound on A (intensity s flop/B in BF16, below the MFMA
// ridge), so the goal is one HBM stream of A per product with the s-wide
// arithmetic on v_mfma_f32_16x16x32_bf16.
//
// Operand layout of that instruction (lane l of a wavefront): the A operand
// holds row l % 16, k = 8 (l / 16) + i; the B operand holds column l % 16,
// k = 8 (l / 16) + i; the 16x16 FP32 result holds row 4 (l / 16) + i, column
// l % 16 (i = 0..7 for the operands, 0..3 for the result).
//
// * Omega is rounded to BF16 once (k_omega_bf16), in place as well, so the
//   s x s core uses exactly the test matrix the products used; the BF16 copy is
//   column-major [c][k], zero past n and past s.
// * W = A Omega: a block owns 128 rows (a wavefront 32: two row tiles) and all
//   s columns for a K range; A fragments go straight from HBM to registers
//   (16 contiguous bytes of a row per lane), the Omega tile of each 32-wide K
//   step is staged in LDS (double-buffered) and shared by the four wavefronts.
// * d o W is split into BF16 hi + lo parts (k_w_split): the product with both
//   keeps ~16 significant bits of d o W, so Y carries FP32-level error.
// * Y = A^T (d o W): A's rows are contiguous in j, but the instruction needs 8
//   consecutive k = r per lane, so each 32-row x 128-column A tile is written
//   to LDS transposed ([j][r]) and read back as 16-byte fragments; the hi/lo
//   tiles of d o W are staged in LDS beside it.  A wavefront loads 16 rows x 4
//   column chunks, and row j of the transposed tile keeps its 32 entries at
//   positions rotated by 16 ((j / 8) mod 4) in a 72-wide row, so the 2-byte
//   stores of one instruction spread over all 32 banks and the fragment reads
//   still take the minimum two passes.
// Results are per-K-split partials, summed in a fixed order by the consumers.
//
// The same two products serve a batch of problems sharing one matrix: with
// P = [p_1 .. p_B] in place of Omega, T = A P and A^T (D o T) give every problem's
// H p for two streams of A (BF16: P and T as hi + lo parts; FP32 matrix: FP32
// operands on v_mfma_f32_16x16x4_f32, the second product formed as (T^T A)^T so
// that A's rows feed the instruction as loaded).
#include <algorithm>

#include "device.hpp"

namespace genios {

namespace {

typedef __attribute__((__vector_size__(8 * sizeof(__bf16)))) __bf16 bf16x8;
typedef __attribute__((__vector_size__(4 * sizeof(float)))) float floatx4;

constexpr int kMK = 32;        // K step of one instruction
constexpr int kPitch = 40;     // LDS row pitch in 16-bit elements (32 + 8: 80 bytes)
constexpr int kWRows = 128;    // rows of A per block in W = A Omega
constexpr int kYCols = 128;    // columns of A per block in Y = A^T W
constexpr int kPitchT = 72;    // LDS row pitch of the transposed A tile (16-bit elements)

__device__ __forceinline__ uint16_t f32_to_bf16_rne(float f) {
  uint32_t u = __float_as_uint(f);
  if ((u & 0x7f800000u) == 0x7f800000u && (u & 0x007fffffu)) return 0x7fc0;  // NaN
  u += 0x7fffu + ((u >> 16) & 1u);
  return (uint16_t)(u >> 16);
}

__device__ __forceinline__ bf16x8 as_bf16x8(const uint4& q) {
  return __builtin_bit_cast(bf16x8, q);
}

__device__ __forceinline__ floatx4 mfma(const uint4& a, const uint4& b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(as_bf16x8(a), as_bf16x8(b), c, 0, 0, 0);
}

// Omega (n x SP column-major, FP32) -> BF16 copy [c][kpad] (zero past n) and
// Omega rounded to the same values in place.
__global__ __launch_bounds__(256) void k_omega_bf16(int64_t n, int sp, int64_t kpad,
                                                    float* __restrict__ omega,
                                                    uint16_t* __restrict__ o16) {
  const int b = blockIdx.y;
  float* Ob = omega + (int64_t)b * n * sp;
  uint16_t* O16 = o16 + (int64_t)b * sp * kpad;
  const int64_t total = (int64_t)sp * kpad;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e / kpad);
    const int64_t k = e - (int64_t)c * kpad;
    uint16_t h = 0;
    if (k < n) {
      h = f32_to_bf16_rne(Ob[(int64_t)c * n + k]);
      Ob[(int64_t)c * n + k] = __uint_as_float((uint32_t)h << 16);
    }
    O16[e] = h;
  }
}

// True if any of the `count` flags (stride `gstride` ints) is set, or gate is NULL.
__device__ __forceinline__ bool any_flag(const int32_t* gate, int gstride, int count) {
  if (gate == nullptr) return true;
  __shared__ int s_any;
  if (threadIdx.x == 0) s_any = 0;
  __syncthreads();
  for (int i = threadIdx.x; i < count; i += blockDim.x)
    if (gate[(int64_t)i * gstride] != 0) s_any = 1;
  __syncthreads();
  return s_any != 0;
}

// Wpart[b][ks][c][r] = sum_{k in split ks} A[r][k] Omega[k][c]; with LO the operand is
// the sum of two BF16 parts (hi + lo of an FP32 block), both staged per step.
// A step covers KS = KC x 32 values of k: while the KC instructions per column tile
// of the current step run, the A fragments and the Omega tile [SP][KS] of the next
// step are in flight, so a block waits for memory once per KC instructions.  The
// Omega tile sits in dynamic LDS, row pitch KS + 8 (conflict-free 16-byte staging
// stores and fragment reads); tile chunks past kpad are stored as zeros.  Measured
// at 20000 x 40000, s = 128: 572 us with KS = 64 (four blocks per CU), 593 with 32,
// 645 with 128 (two blocks per CU: the 628 blocks take 1.23 rounds).
template <int SP, bool LO, int KS>
__global__ __launch_bounds__(256, 3) void k_sketch_w_mfma(const uint16_t* __restrict__ A,
                                                       int64_t lda, int64_t strideA, int m, int n,
                                                       const uint16_t* __restrict__ o16,
                                                       const uint16_t* __restrict__ o16lo,
                                                       int64_t kpad, float* __restrict__ wpart,
                                                       int kchunk, int64_t ks_stride,
                                                       int64_t prob_stride,
                                                       const int32_t* __restrict__ gate,
                                                       int gstride, int gcount) {
  constexpr int NT = SP / 16;     // column tiles
  constexpr int NO = LO ? 2 : 1;  // operand parts
  constexpr int KC = KS / kMK;    // instructions per column tile per step
  constexpr int PITCH = KS + 8;   // LDS row pitch, 16-bit elements
  constexpr int TILE = SP * PITCH;
  extern __shared__ __align__(16) uint16_t os_dyn[];  // [NO][2][SP][PITCH]
  auto os = [&](int o, int buf) { return os_dyn + (o * 2 + buf) * TILE; };
  if (!any_flag(gate, gstride, gcount)) return;
  const int b = blockIdx.z, ks = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int row0 = blockIdx.x * kWRows + wave * 32;
  const int k0 = ks * kchunk;
  const int k1 = min(n, k0 + kchunk);
  const uint16_t* Ab = A + (int64_t)b * strideA;
  const uint16_t* Obp[NO];
  Obp[0] = o16 + (int64_t)b * SP * kpad;
  if constexpr (LO) Obp[NO - 1] = o16lo + (int64_t)b * SP * kpad;
  // this lane's A rows (clamped: rows past m are computed but not stored)
  const uint16_t* arow[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) arow[t] = Ab + (int64_t)min(row0 + 16 * t + (lane & 15), m - 1) * lda;
  const int kl = 8 * (lane >> 4);  // this lane's k offset inside an instruction's 32
  floatx4 acc[2][NT];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int c = 0; c < NT; ++c) acc[t][c] = floatx4{0.f, 0.f, 0.f, 0.f};
  // Omega tile loader: SP columns x KS k = SP * KS / 8 chunks of 16 bytes; a thread's
  // chunks share one k offset (part), since 256 is a multiple of KS / 8
  constexpr int PARTS = KS / 8;
  constexpr int OCH = SP * PARTS;
  constexpr int OQ = (OCH + 255) / 256;
  static_assert(256 % PARTS == 0, "a thread's chunks share their k offset");
  const int part = tid % PARTS;
  // (loads are unconditional -- chunk indices past the tile re-read chunk 0, chunks
  // past kpad read offset 0 -- so the staging registers stay registers; the LDS
  // stores are guarded, and chunks past kpad are stored as zeros)
  auto load_omega = [&](int kk, uint4 (&reg)[NO][OQ]) {
    const int kof = kk + 8 * part + 8 <= kpad ? kk + 8 * part : 0;
#pragma unroll
    for (int o = 0; o < NO; ++o)
#pragma unroll
      for (int q = 0; q < OQ; ++q) {
        const int ch = tid + 256 * q < OCH ? tid + 256 * q : 0;
        reg[o][q] = *reinterpret_cast<const uint4*>(Obp[o] + (int64_t)(ch / PARTS) * kpad + kof);
      }
  };
  auto store_omega = [&](int kk, int buf, const uint4 (&reg)[NO][OQ]) {
    const bool in = kk + 8 * part + 8 <= kpad;
#pragma unroll
    for (int o = 0; o < NO; ++o)
#pragma unroll
      for (int q = 0; q < OQ; ++q) {
        const int ch = tid + 256 * q;
        if (ch < OCH)
          *reinterpret_cast<uint4*>(&os(o, buf)[(ch / PARTS) * PITCH + 8 * part]) =
              in ? reg[o][q] : make_uint4(0u, 0u, 0u, 0u);
      }
  };
  // A fragments of a step: columns past n read column 0 (their Omega rows are 0)
  auto load_a = [&](int kk, uint4 (&fa)[2][KC]) {
#pragma unroll
    for (int i = 0; i < KC; ++i) {
      const int k = kk + kMK * i + kl;
      const int kc = k < n ? k : 0;
#pragma unroll
      for (int t = 0; t < 2; ++t) fa[t][i] = *reinterpret_cast<const uint4*>(arow[t] + kc);
    }
  };
  uint4 oreg[NO][OQ];
  uint4 fa[2][KC], fn[2][KC];
  if (k0 < k1) {
    load_omega(k0, oreg);
    store_omega(k0, 0, oreg);
    load_a(k0, fa);
  }
  __syncthreads();
  int buf = 0;
  for (int kk = k0; kk < k1; kk += KS) {
    const bool more = kk + KS < k1;
    const int kn = more ? kk + KS : kk;  // the last step re-reads its own tile (unused)
    load_omega(kn, oreg);
    load_a(kn, fn);
#pragma unroll
    for (int i = 0; i < KC; ++i)
#pragma unroll
      for (int c = 0; c < NT; ++c) {
#pragma unroll
        for (int o = 0; o < NO; ++o) {
          const uint4 fb = *reinterpret_cast<const uint4*>(
              &os(o, buf)[(16 * c + (lane & 15)) * PITCH + kMK * i + kl]);
#pragma unroll
          for (int t = 0; t < 2; ++t) acc[t][c] = mfma(fa[t][i], fb, acc[t][c]);
        }
      }
    if (more) store_omega(kn, buf ^ 1, oreg);
    __syncthreads();
    buf ^= 1;
#pragma unroll
    for (int i = 0; i < KC; ++i) {
      fa[0][i] = fn[0][i];
      fa[1][i] = fn[1][i];
    }
  }
  float* Wb = wpart + (int64_t)b * prob_stride + (int64_t)ks * ks_stride;
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int c = 0; c < NT; ++c)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = row0 + 16 * t + 4 * (lane >> 4) + i;
        if (r < m) Wb[(int64_t)(16 * c + (lane & 15)) * m + r] = acc[t][c][i];
      }
}

// K step of the W product (both operand forms): 64, two instructions per column
// tile per step.
template <bool LO>
constexpr int w_step() {
  return 64;
}

// Launch of k_sketch_w_mfma with its dynamic LDS; the K range per split, a multiple
// of the step, is derived here from the split count.
template <int SP, bool LO>
hipError_t launch_w_mfma(dim3 grid, hipStream_t st, const uint16_t* A, int64_t lda,
                         int64_t strideA, int m, int n, const uint16_t* o16,
                         const uint16_t* o16lo, int64_t kpad, float* wpart, int splits,
                         int64_t ks_stride, int64_t prob_stride, const int32_t* gate, int gstride,
                         int gcount) {
  constexpr int KS = w_step<LO>();
  constexpr size_t lds = (size_t)(LO ? 2 : 1) * 2 * SP * (KS + 8) * sizeof(uint16_t);
  auto* fn = &k_sketch_w_mfma<SP, LO, KS>;
  static bool attr = false;  // set once per instantiation
  if (lds > 64 * 1024 && !attr) {
    hipError_t e = hipFuncSetAttribute(reinterpret_cast<const void*>(fn),
                                       hipFuncAttributeMaxDynamicSharedMemorySize, (int)lds);
    if (e != hipSuccess) return e;
    attr = true;
  }
  int kchunk = (int)((n + splits - 1) / splits);
  kchunk = (kchunk + KS - 1) / KS * KS;
  hipLaunchKernelGGL(fn, grid, dim3(256), lds, st, A, lda, strideA, m, n, o16, o16lo, kpad, wpart,
                     kchunk, ks_stride, prob_stride, gate, gstride, gcount);
  return hipGetLastError();
}

// (d o sum_ks Wpart) -> BF16 hi and lo parts [c][kpad], zero past m.  Column c < dcols
// is weighted by d + c d_cstride (d_cstride = 0: one d for every column).
__global__ __launch_bounds__(256) void k_w_split(int64_t m, int sp, int ksW,
                                                 const float* __restrict__ wpart,
                                                 int64_t ks_stride, int64_t prob_stride,
                                                 const float* __restrict__ d, int64_t d_stride,
                                                 int64_t d_cstride, int dcols,
                                                 int64_t kpad, uint16_t* __restrict__ hi,
                                                 uint16_t* __restrict__ lo,
                                                 const int32_t* __restrict__ gate, int gstride,
                                                 int gcount) {
  if (!any_flag(gate, gstride, gcount)) return;
  const int b = blockIdx.y;
  const float* Wp = wpart + (int64_t)b * prob_stride;
  const float* db = d ? d + (int64_t)b * d_stride : nullptr;
  uint16_t* H = hi + (int64_t)b * sp * kpad;
  uint16_t* L = lo + (int64_t)b * sp * kpad;
  const int64_t total = (int64_t)sp * kpad;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e / kpad);
    const int64_t r = e - (int64_t)c * kpad;
    uint16_t h = 0, l = 0;
    if (r < m) {
      float w = 0.f;
      for (int k = 0; k < ksW; ++k) w += Wp[(int64_t)k * ks_stride + (int64_t)c * m + r];
      if (db && c < dcols) w *= db[(int64_t)c * d_cstride + r];
      h = f32_to_bf16_rne(w);
      l = f32_to_bf16_rne(w - __uint_as_float((uint32_t)h << 16));
    }
    H[e] = h;
    L[e] = l;
  }
}

// Ypart[b][ks][c][j] = sum_{r in split ks} A[r][j] (hi + lo)[c][r]
template <int SP>
__global__ __launch_bounds__(256) void k_sketch_y_mfma(const uint16_t* __restrict__ A,
                                                       int64_t lda, int64_t strideA, int m, int n,
                                                       const uint16_t* __restrict__ whi,
                                                       const uint16_t* __restrict__ wlo,
                                                       int64_t kpad, float* __restrict__ ypart,
                                                       int rchunk, int64_t ks_stride,
                                                       int64_t prob_stride, int64_t ldy,
                                                       const int32_t* __restrict__ gate,
                                                       int gstride, int gcount) {
  constexpr int NT = SP / 16;
  __shared__ __align__(16) uint16_t at[kYCols * kPitchT];      // A tile transposed: [j][r]
  // hi, lo tiles [c][r], plus one spare row that threads past the tile write into
  // (never read), so every staging store is unconditional
  __shared__ __align__(16) uint16_t ws[2][(SP + 1) * kPitch];
  if (!any_flag(gate, gstride, gcount)) return;
  const int b = blockIdx.z, ks = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int j0 = blockIdx.x * kYCols;
  const int r0 = ks * rchunk;
  const int r1 = min(m, r0 + rchunk);
  const uint16_t* Ab = A + (int64_t)b * strideA;
  const uint16_t* Hb = whi + (int64_t)b * SP * kpad;
  const uint16_t* Lb = wlo + (int64_t)b * SP * kpad;
  const int kl = 8 * (lane >> 4);
  floatx4 acc[2][NT];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int c = 0; c < NT; ++c) acc[t][c] = floatx4{0.f, 0.f, 0.f, 0.f};
  // A tile: 32 rows x 128 columns = 512 chunks of 8 columns, 2 per thread:
  // thread -> rows tr = (lane mod 16) + 16 h (h = 0, 1), chunk tc = 4 wave + lane / 16.
  // Rows past m are clamped (their W rows are 0), chunks past n read column 0
  // (their results are not stored).
  const int tc = 4 * wave + (lane >> 4);
  // position of entry r of transposed row j (rotation by 16 ((j / 8) mod 4) in a 64 ring)
  auto tpos = [](int j, int r) { return j * kPitchT + ((r + 16 * ((j >> 3) & 3)) & 63); };
  for (int rr = r0; rr < r1; rr += kMK) {
    auto load_chunk = [&](int h) {
      const int tr = (lane & 15) + 16 * h;
      const int row = min(rr + tr, m - 1);
      const int j = j0 + 8 * tc;
      return *reinterpret_cast<const uint4*>(Ab + (int64_t)row * lda + (j < n ? j : 0));
    };
    const uint4 av0 = load_chunk(0), av1 = load_chunk(1);
    // hi / lo tiles: SP columns x 32 r each = WCH chunks of 16 bytes, at most two
    // per thread (named registers; chunk indices past the tile re-read chunk 0)
    constexpr int WCH = SP * 4;
    static_assert(WCH <= 512, "at most two staging chunks per thread");
    auto wchunk = [&](int ch) { return ch < WCH ? ch : 0; };
    auto wload = [&](const uint16_t* base, int ch) {
      const int c = wchunk(ch) >> 2, part = wchunk(ch) & 3;
      return *reinterpret_cast<const uint4*>(base + (int64_t)c * kpad + rr + 8 * part);
    };
    const uint4 wh0 = wload(Hb, tid), wl0 = wload(Lb, tid);
    uint4 wh1{}, wl1{};
    if constexpr (WCH > 256) {
      wh1 = wload(Hb, tid + 256);
      wl1 = wload(Lb, tid + 256);
    }
    __syncthreads();  // previous step's reads of the LDS tiles are done
    auto store_transposed = [&](int h, const uint4& v) {
      const int tr = (lane & 15) + 16 * h;
      // the 8 rows j = 8 tc .. 8 tc + 7 share (j / 8) mod 4 = tc mod 4
      uint16_t* dst = &at[(8 * tc) * kPitchT + ((tr + 16 * (tc & 3)) & 63)];
      dst[0 * kPitchT] = (uint16_t)(v.x & 0xffffu);
      dst[1 * kPitchT] = (uint16_t)(v.x >> 16);
      dst[2 * kPitchT] = (uint16_t)(v.y & 0xffffu);
      dst[3 * kPitchT] = (uint16_t)(v.y >> 16);
      dst[4 * kPitchT] = (uint16_t)(v.z & 0xffffu);
      dst[5 * kPitchT] = (uint16_t)(v.z >> 16);
      dst[6 * kPitchT] = (uint16_t)(v.w & 0xffffu);
      dst[7 * kPitchT] = (uint16_t)(v.w >> 16);
    };
    store_transposed(0, av0);
    store_transposed(1, av1);
    auto wstore = [&](int ch, const uint4& h, const uint4& l) {
      const int o = ch < WCH ? (ch >> 2) * kPitch + 8 * (ch & 3) : SP * kPitch;
      *reinterpret_cast<uint4*>(&ws[0][o]) = h;
      *reinterpret_cast<uint4*>(&ws[1][o]) = l;
    };
    wstore(tid, wh0, wl0);
    if constexpr (WCH > 256) wstore(tid + 256, wh1, wl1);
    __syncthreads();
    uint4 fa[2];
#pragma unroll
    for (int t = 0; t < 2; ++t)
      fa[t] = *reinterpret_cast<const uint4*>(&at[tpos(32 * wave + 16 * t + (lane & 15), kl)]);
#pragma unroll
    for (int c = 0; c < NT; ++c) {
      const uint4 fh = *reinterpret_cast<const uint4*>(&ws[0][(16 * c + (lane & 15)) * kPitch + kl]);
      const uint4 fl = *reinterpret_cast<const uint4*>(&ws[1][(16 * c + (lane & 15)) * kPitch + kl]);
#pragma unroll
      for (int t = 0; t < 2; ++t) {
        acc[t][c] = mfma(fa[t], fh, acc[t][c]);
        acc[t][c] = mfma(fa[t], fl, acc[t][c]);
      }
    }
  }
  float* Yb = ypart + (int64_t)b * prob_stride + (int64_t)ks * ks_stride;
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int c = 0; c < NT; ++c)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int j = j0 + 32 * wave + 16 * t + 4 * (lane >> 4) + i;
        if (j < n) Yb[(int64_t)(16 * c + (lane & 15)) * ldy + j] = acc[t][c][i];
      }
}

template <int SP>
hipError_t sketch_mfma_sp(const MatArg& A, int64_t batch, const float* d, int64_t d_stride,
                          const SketchWs& ws, hipStream_t st) {
  const int m = (int)A.m, n = (int)A.n;
  const uint16_t* Ap = static_cast<const uint16_t*>(A.ptr);
  const int64_t kpn = (A.n + kMK - 1) / kMK * kMK, kpm = (A.m + kMK - 1) / kMK * kMK;
  {
    const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((SP * kpn + 255) / 256, 2048));
    hipLaunchKernelGGL(k_omega_bf16, dim3(nb, (unsigned)batch), dim3(256), 0, st, A.n, SP, kpn,
                       static_cast<float*>(ws.omega), ws.o16);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  {
    dim3 grid((unsigned)((m + kWRows - 1) / kWRows), (unsigned)ws.ksW, (unsigned)batch);
    hipError_t e = launch_w_mfma<SP, false>(grid, st, Ap, A.lda, A.strideA, m, n, ws.o16,
                                            (const uint16_t*)nullptr, kpn,
                                            static_cast<float*>(ws.Wpart), ws.ksW,
                                            (int64_t)m * SP, (int64_t)ws.ksW * m * SP,
                                            (const int32_t*)nullptr, 0, 0);
    if (e != hipSuccess) return e;
  }
  {
    const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((SP * kpm + 255) / 256, 2048));
    hipLaunchKernelGGL(k_w_split, dim3(nb, (unsigned)batch), dim3(256), 0, st, A.m, SP, ws.ksW,
                       static_cast<const float*>(ws.Wpart), (int64_t)m * SP,
                       (int64_t)ws.ksW * m * SP, d, d_stride, (int64_t)0, SP, kpm, ws.w16,
                       ws.w16 + (size_t)batch * SP * kpm, (const int32_t*)nullptr, 0, 0);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  {
    int rchunk = (int)((A.m + ws.ksY - 1) / ws.ksY);
    rchunk = (rchunk + kMK - 1) / kMK * kMK;
    dim3 grid((unsigned)((n + kYCols - 1) / kYCols), (unsigned)ws.ksY, (unsigned)batch);
    hipLaunchKernelGGL(k_sketch_y_mfma<SP>, grid, dim3(256), 0, st, Ap, A.lda, A.strideA, m, n,
                       ws.w16, ws.w16 + (size_t)batch * SP * kpm, kpm,
                       static_cast<float*>(ws.Ypart), rchunk, (int64_t)n * SP,
                       (int64_t)ws.ksY * n * SP, (int64_t)n, (const int32_t*)nullptr, 0, 0);
    return hipGetLastError();
  }
}

// P (n x B FP32, column c at P + c pstride) -> BF16 hi and lo parts [c][kpad], zero
// past n and for the padding columns c >= B.
__global__ __launch_bounds__(256) void k_cols_split(int64_t n, int B, int sp,
                                                    const float* __restrict__ P, int64_t pstride,
                                                    int64_t kpad, uint16_t* __restrict__ hi,
                                                    uint16_t* __restrict__ lo,
                                                    const int32_t* __restrict__ gate, int gstride,
                                                    int gcount) {
  if (!any_flag(gate, gstride, gcount)) return;
  const int64_t total = (int64_t)sp * kpad;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e / kpad);
    const int64_t k = e - (int64_t)c * kpad;
    const float v = (c < B && k < n) ? P[(int64_t)c * pstride + k] : 0.f;
    const uint16_t h = f32_to_bf16_rne(v);
    hi[e] = h;
    lo[e] = f32_to_bf16_rne(v - __uint_as_float((uint32_t)h << 16));
  }
}

// ---- the same products with the FP32 operand (v_mfma_f32_16x16x4_f32) ----------
// A lane's 16-byte fragment of A holds 4 consecutive k; instruction i of a 16-wide
// K step takes component i, so lane group g = l / 16 covers k = 4 g + i and the
// other operand is read with the same k order.  P and T stay FP32: the products are
// FP32 products with FP32 accumulation, in another summation order than the fused
// kernel's.
constexpr int kFK = 16;       // K step (4 instructions)
constexpr int kFPitch = 20;   // LDS row pitch in floats (16 + 4: 80 bytes)
constexpr int kFYCols = 256;  // columns of A per block in A^T T (64 per wavefront)

__device__ __forceinline__ floatx4 mfma_f32(float a, float b, floatx4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

__device__ __forceinline__ float comp(const float4& v, int i) {
  return i == 0 ? v.x : i == 1 ? v.y : i == 2 ? v.z : v.w;
}

// P (n x B FP32, column c at P + c pstride) -> [c][kpad] FP32, zero past n and for the
// padding columns c >= B.
__global__ __launch_bounds__(256) void k_cols_f32(int64_t n, int B, int sp,
                                                  const float* __restrict__ P, int64_t pstride,
                                                  int64_t kpad, float* __restrict__ out,
                                                  const int32_t* __restrict__ gate, int gstride,
                                                  int gcount) {
  if (!any_flag(gate, gstride, gcount)) return;
  const int64_t total = (int64_t)sp * kpad;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e / kpad);
    const int64_t k = e - (int64_t)c * kpad;
    out[e] = (c < B && k < n) ? P[(int64_t)c * pstride + k] : 0.f;
  }
}

// Tpart[ks][c][r] = sum_{k in split ks} A[r][k] P[c][k]: a block owns 128 rows (a
// wavefront 32: two row tiles) and all SP columns for a K range, in steps of 32 k: a
// lane loads 8 consecutive k of its row (two 16-byte fragments, so the four lanes of a
// row read 128 contiguous bytes), and instruction (h, i) takes k = 8 g + 4 h + i.  The
// P tile of each step is staged in LDS (double-buffered) and shared by the four
// wavefronts.  kchunk is a multiple of 32; P entries at or past kpad read as 0.
constexpr int kFW = 32;       // K step of the FP32 W kernel
constexpr int kFWPitch = 36;  // its LDS row pitch in floats (32 + 4: 144 bytes)
template <int SP>
__global__ __launch_bounds__(256) void k_mrhs_w_f32(const float* __restrict__ A, int64_t lda,
                                                    int m, int n, const float* __restrict__ pc,
                                                    int64_t kpad, float* __restrict__ tpart,
                                                    int kchunk, int64_t ks_stride,
                                                    const int32_t* __restrict__ gate, int gstride,
                                                    int gcount) {
  constexpr int NT = SP / 16;
  __shared__ __align__(16) float os[2][SP * kFWPitch];
  if (!any_flag(gate, gstride, gcount)) return;
  const int ks = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int row0 = blockIdx.x * kWRows + wave * 32;
  const int k0 = ks * kchunk;
  const int k1 = min(n, k0 + kchunk);
  const float* arow[2];
#pragma unroll
  for (int t = 0; t < 2; ++t) arow[t] = A + (int64_t)min(row0 + 16 * t + (lane & 15), m - 1) * lda;
  const int kl = 8 * (lane >> 4);
  floatx4 acc[2][NT];
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int c = 0; c < NT; ++c) acc[t][c] = floatx4{0.f, 0.f, 0.f, 0.f};
  // P tile: SP columns x 32 k = SP * 8 chunks of 16 bytes (chunk indices past the tile
  // re-read chunk 0 and offsets at or past kpad read offset 0, then count as 0; only the
  // LDS stores are guarded)
  constexpr int OCH = SP * 8;
  constexpr int OQ = (OCH + 255) / 256;
  auto load_p = [&](int kk, float4 (&reg)[OQ]) {
#pragma unroll
    for (int q = 0; q < OQ; ++q) {
      const int ch = tid + 256 * q < OCH ? tid + 256 * q : 0;
      const int64_t k = kk + 4 * (ch & 7);
      const float4 v = *reinterpret_cast<const float4*>(pc + (int64_t)(ch >> 3) * kpad + (k < kpad ? k : 0));
      reg[q] = k < kpad ? v : make_float4(0.f, 0.f, 0.f, 0.f);
    }
  };
  auto store_p = [&](int buf, const float4 (&reg)[OQ]) {
#pragma unroll
    for (int q = 0; q < OQ; ++q) {
      const int ch = tid + 256 * q;
      if (ch < OCH) *reinterpret_cast<float4*>(&os[buf][(ch >> 3) * kFWPitch + 4 * (ch & 7)]) = reg[q];
    }
  };
  // columns past n read column 0 (their P rows are 0); n % 8 == 0 keeps a lane's 8 whole
  auto load_a = [&](int kk, float4 (&fa)[2][2]) {
    const int k = kk + kl;
    const int kc = k < n ? k : 0;
#pragma unroll
    for (int t = 0; t < 2; ++t)
#pragma unroll
      for (int h = 0; h < 2; ++h) fa[t][h] = *reinterpret_cast<const float4*>(arow[t] + kc + 4 * h);
  };
  float4 preg[OQ];
  float4 fa[2][2], fn[2][2];
  if (k0 < k1) {
    load_p(k0, preg);
    store_p(0, preg);
    load_a(k0, fa);
  }
  __syncthreads();
  int buf = 0;
  for (int kk = k0; kk < k1; kk += kFW) {
    const bool more = kk + kFW < k1;
    const int kn = more ? kk + kFW : kk;
    load_p(kn, preg);
    load_a(kn, fn);
#pragma unroll
    for (int c = 0; c < NT; ++c) {
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        const float4 fb =
            *reinterpret_cast<const float4*>(&os[buf][(16 * c + (lane & 15)) * kFWPitch + kl + 4 * h]);
#pragma unroll
        for (int i = 0; i < 4; ++i)
#pragma unroll
          for (int t = 0; t < 2; ++t)
            acc[t][c] = mfma_f32(comp(fa[t][h], i), comp(fb, i), acc[t][c]);
      }
    }
    if (more) store_p(buf ^ 1, preg);
    __syncthreads();
    buf ^= 1;
#pragma unroll
    for (int t = 0; t < 2; ++t) {
      fa[t][0] = fn[t][0];
      fa[t][1] = fn[t][1];
    }
  }
  float* Tb = tpart + (int64_t)ks * ks_stride;
#pragma unroll
  for (int t = 0; t < 2; ++t)
#pragma unroll
    for (int c = 0; c < NT; ++c)
#pragma unroll
      for (int i = 0; i < 4; ++i) {
        const int r = row0 + 16 * t + 4 * (lane >> 4) + i;
        if (r < m) Tb[(int64_t)(16 * c + (lane & 15)) * m + r] = acc[t][c][i];
      }
}

// d_c o sum_ks Tpart -> T [c][kpad] FP32, zero past m (column c < B weighted by
// d + c d_stride when d is given).
__global__ __launch_bounds__(256) void k_t_sum_f32(int64_t m, int sp, int ksW,
                                                   const float* __restrict__ tpart,
                                                   int64_t ks_stride, const float* __restrict__ d,
                                                   int64_t d_stride, int B, int64_t kpad,
                                                   float* __restrict__ T,
                                                   const int32_t* __restrict__ gate, int gstride,
                                                   int gcount) {
  if (!any_flag(gate, gstride, gcount)) return;
  const int64_t total = (int64_t)sp * kpad;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int c = (int)(e / kpad);
    const int64_t r = e - (int64_t)c * kpad;
    float w = 0.f;
    if (r < m) {
      for (int k = 0; k < ksW; ++k) w += tpart[(int64_t)k * ks_stride + (int64_t)c * m + r];
      if (d && c < B) w *= d[(int64_t)c * d_stride + r];
    }
    T[e] = w;
  }
}

// Ypart[ks][c][j] = sum_{r in split ks} T[c][r] A[r][j], formed as (T^T A)^T so that
// A's rows feed the second operand unchanged: lane group g loads rows 4 g + s
// (s = 0..3) of a 16-row step, 4 consecutive columns per lane, and instruction
// (s, q) pairs component s of the T fragment with component q of row s's A
// fragment; result column l % 16 of sub-tile q is j = 4 (l % 16) + q.  The T tile
// of each step is staged in LDS (double-buffered); the next step's A fragments are
// loaded before this step's instructions.
template <int SP>
__global__ __launch_bounds__(256) void k_mrhs_y_f32(const float* __restrict__ A, int64_t lda,
                                                    int m, int n, const float* __restrict__ T,
                                                    int64_t kpad, float* __restrict__ ypart,
                                                    int rchunk, int64_t ks_stride, int64_t ldy,
                                                    const int32_t* __restrict__ gate, int gstride,
                                                    int gcount) {
  constexpr int NT = SP / 16;
  __shared__ __align__(16) float ts[2][SP * kFPitch];
  if (!any_flag(gate, gstride, gcount)) return;
  const int ks = blockIdx.y;
  const int tid = threadIdx.x, lane = tid & 63, wave = tid >> 6;
  const int jl = blockIdx.x * kFYCols + 64 * wave + 4 * (lane & 15);  // this lane's 4 columns
  const int jc = jl < n ? jl : 0;  // columns past n read column 0 (not stored)
  const int r0 = ks * rchunk;
  const int r1 = min(m, r0 + rchunk);
  const int g4 = 4 * (lane >> 4);
  floatx4 acc[NT][4];
#pragma unroll
  for (int c = 0; c < NT; ++c)
#pragma unroll
    for (int q = 0; q < 4; ++q) acc[c][q] = floatx4{0.f, 0.f, 0.f, 0.f};
  constexpr int OCH = SP * 4;
  constexpr int OQ = (OCH + 255) / 256;
  auto load_t = [&](int rr, float4 (&reg)[OQ]) {
#pragma unroll
    for (int q = 0; q < OQ; ++q) {
      const int ch = tid + 256 * q < OCH ? tid + 256 * q : 0;
      reg[q] = *reinterpret_cast<const float4*>(T + (int64_t)(ch >> 2) * kpad + rr + 4 * (ch & 3));
    }
  };
  auto store_t = [&](int buf, const float4 (&reg)[OQ]) {
#pragma unroll
    for (int q = 0; q < OQ; ++q) {
      const int ch = tid + 256 * q;
      if (ch < OCH) *reinterpret_cast<float4*>(&ts[buf][(ch >> 2) * kFPitch + 4 * (ch & 3)]) = reg[q];
    }
  };
  // rows past m are clamped (their T entries are 0)
  auto load_a = [&](int rr, float4 (&fa)[4]) {
#pragma unroll
    for (int s = 0; s < 4; ++s)
      fa[s] = *reinterpret_cast<const float4*>(A + (int64_t)min(rr + g4 + s, m - 1) * lda + jc);
  };
  float4 treg[OQ];
  float4 fa[4], fn[4];
  if (r0 < r1) {
    load_t(r0, treg);
    store_t(0, treg);
    load_a(r0, fa);
  }
  __syncthreads();
  int buf = 0;
  for (int rr = r0; rr < r1; rr += kFK) {
    const bool more = rr + kFK < r1;
    const int rn = more ? rr + kFK : rr;
    load_t(rn, treg);
    load_a(rn, fn);
#pragma unroll
    for (int c = 0; c < NT; ++c) {
      const float4 ft = *reinterpret_cast<const float4*>(&ts[buf][(16 * c + (lane & 15)) * kFPitch + g4]);
#pragma unroll
      for (int s = 0; s < 4; ++s)
#pragma unroll
        for (int q = 0; q < 4; ++q) acc[c][q] = mfma_f32(comp(ft, s), comp(fa[s], q), acc[c][q]);
    }
    if (more) store_t(buf ^ 1, treg);
    __syncthreads();
    buf ^= 1;
#pragma unroll
    for (int s = 0; s < 4; ++s) fa[s] = fn[s];
  }
  if (jl >= n) return;
  float* Yb = ypart + (int64_t)ks * ks_stride;
#pragma unroll
  for (int c = 0; c < NT; ++c)
#pragma unroll
    for (int i = 0; i < 4; ++i) {
      const int col = 16 * c + g4 + i;
      *reinterpret_cast<float4*>(Yb + (int64_t)col * ldy + jl) =
          make_float4(acc[c][0][i], acc[c][1][i], acc[c][2][i], acc[c][3][i]);
    }
}

// H p for B problems sharing A (FP32): T = A P, then (T^T A)^T, both on the matrix
// cores in FP32; P and T [c][kpad] FP32 in the space of the BF16 hi + lo parts.
template <int SP>
hipError_t mrhs_f32_sp(const MatArg& A, int B, const float* P, int64_t pstride, const float* d,
                       int64_t d_stride, const MrhsWs& ws, float* ypart, int64_t ldy,
                       const int32_t* gate, int gstride, hipStream_t st) {
  const int m = (int)A.m, n = (int)A.n;
  const float* Ap = static_cast<const float*>(A.ptr);
  const int64_t kpn = (A.n + kMK - 1) / kMK * kMK, kpm = (A.m + kMK - 1) / kMK * kMK;
  float* pc = reinterpret_cast<float*>(ws.p16);
  float* tc = reinterpret_cast<float*>(ws.w16);
  {
    const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((SP * kpn + 255) / 256, 2048));
    hipLaunchKernelGGL(k_cols_f32, dim3(nb), dim3(256), 0, st, A.n, B, SP, P, pstride, kpn, pc,
                       gate, gstride, B);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  {
    int kchunk = (int)((A.n + ws.ksW - 1) / ws.ksW);
    kchunk = (kchunk + kFW - 1) / kFW * kFW;
    dim3 grid((unsigned)((m + kWRows - 1) / kWRows), (unsigned)ws.ksW, 1u);
    hipLaunchKernelGGL(k_mrhs_w_f32<SP>, grid, dim3(256), 0, st, Ap, A.lda, m, n, pc, kpn,
                       ws.wpart, kchunk, (int64_t)m * SP, gate, gstride, B);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  {
    const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((SP * kpm + 255) / 256, 2048));
    hipLaunchKernelGGL(k_t_sum_f32, dim3(nb), dim3(256), 0, st, A.m, SP, ws.ksW, ws.wpart,
                       (int64_t)m * SP, d, d_stride, B, kpm, tc, gate, gstride, B);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  int rchunk = (int)((A.m + ws.ksYf - 1) / ws.ksYf);
  rchunk = (rchunk + kMK - 1) / kMK * kMK;
  dim3 grid((unsigned)((n + kFYCols - 1) / kFYCols), (unsigned)ws.ksYf, 1u);
  hipLaunchKernelGGL(k_mrhs_y_f32<SP>, grid, dim3(256), 0, st, Ap, A.lda, m, n, tc, kpm, ypart,
                     rchunk, (int64_t)SP * ldy, ldy, gate, gstride, B);
  return hipGetLastError();
}

// H p for B problems sharing A (BF16), H = A^T diag(d_c) A for problem c when d is given
// (d_c at d + c d_stride): T = A [p_1 .. p_B] (P in BF16 hi + lo parts, one
// pass over A), then A^T (T in BF16 hi + lo parts, one pass): two streams of A for
// all B right-hand sides.  Output: ypart[ks][c][j] with column stride ldy.
template <int SP>
hipError_t mrhs_sp(const MatArg& A, int B, const float* P, int64_t pstride, const float* d,
                   int64_t d_stride, const MrhsWs& ws, float* ypart, int64_t ldy,
                   const int32_t* gate, int gstride, hipStream_t st) {
  const int m = (int)A.m, n = (int)A.n;
  const uint16_t* Ap = static_cast<const uint16_t*>(A.ptr);
  const int64_t kpn = (A.n + kMK - 1) / kMK * kMK, kpm = (A.m + kMK - 1) / kMK * kMK;
  uint16_t* ph = ws.p16;
  uint16_t* pl = ws.p16 + (size_t)SP * kpn;
  uint16_t* th = ws.w16;
  uint16_t* tl = ws.w16 + (size_t)SP * kpm;
  {
    const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((SP * kpn + 255) / 256, 2048));
    hipLaunchKernelGGL(k_cols_split, dim3(nb), dim3(256), 0, st, A.n, B, SP, P, pstride, kpn, ph,
                       pl, gate, gstride, B);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  {
    dim3 grid((unsigned)((m + kWRows - 1) / kWRows), (unsigned)ws.ksW, 1u);
    hipError_t e = launch_w_mfma<SP, true>(grid, st, Ap, A.lda, (int64_t)0, m, n, ph, pl, kpn,
                                           ws.wpart, ws.ksW, (int64_t)m * SP,
                                           (int64_t)ws.ksW * m * SP, gate, gstride, B);
    if (e != hipSuccess) return e;
  }
  {
    const unsigned nb = (unsigned)std::max<int64_t>(1, std::min<int64_t>((SP * kpm + 255) / 256, 2048));
    hipLaunchKernelGGL(k_w_split, dim3(nb, 1u), dim3(256), 0, st, A.m, SP, ws.ksW, ws.wpart,
                       (int64_t)m * SP, (int64_t)ws.ksW * m * SP, d, (int64_t)0, d_stride,
                       B, kpm, th, tl, gate, gstride, B);
    hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  int rchunk = (int)((A.m + ws.ksY - 1) / ws.ksY);
  rchunk = (rchunk + kMK - 1) / kMK * kMK;
  dim3 grid((unsigned)((n + kYCols - 1) / kYCols), (unsigned)ws.ksY, 1u);
  hipLaunchKernelGGL(k_sketch_y_mfma<SP>, grid, dim3(256), 0, st, Ap, A.lda, (int64_t)0, m, n, th,
                     tl, kpm, ypart, rchunk, (int64_t)SP * ldy, (int64_t)0, ldy, gate, gstride,
                     B);
  return hipGetLastError();
}

}  // namespace

int mrhs_pad(int B) { return B <= 16 ? 16 : B <= 32 ? 32 : B <= 64 ? 64 : 128; }

bool mrhs_eligible(const MatArg& A, VType vt, int64_t B, const MrhsWs& ws) {
  return vt == VT_F32 && (A.mt == MT_BF16 || A.mt == MT_F32) && A.strideA == 0 && B >= 2 &&
         B <= 128 && ws.p16 != nullptr && ws.sp == mrhs_pad((int)B) && A.n % 8 == 0 &&
         A.lda % 8 == 0 && reinterpret_cast<uintptr_t>(A.ptr) % 16 == 0;
}

hipError_t launch_mrhs_hvp(const MatArg& A, int B, const float* P, int64_t pstride,
                           const float* d, int64_t d_stride, const MrhsWs& ws, float* ypart,
                           int64_t ldy, const int32_t* gate, int gstride, hipStream_t st) {
  if (A.mt == MT_F32) {
    switch (ws.sp) {
      case 16: return mrhs_f32_sp<16>(A, B, P, pstride, d, d_stride, ws, ypart, ldy, gate, gstride, st);
      case 32: return mrhs_f32_sp<32>(A, B, P, pstride, d, d_stride, ws, ypart, ldy, gate, gstride, st);
      case 64: return mrhs_f32_sp<64>(A, B, P, pstride, d, d_stride, ws, ypart, ldy, gate, gstride, st);
      case 128: return mrhs_f32_sp<128>(A, B, P, pstride, d, d_stride, ws, ypart, ldy, gate, gstride, st);
      default: return hipErrorInvalidValue;
    }
  }
  switch (ws.sp) {
    case 16: return mrhs_sp<16>(A, B, P, pstride, d, d_stride, ws, ypart, ldy, gate, gstride, st);
    case 32: return mrhs_sp<32>(A, B, P, pstride, d, d_stride, ws, ypart, ldy, gate, gstride, st);
    case 64: return mrhs_sp<64>(A, B, P, pstride, d, d_stride, ws, ypart, ldy, gate, gstride, st);
    case 128: return mrhs_sp<128>(A, B, P, pstride, d, d_stride, ws, ypart, ldy, gate, gstride, st);
    default: return hipErrorInvalidValue;
  }
}

bool sketch_mfma_eligible(const MatArg& A, VType vt, const SketchWs& ws) {
  return vt == VT_F32 && A.mt == MT_BF16 && ws.o16 != nullptr && ws.w16 != nullptr &&
         A.n % 8 == 0 && A.lda % 8 == 0 && A.strideA % 8 == 0 &&
         reinterpret_cast<uintptr_t>(A.ptr) % 16 == 0;
}

hipError_t launch_sketch_mfma(const MatArg& A, int64_t batch, int sp, const float* d,
                              int64_t d_stride, const SketchWs& ws, hipStream_t st) {
  switch (sp) {
    case 16: return sketch_mfma_sp<16>(A, batch, d, d_stride, ws, st);
    case 32: return sketch_mfma_sp<32>(A, batch, d, d_stride, ws, st);
    case 64: return sketch_mfma_sp<64>(A, batch, d, d_stride, ws, st);
    case 128: return sketch_mfma_sp<128>(A, batch, d, d_stride, ws, st);
    default: return hipErrorInvalidValue;
  }
}

}  // namespace genios
