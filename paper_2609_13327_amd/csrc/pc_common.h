// Shared device helpers for the gfx950 kernels: MFMA fragment types, the
// FP64 MFMA tile accumulator, reductions and rounding to bfloat16.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

namespace pc {

typedef double d4 __attribute__((ext_vector_type(4)));
typedef float f4 __attribute__((ext_vector_type(4)));
typedef short s8 __attribute__((ext_vector_type(8)));

constexpr int WAVE = 64;

__device__ __forceinline__ int lane_id() { return threadIdx.x & (WAVE - 1); }
__device__ __forceinline__ int wave_id() { return threadIdx.x / WAVE; }

// One v_mfma_f64_16x16x4 step.  Operand layout (64 lanes):
//   A (16 x 4): lane l holds A[l % 16][l / 16]
//   B (4 x 16): lane l holds B[l / 16][l % 16]
//   D (16 x 16): lane l holds D[l / 16 + 4 * v][l % 16], v = 0..3
//                (rows interleaved across the four lane groups; measured)
__device__ __forceinline__ d4 mfma_f64(double a, double b, d4 c) {
  return __builtin_amdgcn_mfma_f64_16x16x4f64(a, b, c, 0, 0, 0);
}

// v_mfma_f32_16x16x4_f32: A/B lane layout as the f64 form, fp32 operands.
__device__ __forceinline__ f4 mfma_f32(float a, float b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x4f32(a, b, c, 0, 0, 0);
}

// v_mfma_f32_16x16x32_bf16: lane l holds 8 consecutive k of row (A) or
// column (B) l % 16, k block l / 16; D fp32.
__device__ __forceinline__ f4 mfma_bf16(s8 a, s8 b, f4 c) {
  return __builtin_amdgcn_mfma_f32_16x16x32_bf16(a, b, c, 0, 0, 0);
}

// Round a binary64 value to the nearest bfloat16, ties to even, from the bit
// layouts: the binary64 significand is cut to 8 significant bits.  Values
// below the smallest normal bfloat16 (2^-126) become a signed zero; inputs
// are finite and far below the bfloat16 overflow threshold.
__device__ __forceinline__ unsigned short f64_to_bf16_rne(double x) {
  unsigned long long u = (unsigned long long)__double_as_longlong(x);
  unsigned short sign = (unsigned short)((u >> 48) & 0x8000u);
  int e = (int)((u >> 52) & 0x7ff);            // biased binary64 exponent
  if (e < 1023 - 126) return sign;             // |x| < 2^-126 (also zero)
  unsigned long long mant = u & 0xfffffffffffffULL;  // 52 fraction bits
  unsigned long long keep = mant >> 45;        // top 7 fraction bits
  unsigned long long rest = mant & ((1ULL << 45) - 1);
  const unsigned long long half = 1ULL << 44;
  if (rest > half || (rest == half && (keep & 1ULL))) keep += 1;
  int eb = e - 1023 + 127;                     // bfloat16 biased exponent
  if (keep == 128) { keep = 0; eb += 1; }      // carry into the exponent
  return (unsigned short)(sign | (unsigned short)(eb << 7) | (unsigned short)keep);
}

__device__ __forceinline__ float bf16_to_f32(unsigned short h) {
  return __uint_as_float(((unsigned int)h) << 16);
}

template <typename T>
__device__ __forceinline__ T wave_sum(T v) {
  for (int off = WAVE / 2; off > 0; off >>= 1) v += __shfl_xor(v, off, WAVE);
  return v;
}

template <typename T>
__device__ __forceinline__ T wave_max(T v) {
  for (int off = WAVE / 2; off > 0; off >>= 1) {
    T o = __shfl_xor(v, off, WAVE);
    v = v > o ? v : o;
  }
  return v;
}

// FP64 MFMA accumulator for a BM x BN workgroup tile computed by WM x WN
// waves; each wave owns a (BM/WM) x (BN/WN) sub-tile of 16x16 fragments.
// LDS operand layout: As[k][row] with row stride LDA, Bs[k][col] with stride LDB.
template <int BM, int BN, int WM, int WN>
struct TileF64 {
  static constexpr int TM = BM / WM, TN = BN / WN;
  static constexpr int FM = TM / 16, FN = TN / 16;
  static_assert(TM % 16 == 0 && TN % 16 == 0, "wave tile must be a multiple of 16");
  d4 acc[FM][FN];

  __device__ __forceinline__ void zero() {
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  }

  // Consume KC rows of k from LDS.  With XA (XB) the operand is stored
  // row-XOR swizzled: element (k, m) at k * LDA + (m ^ k), k < 16 (a
  // permutation inside each aligned group of 16 columns).
  template <int KC, int LDA, int LDB, bool XA = false, bool XB = false>
  __device__ __forceinline__ void mma(const double* As, const double* Bs) {
    static_assert((!XA && !XB) || KC <= 16, "the swizzle permutes within groups of 16");
    const int lane = lane_id(), w = wave_id();
    const int wm = w / WN, wn = w % WN;
    const int r = lane & 15, kq = lane >> 4;
#pragma unroll
    for (int kk = 0; kk < KC; kk += 4) {
      double a[FM], b[FN];
      const int k = kk + kq;
#pragma unroll
      for (int i = 0; i < FM; ++i) a[i] = As[k * LDA + wm * TM + i * 16 + (XA ? (r ^ k) : r)];
#pragma unroll
      for (int j = 0; j < FN; ++j) b[j] = Bs[k * LDB + wn * TN + j * 16 + (XB ? (r ^ k) : r)];
#pragma unroll
      for (int i = 0; i < FM; ++i)
#pragma unroll
        for (int j = 0; j < FN; ++j) acc[i][j] = mfma_f64(a[i], b[j], acc[i][j]);
    }
  }

  // Visit every accumulator element with its (row, col) inside the tile.
  template <typename F>
  __device__ __forceinline__ void for_each(F&& f) const {
    const int lane = lane_id(), w = wave_id();
    const int wm = w / WN, wn = w % WN;
#pragma unroll
    for (int i = 0; i < FM; ++i)
#pragma unroll
      for (int j = 0; j < FN; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int row = wm * TM + i * 16 + (lane >> 4) + 4 * v;
          const int col = wn * TN + j * 16 + (lane & 15);
          f(row, col, acc[i][j][v]);
        }
  }
};

}  // namespace pc
