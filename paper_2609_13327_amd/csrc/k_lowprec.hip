// Reduced-precision Gram: the Gram of ONE rounded copy of Z,
//     Zt[i, (k,m)] = round(z),   Gt = Zt^T Zt  on MFMA, fp32 accumulation,
// stored in FP64.  Z (and Zt) is never stored: every operand tile is formed
// while it is staged into LDS.  Rounding Z itself (each product once, not
// diag(s) W) keeps Gt the Gram of an elementwise-perturbed Z, so FP64
// refinement on the least-squares residual contracts at a rate set by
// kappa(Z) * u_low rather than kappa(Z)^2 * u_low.
//
// What z is rounded from:
//   fp32:           z = E[i, k] * W[j(i), m] in FP64, rounded once to fp32;
//   bf16, bf16x3:   z = fl32(E32[i, k] * W32[j(i), m]), the fp32 product of
//                   fp32 copies of E and W (rounded to nearest even once per
//                   plan), then rounded to bf16.  The fp32 product carries a
//                   relative error of at most 3 * 2^-24, far below the bf16
//                   rounding (2^-9) it feeds; forming it costs one fp32
//                   multiply and half a packed conversion per element, which
//                   keeps the formation (repeated for every tile an element
//                   enters) from dominating the bf16 MFMAs.
//
// Split bfloat16 (three products): z = hi + lo with hi = bf16(z) and
// lo = bf16(z - hi) (the subtraction is exact in fp32), and
//     Gt = Hi^T Hi + Hi^T Lo + Lo^T Hi
// accumulated in fp32 (the Lo^T Lo term, 2^-16 relative, is dropped): the
// operand error falls from 2^-9 to about 2^-17 for three bf16 products.
//
// Accumulation: the MFMAs accumulate in fp32 over at most 256 rows of the
// contraction at a time; each such partial Gram is then added into an FP64
// accumulator.  A single fp32 sum over all n rows would carry a relative
// error of about u32 sqrt(n) (1e-5 measured at n = 131072, mostly on the
// diagonal), a perturbation that is not the Gram of a perturbed Z, and
// refinement then contracts at kappa(Z)^2 * 1e-5 instead of kappa(Z) u_low;
// with 256-row partials it is about u32 * 256 / sqrt(n).
//
// Tiles are 128 x 128 of the lower triangle (a0 >= b0): four waves own
// 64 x 64 quadrants.  Accumulator layout of the f32 16x16 MFMAs (measured):
// lane l holds rows 4 * (l / 16) + v, column l % 16.
#include "pc_common.h"
#include "pc_internal.h"

#include <algorithm>

namespace pc {

constexpr int LT = 128;
constexpr int LP_BF16 = 2, LP_FP32 = 1, LP_BF16X3 = 3;   // the pc_precision codes
constexpr int FLUSH_ROWS = 256;                          // contraction rows per fp32 partial

// acc64 += acc32, acc32 = 0 (the fp32 partial Gram into the FP64 accumulator)
template <int TI, int TJ>
__device__ __forceinline__ void flush_partial(f4 (&acc)[TI][TJ], double (&acc64)[TI][TJ][4]) {
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
#pragma unroll
      for (int v = 0; v < 4; ++v) acc64[i][j][v] += (double)acc[i][j][v];
      acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
    }
}

__device__ __forceinline__ void lower_tile(int64_t t, int64_t& ta, int64_t& tb) {
  int64_t a = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((a + 1) * (a + 2) / 2 <= t) ++a;
  while (a * (a + 1) / 2 > t) --a;
  ta = a;
  tb = t - a * (a + 1) / 2;
}

// Store the lower-triangle part of a 128 x 128 FP64 accumulator tile held by
// waves of TI x TJ MFMA blocks (16 x 16): this wave's block (i, j) covers
// rows b0 + r0 + 16 i .. and columns a0 + c0 + 16 j ...
template <int TI, int TJ>
__device__ __forceinline__ void store_tile(const LowGramInst& g, int64_t a0, int64_t b0, int r0, int c0,
                                           const double (&acc64)[TI][TJ][4]) {
  const int lane = lane_id(), r = lane & 15, kq = lane >> 4;
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t b = b0 + r0 + i * 16 + 4 * kq + v;   // row of the product = lower index
        const int64_t a = a0 + c0 + j * 16 + r;            // column = higher index
        if (a < g.KM && b < g.KM && a >= b) g.G[a + b * g.ldG] = acc64[i][j][v];
      }
}

// ---------------------------------------------------------------- bf16 (and split bf16)
// Contraction rows per stage: two 32-row MFMA steps, so that each
// workgroup has twice the operand bytes of a 32-row stage in flight while
// the MFMAs of the previous stage run (the stage loop waits on load latency,
// not on the MFMAs).  Padded LDS row stride in bf16 elements.
constexpr int BKC = 64, KH = BKC / 32, BST = BKC + 8;
static_assert(BKC == kLowRowPad, "the fp32 copies are padded to whole stages");

typedef float f2v __attribute__((ext_vector_type(2)));
typedef __bf16 b2v __attribute__((ext_vector_type(2)));

// Two fp32 values to a packed pair of bf16 (round to nearest even).
__device__ __forceinline__ unsigned pack_bf16(float x, float y) {
  return __builtin_bit_cast(unsigned, __builtin_convertvector(f2v{x, y}, b2v));
}
__device__ __forceinline__ float lo_half_f32(unsigned p) { return __uint_as_float(p << 16); }
__device__ __forceinline__ float hi_half_f32(unsigned p) { return __uint_as_float(p & 0xffff0000u); }

// Raw fp32 values of 8 consecutive rows of one Z column: the member column
// e (rows i0 ..) and the mode column w (rows j0 ..).  WM: how the rows j of
// W follow the rows i of Z: 0: j = i (one level); 1: j = i mod n_h with n_h a
// multiple of 8 (the 8 rows never wrap); 2: the 8 rows may wrap (one by one).
struct Raw8 { float4 e0, e1, w0, w1; };

template <int WM>
__device__ __forceinline__ void load8(const float* e, const float* w, int64_t j0, int64_t n_h, Raw8& r) {
  r.e0 = *reinterpret_cast<const float4*>(e);
  r.e1 = *reinterpret_cast<const float4*>(e + 4);
  if constexpr (WM < 2) {
    r.w0 = *reinterpret_cast<const float4*>(w + j0);
    r.w1 = *reinterpret_cast<const float4*>(w + j0 + 4);
  } else {
    float v[8];
    int64_t j = j0;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      v[q] = w[j];
      if (++j == n_h) j = 0;
    }
    r.w0 = float4{v[0], v[1], v[2], v[3]};
    r.w1 = float4{v[4], v[5], v[6], v[7]};
  }
}

// The fp32 products z = e w of the 8 rows packed to bf16 (hi) and, for the
// split form, the packed remainders bf16(z - hi) (lo).
template <bool X3>
__device__ __forceinline__ void form8(const Raw8& r, s8& hi, s8& lo) {
  const float z[8] = {r.e0.x * r.w0.x, r.e0.y * r.w0.y, r.e0.z * r.w0.z, r.e0.w * r.w0.w,
                      r.e1.x * r.w1.x, r.e1.y * r.w1.y, r.e1.z * r.w1.z, r.e1.w * r.w1.w};
  unsigned h[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) h[q] = pack_bf16(z[2 * q], z[2 * q + 1]);
  hi = __builtin_bit_cast(s8, h);
  if constexpr (X3) {
    unsigned l[4];
#pragma unroll
    for (int q = 0; q < 4; ++q)
      l[q] = pack_bf16(z[2 * q] - lo_half_f32(h[q]), z[2 * q + 1] - hi_half_f32(h[q]));
    lo = __builtin_bit_cast(s8, l);
  }
}

// Waves per workgroup of the bf16 tiles: 2 x (BF_WAVES / 2), each wave owns
// 64 rows x (256 / BF_WAVES) columns of the 128 x 128 tile; a thread stages
// BF_NH columns per side.
constexpr int BF_WAVES = 8;
constexpr int BF_THREADS = 64 * BF_WAVES;
constexpr int BF_NH = 8 / BF_WAVES;

// One 128 x 128 tile (a0.., b0..) of the lower triangle, a0 >= b0, from the
// staged fp32 copies (E32: ldE32 rows, zero beyond n, and a zero column K
// used for the columns beyond K M).  X3: the split-bf16 form (hi and lo
// operands, three products).  Thread t stages rows 32 h + 8 (t % 4) .. (h
// < KH) of the chunk for tile column t / 4 on both sides.  The loads of
// chunk c + 1 are issued before the MFMAs of chunk c and formed into the
// other LDS buffer after them.
template <bool X3, int WM>
__device__ __forceinline__ void gram_bf16_tile_w(const LowGramInst& g, int64_t a0, int64_t b0,
                                                 unsigned short (&As)[2][X3 ? 2 : 1][LT * BST],
                                                 unsigned short (&Bs)[2][X3 ? 2 : 1][LT * BST]) {
  constexpr int NP = X3 ? 2 : 1;   // operand parts in LDS: hi (and lo)
  constexpr int WN = BF_WAVES / 2, CW = 128 / WN;   // waves along the columns, columns per wave
  const int t = threadIdx.x, lane = lane_id(), w = wave_id();
  const int wm = w / WN, wn = w % WN, r = lane & 15, kq = lane >> 4;
  const int seg = t & 3, col = t >> 2;           // 8-row segment of each 32-row half, first tile column
  const float* pe[2][BF_NH];
  const float* pw[2][BF_NH];
#pragma unroll
  for (int side = 0; side < 2; ++side)
#pragma unroll
    for (int h = 0; h < BF_NH; ++h) {
      const int64_t c = (side ? a0 : b0) + col + (128 / BF_NH) * h;
      int64_t k = g.K, m = 0;                      // beyond the last column: the zero member column
      if (c < g.KM) { k = c / g.M; m = c - k * g.M; }
      pe[side][h] = g.E32 + k * g.ldE32;
      pw[side][h] = g.W32 + m * g.ldW32;
    }
  const int64_t nchunks = g.ldE32 / BKC;         // ldE32 is a multiple of BKC (zero rows beyond n)
  int64_t jn = (int64_t)seg * 8 % g.n_h;         // W row of the next stage's first half (n_w > 1)
  auto load = [&](int64_t c, Raw8 (&raw)[2][BF_NH][KH]) {
    int64_t jh = jn;
#pragma unroll
    for (int hh = 0; hh < KH; ++hh) {
      const int64_t i0 = c * BKC + hh * 32 + seg * 8;
      const int64_t j0 = WM == 0 ? i0 : jh;
#pragma unroll
      for (int h = 0; h < BF_NH; ++h) {
        load8<WM>(pe[0][h] + i0, pw[0][h], j0, g.n_h, raw[0][h][hh]);
        load8<WM>(pe[1][h] + i0, pw[1][h], j0, g.n_h, raw[1][h][hh]);
      }
      if constexpr (WM != 0) {
        jh += 32;
        while (jh >= g.n_h) jh -= g.n_h;
      }
    }
    if constexpr (WM != 0) {
      jn += BKC;
      while (jn >= g.n_h) jn -= g.n_h;
    }
  };
  auto convert_store = [&](const Raw8 (&raw)[2][BF_NH][KH], int buf) {
#pragma unroll
    for (int hh = 0; hh < KH; ++hh)
#pragma unroll
      for (int h = 0; h < BF_NH; ++h) {
        const int o = (col + (128 / BF_NH) * h) * BST + hh * 32 + seg * 8;
        s8 hi, lo;
        form8<X3>(raw[0][h][hh], hi, lo);
        *reinterpret_cast<s8*>(&As[buf][0][o]) = hi;
        if constexpr (X3) *reinterpret_cast<s8*>(&As[buf][NP - 1][o]) = lo;
        form8<X3>(raw[1][h][hh], hi, lo);
        *reinterpret_cast<s8*>(&Bs[buf][0][o]) = hi;
        if constexpr (X3) *reinterpret_cast<s8*>(&Bs[buf][NP - 1][o]) = lo;
      }
  };
  constexpr int TI = 4, TJ = CW / 16;            // this wave: rows wm*64 + 16 i, columns wn*CW + 16 j
  f4 acc[TI][TJ];
  double acc64[TI][TJ][4];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
      acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int v = 0; v < 4; ++v) acc64[i][j][v] = 0.0;
    }
  auto mma = [&](int buf) {
#pragma unroll
    for (int hh = 0; hh < KH; ++hh) {
      const int ko = hh * 32 + kq * 8;
      s8 af[TI], bf[TJ];
#pragma unroll
      for (int i = 0; i < TI; ++i) af[i] = *reinterpret_cast<const s8*>(&As[buf][0][(wm * 64 + i * 16 + r) * BST + ko]);
#pragma unroll
      for (int j = 0; j < TJ; ++j) bf[j] = *reinterpret_cast<const s8*>(&Bs[buf][0][(wn * CW + j * 16 + r) * BST + ko]);
      if constexpr (X3) {
        s8 al[TI], bl[TJ];
#pragma unroll
        for (int i = 0; i < TI; ++i)
          al[i] = *reinterpret_cast<const s8*>(&As[buf][NP - 1][(wm * 64 + i * 16 + r) * BST + ko]);
#pragma unroll
        for (int j = 0; j < TJ; ++j)
          bl[j] = *reinterpret_cast<const s8*>(&Bs[buf][NP - 1][(wn * CW + j * 16 + r) * BST + ko]);
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
          for (int j = 0; j < TJ; ++j) {
            acc[i][j] = mfma_bf16(al[i], bf[j], acc[i][j]);   // small terms first
            acc[i][j] = mfma_bf16(af[i], bl[j], acc[i][j]);
            acc[i][j] = mfma_bf16(af[i], bf[j], acc[i][j]);
          }
      } else {
#pragma unroll
        for (int i = 0; i < TI; ++i)
#pragma unroll
          for (int j = 0; j < TJ; ++j) acc[i][j] = mfma_bf16(af[i], bf[j], acc[i][j]);
      }
    }
  };
  Raw8 ra[2][BF_NH][KH];
  load(0, ra);
  convert_store(ra, 0);
  __syncthreads();
  for (int64_t c = 0; c < nchunks; ++c) {
    const bool more = c + 1 < nchunks;
    if (more) load(c + 1, ra);
    mma((int)(c & 1));
    if ((c + 1) % (FLUSH_ROWS / BKC) == 0) flush_partial(acc, acc64);
    if (more) convert_store(ra, (int)((c + 1) & 1));
    __syncthreads();
  }
  flush_partial(acc, acc64);
  store_tile(g, a0, b0, wm * 64, wn * CW, acc64);
}

template <bool X3>
__device__ __forceinline__ void gram_bf16_tile(const LowGramInst& g, int64_t a0, int64_t b0) {
  constexpr int NP = X3 ? 2 : 1;
  __shared__ __attribute__((aligned(16))) unsigned short As[2][NP][LT * BST];   // rows b (lower index block)
  __shared__ __attribute__((aligned(16))) unsigned short Bs[2][NP][LT * BST];   // cols a
  if (g.n_w == 1) gram_bf16_tile_w<X3, 0>(g, a0, b0, As, Bs);
  else if (g.n_h % 8 == 0) gram_bf16_tile_w<X3, 1>(g, a0, b0, As, Bs);
  else gram_bf16_tile_w<X3, 2>(g, a0, b0, As, Bs);
}

// ---------------------------------------------------------------- fp32
// 24 contraction rows per stage (6 per thread): half as many again operand
// bytes in flight per workgroup as a 16-row stage, at 224 registers per lane
// (32 rows would spill).  A partial covers F_FLUSH stages (240 rows).
constexpr int FKC = 24, FR = FKC / 4, FST = FKC + 1;
constexpr int F_FLUSH = FLUSH_ROWS / FKC;

// Raw FP64 values of FR consecutive rows of one Z column.
struct RawF { double e[FR], w[FR]; };

// One 128 x 128 tile of the fp32 Gram: the FP64 products rounded once to
// fp32 (IEEE round to nearest even), fp32 MFMAs, 240-row partials into FP64.
// 8 waves (2 x 4, each 64 x 32); thread t stages rows FR (t % 4) .. of a
// chunk for tile column t / 4 on both sides.  The loads of chunk
// c + 1 are issued before the MFMAs of chunk c and converted after them.
// ONE: n_w = 1 and every chunk but a ragged last one is read as contiguous
// rows without checks; otherwise each row is checked and j = i mod n_h.
template <bool ONE, class WS>
__device__ __forceinline__ void gram_f32_tile_w(const LowGramInst& g, WS ws, int64_t a0, int64_t b0,
                                                float (&As)[2][LT * FST], float (&Bs)[2][LT * FST]) {
  const int t = threadIdx.x, lane = lane_id(), w = wave_id();
  const int wm = w >> 2, wn = w & 3, r = lane & 15, kq = lane >> 4;
  const int seg = t & 3, col = t >> 2;
  const double* pe[2];
  int64_t mc[2];
  bool valid[2];
#pragma unroll
  for (int side = 0; side < 2; ++side) {
    const int64_t c = (side ? a0 : b0) + col;
    valid[side] = c < g.KM;
    int64_t k = 0, m = 0;
    if (valid[side]) { k = c / g.M; m = c - k * g.M; }
    pe[side] = g.E + k * g.ldE;
    mc[side] = m;
  }
  const int64_t nchunks = (g.n + FKC - 1) / FKC;
  const int64_t nfull = ONE ? g.n / FKC : 0;     // chunks read without row checks
  int64_t jn = (int64_t)seg * FR % g.n_h;        // row of W for the next chunk to load (checked path)
  RawF raw[2];
  auto load = [&](int64_t c) {
    const int64_t i0 = c * FKC + seg * FR;
    if (ONE && c < nfull) {
#pragma unroll
      for (int side = 0; side < 2; ++side)
#pragma unroll
        for (int q = 0; q < FR; ++q) {
          raw[side].e[q] = pe[side][i0 + q];
          raw[side].w[q] = ws(i0 + q, mc[side]);
        }
      return;
    }
    int64_t j = ONE ? i0 : jn;
#pragma unroll
    for (int q = 0; q < FR; ++q) {
      const bool in = i0 + q < g.n;
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        raw[side].e[q] = in ? pe[side][i0 + q] : 0.0;
        raw[side].w[q] = in ? ws(j, mc[side]) : 0.0;
      }
      if (++j == g.n_h) j = 0;
    }
    if (!ONE) {
      jn += FKC;
      while (jn >= g.n_h) jn -= g.n_h;
    }
  };
  auto convert_store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < FR; ++q) {
      As[buf][col * FST + seg * FR + q] = valid[0] ? (float)(raw[0].e[q] * raw[0].w[q]) : 0.f;
      Bs[buf][col * FST + seg * FR + q] = valid[1] ? (float)(raw[1].e[q] * raw[1].w[q]) : 0.f;
    }
  };
  constexpr int TI = 4, TJ = 2;
  f4 acc[TI][TJ];
  double acc64[TI][TJ][4];
#pragma unroll
  for (int i = 0; i < TI; ++i)
#pragma unroll
    for (int j = 0; j < TJ; ++j) {
      acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int v = 0; v < 4; ++v) acc64[i][j][v] = 0.0;
    }
  load(0);
  convert_store(0);
  __syncthreads();
  for (int64_t c = 0; c < nchunks; ++c) {
    const bool more = c + 1 < nchunks;
    if (more) load(c + 1);
    const float* Ab = As[c & 1];
    const float* Bb = Bs[c & 1];
#pragma unroll
    for (int kk = 0; kk < FKC; kk += 4) {
      float af[TI], bf[TJ];
#pragma unroll
      for (int i = 0; i < TI; ++i) af[i] = Ab[(wm * 64 + i * 16 + r) * FST + kk + kq];
#pragma unroll
      for (int j = 0; j < TJ; ++j) bf[j] = Bb[(wn * 32 + j * 16 + r) * FST + kk + kq];
#pragma unroll
      for (int i = 0; i < TI; ++i)
#pragma unroll
        for (int j = 0; j < TJ; ++j) acc[i][j] = mfma_f32(af[i], bf[j], acc[i][j]);
    }
    if ((c + 1) % F_FLUSH == 0) flush_partial(acc, acc64);
    if (more) convert_store((int)((c + 1) & 1));
    __syncthreads();
  }
  flush_partial(acc, acc64);
  store_tile(g, a0, b0, wm * 64, wn * 32, acc64);
}

__device__ __forceinline__ void gram_f32_tile(const LowGramInst& g, int64_t a0, int64_t b0) {
  __shared__ float As[2][LT * FST];
  __shared__ float Bs[2][LT * FST];
  if (g.W) {
    const WDense ws{g.W, g.ldW};
    if (g.n_w == 1) gram_f32_tile_w<true>(g, ws, a0, b0, As, Bs);
    else gram_f32_tile_w<false>(g, ws, a0, b0, As, Bs);
  } else {
    const WSep ws{g.U, g.ldU, g.Phi, g.ldPhi, g.n_lon, g.inv_lon};
    if (g.n_w == 1) gram_f32_tile_w<true>(g, ws, a0, b0, As, Bs);
    else gram_f32_tile_w<false>(g, ws, a0, b0, As, Bs);
  }
}

template <int MODE>
__device__ __forceinline__ void gram_lp_tile(const LowGramInst& g, int64_t a0, int64_t b0) {
  if constexpr (MODE == LP_FP32) gram_f32_tile(g, a0, b0);
  else gram_bf16_tile<MODE == LP_BF16X3>(g, a0, b0);
}

template <int MODE>
constexpr int lp_threads() { return MODE == LP_FP32 ? 512 : BF_THREADS; }

// One instance: workgroup b takes tile tiles[b] = (tile row, tile column) of
// the lower triangle, in the order of lowgram_tile_order.
template <int MODE>
__global__ __launch_bounds__(lp_threads<MODE>()) void gram_lowprec_kernel(LowGramInst g,
                                                                        const int* __restrict__ tiles) {
  gram_lp_tile<MODE>(g, (int64_t)tiles[2 * blockIdx.x] * LT, (int64_t)tiles[2 * blockIdx.x + 1] * LT);
}

// Several instances in one launch: workgroup b takes tiles[b] (instance,
// tile row, tile column); the host lists the tiles longest contraction first,
// so the short ones fill the end of the launch.  Tiles of instances whose
// mode differs from the launch's are skipped (mode[inst] != MODE).
template <int MODE>
__global__ __launch_bounds__(lp_threads<MODE>()) void gram_lowprec_batch_kernel(
    const LowGramTile* __restrict__ tiles, const LowGramInst* __restrict__ insts, const int* __restrict__ mode) {
  const LowGramTile tl = tiles[blockIdx.x];
  if (mode[tl.inst] != MODE) return;
  const LowGramInst g = insts[tl.inst];
  gram_lp_tile<MODE>(g, (int64_t)tl.ta * LT, (int64_t)tl.tb * LT);
}

// Order of the lower-triangle tiles (ta >= tb) of a K M x K M Gram in
// 128-column blocks.  When 128 divides M, block t holds member t / (M/128)
// and the 128 modes of mode block t % (M/128): the tiles are grouped by the
// (unordered) pair of mode blocks they read, so the workgroups running at
// one time share those columns of W in the caches; inside a group, tiles
// sharing their column block a follow each other.  Otherwise plain row order.
std::vector<int> lowgram_tile_order(int64_t KM, int64_t M) {
  const int64_t T = ceil_div(KM, LT);
  std::vector<int> out;
  out.reserve((size_t)(T * (T + 1)));
  if (M % LT != 0) {
    for (int64_t a = 0; a < T; ++a)
      for (int64_t b = 0; b <= a; ++b) { out.push_back((int)a); out.push_back((int)b); }
    return out;
  }
  const int64_t nb = M / LT, K = KM / M;
  for (int64_t p = 0; p < nb; ++p)
    for (int64_t q = p; q < nb; ++q)
      for (int64_t ka = 0; ka < K; ++ka)
        for (int64_t kb = 0; kb < K; ++kb) {
          // the tiles with mode blocks {p, q}: (ka q, kb p) and (ka p, kb q)
          const int64_t cand[2][2] = {{ka * nb + q, kb * nb + p}, {ka * nb + p, kb * nb + q}};
          for (int v = 0; v < (p == q ? 1 : 2); ++v) {
            const int64_t a = cand[v][0], b = cand[v][1];
            if (a >= b) { out.push_back((int)a); out.push_back((int)b); }
          }
        }
  return out;
}

static LowGramInst lowgram_args(const Inst& in) {
  const WSep sep = wsep(in);
  return LowGramInst{in.E, in.ldE, in.W, in.ldW, in.U, in.ldU, in.Phi, in.ldPhi, in.n_lon, sep.inv,
                     in.E32, in.ldE32, in.W32, in.ldW32, in.n, in.n_h, in.n_w, in.K, in.M, in.KM, in.G, in.KMp};
}

// fp32 copies of E and W for the bf16 forms (round to nearest even); the
// padding (rows beyond n and n_h, the zero member column K) is never written.
__global__ __launch_bounds__(256) void stage_f32_kernel(const double* __restrict__ A, int64_t ldA, int64_t rows,
                                                        int64_t cols, float* __restrict__ B, int64_t ldB) {
  const int64_t total = rows * cols;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t c = e / rows, i = e - c * rows;
    B[i + c * ldB] = (float)A[i + c * ldA];
  }
}

// The fp32 copy of the modes, from either source (the FP64 value rounded once).
template <class WS>
__global__ __launch_bounds__(256) void stage_w32_kernel(WS w, int64_t n_h, int64_t M, float* __restrict__ B,
                                                        int64_t ldB) {
  const int64_t total = n_h * M;
  for (int64_t e = (int64_t)blockIdx.x * 256 + threadIdx.x; e < total; e += (int64_t)gridDim.x * 256) {
    const int64_t m = e / n_h, j = e - m * n_h;
    B[j + m * ldB] = (float)w(j, m);
  }
}

hipError_t launch_stage_f32(const Inst& in, hipStream_t s) {
  if (!in.E32 || !in.W32) return hipErrorInvalidValue;
  const unsigned ge = (unsigned)std::min<int64_t>(ceil_div(in.n * in.K, 256), 8192);
  hipLaunchKernelGGL(stage_f32_kernel, dim3(ge), dim3(256), 0, s, in.E, in.ldE, in.n, in.K, in.E32, in.ldE32);
  const unsigned gw = (unsigned)std::min<int64_t>(ceil_div(in.n_h * in.M, 256), 8192);
  if (in.W)
    hipLaunchKernelGGL(stage_w32_kernel<WDense>, dim3(gw), dim3(256), 0, s, wdense(in), in.n_h, in.M, in.W32,
                       in.ldW32);
  else
    hipLaunchKernelGGL(stage_w32_kernel<WSep>, dim3(gw), dim3(256), 0, s, wsep(in), in.n_h, in.M, in.W32,
                       in.ldW32);
  return hipGetLastError();
}

LowGramBatch* make_lowgram_batch(const std::vector<Inst>& insts) {
  std::vector<LowGramInst> hi(insts.size());
  std::vector<LowGramTile> ht;
  for (size_t i = 0; i < insts.size(); ++i) {
    const Inst& in = insts[i];
    hi[i] = lowgram_args(in);
    const std::vector<int> order = lowgram_tile_order(in.KM, in.M);
    for (size_t u = 0; u + 1 < order.size(); u += 2) ht.push_back(LowGramTile{(int)i, order[u], order[u + 1], 0});
  }
  std::stable_sort(ht.begin(), ht.end(), [&](const LowGramTile& x, const LowGramTile& y) {
    return insts[x.inst].n > insts[y.inst].n;
  });
  LowGramBatch* b = new LowGramBatch{};
  b->ntiles = (int64_t)ht.size();
  b->count = (int)insts.size();
  hipError_t e = hipMalloc((void**)&b->tiles, sizeof(LowGramTile) * ht.size());
  if (e == hipSuccess) e = hipMalloc((void**)&b->insts, sizeof(LowGramInst) * hi.size());
  if (e == hipSuccess) e = hipMalloc((void**)&b->mode, sizeof(int) * hi.size());
  if (e == hipSuccess) e = hipMemcpy(b->tiles, ht.data(), sizeof(LowGramTile) * ht.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(b->insts, hi.data(), sizeof(LowGramInst) * hi.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    free_lowgram_batch(b);
    return nullptr;
  }
  return b;
}

void free_lowgram_batch(LowGramBatch* b) {
  if (!b) return;
  (void)hipFree(b->tiles);
  (void)hipFree(b->insts);
  (void)hipFree(b->mode);
  delete b;
}

hipError_t set_lowgram_modes(const LowGramBatch* b, const int* modes, hipStream_t s) {
  return hipMemcpyAsync(b->mode, modes, sizeof(int) * (size_t)b->count, hipMemcpyHostToDevice, s);
}

hipError_t launch_gram_lowprec_batch(const LowGramBatch* b, int precision, hipStream_t s) {
  if (b->ntiles <= 0) return hipSuccess;
  const dim3 grid((unsigned)b->ntiles);
  if (precision == LP_BF16)
    hipLaunchKernelGGL(gram_lowprec_batch_kernel<LP_BF16>, grid, dim3(lp_threads<LP_BF16>()), 0, s, b->tiles,
                       b->insts, b->mode);
  else if (precision == LP_BF16X3)
    hipLaunchKernelGGL(gram_lowprec_batch_kernel<LP_BF16X3>, grid, dim3(lp_threads<LP_BF16X3>()), 0, s, b->tiles,
                       b->insts, b->mode);
  else if (precision == LP_FP32)
    hipLaunchKernelGGL(gram_lowprec_batch_kernel<LP_FP32>, grid, dim3(lp_threads<LP_FP32>()), 0, s, b->tiles,
                       b->insts, b->mode);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_gram_lowprec(const Inst& in, int precision, hipStream_t s) {
  if (!in.lp_tiles || in.lp_ntiles <= 0) return hipErrorInvalidValue;
  const dim3 grid((unsigned)in.lp_ntiles);
  const LowGramInst g = lowgram_args(in);
  if (precision == LP_BF16)
    hipLaunchKernelGGL(gram_lowprec_kernel<LP_BF16>, grid, dim3(lp_threads<LP_BF16>()), 0, s, g, in.lp_tiles);
  else if (precision == LP_BF16X3)
    hipLaunchKernelGGL(gram_lowprec_kernel<LP_BF16X3>, grid, dim3(lp_threads<LP_BF16X3>()), 0, s, g, in.lp_tiles);
  else if (precision == LP_FP32)
    hipLaunchKernelGGL(gram_lowprec_kernel<LP_FP32>, grid, dim3(lp_threads<LP_FP32>()), 0, s, g, in.lp_tiles);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace pc
