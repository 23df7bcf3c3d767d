// Reduced-precision Gram: the Gram of ONE rounded copy of Z,
//     Zt[i, (k,m)] = round(E[i, k] * W[j(i), m])   (product in FP64, rounded once
//                                                  to nearest even: bf16 or fp32),
//     Gt = Zt^T Zt  on MFMA with fp32 accumulation, stored in FP64.
// Z (and Zt) is never stored: every operand tile is formed while it is
// staged into LDS, from E and W read in FP64.  Rounding Z itself (not E and W
// separately, and not diag(s) W) keeps Gt the Gram of a perturbed Z, so FP64
// refinement on the least-squares residual contracts at a rate set by
// kappa(Z) * u_low rather than kappa(Z)^2 * u_low.
//
// Split bfloat16 (three products): z = hi + lo with hi = bf16(z) and
// lo = bf16(z - hi) (the subtraction is exact in FP64), and
//     Gt = Hi^T Hi + Hi^T Lo + Lo^T Hi
// accumulated in fp32 (the Lo^T Lo term, 2^-16 relative, is dropped): the
// operand error falls from 2^-9 to about 2^-17 for three bf16 products.
//
// Accumulation: the MFMAs accumulate in fp32 over 256 rows of the
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
__device__ __forceinline__ void flush_partial(f4 (&acc)[4][4], double (&acc64)[4][4][4]) {
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
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

// The FP64 products z = E[i, k] W[j(i), m] of one column (k, m) of Z for the
// Q consecutive rows i0 .. i0 + Q - 1 (zero beyond the last row n or the last
// column KM).  j(i) = i mod n_h (the level segments share W).
template <int Q>
__device__ __forceinline__ void z_rows(const LowGramInst& g, int64_t col, int64_t i0, double (&z)[Q]) {
  if (col >= g.KM) {
#pragma unroll
    for (int q = 0; q < Q; ++q) z[q] = 0.0;
    return;
  }
  const int64_t k = col / g.M, m = col - k * g.M;
  const double* e = g.E + k * g.ldE;
  const double* w = g.W + m * g.ldW;
  if (g.n_w == 1 && i0 + Q <= g.n) {
#pragma unroll
    for (int q = 0; q < Q; ++q) z[q] = e[i0 + q] * w[i0 + q];
    return;
  }
  int64_t j = i0 % g.n_h;
#pragma unroll
  for (int q = 0; q < Q; ++q) {
    const int64_t i = i0 + q;
    z[q] = (i < g.n) ? e[i] * w[j] : 0.0;
    if (++j == g.n_h) j = 0;
  }
}

// ---------------------------------------------------------------- bf16 (and split bf16)
constexpr int BKC = 32, BST = BKC + 8;   // k per stage, padded LDS row stride (bf16 elements)

__device__ __forceinline__ s8 pack8(const unsigned short (&h)[8]) {
  s8 v;
#pragma unroll
  for (int q = 0; q < 8; ++q) v[q] = (short)h[q];
  return v;
}

// One 128 x 128 tile (a0.., b0..) of the lower triangle, a0 >= b0.  X3: the
// split-bf16 form (hi and lo operands, three products).
template <bool X3>
__device__ __forceinline__ void gram_bf16_tile(const LowGramInst& g, int64_t a0, int64_t b0) {
  constexpr int NP = X3 ? 2 : 1;   // operand parts in LDS: hi (and lo)
  __shared__ __attribute__((aligned(16))) unsigned short As[2][NP][LT * BST];   // rows b (lower index block)
  __shared__ __attribute__((aligned(16))) unsigned short Bs[2][NP][LT * BST];   // cols a
  const int t = threadIdx.x, lane = lane_id(), w = wave_id();
  const int wm = w >> 1, wn = w & 1, r = lane & 15, kq = lane >> 4;
  const int seg = t & 3, row = t >> 2;           // 8-row segment of a 32-row chunk, tile column
  const int64_t nchunks = (g.n + BKC - 1) / BKC;
  s8 va[2][NP], vb[2][NP];
  auto form = [&](int64_t c) {
    const int64_t i0 = c * BKC + seg * 8;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
#pragma unroll
      for (int side = 0; side < 2; ++side) {
        double z[8];
        z_rows<8>(g, (side ? a0 : b0) + row + 64 * h, i0, z);
        unsigned short hi[8], lo[8];
#pragma unroll
        for (int q = 0; q < 8; ++q) {
          hi[q] = f64_to_bf16_rne(z[q]);
          if (X3) lo[q] = f64_to_bf16_rne(z[q] - (double)bf16_to_f32(hi[q]));
        }
        s8* dst = side ? vb[h] : va[h];
        dst[0] = pack8(hi);
        if (X3) dst[NP - 1] = pack8(lo);
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int p = 0; p < NP; ++p) {
        *reinterpret_cast<s8*>(&As[buf][p][(row + 64 * h) * BST + seg * 8]) = va[h][p];
        *reinterpret_cast<s8*>(&Bs[buf][p][(row + 64 * h) * BST + seg * 8]) = vb[h][p];
      }
  };
  f4 acc[4][4];
  double acc64[4][4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int v = 0; v < 4; ++v) acc64[i][j][v] = 0.0;
    }
  form(0);
  store(0);
  __syncthreads();
  for (int64_t c = 0; c < nchunks; ++c) {
    const bool more = c + 1 < nchunks;
    if (more) form(c + 1);
    const int buf = (int)(c & 1);
    s8 af[4], bf[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) af[i] = *reinterpret_cast<const s8*>(&As[buf][0][(wm * 64 + i * 16 + r) * BST + kq * 8]);
#pragma unroll
    for (int j = 0; j < 4; ++j) bf[j] = *reinterpret_cast<const s8*>(&Bs[buf][0][(wn * 64 + j * 16 + r) * BST + kq * 8]);
    if constexpr (X3) {
      s8 al[4], bl[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) al[i] = *reinterpret_cast<const s8*>(&As[buf][NP - 1][(wm * 64 + i * 16 + r) * BST + kq * 8]);
#pragma unroll
      for (int j = 0; j < 4; ++j) bl[j] = *reinterpret_cast<const s8*>(&Bs[buf][NP - 1][(wn * 64 + j * 16 + r) * BST + kq * 8]);
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          acc[i][j] = mfma_bf16(al[i], bf[j], acc[i][j]);   // small terms first
          acc[i][j] = mfma_bf16(af[i], bl[j], acc[i][j]);
          acc[i][j] = mfma_bf16(af[i], bf[j], acc[i][j]);
        }
    } else {
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = mfma_bf16(af[i], bf[j], acc[i][j]);
    }
    if ((c + 1) % (FLUSH_ROWS / BKC) == 0) flush_partial(acc, acc64);
    if (more) store((c + 1) & 1);
    __syncthreads();
  }
  flush_partial(acc, acc64);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t b = b0 + wm * 64 + i * 16 + 4 * kq + v;   // row of the product = lower index
        const int64_t a = a0 + wn * 64 + j * 16 + r;            // column = higher index
        if (a < g.KM && b < g.KM && a >= b) g.G[a + b * g.ldG] = acc64[i][j][v];
      }
}

// ---------------------------------------------------------------- fp32
constexpr int FKC = 16, FST = FKC + 1;

__device__ __forceinline__ void gram_f32_tile(const LowGramInst& g, int64_t a0, int64_t b0) {
  __shared__ float As[2][LT * FST];
  __shared__ float Bs[2][LT * FST];
  const int t = threadIdx.x, lane = lane_id(), w = wave_id();
  const int wm = w >> 1, wn = w & 1, r = lane & 15, kq = lane >> 4;
  const int seg = t & 3, row = t >> 2;           // 4 rows of a 16-row chunk, tile column
  const int64_t nchunks = (g.n + FKC - 1) / FKC;
  f4 va[2], vb[2];
  auto form = [&](int64_t c) {
    const int64_t i0 = c * FKC + seg * 4;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      double za[4], zb[4];
      z_rows<4>(g, b0 + row + 64 * h, i0, za);
      z_rows<4>(g, a0 + row + 64 * h, i0, zb);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        va[h][q] = (float)za[q];   // IEEE round to nearest even
        vb[h][q] = (float)zb[q];
      }
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int h = 0; h < 2; ++h)
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        As[buf][(row + 64 * h) * FST + seg * 4 + q] = va[h][q];
        Bs[buf][(row + 64 * h) * FST + seg * 4 + q] = vb[h][q];
      }
  };
  f4 acc[4][4];
  double acc64[4][4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) {
      acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
#pragma unroll
      for (int v = 0; v < 4; ++v) acc64[i][j][v] = 0.0;
    }
  form(0);
  store(0);
  __syncthreads();
  for (int64_t c = 0; c < nchunks; ++c) {
    const bool more = c + 1 < nchunks;
    if (more) form(c + 1);
    const float* Ab = As[c & 1];
    const float* Bb = Bs[c & 1];
#pragma unroll
    for (int kk = 0; kk < FKC; kk += 4) {
      float af[4], bf[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) af[i] = Ab[(wm * 64 + i * 16 + r) * FST + kk + kq];
#pragma unroll
      for (int j = 0; j < 4; ++j) bf[j] = Bb[(wn * 64 + j * 16 + r) * FST + kk + kq];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = mfma_f32(af[i], bf[j], acc[i][j]);
    }
    if ((c + 1) % (FLUSH_ROWS / FKC) == 0) flush_partial(acc, acc64);
    if (more) store((c + 1) & 1);
    __syncthreads();
  }
  flush_partial(acc, acc64);
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t b = b0 + wm * 64 + i * 16 + 4 * kq + v;
        const int64_t a = a0 + wn * 64 + j * 16 + r;
        if (a < g.KM && b < g.KM && a >= b) g.G[a + b * g.ldG] = acc64[i][j][v];
      }
}

template <int MODE>
__device__ __forceinline__ void gram_lp_tile(const LowGramInst& g, int64_t a0, int64_t b0) {
  if constexpr (MODE == LP_FP32) gram_f32_tile(g, a0, b0);
  else gram_bf16_tile<MODE == LP_BF16X3>(g, a0, b0);
}

// One instance: the lower tile pairs in XCD-contiguous ranges.
template <int MODE>
__global__ __launch_bounds__(256) void gram_lowprec_kernel(LowGramInst g, int64_t ntile_pairs) {
  const int64_t per = (ntile_pairs + 7) / 8;
  const int64_t u = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (u >= ntile_pairs) return;
  int64_t ta, tb;
  lower_tile(u, ta, tb);                         // ta >= tb
  gram_lp_tile<MODE>(g, ta * LT, tb * LT);
}

// Several instances in one launch: workgroup b takes tiles[b] (instance,
// tile row, tile column); the host lists the tiles longest contraction first,
// so the short ones fill the end of the launch.  Tiles of instances whose
// mode differs from the launch's are skipped (mode[inst] != MODE).
template <int MODE>
__global__ __launch_bounds__(256) void gram_lowprec_batch_kernel(const LowGramTile* __restrict__ tiles,
                                                                 const LowGramInst* __restrict__ insts,
                                                                 const int* __restrict__ mode) {
  const LowGramTile tl = tiles[blockIdx.x];
  if (mode[tl.inst] != MODE) return;
  const LowGramInst g = insts[tl.inst];
  gram_lp_tile<MODE>(g, (int64_t)tl.ta * LT, (int64_t)tl.tb * LT);
}

static LowGramInst lowgram_args(const Inst& in) {
  return LowGramInst{in.E, in.ldE, in.W, in.ldW, in.n, in.n_h, in.n_w, in.M, in.KM, in.G, in.KMp};
}

LowGramBatch* make_lowgram_batch(const std::vector<Inst>& insts) {
  std::vector<LowGramInst> hi(insts.size());
  std::vector<LowGramTile> ht;
  for (size_t i = 0; i < insts.size(); ++i) {
    const Inst& in = insts[i];
    hi[i] = lowgram_args(in);
    const int64_t nt = ceil_div(in.KM, LT);
    for (int64_t a = 0; a < nt; ++a)
      for (int64_t b = 0; b <= a; ++b) ht.push_back(LowGramTile{(int)i, (int)a, (int)b, 0});
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
    hipLaunchKernelGGL(gram_lowprec_batch_kernel<LP_BF16>, grid, dim3(256), 0, s, b->tiles, b->insts, b->mode);
  else if (precision == LP_BF16X3)
    hipLaunchKernelGGL(gram_lowprec_batch_kernel<LP_BF16X3>, grid, dim3(256), 0, s, b->tiles, b->insts, b->mode);
  else if (precision == LP_FP32)
    hipLaunchKernelGGL(gram_lowprec_batch_kernel<LP_FP32>, grid, dim3(256), 0, s, b->tiles, b->insts, b->mode);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

hipError_t launch_gram_lowprec(const Inst& in, int precision, hipStream_t s) {
  const int64_t nt = ceil_div(in.KM, LT);
  const int64_t pairs = nt * (nt + 1) / 2;
  const dim3 grid((unsigned)(8 * ((pairs + 7) / 8)));
  const LowGramInst g = lowgram_args(in);
  if (precision == LP_BF16)
    hipLaunchKernelGGL(gram_lowprec_kernel<LP_BF16>, grid, dim3(256), 0, s, g, pairs);
  else if (precision == LP_BF16X3)
    hipLaunchKernelGGL(gram_lowprec_kernel<LP_BF16X3>, grid, dim3(256), 0, s, g, pairs);
  else if (precision == LP_FP32)
    hipLaunchKernelGGL(gram_lowprec_kernel<LP_FP32>, grid, dim3(256), 0, s, g, pairs);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

}  // namespace pc
