// Reduced-precision Gram: the exact Gram of ONE rounded copy of Z,
//     Zt[i, (k,m)] = round(E[i, k] * W[j(i), m])   (bf16 or fp32, round to nearest even),
//     Gt = Zt^T Zt  on MFMA with fp32 accumulation, stored in FP64.
// Rounding Z itself (not E and W separately, and not diag(s) W) keeps Gt the
// Gram of a perturbed Z, so FP64 refinement on the least-squares residual
// contracts at a rate set by kappa(Z) * u_low rather than kappa(Z)^2 * u_low.
//
// Staging writes Zt column-major with the rows padded to a multiple of 64
// (zero rows), 2 bytes (bf16) or 4 bytes (fp32) per element.  The Gram then
// is a plain lower-triangular product over 128 x 128 tiles: four waves own
// 64 x 64 quadrants.  Accumulator layout of the f32 16x16 MFMAs (measured):
// lane l holds rows 4 * (l / 16) + v, column l % 16.
#include "pc_common.h"
#include "pc_internal.h"

#include <algorithm>

namespace pc {

constexpr int LT = 128;

template <typename T> struct Round;
template <> struct Round<unsigned short> {
  __device__ static unsigned short go(double x) { return f64_to_bf16_rne(x); }
};
template <> struct Round<float> {
  __device__ static float go(double x) { return (float)x; }   // IEEE round to nearest even
};

template <typename T>
__global__ void stage_z_kernel(const double* __restrict__ E, int64_t ldE, const double* __restrict__ W,
                               int64_t ldW, int64_t n, int64_t n_h, int64_t M, int64_t ldz,
                               T* __restrict__ Zt) {
  const int64_t a = blockIdx.y;          // column (k, m)
  const int64_t k = a / M, m = a % M;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < ldz; i += (int64_t)gridDim.x * blockDim.x) {
    T v;
    if (i < n) v = Round<T>::go(E[i + k * ldE] * W[(i % n_h) + m * ldW]);
    else v = T(0);
    Zt[i + a * ldz] = v;
  }
}

__device__ __forceinline__ void lower_tile(int64_t t, int64_t& ta, int64_t& tb) {
  int64_t a = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((a + 1) * (a + 2) / 2 <= t) ++a;
  while (a * (a + 1) / 2 > t) --a;
  ta = a;
  tb = t - a * (a + 1) / 2;
}

// ---------------------------------------------------------------- bf16
constexpr int BKC = 32, BST = BKC + 8;   // k per stage, padded LDS row stride (bf16 elements)

// One 128 x 128 tile (a0.., b0..) of the lower triangle, a0 >= b0.
__device__ __forceinline__ void gram_bf16_tile(const unsigned short* __restrict__ Zt, int64_t ldz, int64_t KM,
                                               int64_t a0, int64_t b0, double* __restrict__ G, int64_t ldG) {
  __shared__ __attribute__((aligned(16))) unsigned short As[2][LT * BST];   // rows b (lower index block)
  __shared__ __attribute__((aligned(16))) unsigned short Bs[2][LT * BST];   // cols a
  const int t = threadIdx.x, lane = lane_id(), w = wave_id();
  const int wm = w >> 1, wn = w & 1, r = lane & 15, kq = lane >> 4;
  const int seg = t & 3, row = t >> 2;           // 16-byte segment of a 64-byte row chunk
  const int64_t nchunks = ldz / BKC;
  s8 va[2], vb[2];
  auto load = [&](int64_t c) {
    const int64_t i0 = c * BKC + seg * 8;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t rb = b0 + row + 64 * h, ra = a0 + row + 64 * h;
      s8 zero = {0, 0, 0, 0, 0, 0, 0, 0};
      va[h] = (rb < KM) ? *reinterpret_cast<const s8*>(Zt + rb * ldz + i0) : zero;
      vb[h] = (ra < KM) ? *reinterpret_cast<const s8*>(Zt + ra * ldz + i0) : zero;
    }
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      *reinterpret_cast<s8*>(&As[buf][(row + 64 * h) * BST + seg * 8]) = va[h];
      *reinterpret_cast<s8*>(&Bs[buf][(row + 64 * h) * BST + seg * 8]) = vb[h];
    }
  };
  f4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  load(0);
  store(0);
  __syncthreads();
  for (int64_t c = 0; c < nchunks; ++c) {
    const bool more = c + 1 < nchunks;
    if (more) load(c + 1);
    const unsigned short* Ab = As[c & 1];
    const unsigned short* Bb = Bs[c & 1];
    s8 af[4], bf[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) af[i] = *reinterpret_cast<const s8*>(&Ab[(wm * 64 + i * 16 + r) * BST + kq * 8]);
#pragma unroll
    for (int j = 0; j < 4; ++j) bf[j] = *reinterpret_cast<const s8*>(&Bb[(wn * 64 + j * 16 + r) * BST + kq * 8]);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = mfma_bf16(af[i], bf[j], acc[i][j]);
    if (more) store((c + 1) & 1);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t b = b0 + wm * 64 + i * 16 + 4 * kq + v;   // row of the product = lower index
        const int64_t a = a0 + wn * 64 + j * 16 + r;            // column = higher index
        if (a < KM && b < KM && a >= b) G[a + b * ldG] = (double)acc[i][j][v];
      }
}

__global__ __launch_bounds__(256) void gram_bf16_kernel(const unsigned short* __restrict__ Zt, int64_t ldz,
                                                        int64_t KM, int64_t ntile_pairs, double* __restrict__ G,
                                                        int64_t ldG) {
  const int64_t per = (ntile_pairs + 7) / 8;
  const int64_t u = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (u >= ntile_pairs) return;
  int64_t ta, tb;
  lower_tile(u, ta, tb);                         // ta >= tb
  gram_bf16_tile(Zt, ldz, KM, ta * LT, tb * LT, G, ldG);
}

// ---------------------------------------------------------------- fp32
constexpr int FKC = 16, FST = FKC + 1;

__device__ __forceinline__ void gram_f32_tile(const float* __restrict__ Zt, int64_t ldz, int64_t KM, int64_t a0,
                                              int64_t b0, double* __restrict__ G, int64_t ldG) {
  __shared__ float As[2][LT * FST];
  __shared__ float Bs[2][LT * FST];
  const int t = threadIdx.x, lane = lane_id(), w = wave_id();
  const int wm = w >> 1, wn = w & 1, r = lane & 15, kq = lane >> 4;
  const int seg = t & 3, row = t >> 2;           // 4 floats of a 16-float row chunk
  const int64_t nchunks = ldz / FKC;
  f4 va[2], vb[2];
  auto load = [&](int64_t c) {
    const int64_t i0 = c * FKC + seg * 4;
#pragma unroll
    for (int h = 0; h < 2; ++h) {
      const int64_t rb = b0 + row + 64 * h, ra = a0 + row + 64 * h;
      const f4 zero = {0.f, 0.f, 0.f, 0.f};
      va[h] = (rb < KM) ? *reinterpret_cast<const f4*>(Zt + rb * ldz + i0) : zero;
      vb[h] = (ra < KM) ? *reinterpret_cast<const f4*>(Zt + ra * ldz + i0) : zero;
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
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  load(0);
  store(0);
  __syncthreads();
  for (int64_t c = 0; c < nchunks; ++c) {
    const bool more = c + 1 < nchunks;
    if (more) load(c + 1);
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
    if (more) store((c + 1) & 1);
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t b = b0 + wm * 64 + i * 16 + 4 * kq + v;
        const int64_t a = a0 + wn * 64 + j * 16 + r;
        if (a < KM && b < KM && a >= b) G[a + b * ldG] = (double)acc[i][j][v];
      }
}

__global__ __launch_bounds__(256) void gram_f32_kernel(const float* __restrict__ Zt, int64_t ldz, int64_t KM,
                                                       int64_t ntile_pairs, double* __restrict__ G, int64_t ldG) {
  const int64_t per = (ntile_pairs + 7) / 8;
  const int64_t u = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (u >= ntile_pairs) return;
  int64_t ta, tb;
  lower_tile(u, ta, tb);
  gram_f32_tile(Zt, ldz, KM, ta * LT, tb * LT, G, ldG);
}

// Several instances in one launch: workgroup b takes tiles[b] (instance,
// tile row, tile column); the host lists the tiles longest contraction first,
// so the short ones fill the end of the launch.
template <typename T>
__global__ __launch_bounds__(256) void gram_lowprec_batch_kernel(const LowGramTile* __restrict__ tiles,
                                                                 const LowGramInst* __restrict__ insts) {
  const LowGramTile tl = tiles[blockIdx.x];
  const LowGramInst in = insts[tl.inst];
  if constexpr (sizeof(T) == 2)
    gram_bf16_tile(reinterpret_cast<const unsigned short*>(in.Zt), in.ldz, in.KM, (int64_t)tl.ta * LT,
                   (int64_t)tl.tb * LT, in.G, in.ldG);
  else
    gram_f32_tile(reinterpret_cast<const float*>(in.Zt), in.ldz, in.KM, (int64_t)tl.ta * LT, (int64_t)tl.tb * LT,
                  in.G, in.ldG);
}

hipError_t launch_stage_z(const Inst& in, int precision, hipStream_t s) {
  if (!in.Zt) return hipErrorInvalidValue;
  const unsigned gx = (unsigned)std::min<int64_t>(ceil_div(in.ldz, 256), 64);
  if (precision == 2)
    hipLaunchKernelGGL(stage_z_kernel<unsigned short>, dim3(gx, (unsigned)in.KM), dim3(256), 0, s, in.E, in.ldE,
                       in.W, in.ldW, in.n, in.n_h, in.M, in.ldz, reinterpret_cast<unsigned short*>(in.Zt));
  else
    hipLaunchKernelGGL(stage_z_kernel<float>, dim3(gx, (unsigned)in.KM), dim3(256), 0, s, in.E, in.ldE, in.W,
                       in.ldW, in.n, in.n_h, in.M, in.ldz, reinterpret_cast<float*>(in.Zt));
  return hipGetLastError();
}

LowGramBatch* make_lowgram_batch(const std::vector<Inst>& insts) {
  std::vector<LowGramInst> hi(insts.size());
  std::vector<LowGramTile> ht;
  for (size_t i = 0; i < insts.size(); ++i) {
    const Inst& in = insts[i];
    hi[i] = LowGramInst{in.Zt, in.ldz, in.KM, in.G, in.KMp};
    const int64_t nt = ceil_div(in.KM, LT);
    for (int64_t a = 0; a < nt; ++a)
      for (int64_t b = 0; b <= a; ++b) ht.push_back(LowGramTile{(int)i, (int)a, (int)b, 0});
  }
  std::stable_sort(ht.begin(), ht.end(), [&](const LowGramTile& x, const LowGramTile& y) {
    return insts[x.inst].ldz > insts[y.inst].ldz;
  });
  LowGramBatch* b = new LowGramBatch{};
  b->ntiles = (int64_t)ht.size();
  hipError_t e = hipMalloc((void**)&b->tiles, sizeof(LowGramTile) * ht.size());
  if (e == hipSuccess) e = hipMalloc((void**)&b->insts, sizeof(LowGramInst) * hi.size());
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
  delete b;
}

hipError_t launch_gram_lowprec_batch(const LowGramBatch* b, int precision, hipStream_t s) {
  if (b->ntiles <= 0) return hipSuccess;
  if (precision == 2)
    hipLaunchKernelGGL(gram_lowprec_batch_kernel<unsigned short>, dim3((unsigned)b->ntiles), dim3(256), 0, s,
                       b->tiles, b->insts);
  else
    hipLaunchKernelGGL(gram_lowprec_batch_kernel<float>, dim3((unsigned)b->ntiles), dim3(256), 0, s, b->tiles,
                       b->insts);
  return hipGetLastError();
}

hipError_t launch_gram_lowprec(const Inst& in, int precision, hipStream_t s) {
  if (!in.Zt) return hipErrorInvalidValue;
  const int64_t nt = ceil_div(in.KM, LT);
  const int64_t pairs = nt * (nt + 1) / 2;
  const unsigned gx = (unsigned)std::min<int64_t>(ceil_div(in.ldz, 256), 64);
  const unsigned grid = (unsigned)(8 * ((pairs + 7) / 8));
  if (precision == 2) {   // bf16
    unsigned short* Z = reinterpret_cast<unsigned short*>(in.Zt);
    hipLaunchKernelGGL(stage_z_kernel<unsigned short>, dim3(gx, (unsigned)in.KM), dim3(256), 0, s, in.E, in.ldE,
                       in.W, in.ldW, in.n, in.n_h, in.M, in.ldz, Z);
    hipLaunchKernelGGL(gram_bf16_kernel, dim3(grid), dim3(256), 0, s, Z, in.ldz, in.KM, pairs, in.G, in.KMp);
  } else {                // fp32
    float* Z = reinterpret_cast<float*>(in.Zt);
    hipLaunchKernelGGL(stage_z_kernel<float>, dim3(gx, (unsigned)in.KM), dim3(256), 0, s, in.E, in.ldE, in.W,
                       in.ldW, in.n, in.n_h, in.M, in.ldz, Z);
    hipLaunchKernelGGL(gram_f32_kernel, dim3(grid), dim3(256), 0, s, Z, in.ldz, in.KM, pairs, in.G, in.KMp);
  }
  return hipGetLastError();
}

}  // namespace pc
