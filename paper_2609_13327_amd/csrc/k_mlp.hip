// Kernels of the two-layer GELU network used as a warm start for CG on the
// normal equations: forward, relative-MSE loss, backward and Adam.
//
// Batches are row-major (one sample per row).  Every matrix product is one
// MFMA GEMM kernel: operands are read from fp32 global memory and converted
// once, while staged into LDS, to the MFMA operand type T -- bf16 (round to
// nearest even, 16x16x32 MFMA) or fp32 (16x16x4 MFMA) -- and accumulated in
// fp32.  Which operand dimension is contiguous in memory is a template flag,
// so X W^T, dY^T H and dY W all use the same kernel.  Small products split
// the contraction over workgroups into fp32 partial tiles that a separate
// epilogue kernel sums in a fixed order (deterministic).
//
// Accumulator layout of both fp32-output 16x16 MFMAs (measured): lane l holds
// rows 4 * (l / 16) + v, column l % 16.
#include "pc_common.h"
#include "pc_internal.h"

#include <algorithm>

namespace pc {

constexpr int GT = 128;   // workgroup tile (rows and columns)
constexpr int GKC = 32;   // contraction per LDS stage

// fp32 -> bf16, round to nearest even (finite inputs): add 0x7fff plus the
// lowest kept bit, then truncate.
__device__ __forceinline__ unsigned short f32_to_bf16_rne(float x) {
  unsigned int u = __float_as_uint(x);
  u += 0x7fffu + ((u >> 16) & 1u);
  return (unsigned short)(u >> 16);
}

__device__ __forceinline__ float gelu_f(float a) { return 0.5f * a * (1.0f + erff(a * 0.70710678118654752f)); }
__device__ __forceinline__ float gelu_grad_f(float a) {
  return 0.5f * (1.0f + erff(a * 0.70710678118654752f)) + a * 0.39894228040143268f * expf(-0.5f * a * a);
}

template <typename T> struct OpT;
template <> struct OpT<unsigned short> {
  static constexpr int LS = GKC + 8;   // LDS row stride (elements)
  __device__ static unsigned short cvt(float x) { return f32_to_bf16_rne(x); }
};
template <> struct OpT<float> {
  static constexpr int LS = GKC + 4;
  __device__ static float cvt(float x) { return x; }
};

// Stage 32 contraction indices of a 128-row operand tile.  KC (contiguous
// along k): thread t covers row t/2, k [16 (t%2), +16).  Otherwise
// (contiguous along the row index): thread t covers k = t/8 and rows
// [16 (t%8), +16).  Out-of-range elements read as zero.
template <bool KCONT>
struct Stage {
  float v[16];
  __device__ void load(const float* __restrict__ P, int64_t srow, int64_t sk, int64_t row0, int64_t nrow,
                       int64_t k0, int64_t K, bool vec) {
    const int t = threadIdx.x;
    if (KCONT) {
      const int64_t row = row0 + (t >> 1), kb = k0 + 16 * (t & 1);
      if (vec && row < nrow && kb + 16 <= K) {
        const float4* p = reinterpret_cast<const float4*>(P + row * srow + kb);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float4 x = p[q];
          v[4 * q] = x.x; v[4 * q + 1] = x.y; v[4 * q + 2] = x.z; v[4 * q + 3] = x.w;
        }
      } else {
#pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = (row < nrow && kb + q < K) ? P[row * srow + kb + q] : 0.f;
      }
    } else {
      const int64_t k = k0 + (t >> 3), rb = row0 + 16 * (t & 7);
      if (vec && k < K && rb + 16 <= nrow) {
        const float4* p = reinterpret_cast<const float4*>(P + k * sk + rb);
#pragma unroll
        for (int q = 0; q < 4; ++q) {
          const float4 x = p[q];
          v[4 * q] = x.x; v[4 * q + 1] = x.y; v[4 * q + 2] = x.z; v[4 * q + 3] = x.w;
        }
      } else {
#pragma unroll
        for (int q = 0; q < 16; ++q) v[q] = (k < K && rb + q < nrow) ? P[k * sk + rb + q] : 0.f;
      }
    }
  }
  template <typename T>
  __device__ void store(T* __restrict__ S) const {   // S[row * LS + k]
    constexpr int LS = OpT<T>::LS;
    const int t = threadIdx.x;
    if (KCONT) {
      T* d = S + (t >> 1) * LS + 16 * (t & 1);
#pragma unroll
      for (int q = 0; q < 16; ++q) d[q] = OpT<T>::cvt(v[q]);
    } else {
      T* d = S + 16 * (t & 7) * LS + (t >> 3);
#pragma unroll
      for (int q = 0; q < 16; ++q) d[q * LS] = OpT<T>::cvt(v[q]);
    }
  }
};

// Fragment product of one LDS stage for a 64 x 64 wave sub-tile.
template <typename T> struct Frag;
template <> struct Frag<unsigned short> {
  __device__ static void mma(const unsigned short* As, const unsigned short* Bs, int wm, int wn, f4 (&acc)[4][4]) {
    constexpr int LS = OpT<unsigned short>::LS;
    const int lane = lane_id(), r = lane & 15, kq = lane >> 4;
    s8 af[4], bf[4];
#pragma unroll
    for (int i = 0; i < 4; ++i) af[i] = *reinterpret_cast<const s8*>(&As[(wm * 64 + i * 16 + r) * LS + kq * 8]);
#pragma unroll
    for (int j = 0; j < 4; ++j) bf[j] = *reinterpret_cast<const s8*>(&Bs[(wn * 64 + j * 16 + r) * LS + kq * 8]);
#pragma unroll
    for (int i = 0; i < 4; ++i)
#pragma unroll
      for (int j = 0; j < 4; ++j) acc[i][j] = mfma_bf16(af[i], bf[j], acc[i][j]);
  }
};
template <> struct Frag<float> {
  __device__ static void mma(const float* As, const float* Bs, int wm, int wn, f4 (&acc)[4][4]) {
    constexpr int LS = OpT<float>::LS;
    const int lane = lane_id(), r = lane & 15, kq = lane >> 4;
#pragma unroll
    for (int kk = 0; kk < GKC; kk += 4) {
      float af[4], bf[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) af[i] = As[(wm * 64 + i * 16 + r) * LS + kk + kq];
#pragma unroll
      for (int j = 0; j < 4; ++j) bf[j] = Bs[(wn * 64 + j * 16 + r) * LS + kk + kq];
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = mfma_f32(af[i], bf[j], acc[i][j]);
    }
  }
};

__device__ __forceinline__ float mlp_epilogue(const MlpGemm& g, int64_t m, int64_t n, float v) {
  switch (g.mode) {
    case MLP_EPI_BIAS_GELU: {
      const float a = v + g.bias[n];
      g.C[m * g.ldc + n] = a;
      g.C2[m * g.ldc + n] = gelu_f(a);
      return a;
    }
    case MLP_EPI_BIAS:
      g.C[m * g.ldc + n] = v + g.bias[n];
      return v;
    case MLP_EPI_GELU_GRAD:
      g.C[m * g.ldc + n] = v * gelu_grad_f(g.aux[m * g.ldc + n]);
      return v;
    default:
      g.C[m * g.ldc + n] = v;
      return v;
  }
}

// C(m, n) = sum_k A(m, k) B(n, k) over the contraction range of split s.
template <typename T, bool AK, bool BK>
__global__ __launch_bounds__(256) void mlp_gemm_kernel(MlpGemm g) {
  constexpr int LS = OpT<T>::LS;
  __shared__ __attribute__((aligned(16))) T As[2][GT * LS];
  __shared__ __attribute__((aligned(16))) T Bs[2][GT * LS];
  const int64_t tm = (g.M + GT - 1) / GT;
  const int64_t tile = blockIdx.x, s = blockIdx.y;
  const int64_t m0 = (tile % tm) * GT, n0 = (tile / tm) * GT;
  const int64_t kbeg = s * g.kper, kend = std::min<int64_t>(g.K, kbeg + g.kper);
  const int w = wave_id(), wm = w >> 1, wn = w & 1;
  f4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = f4{0.f, 0.f, 0.f, 0.f};
  const int64_t nchunks = kend > kbeg ? (kend - kbeg + GKC - 1) / GKC : 0;
  Stage<AK> sa;
  Stage<BK> sb;
  if (nchunks > 0) {
    sa.load(g.A, g.sam, g.sak, m0, g.M, kbeg, kend, g.vec != 0);
    sb.load(g.B, g.sbn, g.sbk, n0, g.N, kbeg, kend, g.vec != 0);
    sa.store(As[0]);
    sb.store(Bs[0]);
    __syncthreads();
  }
  for (int64_t c = 0; c < nchunks; ++c) {
    const bool more = c + 1 < nchunks;
    if (more) {
      const int64_t k0 = kbeg + (c + 1) * GKC;
      sa.load(g.A, g.sam, g.sak, m0, g.M, k0, kend, g.vec != 0);
      sb.load(g.B, g.sbn, g.sbk, n0, g.N, k0, kend, g.vec != 0);
    }
    Frag<T>::mma(As[c & 1], Bs[c & 1], wm, wn, acc);
    if (more) {
      sa.store(As[(c + 1) & 1]);
      sb.store(Bs[(c + 1) & 1]);
    }
    __syncthreads();
  }
  const int lane = lane_id(), r = lane & 15, kq = lane >> 4;
  float* part = g.partial ? g.partial + s * g.M * g.N : nullptr;
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t m = m0 + wm * 64 + i * 16 + 4 * kq + v;
        const int64_t n = n0 + wn * 64 + j * 16 + r;
        if (m >= g.M || n >= g.N) continue;
        if (part) part[m * g.N + n] = acc[i][j][v];
        else mlp_epilogue(g, m, n, acc[i][j][v]);
      }
}

// Sum the split partials in split order, then apply the epilogue.
__global__ void mlp_split_epilogue_kernel(MlpGemm g, int splits) {
  const int64_t total = g.M * g.N;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total; e += (int64_t)gridDim.x * blockDim.x) {
    float v = 0.f;
    for (int s = 0; s < splits; ++s) v += g.partial[s * total + e];
    mlp_epilogue(g, e / g.N, e % g.N, v);
  }
}

template <typename T>
static hipError_t gemm_dispatch(const MlpGemm& g0, hipStream_t st) {
  MlpGemm g = g0;
  const int64_t tiles = ((g.M + GT - 1) / GT) * ((g.N + GT - 1) / GT);
  int splits = 1;
  if (g.partial && tiles < 512) {
    const int64_t want = (512 + tiles - 1) / tiles;
    const int64_t maxs = std::max<int64_t>(1, g.K / (4 * GKC));
    const int64_t room = g.partial_cap / std::max<int64_t>(1, g.M * g.N);
    splits = (int)std::max<int64_t>(1, std::min<int64_t>({want, maxs, (int64_t)g.max_splits, room}));
  }
  g.kper = ((g.K + splits - 1) / splits + GKC - 1) / GKC * GKC;
  splits = (int)((g.K + g.kper - 1) / g.kper);
  if (splits < 1) splits = 1;
  if (splits == 1) g.partial = nullptr;
  const dim3 grid((unsigned)tiles, (unsigned)splits);
  const bool ak = g.a_kcont != 0, bk = g.b_kcont != 0;
  // 16-byte loads need aligned bases and row strides that are multiples of 4
  const auto al = [](const void* p) { return (reinterpret_cast<uintptr_t>(p) & 15) == 0; };
  g.vec = al(g.A) && al(g.B) && ((ak ? g.sam : g.sak) % 4 == 0) && ((bk ? g.sbn : g.sbk) % 4 == 0);
  if (ak && bk) hipLaunchKernelGGL((mlp_gemm_kernel<T, true, true>), grid, dim3(256), 0, st, g);
  else if (ak && !bk) hipLaunchKernelGGL((mlp_gemm_kernel<T, true, false>), grid, dim3(256), 0, st, g);
  else if (!ak && !bk) hipLaunchKernelGGL((mlp_gemm_kernel<T, false, false>), grid, dim3(256), 0, st, g);
  else hipLaunchKernelGGL((mlp_gemm_kernel<T, false, true>), grid, dim3(256), 0, st, g);
  if (splits > 1) {
    const unsigned eg = (unsigned)std::min<int64_t>(ceil_div(g.M * g.N, 256), 4096);
    hipLaunchKernelGGL(mlp_split_epilogue_kernel, dim3(eg), dim3(256), 0, st, g, splits);
  }
  return hipGetLastError();
}

hipError_t launch_mlp_gemm(const MlpGemm& g, int bf16, hipStream_t s) {
  if (g.M <= 0 || g.N <= 0) return hipSuccess;
  return bf16 ? gemm_dispatch<unsigned short>(g, s) : gemm_dispatch<float>(g, s);
}

// Relative MSE per row and its gradient:
//   loss_b = ||Y_b - T_b||^2 / ||T_b||^2,  dY_b = (2 / B) (Y_b - T_b) / ||T_b||^2.
// One workgroup per row.
__global__ __launch_bounds__(256) void mlp_loss_kernel(const float* __restrict__ Y, int64_t ldY,
                                                       const float* __restrict__ T, int64_t ldT, int64_t d,
                                                       int64_t B, float* __restrict__ dY, float* __restrict__ row_loss) {
  __shared__ double red[2][4];
  const int64_t b = blockIdx.x;
  double num = 0.0, den = 0.0;
  for (int64_t i = threadIdx.x; i < d; i += 256) {
    const double y = Y[b * ldY + i], t = T[b * ldT + i];
    num += (y - t) * (y - t);
    den += t * t;
  }
  num = wave_sum(num);
  den = wave_sum(den);
  if (lane_id() == 0) { red[0][wave_id()] = num; red[1][wave_id()] = den; }
  __syncthreads();
  num = red[0][0] + red[0][1] + red[0][2] + red[0][3];
  den = red[1][0] + red[1][1] + red[1][2] + red[1][3];
  const double scale = den > 0.0 ? 2.0 / ((double)B * den) : 0.0;
  for (int64_t i = threadIdx.x; i < d; i += 256)
    dY[b * d + i] = (float)(scale * ((double)Y[b * ldY + i] - (double)T[b * ldT + i]));
  if (threadIdx.x == 0) row_loss[b] = den > 0.0 ? (float)(num / den) : 0.f;
}

__global__ void mlp_mean_kernel(const float* __restrict__ v, int64_t n, float* __restrict__ out) {
  __shared__ double red[4];
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) s += v[i];
  s = wave_sum(s);
  if (lane_id() == 0) red[wave_id()] = s;
  __syncthreads();
  if (threadIdx.x == 0) *out = (float)((red[0] + red[1] + red[2] + red[3]) / (double)n);
}

// out[n] = sum_b G[b * ld + n] (bias gradients), rows summed in order.
__global__ void mlp_colsum_kernel(const float* __restrict__ G, int64_t ld, int64_t rows, int64_t cols,
                                  float* __restrict__ out) {
  const int64_t n = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (n >= cols) return;
  float s = 0.f;
  for (int64_t b = 0; b < rows; ++b) s += G[b * ld + n];
  out[n] = s;
}

hipError_t launch_mlp_loss(const float* Y, int64_t ldY, const float* T, int64_t ldT, int64_t d, int64_t B,
                           float* dY, float* row_loss, float* loss, hipStream_t s) {
  if (B <= 0) return hipSuccess;
  hipLaunchKernelGGL(mlp_loss_kernel, dim3((unsigned)B), dim3(256), 0, s, Y, ldY, T, ldT, d, B, dY, row_loss);
  hipLaunchKernelGGL(mlp_mean_kernel, dim3(1), dim3(256), 0, s, row_loss, B, loss);
  return hipGetLastError();
}

hipError_t launch_mlp_colsum(const float* G, int64_t ld, int64_t rows, int64_t cols, float* out, hipStream_t s) {
  if (cols <= 0) return hipSuccess;
  hipLaunchKernelGGL(mlp_colsum_kernel, dim3((unsigned)ceil_div(cols, 256)), dim3(256), 0, s, G, ld, rows, cols, out);
  return hipGetLastError();
}

// Adam with bias correction over every parameter (one flat array).  The
// coefficients 1 - beta and the bias corrections come from the host in
// double precision (1 - 0.999 formed in fp32 would be off by 1e-5).
__global__ void mlp_adam_kernel(float* __restrict__ p, const float* __restrict__ g, float* __restrict__ m,
                                float* __restrict__ v, int64_t n, AdamCoef c) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) {
    const float gi = g[i];
    const float mi = c.b1 * m[i] + c.omb1 * gi;
    const float vi = c.b2 * v[i] + c.omb2 * gi * gi;
    m[i] = mi;
    v[i] = vi;
    p[i] -= c.lr * (mi / c.bc1) / (sqrtf(vi / c.bc2) + c.eps);
  }
}

hipError_t launch_mlp_adam(float* p, const float* g, float* m, float* v, int64_t n, const AdamCoef& c,
                           hipStream_t s) {
  const unsigned gx = (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(n, 256), 8192));
  hipLaunchKernelGGL(mlp_adam_kernel, dim3(gx), dim3(256), 0, s, p, g, m, v, n, c);
  return hipGetLastError();
}

// Warm-start input: row r of Xh = b_r / ||b_r|| (fp32), nrm[r] = ||b_r||.
// b is column r of the FP64 column-major B.  One workgroup per column.
__global__ __launch_bounds__(256) void ws_prep_kernel(const double* __restrict__ Bm, int64_t ldB, int64_t d,
                                                      float* __restrict__ Xh, int64_t ldX, double* __restrict__ nrm) {
  __shared__ double red[4];
  const int64_t r = blockIdx.x;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < d; i += 256) {
    const double x = Bm[i + r * ldB];
    s += x * x;
  }
  s = wave_sum(s);
  if (lane_id() == 0) red[wave_id()] = s;
  __syncthreads();
  const double nb = sqrt(red[0] + red[1] + red[2] + red[3]);
  const double inv = nb > 0.0 ? 1.0 / nb : 0.0;
  for (int64_t i = threadIdx.x; i < d; i += 256) Xh[r * ldX + i] = (float)(Bm[i + r * ldB] * inv);
  if (threadIdx.x == 0) nrm[r] = nb;
}

// y0[:, r] = ||b_r|| * row r of Yh (FP64 column-major output).
__global__ void ws_finish_kernel(const float* __restrict__ Yh, int64_t ldYh, const double* __restrict__ nrm,
                                 int64_t d, double* __restrict__ Y0, int64_t ldY0) {
  const int64_t r = blockIdx.y;
  const double nb = nrm[r];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < d; i += (int64_t)gridDim.x * blockDim.x)
    Y0[i + r * ldY0] = nb * (double)Yh[r * ldYh + i];
}

// Training pairs from solved systems: row r of X = b_r / ||b_r||, row r of
// T = y_r / ||b_r|| (b_r, y_r columns of the FP64 column-major B and Y).
__global__ __launch_bounds__(256) void pairs_kernel(const double* __restrict__ Bm, int64_t ldB,
                                                    const double* __restrict__ Ym, int64_t ldY, int64_t d,
                                                    float* __restrict__ X, int64_t ldX, float* __restrict__ T,
                                                    int64_t ldT) {
  __shared__ double red[4];
  const int64_t r = blockIdx.x;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < d; i += 256) {
    const double x = Bm[i + r * ldB];
    s += x * x;
  }
  s = wave_sum(s);
  if (lane_id() == 0) red[wave_id()] = s;
  __syncthreads();
  const double nb = sqrt(red[0] + red[1] + red[2] + red[3]);
  const double inv = nb > 0.0 ? 1.0 / nb : 0.0;
  for (int64_t i = threadIdx.x; i < d; i += 256) {
    X[r * ldX + i] = (float)(Bm[i + r * ldB] * inv);
    T[r * ldT + i] = (float)(Ym[i + r * ldY] * inv);
  }
}

hipError_t launch_training_pairs(const double* Bm, int64_t ldB, const double* Ym, int64_t ldY, int64_t d, int64_t N,
                                 float* X, int64_t ldX, float* T, int64_t ldT, hipStream_t s) {
  if (N <= 0) return hipSuccess;
  hipLaunchKernelGGL(pairs_kernel, dim3((unsigned)N), dim3(256), 0, s, Bm, ldB, Ym, ldY, d, X, ldX, T, ldT);
  return hipGetLastError();
}

hipError_t launch_ws_prep(const double* Bm, int64_t ldB, int64_t d, int64_t R, float* Xh, int64_t ldX, double* nrm,
                          hipStream_t s) {
  if (R <= 0) return hipSuccess;
  hipLaunchKernelGGL(ws_prep_kernel, dim3((unsigned)R), dim3(256), 0, s, Bm, ldB, d, Xh, ldX, nrm);
  return hipGetLastError();
}

hipError_t launch_ws_finish(const float* Yh, int64_t ldYh, const double* nrm, int64_t d, int64_t R, double* Y0,
                            int64_t ldY0, hipStream_t s) {
  if (R <= 0) return hipSuccess;
  const unsigned gx = (unsigned)std::min<int64_t>(ceil_div(d, 256), 64);
  hipLaunchKernelGGL(ws_finish_kernel, dim3(gx, (unsigned)R), dim3(256), 0, s, Yh, ldYh, nrm, d, Y0, ldY0);
  return hipGetLastError();
}

}  // namespace pc
