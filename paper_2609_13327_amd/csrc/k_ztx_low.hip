// Reduced-precision Z^T x on MFMA with fp32 accumulation, stored in FP64:
//     B = Zt^T Xt,
// the right-hand side of the normal equations of a reduced-precision solve
// (the refinement's Z^T r stays FP64).  Zt is the same rounded Z whose Gram
// the reduced-precision modes contract, and Xt the rounded right-hand sides:
//   fp32:  Zt[i, (k,m)] = fp32(E[i,k] W[j,m])        (FP64 product, rounded once)
//          Xt = fp32(X)                               v_mfma_f32_16x16x4_f32
//   bf16:  Zt[i, (k,m)] = bf16(fl32(fp32(E[i,k]) fp32(W[j,m])))
//          Xt = bf16(fp32(X))                         v_mfma_f32_16x16x32_bf16
// with j = i mod n_h (row i = l n_h + j: level l, grid column j).  All
// roundings are to nearest even.  The contraction runs over all n rows of Z:
// the rounding is per element of Z, so the level sum cannot come first as it
// does in FP64.
//
// Tile: 64 right-hand sides x 64 modes of QKB consecutive members (4, or 2
// or 1 when larger tiles would leave compute units without one), four waves
// (2 x 2) of 32 x 32 per member; chunks of 32 rows staged in LDS (double
// buffered, the next chunk's loads issued before the current chunk's
// MFMAs).  The X and W rows of a chunk serve all the tile's members: each member's
// E column scales the W rows when the operand fragment is formed and
// rounded.  Tiles are dealt out in contiguous ranges per XCD.
#include "pc_common.h"
#include "pc_internal.h"

#include <algorithm>

namespace pc {

namespace {

constexpr int QT = 64, QKC = 32;
constexpr int QLD = QT + 1;      // fp32 form: LDS row stride (one row of Z per LDS row)
constexpr int QBS = QKC + 8;     // bf16 form: bf16 stride of an X column (80 bytes)
constexpr int QWS = QKC + 4;     // bf16 form: fp32 stride of a W or E column (144 bytes)
constexpr int LP_FP32 = 1, LP_BF16 = 2;   // the pc_precision codes of the two forms

template <class WS>
struct ZtxLowArgs {
  const double* E; int64_t ldE;
  WS w;
  const double* X; int64_t ldX;
  double* B; int64_t ldB;
  int64_t n, n_h, K, M, R;
  int ntr, ntm, ntk;
};

// Tile of workgroup blockIdx.x: contiguous ranges of tiles per XCD
// (workgroups are dealt round robin over the 8 XCDs).  False past the end.
template <int QKB, class A>
__device__ __forceinline__ bool ztx_low_tile(const A& a, int64_t& r0, int64_t& m0, int64_t& k0) {
  const int64_t units = (int64_t)a.ntr * a.ntm * a.ntk;
  const int64_t per = (units + 7) / 8;
  int64_t u = (blockIdx.x % 8) * per + blockIdx.x / 8;
  if (u >= units) return false;
  const int tr = (int)(u % a.ntr); u /= a.ntr;
  const int tm = (int)(u % a.ntm);
  k0 = (u / a.ntm) * QKB;
  r0 = (int64_t)tr * QT;
  m0 = (int64_t)tm * QT;
  return true;
}

typedef float f2v __attribute__((ext_vector_type(2)));
typedef __bf16 b2v __attribute__((ext_vector_type(2)));

// Two fp32 values to a packed pair of bf16 (round to nearest even).
__device__ __forceinline__ unsigned pack2(float x, float y) {
  return __builtin_bit_cast(unsigned, __builtin_convertvector(f2v{x, y}, b2v));
}

// ------------------------------------------------------------------- fp32
// Thread t stages row t % 32 of the chunk for the tile columns t / 32 + 8 q
// (q < 8) of X and W; threads t < 32 QKB stage row t % 32 of member t / 32.
template <int QKB, bool ONE, class WS>
__global__ __launch_bounds__(256) void ztx_f32_kernel(ZtxLowArgs<WS> a) {
  __shared__ float Xs[2][QKC * QLD];
  __shared__ double Ws[2][QKC * QLD];
  __shared__ double Es[2][QKC * QKB];
  int64_t r0, m0, k0;
  if (!ztx_low_tile<QKB>(a, r0, m0, k0)) return;
  const int t = threadIdx.x, lane = lane_id(), w = wave_id();
  const int wm = w >> 1, wn = w & 1, rr = lane & 15, kq = lane >> 4;
  const int jj = t % QKC, c0 = t / QKC;          // staged row of the chunk, first staged column
  const int64_t nchunks = (a.n + QKC - 1) / QKC;
  int64_t jw = ONE ? 0 : jj % a.n_h;             // W row of this thread's next chunk (levels > 1)
  const bool estage = t < QKC * QKB;
  const int eb = t / QKC;
  const bool ecol = estage && k0 + eb < a.K;
  double xv[8], wv[8], ev = 0.0;
  auto load = [&](int64_t c) {
    const int64_t i = c * QKC + jj;
    const bool row = i < a.n;
    const int64_t j = ONE ? i : jw;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int col = c0 + 8 * q;
      xv[q] = (row && r0 + col < a.R) ? a.X[i + (r0 + col) * a.ldX] : 0.0;
      wv[q] = (row && m0 + col < a.M) ? a.w(j, m0 + col) : 0.0;
    }
    if (estage) ev = (row && ecol) ? a.E[i + (k0 + eb) * a.ldE] : 0.0;
    if constexpr (!ONE) jw = (jw + QKC) % a.n_h;
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int col = c0 + 8 * q;
      Xs[buf][jj * QLD + col] = (float)xv[q];
      Ws[buf][jj * QLD + col] = wv[q];
    }
    if (estage) Es[buf][jj * QKB + eb] = ev;
  };
  f4 acc[QKB][2][2];
#pragma unroll
  for (int b = 0; b < QKB; ++b)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[b][i][j] = f4{0.f, 0.f, 0.f, 0.f};
  load(0);
  store(0);
  __syncthreads();
  for (int64_t c = 0; c < nchunks; ++c) {
    const bool more = c + 1 < nchunks;
    if (more) load(c + 1);
    const float* Xb = Xs[c & 1];
    const double* Wb = Ws[c & 1];
    const double* Eb = Es[c & 1];
#pragma unroll
    for (int kk = 0; kk < QKC; kk += 4) {
      const int krow = kk + kq;
      float xa[2];
      double wr[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) xa[i] = Xb[krow * QLD + wm * 32 + i * 16 + rr];
#pragma unroll
      for (int j = 0; j < 2; ++j) wr[j] = Wb[krow * QLD + wn * 32 + j * 16 + rr];
#pragma unroll
      for (int b = 0; b < QKB; ++b) {
        const double e = Eb[krow * QKB + b];
#pragma unroll
        for (int j = 0; j < 2; ++j) {
          const float z = (float)(wr[j] * e);   // the FP64 product rounded once
#pragma unroll
          for (int i = 0; i < 2; ++i) acc[b][i][j] = mfma_f32(xa[i], z, acc[b][i][j]);
        }
      }
    }
    if (more) store((int)((c + 1) & 1));
    __syncthreads();
  }
  // D of the f32 MFMA: lane l holds rows 4 (l / 16) + v (right-hand sides), column l % 16 (modes)
#pragma unroll
  for (int b = 0; b < QKB; ++b) {
    const int64_t k = k0 + b;
    if (k >= a.K) break;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t r = r0 + wm * 32 + i * 16 + 4 * kq + v;
          const int64_t m = m0 + wn * 32 + j * 16 + rr;
          if (r < a.R && m < a.M) a.B[(k * a.M + m) + r * a.ldB] = (double)acc[b][i][j][v];
        }
  }
}

// ------------------------------------------------------------------- bf16
// Thread t stages rows 8 (t % 4) .. + 7 of the chunk for tile column t / 4
// of X and of W; threads t < 4 QKB stage those rows of member t / 4.  LDS
// holds X as bf16 (one column of 32 rows per LDS row), W and E as fp32 copies.
template <int QKB, bool ONE, class WS>
__global__ __launch_bounds__(256) void ztx_bf16_kernel(ZtxLowArgs<WS> a) {
  __shared__ __attribute__((aligned(16))) unsigned short Xs[2][QT * QBS];
  __shared__ __attribute__((aligned(16))) float Ws[2][QT * QWS];
  __shared__ __attribute__((aligned(16))) float Es[2][QKB * QWS];
  int64_t r0, m0, k0;
  if (!ztx_low_tile<QKB>(a, r0, m0, k0)) return;
  const int t = threadIdx.x, lane = lane_id(), w = wave_id();
  const int wm = w >> 1, wn = w & 1, rr = lane & 15, kq = lane >> 4;
  const int seg = t & 3, col = t >> 2;
  const int64_t nchunks = (a.n + QKC - 1) / QKC;
  const bool xcol = r0 + col < a.R, wcol = m0 + col < a.M;
  const bool estage = t < 4 * QKB;
  const bool ecol = estage && k0 + (t >> 2) < a.K;
  const double* xp = a.X + (xcol ? (r0 + col) * a.ldX : 0);
  const double* ep = a.E + (ecol ? (k0 + (t >> 2)) * a.ldE : 0);
  double xr[8], wr[8], er[8];
  auto load = [&](int64_t c) {
    const int64_t i0 = c * QKC + seg * 8;
    int64_t j = ONE ? i0 : i0 % a.n_h;
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const bool row = i0 + q < a.n;
      xr[q] = (row && xcol) ? xp[i0 + q] : 0.0;
      wr[q] = (row && wcol) ? a.w(ONE ? i0 + q : j, m0 + col) : 0.0;
      if (estage) er[q] = (row && ecol) ? ep[i0 + q] : 0.0;
      if constexpr (!ONE) {
        if (++j == a.n_h) j = 0;
      }
    }
  };
  auto store = [&](int buf) {
    unsigned p[4];
#pragma unroll
    for (int q = 0; q < 4; ++q) p[q] = pack2((float)xr[2 * q], (float)xr[2 * q + 1]);
    *reinterpret_cast<s8*>(&Xs[buf][col * QBS + seg * 8]) = __builtin_bit_cast(s8, p);
    float* wd = &Ws[buf][col * QWS + seg * 8];
    *reinterpret_cast<float4*>(wd) = float4{(float)wr[0], (float)wr[1], (float)wr[2], (float)wr[3]};
    *reinterpret_cast<float4*>(wd + 4) = float4{(float)wr[4], (float)wr[5], (float)wr[6], (float)wr[7]};
    if (estage) {
      float* ed = &Es[buf][(t >> 2) * QWS + seg * 8];
      *reinterpret_cast<float4*>(ed) = float4{(float)er[0], (float)er[1], (float)er[2], (float)er[3]};
      *reinterpret_cast<float4*>(ed + 4) = float4{(float)er[4], (float)er[5], (float)er[6], (float)er[7]};
    }
  };
  f4 acc[QKB][2][2];
#pragma unroll
  for (int b = 0; b < QKB; ++b)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[b][i][j] = f4{0.f, 0.f, 0.f, 0.f};
  load(0);
  store(0);
  __syncthreads();
  for (int64_t c = 0; c < nchunks; ++c) {
    const bool more = c + 1 < nchunks;
    if (more) load(c + 1);
    const int buf = (int)(c & 1);
    s8 xf[2];
#pragma unroll
    for (int i = 0; i < 2; ++i) xf[i] = *reinterpret_cast<const s8*>(&Xs[buf][(wm * 32 + i * 16 + rr) * QBS + kq * 8]);
    float4 w0[2], w1[2];
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const float* ws = &Ws[buf][(wn * 32 + j * 16 + rr) * QWS + kq * 8];
      w0[j] = *reinterpret_cast<const float4*>(ws);
      w1[j] = *reinterpret_cast<const float4*>(ws + 4);
    }
#pragma unroll
    for (int b = 0; b < QKB; ++b) {
      const float* es = &Es[buf][b * QWS + kq * 8];
      const float4 e0 = *reinterpret_cast<const float4*>(es);
      const float4 e1 = *reinterpret_cast<const float4*>(es + 4);
#pragma unroll
      for (int j = 0; j < 2; ++j) {
        // the fp32 products of the fp32 copies, rounded to bf16
        unsigned p[4];
        p[0] = pack2(e0.x * w0[j].x, e0.y * w0[j].y);
        p[1] = pack2(e0.z * w0[j].z, e0.w * w0[j].w);
        p[2] = pack2(e1.x * w1[j].x, e1.y * w1[j].y);
        p[3] = pack2(e1.z * w1[j].z, e1.w * w1[j].w);
        const s8 zf = __builtin_bit_cast(s8, p);
#pragma unroll
        for (int i = 0; i < 2; ++i) acc[b][i][j] = mfma_bf16(xf[i], zf, acc[b][i][j]);
      }
    }
    if (more) store((int)((c + 1) & 1));
    __syncthreads();
  }
#pragma unroll
  for (int b = 0; b < QKB; ++b) {
    const int64_t k = k0 + b;
    if (k >= a.K) break;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t r = r0 + wm * 32 + i * 16 + 4 * kq + v;
          const int64_t m = m0 + wn * 32 + j * 16 + rr;
          if (r < a.R && m < a.M) a.B[(k * a.M + m) + r * a.ldB] = (double)acc[b][i][j][v];
        }
  }
}

template <class WS>
hipError_t run_ztx_low(const Inst& in, WS w, int precision, const double* X, int64_t ldX, int64_t R, double* B,
                       int64_t ldB, hipStream_t s) {
  ZtxLowArgs<WS> a;
  a.E = in.E; a.ldE = in.ldE; a.w = w; a.X = X; a.ldX = ldX; a.B = B; a.ldB = ldB;
  a.n = in.n; a.n_h = in.n_h; a.K = in.K; a.M = in.M; a.R = R;
  a.ntr = (int)ceil_div(R, QT); a.ntm = (int)ceil_div(in.M, QT);
  if (precision != LP_FP32 && precision != LP_BF16) return hipErrorInvalidValue;
  int dev = 0, cus = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (cus <= 0) cus = 256;
  // members per tile: 4, halved while the launch would give fewer than two
  // workgroups per compute unit
  const int64_t base = (int64_t)a.ntr * a.ntm;
  int kb = 4;
  while (kb > 1 && base * ceil_div(in.K, kb) < 2 * (int64_t)cus) kb /= 2;
  a.ntk = (int)ceil_div(in.K, kb);
  const int64_t units = base * a.ntk;
  const dim3 grid((unsigned)(8 * ((units + 7) / 8)));
  const bool one = in.n_w == 1;
  const bool f32 = precision == LP_FP32;
#define PC_ZTX_LOW_LAUNCH(KB)                                                                   \
  if (f32) {                                                                                   \
    if (one) hipLaunchKernelGGL((ztx_f32_kernel<KB, true, WS>), grid, dim3(256), 0, s, a);     \
    else hipLaunchKernelGGL((ztx_f32_kernel<KB, false, WS>), grid, dim3(256), 0, s, a);        \
  } else {                                                                                     \
    if (one) hipLaunchKernelGGL((ztx_bf16_kernel<KB, true, WS>), grid, dim3(256), 0, s, a);    \
    else hipLaunchKernelGGL((ztx_bf16_kernel<KB, false, WS>), grid, dim3(256), 0, s, a);       \
  }
  if (kb == 4) { PC_ZTX_LOW_LAUNCH(4) }
  else if (kb == 2) { PC_ZTX_LOW_LAUNCH(2) }
  else { PC_ZTX_LOW_LAUNCH(1) }
#undef PC_ZTX_LOW_LAUNCH
  return hipGetLastError();
}

}  // namespace

hipError_t launch_ztx_lowprec(const Inst& in, int precision, const double* X, int64_t ldX, int64_t R, double* B,
                              int64_t ldB, hipStream_t s) {
  if (R <= 0) return hipSuccess;
  return in.W ? run_ztx_low(in, wdense(in), precision, X, ldX, R, B, ldB, s)
              : run_ztx_low(in, wsep(in), precision, X, ldX, R, B, ldB, s);
}

}  // namespace pc
