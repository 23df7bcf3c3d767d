// The paper's own left inverse for the square case n_w = K (Sec. 3.9,
// eq. InverseSquareRootSwift; steps V1-V5 of Sec. 3.10), behind
// pc_swift_build / pc_swift_apply / pc_swift_destroy (include/pcsqrt.h).
//
//   V1   for every grid column m: w^(m) = A_m^{-1} x^(m), with A_m the K x K
//        block of the member matrix holding the rows of column m
//        (A_m[l, k] = E[l n_h + m, k]) and x^(m) the K values of x there;
//   V2-3 regroup by member: w_k = (w^(0)_k, ..., w^(n_h - 1)_k);
//   V4   x~_k = Delta_b^{-1/2} V_b^T w_k;
//   V5   x~ = (x~_0; ...; x~_{K-1}), row k L + l.
//
// The paper factors each A_m by SVD; here each A_m is inverted once by
// Gauss-Jordan elimination with partial pivoting (the same A_m^{-1} up to
// rounding), at build time, one workgroup per grid column.  V1 then is a
// small FP64 MFMA product per column and right-hand-side tile (after a
// transpose that groups the right-hand sides by grid column), written as the
// rows of an n_h x (K R) matrix whose column k R + r is w_k of right-hand side r:
// that is the regrouping of V2-V3, and V4 becomes one FP64 MFMA product
// V_b^T (L x n_h) times that matrix, scaled by delta^{-1/2} and scattered to
// the member segments of V5.
#include <algorithm>
#include <cmath>
#include <new>

#include "gemm_core.h"
#include "pc_internal.h"
#include "pcsqrt.h"

namespace pc {

constexpr int SW_KMAX = 64;            // K <= 64: one column's block and its inverse fit in LDS
constexpr int SW_LD = 2 * SW_KMAX + 1;

// Gauss-Jordan on [A_m | I] in LDS; writes A_m^{-1} (column-major K x K) to
// Ainv + m K^2.  A pivot with |p| <= K u max|A_m| marks the block singular
// (bad[m] = 1; the inverse is then not used).
__global__ __launch_bounds__(256) void swift_invert_kernel(const double* __restrict__ E, int64_t ldE, int64_t n_h,
                                                           int K, double* __restrict__ Ainv, int* __restrict__ bad) {
  __shared__ double T[SW_KMAX][SW_LD];
  __shared__ double red_v[4];
  __shared__ int red_i[4];
  __shared__ int piv;
  __shared__ double amax;
  const int64_t m = blockIdx.x;
  const int t = threadIdx.x, K2 = 2 * K;
  double mx = 0.0;
  for (int e = t; e < K * K2; e += 256) {
    const int l = e / K2, c = e % K2;
    double v;
    if (c < K) {
      v = E[(int64_t)l * n_h + m + (int64_t)c * ldE];
      mx = fmax(mx, fabs(v));
    } else {
      v = (c - K == l) ? 1.0 : 0.0;
    }
    T[l][c] = v;
  }
  mx = wave_max(mx);
  if (lane_id() == 0) red_v[wave_id()] = mx;
  __syncthreads();
  if (t == 0) amax = fmax(fmax(red_v[0], red_v[1]), fmax(red_v[2], red_v[3]));
  __syncthreads();
  const double thr = (double)K * 0x1p-53 * amax;
  int singular = 0;
  for (int j = 0; j < K; ++j) {
    // pivot: the row i >= j with the largest |T[i][j]| (first such row on ties)
    if (t < 64) {
      double bv = -1.0;
      int bi = j;
      for (int i = j + t; i < K; i += 64) {
        const double a = fabs(T[i][j]);
        if (a > bv) { bv = a; bi = i; }
      }
      for (int off = 32; off > 0; off >>= 1) {
        const double ov = __shfl_xor(bv, off, 64);
        const int oi = __shfl_xor(bi, off, 64);
        if (ov > bv || (ov == bv && oi < bi)) { bv = ov; bi = oi; }
      }
      if (t == 0) piv = bi;
    }
    __syncthreads();
    const int p = piv;
    if (p != j)
      for (int c = t; c < K2; c += 256) {
        const double a = T[j][c];
        T[j][c] = T[p][c];
        T[p][c] = a;
      }
    __syncthreads();
    const double d = T[j][j];
    if (!(fabs(d) > thr)) singular = 1;
    const double inv = 1.0 / d;
    __syncthreads();
    for (int c = t; c < K2; c += 256) T[j][c] *= inv;
    __syncthreads();
    for (int e = t; e < K * K2; e += 256) {
      const int i = e / K2, c = e % K2;
      if (i != j && c != j) T[i][c] = fma(-T[i][j], T[j][c], T[i][c]);
    }
    __syncthreads();
    for (int i = t; i < K; i += 256)
      if (i != j) T[i][j] = 0.0;
    __syncthreads();
  }
  double* out = Ainv + m * (int64_t)K * K;
  for (int e = t; e < K * K; e += 256) {
    const int i = e % K, c = e / K;
    out[i + (int64_t)c * K] = T[i][K + c];
  }
  if (t == 0) bad[m] = singular;
}

// V1 reads the K values of x in grid column m, x[l n_h + m] (l < K), for
// every right-hand side: a stride of n_h between them.  First X is
// transposed into Xt[(m K + l) R + r] (one 64 x 64 tile of (grid column,
// right-hand side) per workgroup and level, through LDS, so that both the
// reads along m and the writes along r are coalesced); then per grid column
// one FP64 MFMA product Wm[m, k R + r] = sum_l Ainv_m[k, l] Xt[m, l, r]
// (swift_v1 of SwiftV1Prob), whose operands are contiguous blocks.
__global__ __launch_bounds__(256) void swift_xt_kernel(const double* __restrict__ X, int64_t ldX, int64_t n_h, int K,
                                                       int64_t R, double* __restrict__ Xt) {
  __shared__ double T[64][65];
  const int64_t m0 = (int64_t)blockIdx.x * 64, r0 = (int64_t)blockIdx.y * 64;
  const int64_t l = blockIdx.z;
  const int t = threadIdx.x, a = t & 63, g = t >> 6;
#pragma unroll 4
  for (int j = g; j < 64; j += 4) {          // read along m (contiguous in X)
    const int64_t m = m0 + a, r = r0 + j;
    T[j][a] = (m < n_h && r < R) ? X[l * n_h + m + r * ldX] : 0.0;
  }
  __syncthreads();
#pragma unroll 4
  for (int i = g; i < 64; i += 4) {          // write along r (contiguous in Xt)
    const int64_t m = m0 + i, r = r0 + a;
    if (m < n_h && r < R) Xt[(m * K + l) * R + r] = T[a][i];
  }
}

// V1 per grid column m and tile of 64 right-hand sides:
// Wm[m, k R + r] = sum_l Ainv_m[k, l] Xt[m, l, r] (rows k of the product, columns r).
struct SwiftV1Prob {
  static constexpr int BM = 64, BN = 64, WM = 2, WN = 2, KC = 16;
  static constexpr int LDA = BM + 1, LDB = BN;
  static constexpr int NA = BM * KC / 256, NB_ = BN * KC / 256;
  const double* Ainv; int K;
  const double* Xt;
  double* Wm; int64_t ldw;
  int64_t R; int nrt;

  struct Ctx { bool valid; int64_t m, r0; int nchunks; };
  struct ARegs { double v[NA]; };
  struct BRegs { double v[NB_]; };

  __device__ Ctx ctx(int b) const {
    Ctx c;
    c.valid = true;
    c.m = b / nrt;
    c.r0 = (int64_t)(b % nrt) * BN;
    c.nchunks = (K + KC - 1) / KC;
    return c;
  }
  __device__ void loadA(const Ctx& c, int chunk, ARegs& r) const {
    const double* A = Ainv + c.m * (int64_t)K * K;
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = threadIdx.x + 256 * q, row = e % BM, kk = e / BM;   // row k contiguous
      const int l = chunk * KC + kk;
      r.v[q] = (row < K && l < K) ? A[row + l * K] : 0.0;
    }
  }
  __device__ void storeA(const ARegs& r, double* As) const {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = threadIdx.x + 256 * q;
      As[(e / BM) * LDA + e % BM] = r.v[q];
    }
  }
  __device__ void loadB(const Ctx& c, int chunk, BRegs& r) const {
    const double* B = Xt + c.m * (int64_t)K * R;
#pragma unroll
    for (int q = 0; q < NB_; ++q) {
      const int e = threadIdx.x + 256 * q, col = e % BN, kk = e / BN;  // right-hand side contiguous
      const int l = chunk * KC + kk;
      r.v[q] = (c.r0 + col < R && l < K) ? B[(int64_t)l * R + c.r0 + col] : 0.0;
    }
  }
  __device__ void storeB(const BRegs& r, double* Bs) const {
#pragma unroll
    for (int q = 0; q < NB_; ++q) {
      const int e = threadIdx.x + 256 * q;
      Bs[(e / BN) * LDB + e % BN] = r.v[q];
    }
  }
  __device__ void epilogue(const Ctx& c, const TileF64<BM, BN, WM, WN>& acc) const {
    acc.for_each([&](int row, int col, double v) {
      const int64_t r = c.r0 + col;
      if (row >= K || r >= R) return;
      Wm[c.m * ldw + (int64_t)row * R + r] = v;
    });
  }
};

// V4-V5: Y[k L + l, r] = delta_l^{-1/2} sum_m Vb[m, l] Wm[m, k R + r], as a
// GEMM C (L x K R) = Vb^T Wm over 64 x 64 tiles, contraction over m in
// chunks of 32 (twice the bytes in flight of 16-deep chunks, half the barriers).
struct SwiftProjProb {
  static constexpr int BM = 64, BN = 64, WM = 2, WN = 2, KC = 32;
  static constexpr int LDA = BM + 1, LDB = BN;
  static constexpr int NA = BM * KC / 256, NB_ = BN * KC / 256;
  const double* Vb; int64_t ldV;
  const double* Wm; int64_t ldw;
  const double* rsd;               // delta^{-1/2}
  double* Y; int64_t ldY;
  int64_t L, NC, n_h, R;
  int64_t tm, ntiles;

  struct Ctx { bool valid; int64_t l0, c0; int nchunks; };
  struct ARegs { double v[NA]; };
  struct BRegs { double v[NB_]; };

  __device__ Ctx ctx(int b) const {
    Ctx c;
    c.valid = b < ntiles;
    c.l0 = (int64_t)(b % tm) * BM;
    c.c0 = (int64_t)(b / tm) * BN;
    c.nchunks = (int)((n_h + KC - 1) / KC);
    return c;
  }
  __device__ void loadA(const Ctx& c, int chunk, ARegs& r) const {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = threadIdx.x + 256 * q, kk = e % KC, row = e / KC;   // along m (contiguous in Vb)
      const int64_t l = c.l0 + row, m = (int64_t)chunk * KC + kk;
      r.v[q] = (l < L && m < n_h) ? Vb[m + l * ldV] : 0.0;
    }
  }
  __device__ void storeA(const ARegs& r, double* As) const {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = threadIdx.x + 256 * q;
      As[(e % KC) * LDA + e / KC] = r.v[q];
    }
  }
  __device__ void loadB(const Ctx& c, int chunk, BRegs& r) const {
#pragma unroll
    for (int q = 0; q < NB_; ++q) {
      const int e = threadIdx.x + 256 * q, col = e % BN, kk = e / BN;
      const int64_t cc = c.c0 + col, m = (int64_t)chunk * KC + kk;
      r.v[q] = (cc < NC && m < n_h) ? Wm[m * ldw + cc] : 0.0;
    }
  }
  __device__ void storeB(const BRegs& r, double* Bs) const {
#pragma unroll
    for (int q = 0; q < NB_; ++q) {
      const int e = threadIdx.x + 256 * q;
      Bs[(e / BN) * LDB + e % BN] = r.v[q];
    }
  }
  __device__ void epilogue(const Ctx& c, const TileF64<BM, BN, WM, WN>& acc) const {
    acc.for_each([&](int row, int col, double v) {
      const int64_t l = c.l0 + row, cc = c.c0 + col;
      if (l >= L || cc >= NC) return;
      const int64_t k = cc / R, r = cc % R;
      Y[k * L + l + r * ldY] = v * rsd[l];
    });
  }
};

__global__ void swift_rsqrt_kernel(const double* __restrict__ delta, int64_t L, double* __restrict__ rsd,
                                   int* __restrict__ bad) {
  for (int64_t l = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; l < L; l += (int64_t)gridDim.x * blockDim.x) {
    const double d = delta[l];
    if (!(d > 0.0) || !isfinite(d)) atomicOr(bad, 1);
    rsd[l] = 1.0 / sqrt(d);
  }
}

__global__ void swift_any_kernel(const int* __restrict__ flags, int64_t n, int* __restrict__ out) {
  int v = 0;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x)
    v |= flags[i];
  if (v) atomicOr(out, 1);
}

}  // namespace pc

struct pc_swift {
  int device = 0;
  int64_t n_h = 0, K = 0, L = 0, max_rhs = 0;
  const double* E = nullptr; int64_t ldE = 0;
  const double* Vb = nullptr; int64_t ldV = 0;
  double* Ainv = nullptr;   // n_h blocks K x K
  double* rsd = nullptr;    // L: delta^{-1/2}
  double* Wm = nullptr;     // n_h x (K max_rhs), row-major
  double* Xt = nullptr;     // n_h K max_rhs: the right-hand sides grouped by grid column
  int* bad = nullptr;       // n_h singular flags, then [n_h] delta flag, [n_h + 1] any
};

static void swift_free(pc_swift* s) {
  if (!s) return;
  (void)hipDeviceSynchronize();
  (void)hipFree(s->Ainv);
  (void)hipFree(s->rsd);
  (void)hipFree(s->Wm);
  (void)hipFree(s->Xt);
  (void)hipFree(s->bad);
  delete s;
}

extern "C" pc_status pc_swift_build(int64_t n_h, int64_t K, int64_t L, const double* E, int64_t ldE,
                                    const double* Vb, int64_t ldV, const double* delta, int64_t max_rhs,
                                    void* stream, pc_swift** out) {
  if (!out) return PC_ERR_INVALID_ARG;
  *out = nullptr;
  if (n_h < 1 || K < 1 || L < 1 || max_rhs < 0) return PC_ERR_SHAPE;
  if (K > pc::SW_KMAX || L > n_h) return PC_ERR_SHAPE;
  if (!E || !Vb || !delta || ldE < n_h * K || ldV < n_h) return PC_ERR_INVALID_ARG;
  pc_swift* s = new (std::nothrow) pc_swift();
  if (!s) return PC_ERR_OOM;
  (void)hipGetDevice(&s->device);
  s->n_h = n_h; s->K = K; s->L = L; s->max_rhs = std::max<int64_t>(max_rhs, 1);
  s->E = E; s->ldE = ldE; s->Vb = Vb; s->ldV = ldV;
  hipStream_t st = (hipStream_t)stream;
  bool ok = hipMalloc((void**)&s->Ainv, sizeof(double) * (size_t)(n_h * K * K)) == hipSuccess &&
            hipMalloc((void**)&s->rsd, sizeof(double) * (size_t)L) == hipSuccess &&
            hipMalloc((void**)&s->Wm, sizeof(double) * (size_t)(n_h * K * s->max_rhs)) == hipSuccess &&
            hipMalloc((void**)&s->Xt, sizeof(double) * (size_t)(n_h * K * s->max_rhs)) == hipSuccess &&
            hipMalloc((void**)&s->bad, sizeof(int) * (size_t)(n_h + 2)) == hipSuccess;
  if (!ok) { swift_free(s); return PC_ERR_OOM; }
  int h[2] = {0, 0};
  ok = pc::launch_fill_int(s->bad + n_h, 0, 2, st) == hipSuccess;
  if (ok) {
    hipLaunchKernelGGL(pc::swift_rsqrt_kernel, dim3((unsigned)std::min<int64_t>(pc::ceil_div(L, 256), 64)), dim3(256),
                       0, st, delta, L, s->rsd, s->bad + n_h);
    hipLaunchKernelGGL(pc::swift_invert_kernel, dim3((unsigned)n_h), dim3(256), 0, st, E, ldE, n_h, (int)K, s->Ainv,
                       s->bad);
    hipLaunchKernelGGL(pc::swift_any_kernel, dim3((unsigned)std::min<int64_t>(pc::ceil_div(n_h, 256), 64)), dim3(256),
                       0, st, s->bad, n_h, s->bad + n_h + 1);
    ok = hipGetLastError() == hipSuccess &&
         hipMemcpyAsync(h, s->bad + n_h, sizeof(int) * 2, hipMemcpyDeviceToHost, st) == hipSuccess &&
         hipStreamSynchronize(st) == hipSuccess;
  }
  if (!ok) { swift_free(s); return PC_ERR_DEVICE; }
  if (h[0]) { swift_free(s); return PC_ERR_INVALID_ARG; }   // an eigenvalue not positive
  if (h[1]) { swift_free(s); return PC_ERR_NOT_SPD; }       // a singular block A_m
  *out = s;
  return PC_OK;
}

extern "C" pc_status pc_swift_apply(pc_swift* s, const double* X, int64_t ldX, int64_t R, double* Y, int64_t ldY,
                                    void* stream) {
  if (!s || R < 0) return PC_ERR_INVALID_ARG;
  if (R == 0) return PC_OK;
  if (R > s->max_rhs) return PC_ERR_TOO_MANY_RHS;
  if (!X || !Y || ldX < s->n_h * s->K || ldY < s->K * s->L) return PC_ERR_INVALID_ARG;
  (void)hipSetDevice(s->device);
  hipStream_t st = (hipStream_t)stream;
  const int64_t ldw = s->K * R;
  hipLaunchKernelGGL(pc::swift_xt_kernel, dim3((unsigned)pc::ceil_div(s->n_h, 64), (unsigned)pc::ceil_div(R, 64),
                                                (unsigned)s->K),
                     dim3(256), 0, st, X, ldX, s->n_h, (int)s->K, R, s->Xt);
  pc::SwiftV1Prob v1;
  v1.Ainv = s->Ainv; v1.K = (int)s->K; v1.Xt = s->Xt; v1.Wm = s->Wm; v1.ldw = ldw; v1.R = R;
  v1.nrt = (int)pc::ceil_div(R, pc::SwiftV1Prob::BN);
  hipLaunchKernelGGL(pc::gemm_f64_kernel<pc::SwiftV1Prob>, dim3((unsigned)(s->n_h * v1.nrt)), dim3(256), 0, st, v1);
  pc::SwiftProjProb g;
  g.Vb = s->Vb; g.ldV = s->ldV; g.Wm = s->Wm; g.ldw = ldw; g.rsd = s->rsd; g.Y = Y; g.ldY = ldY;
  g.L = s->L; g.NC = s->K * R; g.n_h = s->n_h; g.R = R;
  g.tm = pc::ceil_div(s->L, pc::SwiftProjProb::BM);
  g.ntiles = g.tm * pc::ceil_div(g.NC, pc::SwiftProjProb::BN);
  hipLaunchKernelGGL(pc::gemm_f64_kernel<pc::SwiftProjProb>, dim3((unsigned)g.ntiles), dim3(256), 0, st, g);
  return hipGetLastError() == hipSuccess ? PC_OK : PC_ERR_DEVICE;
}

extern "C" pc_status pc_swift_destroy(pc_swift* s) {
  swift_free(s);
  return PC_OK;
}
