// Products with the modulated square root Z, never forming Z (FP64, MFMA).
//
//  Z^T x  (the start of the solve and of every refinement step):
//      b[k*M + m, r] = sum_j W[j, m] * u[j, (k, r)],
//      u[j, (k, r)]  = sum_l E[l*n_h + j, k] * X[l*n_h + j, r]
//    a per-grid-column contraction over the levels (the shape of the
//    paper's column step V1) followed by a projection on the modes (the
//    shape of its member step V4).  GEMM rows = (k, r), cols = m, depth = j;
//    the u operand is formed while it is staged in LDS.
//
//  Z y  (the back-transform, and the residual x - Z y of refinement):
//      (Z y)[i, r] = sum_{k,m} E[i, k] * W[j(i), m] * Y[k*M + m, r],
//    GEMM rows = r, cols = i, depth = (k, m); the Z operand E[i,k] W[j,m] is
//    formed while it is staged in LDS.
#include "gemm_core.h"
#include "pc_internal.h"

namespace pc {

// ------------------------------------------------------------------ Z^T X
template <int BM_, int BN_, int WM_, int WN_>
struct ZtxProb {
  static constexpr int BM = BM_, BN = BN_, WM = WM_, WN = WN_, KC = 16;
  static constexpr int LDA = BM + 1, LDB = BN + 1;
  static constexpr int NA = BM * KC / 256, NB_ = BN * KC / 256;
  static_assert(NA >= 1 && NB_ >= 1, "tile too small for 256 threads");
  const double* E; int64_t ldE;
  const double* W; int64_t ldW;
  const double* X; int64_t ldX;
  double* Bout; int64_t ldB;
  int64_t n_h, n_w, K, M, R, KR;
  int ntr, ntc;   // tiles along rows (k,r) and cols (m)

  struct Ctx { bool valid; int64_t c0, m0; int nchunks; };
  struct ARegs { double v[NA]; };
  struct BRegs { double v[NB_]; };

  __device__ Ctx ctx(int tile) const {
    Ctx c;
    const int tr = tile % ntr, tc = tile / ntr;
    c.valid = tc < ntc;
    c.c0 = (int64_t)tr * BM;
    c.m0 = (int64_t)tc * BN;
    c.nchunks = (int)((n_h + KC - 1) / KC);
    return c;
  }
  // element e of this thread: jj = e_index % KC (fastest, coalesced), row = e_index / KC
  __device__ void loadA(const Ctx& c, int chunk, ARegs& r) const {
    const int t = threadIdx.x;
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int e = t + 256 * i;
      const int jj = e % KC, row = e / KC;
      const int64_t j = (int64_t)chunk * KC + jj, cc = c.c0 + row;
      double s = 0.0;
      if (j < n_h && cc < KR) {
        const int64_t k = cc / R, rr = cc % R;
        const double* Ek = E + k * ldE + j;
        const double* Xr = X + rr * ldX + j;
        for (int64_t l = 0; l < n_w; ++l) s += Ek[l * n_h] * Xr[l * n_h];
      }
      r.v[i] = s;
    }
  }
  __device__ void storeA(const ARegs& r, double* As) const {
    const int t = threadIdx.x;
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int e = t + 256 * i;
      As[(e % KC) * LDA + e / KC] = r.v[i];
    }
  }
  __device__ void loadB(const Ctx& c, int chunk, BRegs& r) const {
    const int t = threadIdx.x;
#pragma unroll
    for (int i = 0; i < NB_; ++i) {
      const int e = t + 256 * i;
      const int jj = e % KC, col = e / KC;
      const int64_t j = (int64_t)chunk * KC + jj, m = c.m0 + col;
      r.v[i] = (j < n_h && m < M) ? W[j + m * ldW] : 0.0;
    }
  }
  __device__ void storeB(const BRegs& r, double* Bs) const {
    const int t = threadIdx.x;
#pragma unroll
    for (int i = 0; i < NB_; ++i) {
      const int e = t + 256 * i;
      Bs[(e % KC) * LDB + e / KC] = r.v[i];
    }
  }
  __device__ void epilogue(const Ctx& c, const TileF64<BM, BN, WM, WN>& acc) const {
    acc.for_each([&](int row, int col, double v) {
      const int64_t cc = c.c0 + row, m = c.m0 + col;
      if (cc >= KR || m >= M) return;
      const int64_t k = cc / R, rr = cc % R;
      Bout[(k * M + m) + rr * ldB] = v;
    });
  }
};

template <class P>
static hipError_t run_ztx(const Inst& in, const double* X, int64_t ldX, int64_t R, double* B, int64_t ldB,
                          hipStream_t s) {
  P pr;
  pr.E = in.E; pr.ldE = in.ldE; pr.W = in.W; pr.ldW = in.ldW;
  pr.X = X; pr.ldX = ldX; pr.Bout = B; pr.ldB = ldB;
  pr.n_h = in.n_h; pr.n_w = in.n_w; pr.K = in.K; pr.M = in.M; pr.R = R; pr.KR = in.K * R;
  pr.ntr = (int)ceil_div(pr.KR, P::BM);
  pr.ntc = (int)ceil_div(in.M, P::BN);
  const int64_t tiles = (int64_t)pr.ntr * pr.ntc;
  hipLaunchKernelGGL(gemm_f64_kernel<P>, dim3((unsigned)tiles), dim3(256), 0, s, pr);
  return hipGetLastError();
}

hipError_t launch_ztx(const Inst& in, const double* X, int64_t ldX, int64_t R, double* B, int64_t ldB,
                      hipStream_t s) {
  if (R <= 0) return hipSuccess;
  if (in.M <= 32) return run_ztx<ZtxProb<128, 32, 4, 1>>(in, X, ldX, R, B, ldB, s);
  return run_ztx<ZtxProb<64, 64, 2, 2>>(in, X, ldX, R, B, ldB, s);
}

// ------------------------------------------------------------------- Z Y
template <int BM_, int BN_, int WM_, int WN_>
struct ZyProb {
  static constexpr int BM = BM_, BN = BN_, WM = WM_, WN = WN_, KC = 16;
  static constexpr int LDA = BM + 1, LDB = BN;
  static constexpr int NA = BM * KC / 256, NB_ = BN * KC / 256;
  static_assert(NA >= 1 && NB_ >= 1, "tile too small for 256 threads");
  const double* E; int64_t ldE;
  const double* W; int64_t ldW;
  const double* Y; int64_t ldY;
  const double* Xs; int64_t ldXs;   // optional: out = Xs - Z Y
  double* Out; int64_t ldO;
  int64_t n_h, n, K, M, KM, R;
  int ntr, ntc;   // tiles along rows (r) and cols (i)

  struct Ctx { bool valid; int64_t r0, i0; int nchunks; };
  struct ARegs { double v[NA]; };
  struct BRegs { double v[NB_]; };

  __device__ Ctx ctx(int tile) const {
    Ctx c;
    const int tr = tile % ntr, tc = tile / ntr;
    c.valid = tc < ntc;
    c.r0 = (int64_t)tr * BM;
    c.i0 = (int64_t)tc * BN;
    c.nchunks = (int)((KM + KC - 1) / KC);
    return c;
  }
  __device__ void loadA(const Ctx& c, int chunk, ARegs& r) const {
    const int t = threadIdx.x;
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int e = t + 256 * i;
      const int kk = e % KC, row = e / KC;
      const int64_t q = (int64_t)chunk * KC + kk, rr = c.r0 + row;
      r.v[i] = (q < KM && rr < R) ? Y[q + rr * ldY] : 0.0;
    }
  }
  __device__ void storeA(const ARegs& r, double* As) const {
    const int t = threadIdx.x;
#pragma unroll
    for (int i = 0; i < NA; ++i) {
      const int e = t + 256 * i;
      As[(e % KC) * LDA + e / KC] = r.v[i];
    }
  }
  __device__ void loadB(const Ctx& c, int chunk, BRegs& r) const {
    const int t = threadIdx.x;
#pragma unroll
    for (int i = 0; i < NB_; ++i) {
      const int e = t + 256 * i;
      const int col = e % BN, kk = e / BN;
      const int64_t q = (int64_t)chunk * KC + kk, ii = c.i0 + col;
      double z = 0.0;
      if (q < KM && ii < n) {
        const int64_t k = q / M, m = q % M, j = ii % n_h;
        z = E[ii + k * ldE] * W[j + m * ldW];
      }
      r.v[i] = z;
    }
  }
  __device__ void storeB(const BRegs& r, double* Bs) const {
    const int t = threadIdx.x;
#pragma unroll
    for (int i = 0; i < NB_; ++i) {
      const int e = t + 256 * i;
      Bs[(e / BN) * LDB + e % BN] = r.v[i];
    }
  }
  __device__ void epilogue(const Ctx& c, const TileF64<BM, BN, WM, WN>& acc) const {
    acc.for_each([&](int row, int col, double v) {
      const int64_t rr = c.r0 + row, ii = c.i0 + col;
      if (rr >= R || ii >= n) return;
      Out[ii + rr * ldO] = Xs ? Xs[ii + rr * ldXs] - v : v;
    });
  }
};

template <class P>
static hipError_t run_zy(const Inst& in, const double* Y, int64_t ldY, int64_t R, const double* Xs,
                         int64_t ldXs, double* out, int64_t ldOut, hipStream_t s) {
  P pr;
  pr.E = in.E; pr.ldE = in.ldE; pr.W = in.W; pr.ldW = in.ldW;
  pr.Y = Y; pr.ldY = ldY; pr.Xs = Xs; pr.ldXs = ldXs; pr.Out = out; pr.ldO = ldOut;
  pr.n_h = in.n_h; pr.n = in.n; pr.K = in.K; pr.M = in.M; pr.KM = in.KM; pr.R = R;
  pr.ntr = (int)ceil_div(R, P::BM);
  pr.ntc = (int)ceil_div(in.n, P::BN);
  const int64_t tiles = (int64_t)pr.ntr * pr.ntc;
  hipLaunchKernelGGL(gemm_f64_kernel<P>, dim3((unsigned)tiles), dim3(256), 0, s, pr);
  return hipGetLastError();
}

hipError_t launch_zy(const Inst& in, const double* Y, int64_t ldY, int64_t R, const double* Xs, int64_t ldXs,
                     double* out, int64_t ldOut, hipStream_t s) {
  if (R <= 0) return hipSuccess;
  if (R <= 16) return run_zy<ZyProb<16, 128, 1, 4>>(in, Y, ldY, R, Xs, ldXs, out, ldOut, s);
  if (R <= 32) return run_zy<ZyProb<32, 128, 1, 4>>(in, Y, ldY, R, Xs, ldXs, out, ldOut, s);
  return run_zy<ZyProb<64, 64, 2, 2>>(in, Y, ldY, R, Xs, ldXs, out, ldOut, s);
}

}  // namespace pc
