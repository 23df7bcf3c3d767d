// Products with the modulated square root Z, never forming Z (FP64, MFMA).
//
//  Z^T x  (the start of the solve and of every refinement step):
//      b[k*M + m, r] = sum_i E[i, k] W[j(i), m] X[i, r],   j(i) = i mod n_h,
//    per member a GEMM X^T (diag(e_k) W) over the n rows of Z; the
//    scaling by e_k is applied when the MFMA operand is formed.
//
//  Z y  (the back-transform, the residual x - Z y of refinement, and the
//  Hybrid product (1 - beta) v + beta Z (Z^T v)): out = alpha xs + beta (Z y),
//      (Z y)[i, r] = sum_{k,m} E[i, k] * W[j(i), m] * Y[k*M + m, r],
//    GEMM rows = r, cols = i, depth = (k, m); the Z operand E[i,k] W[j,m] is
//    formed while it is staged in LDS.
#include "gemm_core.h"
#include "pc_internal.h"

#include <algorithm>

namespace pc {

// ------------------------------------------------------------------ Z^T X
// b_k = (X^T Z_k)^T with Z_k[i, m] = E[i, k] W[j(i), m], the contraction over
// the n rows i = l n_h + j of Z (j(i) = i mod n_h; one level: j = i);
// tile = 64 right-hand sides x 64 modes of KB consecutive members k (KB = 4,
// or 2 or 1 when larger tiles would leave compute units without one).  The
// staged X and W rows serve all of the tile's members: each member's column
// of E scales the W rows when the MFMA fragment is read.  Several levels run
// through the same MFMA contraction over all n rows rather than forming the
// level sums sum_l E[l n_h + j, k] X[l n_h + j, r] first: that operand would
// be re-formed for every mode tile from n_w scalar loads of each factor per
// element.  With few tiles the row range is split in two halves accumulated
// with two atomic adds onto a zeroed output (two addends onto zero: the same
// result in either order).
constexpr int ZT = 64, ZKC = 32, ZLD = ZT + 1;
constexpr int ZNQ = ZKC * ZT / 256;     // X and W values staged per thread and chunk

template <class WS>
struct Ztx1Args {
  const double* E; int64_t ldE;
  WS w;
  const double* X; int64_t ldX;
  double* B; int64_t ldB;
  int64_t n, n_h, K, M, R;
  int ntr, ntm, ntk, split;
  int64_t jlen;
  const int* skip;
};

template <int ZKB, bool ONE, class WS>
__global__ __launch_bounds__(256) void ztx1_kernel(Ztx1Args<WS> a) {
  if (a.skip && *a.skip) return;
  __shared__ double Xs[2][ZKC * ZLD];
  __shared__ double Ws[2][ZKC * ZLD];
  __shared__ double Es[2][ZKC * ZKB];
  const int64_t ntiles = (int64_t)a.ntr * a.ntm * a.ntk;
  const int64_t units = ntiles * a.split;
  const int64_t per = (units + 7) / 8;
  const int64_t u = (blockIdx.x % 8) * per + blockIdx.x / 8;     // contiguous ranges per XCD
  if (u >= units) return;
  const int part = (int)(u / ntiles);
  int64_t tile = u % ntiles;
  const int tr = (int)(tile % a.ntr); tile /= a.ntr;
  const int tm = (int)(tile % a.ntm);
  const int64_t k0 = (tile / a.ntm) * ZKB;                         // first member of the tile
  const int64_t r0 = (int64_t)tr * ZT, m0 = (int64_t)tm * ZT;
  const int64_t jbeg = (int64_t)part * a.jlen;
  const int64_t jend = jbeg + a.jlen < a.n ? jbeg + a.jlen : a.n;
  const int nchunks = (int)((jend - jbeg + ZKC - 1) / ZKC);
  const int t = threadIdx.x, lane = lane_id(), w = wave_id();
  const int wm = w >> 1, wn = w & 1, rr = lane & 15, kq = lane >> 4;

  double xv[ZNQ], wv[ZNQ], ev = 0.0;
  // every element this thread stages is in row t % ZKC of the chunk; its W row
  // for the next chunk to load (several levels)
  int64_t jw = ONE ? 0 : (jbeg + t % ZKC) % a.n_h;
  // E: thread t < ZKC * ZKB stages member t / ZKC, row t % ZKC (zero past K)
  const int ej = t % ZKC, ek = t / ZKC;
  const bool estage = t < ZKC * ZKB;
  const double* Ek = a.E + (k0 + ek) * a.ldE;
  const bool evalid = estage && k0 + ek < a.K;
  auto load = [&](int chunk) {
    const int64_t j0 = jbeg + (int64_t)chunk * ZKC;
#pragma unroll
    for (int q = 0; q < ZNQ; ++q) {
      const int e = t + 256 * q, jj = e % ZKC, col = e / ZKC;
      const int64_t j = j0 + jj;
      xv[q] = (j < jend && r0 + col < a.R) ? a.X[j + (r0 + col) * a.ldX] : 0.0;
      wv[q] = (j < jend && m0 + col < a.M) ? a.w(ONE ? j : jw, m0 + col) : 0.0;
    }
    if (estage) ev = (evalid && j0 + ej < jend) ? Ek[j0 + ej] : 0.0;
    if constexpr (!ONE) jw = (jw + ZKC) % a.n_h;
  };
  auto store = [&](int buf) {
#pragma unroll
    for (int q = 0; q < ZNQ; ++q) {
      const int e = t + 256 * q, jj = e % ZKC, col = e / ZKC;
      Xs[buf][jj * ZLD + col] = xv[q];
      Ws[buf][jj * ZLD + col] = wv[q];
    }
    if (estage) Es[buf][ej * ZKB + ek] = ev;
  };
  d4 acc[ZKB][2][2];
#pragma unroll
  for (int b = 0; b < ZKB; ++b)
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j) acc[b][i][j] = d4{0.0, 0.0, 0.0, 0.0};
  if (nchunks > 0) {
    load(0);
    store(0);
    __syncthreads();
    for (int c = 0; c < nchunks; ++c) {
      const bool more = c + 1 < nchunks;
      if (more) load(c + 1);
      const double* Xb = Xs[c & 1];
      const double* Wb = Ws[c & 1];
      const double* Eb = Es[c & 1];
#pragma unroll
      for (int kk = 0; kk < ZKC; kk += 4) {
        const int krow = kk + kq;
        double av[2], wr[2];
#pragma unroll
        for (int i = 0; i < 2; ++i) av[i] = Xb[krow * ZLD + wm * 32 + i * 16 + rr];
#pragma unroll
        for (int j = 0; j < 2; ++j) wr[j] = Wb[krow * ZLD + wn * 32 + j * 16 + rr];
#pragma unroll
        for (int b = 0; b < ZKB; ++b) {
          const double e = Eb[krow * ZKB + b];
#pragma unroll
          for (int i = 0; i < 2; ++i)
#pragma unroll
            for (int j = 0; j < 2; ++j) acc[b][i][j] = mfma_f64(av[i], wr[j] * e, acc[b][i][j]);
        }
      }
      if (more) store((c + 1) & 1);
      __syncthreads();
    }
  }
#pragma unroll
  for (int b = 0; b < ZKB; ++b) {
    const int64_t k = k0 + b;
    if (k >= a.K) break;
#pragma unroll
    for (int i = 0; i < 2; ++i)
#pragma unroll
      for (int j = 0; j < 2; ++j)
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const int64_t r = r0 + wm * 32 + i * 16 + kq + 4 * v;
          const int64_t m = m0 + wn * 32 + j * 16 + rr;
          if (r >= a.R || m >= a.M) continue;
          double* dst = &a.B[(k * a.M + m) + r * a.ldB];
          if (a.split == 1) *dst = acc[b][i][j][v];
          else atomicAdd(dst, acc[b][i][j][v]);
        }
  }
}

__global__ void zero_block_kernel(double* B, int64_t ld, int64_t rows, int64_t cols, const int* skip) {
  if (skip && *skip) return;
  const int64_t c = blockIdx.y;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < rows; i += (int64_t)gridDim.x * blockDim.x)
    B[i + c * ld] = 0.0;
}

template <class WS>
static hipError_t run_ztx1(const Inst& in, WS w, const double* X, int64_t ldX, int64_t R, double* B, int64_t ldB,
                           hipStream_t s, const int* skip) {
  Ztx1Args<WS> a;
  a.skip = skip;
  a.E = in.E; a.ldE = in.ldE; a.w = w; a.X = X; a.ldX = ldX; a.B = B; a.ldB = ldB;
  a.n = in.n; a.n_h = in.n_h; a.K = in.K; a.M = in.M; a.R = R;
  a.ntr = (int)ceil_div(R, ZT); a.ntm = (int)ceil_div(in.M, ZT);
  int dev = 0, cus = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (cus <= 0) cus = 256;
  // members per tile: 4, halved while the launch (with a split row range)
  // would still give fewer than two workgroups per compute unit
  const int64_t base = (int64_t)a.ntr * a.ntm;
  int kb = 4;
  while (kb > 1 && base * ceil_div(in.K, kb) * (in.n >= 4 * ZKC ? 2 : 1) < 2 * (int64_t)cus) kb /= 2;
  a.ntk = (int)ceil_div(in.K, kb);
  const int64_t ntiles = base * a.ntk;
  a.split = (ntiles < 2 * (int64_t)cus && in.n >= 4 * ZKC) ? 2 : 1;
  if (in.tune_ztx_split == 1 || (in.tune_ztx_split == 2 && in.n >= 2 * ZKC)) a.split = in.tune_ztx_split;
  a.jlen = round_up(ceil_div(in.n, a.split), ZKC);
  if (a.split == 2) {
    const unsigned gx = (unsigned)std::min<int64_t>(ceil_div(in.KM, 256), 64);
    hipLaunchKernelGGL(zero_block_kernel, dim3(gx, (unsigned)R), dim3(256), 0, s, B, ldB, in.KM, R, skip);
  }
  const int64_t units = ntiles * a.split;
  const dim3 grid((unsigned)(8 * ((units + 7) / 8)));
  const bool one = in.n_w == 1;
  if (kb == 4) {
    if (one) hipLaunchKernelGGL((ztx1_kernel<4, true, WS>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((ztx1_kernel<4, false, WS>), grid, dim3(256), 0, s, a);
  } else if (kb == 2) {
    if (one) hipLaunchKernelGGL((ztx1_kernel<2, true, WS>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((ztx1_kernel<2, false, WS>), grid, dim3(256), 0, s, a);
  } else {
    if (one) hipLaunchKernelGGL((ztx1_kernel<1, true, WS>), grid, dim3(256), 0, s, a);
    else hipLaunchKernelGGL((ztx1_kernel<1, false, WS>), grid, dim3(256), 0, s, a);
  }
  return hipGetLastError();
}

template <class WS>
static hipError_t ztx_for(const Inst& in, WS w, const double* X, int64_t ldX, int64_t R, double* B, int64_t ldB,
                          hipStream_t s, const int* skip) {
  return run_ztx1(in, w, X, ldX, R, B, ldB, s, skip);
}

hipError_t launch_ztx(const Inst& in, const double* X, int64_t ldX, int64_t R, double* B, int64_t ldB,
                      hipStream_t s, const int* skip) {
  if (R <= 0) return hipSuccess;
  return in.W ? ztx_for(in, wdense(in), X, ldX, R, B, ldB, s, skip)
              : ztx_for(in, wsep(in), X, ldX, R, B, ldB, s, skip);
}

// ------------------------------------------------------------------- Z Y
template <int BM_, int BN_, int WM_, int WN_, class WS>
struct ZyProb {
  static constexpr int BM = BM_, BN = BN_, WM = WM_, WN = WN_, KC = 16;
  static constexpr int LDA = BM + 1, LDB = BN;
  static constexpr int NA = BM * KC / 256, NB_ = BN * KC / 256;
  static_assert(NA >= 1 && NB_ >= 1, "tile too small for 256 threads");
  const double* E; int64_t ldE;
  WS w;
  const double* Y; int64_t ldY;
  const double* Xs; int64_t ldXs;   // optional: out = alpha Xs + beta Z Y (else beta Z Y)
  double alpha, beta;
  double* Out; int64_t ldO;
  int64_t n_h, n, K, M, KM, R;
  int ntr, ntc;   // tiles along rows (r) and cols (i)
  const int* skip;

  struct Ctx { bool valid; int64_t r0, i0; int nchunks; };
  struct ARegs { double v[NA]; };
  struct BRegs { double v[NB_]; };

  __device__ Ctx ctx(int tile) const {
    Ctx c;
    const int tr = tile % ntr, tc = tile / ntr;
    c.valid = tc < ntc && !(skip && *skip);
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
        z = E[ii + k * ldE] * w(j, m);
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
      Out[ii + rr * ldO] = Xs ? fma(beta, v, alpha * Xs[ii + rr * ldXs]) : beta * v;
    });
  }
};

template <class P, class WS>
static hipError_t run_zy(const Inst& in, WS w, const double* Y, int64_t ldY, int64_t R, const double* Xs,
                         int64_t ldXs, double alpha, double beta, double* out, int64_t ldOut, hipStream_t s,
                         const int* skip) {
  P pr;
  pr.skip = skip;
  pr.alpha = alpha; pr.beta = beta;
  pr.E = in.E; pr.ldE = in.ldE; pr.w = w;
  pr.Y = Y; pr.ldY = ldY; pr.Xs = Xs; pr.ldXs = ldXs; pr.Out = out; pr.ldO = ldOut;
  pr.n_h = in.n_h; pr.n = in.n; pr.K = in.K; pr.M = in.M; pr.KM = in.KM; pr.R = R;
  pr.ntr = (int)ceil_div(R, P::BM);
  pr.ntc = (int)ceil_div(in.n, P::BN);
  const int64_t tiles = (int64_t)pr.ntr * pr.ntc;
  hipLaunchKernelGGL(gemm_f64_kernel<P>, dim3((unsigned)tiles), dim3(256), 0, s, pr);
  return hipGetLastError();
}

// Single level (n_w = 1): out[j, r] = (alpha Xs[j, r] +) beta sum_k E[j,k] sum_m W[j,m] Y[k*M+m, r].
// Tile: 64 right-hand sides x 256 grid columns, four waves of 64 x 64.  The
// contraction runs mode chunk by mode chunk (16 modes) on the outside and
// member by member inside: a chunk of W rows is staged once and serves all
// K members (each member's column of E scales it when the MFMA fragment is
// read), so W is read once per tile instead of once per member; per member
// only 16 rows of Y and 256 values of E are staged (double-buffered).
constexpr int YR = 64, YJ = 256, YKC = 16;
constexpr int YLD = YR + 16, WLD = YJ + 16;   // row strides: the four row groups of a fragment read on distinct banks

template <class WS>
struct Zy1Args {
  const double* E; int64_t ldE;
  WS w;
  const double* Y; int64_t ldY;
  const double* Xs; int64_t ldXs;
  double alpha, beta;
  double* Out; int64_t ldO;
  int64_t n_h, K, M, KM, R;
  int ntr, ntj;
  const int* skip;
};

template <class WS>
__global__ __launch_bounds__(256, 2) void zy1_kernel(Zy1Args<WS> a) {
  if (a.skip && *a.skip) return;
  __shared__ double Ws[YKC * WLD];         // Ws[m][j]: W rows of the current mode chunk
  __shared__ double Ys[2][YKC * YLD];      // Ys[m][r]: Y rows of one member in that chunk
  __shared__ double Es[2][YJ];             // the member's E values on the tile's grid columns
  const int64_t ntiles = (int64_t)a.ntr * a.ntj;
  const int64_t per = (ntiles + 7) / 8;
  const int64_t u = (blockIdx.x % 8) * per + blockIdx.x / 8;   // contiguous ranges per XCD
  if (u >= ntiles) return;
  const int tr = (int)(u % a.ntr), tj = (int)(u / a.ntr);
  const int64_t r0 = (int64_t)tr * YR, j0 = (int64_t)tj * YJ;
  const int t = threadIdx.x, lane = lane_id(), w = wave_id();
  const int rr = lane & 15, kq = lane >> 4;
  const int64_t mchunks = (a.M + YKC - 1) / YKC;
  const int64_t jt = j0 + t;                     // this thread's grid column for W and E staging
  const bool jin = jt < a.n_h;
  double yv[4], ev = 0.0;
  auto load_member = [&](int64_t mc, int64_t k) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = t + 256 * q, mm = e % YKC, col = e / YKC;
      const int64_t m = mc * YKC + mm, r = r0 + col;
      yv[q] = (m < a.M && r < a.R) ? a.Y[k * a.M + m + r * a.ldY] : 0.0;
    }
    ev = jin ? a.E[jt + k * a.ldE] : 0.0;
  };
  auto store_member = [&](int buf) {
#pragma unroll
    for (int q = 0; q < 4; ++q) {
      const int e = t + 256 * q;
      Ys[buf][(e % YKC) * YLD + e / YKC] = yv[q];
    }
    Es[buf][t] = ev;
  };
  d4 acc[4][4];
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  const int64_t steps = mchunks * a.K;           // (mode chunk, member) pairs, member fastest
  load_member(0, 0);
  for (int64_t st = 0; st < steps; ++st) {
    const int64_t mc = st / a.K, k = st - mc * a.K;
    const int buf = (int)(st & 1);
    if (k == 0) {
      // a new mode chunk: all its W loads in flight together (clamped,
      // valid indices; out-of-range values zeroed when stored), then every
      // wave is past the last fragment reads of Ws
      double wv[YKC];
#pragma unroll
      for (int mm = 0; mm < YKC; ++mm) {
        const int64_t m = mc * YKC + mm;
        wv[mm] = a.w(jin ? jt : 0, m < a.M ? m : a.M - 1);
      }
      __syncthreads();
#pragma unroll
      for (int mm = 0; mm < YKC; ++mm) Ws[mm * WLD + t] = (jin && mc * YKC + mm < a.M) ? wv[mm] : 0.0;
    }
    store_member(buf);
    __syncthreads();
    if (st + 1 < steps) {
      const int64_t st1 = st + 1, mc1 = st1 / a.K;
      load_member(mc1, st1 - mc1 * a.K);
    }
    const double* Yb = Ys[buf];
    const double* Eb = Es[buf];
#pragma unroll
    for (int kk = 0; kk < YKC; kk += 4) {
      const int mrow = kk + kq;
      double av[4], bv[4];
#pragma unroll
      for (int i = 0; i < 4; ++i) av[i] = Yb[mrow * YLD + i * 16 + rr];
#pragma unroll
      for (int j = 0; j < 4; ++j) {
        const int jc = w * 64 + j * 16 + rr;
        bv[j] = Ws[mrow * WLD + jc] * Eb[jc];    // z = E[j, k] W[j, m]
      }
#pragma unroll
      for (int i = 0; i < 4; ++i)
#pragma unroll
        for (int j = 0; j < 4; ++j) acc[i][j] = mfma_f64(av[i], bv[j], acc[i][j]);
    }
  }
#pragma unroll
  for (int i = 0; i < 4; ++i)
#pragma unroll
    for (int j = 0; j < 4; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int64_t r = r0 + i * 16 + kq + 4 * v;
        const int64_t jj = j0 + w * 64 + j * 16 + rr;
        if (r >= a.R || jj >= a.n_h) continue;
        const double val = acc[i][j][v];
        a.Out[jj + r * a.ldO] = a.Xs ? fma(a.beta, val, a.alpha * a.Xs[jj + r * a.ldXs]) : a.beta * val;
      }
}

template <class WS>
static hipError_t zy_for(const Inst& in, WS w, const double* Y, int64_t ldY, int64_t R, const double* Xs,
                         int64_t ldXs, double alpha, double beta, double* out, int64_t ldOut, hipStream_t s,
                         const int* skip) {
  if (in.n_w == 1) {
    Zy1Args<WS> a;
    a.skip = skip;
    a.alpha = alpha; a.beta = beta;
    a.E = in.E; a.ldE = in.ldE; a.w = w; a.Y = Y; a.ldY = ldY; a.Xs = Xs; a.ldXs = ldXs;
    a.Out = out; a.ldO = ldOut; a.n_h = in.n_h; a.K = in.K; a.M = in.M; a.KM = in.KM; a.R = R;
    a.ntr = (int)ceil_div(R, YR); a.ntj = (int)ceil_div(in.n_h, YJ);
    const int64_t ntiles = (int64_t)a.ntr * a.ntj;
    hipLaunchKernelGGL(zy1_kernel<WS>, dim3((unsigned)(8 * ((ntiles + 7) / 8))), dim3(256), 0, s, a);
    return hipGetLastError();
  }
  if (R <= 16) return run_zy<ZyProb<16, 128, 1, 4, WS>>(in, w, Y, ldY, R, Xs, ldXs, alpha, beta, out, ldOut, s, skip);
  if (R <= 32) return run_zy<ZyProb<32, 128, 1, 4, WS>>(in, w, Y, ldY, R, Xs, ldXs, alpha, beta, out, ldOut, s, skip);
  return run_zy<ZyProb<64, 64, 2, 2, WS>>(in, w, Y, ldY, R, Xs, ldXs, alpha, beta, out, ldOut, s, skip);
}

hipError_t launch_zy_axpby(const Inst& in, const double* Y, int64_t ldY, int64_t R, const double* Xs,
                           int64_t ldXs, double alpha, double beta, double* out, int64_t ldOut, hipStream_t s,
                           const int* skip) {
  if (R <= 0) return hipSuccess;
  return in.W ? zy_for(in, wdense(in), Y, ldY, R, Xs, ldXs, alpha, beta, out, ldOut, s, skip)
              : zy_for(in, wsep(in), Y, ldY, R, Xs, ldXs, alpha, beta, out, ldOut, s, skip);
}

hipError_t launch_zy(const Inst& in, const double* Y, int64_t ldY, int64_t R, const double* Xs, int64_t ldXs,
                     double* out, int64_t ldOut, hipStream_t s, const int* skip) {
  // x - Z y exactly as a subtraction (fma(-1, v, 1 * x) rounds once), else Z y
  return launch_zy_axpby(in, Y, ldY, R, Xs, ldXs, 1.0, Xs ? -1.0 : 1.0, out, ldOut, s, skip);
}

}  // namespace pc
