// FP64 Gram of the modulated square root, assembled without forming Z.
//
// Per grid column j the n_w x K block A_j (the rows of the members in column
// j, the paper's A_m of Sec. 3.9) gives S_j = A_j^T A_j.  Because the
// localization is horizontal (equal blocks C_b, Sec. 3.7) every level shares
// W, so
//     G_{(k,m),(k',m')} = sum_j S_j[k,k'] * W[j,m] * W[j,m'].
// G is symmetric in (k,k') and in (m,m') separately; only k <= k' and
// m <= m' are computed.  Written as a GEMM over j,
//     C[p, q] = sum_j S[j, p] * T[j, q],   p = (k <= k'),  q = (m <= m'),
//     T[j, q] = W[j, m] * W[j, m'],
// with the T operand formed on the fly from W while it is staged in LDS.
#include "gemm_core.h"
#include "pc_internal.h"

namespace pc {

// ---------------------------------------------------------------- pair table
__global__ void pairs_init_kernel(int K, int* pairs) {
  // packed order: p runs over k' (outer) and k <= k' (inner)
  int kp = blockIdx.x;
  for (int k = threadIdx.x; k <= kp; k += blockDim.x) {
    int p = kp * (kp + 1) / 2 + k;
    pairs[2 * p] = k;
    pairs[2 * p + 1] = kp;
  }
}

hipError_t launch_pairs_init(const Inst& in, hipStream_t s) {
  hipLaunchKernelGGL(pairs_init_kernel, dim3((unsigned)in.K), dim3(256), 0, s, (int)in.K, in.pairs);
  return hipGetLastError();
}

// ---------------------------------------------------- per-column Grams S_j
// Block: JB grid columns x 256 pairs.  E rows of one level are staged in LDS,
// each thread accumulates its pair over the block's columns and all levels.
constexpr int CG_JB = 32;

__global__ __launch_bounds__(256) void column_grams_kernel(const double* __restrict__ E, int64_t ldE,
                                                           int64_t n_h, int64_t n_w, int K, int64_t P,
                                                           const int* __restrict__ pairs, int jb,
                                                           double* __restrict__ S) {
  extern __shared__ double Es[];  // jb x K, Es[k * jb + jj]
  const int64_t j0 = (int64_t)blockIdx.x * jb;
  const int64_t p = (int64_t)blockIdx.y * 256 + threadIdx.x;
  int k = 0, kp = 0;
  if (p < P) { k = pairs[2 * p]; kp = pairs[2 * p + 1]; }
  double acc[CG_JB];
#pragma unroll
  for (int jj = 0; jj < CG_JB; ++jj) acc[jj] = 0.0;
  for (int64_t l = 0; l < n_w; ++l) {
    __syncthreads();
    for (int idx = threadIdx.x; idx < jb * K; idx += 256) {
      int jj = idx % jb, kk = idx / jb;
      int64_t j = j0 + jj;
      Es[idx] = (j < n_h) ? E[l * n_h + j + (int64_t)kk * ldE] : 0.0;
    }
    __syncthreads();
    if (p < P) {
#pragma unroll
      for (int jj = 0; jj < CG_JB; ++jj)
        if (jj < jb) acc[jj] += Es[k * jb + jj] * Es[kp * jb + jj];
    }
  }
  if (p < P) {
#pragma unroll
    for (int jj = 0; jj < CG_JB; ++jj)
      if (jj < jb && j0 + jj < n_h) S[(j0 + jj) * P + p] = acc[jj];
  }
}

hipError_t launch_column_grams(const Inst& in, hipStream_t s) {
  int jb = CG_JB;
  while (jb > 1 && (int64_t)jb * in.K * 8 > 48 * 1024) jb /= 2;
  dim3 grid((unsigned)ceil_div(in.n_h, jb), (unsigned)ceil_div(in.P, 256));
  size_t shm = (size_t)jb * in.K * sizeof(double);
  hipLaunchKernelGGL(column_grams_kernel, grid, dim3(256), shm, s, in.E, in.ldE, in.n_h, in.n_w,
                     (int)in.K, in.P, in.pairs, jb, in.S);
  return hipGetLastError();
}

// -------------------------------------------------------------- FP64 Gram
// Tile: 128 pairs p x 128 mode pairs q (8 values of m x 16 values of m').
struct GramF64Prob {
  static constexpr int BM = 128, BN = 128, WM = 2, WN = 2, KC = 16;
  static constexpr int LDA = BM, LDB = BN;
  const double* S; const double* W; int64_t ldW;
  int64_t n_h, M, P;
  const int* pairs; const int* qtiles;
  int npt, nq;
  double* G; int64_t ldG;

  struct Ctx { bool valid; int64_t p0; int m0, mp0; int nchunks; };
  struct ARegs { double v[8]; };
  struct BRegs { double v[8]; };

  __device__ Ctx ctx(int tile) const {
    Ctx c;
    int pt = tile / nq, qi = tile % nq;
    c.valid = pt < npt;
    c.p0 = (int64_t)pt * BM;
    c.m0 = qtiles[2 * qi];
    c.mp0 = qtiles[2 * qi + 1];
    c.nchunks = (int)ceil_div_dev(n_h, KC);
    return c;
  }
  __device__ static int64_t ceil_div_dev(int64_t a, int64_t b) { return (a + b - 1) / b; }

  __device__ void loadA(const Ctx& c, int chunk, ARegs& r) const {
    const int t = threadIdx.x, pl = t & 127;
    const int64_t p = c.p0 + pl;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int64_t j = (int64_t)chunk * KC + (t >> 7) + 2 * i;
      r.v[i] = (j < n_h && p < P) ? S[j * P + p] : 0.0;
    }
  }
  __device__ void storeA(const ARegs& r, double* As) const {
    const int t = threadIdx.x;
#pragma unroll
    for (int i = 0; i < 8; ++i) As[((t >> 7) + 2 * i) * LDA + (t & 127)] = r.v[i];
  }
  __device__ void loadB(const Ctx& c, int chunk, BRegs& r) const {
    const int t = threadIdx.x, ql = t & 127;
    const int64_t m = c.m0 + (ql >> 4), mp = c.mp0 + (ql & 15);
    const bool ok = m < M && mp < M;
#pragma unroll
    for (int i = 0; i < 8; ++i) {
      const int64_t j = (int64_t)chunk * KC + (t >> 7) + 2 * i;
      r.v[i] = (ok && j < n_h) ? W[j + m * ldW] * W[j + mp * ldW] : 0.0;
    }
  }
  __device__ void storeB(const BRegs& r, double* Bs) const {
    const int t = threadIdx.x;
#pragma unroll
    for (int i = 0; i < 8; ++i) Bs[((t >> 7) + 2 * i) * LDB + (t & 127)] = r.v[i];
  }
  __device__ void epilogue(const Ctx& c, const TileF64<BM, BN, WM, WN>& acc) const {
    acc.for_each([&](int row, int col, double v) {
      const int64_t p = c.p0 + row;
      if (p >= P) return;
      const int64_t m = c.m0 + (col >> 4), mp = c.mp0 + (col & 15);
      if (mp >= M || m > mp) return;
      const int64_t k = pairs[2 * p], kp = pairs[2 * p + 1];
      G[(kp * M + mp) + (k * M + m) * ldG] = v;
      if (k != kp && m != mp) G[(kp * M + m) + (k * M + mp) * ldG] = v;
    });
  }
};

hipError_t launch_gram_f64(const Inst& in, hipStream_t s) {
  GramF64Prob pr;
  pr.S = in.S; pr.W = in.W; pr.ldW = in.ldW;
  pr.n_h = in.n_h; pr.M = in.M; pr.P = in.P;
  pr.pairs = in.pairs; pr.qtiles = in.qtiles;
  pr.npt = (int)ceil_div(in.P, GramF64Prob::BM); pr.nq = in.nq;
  pr.G = in.G; pr.ldG = in.KMp;
  const int64_t tiles = (int64_t)pr.npt * pr.nq;
  hipLaunchKernelGGL(gemm_f64_kernel<GramF64Prob>, dim3((unsigned)tiles), dim3(256), 0, s, pr);
  return hipGetLastError();
}

// ------------------------------------ padding of the Gram and its diagonal
// Rows/cols KM..KMp-1 become the identity so the blocked factorization can
// run on whole NB blocks; diag0 keeps the pre-factorization diagonal.
__global__ void gram_pad_diag_kernel(double* G, int64_t ld, int64_t KM, int64_t KMp, double* diag0) {
  int64_t c = blockIdx.x;  // column
  if (c >= KM) {
    for (int64_t r = threadIdx.x; r < KMp; r += blockDim.x) G[r + c * ld] = (r == c) ? 1.0 : 0.0;
  } else {
    for (int64_t r = KM + threadIdx.x; r < KMp; r += blockDim.x) G[r + c * ld] = 0.0;
  }
  if (threadIdx.x == 0) diag0[c] = (c >= KM) ? 1.0 : G[c + c * ld];
}

hipError_t launch_gram_pad_and_diag(const Inst& in, hipStream_t s) {
  hipLaunchKernelGGL(gram_pad_diag_kernel, dim3((unsigned)in.KMp), dim3(64), 0, s, in.G, in.KMp,
                     in.KM, in.KMp, in.diag0);
  return hipGetLastError();
}

}  // namespace pc
