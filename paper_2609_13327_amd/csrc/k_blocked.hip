// FP64 MFMA products of column-major panels for the blocked outer
// factorization of large Grams and the blocked triangular solves:
//   C(i, j) = alpha sum_k A(i, k) B(j, k)            (overwrite), or
//   C(i, j) = C(i, j) + alpha sum_k A(i, k) B(j, k)  (accumulate),
// optionally on the lower triangle only (tiles with i >= j; inside a
// diagonal tile only i >= j is written).  Each operand is read either along
// its columns (A(i, k) at A[i + k lda]) or, with TA / TB, along k
// (A(i, k) at A[k + i lda]); both reads are coalesced.  Waves own 64 x 64
// sub-tiles; the contraction is staged through LDS 16 k at a time (k-major
// operands row-XOR swizzled, so that their transposing stores spread over
// the banks).  Large products use 256 x 128 workgroup tiles (8 waves, two
// per SIMD): a third less operand traffic per flop than 128 x 128 (four
// waves, two workgroups per compute unit).
#include "pc_common.h"
#include "pc_internal.h"
#include "gemm_core.h"

#include <algorithm>

namespace pc {

template <int BM_, int BN_, int WM_, int WN_, bool TA = false, bool TB = false>
struct NtGemmProb {
  static constexpr int BM = BM_, BN = BN_, WM = WM_, WN = WN_, KC = 16;
  static constexpr int NT = 64 * WM * WN;          // threads
  // two waves per SIMD: two 4-wave workgroups (or one of 8 waves) per compute unit
  static constexpr int OCC = 2;
  static constexpr bool XA = TA, XB = TB;
  static constexpr int LDA = TA ? BM : BM + 8, LDB = TB ? BN : BN + 8;
  static constexpr int NA = BM * KC / NT, NB_ = BN * KC / NT;
  static constexpr int RT = BM / BN;              // column tiles per row tile (lower-triangle mode)
  static constexpr int LG = 8;                    // tile rows per group (lower-triangle mode, RT = 1)
  static_assert(NA >= 2 && NB_ >= 2 && BM * KC % (2 * NT) == 0 && BN * KC % (2 * NT) == 0, "tile / thread mismatch");
  static_assert(BM % BN == 0, "row tiles must cover whole column tiles");
  const double* A; int64_t lda;
  const double* B; int64_t ldb;
  double* C; int64_t ldc;
  int64_t M, N, K;
  double alpha;
  int accumulate, lower;
  int64_t tm, tn, ntiles;
  const int* skip;                                 // nonzero *skip: the product is not applied
  int tri_b;                                       // B(j, k) = 0 for k > j: column tile j0.. contracts k < j0 + BN only

  struct Ctx { bool valid; int64_t i0, j0; int nchunks; };

  __device__ Ctx ctx(int b) const {
    Ctx c;
    const int64_t per = (ntiles + 7) / 8;
    const int64_t u = (b % 8) * per + b / 8;      // consecutive tiles on one XCD
    c.valid = u < ntiles && !(skip && *skip);
    c.i0 = c.j0 = 0;
    c.nchunks = 0;
    if (!c.valid) return c;                       // (the orders below assume u < ntiles)
    int64_t ti, tj;
    if (lower && RT == 1) {
      // groups of LG tile rows; inside a group column by column, so that the
      // tiles an XCD runs at once share a few row strips of both operands
      // (the group before row r0 = g LG holds r0 (r0 + 1) / 2 tiles)
      int64_t g = (int64_t)((sqrt(8.0 * (double)u + 1.0) - 1.0) * 0.5) / LG;
      while ((g + 1) * LG <= tm && ((g + 1) * LG) * ((g + 1) * LG + 1) / 2 <= u) ++g;
      while (g > 0 && (g * LG) * (g * LG + 1) / 2 > u) --g;
      const int64_t r0 = g * LG, rows = (r0 + LG <= tm ? LG : tm - r0);
      int64_t v = u - r0 * (r0 + 1) / 2;
      if (v < r0 * rows) {                        // columns left of the group's diagonal block
        tj = v / rows;
        ti = r0 + v % rows;
      } else {                                    // the diagonal block: column r0 + d has rows - d tiles
        v -= r0 * rows;
        int64_t d = 0;
        while (d + 1 < rows && v >= rows - d) { v -= rows - d; ++d; }
        tj = r0 + d;
        ti = tj + v;
      }
    } else if (lower) {
      // tile row ti holds the RT (ti + 1) column tiles that reach the lower
      // triangle (RT = BM / BN); rows before it hold RT ti (ti + 1) / 2
      ti = (int64_t)((sqrt(8.0 * (double)u / RT + 1.0) - 1.0) * 0.5);
      while (RT * (ti + 1) * (ti + 2) / 2 <= u) ++ti;
      while (RT * ti * (ti + 1) / 2 > u) --ti;
      tj = u - RT * ti * (ti + 1) / 2;
    } else {
      // column tiles fastest: the tiles of a row strip of A run together
      ti = u / tn;
      tj = u % tn;
    }
    c.i0 = ti * BM;
    c.j0 = tj * BN;
    const int64_t kend = tri_b && c.j0 + BN < K ? c.j0 + BN : K;
    c.nchunks = (int)((kend + KC - 1) / KC);
    return c;
  }
  // Thread t's share of a chunk, in pairs of elements adjacent in memory
  // (one 16-byte load each): a column-major operand pairs rows (pair index
  // fixed per thread, k steps NT / (BR/2) per q), a k-major one pairs k
  // (k pair fixed, row steps NT / (KC/2) per q).  K is a multiple of KC and
  // the host checks the alignment (even leading dimensions and column-major
  // row counts, 16-byte aligned bases), so every k is inside; row pairs past
  // the edge read the last pair (their products only reach outputs that are
  // not written).  The loads are unconditional and nothing is selected on
  // their values, so the chunk's products never wait for them.
  struct ARegs { double x[NA / 2], y[NA / 2]; };
  struct BRegs { double x[NB_ / 2], y[NB_ / 2]; };
  template <bool T, int BR, int NP>
  __device__ static void load_slab(const double* X, int64_t ldx, int64_t r0, int64_t rows, int64_t k0, double* vx,
                                   double* vy) {
    const int t = threadIdx.x;
    if (!T) {
      constexpr int STEP = NT / (BR / 2);              // k per q
      const int pr = t % (BR / 2), kk = t / (BR / 2);
      const int64_t r = r0 + 2 * pr <= rows - 2 ? r0 + 2 * pr : rows - 2;
      const double* p = X + r + (k0 + kk) * ldx;
      const int64_t qs = (int64_t)STEP * ldx;
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        const double2 u = *reinterpret_cast<const double2*>(p + q * qs);
        vx[q] = u.x;
        vy[q] = u.y;
      }
    } else {
      constexpr int STEP = NT / (KC / 2);              // rows per q
      const int kp = t % (KC / 2), row = t / (KC / 2);
      const double* p = X + k0 + 2 * kp;
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        const int64_t r = r0 + row + STEP * q;
        const double2 u = *reinterpret_cast<const double2*>(p + (r < rows ? r : rows - 1) * ldx);
        vx[q] = u.x;
        vy[q] = u.y;
      }
    }
  }
  template <bool T, int BR, int NP, int LD>
  __device__ static void store_slab(const double* vx, const double* vy, double* S) {
    const int t = threadIdx.x;
    if (!T) {
      constexpr int STEP = NT / (BR / 2);
      const int pr = t % (BR / 2), kk = t / (BR / 2);
#pragma unroll
      for (int q = 0; q < NP; ++q) *reinterpret_cast<double2*>(S + (kk + STEP * q) * LD + 2 * pr) = double2{vx[q], vy[q]};
    } else {
      constexpr int STEP = NT / (KC / 2);
      const int kp = t % (KC / 2), row = t / (KC / 2), k = 2 * kp;
#pragma unroll
      for (int q = 0; q < NP; ++q) {
        S[k * LD + ((row + STEP * q) ^ k)] = vx[q];
        S[(k + 1) * LD + ((row + STEP * q) ^ (k + 1))] = vy[q];
      }
    }
  }
  __device__ void loadA(const Ctx& c, int chunk, ARegs& r) const {
    load_slab<TA, BM, NA / 2>(A, lda, c.i0, M, (int64_t)chunk * KC, r.x, r.y);
  }
  __device__ void storeA(const ARegs& r, double* As) const { store_slab<TA, BM, NA / 2, LDA>(r.x, r.y, As); }
  __device__ void loadB(const Ctx& c, int chunk, BRegs& r) const {
    load_slab<TB, BN, NB_ / 2>(B, ldb, c.j0, N, (int64_t)chunk * KC, r.x, r.y);
  }
  __device__ void storeB(const BRegs& r, double* Bs) const { store_slab<TB, BN, NB_ / 2, LDB>(r.x, r.y, Bs); }
  // A tile inside C (and strictly below the diagonal in lower mode) reads
  // the 16 C values of a fragment row with unconditional loads before it
  // writes any of them: an edge test per element would make every load wait
  // for the previous one.  Edge tiles test each element.
  __device__ void epilogue(const Ctx& c, const TileF64<BM, BN, WM, WN>& acc) const {
    using Tile = TileF64<BM, BN, WM, WN>;
    const bool inside = c.i0 + BM <= M && c.j0 + BN <= N && (!lower || c.i0 >= c.j0 + BN);
    if (inside) {
      const int lane = lane_id(), w = wave_id();
      const int wm = w / WN, wn = w % WN;
      double* Cw = C + (c.i0 + wm * Tile::TM + (lane >> 4)) + (c.j0 + wn * Tile::TN + (lane & 15)) * ldc;
#pragma unroll
      for (int i = 0; i < Tile::FM; ++i) {
        double old[Tile::FN][4];
        if (accumulate) {
#pragma unroll
          for (int j = 0; j < Tile::FN; ++j)
#pragma unroll
            for (int v = 0; v < 4; ++v) old[j][v] = Cw[(i * 16 + 4 * v) + (int64_t)(j * 16) * ldc];
        }
#pragma unroll
        for (int j = 0; j < Tile::FN; ++j)
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const double x = alpha * acc.acc[i][j][v];
            Cw[(i * 16 + 4 * v) + (int64_t)(j * 16) * ldc] = accumulate ? old[j][v] + x : x;
          }
      }
      return;
    }
    acc.for_each([&](int row, int col, double v) {
      const int64_t i = c.i0 + row, j = c.j0 + col;
      if (i >= M || j >= N || (lower && i < j)) return;
      double* p = C + i + j * ldc;
      *p = accumulate ? *p + alpha * v : alpha * v;
    });
  }
};

using NtGemm128 = NtGemmProb<128, 128, 2, 2>;
using NtGemm256 = NtGemmProb<256, 128, 4, 2>;

// The loaders read pairs of adjacent elements with 16-byte loads: even
// leading dimensions, 16-byte aligned bases, and an even row count for an
// operand read along its columns.
static bool pair_loads_ok(const double* X, int64_t ldx, int64_t rows, bool kmajor) {
  return ((uintptr_t)X % 16 == 0) && ldx % 2 == 0 && (kmajor || (rows % 2 == 0 && rows >= 2));
}

template <class P>
static hipError_t run_nt_gemm(const double* A, int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc,
                              int64_t M, int64_t N, int64_t K, double alpha, int accumulate, int lower,
                              hipStream_t s, const int* skip = nullptr, int tri_b = 0) {
  if (!pair_loads_ok(A, lda, M, P::XA) || !pair_loads_ok(B, ldb, N, P::XB)) return hipErrorInvalidValue;
  P g;
  g.A = A; g.lda = lda; g.B = B; g.ldb = ldb; g.C = C; g.ldc = ldc;
  g.M = M; g.N = N; g.K = K; g.alpha = alpha; g.accumulate = accumulate; g.lower = lower; g.skip = skip;
  g.tri_b = tri_b;
  g.tm = ceil_div(M, P::BM);
  g.tn = ceil_div(N, P::BN);
  g.ntiles = lower ? P::RT * g.tm * (g.tm + 1) / 2 : g.tm * g.tn;
  const int64_t grid = 8 * ((g.ntiles + 7) / 8);
  hipLaunchKernelGGL(gemm_f64_kernel<P>, dim3((unsigned)grid), dim3(P::NT), 0, s, g);
  return hipGetLastError();
}

hipError_t launch_nt_gemm(const double* A, int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc,
                          int64_t M, int64_t N, int64_t K, double alpha, int accumulate, int lower, hipStream_t s,
                          int tile, int tri_b) {
  if (M <= 0 || N <= 0) return hipSuccess;
  if (K % 16 != 0) return hipErrorInvalidValue;      // whole chunks of k (the loaders read no edge)
  // tile 1: 128 x 128, tile 2: 256 x 128; 0: 256 x 128 once there are enough
  // of them to fill the device twice
  const int64_t t256 = lower ? ceil_div(M, 256) * (ceil_div(M, 256) + 1) : ceil_div(M, 256) * ceil_div(N, 128);
  if (tile == 2 || (tile == 0 && t256 >= 512))
    return run_nt_gemm<NtGemm256>(A, lda, B, ldb, C, ldc, M, N, K, alpha, accumulate, lower, s, nullptr, tri_b);
  return run_nt_gemm<NtGemm128>(A, lda, B, ldb, C, ldc, M, N, K, alpha, accumulate, lower, s, nullptr, tri_b);
}

// Products of the blocked solves (rectangular, accumulate into C):
//   tb:      C(i, j) += alpha sum_k A(i, k) B(k, j)      A column-major, B read along k
//   ta, tb:  C(i, j) += alpha sum_k A(k, i) B(k, j)      both read along k
using GemmNK = NtGemmProb<128, 128, 2, 2, false, true>;
using GemmKK = NtGemmProb<128, 128, 2, 2, true, true>;

hipError_t launch_solve_gemm(bool ta, const double* A, int64_t lda, const double* B, int64_t ldb, double* C,
                             int64_t ldc, int64_t M, int64_t N, int64_t K, double alpha, const int* skip,
                             hipStream_t s) {
  if (M <= 0 || N <= 0 || K <= 0) return hipSuccess;
  if (K % 16 != 0) return hipErrorInvalidValue;      // whole chunks of k (the loaders read no edge)
  return ta ? run_nt_gemm<GemmKK>(A, lda, B, ldb, C, ldc, M, N, K, alpha, 1, 0, s, skip)
            : run_nt_gemm<GemmNK>(A, lda, B, ldb, C, ldc, M, N, K, alpha, 1, 0, s, skip);
}

// dst (rows x cols, ld ldd) = src (ld lds)
__global__ void copy_panel_kernel(const double* __restrict__ src, int64_t lds, double* __restrict__ dst, int64_t ldd,
                                  int64_t rows) {
  const int64_t c = blockIdx.y;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < rows; r += (int64_t)gridDim.x * blockDim.x)
    dst[r + c * ldd] = src[r + c * lds];
}

hipError_t launch_copy_panel(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t rows, int64_t cols,
                             hipStream_t s) {
  if (rows <= 0 || cols <= 0) return hipSuccess;
  const unsigned gx = (unsigned)std::min<int64_t>(ceil_div(rows, 256), 128);
  hipLaunchKernelGGL(copy_panel_kernel, dim3(gx, (unsigned)cols), dim3(256), 0, s, src, lds, dst, ldd, rows);
  return hipGetLastError();
}

// n x n identity (ld n)
__global__ void identity_kernel(double* __restrict__ I, int64_t n) {
  const int64_t c = blockIdx.y;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < n; r += (int64_t)gridDim.x * blockDim.x)
    I[r + c * n] = (r == c) ? 1.0 : 0.0;
}

hipError_t launch_identity(double* I, int64_t n, hipStream_t s) {
  const unsigned gx = (unsigned)std::min<int64_t>(ceil_div(n, 256), 16);
  hipLaunchKernelGGL(identity_kernel, dim3(gx, (unsigned)n), dim3(256), 0, s, I, n);
  return hipGetLastError();
}

}  // namespace pc
