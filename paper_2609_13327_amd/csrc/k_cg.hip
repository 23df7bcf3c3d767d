// Block-Jacobi preconditioned conjugate gradients on the normal equations
// G y = b (G = Z^T Z), batched over right-hand sides with per-column scalars.
//
// G is kept as a full symmetric copy Gs (KMp x KMp, the padding is the
// identity, so padded rows stay zero).  The preconditioner inverts the 64 x 64
// diagonal blocks of Gs.  One iteration:
//   Q = Gs P                     (FP64 MFMA GEMM)
//   alpha = rz / p^T q; y += alpha p; r -= alpha q; converged if ||r|| <= tol ||b||
//   z = blockdiag(Gs)^{-1} r
//   beta = r^T z / rz; p = z + beta p
// Column kernels use one workgroup per right-hand side and skip converged
// columns, so a fixed-length loop can run past convergence harmlessly.
#include "pc_common.h"
#include "pc_internal.h"
#include "gemm_core.h"

#include <algorithm>

namespace pc {

// ---------------------------------------------------------------- symmetric copy
// Gs(i, j) = G(max(i, j), min(i, j)) from the lower triangle, by 64 x 64 tiles
// through LDS so both the tile and its transpose are written coalesced.
__global__ __launch_bounds__(256) void gram_symmetrize_kernel(const double* __restrict__ G, int64_t ld,
                                                              int64_t T, double* __restrict__ Gs) {
  __shared__ double tile[64][65];
  int64_t u = blockIdx.x;
  int64_t ti = (int64_t)((sqrt(8.0 * (double)u + 1.0) - 1.0) * 0.5);
  while ((ti + 1) * (ti + 2) / 2 <= u) ++ti;
  while (ti * (ti + 1) / 2 > u) --ti;
  const int64_t tj = u - ti * (ti + 1) / 2;   // ti >= tj
  const int64_t r0 = ti * 64, c0 = tj * 64;
  const int tx = threadIdx.x & 63, ty = threadIdx.x >> 6;
  for (int c = ty; c < 64; c += 4) tile[tx][c] = G[(r0 + tx) + (c0 + c) * ld];
  __syncthreads();
  if (ti == tj) {
    for (int c = ty; c < 64; c += 4) {
      const int a = tx > c ? tx : c, b = tx > c ? c : tx;
      Gs[(r0 + tx) + (c0 + c) * ld] = tile[a][b];
    }
  } else {
    for (int c = ty; c < 64; c += 4) {
      Gs[(r0 + tx) + (c0 + c) * ld] = tile[tx][c];   // lower tile
      Gs[(c0 + tx) + (r0 + c) * ld] = tile[c][tx];   // its transpose in the upper triangle
    }
  }
  (void)T;
}

// The kept FP64 Gram of a plan whose factored Gram is a reduced-precision
// one: the structured FP64 Gram is assembled into Gs (its lower triangle,
// by the FP64 Gram kernels), the padding becomes identity columns and zero
// rows, and the lower triangle is mirrored in place.
__global__ void gram_pad_only_kernel(double* G, int64_t ld, int64_t KM, int64_t KMp) {
  const int64_t c = blockIdx.x;
  const int64_t r0 = c >= KM ? 0 : KM;
  for (int64_t r = r0 + threadIdx.x; r < KMp; r += blockDim.x) G[r + c * ld] = (r == c) ? 1.0 : 0.0;
}

hipError_t launch_kept_fp64_gram(const Inst& in, hipStream_t s) {
  Inst f = in;
  f.G = in.Gs;
  f.G2 = nullptr;
  f.g2_parts = 0;
  hipError_t e = launch_column_grams(f, s);
  if (e == hipSuccess) e = launch_gram_f64(f, s);
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(gram_pad_only_kernel, dim3((unsigned)in.KMp), dim3(256), 0, s, in.Gs, in.KMp, in.KM, in.KMp);
  e = hipGetLastError();
  return e != hipSuccess ? e : launch_gram_symmetrize(f, in.Gs, s);   // in place: reads lower tiles only
}

hipError_t launch_gram_symmetrize(const Inst& in, double* Gs, hipStream_t s) {
  const int64_t T = in.KMp / NB;
  hipLaunchKernelGGL(gram_symmetrize_kernel, dim3((unsigned)(T * (T + 1) / 2)), dim3(256), 0, s, in.G, in.KMp, T, Gs);
  return hipGetLastError();
}

// ---------------------------------------------------------------- block-Jacobi
// One workgroup per diagonal block: Cholesky in LDS, inverse of the factor by
// forward substitution (one thread per column), then Dinv = L^{-T} L^{-1}.
__global__ __launch_bounds__(256) void bj_setup_kernel(const double* __restrict__ Gs, int64_t ld,
                                                       double* __restrict__ Dinv, int* __restrict__ flag) {
  __shared__ double a[64][65];
  __shared__ double li[64][65];
  __shared__ int bad;
  const int64_t t = blockIdx.x, o = t * 64;
  const int tid = threadIdx.x;
  for (int e = tid; e < 4096; e += 256) {
    const int i = e & 63, j = e >> 6;
    a[i][j] = Gs[(o + i) + (o + j) * ld];
  }
  if (tid == 0) bad = 0;
  __syncthreads();
  for (int j = 0; j < 64; ++j) {
    const double piv = a[j][j];
    if (!(piv > 0.0)) {   // uniform: every thread reads the same value
      if (tid == 0) bad = 1;
      break;
    }
    const double dj = sqrt(piv);
    __syncthreads();
    if (tid < 64 && tid > j) a[tid][j] /= dj;
    if (tid == 0) a[j][j] = dj;
    __syncthreads();
    for (int e = tid; e < 4096; e += 256) {
      const int i = e & 63, k = e >> 6;
      if (k > j && i >= k) a[i][k] -= a[i][j] * a[k][j];
    }
    __syncthreads();
  }
  __syncthreads();
  if (bad) {
    if (tid == 0) atomicOr(flag, 1);
    return;
  }
  if (tid < 64) {
    const int c = tid;
    for (int i = 0; i < 64; ++i) {
      if (i < c) { li[i][c] = 0.0; continue; }
      double s = (i == c) ? 1.0 : 0.0;
      for (int k = c; k < i; ++k) s -= a[i][k] * li[k][c];
      li[i][c] = s / a[i][i];
    }
  }
  __syncthreads();
  for (int e = tid; e < 4096; e += 256) {
    const int i = e & 63, j = e >> 6;
    const int k0 = i > j ? i : j;
    double s = 0.0;
    for (int k = k0; k < 64; ++k) s += li[k][i] * li[k][j];
    Dinv[t * 4096 + i + j * 64] = s;
  }
}

hipError_t launch_bj_setup(const double* Gs, int64_t ld, int64_t T, double* Dinv, int* flag, hipStream_t s) {
  hipLaunchKernelGGL(bj_setup_kernel, dim3((unsigned)T), dim3(256), 0, s, Gs, ld, Dinv, flag);
  return hipGetLastError();
}

// Z[block t, cols] = Dinv_t R[block t, cols], 64 columns per workgroup.
__global__ __launch_bounds__(256) void bj_apply_kernel(const double* __restrict__ Dinv, const double* __restrict__ Rm,
                                                       double* __restrict__ Zm, int64_t ld, int64_t R) {
  __shared__ double d[64][65];
  __shared__ double rb[64][65];
  const int64_t t = blockIdx.x, c0 = (int64_t)blockIdx.y * 64, o = t * 64;
  const int tid = threadIdx.x;
  for (int e = tid; e < 4096; e += 256) {
    const int i = e & 63, j = e >> 6;
    d[i][j] = Dinv[t * 4096 + i + j * 64];
    rb[i][j] = (c0 + j < R) ? Rm[(o + i) + (c0 + j) * ld] : 0.0;
  }
  __syncthreads();
  const int i = tid & 63, cq = tid >> 6;
  for (int c = cq; c < 64; c += 4) {
    if (c0 + c >= R) break;
    double s = 0.0;
#pragma unroll 8
    for (int j = 0; j < 64; ++j) s += d[i][j] * rb[j][c];
    Zm[(o + i) + (c0 + c) * ld] = s;
  }
}

hipError_t launch_bj_apply(const double* Dinv, int64_t T, const double* Rm, double* Zm, int64_t ld, int64_t R,
                           hipStream_t s) {
  if (R <= 0) return hipSuccess;
  hipLaunchKernelGGL(bj_apply_kernel, dim3((unsigned)T, (unsigned)ceil_div(R, 64)), dim3(256), 0, s, Dinv, Rm, Zm,
                     ld, R);
  return hipGetLastError();
}

// ---------------------------------------------------------------- Q = Gs P
struct GramMatmul {
  static constexpr int BM = 64, BN = 64, WM = 2, WN = 2, KC = 16;
  static constexpr int LDA = BM + 16, LDB = BN + 1;
  static constexpr int NA = BM * KC / 256, NB_ = BN * KC / 256;
  const double* Gs; const double* P; double* Q;
  int64_t ld, KMp, R;
  int ntr, ntc;
  struct Ctx { bool valid; int64_t i0, c0; int nchunks; };
  struct ARegs { double v[NA]; };
  struct BRegs { double v[NB_]; };
  __device__ Ctx ctx(int tile) const {
    Ctx c;
    const int tr = tile % ntr, tc = tile / ntr;
    c.valid = tc < ntc;
    c.i0 = (int64_t)tr * BM;
    c.c0 = (int64_t)tc * BN;
    c.nchunks = (int)(KMp / KC);
    return c;
  }
  __device__ void loadA(const Ctx& c, int chunk, ARegs& r) const {   // As[k][row] = Gs(i0 + row, k)
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = threadIdx.x + 256 * q, row = e % BM, kk = e / BM;
      r.v[q] = Gs[(c.i0 + row) + ((int64_t)chunk * KC + kk) * ld];
    }
  }
  __device__ void storeA(const ARegs& r, double* As) const {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = threadIdx.x + 256 * q;
      As[(e / BM) * LDA + e % BM] = r.v[q];
    }
  }
  __device__ void loadB(const Ctx& c, int chunk, BRegs& r) const {   // Bs[k][col] = P(k, c0 + col)
#pragma unroll
    for (int q = 0; q < NB_; ++q) {
      const int e = threadIdx.x + 256 * q, kk = e % KC, col = e / KC;
      const int64_t cc = c.c0 + col;
      r.v[q] = cc < R ? P[((int64_t)chunk * KC + kk) + cc * ld] : 0.0;
    }
  }
  __device__ void storeB(const BRegs& r, double* Bs) const {
#pragma unroll
    for (int q = 0; q < NB_; ++q) {
      const int e = threadIdx.x + 256 * q;
      Bs[(e % KC) * LDB + e / KC] = r.v[q];
    }
  }
  __device__ void epilogue(const Ctx& c, const TileF64<BM, BN, WM, WN>& acc) const {
    acc.for_each([&](int row, int col, double v) {
      const int64_t cc = c.c0 + col;
      if (cc < R) Q[(c.i0 + row) + cc * ld] = v;
    });
  }
};

hipError_t launch_gram_matmul(const double* Gs, int64_t KMp, const double* P, double* Q, int64_t ld, int64_t R,
                              hipStream_t s) {
  if (R <= 0) return hipSuccess;
  GramMatmul g;
  g.Gs = Gs; g.P = P; g.Q = Q; g.ld = ld; g.KMp = KMp; g.R = R;
  g.ntr = (int)(KMp / GramMatmul::BM);
  g.ntc = (int)ceil_div(R, GramMatmul::BN);
  hipLaunchKernelGGL(gemm_f64_kernel<GramMatmul>, dim3((unsigned)(g.ntr * g.ntc)), dim3(256), 0, s, g);
  return hipGetLastError();
}

// ---------------------------------------------------------------- column kernels
__device__ __forceinline__ double block_sum(double v, double* red) {
  v = wave_sum(v);
  __syncthreads();
  if (lane_id() == 0) red[wave_id()] = v;
  __syncthreads();
  return red[0] + red[1] + red[2] + red[3];
}

// r = b - Q (Q = Gs y0, or zero for a cold start); b rows >= KM read as zero.
// A column with b = 0 is done with y = 0.
__global__ __launch_bounds__(256) void cg_start_kernel(const double* __restrict__ Bm, int64_t ldB,
                                                       const double* __restrict__ Q, double* __restrict__ Rm,
                                                       double* __restrict__ Y, int64_t ldY, int64_t ld, int64_t KM,
                                                       int64_t KMp, double tol, CgCol* __restrict__ col,
                                                       int* __restrict__ ndone) {
  __shared__ double red[4];
  const int64_t c = blockIdx.x;
  double bb = 0.0, rr = 0.0;
  for (int64_t i = threadIdx.x; i < KMp; i += 256) {
    const double b = i < KM ? Bm[i + c * ldB] : 0.0;
    const double r = b - (Q ? Q[i + c * ld] : 0.0);
    Rm[i + c * ld] = r;
    bb += b * b;
    rr += r * r;
  }
  bb = block_sum(bb, red);
  rr = block_sum(rr, red);
  const double bn = sqrt(bb);
  const bool zero = !(bn > 0.0);
  if (zero)
    for (int64_t i = threadIdx.x; i < KMp; i += 256) Y[i + c * ldY] = 0.0;
  if (threadIdx.x == 0) {
    col[c].bnorm = bn;
    col[c].rz = 0.0;
    col[c].iters = 0;
    col[c].done = (zero || sqrt(rr) <= tol * bn) ? 1 : 0;
    if (col[c].done) atomicAdd(ndone, 1);
  }
}

// rz_new = r^T z; p = z (first) or z + (rz_new / rz) p.
__global__ __launch_bounds__(256) void cg_dir_kernel(const double* __restrict__ Rm, const double* __restrict__ Zm,
                                                     double* __restrict__ P, int64_t ld, int64_t KMp,
                                                     CgCol* __restrict__ col, int first) {
  __shared__ double red[4];
  const int64_t c = blockIdx.x;
  if (col[c].done) return;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < KMp; i += 256) s += Rm[i + c * ld] * Zm[i + c * ld];
  const double rz = block_sum(s, red);
  const double beta = first ? 0.0 : rz / col[c].rz;
  for (int64_t i = threadIdx.x; i < KMp; i += 256) {
    const int64_t e = i + c * ld;
    P[e] = Zm[e] + (first ? 0.0 : beta * P[e]);
  }
  if (threadIdx.x == 0) col[c].rz = rz;
}

// alpha = rz / p^T q; y += alpha p; r -= alpha q; convergence test on ||r||.
__global__ __launch_bounds__(256) void cg_step_kernel(const double* __restrict__ P, const double* __restrict__ Q,
                                                      double* __restrict__ Y, int64_t ldY, double* __restrict__ Rm,
                                                      int64_t ld, int64_t KMp, double tol, CgCol* __restrict__ col,
                                                      int* __restrict__ ndone, int iter) {
  __shared__ double red[4];
  const int64_t c = blockIdx.x;
  if (col[c].done) return;
  double s = 0.0;
  for (int64_t i = threadIdx.x; i < KMp; i += 256) s += P[i + c * ld] * Q[i + c * ld];
  const double pq = block_sum(s, red);
  if (!(pq > 0.0)) {   // breakdown (not positive definite, or exact convergence)
    if (threadIdx.x == 0) { col[c].done = 2; col[c].iters = iter; atomicAdd(ndone, 1); }
    return;
  }
  const double alpha = col[c].rz / pq;
  double rr = 0.0;
  for (int64_t i = threadIdx.x; i < KMp; i += 256) {
    Y[i + c * ldY] += alpha * P[i + c * ld];
    const double r = Rm[i + c * ld] - alpha * Q[i + c * ld];
    Rm[i + c * ld] = r;
    rr += r * r;
  }
  rr = block_sum(rr, red);
  if (threadIdx.x == 0) {
    col[c].iters = iter;
    if (sqrt(rr) <= tol * col[c].bnorm) {
      col[c].done = 1;
      atomicAdd(ndone, 1);
    }
  }
}

hipError_t launch_cg_start(const double* Bm, int64_t ldB, const double* Q, double* Rm, double* Y, int64_t ldY,
                           int64_t ld, int64_t KM, int64_t KMp, int64_t R, double tol, CgCol* col, int* ndone,
                           hipStream_t s) {
  if (R <= 0) return hipSuccess;
  hipLaunchKernelGGL(cg_start_kernel, dim3((unsigned)R), dim3(256), 0, s, Bm, ldB, Q, Rm, Y, ldY, ld, KM, KMp, tol,
                     col, ndone);
  return hipGetLastError();
}

hipError_t launch_cg_dir(const double* Rm, const double* Zm, double* P, int64_t ld, int64_t KMp, int64_t R,
                         CgCol* col, int first, hipStream_t s) {
  if (R <= 0) return hipSuccess;
  hipLaunchKernelGGL(cg_dir_kernel, dim3((unsigned)R), dim3(256), 0, s, Rm, Zm, P, ld, KMp, col, first);
  return hipGetLastError();
}

hipError_t launch_cg_step(const double* P, const double* Q, double* Y, int64_t ldY, double* Rm, int64_t ld,
                          int64_t KMp, int64_t R, double tol, CgCol* col, int* ndone, int iter, hipStream_t s) {
  if (R <= 0) return hipSuccess;
  hipLaunchKernelGGL(cg_step_kernel, dim3((unsigned)R), dim3(256), 0, s, P, Q, Y, ldY, Rm, ld, KMp, tol, col, ndone,
                     iter);
  return hipGetLastError();
}


// ---------------------------------------- member block-Jacobi application
// z[o_k + i] = sum_c Dinv_k[i, c] r[o_k + c] for every member block k
// (o_k = k M), all right-hand sides; Dinv_k is Mp x Mp (ld Mp).
struct MemberApply {
  static constexpr int BM = 64, BN = 64, WM = 2, WN = 2, KC = 16;
  static constexpr int LDA = BM + 16, LDB = BN + 1;
  static constexpr int NA = BM * KC / 256, NB_ = BN * KC / 256;
  const double* Dinv; const double* Rm; double* Zm;
  int64_t ld, M, Mp, R;
  int ntr, ntc, nblk;
  struct Ctx { bool valid; int64_t kb, i0, c0; int nchunks; };
  struct ARegs { double v[NA]; };
  struct BRegs { double v[NB_]; };
  __device__ Ctx ctx(int tile) const {
    Ctx c;
    const int per = ntr * ntc;
    c.kb = tile / per;
    const int u = tile % per, tr = u % ntr, tc = u / ntr;
    c.valid = c.kb < nblk;
    c.i0 = (int64_t)tr * BM;
    c.c0 = (int64_t)tc * BN;
    c.nchunks = (int)((M + KC - 1) / KC);
    return c;
  }
  __device__ void loadA(const Ctx& c, int chunk, ARegs& r) const {   // As[k][row] = Dinv_k(i0 + row, k)
    const double* A = Dinv + c.kb * Mp * Mp;
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = threadIdx.x + 256 * q, row = e % BM, kk = e / BM;
      const int64_t i = c.i0 + row, k = (int64_t)chunk * KC + kk;
      r.v[q] = (i < M && k < M) ? A[i + k * Mp] : 0.0;
    }
  }
  __device__ void storeA(const ARegs& r, double* As) const {
#pragma unroll
    for (int q = 0; q < NA; ++q) {
      const int e = threadIdx.x + 256 * q;
      As[(e / BM) * LDA + e % BM] = r.v[q];
    }
  }
  __device__ void loadB(const Ctx& c, int chunk, BRegs& r) const {   // Bs[k][col] = r(o_k + k, c0 + col)
    const double* B = Rm + c.kb * M;
#pragma unroll
    for (int q = 0; q < NB_; ++q) {
      const int e = threadIdx.x + 256 * q, kk = e % KC, col = e / KC;
      const int64_t k = (int64_t)chunk * KC + kk, cc = c.c0 + col;
      r.v[q] = (k < M && cc < R) ? B[k + cc * ld] : 0.0;
    }
  }
  __device__ void storeB(const BRegs& r, double* Bs) const {
#pragma unroll
    for (int q = 0; q < NB_; ++q) {
      const int e = threadIdx.x + 256 * q;
      Bs[(e % KC) * LDB + e / KC] = r.v[q];
    }
  }
  __device__ void epilogue(const Ctx& c, const TileF64<BM, BN, WM, WN>& acc) const {
    acc.for_each([&](int row, int col, double v) {
      const int64_t i = c.i0 + row, cc = c.c0 + col;
      if (i < M && cc < R) Zm[(c.kb * M + i) + cc * ld] = v;
    });
  }
};

hipError_t launch_member_apply(const double* Dinv, int64_t K, int64_t M, int64_t Mp, const double* Rm, double* Zm,
                               int64_t ld, int64_t R, hipStream_t s) {
  if (R <= 0) return hipSuccess;
  MemberApply g;
  g.Dinv = Dinv; g.Rm = Rm; g.Zm = Zm; g.ld = ld; g.M = M; g.Mp = Mp; g.R = R;
  g.ntr = (int)ceil_div(M, MemberApply::BM);
  g.ntc = (int)ceil_div(R, MemberApply::BN);
  g.nblk = (int)K;
  hipLaunchKernelGGL(gemm_f64_kernel<MemberApply>, dim3((unsigned)(K * g.ntr * g.ntc)), dim3(256), 0, s, g);
  return hipGetLastError();
}

// rows [from, to) of every column set to zero
__global__ void zero_rows_kernel(double* __restrict__ Z, int64_t ld, int64_t from, int64_t to) {
  const int64_t c = blockIdx.y;
  for (int64_t i = from + threadIdx.x; i < to; i += blockDim.x) Z[i + c * ld] = 0.0;
}

hipError_t launch_zero_rows(double* Z, int64_t ld, int64_t from, int64_t to, int64_t R, hipStream_t s) {
  if (R <= 0 || to <= from) return hipSuccess;
  hipLaunchKernelGGL(zero_rows_kernel, dim3(1, (unsigned)R), dim3(64), 0, s, Z, ld, from, to);
  return hipGetLastError();
}

}  // namespace pc
