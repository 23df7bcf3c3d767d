// Blocked right-looking FP64 Cholesky G = L L^T and the two triangular solves.
//
// Block size NB = 64.  Step kb of the factorization:
//   chol_diag    one workgroup factors the NB x NB diagonal block in LDS and,
//                with the same elimination steps, forms its inverse Linv_kb
//   chol_panel   L[ib,kb] = G[ib,kb] * Linv_kb^T for the blocks below (MFMA)
//   chol_update  G[ib,jb] -= L[ib,kb] L[jb,kb]^T for kb < jb <= ib (MFMA)
// A pivot d_j <= 64 * KM * 2^-53 * G_jj marks Z as numerically rank
// deficient (d_j / G_jj is the squared sine between column j of Z and the
// span of the previous columns; for an exactly dependent column it is pure
// rounding noise, bounded by about KM * u), as does a non-finite pivot.
//
// Solves (R right-hand sides, blocks of 64 columns):
//   forward   for kb ascending: z_kb = Linv_kb b_kb;  b_ib -= L[ib,kb] z_kb (ib > kb)
//   backward  for kb descending: y_kb = Linv_kb^T z_kb;  z_ib -= L[kb,ib]^T y_kb (ib < kb)
// Each step is one launch; the workgroups of a step recompute the small
// product with the inverse diagonal block themselves, so no other
// synchronization than stream order is needed.
#include "pc_common.h"
#include "pc_internal.h"

namespace pc {

constexpr int LDT = NB + 1;  // padded LDS stride for the diagonal block

__global__ __launch_bounds__(256) void chol_diag_kernel(double* __restrict__ G, int64_t ld, int64_t KM,
                                                        int64_t kb, const double* __restrict__ diag0,
                                                        double* __restrict__ Linv, int* info) {
  __shared__ double A[NB * LDT];   // A[r * LDT + c], lower triangle used
  __shared__ double X[NB * LDT];   // becomes L^{-1}
  __shared__ int fail;
  if (*info >= 0) return;
  const int t = threadIdx.x;
  const int64_t k0 = kb * NB;
  for (int idx = t; idx < NB * NB; idx += 256) {
    const int r = idx % NB, c = idx / NB;
    A[r * LDT + c] = (r >= c) ? G[(k0 + r) + (k0 + c) * ld] : 0.0;
    X[r * LDT + c] = (r == c) ? 1.0 : 0.0;
  }
  if (t == 0) fail = -1;
  __syncthreads();
  const double thr_scale = 64.0 * (double)KM * 1.1102230246251565e-16;  // 64 KM 2^-53
  for (int j = 0; j < NB; ++j) {
    if (t == 0) {
      const double d = A[j * LDT + j];
      const double ref = diag0[k0 + j];
      if (!(d > thr_scale * ref) || !isfinite(d)) {
        fail = (int)(k0 + j);
      } else {
        A[j * LDT + j] = sqrt(d);
      }
    }
    __syncthreads();
    if (fail >= 0) break;
    const double ljj = A[j * LDT + j];
    const double inv = 1.0 / ljj;
    if (t > j && t < NB) A[t * LDT + j] *= inv;
    if (t <= j) X[j * LDT + t] *= inv;
    __syncthreads();
    // trailing update of A and elimination in X
    const int w = NB - 1 - j;
    for (int idx = t; idx < w * w; idx += 256) {
      const int r = j + 1 + idx / w, c = j + 1 + idx % w;
      if (c <= r) A[r * LDT + c] -= A[r * LDT + j] * A[c * LDT + j];
    }
    for (int idx = t; idx < w * (j + 1); idx += 256) {
      const int r = j + 1 + idx / (j + 1), c = idx % (j + 1);
      X[r * LDT + c] -= A[r * LDT + j] * X[j * LDT + c];
    }
    __syncthreads();
  }
  if (fail >= 0) {
    if (t == 0) *info = fail;   // one diagonal block is factored at a time
    return;
  }
  for (int idx = t; idx < NB * NB; idx += 256) {
    const int r = idx % NB, c = idx / NB;
    if (r >= c) G[(k0 + r) + (k0 + c) * ld] = A[r * LDT + c];
    Linv[kb * NB * NB + r + c * NB] = (r >= c) ? X[r * LDT + c] : 0.0;
  }
}

// L[ib,kb] = G[ib,kb] * Linv^T : one workgroup per 64-row block below the diagonal.
__global__ __launch_bounds__(256) void chol_panel_kernel(double* __restrict__ G, int64_t ld, int64_t kb,
                                                         const double* __restrict__ Linv, const int* info) {
  __shared__ double As[NB * NB];   // As[c * NB + r] = G[i0 + r, k0 + c]
  __shared__ double Bs[NB * NB];   // Bs[c * NB + c'] = Linv[c', c]
  if (*info >= 0) return;
  const int64_t ib = kb + 1 + blockIdx.x;
  const int64_t i0 = ib * NB, k0 = kb * NB;
  const double* Lb = Linv + kb * NB * NB;
  for (int idx = threadIdx.x; idx < NB * NB; idx += 256) {
    const int r = idx % NB, c = idx / NB;
    As[c * NB + r] = G[(i0 + r) + (k0 + c) * ld];
    Bs[c * NB + r] = Lb[r + c * NB];   // r plays c'
  }
  __syncthreads();
  TileF64<NB, NB, 2, 2> acc;
  acc.zero();
  acc.template mma<NB, NB, NB>(As, Bs);
  acc.for_each([&](int r, int c, double v) { G[(i0 + r) + (k0 + c) * ld] = v; });
}

// G[ib,jb] -= L[ib,kb] L[jb,kb]^T for kb < jb <= ib.
__global__ __launch_bounds__(256) void chol_update_kernel(double* __restrict__ G, int64_t ld, int64_t kb,
                                                          int64_t nblk, const int* info) {
  __shared__ double As[NB * NB];   // As[c * NB + r] = L[i0 + r, k0 + c]
  __shared__ double Bs[NB * NB];   // Bs[c * NB + r] = L[j0 + r, k0 + c]
  if (*info >= 0) return;
  // triangular tile index -> (a, b) with b <= a, both in [0, T)
  const int64_t t = blockIdx.x;
  int64_t a = (int64_t)((sqrt(8.0 * (double)t + 1.0) - 1.0) * 0.5);
  while ((a + 1) * (a + 2) / 2 <= t) ++a;
  while (a * (a + 1) / 2 > t) --a;
  const int64_t b = t - a * (a + 1) / 2;
  const int64_t ib = kb + 1 + a, jb = kb + 1 + b;
  if (ib >= nblk) return;
  const int64_t i0 = ib * NB, j0 = jb * NB, k0 = kb * NB;
  for (int idx = threadIdx.x; idx < NB * NB; idx += 256) {
    const int r = idx % NB, c = idx / NB;
    As[c * NB + r] = G[(i0 + r) + (k0 + c) * ld];
    Bs[c * NB + r] = G[(j0 + r) + (k0 + c) * ld];
  }
  __syncthreads();
  TileF64<NB, NB, 2, 2> acc;
  acc.zero();
  acc.template mma<NB, NB, NB>(As, Bs);
  const bool diag = ib == jb;
  acc.for_each([&](int r, int c, double v) {
    if (!diag || r >= c) G[(i0 + r) + (j0 + c) * ld] -= v;
  });
}

hipError_t launch_cholesky(const Inst& in, hipStream_t s) {
  const int64_t nblk = in.KMp / NB, ld = in.KMp;
  for (int64_t kb = 0; kb < nblk; ++kb) {
    hipLaunchKernelGGL(chol_diag_kernel, dim3(1), dim3(256), 0, s, in.G, ld, in.KM, kb, in.diag0, in.Linv,
                       in.info);
    const int64_t T = nblk - kb - 1;
    if (T > 0) {
      hipLaunchKernelGGL(chol_panel_kernel, dim3((unsigned)T), dim3(256), 0, s, in.G, ld, kb, in.Linv,
                         in.info);
      hipLaunchKernelGGL(chol_update_kernel, dim3((unsigned)(T * (T + 1) / 2)), dim3(256), 0, s, in.G, ld,
                         kb, nblk, in.info);
    }
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------- solves
// One forward step.  blockIdx.x = row block offset (0 -> the diagonal block),
// blockIdx.y = 64-column tile of the right-hand sides.
__global__ __launch_bounds__(256) void solve_fwd_kernel(const double* __restrict__ G, int64_t ld, int64_t kb,
                                                        const double* __restrict__ Linv, double* __restrict__ B,
                                                        int64_t ldB, double* __restrict__ Out, int64_t ldO,
                                                        int64_t R) {
  __shared__ double As[NB * NB];
  __shared__ double Bs[NB * NB];
  const int64_t ib = kb + blockIdx.x;
  const int64_t r0 = (int64_t)blockIdx.y * NB;
  const int64_t k0 = kb * NB, i0 = ib * NB;
  const double* Lb = Linv + kb * NB * NB;
  // t = Linv_kb * B[kb block, r tile]
  for (int idx = threadIdx.x; idx < NB * NB; idx += 256) {
    const int r = idx % NB, c = idx / NB;
    As[c * NB + r] = Lb[r + c * NB];
    Bs[r * NB + c] = (r0 + c < R) ? B[(k0 + r) + (r0 + c) * ldB] : 0.0;  // Bs[k][col], k = r
  }
  __syncthreads();
  TileF64<NB, NB, 2, 2> acc;
  acc.zero();
  acc.template mma<NB, NB, NB>(As, Bs);
  if (blockIdx.x == 0) {
    acc.for_each([&](int r, int c, double v) {
      if (r0 + c < R) Out[(k0 + r) + (r0 + c) * ldO] = v;
    });
    return;
  }
  __syncthreads();
  acc.for_each([&](int r, int c, double v) { Bs[r * NB + c] = v; });   // t as the B operand
  for (int idx = threadIdx.x; idx < NB * NB; idx += 256) {
    const int r = idx % NB, c = idx / NB;
    As[c * NB + r] = G[(i0 + r) + (k0 + c) * ld];
  }
  __syncthreads();
  TileF64<NB, NB, 2, 2> acc2;
  acc2.zero();
  acc2.template mma<NB, NB, NB>(As, Bs);
  acc2.for_each([&](int r, int c, double v) {
    if (r0 + c < R) B[(i0 + r) + (r0 + c) * ldB] -= v;
  });
}

// One backward step: blockIdx.x = 0 -> the diagonal block kb, x > 0 -> block kb - x.
__global__ __launch_bounds__(256) void solve_bwd_kernel(const double* __restrict__ G, int64_t ld, int64_t kb,
                                                        const double* __restrict__ Linv, double* __restrict__ Zb,
                                                        int64_t ldZ, double* __restrict__ Out, int64_t ldO,
                                                        int64_t R) {
  __shared__ double As[NB * NB];
  __shared__ double Bs[NB * NB];
  const int64_t ib = kb - blockIdx.x;
  const int64_t r0 = (int64_t)blockIdx.y * NB;
  const int64_t k0 = kb * NB, i0 = ib * NB;
  const double* Lb = Linv + kb * NB * NB;
  // t = Linv_kb^T * Z[kb block]
  for (int idx = threadIdx.x; idx < NB * NB; idx += 256) {
    const int r = idx % NB, c = idx / NB;
    As[r * NB + c] = Lb[r + c * NB];   // As[k][row] = Linv^T[row][k] = Linv[k][row]; here k = r, row = c
    Bs[r * NB + c] = (r0 + c < R) ? Zb[(k0 + r) + (r0 + c) * ldZ] : 0.0;
  }
  __syncthreads();
  TileF64<NB, NB, 2, 2> acc;
  acc.zero();
  acc.template mma<NB, NB, NB>(As, Bs);
  if (blockIdx.x == 0) {
    acc.for_each([&](int r, int c, double v) {
      if (r0 + c < R) Out[(k0 + r) + (r0 + c) * ldO] = v;
    });
    return;
  }
  __syncthreads();
  acc.for_each([&](int r, int c, double v) { Bs[r * NB + c] = v; });
  // L[kb, ib]^T [row][k] = L[k0 + k, i0 + row]
  for (int idx = threadIdx.x; idx < NB * NB; idx += 256) {
    const int k = idx % NB, row = idx / NB;
    As[k * NB + row] = G[(k0 + k) + (i0 + row) * ld];
  }
  __syncthreads();
  TileF64<NB, NB, 2, 2> acc2;
  acc2.zero();
  acc2.template mma<NB, NB, NB>(As, Bs);
  acc2.for_each([&](int r, int c, double v) {
    if (r0 + c < R) Zb[(i0 + r) + (r0 + c) * ldZ] -= v;
  });
}

// Y (KMp x R, ld ldY) <- G^{-1} Y using the factor; Wk is KMp x R scratch.
hipError_t launch_chol_solve(const Inst& in, double* Y, int64_t ldY, int64_t R, double* Wk, int64_t ldW,
                             hipStream_t s) {
  const int64_t nblk = in.KMp / NB, ld = in.KMp;
  const unsigned rt = (unsigned)ceil_div(R, NB);
  // forward: Y is consumed in place (rows below kb updated), z written to Wk
  for (int64_t kb = 0; kb < nblk; ++kb)
    hipLaunchKernelGGL(solve_fwd_kernel, dim3((unsigned)(nblk - kb), rt), dim3(256), 0, s, in.G, ld, kb,
                       in.Linv, Y, ldY, Wk, ldW, R);
  // backward: Wk consumed in place, y written to Y
  for (int64_t kb = nblk - 1; kb >= 0; --kb)
    hipLaunchKernelGGL(solve_bwd_kernel, dim3((unsigned)(kb + 1), rt), dim3(256), 0, s, in.G, ld, kb,
                       in.Linv, Wk, ldW, Y, ldY, R);
  return hipGetLastError();
}

}  // namespace pc
