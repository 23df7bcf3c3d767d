// Small bandwidth-bound helpers: copies with zero padding, the refinement
// update with its per-right-hand-side norms, finiteness checks and fills.
#include "pc_common.h"
#include "pc_internal.h"

namespace pc {

// dst[0:rows_zero_to, r] = (i < rows ? src[i, r] : 0) for every column r.
__global__ void copy_rows_kernel(const double* __restrict__ src, int64_t lds, double* __restrict__ dst,
                                 int64_t ldd, int64_t rows, int64_t rows_zero_to) {
  const int64_t r = blockIdx.y;
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < rows_zero_to;
       i += (int64_t)gridDim.x * blockDim.x)
    dst[i + r * ldd] = (i < rows) ? src[i + r * lds] : 0.0;
}

hipError_t launch_copy_rows(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t rows,
                            int64_t rows_zero_to, int64_t R, hipStream_t s) {
  if (R <= 0 || rows_zero_to <= 0) return hipSuccess;
  unsigned gx = (unsigned)std::min<int64_t>(ceil_div(rows_zero_to, 256), 64);
  hipLaunchKernelGGL(copy_rows_kernel, dim3(gx, (unsigned)R), dim3(256), 0, s, src, lds, dst, ldd, rows,
                     rows_zero_to);
  return hipGetLastError();
}

__global__ void refine_init_kernel(RefineCtl* ctl, RhsCtl* rhs, int64_t R, int budget) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) {
    ctl->done = budget > 0 ? 0 : 1;
    ctl->iters = 0;
    ctl->running = 0;
    ctl->stops = 0;
    ctl->worst = 0ULL;
    ctl->last = 0.0;
    ctl->prev = 0.0;
  }
  if (i < R) rhs[i] = RhsCtl{budget > 0 ? 0 : 1, 0, 0, 0, 0.0, 0.0};
}

hipError_t launch_refine_init(RefineCtl* ctl, RhsCtl* rhs, int64_t R, int budget, hipStream_t s) {
  const int64_t n = std::max<int64_t>(R, 1);
  hipLaunchKernelGGL(refine_init_kernel, dim3((unsigned)ceil_div(n, 256)), dim3(256), 0, s, ctl, rhs, R, budget);
  return hipGetLastError();
}

// The stop rule of one right-hand side after an update of relative size rel
// = max|delta| / max|y|.  Stop at the tolerance, or once the updates stop
// shrinking (two iterations in a row with less than a halving): then the
// contraction ratio rho = last / previous estimates what further iterations
// could still change, last * rho / (1 - rho) for rho < 1, else last (the
// updates fluctuate at the attainable accuracy of the FP64 residual).  The
// result is accepted (1) if that estimate is at most `accept` and rho < 0.9
// (a ratio near 1, from a preconditioner far from the Gram, as for a rounded
// Z much better conditioned than Z, cannot bound the remaining change), and
// reported as stalled (2) otherwise.  It is diverging (3) when the update is
// not finite, or is growing and already as large as y (at the attainable
// accuracy the updates fluctuate in size, so growth alone does not mean
// divergence).
__device__ __forceinline__ void rhs_stop_rule(RhsCtl& c, double rel, double tol, double accept) {
  c.iters += 1;
  c.prev = c.last;
  c.last = rel;
  if (rel <= tol) {
    c.state = 1;
  } else if (!(rel < INFINITY) || (c.iters >= 2 && rel >= 1.0 && rel > c.prev)) {
    c.state = 3;
  } else if (c.iters >= 2 && rel > 0.5 * c.prev) {
    if (++c.stall >= 2) {
      const double rho = rel / c.prev;
      const double est = rho < 1.0 ? rel * rho / (1.0 - rho) : rel;
      c.state = (est <= accept && rho < 0.9) ? 1 : 2;
    }
  } else {
    c.stall = 0;
  }
}

// Y[:, r] += D[:, r] over the first KM rows for every right-hand side still
// running, then its stop rule.  One workgroup per right-hand side.
__global__ __launch_bounds__(256) void refine_update_kernel(double* __restrict__ Y, int64_t ldY,
                                                            const double* __restrict__ D, int64_t ldD,
                                                            int64_t KM, RefineCtl* ctl, RhsCtl* rhs, double tol,
                                                            double accept) {
  __shared__ double red[2][4];
  if (ctl->done) return;
  const int64_t r = blockIdx.x;
  if (rhs[r].state != 0) return;
  double md = 0.0, my = 0.0;
  for (int64_t i = threadIdx.x; i < KM; i += 256) {
    const double d = D[i + r * ldD];
    const double y = Y[i + r * ldY] + d;
    Y[i + r * ldY] = y;
    md = fmax(md, fabs(d));
    my = fmax(my, fabs(y));
  }
  md = wave_max(md);
  my = wave_max(my);
  if (lane_id() == 0) { red[0][wave_id()] = md; red[1][wave_id()] = my; }
  __syncthreads();
  if (threadIdx.x == 0) {
    double a = red[0][0], b = red[1][0];
    for (int w = 1; w < 4; ++w) { a = fmax(a, red[0][w]); b = fmax(b, red[1][w]); }
    double rel = b > 0.0 ? a / b : (a > 0.0 ? INFINITY : 0.0);
    if (!(rel >= 0.0)) rel = INFINITY;   // NaN
    RhsCtl c = rhs[r];
    rhs_stop_rule(c, rel, tol, accept);
    rhs[r] = c;
    atomicMax(&ctl->worst, (unsigned long long)__double_as_longlong(rel));
    if (c.state == 0) atomicAdd(&ctl->running, 1);
    else if (c.state == 2) atomicOr(&ctl->stops, 1);
    else if (c.state == 3) atomicOr(&ctl->stops, 2);
  }
}

hipError_t launch_refine_update(const Inst& in, double* Y, int64_t ldY, const double* Dl, int64_t ldD,
                                int64_t R, RefineCtl* ctl, double tol, double accept, hipStream_t s) {
  if (R <= 0) return hipSuccess;
  hipLaunchKernelGGL(refine_update_kernel, dim3((unsigned)R), dim3(256), 0, s, Y, ldY, Dl, ldD, in.KM, ctl, in.rhs,
                     tol, accept);
  return hipGetLastError();
}

// One thread, after an update: the instance is done when no right-hand side
// is still running; its outcome is the worst of theirs.
__global__ void refine_check_kernel(RefineCtl* ctl) {
  if (ctl->done) return;
  const double worst = __longlong_as_double((long long)ctl->worst);
  ctl->worst = 0ULL;
  ctl->iters += 1;
  ctl->prev = ctl->last;
  ctl->last = worst;
  if (ctl->running == 0) ctl->done = (ctl->stops & 2) ? 3 : (ctl->stops & 1) ? 2 : 1;
  ctl->running = 0;
}

hipError_t launch_refine_check(RefineCtl* ctl, hipStream_t s) {
  hipLaunchKernelGGL(refine_check_kernel, dim3(1), dim3(1), 0, s, ctl);
  return hipGetLastError();
}

__global__ void nonfinite_kernel(const double* __restrict__ A, int64_t ld, int64_t rows, int64_t cols,
                                 int* flag) {
  const int64_t total = rows * cols;
  int bad = 0;
  for (int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; e < total;
       e += (int64_t)gridDim.x * blockDim.x) {
    const int64_t i = e % rows, c = e / rows;
    if (!isfinite(A[i + c * ld])) bad = 1;
  }
  if (bad) atomicOr(flag, 1);
}

hipError_t launch_nonfinite_check(const double* A, int64_t ld, int64_t rows, int64_t cols, int* flag,
                                  hipStream_t s) {
  const int64_t total = rows * cols;
  unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(total, 256), 4096));
  hipLaunchKernelGGL(nonfinite_kernel, dim3(g), dim3(256), 0, s, A, ld, rows, cols, flag);
  return hipGetLastError();
}

__global__ void export_lower_kernel(const double* __restrict__ src, int64_t lds, double* __restrict__ dst,
                                    int64_t ldd, int64_t n) {
  const int64_t c = blockIdx.x;
  for (int64_t r = c + threadIdx.x; r < n; r += blockDim.x) dst[r + c * ldd] = src[r + c * lds];
}

hipError_t launch_export_lower(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t n,
                               hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(export_lower_kernel, dim3((unsigned)n), dim3(256), 0, s, src, lds, dst, ldd, n);
  return hipGetLastError();
}

__global__ void fill_int_kernel(int* p, int v, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = v;
}

hipError_t launch_fill_int(int* p, int v, int64_t count, hipStream_t s) {
  if (count <= 0) return hipSuccess;
  unsigned g = (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(count, 256), 1024));
  hipLaunchKernelGGL(fill_int_kernel, dim3(g), dim3(256), 0, s, p, v, count);
  return hipGetLastError();
}

}  // namespace pc
