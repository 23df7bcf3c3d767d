// Allocation-free factor-and-apply (pc_factor_apply_noalloc, include/pcsqrt.h).
//
// The same kernels as pc_sqrt_build + pc_factor_apply on one FP64 instance,
// with every workspace buffer of the plan (per-column Grams, Gram and factor,
// diagonal-block inverses, final-tile copy, folded solve operators, the
// right-hand-side buffers, DAG counters, task tables) carved out of one
// fixed device array instead of being allocated.  Nothing here calls an
// allocating HIP routine.
#include <algorithm>
#include <mutex>
#include <vector>

#include "pcsqrt.h"
#include "pc_internal.h"

namespace {

constexpr size_t kScratchBytes = (size_t)PC_NOALLOC_WORKSPACE_BYTES;

// The workspace.  Every device the library runs on holds its own copy until
// the process ends; calls on one device share it (and so must not overlap).
static __device__ __align__(256) unsigned char scratch[kScratchBytes];

// Device address of `scratch` per device: the host-side name is only a
// stand-in, so the address is looked up once per device (with that device
// current) and only this address is ever passed to kernels.
std::mutex g_mu;
std::vector<void*> g_ptr;      // indexed by device ordinal, null until looked up

pc_status scratch_address(int dev, unsigned char** out) {
  std::lock_guard<std::mutex> lock(g_mu);
  if (dev < 0) return PC_ERR_DEVICE;
  if ((size_t)dev >= g_ptr.size()) g_ptr.resize((size_t)dev + 1, nullptr);
  if (!g_ptr[(size_t)dev]) {
    void* p = nullptr;
    if (hipGetSymbolAddress(&p, HIP_SYMBOL(scratch)) != hipSuccess || !p) return PC_ERR_DEVICE;
    g_ptr[(size_t)dev] = p;
  }
  *out = (unsigned char*)g_ptr[(size_t)dev];
  return PC_OK;
}

// Bump allocation inside the workspace (256-byte aligned pieces); with a
// null base it only counts.
struct Carve {
  unsigned char* base;
  size_t used = 0;
  template <class T>
  T* take(int64_t count) {
    const size_t off = (used + 255) & ~(size_t)255;
    used = off + sizeof(T) * (size_t)std::max<int64_t>(count, 1);
    return base ? (T*)(base + off) : nullptr;
  }
};

// Lays out every buffer the single-instance FP64 path needs; returns the bytes used.
size_t layout(pc::Inst& in, int64_t R, unsigned char* base) {
  Carve c{base};
  const int64_t KMp = in.KMp, T = KMp / pc::NB;
  in.G = c.take<double>(KMp * KMp);
  in.diag0 = c.take<double>(KMp);
  in.Linv = c.take<double>(T * pc::NB * pc::NB);
  in.Msol = c.take<double>(4 * T * pc::NB * pc::NB);
  in.lt_tiles = T * (T - 1) / 2;
  in.Lt = c.take<double>(std::max<int64_t>(in.lt_tiles, 1) * pc::NB * pc::NB);
  in.S = c.take<double>(in.n_h * in.ldS);
  in.pairs = c.take<int>(2 * in.P);
  in.qtiles = c.take<int>(4 * (int64_t)in.nq);
  in.B = c.take<double>(KMp * R);
  in.Y = c.take<double>(KMp * R);
  in.info = c.take<int>(1);
  in.dag = c.take<int>(T * T + 2 + T * in.nrt_max + 2);
  in.chol_offs = c.take<int64_t>(T);
  (void)c.take<int>(1);   // finiteness flag, located right after (see below)
  return c.used;
}

}  // namespace

extern "C" pc_status pc_factor_apply_noalloc(const pc_instance* inst, const double* X, int64_t ldX, int64_t R,
                                             double* Y, int64_t ldY, void* stream) {
  if (!inst) return PC_ERR_INVALID_ARG;
  const pc_instance& a = *inst;
  if (a.n_h < 1 || a.n_w < 1 || a.K < 1 || a.M < 1 || R < 0) return PC_ERR_SHAPE;
  if (a.K * a.M > a.n_h * a.n_w) return PC_ERR_SHAPE;
  if (!a.E || !a.W || a.ldE < a.n_h * a.n_w || a.ldW < a.n_h) return PC_ERR_INVALID_ARG;
  if (R == 0) return PC_OK;
  if (!X || !Y || ldX < a.n_h * a.n_w || ldY < a.K * a.M) return PC_ERR_INVALID_ARG;

  pc::Inst in;
  in.n_h = a.n_h; in.n_w = a.n_w; in.K = a.K; in.M = a.M;
  in.n = a.n_h * a.n_w; in.KM = a.K * a.M; in.KMp = pc::round_up(in.KM, pc::NB);
  in.P = a.K * (a.K + 1) / 2;
  in.E = a.E; in.ldE = a.ldE; in.W = a.W; in.ldW = a.ldW; in.max_rhs = R;
  in.ldS = pc::round_up(in.P, 128);
  in.nrt_max = (int)pc::ceil_div(R, pc::NB);
  in.tune_gram_split = 1;     // one contraction part: no partial Grams
  in.tune_chol_per_cu = 0;
  const int64_t T = in.KMp / pc::NB;
  // the tile DAG over the whole Gram (the blocked factorization needs more buffers)
  if (in.KMp > 8192) return PC_ERR_WORKSPACE;
  const std::vector<int> qt = pc::make_qtiles(in.M);
  in.nq = (int)(qt.size() / 4);
  std::vector<int64_t> offs;
  in.chol_ntasks = pc::chol_task_offsets((int)T, offs);
  if (layout(in, R, nullptr) > kScratchBytes) return PC_ERR_WORKSPACE;

  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess) return PC_ERR_DEVICE;
  unsigned char* base = nullptr;
  pc_status st = scratch_address(dev, &base);
  if (st != PC_OK) return st;
  const size_t used = layout(in, R, base);
  int* d_flag = (int*)(base + used - sizeof(int));
  hipStream_t s = (hipStream_t)stream;
#define NA_TRY(expr) do { if ((expr) != hipSuccess) return PC_ERR_DEVICE; } while (0)
  // The workspace keeps the previous call's contents: clear what must start
  // at zero (fill kernels, no memset nodes), and upload the task tables.
  // E and W are checked for NaN/Inf first (one sync), as pc_sqrt_build does.
  NA_TRY(pc::launch_fill_int(d_flag, 0, 1, s));
  NA_TRY(pc::launch_copy_rows(nullptr, 0, in.S, in.n_h * in.ldS, 0, in.n_h * in.ldS, 1, s));   // padding pairs
  NA_TRY(pc::launch_copy_rows(nullptr, 0, in.B, in.KMp, 0, in.KMp, R, s));   // padding rows of the solves
  NA_TRY(pc::launch_copy_rows(nullptr, 0, in.Y, in.KMp, 0, in.KMp, R, s));
  NA_TRY(hipMemcpyAsync(in.qtiles, qt.data(), qt.size() * sizeof(int), hipMemcpyHostToDevice, s));
  NA_TRY(hipMemcpyAsync(in.chol_offs, offs.data(), offs.size() * sizeof(int64_t), hipMemcpyHostToDevice, s));
  NA_TRY(pc::launch_nonfinite_check(in.E, in.ldE, in.n, in.K, d_flag, s));
  NA_TRY(pc::launch_nonfinite_check(in.W, in.ldW, in.n_h, in.M, d_flag, s));
  int bad = 0;
  NA_TRY(hipMemcpyAsync(&bad, d_flag, sizeof(int), hipMemcpyDeviceToHost, s));
  NA_TRY(hipStreamSynchronize(s));
  if (bad) return PC_ERR_NONFINITE;
  NA_TRY(pc::launch_pairs_init(in, s));
  NA_TRY(pc::launch_fill_int(in.info, -1, 1, s));
  // Gram, factorization, b = Z^T x, two triangular solves, copy-out
  NA_TRY(pc::launch_column_grams(in, s));
  NA_TRY(pc::launch_gram_f64(in, s));
  NA_TRY(pc::launch_gram_pad_and_diag(in, s));
  NA_TRY(pc::launch_cholesky(in, s));
  int h[3] = {-1, 0, 0};
  NA_TRY(hipMemcpyAsync(&h[0], in.info, sizeof(int), hipMemcpyDeviceToHost, s));
  NA_TRY(hipMemcpyAsync(&h[1], pc::chol_error_flag(in), sizeof(int), hipMemcpyDeviceToHost, s));
  NA_TRY(pc::launch_ztx(in, X, ldX, R, in.Y, in.KMp, s));
  NA_TRY(pc::launch_chol_solve(in, in.Y, in.KMp, R, in.B, in.KMp, s));
  NA_TRY(hipMemcpyAsync(&h[2], pc::chol_error_flag(in), sizeof(int), hipMemcpyDeviceToHost, s));
  NA_TRY(pc::launch_copy_rows(in.Y, in.KMp, Y, ldY, in.KM, in.KM, R, s));
  NA_TRY(hipStreamSynchronize(s));   // also keeps qt / offs alive until their copies are done
#undef NA_TRY
  if (h[1] || h[2]) return PC_ERR_DEVICE;   // a bounded wait expired
  if (h[0] >= 0) return PC_ERR_NOT_SPD;
  return PC_OK;
}
