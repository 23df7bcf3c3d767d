// Internal declarations shared by the host library and the kernel files.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace pc {

constexpr int NB = 64;  // Cholesky / triangular-solve block size

inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }
inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Device-side control of the refinement of one instance.
struct RefineCtl {
  int done;                  // 0 running, 1 converged, 2 stopped above the acceptance level
  int iters;                 // refinement iterations applied
  int stall;                 // consecutive iterations with less than a halving
  int pad;
  unsigned long long worst;  // bits of max over rhs of max|delta| / max|y| (non-negative double)
  double last, prev;         // relative update of the last and the previous iteration
};

// Everything the kernels need to know about one instance.
struct Inst {
  int64_t n_h, n_w, K, M;
  int64_t n, KM, KMp, P;   // n = n_h*n_w, KMp = KM rounded up to NB, P = K(K+1)/2
  const double* E; int64_t ldE;
  const double* W; int64_t ldW;
  int64_t max_rhs;
  // plan-owned device buffers
  double* G = nullptr;       // KMp x KMp, ld = KMp; Gram then its Cholesky factor (lower)
  double* diag0 = nullptr;   // KMp: diagonal of the Gram before factoring
  double* Linv = nullptr;    // (KMp/NB) blocks of NB x NB: inverses of the diagonal blocks of L
  double* S = nullptr;       // n_h x ldS per-column Grams (row j holds the P packed pairs, zero padded)
  int64_t ldS = 0;           // P rounded up to the 128-pair Gram tile
  double* G2 = nullptr;      // second half of a split FP64 Gram (only when the tiles are few)
  void* Zt = nullptr;        // reduced precision: the rounded Z, column-major, ldz rows (bf16 or fp32)
  int64_t ldz = 0;
  int* pairs = nullptr;      // P x 2: (k, k') with k <= k'
  int* qtiles = nullptr;     // nq x 2: (m0, m0') of the mode-pair tiles
  int nq = 0;
  double* B = nullptr;       // KMp x max_rhs: right-hand side of the normal equations
  double* Y = nullptr;       // KMp x max_rhs: solution / iterate
  double* D = nullptr;       // KMp x max_rhs: correction
  double* Rres = nullptr;    // n x max_rhs: least-squares residual x - Z y
  int* info = nullptr;       // device int: first failing pivot column, or -1
  int* dag = nullptr;        // DAG counters: T*T tile states, queue head, error, solve flags, solve head
  int nrt_max = 1;           // 64-column tiles of max_rhs
  int64_t* chol_offs = nullptr;  // first task index of each Cholesky look-ahead iteration
  int64_t chol_ntasks = 0;
  RefineCtl* ctl = nullptr;  // device refinement control
  bool factored = false;
  int iters = 0;
  double last_rel = 0.0;
};

// ---- kernels (launchers return hipError_t of the launch) ----
hipError_t launch_pairs_init(const Inst& in, hipStream_t s);
hipError_t launch_column_grams(const Inst& in, hipStream_t s);
hipError_t launch_gram_f64(const Inst& in, hipStream_t s);
hipError_t launch_gram_lowprec(const Inst& in, int precision, hipStream_t s);
hipError_t launch_gram_pad_and_diag(const Inst& in, hipStream_t s);
hipError_t launch_cholesky(const Inst& in, hipStream_t s);
// `skip` (device int, may be null): when nonzero at run time the kernels exit
// at once; the refinement loop uses it to stop converged instances on the GPU.
hipError_t launch_ztx(const Inst& in, const double* X, int64_t ldX, int64_t R, double* B,
                      int64_t ldB, hipStream_t s, const int* skip = nullptr);
// out = Xsub - Z Y  (Xsub may be null: out = Z Y)
hipError_t launch_zy(const Inst& in, const double* Y, int64_t ldY, int64_t R, const double* Xsub,
                     int64_t ldXs, double* out, int64_t ldOut, hipStream_t s, const int* skip = nullptr);
// in-place Y <- L^{-T} L^{-1} Y on the KMp x R block (ld = ldY), using work buffer Wk
hipError_t launch_chol_solve(const Inst& in, double* Y, int64_t ldY, int64_t R, double* Wk,
                             int64_t ldW, hipStream_t s, const int* skip = nullptr);
hipError_t launch_copy_rows(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t rows,
                            int64_t rows_zero_to, int64_t R, hipStream_t s);
hipError_t launch_refine_init(RefineCtl* ctl, int budget, hipStream_t s);
// Y[:, r] += D[:, r]; the worst relative update goes to ctl->worst.
hipError_t launch_refine_update(const Inst& in, double* Y, int64_t ldY, const double* Dl,
                                int64_t ldD, int64_t R, RefineCtl* ctl, hipStream_t s);
// one thread: decide converged / stalled from ctl->worst, then clear it
hipError_t launch_refine_check(RefineCtl* ctl, double tol, double accept, hipStream_t s);
hipError_t launch_nonfinite_check(const double* A, int64_t ld, int64_t rows, int64_t cols,
                                  int* flag, hipStream_t s);
hipError_t launch_export_lower(const double* src, int64_t lds, double* dst, int64_t ldd,
                               int64_t n, hipStream_t s);
hipError_t launch_fill_int(int* p, int v, int64_t count, hipStream_t s);
int64_t chol_task_offsets(int T, std::vector<int64_t>& offs);
int gram_split_for(const Inst& in);
int check_chol_task_order(int T);

}  // namespace pc
