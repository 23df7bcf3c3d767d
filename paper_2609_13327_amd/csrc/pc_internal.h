// Internal declarations shared by the host library and the kernel files.
#pragma once
#include <hip/hip_runtime.h>
#include <stdint.h>

#include <vector>

namespace pc {

// The localization modes read by the kernels: a dense n_h x M matrix, or
// separable modes generated where they are read,
//   W[a n_lon + i, m] = U[a, m] * Phi[i, m]   (a: latitude row, i: longitude),
// so that no n_h x M array exists (the paper notes that analytic modes can be
// computed when needed instead of stored, Sec. 3.11).  Both return the same
// FP64 value for the same (j, m): fl(U Phi) is the definition of W then.
struct WDense {
  const double* W; int64_t ld;
  __device__ __forceinline__ double operator()(int64_t j, int64_t m) const { return W[j + m * ld]; }
};
struct WSep {
  const double* U; int64_t ldU;
  const double* Phi; int64_t ldPhi;
  int64_t n_lon; double inv;   // inv = 1 / n_lon (row split by a rounded quotient, corrected once)
  __device__ __forceinline__ double operator()(int64_t j, int64_t m) const {
    int64_t a = (int64_t)((double)j * inv);
    int64_t i = j - a * n_lon;
    if (i < 0) { --a; i += n_lon; } else if (i >= n_lon) { ++a; i -= n_lon; }
    return U[a + m * ldU] * Phi[i + m * ldPhi];
  }
};


constexpr int NB = 64;  // Cholesky / triangular-solve block size
constexpr int kLowRowPad = 64;   // row padding of the fp32 copies: the contraction rows of one bf16 Gram stage

inline int64_t round_up(int64_t a, int64_t b) { return (a + b - 1) / b * b; }
inline int64_t ceil_div(int64_t a, int64_t b) { return (a + b - 1) / b; }

// Device-side control of the refinement of one instance.  Every right-hand
// side stops on its own (RhsCtl): once stopped, its iterate is no longer
// updated; the instance is done when none is running.
struct RefineCtl {
  int done;                  // 0 running, 1 all converged, 2 some stalled above the acceptance level, 3 some diverging
  int iters;                 // refinement iterations applied (to the slowest right-hand side)
  int running;               // right-hand sides still running after the last update (counted by it)
  int stops;                 // bit 1: a right-hand side stalled, bit 2: one diverged
  unsigned long long worst;  // bits of max over running rhs of max|delta| / max|y| (non-negative double)
  double last, prev;         // worst relative update of the last and the previous iteration
};

// One right-hand side's refinement (state as RefineCtl::done).
struct RhsCtl {
  int state, iters, stall, pad;
  double last, prev;         // relative update max|delta| / max|y| of the last and the previous iteration
};

// Everything the kernels need to know about one instance.
struct Inst {
  int64_t n_h, n_w, K, M;
  int64_t n, KM, KMp, P;   // n = n_h*n_w, KMp = KM rounded up to NB, P = K(K+1)/2
  const double* E; int64_t ldE;
  const double* W; int64_t ldW;          // dense modes (null for separable modes)
  const double* U = nullptr; int64_t ldU = 0;      // separable modes: n_lat x M latitude factors
  const double* Phi = nullptr; int64_t ldPhi = 0;  // and n_lon x M longitude factors
  int64_t n_lon = 0;
  int64_t max_rhs;
  // plan-owned device buffers
  double* G = nullptr;       // KMp x KMp, ld = KMp; Gram then its Cholesky factor (lower)
  double* diag0 = nullptr;   // KMp: diagonal of the Gram before factoring
  double* Linv = nullptr;    // (KMp/NB) blocks of NB x NB: inverses of the diagonal blocks of L
  double* Lt = nullptr;      // final strictly-lower tiles of L, tile-major, written once per factorization
  double* Msol = nullptr;    // 4 x (KMp/NB) blocks NB x NB: the block solves' folded last two updates
  int64_t lt_tiles = 0;      // capacity of Lt in 64 x 64 tiles
  double* S = nullptr;       // n_h x ldS per-column Grams (row j holds the P packed pairs, zero padded)
  int64_t ldS = 0;           // P rounded up to the 128-pair Gram tile
  double* G2 = nullptr;      // contraction parts 2.. of a split FP64 Gram (only when the tiles are few)
  int g2_parts = 0;          // parts G2 has room for ((g2_parts) x KMp x KMp)
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
  // fp32 copies of E and W for the bf16 Grams: E32 has ldE32 = n rounded up
  // to kLowRowPad rows (zero beyond n) and K + 1 columns (column K zero); W32
  // has ldW32 = n_h rounded up to kLowRowPad rows (zero beyond n_h)
  float* E32 = nullptr; int64_t ldE32 = 0;
  float* W32 = nullptr; int64_t ldW32 = 0;
  int* lp_tiles = nullptr; int64_t lp_ntiles = 0;   // reduced-precision Gram tiles (ta, tb), in launch order
  RefineCtl* ctl = nullptr;  // device refinement control
  RhsCtl* rhs = nullptr;     // max_rhs per-right-hand-side controls
  std::vector<RhsCtl> rhs_host;   // per-right-hand-side outcome of the last apply
  int64_t last_R = 0;        // right-hand sides of the last apply of this instance
  // CG on the stored Gram (plans built with PC_FLAG_KEEP_GRAM)
  double* Gs = nullptr;      // KMp x KMp symmetric copy of the assembled Gram
  double* Dinv = nullptr;    // (KMp/NB) blocks NB x NB: inverses of the diagonal blocks of Gs
  double* cg = nullptr;      // four KMp x max_rhs buffers: r, z, p, q
  struct CgCol* cgcol = nullptr;
  int* cg_flags = nullptr;   // [0] converged columns, [1] block-Jacobi pivot failure
  // member block-Jacobi (PC_FLAG_CG_MEMBER_BLOCKS): inverses of the K diagonal M x M blocks
  int64_t cgm_Mp = 0;        // M rounded up to 64
  double* cgm_Dinv = nullptr;   // K x Mp x Mp
  double* cgm_work = nullptr;   // 2 x Mp x Mp: block copy, forward-solve result
  double* cgm_I = nullptr;      // Mp x Mp identity
  double* cgm_d0 = nullptr;     // Mp: diagonal of the block copy
  double* cgm_Linv = nullptr;   // (Mp/64) x 64 x 64
  int* cgm_ctr = nullptr;       // DAG and solve counters of one block
  int64_t* cgm_offs = nullptr; int64_t cgm_ntasks = 0;
  // launch-shape choices of the autotuner (0: built-in heuristic)
  int tune_gram_split = 0;   // FP64 Gram: 1 to 4 contraction parts
  int tune_ztx_split = 0;    // Z^T x: 1 or 2 contraction parts
  int tune_gemm_tile = 0;    // blocked factorization products: 0 by size, 1 128 x 128, 2 256 x 128 tiles
  int tune_chol_per_cu = 0;  // Cholesky DAG: persistent workgroups per compute unit (1 or 2)
  // blocked outer factorization (large Grams): block columns of blk_NO (0: tile DAG only)
  int64_t blk_NO = 0;
  double* blk_P = nullptr;   // KMp x blk_NO copy of a panel
  double* blk_X = nullptr;   // blk_NO x blk_NO inverse of a diagonal block
  double* blk_I = nullptr;   // blk_NO x blk_NO identity
  int64_t* blk_offs = nullptr; int64_t blk_ntasks = 0;            // DAG order of a full diagonal block
  int64_t* blk_offs_tail = nullptr; int64_t blk_ntasks_tail = 0;  // and of the last, smaller one
  bool factored = false;
  int prec = 0;              // precision of the current Gram (a pc_precision value); the ladder raises it
  int iters = 0;
  double last_rel = 0.0;
};

inline WDense wdense(const Inst& in) { return WDense{in.W, in.ldW}; }
inline WSep wsep(const Inst& in) {
  return WSep{in.U, in.ldU, in.Phi, in.ldPhi, in.n_lon, 1.0 / (double)(in.n_lon > 0 ? in.n_lon : 1)};
}

// Mode-pair tiles of the FP64 Gram (four ints per tile: m0, m0', m1, m1').
std::vector<int> make_qtiles(int64_t M);

// ---- kernels (launchers return hipError_t of the launch) ----
hipError_t launch_pairs_init(const Inst& in, hipStream_t s);
hipError_t launch_column_grams(const Inst& in, hipStream_t s);
// Zero rows of the per-column Grams S past n_h (read by the FP64 Gram's last chunk).
constexpr int kGramZeroRows = 32;
hipError_t launch_gram_f64(const Inst& in, hipStream_t s);
hipError_t launch_gram_lowprec(const Inst& in, int precision, hipStream_t s);
// fp32 copies E32, W32 of E and W (the bf16 forms' operands), before their Gram
hipError_t launch_stage_f32(const Inst& in, hipStream_t s);
// launch order of the lower-triangle 128 x 128 tiles of a reduced-precision
// Gram: (ta, tb) pairs, grouped by the pair of 128-mode blocks they read
std::vector<int> lowgram_tile_order(int64_t KM, int64_t M);
// reduced-precision Grams of several instances in one launch (after each
// instance's rounded Z has been staged)
// (the rounded Z is formed tile by tile from E and W inside the Gram kernel)
struct LowGramInst {
  const double* E; int64_t ldE;
  const double* W; int64_t ldW;       // dense modes, or null: separable (U, Phi)
  const double* U; int64_t ldU;
  const double* Phi; int64_t ldPhi;
  int64_t n_lon; double inv_lon;
  const float* E32; int64_t ldE32;   // fp32 copies (bf16 forms only)
  const float* W32; int64_t ldW32;
  int64_t n, n_h, n_w, K, M, KM;
  double* G; int64_t ldG;
};
struct LowGramTile { int inst, ta, tb, pad; };
struct LowGramBatch {
  LowGramTile* tiles = nullptr; LowGramInst* insts = nullptr; int* mode = nullptr;
  int64_t ntiles = 0; int count = 0;
};
LowGramBatch* make_lowgram_batch(const std::vector<Inst>& insts);
void free_lowgram_batch(LowGramBatch* b);
// per-instance precision codes (host array of b->count); a batched launch of
// one precision computes only the instances of that precision
hipError_t set_lowgram_modes(const LowGramBatch* b, const int* modes, hipStream_t s);
hipError_t launch_gram_lowprec_batch(const LowGramBatch* b, int precision, hipStream_t s);
hipError_t launch_gram_pad_and_diag(const Inst& in, hipStream_t s);
// after_reset (may be null) is recorded once the tile states are reset,
// before the factorization starts (unblocked factorizations only)
hipError_t launch_cholesky(const Inst& in, hipStream_t s, hipEvent_t after_reset = nullptr);
hipError_t launch_solve_fold(const Inst& in, hipStream_t s);
int* chol_error_flag(const Inst& in);   // device int set when a bounded wait of the factorization expired
// `skip` (device int, may be null): when nonzero at run time the kernels exit
// at once; the refinement loop uses it to stop converged instances on the GPU.
hipError_t launch_ztx(const Inst& in, const double* X, int64_t ldX, int64_t R, double* B,
                      int64_t ldB, hipStream_t s, const int* skip = nullptr);
// B = Zt^T Xt with the rounded operands of a reduced-precision form
// (precision PC_PREC_FP32_REFINE: fp32; PC_PREC_BF16_REFINE: bf16), MFMA
// with fp32 accumulation, stored in FP64 (hipErrorInvalidValue otherwise)
hipError_t launch_ztx_lowprec(const Inst& in, int precision, const double* X, int64_t ldX, int64_t R, double* B,
                              int64_t ldB, hipStream_t s);
// out = Xsub - Z Y  (Xsub may be null: out = Z Y)
hipError_t launch_zy(const Inst& in, const double* Y, int64_t ldY, int64_t R, const double* Xsub,
                     int64_t ldXs, double* out, int64_t ldOut, hipStream_t s, const int* skip = nullptr);
// out = alpha Xs + beta (Z Y) (Xs may be null: beta (Z Y)); out may alias Xs
hipError_t launch_zy_axpby(const Inst& in, const double* Y, int64_t ldY, int64_t R, const double* Xs,
                           int64_t ldXs, double alpha, double beta, double* out, int64_t ldOut, hipStream_t s,
                           const int* skip = nullptr);
// in-place Y <- L^{-T} L^{-1} Y on the KMp x R block (ld = ldY), using work buffer Wk
// (first_pass = 1: Wk already holds L^{-1} Y, only the backward pass runs)
hipError_t launch_chol_solve(const Inst& in, double* Y, int64_t ldY, int64_t R, double* Wk,
                             int64_t ldW, hipStream_t s, const int* skip = nullptr, int first_pass = 0);
// in.B <- L^{-1} in.Y (R right-hand sides) while the unblocked factorization runs on another stream
hipError_t launch_chol_solve_fwd_concurrent(const Inst& in, int64_t R, hipStream_t s);
int* chol_solve_fwd_error_flag(const Inst& in);   // device int set when one of its bounded waits expired
hipError_t launch_copy_rows(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t rows,
                            int64_t rows_zero_to, int64_t R, hipStream_t s);
hipError_t launch_refine_init(RefineCtl* ctl, RhsCtl* rhs, int64_t R, int budget, hipStream_t s);
// Y[:, r] += D[:, r]; the worst relative update goes to ctl->worst.
// (per right-hand side: stop rule of refine_check_kernel on its own updates)
hipError_t launch_refine_update(const Inst& in, double* Y, int64_t ldY, const double* Dl,
                                int64_t ldD, int64_t R, RefineCtl* ctl, double tol, double accept, hipStream_t s);
// one thread: the instance is done once no right-hand side is running
hipError_t launch_refine_check(RefineCtl* ctl, hipStream_t s);
hipError_t launch_nonfinite_check(const double* A, int64_t ld, int64_t rows, int64_t cols,
                                  int* flag, hipStream_t s);
hipError_t launch_export_lower(const double* src, int64_t lds, double* dst, int64_t ldd,
                               int64_t n, hipStream_t s);
hipError_t launch_fill_int(int* p, int v, int64_t count, hipStream_t s);
// C = alpha A B^T (or C += alpha A B^T when accumulate), column-major, FP64 MFMA;
// lower != 0 writes only the lower triangle (i >= j) of a square C
// tile: 0 by size, 1: 128 x 128 tiles, 2: 256 x 128 tiles; K must be a
// multiple of 16 (hipErrorInvalidValue otherwise; the blocked paths use
// multiples of 64)
// tri_b != 0: B(j, k) = 0 for k > j (a lower-triangular B), so each column
// tile contracts only the k up to its last column
hipError_t launch_nt_gemm(const double* A, int64_t lda, const double* B, int64_t ldb, double* C, int64_t ldc,
                          int64_t M, int64_t N, int64_t K, double alpha, int accumulate, int lower, hipStream_t s,
                          int tile = 0, int tri_b = 0);
// C (M x N) += alpha opA opB^T for the blocked solves: opA(i, k) = A[i + k lda]
// (or A[k + i lda] with ta), opB(j, k) = B[k + j ldb]; nothing when *skip != 0;
// K a multiple of 16.
hipError_t launch_solve_gemm(bool ta, const double* A, int64_t lda, const double* B, int64_t ldb, double* C,
                             int64_t ldc, int64_t M, int64_t N, int64_t K, double alpha, const int* skip,
                             hipStream_t s);
hipError_t launch_copy_panel(const double* src, int64_t lds, double* dst, int64_t ldd, int64_t rows, int64_t cols,
                             hipStream_t s);
hipError_t launch_identity(double* I, int64_t n, hipStream_t s);
int64_t chol_task_offsets(int T, std::vector<int64_t>& offs, int G = 0);   // G <= 0: the default group
// All instances of a plan in one persistent Cholesky launch and one pair of
// solve launches (task lists interleaved, largest instance first).
struct DagBatch;
DagBatch* make_dag_batch(const std::vector<Inst>& insts);   // null on allocation failure
void free_dag_batch(DagBatch* b);
int* dag_batch_error(const DagBatch* b);                    // device int: a bounded wait expired
hipError_t launch_cholesky_batch(const DagBatch* b, hipStream_t s, int per_cu = 0);
hipError_t set_batch_rhs(const DagBatch* b, const int64_t* R, hipStream_t s);   // R: host, one per instance
// G^{-1} on the plan buffers of every instance: Y (refine = 0) or D (refine = 1, skipping
// converged instances), with B as the work buffer
hipError_t launch_chol_solve_batch(const DagBatch* b, int refine, hipStream_t s);
int gram_split_for(const Inst& in);      // contraction parts the FP64 Gram would use untuned (1 to 4)
int gram_parts_used(const Inst& in);     // contraction parts of the next FP64 Gram launch
int check_chol_task_order(int T, int G = 0);

// ---------------------------------------------------------------- learned warm start
enum { MLP_EPI_STORE = 0, MLP_EPI_BIAS_GELU = 1, MLP_EPI_BIAS = 2, MLP_EPI_GELU_GRAD = 3 };
// C(m, n) = sum_k A(m, k) B(n, k), fp32 in global memory, MFMA operands bf16 or fp32.
//   A(m, k) = A[m * sam + k * sak], B(n, k) = B[n * sbn + k * sbk]; a_kcont / b_kcont
//   say which index is contiguous (sak == 1 / sbk == 1).  Output row-major, ld ldc.
//   partial (max_splits * M * N floats) allows a split contraction; may be null.
struct MlpGemm {
  const float* A; int64_t sam, sak;
  const float* B; int64_t sbn, sbk;
  int64_t M, N, K;
  int a_kcont, b_kcont;
  int mode;
  float* C; int64_t ldc;
  const float* bias;       // per column n (BIAS modes)
  float* C2;               // gelu(C) (BIAS_GELU), ld ldc
  const float* aux;        // pre-activation (GELU_GRAD), ld ldc
  float* partial; int max_splits; int64_t partial_cap;   // partial holds partial_cap floats
  int64_t kper; int vec;   // set by the launcher
};
hipError_t launch_mlp_gemm(const MlpGemm& g, int bf16, hipStream_t s);
hipError_t launch_mlp_loss(const float* Y, int64_t ldY, const float* T, int64_t ldT, int64_t d, int64_t B,
                           float* dY, float* row_loss, float* loss, hipStream_t s);
hipError_t launch_mlp_colsum(const float* G, int64_t ld, int64_t rows, int64_t cols, float* out, hipStream_t s);
// Adam coefficients: beta1, beta2, 1 - beta1, 1 - beta2, bias corrections 1 - beta^t
struct AdamCoef { float lr, b1, b2, omb1, omb2, bc1, bc2, eps; };
hipError_t launch_mlp_adam(float* p, const float* g, float* m, float* v, int64_t n, const AdamCoef& c,
                           hipStream_t s);
hipError_t launch_training_pairs(const double* Bm, int64_t ldB, const double* Ym, int64_t ldY, int64_t d, int64_t N,
                                 float* X, int64_t ldX, float* T, int64_t ldT, hipStream_t s);
hipError_t launch_ws_prep(const double* Bm, int64_t ldB, int64_t d, int64_t R, float* Xh, int64_t ldX, double* nrm,
                          hipStream_t s);
hipError_t launch_ws_finish(const float* Yh, int64_t ldYh, const double* nrm, int64_t d, int64_t R, double* Y0,
                            int64_t ldY0, hipStream_t s);

// ---------------------------------------------------------------- CG on the stored Gram
struct CgCol { double bnorm, rz; int done, iters; };
// symmetric full copy of the assembled (padded) Gram: Gs = G + tril(G, -1)^T
hipError_t launch_gram_symmetrize(const Inst& in, double* Gs, hipStream_t s);
// the structured FP64 Gram assembled straight into in.Gs (symmetric, padded),
// for plans whose factored Gram is a reduced-precision one
hipError_t launch_kept_fp64_gram(const Inst& in, hipStream_t s);
// Dinv[t] = inverse of the t-th 64 x 64 diagonal block of Gs (block-Jacobi); flag set if not SPD
hipError_t launch_bj_setup(const double* Gs, int64_t ld, int64_t T, double* Dinv, int* flag, hipStream_t s);
// Z = blockdiag(Dinv) Rm on KMp x R
hipError_t launch_bj_apply(const double* Dinv, int64_t T, const double* Rm, double* Zm, int64_t ld, int64_t R,
                           hipStream_t s);
// Q = Gs P (KMp x KMp times KMp x R), all ld = ld
hipError_t launch_member_apply(const double* Dinv, int64_t K, int64_t M, int64_t Mp, const double* Rm, double* Zm,
                               int64_t ld, int64_t R, hipStream_t s);
hipError_t launch_zero_rows(double* Z, int64_t ld, int64_t from, int64_t to, int64_t R, hipStream_t s);
hipError_t launch_member_block_inverse(const double* Gs, int64_t ld, int64_t o, int64_t M, int64_t Mp, double* D,
                                       double* d0, double* Linv, int* ctr, const int64_t* offs, int64_t ntasks,
                                       const double* I, double* Wk, double* Dinv, int* info, hipStream_t s);
hipError_t launch_gram_matmul(const double* Gs, int64_t KMp, const double* P, double* Q, int64_t ld, int64_t R,
                              hipStream_t s);
// r = b - Q (Q may be null: cold start, y = 0); a zero column b gives y = 0 and is done
hipError_t launch_cg_start(const double* Bm, int64_t ldB, const double* Q, double* Rm, double* Y, int64_t ldY,
                           int64_t ld, int64_t KM, int64_t KMp, int64_t R, double tol, CgCol* col, int* ndone,
                           hipStream_t s);
hipError_t launch_cg_dir(const double* Rm, const double* Zm, double* P, int64_t ld, int64_t KMp, int64_t R,
                         CgCol* col, int first, hipStream_t s);
hipError_t launch_cg_step(const double* P, const double* Q, double* Y, int64_t ldY, double* Rm, int64_t ld,
                          int64_t KMp, int64_t R, double tol, CgCol* col, int* ndone, int iter, hipStream_t s);

}  // namespace pc

// The network object behind the C handle pc_mlp (include/pcsqrt.h).
struct pc_mlp {
  int device = 0;
  int64_t d = 0, h = 0, max_batch = 0;
  int bf16 = 1;
  int64_t nparams = 0;       // h*d + h + d*h + d
  float* params = nullptr;   // [W1 (h x d, row-major) | b1 (h) | W2 (d x h, row-major) | b2 (d)]
  float* grads = nullptr;    // same layout
  float* m = nullptr;        // Adam moments, same layout
  float* v = nullptr;
  int64_t step = 0;          // Adam steps taken
  // activations for max_batch rows
  float* Apre = nullptr;     // B x h pre-activation
  float* H = nullptr;        // B x h
  float* Y = nullptr;        // B x d output
  float* dY = nullptr;       // B x d
  float* dA = nullptr;       // B x h
  float* row_loss = nullptr; // B
  float* loss = nullptr;     // 1
  float* Xh = nullptr;       // B x d normalized warm-start input
  double* nrm = nullptr;     // B norms of the warm-start inputs
  float* partial = nullptr;  // split-contraction partials: max_splits x B x max(d, h)
  int max_splits = 16;
};

