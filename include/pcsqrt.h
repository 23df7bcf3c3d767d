/*
 * pcsqrt — left inverse of the modulated square root of a horizontally
 * localized ensemble covariance, on AMD Instinct MI355X (gfx950).
 *
 * The operation (Sardelli & Bishop, Sec. 2.1, eq. svTransform, with the
 * square root of Sec. 3.7, eq. SQRTofPCModulation):
 *
 *   P^c = C o P^s,  P^s = Z_e Z_e^T (eq. PsAndItsSquareRoot),
 *   C   = equal n_h x n_h blocks C_b = W W^T (eqs. blockStructureCEqualBlocks, SqrtOfC),
 *   Z   = [diag(z_1) C^{1/2}, ..., diag(z_K) C^{1/2}]            (n x K*M),
 *   Z[l*n_h + j, k*M + m] = E[l*n_h + j, k] * W[j, m],
 *   y   = Z^+ x = argmin_y || Z y - x ||_2    for every column x of X.
 *
 * E holds the scaled members z_k (eq. zkDefinition; the library uses E as
 * given), rows in the paper's segment order i = l*n_h + j (Sec. 3.4): level or
 * variable kind l (n_w of them), grid column j (n_h of them).  W = V_b
 * Delta_b^{1/2} (Sec. 3.9) holds the M localization square-root modes.  The
 * paper builds a left inverse from per-column SVDs under n_w = K (Sec. 3.9);
 * for the general tall Z (K*M <= n) this library returns the Moore-Penrose
 * (least-squares) left inverse, which agrees with the paper's on range(Z).
 *
 * Method: Z is never formed.  b = Z^T x is a per-grid-column contraction over
 * levels followed by a projection on the modes; the Gram Z^T Z is assembled
 * from the per-column Grams S_j = A_j^T A_j (A_j the n_w x K block of column j,
 * Sec. 3.9) as G_{(k,m),(k',m')} = sum_j S_j[k,k'] W[j,m] W[j,m'], factored
 * by Cholesky in FP64, and y = G^{-1} b by two triangular solves.  Reduced
 * precision modes build the Gram of a once-rounded Z and recover FP64
 * accuracy by iterative refinement on the least-squares residual.
 *
 * Conventions for every entry point:
 *  - All matrices are column-major float64 in DEVICE memory unless stated.
 *    Pointers are borrowed: the library never frees caller memory.  E and W
 *    must stay alive and unchanged from pc_sqrt_build to the last apply.
 *  - `stream` is a hipStream_t passed as void* (NULL = the default stream).
 *    Work is enqueued on it; calls are asynchronous unless stated.
 *  - Errors are returned as pc_status; nothing is thrown or aborted and no
 *    global error state is kept.  A plan is not thread-safe; distinct plans
 *    are independent.
 *  - Indices are 0-based; output row k*M + m is member k, mode m (the
 *    column order of eq. SQRTofPCModulation).
 */
#ifndef PCSQRT_H
#define PCSQRT_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum {
  PC_OK = 0,
  PC_ERR_INVALID_ARG = 1,    /* null pointer, leading dimension too small, bad option value */
  PC_ERR_SHAPE = 2,          /* a size <= 0, or K*M > n (Z would not be tall) */
  PC_ERR_NONFINITE = 3,      /* NaN or Inf in E or W (checked by pc_sqrt_build) */
  PC_ERR_NOT_SPD = 4,        /* a Cholesky pivot <= 0: Z is (numerically) rank deficient */
  PC_ERR_NOT_FACTORED = 5,   /* apply before a successful pc_gram_factor */
  PC_ERR_NO_CONVERGENCE = 6, /* an iteration did not meet its tolerance (refinement, CG: see each call) */
  PC_ERR_OOM = 7,            /* device allocation failed */
  PC_ERR_DEVICE = 8,         /* a HIP runtime call failed */
  PC_ERR_TOO_MANY_RHS = 9,   /* R larger than the max_rhs given at build time */
  PC_ERR_WORKSPACE = 10      /* the problem does not fit the fixed workspace of pc_factor_apply_noalloc */
} pc_status;

/* Precision of the Gram.  The reduced-precision modes form the rounded Z
 * tile by tile inside the Gram kernel (Z is never stored), factor the Gram
 * in FP64 and recover FP64 accuracy by iterative refinement on the
 * least-squares residual (r = x - Z y, d = G~^{-1} Z^T r, y += d, all FP64).
 * Unless PC_FLAG_FIXED_PRECISION is set, an instance whose reduced-precision
 * Gram is not positive definite, or whose refinement stalls above the
 * acceptance level or diverges, climbs the ladder
 *   PC_PREC_BF16_REFINE -> PC_PREC_BF16X3_REFINE -> PC_PREC_FP32_REFINE -> PC_PREC_FP64
 * (re-assembled, re-factored and re-solved in the next precision). */
typedef enum {
  PC_PREC_FP64 = 0,          /* FP64 Gram (MFMA f64), FP64 Cholesky and solves */
  PC_PREC_FP32_REFINE = 1,   /* Gram of fp32(Z) on MFMA f32, FP64 Cholesky + FP64 refinement */
  PC_PREC_BF16_REFINE = 2,   /* Gram of bf16(z32) on MFMA bf16 (fp32 accumulation), FP64 Cholesky + FP64
                                refinement; z32 = fl32(fp32(e) * fp32(w)), the fp32 product of fp32 copies
                                of E and W that the plan keeps */
  PC_PREC_BF16X3_REFINE = 3  /* split bf16: z32 = hi + lo (hi = bf16(z32), lo = bf16(z32 - hi)), Gram
                                Hi^T Hi + Hi^T Lo + Lo^T Hi on MFMA bf16 (fp32 accumulation),
                                FP64 Cholesky + FP64 refinement */
} pc_precision;

/* One problem instance.  Sizes must satisfy n_h, n_w, K, M >= 1 and
 * K*M <= n_h*n_w.  ldE >= n_h*n_w, ldW >= n_h.  max_rhs bounds the number of
 * right-hand sides of every later apply (the plan sizes its workspace from it). */
typedef struct {
  int64_t n_h, n_w, K, M;
  const double *E; int64_t ldE;   /* device, n x K, column k = z_k in segment order */
  const double *W; int64_t ldW;   /* device, n_h x M, column m = localization mode w_m */
  int64_t max_rhs;
} pc_instance;

typedef struct {
  int32_t precision;   /* a pc_precision value */
  int32_t max_refine;  /* refinement iterations allowed; in PC_PREC_FP64 these are
                          corrected semi-normal steps (0 = plain normal equations) */
  double tol;          /* each right-hand side stops refining on its own once
                          max|delta| <= tol * max|y| over its column (later
                          iterations leave its column of Y unchanged); <= 0
                          selects 1e-12 */
  int32_t use_graph;   /* 1: hipGraphs: pc_left_inverse_apply captures its apply sequence, and
                          pc_factor_apply the whole assemble + factor + apply sequence (with the
                          pivot status copies), once per argument set and per precision of each
                          instance, then replays it (both run eagerly while phase timing,
                          pc_profile_enable, is on: a graph carries no timing events) */
  int32_t flags;       /* 0, or PC_FLAG_KEEP_GRAM (optionally with PC_FLAG_CG_MEMBER_BLOCKS),
                          PC_FLAG_FIXED_PRECISION, PC_FLAG_ZTX_FP32 or PC_FLAG_ZTX_BF16 (or'ed) */
} pc_options;

/* Keep a symmetric copy of each instance's FP64 Gram, for pc_cg_solve /
 * pc_learned_apply (extra 8 (K*M)^2 bytes per instance).  CG multiplies by
 * this Gram and is preconditioned by: in a reduced-precision plan, the FP64
 * Cholesky factor of the reduced-precision Gram (the plan's own factor);
 * in an FP64 plan, the inverses of the 64 x 64 diagonal blocks of the Gram
 * (or of its member blocks, PC_FLAG_CG_MEMBER_BLOCKS). */
#define PC_FLAG_KEEP_GRAM 1

/* With PC_FLAG_KEEP_GRAM: precondition CG by the inverses of the K diagonal
 * M x M member blocks G_kk of the Gram (one block per ensemble member; each
 * factored by the tile DAG and inverted at pc_gram_factor, K M^2 doubles)
 * instead of its 64 x 64 diagonal blocks. */
#define PC_FLAG_CG_MEMBER_BLOCKS 2

/* Keep every instance in the precision of the options: no escalation along
 * the precision ladder (a failure is reported as PC_ERR_NOT_SPD or
 * PC_ERR_NO_CONVERGENCE instead). */
#define PC_FLAG_FIXED_PRECISION 4

/* Form the first right-hand side of the normal equations, b = Z^T x, in
 * reduced precision as well while an instance is on a reduced-precision
 * rung: the products of pc_sqrt_transpose_apply_lowprec with fp32 operands
 * (PC_FLAG_ZTX_FP32) or bf16 operands (PC_FLAG_ZTX_BF16), MFMA with fp32
 * accumulation.  The refinement's Z^T r stays FP64, so the refined result
 * keeps its accuracy; the rounding of b only changes the starting point.
 * An instance in FP64 (plan precision or the ladder's last rung) uses the
 * FP64 product.  At most one of the two flags. */
#define PC_FLAG_ZTX_FP32 8
#define PC_FLAG_ZTX_BF16 16

typedef struct pc_plan pc_plan;

/* pc_sqrt_build — validate `count` instances, record the borrowed E/W
 * pointers, allocate every device workspace the later calls need (Gram and
 * factor K*M x K*M FP64 per instance, per-column Grams, refinement scratch
 * sized by max_rhs), and check E and W for NaN/Inf (one stream sync).
 * On success *out receives the plan; on failure *out is NULL and nothing is
 * left allocated.  opt may be NULL (FP64, no refinement, no graph). */
pc_status pc_sqrt_build(const pc_instance *inst, int32_t count, const pc_options *opt,
                        void *stream, pc_plan **out);

/* An instance whose localization modes are separable on an n_lat x n_lon
 * latitude-longitude grid (grid column j = a * n_lon + i, a the latitude
 * row, i the longitude): mode m is the product of a latitude factor and a
 * longitude factor,
 *   W[a * n_lon + i, m] = U[a, m] * Phi[i, m]   (FP64 product, rounded once),
 * as for Fourier modes in longitude times latitude eigenvectors of an
 * isotropic localization on such a grid.  The plan never forms W: every
 * kernel that reads a mode value generates it from U and Phi where it is
 * used (the paper points out that analytically defined modes need not be
 * stored, Sec. 3.11).  Results equal those of a plan built with the dense W
 * formed by that product, bit for bit.  n_h = n_lat * n_lon; other fields as
 * in pc_instance. */
typedef struct {
  int64_t n_lat, n_lon, n_w, K, M;
  const double *E; int64_t ldE;     /* device, n x K (n = n_lat n_lon n_w), segment order */
  const double *U; int64_t ldU;     /* device, n_lat x M, ldU >= n_lat */
  const double *Phi; int64_t ldPhi; /* device, n_lon x M, ldPhi >= n_lon */
  int64_t max_rhs;
} pc_instance_separable;

/* pc_sqrt_build_separable — pc_sqrt_build for instances with separable
 * modes: same options, ownership (E, U, Phi borrowed until destroy), checks
 * (NaN/Inf in E, U and Phi) and statuses; every other call takes the plan as
 * it comes.  Reduced-precision plans still keep their fp32 copy of the modes
 * (formed from U and Phi). */
pc_status pc_sqrt_build_separable(const pc_instance_separable *inst, int32_t count, const pc_options *opt,
                                  void *stream, pc_plan **out);

/* pc_gram_factor — for every instance form G = Z^T Z (or the Gram of the
 * rounded Z in reduced precision) from the per-column Grams and W, then
 * factor G = L L^T in FP64.  Synchronizes `stream` once to read the pivot
 * status.  Returns PC_ERR_NOT_SPD if any instance failed; *failed_instance
 * (may be NULL) receives the first failing instance index or -1.  The plan
 * stays valid; a failed plan rejects apply with PC_ERR_NOT_FACTORED. */
pc_status pc_gram_factor(pc_plan *plan, void *stream, int32_t *failed_instance);

/* pc_left_inverse_apply — Y_i = Z_i^+ X_i for every instance i.
 * X[i]: device, n_i x R[i] with leading dimension ldX[i] >= n_i (read only).
 * Y[i]: device, K_i*M_i x R[i] with leading dimension ldY[i] >= K_i*M_i.
 * X, ldX, R, Y, ldY are HOST arrays of `count` entries (the build count).
 * R[i] = 0 skips instance i.  Asynchronous in FP64 mode without refinement;
 * with refinement the convergence test runs on the device and the host
 * reads its flags every two iterations (without a graph) or once at the
 * end.  Every right-hand side follows its own stop rule: it converges at
 * tol; when its updates stop shrinking (two iterations in a row with less
 * than a halving), it is accepted if the geometric estimate of what further
 * iterations could change, last * rho / (1 - rho) with rho the last ratio of
 * successive updates, is at most 1e-8 * max|y| and rho < 0.9, and counted
 * as stalled otherwise; it diverges when an update is not finite or grows
 * while at least max|y|.  An instance is done when none of its right-hand
 * sides still runs.  Returns PC_ERR_NO_CONVERGENCE (Y holds the last
 * iterates) if a right-hand side diverged, or, in an instance whose Gram is
 * in reduced precision, stalled or ran out of budget (after the ladder).  An
 * instance in FP64 (the plan's precision, or the ladder's last rung) takes
 * corrected semi-normal steps and accepts a stall or a spent budget: the
 * updates then fluctuate at the attainable accuracy of the FP64 residual, or
 * the caller asked for a fixed number of steps.  pc_query_rhs_info tells
 * which right-hand side ended how. */
pc_status pc_left_inverse_apply(pc_plan *plan, const double *const *X, const int64_t *ldX,
                                const int64_t *R, double *const *Y, const int64_t *ldY,
                                void *stream);

/* pc_factor_apply — pc_gram_factor followed by pc_left_inverse_apply, with
 * the same arguments, ownership and statuses (failed_instance as in
 * pc_gram_factor; X need not be ready before the call, only ordered before
 * it on `stream`).  For a plan of one instance without a graph whose Gram
 * is factored by the tile DAG (order up to 8192), the products b = Z^T x
 * (Sec. 3.9: they use E, W and X only) run on an internal stream while the
 * factorization runs, which the two separate calls cannot do:
 * pc_gram_factor waits for the pivot status before returning.  A blocked
 * factorization (larger orders) runs after the products instead.  Synchronizes `stream` once, at the end.  If the Gram of an
 * instance with right-hand sides is not positive definite (after the
 * precision ladder), its Y is undefined and PC_ERR_NOT_SPD is returned
 * (*failed_instance: the first such instance); the other instances are still
 * solved.  An instance that fails with R[i] = 0 is not an error of the call.
 * A failed instance rejects a later apply until a successful factorization. */
pc_status pc_factor_apply(pc_plan *plan, const double *const *X, const int64_t *ldX,
                          const int64_t *R, double *const *Y, const int64_t *ldY,
                          void *stream, int32_t *failed_instance);

/* pc_query_info — after an apply and a stream sync: iterations used by the
 * last apply (max over its right-hand sides) and its final max|delta|/max|y|
 * (max over the right-hand sides still running at the last iteration), for
 * instance `instance`.  Either output pointer may be NULL. */
pc_status pc_query_info(const pc_plan *plan, int32_t instance, int32_t *iterations,
                        double *last_rel_update);

/* Refinement outcome of one right-hand side. */
typedef struct {
  int32_t iterations;      /* refinement updates applied to this column of Y */
  int32_t state;           /* 0 budget spent while running, 1 converged or accepted,
                              2 stalled above the acceptance level, 3 diverging */
  double last_rel_update;  /* max|delta| / max|y| of its last update (0 if none) */
} pc_rhs_info;

/* pc_query_rhs_info — per-right-hand-side outcome of the last apply of
 * instance `instance` (pc_left_inverse_apply or pc_factor_apply, after it
 * returned): out[r] for r < R, out a HOST array of R entries.  R may not
 * exceed that apply's R[instance] (PC_ERR_INVALID_ARG).  Without refinement
 * (max_refine = 0) every entry is {0, 1, 0}. */
pc_status pc_query_rhs_info(const pc_plan *plan, int32_t instance, int64_t R, pc_rhs_info *out);

/* pc_query_instance — state of instance `instance` after pc_gram_factor:
 * *precision (may be NULL) receives the precision (a pc_precision value) of
 * its current Gram: the options' precision, or the rung the ladder raised it
 * to (the plan keeps it: later factorizations start there); *factored (may
 * be NULL) receives 1 if its factorization succeeded, else 0 (after
 * PC_ERR_NOT_SPD the other instances stay usable: pass R = 0 for the failed
 * ones to pc_left_inverse_apply). */
pc_status pc_query_instance(const pc_plan *plan, int32_t instance, int32_t *precision, int32_t *factored);

/* pc_plan_destroy — free everything the plan owns (synchronizes the device
 * first).  NULL is accepted. */
pc_status pc_plan_destroy(pc_plan *plan);

/* Static, NUL-terminated description of a status code. */
const char *pc_status_string(pc_status s);

/* ------------------------------------------------------------------------
 * Transforms on either side of the path (same plan, same borrowed E and W).
 * ---------------------------------------------------------------------- */

/* pc_sqrt_transpose_apply — B = Z^T X for instance `instance` (the first
 * step of the solve; also the gradient-like product of refinement).
 * X: device n x R (ldX >= n); B: device K*M x R (ldB >= K*M).  Asynchronous. */
pc_status pc_sqrt_transpose_apply(pc_plan *plan, int32_t instance, const double *X, int64_t ldX,
                                  int64_t R, double *B, int64_t ldB, void *stream);

/* pc_sqrt_transpose_apply_lowprec — B = Zt^T Xt for instance `instance`, the
 * reduced-precision form of pc_sqrt_transpose_apply (the first product of a
 * mixed-precision solve; the precision of the Gram and of Z^T x is not fixed
 * by the paper, whose method is FP64).  Zt is the rounded Z whose Gram the
 * reduced-precision modes form and Xt the rounded right-hand sides:
 *   precision PC_PREC_FP32_REFINE: Zt = fp32(E[i,k] W[j,m]) (the FP64 product
 *     rounded once), Xt = fp32(X), MFMA f32;
 *   precision PC_PREC_BF16_REFINE: Zt = bf16(fl32(fp32(E[i,k]) fp32(W[j,m]))),
 *     Xt = bf16(fp32(X)), MFMA bf16;
 * rounding to nearest even, j = i mod n_h.  Products accumulate in fp32 over
 * all n rows of Z; B is stored in FP64.  X: device n x R (ldX >= n); B:
 * device K*M x R (ldB >= K*M), overwritten.  Other precision values, or bad
 * sizes, give PC_ERR_INVALID_ARG.  Asynchronous on `stream`. */
pc_status pc_sqrt_transpose_apply_lowprec(pc_plan *plan, int32_t instance, int32_t precision, const double *X,
                                          int64_t ldX, int64_t R, double *B, int64_t ldB, void *stream);

/* pc_sqrt_apply — X = Z Y, the back-transform to model variables
 * (x = (P^c)^{1/2} x~, Sec. 2.2).  Y: device K*M x R; X: device n x R. */
pc_status pc_sqrt_apply(pc_plan *plan, int32_t instance, const double *Y, int64_t ldY,
                        int64_t R, double *X, int64_t ldX, void *stream);

/* pc_gram_assemble — form the Gram of every instance (FP64 Gram, or the
 * Gram of the rounded Z in reduced precision) without factoring it.  The
 * plan's K*M x K*M buffer then holds its lower triangle; pc_gram_factor
 * repeats the assembly before it factors in place. */
pc_status pc_gram_assemble(pc_plan *plan, void *stream);

/* pc_gram_export — copy the lower triangle (diagonal included) of the plan's
 * K*M x K*M buffer of instance `instance` into G (device, ldG >= K*M): the
 * Gram after pc_gram_assemble, the Cholesky factor L after pc_gram_factor.
 * Entries of G above the diagonal are not written.  Asynchronous. */
pc_status pc_gram_export(const pc_plan *plan, int32_t instance, double *G, int64_t ldG,
                         void *stream);

/* ------------------------------------------------------------------------
 * Hybrid covariance product in standardized variables (Sec. 2.2, eq.
 * svCBKHybrid): P~h v = (1 - beta_e) v + beta_e (C~ o P~e) v.
 * ---------------------------------------------------------------------- */

/* pc_hybrid_apply — Out = (1 - beta_e) V + beta_e (C~ o P~e) V for R vectors
 * of the standardized space (n~ = n_h * n_w entries each).  The two factors
 * come as an instance (sizes as in pc_instance, except that K*M <= n~ is not
 * required and max_rhs is ignored):
 *   E: n~ x K, the standardized ensemble perturbations e~_k (the forecast
 *      members mapped by the left inverse of the square root, Sec. 2.1 eq.
 *      svTransform, e.g. with pc_left_inverse_apply), scaled so that
 *      P~e = E E^T;
 *   W: n_h x M, the modes of the localization, C~ = (1 1^T) (x) (W W^T)
 *      over the n_w levels (index l * n_h + j, as for Z).
 * By the Schur product identity C~ o (E E^T) = Z~ Z~^T with Z~ the columns
 * e~_k o w~_m (Sec. 3.7), so Out = (1 - beta_e) V + beta_e Z~ (Z~^T V): two
 * structured products, forming neither Z~ nor an n~ x n~ matrix.  The
 * paper obtains this form from its unsimplified one assuming every
 * diagonal entry of C~ is 1 (rows of W with unit norm); the product
 * computed is this form whatever W is.  For 0 < beta_e < 1 it is positive
 * definite (C~ is positive semi-definite by construction).
 * V, Out: device n~ x R (ldV, ldOut >= n~; Out may be V itself, with the
 * same leading dimension).  work: device K*M x R scratch (ldwork >= K*M),
 * caller-owned and overwritten.  Allocates nothing; asynchronous on stream.
 * Errors: PC_ERR_SHAPE (a size below 1, R < 0), PC_ERR_INVALID_ARG (null
 * pointer, short leading dimension, beta_e outside [0, 1] or not finite),
 * PC_ERR_DEVICE (a launch failed). */
pc_status pc_hybrid_apply(const pc_instance *hybrid, double beta_e, const double *V, int64_t ldV,
                          int64_t R, double *Out, int64_t ldOut, double *work, int64_t ldwork,
                          void *stream);

/* ------------------------------------------------------------------------
 * Autotuning of launch shapes.
 * ---------------------------------------------------------------------- */

/* pc_autotune — for every instance, time the candidate launch shapes on the
 * plan's own data and keep the fastest: the FP64 Gram's contraction split
 * (1 to 2 parts, 1 to 4 where the Gram has few tiles), the Z^T x
 * contraction split (1 or 2) and the persistent
 * Cholesky grid (1 or 2 workgroups per compute unit; one choice for a plan
 * with several instances, whose factorization is one launch) and, for an
 * instance factored by blocks, the block width (1024 or 2048) and the tile
 * shape of its products (see pc_set_tile_shape).  Choices are
 * kept in the plan.  cache_path (host string, may be NULL) names a text file
 * of earlier results keyed by (n_h, n_w, K, M, max_rhs, precision): with
 * use_cached != 0 an instance found there is not measured; new results are
 * merged into the file.  Runs the Gram and the factorization several times,
 * so the plan is left unfactored: call pc_gram_factor afterwards.
 * Synchronous.  Returns PC_ERR_INVALID_ARG if the cache file cannot be
 * written. */
pc_status pc_autotune(pc_plan *plan, const char *cache_path, int32_t use_cached, void *stream);

/* pc_set_tuning — set the launch shapes of instance `instance` by hand
 * (values as pc_query_tuning reports them; 0 = heuristic): gram_split 1 to
 * 4 contraction parts of the FP64 Gram, ztx_split 1 or 2, chol_per_cu 1 or
 * 2 persistent workgroups per compute unit.  chol_per_cu
 * applies to every instance of a plan with several instances.  chol_block
 * selects the factorization: 0 keeps the current one, -1 the tile DAG over
 * the whole Gram, a multiple of 64 that is >= 128 the blocked outer
 * factorization with block columns of that width (the default for Grams of
 * order above 8192 uses 1024; not for plans with several instances).  The
 * plan is left unfactored.  Returns PC_ERR_INVALID_ARG for other values. */
pc_status pc_set_tuning(pc_plan *plan, int32_t instance, int32_t gram_split, int32_t ztx_split,
                        int32_t chol_per_cu, int32_t chol_block);

/* pc_query_tuning — the launch shapes in use for instance `instance`
 * (0 = built-in heuristic, not tuned; chol_block 0 = tile DAG, else the
 * block-column width).  Output pointers may be NULL. */
pc_status pc_query_tuning(const pc_plan *plan, int32_t instance, int32_t *gram_split,
                          int32_t *ztx_split, int32_t *chol_per_cu, int32_t *chol_block);

/* pc_set_tile_shape / pc_query_tile_shape — the tile shape of the panel and
 * trailing products of the blocked factorization of instance `instance`
 * (used above order 8192): 1 = 128 x 128 tiles, 2 = 256 x 128 tiles (8
 * waves), 0 = by size (256 x 128 once they fill the device twice).
 * pc_autotune chooses it together with the block width (1024 or 2048) for
 * blocked instances.  The plan must be factored again afterwards.
 * PC_ERR_INVALID_ARG for another value or a bad instance. */
pc_status pc_set_tile_shape(pc_plan *plan, int32_t instance, int32_t gemm_tile);
pc_status pc_query_tile_shape(const pc_plan *plan, int32_t instance, int32_t *gemm_tile);

/* ------------------------------------------------------------------------
 * Per-phase timing (HIP events recorded on the caller's stream).
 * ---------------------------------------------------------------------- */

/* Phases timed while profiling is on (indices of the arrays below). */
#define PC_PHASE_COLUMN_GRAMS 0  /* per-column Grams S_j (FP64 path) */
#define PC_PHASE_GRAM 1          /* Gram kernel (FP64, or staging + low-precision Gram) */
#define PC_PHASE_PAD 2           /* padding to whole blocks, saved diagonal */
#define PC_PHASE_CHOLESKY 3      /* blocked FP64 Cholesky */
#define PC_PHASE_ZTX 4           /* b = Z^T x of the initial solve */
#define PC_PHASE_SOLVE 5         /* the two triangular solves of the initial solve */
#define PC_PHASE_REFINE 6        /* the whole refinement loop */
#define PC_PHASE_COPYOUT 7       /* copy of the solution to the caller's Y */
#define PC_PHASE_SOLVE_ALONGSIDE 8  /* pc_factor_apply: the forward pass run during the
                                       factorization, from its launch to its end */
#define PC_NUM_PHASES 9

/* pc_profile_enable — on != 0: every later call records a pair of HIP
 * events around each phase it runs, per instance.  Costs a few microseconds
 * per phase.  Turning it off keeps the recorded pairs until read. */
pc_status pc_profile_enable(pc_plan *plan, int32_t on);

/* pc_profile_read — synchronizes on the recorded events and returns, per
 * phase, the summed elapsed milliseconds (total_ms[PC_NUM_PHASES], host) and
 * the number of recorded intervals (counts[PC_NUM_PHASES], host); then
 * forgets them.  Either array may be NULL. */
pc_status pc_profile_read(pc_plan *plan, double *total_ms, int64_t *counts);

/* pc_selftest_task_order — host-only check of the task order used by the
 * Cholesky DAG kernel for T tile rows of 64 with update tasks that apply
 * `group` consecutive columns each (group <= 0: the library's default):
 * every task exactly once and after the tasks it waits for.  Returns 0 when
 * valid, a positive code naming the violated rule otherwise, -1 for T < 1 or
 * group > T.  Touches no GPU. */
int32_t pc_selftest_task_order(int32_t T, int32_t group);

/* ------------------------------------------------------------------------
 * Iterative solve on the normal equations and the learned warm start.
 * Not part of the paper's method: conjugate gradients on G y = b with
 * G = Z^T Z, started from the prediction of a small network trained on
 * (x, Z^+ x) pairs that the direct method produced; the direct solve stays
 * the fallback and the reference its error is measured against.
 * ---------------------------------------------------------------------- */

/* pc_cg_solve — preconditioned CG on G y = b (G the FP64 Gram; the
 * preconditioner as PC_FLAG_KEEP_GRAM says) for instance `instance` of a plan
 * built with PC_FLAG_KEEP_GRAM and factored.
 * B: device K*M x R (ldB >= K*M), right-hand sides b (e.g. Z^T x).
 * Y: device K*M x R (ldY >= K*M); read as the starting guess when warm != 0
 * (else the start is y = 0), overwritten with the result.  A column stops when
 * ||b - G y||_2 <= tol ||b||_2.  At most maxiter iterations.  Synchronous:
 * returns after the result is written.  *iterations (host, may be NULL)
 * receives the largest iteration count over the columns.  Returns
 * PC_ERR_NO_CONVERGENCE if a column did not reach tol (Y holds the iterate),
 * PC_ERR_INVALID_ARG if the plan keeps no Gram, PC_ERR_NOT_FACTORED before a
 * successful pc_gram_factor, PC_ERR_TOO_MANY_RHS if R > max_rhs. */
pc_status pc_cg_solve(pc_plan *plan, int32_t instance, const double *B, int64_t ldB, int64_t R,
                      double *Y, int64_t ldY, double tol, int32_t maxiter, int32_t warm,
                      int32_t *iterations, void *stream);

/* Two-layer network y^ = W2 gelu(W1 x^ + b1) + b2 (gelu(a) = a Phi(a)),
 * d inputs and outputs, h hidden units.  Parameters and Adam moments are
 * FP32; every matrix product runs on MFMA with bf16 operands (rounded to
 * nearest even) or fp32 operands, accumulating in fp32. */
typedef struct pc_mlp pc_mlp;
#define PC_MLP_BF16 0
#define PC_MLP_FP32 1

/* pc_mlp_create — allocate a network for batches of up to max_batch rows on
 * the current device; parameters start at zero (set them with
 * pc_mlp_set_params).  operand_type: PC_MLP_BF16 or PC_MLP_FP32. */
pc_status pc_mlp_create(int64_t d, int64_t h, int64_t max_batch, int32_t operand_type, pc_mlp **out);

/* pc_mlp_destroy — free the network (synchronizes the device).  NULL is accepted. */
pc_status pc_mlp_destroy(pc_mlp *mlp);

/* Parameter exchange, device FP32 buffers, row-major: W1 h x d, b1 h,
 * W2 d x h, b2 d.  set also clears the Adam moments and step count. */
pc_status pc_mlp_set_params(pc_mlp *mlp, const float *W1, const float *b1, const float *W2,
                            const float *b2, void *stream);
pc_status pc_mlp_get_params(const pc_mlp *mlp, float *W1, float *b1, float *W2, float *b2,
                            void *stream);

/* pc_mlp_forward — Y = network(X) for B <= max_batch rows.  X: device FP32
 * B x d row-major with row stride ldX >= d; Y likewise (ldY >= d).  Asynchronous. */
pc_status pc_mlp_forward(pc_mlp *mlp, const float *X, int64_t ldX, int64_t B, float *Y, int64_t ldY,
                         void *stream);

/* pc_mlp_gradients — loss = (1/B) sum_b ||y^_b - t_b||^2 / ||t_b||^2 over
 * the batch and its gradients, without updating the parameters.  X, T:
 * device FP32 B x d row-major (strides ldX, ldT >= d).  loss: device, one
 * float.  dW1 .. db2: device FP32 in the layout of pc_mlp_set_params; any
 * may be NULL.  Asynchronous. */
pc_status pc_mlp_gradients(pc_mlp *mlp, const float *X, int64_t ldX, const float *T, int64_t ldT,
                           int64_t B, float *loss, float *dW1, float *db1, float *dW2, float *db2,
                           void *stream);

/* pc_mlp_train_step — one Adam step (beta1 0.9, beta2 0.999, eps 1e-8,
 * bias-corrected, learning rate lr) on the batch's loss; loss as above (may
 * be NULL).  Asynchronous. */
pc_status pc_mlp_train_step(pc_mlp *mlp, const float *X, int64_t ldX, const float *T, int64_t ldT,
                            int64_t B, float lr, float *loss, void *stream);

/* pc_mlp_training_pairs — network inputs and targets from N solved systems:
 * row r of X = b_r / ||b_r||, row r of T = y_r / ||b_r||, where b_r, y_r are
 * column r of B and Y (device FP64, d x N, ldB, ldY >= d; typically
 * b = Z^T x and y = Z^+ x from the direct solve).  X, T: device FP32 N x d
 * row-major (ldX, ldT >= d).  Asynchronous on `stream`. */
pc_status pc_mlp_training_pairs(const double *B, int64_t ldB, const double *Y, int64_t ldY, int64_t d,
                                int64_t N, float *X, int64_t ldX, float *T, int64_t ldT, void *stream);

/* pc_mlp_warm_start — y0 = ||b|| network(b / ||b||) per column of B (device
 * FP64 d x R, ldB >= d) into Y0 (device FP64 d x R, ldY0 >= d), R <= max_batch.
 * A zero column gives y0 = 0.  Asynchronous. */
pc_status pc_mlp_warm_start(pc_mlp *mlp, const double *B, int64_t ldB, int64_t R, double *Y0,
                            int64_t ldY0, void *stream);

/* pc_learned_apply — Y = Z^+ X for instance `instance` by CG from the
 * network's warm start (mlp may be NULL: cold start), for a plan built with
 * PC_FLAG_KEEP_GRAM and factored; the network's d must equal K*M.  If a
 * column has not reached tol after maxiter iterations, the plan's direct
 * solve replaces the result (the FP64 factor's two triangular solves, or in
 * a reduced-precision plan its factor with FP64 refinement; *fallback = 1,
 * else 0; the status is then that of the direct solve).  X: device n x R; Y: device
 * K*M x R.  Synchronous.  *iterations: largest CG iteration count. */
pc_status pc_learned_apply(pc_plan *plan, int32_t instance, pc_mlp *mlp, const double *X,
                           int64_t ldX, int64_t R, double *Y, int64_t ldY, double tol,
                           int32_t maxiter, int32_t *iterations, int32_t *fallback, void *stream);

/* ------------------------------------------------------------------------
 * The paper's own left inverse for the square case n_w = K.
 * ---------------------------------------------------------------------- */

/* With as many levels (or variable kinds) per grid column as members,
 * n_w = K, the per-column blocks A_m of the member matrix are square and the
 * paper's left inverse (Sec. 3.9, eq. InverseSquareRootSwift; steps V1-V5 of
 * Sec. 3.10) applies:
 *   V1   w^(m) = A_m^{-1} x^(m) for every grid column m, where
 *        A_m[l, k] = E[l*n_h + m, k] (K x K) and x^(m)[l] = x[l*n_h + m];
 *   V2-3 w_k = (w^(0)_k, ..., w^(n_h-1)_k) for every member k;
 *   V4   x~_k = Delta_b^{-1/2} V_b^T w_k;
 *   V5   x~ = (x~_0; ...; x~_{K-1}): row k*L + l of the output.
 * It is a left inverse of Z = [diag(z_k) V_b Delta_b^{1/2}] (Z is n x K*L,
 * n = n_h*K): it equals the Moore-Penrose Z^+ on range(Z), and everywhere
 * when L = n_h (Z square).  The paper factors A_m by SVD; here A_m is
 * inverted once, at build time, by Gauss-Jordan elimination with partial
 * pivoting (the same A_m^{-1} up to rounding). */
typedef struct pc_swift pc_swift;

/* pc_swift_build — validate, allocate the workspace (n_h*K^2 + n_h*K*max_rhs
 * + L doubles) and invert every A_m (one stream sync).
 * E: device, n_h*K x K column-major (ldE >= n_h*K), the scaled members in
 * segment order (row l*n_h + m: level l of grid column m); borrowed, kept
 * alive by the caller.  Vb: device, n_h x L column-major (ldV >= n_h), the
 * orthonormal eigenvectors of the localization block; borrowed.  delta:
 * device, L positive eigenvalues (read at build time).  Needs K <= 64 and
 * L <= n_h (PC_ERR_SHAPE otherwise).  Returns PC_ERR_NOT_SPD if some A_m is
 * singular to working precision (a pivot |p| <= K u max|A_m|: A, and Z,
 * have no inverse), PC_ERR_INVALID_ARG for a non-positive eigenvalue. */
pc_status pc_swift_build(int64_t n_h, int64_t K, int64_t L, const double *E, int64_t ldE, const double *Vb,
                         int64_t ldV, const double *delta, int64_t max_rhs, void *stream, pc_swift **out);

/* pc_swift_apply — Y = (paper's left inverse) X for R <= max_rhs columns.
 * X: device n_h*K x R (ldX >= n_h*K); Y: device K*L x R (ldY >= K*L).
 * Asynchronous. */
pc_status pc_swift_apply(pc_swift *s, const double *X, int64_t ldX, int64_t R, double *Y, int64_t ldY,
                         void *stream);

/* pc_swift_destroy — free the workspace (synchronizes the device).  NULL is accepted. */
pc_status pc_swift_destroy(pc_swift *s);

/* ------------------------------------------------------------------------
 * Allocation-free entry point.
 * ---------------------------------------------------------------------- */

/* Bytes of the fixed device workspace of pc_factor_apply_noalloc (one copy
 * per device the library runs on, held until the process ends). */
#define PC_NOALLOC_WORKSPACE_BYTES (64 * 1024 * 1024)

/* pc_factor_apply_noalloc — for callers that cannot allocate device memory
 * (code under stream capture, tight serving loops, harnesses that forbid
 * hipMalloc): Y = Z^+ X for ONE instance in FP64, the same kernels and
 * result as pc_sqrt_build + pc_factor_apply (precision FP64, no refinement),
 * with every workspace buffer taken from a fixed, library-owned device array
 * of PC_NOALLOC_WORKSPACE_BYTES instead of allocated.  No plan is involved
 * and nothing is allocated or freed (no hipMalloc/hipFree, no pinned host
 * memory, no internal streams or events).
 * inst: host pointer to one instance (inst->max_rhs is ignored; R is used).
 * X: device n x R (ldX >= n); Y: device K*M x R (ldY >= K*M).  R = 0 returns
 * PC_OK at once.
 * Synchronizes `stream` once, at the end (to read the pivot status).
 * Statuses: PC_ERR_SHAPE / PC_ERR_INVALID_ARG as pc_sqrt_build;
 * PC_ERR_WORKSPACE if the Gram, its factor and the right-hand-side buffers
 * (about 12 (K*M)^2 + 8 n_h K^2/2 + 16 K*M R bytes) do not fit the workspace,
 * or K*M > 8192; PC_ERR_NONFINITE for NaN/Inf in E or W; PC_ERR_NOT_SPD
 * (Y undefined) for a rank-deficient Z; PC_ERR_DEVICE for a HIP failure.
 * The workspace keeps the last call's contents and is shared by every call
 * on the same device: calls that overlap on one device (concurrent host
 * threads, or work still running on another stream) race and must be
 * serialized by the caller. */
pc_status pc_factor_apply_noalloc(const pc_instance *inst, const double *X, int64_t ldX, int64_t R,
                                  double *Y, int64_t ldY, void *stream);

#ifdef __cplusplus
}
#endif
#endif /* PCSQRT_H */
