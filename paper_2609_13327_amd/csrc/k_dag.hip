// Persistent tile-DAG kernels: FP64 Cholesky G = L L^T and the two
// triangular solves, on 64 x 64 tiles.
//
// A fixed grid of workgroups (two per compute unit) takes tasks from a global
// counter in a topological order and waits on per-tile counters before it
// runs a task, so independent tiles proceed while the critical path (the
// factorization of the diagonal tiles) is never held up by kernel launches.
//
// Cholesky tasks (T = KMp / 64 tile rows):
//   DIAG(k)     the diagonal step: for k >= 1 first the panel tile below the
//               previous diagonal, L_{k,k-1} = (G_{k,k-1} - L_{k,k-2}
//               L_{k-1,k-2}^T) L_{k-1,k-1}^{-T}, then the last update of the
//               diagonal tile G_kk -= L_{k,k-1} L_{k,k-1}^T, then its
//               factorization (blocked by 16, MFMA updates) and inverse
//   TRSM(i,k)   L_ik = (G_ik - L_{i,k-1} L_{k,k-1}^T) L_kk^{-T} for i >= k+2
//               (MFMA, with the inverse; the update only when k >= 1)
//   GEMM(i,j,k) G_ij -= sum_{kk = kb..k} L_i,kk L_j,kk^T for k <= j - 2 (the
//               earlier updates), kb = G floor(k / G): the updates come in
//               groups of G consecutive columns, one task per tile and group,
//               so that G_ij makes one round trip to memory per group
// Fusing a tile's last update into its TRSM/DIAG keeps the updated tile in
// the same workgroup, and DIAG chains the whole diagonal step in one
// workgroup, so the critical path crosses one workgroup hand-over per tile
// row: DIAG(k) -> DIAG(k+1).  DIAG(k+1) loads and updates its operands before
// it waits for DIAG(k)'s inverse.
// Order (look-ahead of one step): DIAG(0); then for every k: DIAG(k+1),
// TRSM(i,k) for i >= k+2, then the non-final update tasks ending at column k:
// GEMM(i,j,k) for all j >= k+2 when k closes a group ((k + 1) % G == 0),
// else only for j = k + 2 (a tile whose last non-final update is k).  A
// closing group's tasks beyond its first three columns are spread over the
// next G - 1 iterations (interleaved columns, ahead of those iterations' own
// tasks), so that the next diagonal steps are not queued behind a whole
// triangle of updates; each still comes before any task that needs it.
// Every task appears after the tasks it needs, which makes the waits
// deadlock-free: a waiting workgroup only waits for a task that another
// running workgroup has already taken.
// state[i*T + j] counts the updates applied to tile (i,j); it becomes j + 1
// once the tile is final.
//
// Pivot test: d_j <= 64 * KM * 2^-53 * G_jj or a non-finite pivot marks Z as
// numerically rank deficient (d_j / G_jj is the squared sine between column
// j of Z and the span of the previous columns; for a dependent column it is
// rounding noise of order KM * u).  The failing column goes to *info and every
// waiting workgroup abandons the DAG.
//
// Every wait is bounded: after kSpinLimit polls the workgroup records an
// error in *err and leaves, so the kernel always terminates.
#include "pc_common.h"
#include "pc_internal.h"

namespace pc {

constexpr int T64 = 64;
constexpr int LDP = T64 + 1;          // padded LDS stride
constexpr int kSolveWaves = 8;        // waves per workgroup of the solves (not the one run alongside)
constexpr long long kSpinLimit = 1LL << 22;   // polls: a few seconds at most

// Every buffer these kernels touch is in device (global) memory.  Task
// arguments are read from LDS or device memory, which leaves their pointers
// generic; casting them to the global address space keeps the accesses
// global_load/store instead of flat ones.
typedef __attribute__((address_space(1))) double gdouble;
typedef __attribute__((address_space(1))) int gint;
__device__ __forceinline__ gdouble* gp(const double* p) { return (gdouble*)p; }
__device__ __forceinline__ gint* gp(const int* p) { return (gint*)p; }

__device__ __forceinline__ int ld_acquire(const int* p) {
  return __hip_atomic_load(gp(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

__device__ __forceinline__ void st_release(int* p, int v) {
  __hip_atomic_store(gp(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// Tile data that other workgroups read while the kernel runs is moved with
// device-coherent accesses (relaxed atomics at agent scope: they go past the
// per-XCD L2 caches), so that no cache-wide write-back or invalidate is needed.
__device__ __forceinline__ double ld_c(const double* p) {
  return __hip_atomic_load(gp(p), __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}
__device__ __forceinline__ void st_c(double* p, double v) {
  __hip_atomic_store(gp(p), v, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
}

// All threads: wait until this workgroup's coherent stores have completed,
// then thread 0 publishes `v` in *flag.
__device__ __forceinline__ void publish(int* flag, int v) {
  __builtin_amdgcn_s_waitcnt(0);
  __syncthreads();
  if (threadIdx.x == 0) st_release(flag, v);
}

// Thread 0 waits until *flag >= v (or the DAG is abandoned); the coherent
// loads that follow see the producer's data.  Returns false if the task must
// be skipped.
__device__ __forceinline__ bool wait_ge(const int* flag, int v, const int* info, int* err, int* sh) {
  if (threadIdx.x == 0) {
    int ok = 1;
    long long spins = 0;
    while (ld_acquire(flag) < v) {
      // the abandon conditions are polled every 8th time, so that a poll
      // costs one round trip to memory
      if ((++spins & 7) == 0 && (ld_acquire(info) >= 0 || ld_acquire(err) != 0)) { ok = 0; break; }
      if (spins > kSpinLimit) { atomicOr((int*)gp(err), 1); ok = 0; break; }
      __builtin_amdgcn_s_sleep(1);
    }
    *sh = ok;
  }
  __syncthreads();
  const bool ok = *sh != 0;
  __syncthreads();
  return ok;
}

struct TaskDesc { int type, i, j, k; };   // type 0 DIAG(k), 1 TRSM(i,k), 2 GEMM(i,j,k)

constexpr int kGemmGroup = 6;   // columns of updates per GEMM task
constexpr int kNearCols = 3;    // columns of a closing group's tasks emitted in its own iteration

// Whether iteration k closes a group of updates, and its GEMM task count.
__host__ __device__ inline bool gemm_group_end(int k, int G) { return (k + 1) % G == 0; }
__host__ __device__ inline int64_t gemm_task_count(int T, int k, int G) {
  const int64_t m2 = T - k - 2;
  return gemm_group_end(k, G) ? m2 * (m2 + 1) / 2 : m2;
}

// The tasks of a closing group (k0) in columns j >= k0 + 2 + kNearCols are
// spread over the next G - 1 iterations: iteration k0 + d takes columns
// k0 + 1 + kNearCols + d, then every G - 1.  The last group end before
// iteration k whose tasks it carries, or -1.
__host__ __device__ inline int deferred_group(int k, int G) {
  if (G < 2) return -1;
  const int d = 1 + k % G;
  return (d <= G - 1 && k - d >= 0) ? k - d : -1;
}
__host__ __device__ inline int deferred_col0(int k0, int k) { return k0 + 1 + kNearCols + (k - k0); }
// Tasks in the columns j0, j0 + B, ... below T (column j holds T - j tiles).
__host__ __device__ inline int64_t strided_cols_tasks(int T, int j0, int B, int64_t* ncols = nullptr) {
  const int64_t n = j0 < T ? (T - 1 - j0) / B + 1 : 0;
  if (ncols) *ncols = n;
  return n * (int64_t)(T - j0) - (int64_t)B * n * (n - 1) / 2;
}
// GEMM tasks of iteration k in the order below: the deferred ones first, then
// its own (a closing group's near columns, else the single column k + 2).
__host__ __device__ inline int64_t gemm_section_count(int T, int k, int G) {
  int64_t c = 0;
  const int k0 = deferred_group(k, G);
  if (k0 >= 0) c += strided_cols_tasks(T, deferred_col0(k0, k), G - 1);
  if (gemm_group_end(k, G)) {
    const int jend = G >= 2 ? (k + 2 + kNearCols < T ? k + 2 + kNearCols : T) : T;
    for (int j = k + 2; j < jend; ++j) c += T - j;
  } else if (k + 2 < T) {
    c += T - k - 2;
  }
  return c;
}

// t -> task in the order described above; offs[k] is the first index of
// iteration k (k = 0..T-2) and offs[T-1] the task count.
__host__ __device__ TaskDesc decode_task(int64_t t, int T, const int64_t* offs, int G) {
  TaskDesc d{0, 0, 0, 0};
  if (t == 0) return d;                    // DIAG(0)
  int lo = 0, hi = T - 2;                  // largest k with offs[k] <= t
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (offs[mid] <= t) lo = mid; else hi = mid - 1;
  }
  const int k = lo;
  const int64_t u = t - offs[k];
  const int m1 = T - k - 1;                // DIAG(k+1) and the T-k-2 TRSM(i,k)
  if (u < m1) {
    if (u == 0) { d.type = 0; d.i = d.j = d.k = k + 1; }
    else { d.type = 1; d.i = k + 1 + (int)u; d.j = d.k = k; }
    return d;
  }
  int64_t w = u - m1;
  d.type = 2;
  const int k0 = deferred_group(k, G);
  if (k0 >= 0) {
    const int j0 = deferred_col0(k0, k), B = G - 1;
    int64_t n;
    const int64_t nd = strided_cols_tasks(T, j0, B, &n);
    if (w < nd) {
      // column s of the run: the largest s with C(s) = s A - B s (s - 1) / 2 <= w
      const double A = (double)(T - j0), h = A + 0.5 * B;
      int64_t sc = (int64_t)((h - sqrt(fmax(h * h - 2.0 * B * (double)w, 0.0))) / B);
      auto C = [&](int64_t x) { return x * (int64_t)(T - j0) - (int64_t)B * x * (x - 1) / 2; };
      if (sc > n - 1) sc = n - 1;
      if (sc < 0) sc = 0;
      while (sc + 1 < n && C(sc + 1) <= w) ++sc;
      while (sc > 0 && C(sc) > w) --sc;
      d.j = j0 + (int)sc * B;
      d.i = d.j + (int)(w - C(sc));
      d.k = k0;
      return d;
    }
    w -= nd;
  }
  d.k = k;
  if (!gemm_group_end(k, G)) {             // column k + 2 only
    d.i = k + 2 + (int)w; d.j = k + 2;
    return d;
  }
  int j = k + 2;                           // near columns (all of them when G = 1)
  while (w >= T - j) { w -= T - j; ++j; }
  d.j = j; d.i = j + (int)w;
  return d;
}

struct CholArgs {
  double* G; int64_t ld; int T; int64_t KM;
  const double* diag0; double* Linv;
  double* Lt;               // final strictly-lower tiles, tile-major (null: read them from G)
  int* state; int* head; int* info; int* err;
  const int64_t* offs; int64_t ntasks;
  int grp;                  // update columns per GEMM task (the order in offs was built for it)
  int64_t col_off;          // column of G's first row/column in the whole matrix (failure reports)
};

// 64 x 64 tile of column-major `M` (rows r0.., cols c0..) into LDS as
// S[c * 64 + r] (the [k][row] operand layout when the tile's columns are the
// contraction index), scaled by `scale`.  Each thread issues its 16
// coherent loads before it writes any of them, so they are in flight together.
__device__ __forceinline__ void tile_to_lds(const double* M, int64_t ld, int64_t r0, int64_t c0, double* S,
                                            double scale = 1.0) {
#pragma unroll
  for (int h = 0; h < 2; ++h) {            // two rounds of 8 loads in flight
    double v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) {
      const int idx = threadIdx.x + 256 * (8 * h + q), r = idx % T64, c = idx / T64;
      v[q] = ld_c(&M[(r0 + r) + (c0 + c) * ld]);
    }
#pragma unroll
    for (int q = 0; q < 8; ++q) S[threadIdx.x + 256 * (8 * h + q)] = scale * v[q];
  }
}

// Accumulator of a 64x64 tile (2x2 waves of 32x32) <-> column-major memory.
template <int WM, int WN>
__device__ __forceinline__ void tile_to_acc(const double* M, int64_t ld, int64_t r0, int64_t c0,
                                            TileF64<T64, T64, WM, WN>& acc, int64_t ncols_valid) {
  using Tile = TileF64<T64, T64, WM, WN>;
  const int lane = lane_id(), w = wave_id(), wm = w / WN, wn = w % WN;
#pragma unroll
  for (int fi = 0; fi < Tile::FM; ++fi)
#pragma unroll
    for (int fj = 0; fj < Tile::FN; ++fj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = wm * Tile::TM + fi * 16 + (lane >> 4) + 4 * v;
        const int c = wn * Tile::TN + fj * 16 + (lane & 15);
        acc.acc[fi][fj][v] = (c < ncols_valid) ? ld_c(&M[(r0 + r) + (c0 + c) * ld]) : 0.0;
      }
}

// Loads of one 64 x 64 column-major tile into registers, 16 per thread, in
// the order tile_store_lds writes them (S[c * 64 + r] layout).
struct TileRegs { double v[16]; };
__device__ __forceinline__ void tile_load(const double* M, int64_t ld, int64_t r0, int64_t c0, TileRegs& t) {
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int idx = threadIdx.x + 256 * q, r = idx % T64, c = idx / T64;
    t.v[q] = ld_c(&M[(r0 + r) + (c0 + c) * ld]);
  }
}
__device__ __forceinline__ void tile_store_lds(const TileRegs& t, double* S, double scale) {
#pragma unroll
  for (int q = 0; q < 16; ++q) S[threadIdx.x + 256 * q] = scale * t.v[q];
}

// Row-XOR layout of a 64 x 64 operand: element (k, n) at k * 64 + (n ^ k).
// Writing it from a column of the source (k runs across the lanes) and
// reading MFMA fragments (n runs across 16 lanes, four rows of k) both spread
// over all LDS banks, which a transposing store into the plain layout does
// not (every lane of the wave on one bank).
__device__ __forceinline__ int xs64(int k, int n) { return k * T64 + (n ^ k); }
// Accumulator tile -> LDS in a swizzled column-major layout (element (r, c)
// at c * 64 + ((r + c) & 63): conflict-free both for the accumulator's
// column-strided writes and for the column-contiguous reads below).
__device__ __forceinline__ int sw64(int r, int c) { return c * T64 + ((r + c) & (T64 - 1)); }
template <int WM, int WN>
__device__ __forceinline__ void acc_to_lds_sw(const TileF64<T64, T64, WM, WN>& acc, double* S) {
  acc.for_each([&](int r, int c, double v) { S[sw64(r, c)] = v; });
}

// Coherent, coalesced store of an LDS tile (swizzled layout) plus `add`
// (registers in the tile_load order) to column-major M: each store
// instruction of a wave writes 64 consecutive doubles of one column.
// cols_valid limits the columns written; lower_only keeps r >= c.
template <int NT = 256>
__device__ __forceinline__ void lds_sw_to_global(const double* S, const TileRegs* add, double* M, int64_t ld,
                                                 int64_t r0, int64_t c0, int64_t cols_valid, bool lower_only) {
#pragma unroll
  for (int q = 0; q < T64 * T64 / NT; ++q) {
    const int idx = threadIdx.x + NT * q, r = idx % T64, c = idx / T64;
    const double v = S[sw64(r, c)] + (add ? add->v[q] : 0.0);
    if (c < cols_valid && (!lower_only || r >= c)) st_c(&M[(r0 + r) + (c0 + c) * ld], v);
  }
}

// Final tiles L_ik (i > k) are also written once, tile-major, to a buffer
// that nothing reads before its producer has published the tile: those reads
// can go through the caches (no stale line can exist), unlike the tiles of G,
// which change while the kernel runs.
__device__ __forceinline__ int64_t lt_off(int i, int k) {
  return ((int64_t)i * (i - 1) / 2 + k) * (T64 * T64);
}
__device__ __forceinline__ void ltile_load(const CholArgs& a, int i, int k, TileRegs& t) {
  if (a.Lt) {
    const gdouble* p = gp(a.Lt) + lt_off(i, k);
#pragma unroll
    for (int q = 0; q < 16; ++q) t.v[q] = p[threadIdx.x + 256 * q];
  } else {
    tile_load(a.G, a.ld, (int64_t)i * T64, (int64_t)k * T64, t);
  }
}

// X Linv^T for a 64 x 64 tile X (As[c * 64 + r] = X[r][c]) and the inverse of
// a diagonal tile (Bs[c * 64 + r] = Linv[r][c]).  Linv is lower triangular,
// so output columns 16 f.. need only the first 16 (f + 1) contraction
// indices.  The product is formed transposed: wave w computes rows 16 w.. of
// the four 16-column fragments, acc4[f][v] being element
// (16 w + (lane & 15), 16 f + (lane >> 4) + 4 v), so that 16 lanes hold 16
// consecutive rows of a column (coalesced column-major stores, and
// conflict-free LDS stores into a column-major tile).
__device__ __forceinline__ void mul_linv_t(const double* As, const double* Bs, d4 acc4[4]) {
  const int l = lane_id(), w = __builtin_amdgcn_readfirstlane(wave_id());
#pragma unroll
  for (int f = 0; f < 4; ++f) acc4[f] = d4{0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int kk = 0; kk < T64; kk += 4) {
    const double xv = As[(kk + (l >> 4)) * T64 + 16 * w + (l & 15)];
#pragma unroll
    for (int f = kk / 16; f < 4; ++f)
      acc4[f] = mfma_f64(Bs[(kk + (l >> 4)) * T64 + 16 * f + (l & 15)], xv, acc4[f]);
  }
}
__device__ __forceinline__ double fr_a(const double* M, int ld, int r0, int c0, int kk) {
  const int l = lane_id();
  return M[(r0 + (l & 15)) * ld + c0 + kk + (l >> 4)];
}
__device__ __forceinline__ double fr_b(const double* M, int ld, int r0, int c0, int kk) {
  const int l = lane_id();
  return M[(r0 + kk + (l >> 4)) * ld + c0 + (l & 15)];
}
__device__ __forceinline__ void fr_store(double* M, int ld, int r0, int c0, const d4& acc) {
  const int l = lane_id();
#pragma unroll
  for (int v = 0; v < 4; ++v) M[(r0 + (l >> 4) + 4 * v) * ld + c0 + (l & 15)] = acc[v];
}
__device__ __forceinline__ d4 fr_load(const double* M, int ld, int r0, int c0) {
  const int l = lane_id();
  d4 acc;
#pragma unroll
  for (int v = 0; v < 4; ++v) acc[v] = M[(r0 + (l >> 4) + 4 * v) * ld + c0 + (l & 15)];
  return acc;
}

// Broadcast of lane l of each row of 16 lanes to the whole row (DPP
// row_newbcast: one VALU move, no scalar round trip).  `l` must fold to a
// constant after unrolling.
__device__ __forceinline__ double bcast16(double v, int l) {
#define PC_BC(n) case n: return __builtin_amdgcn_mov_dpp(v, 0x150 + n, 0xf, 0xf, false);
  switch (l) {
    PC_BC(0) PC_BC(1) PC_BC(2) PC_BC(3) PC_BC(4) PC_BC(5) PC_BC(6) PC_BC(7)
    PC_BC(8) PC_BC(9) PC_BC(10) PC_BC(11) PC_BC(12) PC_BC(13) PC_BC(14)
    default: return __builtin_amdgcn_mov_dpp(v, 0x15f, 0xf, 0xf, false);
  }
#undef PC_BC
}

// Blocks of the inverse Y of the 64 x 64 factor in A, by one wave each:
// Y_pp = X_pp (from the panel sweeps) and, for p > q,
//     Y_pq = -X_pp S_pq,   S_pq = L_pq X_qq + sum_{q<m<p} L_pm Y_mq.
// Y blocks (p > q) are kept transposed in the upper triangle of A (rows
// 16q.., columns 16p..), which the factor never touches.  inv_sum adds the
// terms m0 <= m < m1 of S_pq (m = q is L_pq X_qq) to s4; inv_finish forms
// Y_pq from S_pq through the wave's 16 x 16 scratch Sw.
__device__ __forceinline__ d4 inv_sum(const double* A, const double* X, int p, int q, int m0, int m1, d4 s4) {
  // each block's eight operands are read before its four products
  double av[4], bv[4];
  if (m0 == q) {
    // B[k][n] = X_qq[k][n]
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      av[u] = fr_a(A, LDP, 16 * p, 16 * q, 4 * u);
      bv[u] = fr_b(X + q * 256, 16, 0, 0, 4 * u);
    }
    __builtin_amdgcn_sched_barrier(0);    // keep the reads ahead of the products
#pragma unroll
    for (int u = 0; u < 4; ++u) s4 = mfma_f64(av[u], bv[u], s4);
    ++m0;
  }
  // B[k][n] = Y_mq[k][n] = A[16q + n][16m + k]
  for (int m = m0; m < m1; ++m) {
#pragma unroll
    for (int u = 0; u < 4; ++u) {
      av[u] = fr_a(A, LDP, 16 * p, 16 * m, 4 * u);
      bv[u] = fr_a(A, LDP, 16 * q, 16 * m, 4 * u);
    }
    __builtin_amdgcn_sched_barrier(0);
#pragma unroll
    for (int u = 0; u < 4; ++u) s4 = mfma_f64(av[u], bv[u], s4);
  }
  return s4;
}
__device__ __forceinline__ void inv_finish(double* A, const double* X, double* Sw, int p, int q, const d4& s4) {
  fr_store(Sw, 16, 0, 0, s4);
  double av[4], bv[4];
#pragma unroll
  for (int u = 0; u < 4; ++u) {
    av[u] = -fr_a(X + p * 256, 16, 0, 0, 4 * u);
    bv[u] = fr_b(Sw, 16, 0, 0, 4 * u);
  }
  __builtin_amdgcn_sched_barrier(0);
  d4 y4 = {0.0, 0.0, 0.0, 0.0};
#pragma unroll
  for (int u = 0; u < 4; ++u) y4 = mfma_f64(av[u], bv[u], y4);
  const int l = lane_id();
#pragma unroll
  for (int v = 0; v < 4; ++v) A[(16 * q + (l & 15)) * LDP + 16 * p + (l >> 4) + 4 * v] = y4[v];
}
__device__ __forceinline__ void inv_offdiag_block(double* A, const double* X, double* Sw, int p, int q) {
  inv_finish(A, X, Sw, p, q, inv_sum(A, X, p, q, q, p, d4{0.0, 0.0, 0.0, 0.0}));
}

// Pivot threshold of column 64 k + t (t < 64) of the tile, from the
// diagonal of G before the factorization (see the pivot test above).
__device__ __forceinline__ double pivot_threshold(const CholArgs& a, int k) {
  const int t = threadIdx.x;
  return t < T64 ? gp(a.diag0)[(int64_t)k * T64 + t] * (64.0 * (double)a.KM * 1.1102230246251565e-16) : 0.0;
}

// Diagonal tile, blocked by 16.  For each 16-column panel one wave factors
// the whole column panel (rows c..63) right-looking, column by column: every
// row of 16 lanes holds a copy of the 16 x 16 diagonal block (lane r: row r)
// and up to 16 rows of the panel below it, so the broadcasts of L_qj that
// the updates need stay inside a row (DPP) and the panel is solved in the
// same sweep.  The trailing lower part is then updated with MFMA.
// The lanes of the sweep that hold no panel row (always the last row of 16
// lanes) sweep rows of the identity instead, which gives rows of
// L_pp^{-T}: the inverse X_pp of the diagonal block comes out of the same
// instructions.  The off-diagonal blocks of the inverse are formed by the
// waves that the sweeps leave idle: Y_10 with panel 2; Y_21, Y_20 and the
// parts of S_32, S_31, S_30 that do not need them with panel 3; after it
// only the last terms and the products with X_33.
// LDS: A (64 x 65), X (4 x 16 x 16), sweep scratch (64 x 16) and pivot
// thresholds (64), then the inverse's scratch (4 x 256).
// Factor the 64 x 64 lower triangle held in A (LDS, row-major, stride LDP)
// and form its inverse; publish the inverse (Linv) and the factor of tile
// (k,k).  If pend_flag is set, the flag is published after the first panel
// (the caller's coherent stores have completed by then).
__device__ __noinline__ void potrf_factor(const CholArgs& a, int k, double* A, double* X, double* Sc, int* sh,
                                         int* pend_flag, int pend_val, double thr_t) {
  const int t = threadIdx.x, lane = lane_id(), w = wave_id();
  const int64_t k0 = (int64_t)k * T64;
  double* Sy = Sc + 1024 + T64;          // inverse scratch, 256 per wave
  if (t == 0) sh[1] = -1;
  // pivot thresholds of the 64 columns (fetched by the caller)
  if (t < T64) Sc[1024 + t] = thr_t;
  __syncthreads();
  d4 sacc = {0.0, 0.0, 0.0, 0.0};          // this wave's part of S_3q, q = 3 - w
  for (int p = 0; p < 4; ++p) {
    const int c = 16 * p;
    if (w == 0) {
      // lane 16 s + r: diagonal-block row c + r (dg) and panel row
      // c + 16 + 16 s + r (pr) when that row exists.  Branch-free: the
      // pivots are checked once at the end.
      const int r = lane & 15, s = lane >> 4;
      const int prow = c + 16 + 16 * s + r;
      const bool has = prow < T64;
      const int lrow = has ? prow : c + r;      // rows past the tile sweep a row of the identity
      double dg[16], pr[16];
#pragma unroll
      for (int q = 0; q < 16; ++q) dg[q] = A[(c + r) * LDP + c + q];
#pragma unroll
      for (int q = 0; q < 16; ++q) pr[q] = A[lrow * LDP + c + q];
      // identity rows: 0 * v keeps the loads above unconditional (a select
      // that dropped v would have them issued one by one under a branch)
#pragma unroll
      for (int q = 0; q < 16; ++q) pr[q] = has ? pr[q] : fma(0.0, pr[q], q == r ? 1.0 : 0.0);
      int fail = 16;                      // first failing pivot of this panel
#pragma unroll
      for (int j = 0; j < 16; ++j) {
        const double piv = bcast16(dg[j], j);
        const double thr = Sc[1024 + c + j];
        if (!(piv > thr && isfinite(piv))) fail = fail < j ? fail : j;
        // 1/sqrt(piv): the hardware estimate and two Newton steps
        // y <- y + y (1 - piv y^2) / 2 (each squares the relative error: the
        // estimate's ~1e-7 becomes ~1e-14, then rounding level, so the column
        // scaling adds nothing to the factor's own rounding error; a failing
        // pivot is caught above and its value never used)
        const double y0 = __builtin_amdgcn_rsq(piv);
        const double y1 = fma(0.5 * y0, fma(-piv * y0, y0, 1.0), y0);
        const double inv = fma(0.5 * y1, fma(-piv * y1, y1, 1.0), y1);
        dg[j] *= inv;                     // lanes r > j: L_rj; lane j: piv / sqrt(piv) = L_jj
        pr[j] *= inv;
#pragma unroll
        for (int q = j + 1; q < 16; ++q) {
          const double lqj = bcast16(dg[j], q);
          dg[q] = fma(-dg[j], lqj, dg[q]);
          pr[q] = fma(-pr[j], lqj, pr[q]);
        }
        // finish the panel rows' updates in this step (the instruction
        // selector would otherwise defer them and keep every broadcast live)
#pragma unroll
        for (int q = j; q < 16; ++q) asm volatile("" : "+v"(pr[q]));
      }
      // Stores are unconditional (lanes without a panel row write row r of
      // L_pp^{-T} to column r of X_pp from the last row of lanes, and to the
      // sweep scratch from the others), so no part of the sweep is sunk into
      // a branch.  Every row of 16 lanes writes the same diagonal block.
      double* pdst = has ? A + prow * LDP + c : (s == 3 ? X + p * 256 + r : Sc + lane * 16);
      const int pst = (!has && s == 3) ? 16 : 1;
#pragma unroll
      for (int q = 0; q < 16; ++q) A[(c + r) * LDP + c + q] = (q <= r) ? dg[q] : 0.0;
#pragma unroll
      for (int q = 0; q < 16; ++q) pdst[q * pst] = pr[q];
      if (fail < 16 && lane == 0) sh[1] = (int)(a.col_off + k0 + c + fail);
    } else if (p == 2) {
      if (w == 2) inv_offdiag_block(A, X, Sy + 2 * 256, 1, 0);
    } else if (p == 3) {
      if (w == 1) {
        sacc = inv_sum(A, X, 3, 2, 2, 3, sacc);                  // S_32 = L_32 X_22
      } else if (w == 2) {
        inv_offdiag_block(A, X, Sy + 2 * 256, 2, 1);             // Y_21
        sacc = inv_sum(A, X, 3, 1, 1, 2, sacc);                  // L_31 X_11
      } else {
        inv_offdiag_block(A, X, Sy + 3 * 256, 2, 0);             // Y_20
        sacc = inv_sum(A, X, 3, 0, 0, 2, sacc);                  // L_30 X_00 + L_31 Y_10
      }
    }
    __syncthreads();
    if (sh[1] >= 0) {
      if (t == 0) st_release(a.info, sh[1]);
      return;
    }
    const int nf = 3 - p;                 // 16-row fragments below the diagonal block
    // trailing lower fragments (fi >= fj) of A[c+16:, c+16:] -= P P^T
    for (int f = w; f < nf * (nf + 1) / 2; f += 4) {
      int fi = 0;
      while ((fi + 1) * (fi + 2) / 2 <= f) ++fi;
      const int fj = f - fi * (fi + 1) / 2;
      const int ri = c + 16 + 16 * fi, rj = c + 16 + 16 * fj;
      d4 acc = fr_load(A, LDP, ri, rj);
#pragma unroll
      for (int kk = 0; kk < 16; kk += 4)
        acc = mfma_f64(-fr_a(A, LDP, ri, c, kk), fr_a(A, LDP, rj, c, kk), acc);
      fr_store(A, LDP, ri, rj, acc);
    }
    if (p == 0 && pend_flag) __builtin_amdgcn_s_waitcnt(0);
    if (p < 3) __syncthreads();           // the last panel has no trailing part
    if (p == 0 && pend_flag && t == 0) st_release(pend_flag, pend_val);
  }
  // the rest of block row 3 of the inverse: the terms with Y_21 and Y_20,
  // then the products with X_33 (from the last sweep)
  if (w >= 1) {
    if (w >= 2) sacc = inv_sum(A, X, 3, 3 - w, 2, 3, sacc);     // + L_32 Y_21, + L_32 Y_20
    inv_finish(A, X, Sy + w * 256, 3, 3 - w, sacc);
  }
  __syncthreads();
  // the inverse first (the next panel's solves wait for it), then the flag,
  // then the factor tile itself (read only by later kernels)
  double* Lb = a.Linv + (int64_t)k * T64 * T64;
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int idx = t + 256 * u, r = idx % T64, c = idx / T64;
    const int pr = r >> 4, pc = c >> 4;
    double yv;
    if (pr == pc) yv = X[pr * 256 + (r & 15) * 16 + (c & 15)];
    else if (pr > pc) yv = A[c * LDP + r];          // transposed storage of Y_{pr,pc}
    else yv = 0.0;
    st_c(&Lb[r + c * T64], yv);
  }
  publish(&a.state[(int64_t)k * a.T + k], k + 1);
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int idx = t + 256 * u, r = idx % T64, c = idx / T64;
    if (r >= c) gp(a.G)[(k0 + r) + (k0 + c) * a.ld] = A[r * LDP + c];
  }
}

// DIAG(0): the first diagonal tile as it is.
__device__ __noinline__ void diag0_task(const CholArgs& a, double* A, double* X, double* Sc, int* sh) {
  const int t = threadIdx.x;
  const double thr = pivot_threshold(a, 0);
  double v[16];
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int idx = t + 256 * q, r = idx % T64, c = idx / T64;
    v[q] = (r >= c) ? ld_c(&a.G[r + c * a.ld]) : 0.0;
  }
#pragma unroll
  for (int q = 0; q < 16; ++q) {
    const int idx = t + 256 * q, r = idx % T64, c = idx / T64;
    A[r * LDP + c] = v[q];
  }
  potrf_factor(a, 0, A, X, Sc, sh, nullptr, 0, thr);
}

// DIAG(k), k >= 1 (see the top of the file).  Returns false if the DAG was
// abandoned while waiting.  LDS: As, Bs (two 64 x 64 operands) and then the
// factorization workspace over the same buffer.
__device__ __noinline__ bool diag_task(const CholArgs& a, int k, double* buf, int* sh) {
  double* As = buf;
  double* Bs = buf + T64 * T64;
  const int T = a.T;
  const int64_t k0 = (int64_t)k * T64, p0 = k0 - T64;     // tile rows k and k-1
  int* st = a.state;
  const double thr = pivot_threshold(a, k);
  // operands that are ready before the previous diagonal step ends
  if (k >= 3 && !wait_ge(&st[k * T + k - 1], k - 2, a.info, a.err, &sh[2])) return false;
  if (k >= 2) {
    if (!wait_ge(&st[k * T + k - 2], k - 1, a.info, a.err, &sh[2])) return false;
    if (!wait_ge(&st[(k - 1) * T + k - 2], k - 1, a.info, a.err, &sh[2])) return false;
  }
  TileRegs tp;                                          // G_{k,k-1}
  tile_load(a.G, a.ld, k0, p0, tp);
  if (k >= 2) {                                         // its last update, from column k-2
    TileF64<T64, T64, 2, 2> upd;
    TileRegs ta, tb;
    ltile_load(a, k, k - 2, ta);                        // L_{k,k-2}
    ltile_load(a, k - 1, k - 2, tb);                    // L_{k-1,k-2}
    tile_store_lds(ta, As, -1.0);
    tile_store_lds(tb, Bs, 1.0);
    __syncthreads();
    upd.zero();
    upd.template mma<T64, T64, T64>(Bs, As);          // transposed: accumulator (c, r)
    __syncthreads();
    upd.for_each([&](int c, int r, double v) { As[c * T64 + r] = v; });
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) As[threadIdx.x + 256 * q] += tp.v[q];
  } else {
    tile_store_lds(tp, As, 1.0);
  }
  if (k >= 2 && !wait_ge(&st[k * T + k], k - 1, a.info, a.err, &sh[2])) return false;
  TileRegs td;                                          // G_kk, updated through column k-2
  tile_load(a.G, a.ld, k0, k0, td);
  // the previous diagonal step's inverse
  if (!wait_ge(&st[(k - 1) * T + k - 1], k, a.info, a.err, &sh[2])) return false;
  {
    TileRegs tl;
    tile_load(a.Linv + (int64_t)(k - 1) * T64 * T64, T64, 0, 0, tl);
    tile_store_lds(tl, Bs, 1.0);
  }
  __syncthreads();
  {
    // L_{k,k-1} = G' Linv_{k-1}^T, out from the accumulators (published
    // later) and into As as a column-major tile for the SYRK
    const int l = lane_id(), w = __builtin_amdgcn_readfirstlane(wave_id());
    d4 acc4[4];
    mul_linv_t(As, Bs, acc4);
    double* lt = a.Lt ? a.Lt + lt_off(k, k - 1) : nullptr;
#pragma unroll
    for (int f = 0; f < 4; ++f)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * w + (l & 15), c = 16 * f + (l >> 4) + 4 * v;
        st_c(&a.G[(k0 + r) + (p0 + c) * a.ld], acc4[f][v]);
        if (lt) st_c(&lt[c * T64 + r], acc4[f][v]);
      }
    __syncthreads();
#pragma unroll
    for (int f = 0; f < 4; ++f)
#pragma unroll
      for (int v = 0; v < 4; ++v) As[(16 * f + (l >> 4) + 4 * v) * T64 + 16 * w + (l & 15)] = acc4[f][v];
  }
  __syncthreads();
  double* A = buf;
  {
    // L_{k,k-1} L_{k,k-1}^T on the ten lower 16 x 16 fragments, three or two
    // per wave: w0 (0,0) (3,0) (3,1), w1 (1,0) (1,1) (3,2), w2 (2,0) (2,1),
    // w3 (2,2) (3,3).  w2 and w3 repeat their first fragment as the third
    // (not stored), so the loop has no branch and the operands of the next
    // step are read from LDS while the products of this one run.
    const int l = lane_id(), w = __builtin_amdgcn_readfirstlane(wave_id());
    const int nf = w < 2 ? 3 : 2;
    int fi[3], fj[3];
    fi[0] = w < 2 ? w : 2;  fj[0] = w == 3 ? 2 : (w == 1 ? 0 : 0);
    fi[1] = w == 0 ? 3 : (w == 1 ? 1 : (w == 2 ? 2 : 3));  fj[1] = w == 0 ? 0 : (w == 1 ? 1 : (w == 2 ? 1 : 3));
    fi[2] = w < 2 ? 3 : fi[0];  fj[2] = w == 0 ? 1 : (w == 1 ? 2 : fj[0]);
    d4 sy[3];
#pragma unroll
    for (int u = 0; u < 3; ++u) sy[u] = d4{0.0, 0.0, 0.0, 0.0};
    double ca[3], cb[3];
    auto operands = [&](int kk, double* oa, double* ob) {
      const double* col = As + (kk + (l >> 4)) * T64 + (l & 15);
#pragma unroll
      for (int u = 0; u < 3; ++u) {
        oa[u] = col[16 * fi[u]];
        ob[u] = col[16 * fj[u]];
      }
    };
    operands(0, ca, cb);
#pragma unroll
    for (int kk = 0; kk < T64; kk += 4) {
      double na[3], nb[3];
      if (kk + 4 < T64) operands(kk + 4, na, nb);
#pragma unroll
      for (int u = 0; u < 3; ++u) sy[u] = mfma_f64(ca[u], cb[u], sy[u]);
      if (kk + 4 < T64) {
#pragma unroll
        for (int u = 0; u < 3; ++u) { ca[u] = na[u]; cb[u] = nb[u]; }
      }
    }
    __syncthreads();
#pragma unroll
    for (int u = 0; u < 3; ++u)
      if (u < nf)
#pragma unroll
        for (int v = 0; v < 4; ++v) A[(16 * fi[u] + (l >> 4) + 4 * v) * LDP + 16 * fj[u] + (l & 15)] = -sy[u][v];
  }
  __syncthreads();
  {
    // all sixteen reads first, then the writes (no LDS round trip per element)
    double cur[16];
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int idx = threadIdx.x + 256 * q, r = idx % T64, c = idx / T64;
      cur[q] = A[r * LDP + c];
    }
#pragma unroll
    for (int q = 0; q < 16; ++q) {
      const int idx = threadIdx.x + 256 * q, r = idx % T64, c = idx / T64;
      A[r * LDP + c] = (r >= c) ? cur[q] + td.v[q] : 0.0;
    }
  }
  potrf_factor(a, k, A, buf + T64 * LDP, buf + T64 * LDP + 1024, sh, &st[k * T + k - 1], k, thr);
  return true;
}

// GEMM(i,j,k) with its group: G_ij -= L_i,kk L_j,kk^T for kk = kb..k.  Each
// update is rounded into the tile on its own, in column order, so the result
// is the same for every group size.
__device__ __forceinline__ void gemm_task(const CholArgs& a, int i, int j, int kb, int k, double* As, double* Bs) {
  const int64_t i0 = (int64_t)i * T64, j0 = (int64_t)j * T64;
  // The product is formed transposed, acc(m, n) = -(L_jk L_ik^T)(m, n), so
  // that a lane's accumulator entries run down the columns of G_ij: the tile
  // is read in the accumulator layout and written back from it directly,
  // each wave instruction touching four 128-byte column segments.
  TileF64<T64, T64, 2, 2> acc;
  TileRegs ta, tb;
  // operands first (loads complete in order), G_ij arrives during the product
  ltile_load(a, i, kb, ta);                           // L_i,kb
  ltile_load(a, j, kb, tb);                           // L_j,kb
  const int lane = lane_id(), w = wave_id(), wm = w / 2, wn = w % 2;
  double cr[2][2][4];                                 // G_ij(n, m) at accumulator (m, n)
#pragma unroll
  for (int fi = 0; fi < 2; ++fi)
#pragma unroll
    for (int fj = 0; fj < 2; ++fj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = wm * 32 + fi * 16 + (lane >> 4) + 4 * v, n = wn * 32 + fj * 16 + (lane & 15);
        cr[fi][fj][v] = ld_c(&a.G[(i0 + n) + (j0 + m) * a.ld]);
      }
  for (int kk = kb; kk <= k; ++kk) {
    if (kk > kb) __syncthreads();                     // the previous product has read As, Bs
    tile_store_lds(tb, As, -1.0);                     // As[c][m] = -L_j,kk[m][c]
    tile_store_lds(ta, Bs, 1.0);                      // Bs[c][n] = L_i,kk[n][c]
    __syncthreads();
    if (kk < k) {                                     // next operands, in flight during the product
      ltile_load(a, i, kk + 1, ta);
      ltile_load(a, j, kk + 1, tb);
    }
    acc.zero();
    acc.template mma<T64, T64, T64>(As, Bs);
#pragma unroll
    for (int fi = 0; fi < 2; ++fi)
#pragma unroll
      for (int fj = 0; fj < 2; ++fj)
#pragma unroll
        for (int v = 0; v < 4; ++v) cr[fi][fj][v] += acc.acc[fi][fj][v];
  }
#pragma unroll
  for (int fi = 0; fi < 2; ++fi)
#pragma unroll
    for (int fj = 0; fj < 2; ++fj)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int m = wm * 32 + fi * 16 + (lane >> 4) + 4 * v, n = wn * 32 + fj * 16 + (lane & 15);
        if (i != j || n >= m) st_c(&a.G[(i0 + n) + (j0 + m) * a.ld], cr[fi][fj][v]);
      }
}

// TRSM(i,k): for k >= 1 the tile's last update from column k-1 comes first
// (its operands are final once TRSM(i,k-1) and TRSM(k,k-1) are done), then the
// task waits for POTRF(k) and multiplies by L_kk^{-T}.  Returns false if the
// DAG was abandoned while waiting.
__device__ __noinline__ bool trsm_task(const CholArgs& a, int i, int k, double* As, double* Bs, int* sh) {
  const int64_t i0 = (int64_t)i * T64, k0 = (int64_t)k * T64;
  TileRegs tc;
  if (k >= 1) {
    TileF64<T64, T64, 2, 2> upd;
    TileRegs ta, tb;
    ltile_load(a, i, k - 1, ta);                      // L_{i,k-1}
    ltile_load(a, k, k - 1, tb);                      // L_{k,k-1}
    tile_load(a.G, a.ld, i0, k0, tc);                 // G_ik (arrives while the product runs)
    tile_store_lds(ta, As, -1.0);
    tile_store_lds(tb, Bs, 1.0);
    __syncthreads();
    upd.zero();
    upd.template mma<T64, T64, T64>(Bs, As);          // -L_{i,k-1} L_{k,k-1}^T, transposed
    __syncthreads();
    upd.for_each([&](int c, int r, double v) { As[c * T64 + r] = v; });
    __syncthreads();
#pragma unroll
    for (int q = 0; q < 16; ++q) As[threadIdx.x + 256 * q] += tc.v[q];   // As[c][r] = updated G_ik
  } else {
    tile_load(a.G, a.ld, i0, k0, tc);                 // G_ik
    tile_store_lds(tc, As, 1.0);                      // As[c][r] = G[i0+r][k0+c]
  }
  if (!wait_ge(&a.state[(int64_t)k * a.T + k], k + 1, a.info, a.err, &sh[2])) return false;
  const double* Lb = a.Linv + (int64_t)k * T64 * T64;
  TileRegs tb;
  tile_load(Lb, T64, 0, 0, tb);                       // Bs[c][r] = Linv[r][c]
  tile_store_lds(tb, Bs, 1.0);
  __syncthreads();
  {
    // L_ik = G'_ik Linv_k^T, out straight from the accumulators
    const int l = lane_id(), w = __builtin_amdgcn_readfirstlane(wave_id());
    d4 acc4[4];
    mul_linv_t(As, Bs, acc4);
    double* lt = a.Lt ? a.Lt + lt_off(i, k) : nullptr;
#pragma unroll
    for (int f = 0; f < 4; ++f)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int r = 16 * w + (l & 15), c = 16 * f + (l >> 4) + 4 * v;
        st_c(&a.G[(i0 + r) + (k0 + c) * a.ld], acc4[f][v]);
        if (lt) st_c(&lt[c * T64 + r], acc4[f][v]);
      }
  }
  return true;
}

// A run of consecutive global task indices that belong to one instance of a
// batch: global task gstart + u is that instance's task lstart + u.
struct DagSeg { int64_t gstart, lstart; int inst, pad; };

__device__ __forceinline__ int find_seg(const DagSeg* segs, int n, int64_t g) {
  int lo = 0, hi = n - 1;                  // largest s with segs[s].gstart <= g
  while (lo < hi) {
    const int mid = (lo + hi + 1) / 2;
    if (segs[mid].gstart <= g) lo = mid; else hi = mid - 1;
  }
  return lo;
}

// One instance (inst == null: `one`), or a batch whose instances' task lists
// are interleaved by the segment table.
struct CholBatch {
  const CholArgs* inst; const DagSeg* segs; int nsegs;
  CholArgs one;
  int64_t ntasks; int* head; int* err;
};

__global__ __launch_bounds__(256, 2) void chol_dag_kernel(CholBatch b) {
  // DIAG: tile (64 x 65) + X (4 x 256) + sweep scratch and thresholds
  // (1024 + 64) + inverse scratch (4 x 256) = 7296 doubles;
  // TRSM/GEMM: two 64 x 64 operands = 8192 doubles
  __shared__ double buf[2 * T64 * T64];
  __shared__ int sh[4];
  __shared__ CholArgs sa;
  double* As = buf;
  double* Bs = buf + T64 * T64;
  // Final tiles are read through the caches: drop whatever lines this
  // compute unit's caches still hold from before the launch.
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  for (;;) {
    if (threadIdx.x == 0) sh[0] = atomicAdd(b.head, 1);
    __syncthreads();
    // the task index is the same for the whole workgroup: keep it (and all
    // that is derived from it) in scalar registers
    const int64_t g = __builtin_amdgcn_readfirstlane(sh[0]);
    __syncthreads();
    if (g >= b.ntasks) break;
    // this task's instance arguments, shared through LDS (a private copy
    // would live in scratch memory, since the task functions take a reference)
    int64_t t;
    if (b.inst) {
      const DagSeg sg = b.segs[find_seg(b.segs, b.nsegs, g)];
      if (threadIdx.x == 0) sa = b.inst[sg.inst];
      t = sg.lstart + (g - sg.gstart);
    } else {
      if (threadIdx.x == 0) sa = b.one;
      t = g;
    }
    if (threadIdx.x == 0) sa.err = b.err;
    __syncthreads();
    const CholArgs& a = sa;
    const int T = a.T;
    const TaskDesc d = decode_task(t, T, a.offs, a.grp);
    int* st = a.state;
    if (d.type == 0) {
      // the diagonal step is the critical path: its waves get the highest
      // issue priority against the update tasks sharing the CU
      __builtin_amdgcn_s_setprio(3);
      if (d.k == 0) diag0_task(a, buf, buf + T64 * LDP, buf + T64 * LDP + 1024, sh);
      else diag_task(a, d.k, buf, sh);
      __builtin_amdgcn_s_setprio(0);
    } else if (d.type == 1) {
      const int i = d.i, k = d.k;
      if (k >= 1) {
        if (!wait_ge(&st[i * T + k - 1], k, a.info, a.err, &sh[2])) continue;
        if (!wait_ge(&st[k * T + k - 1], k, a.info, a.err, &sh[2])) continue;
        if (!wait_ge(&st[i * T + k], k - 1, a.info, a.err, &sh[2])) continue;
      }
      __builtin_amdgcn_s_setprio(2);
      const bool done = trsm_task(a, i, k, As, Bs, sh);
      __builtin_amdgcn_s_setprio(0);
      if (!done) continue;
      publish(&st[i * T + k], k + 1);
    } else {
      // L_i,kk is final for every kk <= k once L_ik is (each TRSM waits for
      // the one before it in its tile row)
      const int kb = d.k - d.k % a.grp;
      if (!wait_ge(&st[d.i * T + d.k], d.k + 1, a.info, a.err, &sh[2])) continue;
      if (d.j != d.i && !wait_ge(&st[d.j * T + d.k], d.k + 1, a.info, a.err, &sh[2])) continue;
      if (!wait_ge(&st[d.i * T + d.j], kb, a.info, a.err, &sh[2])) continue;
      gemm_task(a, d.i, d.j, kb, d.k, As, Bs);
      publish(&st[d.i * T + d.j], d.k + 1);
    }
    __syncthreads();
  }
}

// ------------------------------------------------------------------ solves
// Forward: task (i, rt) in order i ascending: acc = B_i - sum_{j<i} L_ij Z_j,
// Z_i = Linv_i acc.  Backward: i descending: acc = Z_i - sum_{j>i} L_ji^T Y_j,
// Y_i = Linv_i^T acc.  flag[i * nrt + rt] = 1 once the block row is written.
// With the folded products (Mf, Mb) the update from the previous block row
// comes last and after the multiplication by the inverse:
//   Z_i = Linv_i (B_i - sum_{j<i-1} L_ij Z_j) - Mf_i Z_{i-1},   Mf_i = Linv_i L_{i,i-1}
//   Y_i = Linv_i^T (Z_i - sum_{j>i+1} L_ji^T Y_j) - Mb_i Y_{i+1}, Mb_i = Linv_i^T L_{i+1,i}^T
// so that the chain from one block row to the next crosses one product.
// With the second folds (Mf2_i = Linv_i L_{i,i-2}, Mb2_i = Linv_i^T L_{i+2,i}^T)
// the block row before that is folded the same way, just before the previous
// one, so that the rest of the task (the older block rows and the product
// with the inverse) runs one step ahead of the chain.
struct SolveArgs {
  const double* G; int64_t ld; int T;
  const double* Linv;
  const double* Mf; const double* Mb;   // folded products (column-major, 64 x 64 per block row) or null
  const double* Mf2; const double* Mb2; // second folds (same layout) or null
  // forward pass run while the factorization runs: the tile states of the
  // factorization (T x T, row-major) and its final tiles; L blocks and the
  // inverses are read once their tiles are published
  const int* cstate; int cT; const double* Lt;
  const double* In; int64_t ldIn;
  double* Out; int64_t ldOut;
  int64_t R; const int64_t* Rp;   // right-hand sides: *Rp when Rp is set, else R
  int nrt;                         // 64-column tiles per block row (task stride, >= ceil(R / 64))
  int* flags; const int* info;
  const int* skip;
};

struct SolveBatch {
  const SolveArgs* inst; const DagSeg* segs; int nsegs;
  SolveArgs one;
  int64_t ntasks; int* head; int* err;
  int backward;
  int swap_io;      // batch descriptors hold the forward pass: swap In/Out for the backward one
};

// The number of leading tiles L_i0, L_i1, .. of tile row i that the running
// factorization has published, at least `need` + 1 once this returns true
// (tiles of a row become final in column order).  Wave 0 reads up to 64
// states per round; the abandon conditions are read every 8th round.
__device__ __forceinline__ bool row_ready(const int* st_row, int i, int need, int* ready, const int* info, int* err,
                                          int* sh) {
  if (threadIdx.x < 64) {
    const int lane = threadIdx.x;
    int have = *ready, ok = 1;
    long long spins = 0;
    while (have <= need) {
      const int jj = have + lane;
      const bool fin = jj >= i || ld_acquire(&st_row[jj]) >= jj + 1;
      const unsigned long long notfin = __ballot(!fin);
      have += notfin ? __builtin_ctzll(notfin) : 64;
      if (have > need) break;
      if ((++spins & 7) == 0 && (ld_acquire(info) >= 0 || ld_acquire(err) != 0)) { ok = 0; break; }
      if (spins > kSpinLimit) { if (lane == 0) atomicOr((int*)gp(err), 1); ok = 0; break; }
      __builtin_amdgcn_s_sleep(1);
    }
    if (lane == 0) { *sh = ok; *ready = have; }
  }
  __syncthreads();
  const bool ok = *sh != 0;
  __syncthreads();
  return ok;
}

// acc += (sa A) B for 64 x 64 operands in LDS, A[k][m] and B[k][n] in the
// plain layout (k * 64 + m) or, with XA / XB, in the row-XOR layout.
template <bool XA, bool XB, int WM = 2, int WN = 2>
__device__ __forceinline__ void mma64_lds(TileF64<T64, T64, WM, WN>& acc, const double* As, const double* Bs,
                                          double sa) {
  using Tile = TileF64<T64, T64, WM, WN>;
  constexpr int FM = Tile::FM, FN = Tile::FN;
  const int lane = lane_id(), w = wave_id();
  const int wm = w / WN, wn = w % WN, rr = lane & 15, kq = lane >> 4;
#pragma unroll 4
  for (int kk = 0; kk < T64; kk += 4) {
    const int k = kk + kq;
    double av[FM], bv[FN];
#pragma unroll
    for (int f = 0; f < FM; ++f) {
      const int m = wm * Tile::TM + f * 16 + rr;
      av[f] = sa * As[XA ? xs64(k, m) : k * T64 + m];
    }
#pragma unroll
    for (int f = 0; f < FN; ++f) {
      const int n = wn * Tile::TN + f * 16 + rr;
      bv[f] = Bs[XB ? xs64(k, n) : k * T64 + n];
    }
#pragma unroll
    for (int fi = 0; fi < FM; ++fi)
#pragma unroll
      for (int fj = 0; fj < FN; ++fj) acc.acc[fi][fj] = mfma_f64(av[fi], bv[fj], acc.acc[fi][fj]);
  }
}

// CONC: the forward pass alongside the factorization (forward only, no
// folded products, tiles and inverses read once published); a variant of its
// own so that it needs no more registers than two waves per SIMD allow and
// shares the compute units with the factorization's workgroups.
// NW: waves per workgroup (4, or 8 to halve each wave's share of a product
// on the chain).
template <bool CONC, int NW>
__global__ __launch_bounds__(64 * NW, CONC ? 2 : 1) void solve_dag_kernel_t(SolveBatch b) {
  constexpr int NT = 64 * NW, PER = T64 * T64 / NT, WM = NW / 2;
  using Acc = TileF64<T64, T64, WM, 2>;
  __shared__ double As[T64 * T64];
  __shared__ double Bs[T64 * T64];
  __shared__ int sh[8];
  __shared__ SolveArgs sa;
  // final tiles (and inverses) of a factorization that runs alongside are
  // read through the caches once published: drop whatever lines this
  // compute unit's caches still hold from before the launch
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
  for (;;) {
    if (threadIdx.x == 0) sh[0] = atomicAdd(b.head, 1);
    __syncthreads();
    // the task index is the same for the whole workgroup: keep it (and all
    // that is derived from it) in scalar registers
    const int64_t g = __builtin_amdgcn_readfirstlane(sh[0]);
    __syncthreads();
    if (g >= b.ntasks) break;
    int64_t t;
    if (threadIdx.x == 0) {
      if (b.inst) {
        const DagSeg sg = b.segs[find_seg(b.segs, b.nsegs, g)];
        sa = b.inst[sg.inst];
        t = sg.lstart + (g - sg.gstart);
      } else {
        sa = b.one;
        t = g;
      }
      if (sa.Rp) sa.R = *sa.Rp;
      if (!CONC && b.swap_io && b.backward) {
        const double* in_ = sa.In; const int64_t ldi = sa.ldIn;
        sa.In = sa.Out; sa.ldIn = sa.ldOut;
        sa.Out = const_cast<double*>(in_); sa.ldOut = ldi;
      }
      sh[1] = (int)t;
      sh[3] = (sa.skip && *sa.skip) ? 1 : 0;
    }
    __syncthreads();
    t = __builtin_amdgcn_readfirstlane(sh[1]);
    const bool skipped = sh[3] != 0;
    const SolveArgs& a = sa;
    if (skipped) { __syncthreads(); continue; }
    const int step = (int)(t / a.nrt), rt = (int)(t % a.nrt);
    if ((int64_t)rt * T64 >= a.R) continue;            // beyond this call's right-hand sides
    const bool bwd = !CONC && b.backward;
    const int i = bwd ? a.T - 1 - step : step;
    const int64_t i0 = (int64_t)i * T64, r0 = (int64_t)rt * T64;
    Acc acc;
    tile_to_acc(a.In, a.ldIn, i0, r0, acc, a.R - r0);    // acc = In[i block, rt]
    // the diagonal block's inverse is static: it travels while the task waits
    // forward: As[k][row] = Linv[row][k]; backward: As[k][row] = Linv[k][row]
    double linv[PER];
    if (!CONC) {
      const gdouble* Lb = gp(a.Linv + (int64_t)i * T64 * T64);
#pragma unroll
      for (int u = 0; u < PER; ++u) {
        const int idx = threadIdx.x + NT * u, p = idx % T64, q = idx / T64;
        linv[u] = bwd ? Lb[q + p * T64] : Lb[idx];
      }
    }
    if (threadIdx.x == 0) sh[4] = 0;                  // leading final tiles of row i (with a.cstate)
    bool ok = true;
    const int nprev = bwd ? (a.T - 1 - i) : i;
    const double* Mfold = bwd ? a.Mb : a.Mf;
    const double* Mfold2 = bwd ? a.Mb2 : a.Mf2;
    const bool fold = !CONC && Mfold != nullptr && nprev > 0;
    const bool fold2 = fold && Mfold2 != nullptr && nprev > 1;
    const int nloop = nprev - (fold ? 1 : 0) - (fold2 ? 1 : 0);   // the folded block rows come last
    for (int s = 0; s < nloop && ok; ++s) {
      const int j = bwd ? a.T - 1 - s : s;               // producers in their own order
      const int64_t j0 = (int64_t)j * T64;
      // operand L block (row-XOR layout): forward L_ij (A[c][r] = L[i0+r][j0+c]); backward L_ji^T
      // (A[c][r] = L[j0+c][i0+r]); Out_j also row-XOR (B[p][q] = Out[j0+p][r0+q])
      if (CONC) {
        if (!row_ready(a.cstate + (int64_t)i * a.cT, i, j, &sh[4], a.info, b.err, &sh[2])) { ok = false; break; }
        const gdouble* lt = gp(a.Lt + lt_off(i, j));   // final tile, column-major
#pragma unroll
        for (int u = 0; u < PER; ++u) {
          const int idx = threadIdx.x + NT * u, p = idx % T64, q = idx / T64;
          As[xs64(q, p)] = lt[idx];                     // A[p][q] = L[i0+p][j0+q]
        }
      } else {
#pragma unroll
        for (int u = 0; u < PER; ++u) {
          const int idx = threadIdx.x + NT * u, p = idx % T64, q = idx / T64;   // p runs along a column of G
          if (!bwd) As[xs64(q, p)] = gp(a.G)[(i0 + p) + (j0 + q) * a.ld];   // A[p][q] = L[i0+p][j0+q]
          else As[xs64(p, q)] = gp(a.G)[(j0 + p) + (i0 + q) * a.ld];              // A[q][p] = L[j0+p][i0+q]
        }
      }
      if (!wait_ge(&a.flags[j * a.nrt + rt], 1, a.info, b.err, &sh[2])) { ok = false; break; }
      {
#pragma unroll
        for (int h = 0; h < 2; ++h) {
          double v[PER / 2];
#pragma unroll
          for (int u = 0; u < PER / 2; ++u) {
            const int idx = threadIdx.x + NT * (PER / 2 * h + u), p = idx % T64, q = idx / T64;  // p: row in block j, q: rhs
            v[u] = (r0 + q < a.R) ? ld_c(&a.Out[(j0 + p) + (r0 + q) * a.ldOut]) : 0.0;
          }
#pragma unroll
          for (int u = 0; u < PER / 2; ++u) {
            const int idx = threadIdx.x + NT * (PER / 2 * h + u), p = idx % T64, q = idx / T64;
            Bs[xs64(p, q)] = v[u];
          }
        }
      }
      __syncthreads();
      mma64_lds<true, true, WM, 2>(acc, As, Bs, -1.0);   // acc -= Lop * Out_j
      __syncthreads();
    }
    if (!ok) continue;
    if (CONC) {
      // the diagonal step's inverse, once published
      if (!wait_ge(&a.cstate[(int64_t)i * a.cT + i], i + 1, a.info, b.err, &sh[2])) continue;
      const double* Lb = a.Linv + (int64_t)i * T64 * T64;
#pragma unroll
      for (int u = 0; u < PER; ++u) linv[u] = ld_c(&Lb[threadIdx.x + NT * u]);
    }
    // Out_i = Linv_i (or its transpose) * acc
    acc.for_each([&](int r, int c, double v) { Bs[r * T64 + c] = v; });
#pragma unroll
    for (int u = 0; u < PER; ++u) As[threadIdx.x + NT * u] = linv[u];
    __syncthreads();
    Acc res;
    res.zero();
    mma64_lds<false, false, WM, 2>(res, As, Bs, 1.0);
    __syncthreads();
    // res -= M_i Out_j for the block row j two steps back, then the previous
    // one (As[k][row] = -M[row][k])
    bool fok = true;
#pragma unroll 1
    for (int d = fold2 ? 2 : 1; d >= 1 && fold; --d) {
      const int j = bwd ? i + d : i - d;
      const int64_t j0 = (int64_t)j * T64;
      const gdouble* Mi = gp((d == 2 ? Mfold2 : Mfold) + (int64_t)i * T64 * T64);
#pragma unroll
      for (int u = 0; u < PER; ++u) As[threadIdx.x + NT * u] = -Mi[threadIdx.x + NT * u];
      if (!wait_ge(&a.flags[j * a.nrt + rt], 1, a.info, b.err, &sh[2])) { fok = false; break; }
#pragma unroll
      for (int h = 0; h < 2; ++h) {
        double v[PER / 2];
#pragma unroll
        for (int u = 0; u < PER / 2; ++u) {
          const int idx = threadIdx.x + NT * (PER / 2 * h + u), p = idx % T64, q = idx / T64;
          v[u] = (r0 + q < a.R) ? ld_c(&a.Out[(j0 + p) + (r0 + q) * a.ldOut]) : 0.0;
        }
#pragma unroll
        for (int u = 0; u < PER / 2; ++u) {
          const int idx = threadIdx.x + NT * (PER / 2 * h + u), p = idx % T64, q = idx / T64;
          Bs[xs64(p, q)] = v[u];
        }
      }
      __syncthreads();
      mma64_lds<false, true, WM, 2>(res, As, Bs, 1.0);
      __syncthreads();
    }
    if (!fok) continue;
    acc_to_lds_sw(res, As);
    __syncthreads();
    lds_sw_to_global<NT>(As, nullptr, a.Out, a.ldOut, i0, r0, a.R - r0, false);
    publish(&a.flags[i * a.nrt + rt], 1);
    __syncthreads();
  }
}

// ----------------------------------------------------------------- resets
__global__ void dag_reset_kernel(int* p, int64_t count) {
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < count; i += (int64_t)gridDim.x * blockDim.x)
    p[i] = 0;
}

// Host check of the task order for T tile rows: every task exactly once, and
// each task after all the tasks it waits for.  Returns 0 when valid.
int check_chol_task_order(int T, int G) {
  if (G <= 0) G = kGemmGroup;
  std::vector<int64_t> offs;
  const int64_t n = chol_task_offsets(T, offs, G);
  int64_t expect = 1;
  for (int k = 0; k + 1 < T; ++k) expect += (int64_t)(T - k - 1) + gemm_task_count(T, k, G);
  if (n != expect) return 1;
  std::vector<int> state((size_t)T * T, 0);      // as on the device: updates applied, j + 1 when final
  auto st = [&](int i, int j) -> int& { return state[(size_t)i * T + j]; };
  for (int64_t t = 0; t < n; ++t) {
    const TaskDesc d = decode_task(t, T, offs.data(), G);
    if (d.i < 0 || d.i >= T || d.j < 0 || d.j >= T || d.k < 0 || d.k >= T) return 2;
    if (d.type == 0) {                            // DIAG(k)
      const int k = d.k;
      if (d.i != k || d.j != k) return 3;
      if (k >= 1) {
        // panel tile (k, k-1): every update but the last (from column k-2) applied
        if (st(k, k - 1) != (k >= 2 ? k - 2 : 0)) return 3;
        if (k >= 2 && (st(k, k - 2) < k - 1 || st(k - 1, k - 2) < k - 1)) return 3;
        if (st(k - 1, k - 1) < k) return 3;       // previous diagonal step done
        st(k, k - 1) = k;
      }
      if (st(k, k) != (k >= 1 ? k - 1 : 0)) return 3;   // diagonal tile: all but the last update
      st(k, k) = k + 1;
    } else if (d.type == 1) {                     // TRSM(i,k), i >= k+2, with the last update when k >= 1
      const int i = d.i, k = d.k;
      if (i < k + 2 || d.j != k) return 4;
      if (k >= 1 && (st(i, k - 1) < k || st(k, k - 1) < k || st(i, k) < k - 1)) return 4;
      if (st(k, k) < k + 1) return 4;
      if (st(i, k) != (k >= 1 ? k - 1 : 0)) return 4;
      st(i, k) = k + 1;
    } else {                                      // GEMM(i,j,k): updates kb..k, k <= j - 2
      const int kb = d.k - d.k % G;
      if (!(d.k + 2 <= d.j && d.j <= d.i)) return 5;
      // the kernel waits for L_ik, L_jk only: the earlier columns must be final by then
      if (st(d.i, d.k) < d.k + 1 || st(d.j, d.k) < d.k + 1) return 6;
      for (int kk = kb; kk <= d.k; ++kk)
        if (st(d.i, kk) < kk + 1 || st(d.j, kk) < kk + 1) return 6;
      if (st(d.i, d.j) != kb) return 6;
      st(d.i, d.j) = d.k + 1;
    }
  }
  for (int i = 0; i < T; ++i)
    for (int j = 0; j <= i; ++j)
      if (st(i, j) != j + 1) return 7;
  return 0;
}

// Workgroups that fit on the device at once for `kernel` (at least one per
// CU), optionally capped at `want` per CU.
template <typename K>
static int persistent_grid(K kernel, int want = 0, int block = 256) {
  int dev = 0, cus = 0, per_cu = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kernel, block, 0) != hipSuccess || per_cu < 1)
    per_cu = 1;
  if (want > 0 && want < per_cu) per_cu = want;
  return (cus > 0 ? cus : 256) * per_cu;
}

int64_t chol_task_offsets(int T, std::vector<int64_t>& offs, int G) {
  if (G <= 0) G = kGemmGroup;
  offs.assign((size_t)std::max(T, 1), 0);
  int64_t t = 1;                                  // DIAG(0)
  for (int k = 0; k + 1 < T; ++k) {
    offs[k] = t;
    t += (T - k - 1) + gemm_section_count(T, k, G);
  }
  if (T >= 1) offs[T - 1] = t;
  return t;
}

static CholArgs chol_args(const Inst& in) {
  CholArgs a;
  const int T = (int)(in.KMp / T64);
  a.G = in.G; a.ld = in.KMp; a.T = T; a.KM = in.KM; a.diag0 = in.diag0; a.Linv = in.Linv; a.Lt = in.Lt;
  a.state = in.dag; a.head = in.dag + (int64_t)T * T; a.err = a.head + 1; a.info = in.info;
  a.offs = in.chol_offs; a.ntasks = in.chol_ntasks; a.grp = kGemmGroup;
  a.col_off = 0;
  return a;
}

// Blocked outer factorization for large Grams: for every block column of
// NO = 1024 (16 tiles), factor the diagonal block with the tile DAG, form
// its inverse by a forward solve on the identity, solve the panel below as
// G_panel L_kk^{-T} and apply the symmetric update to the trailing lower
// triangle with FP64 MFMA products.  The critical path is then 16 diagonal
// steps per block column instead of one per 64-tile row.
// Counters of the blocked path: [0] error flag for the whole factorization,
// then the diagonal block's states and queue head, then the flags and head
// of its inverse (2 (NO/64)^2 + 3 ints in all).
static hipError_t launch_cholesky_blocked(const Inst& in, hipStream_t s) {
  const int64_t ld = in.KMp, NO = in.blk_NO;
  int* err = in.dag;
  hipLaunchKernelGGL(dag_reset_kernel, dim3(1), dim3(64), 0, s, err, (int64_t)1);
  for (int64_t k0 = 0; k0 < in.KMp; k0 += NO) {
    const int64_t nb = std::min<int64_t>(NO, in.KMp - k0), m = in.KMp - k0 - nb;
    const int Ts = (int)(nb / T64);
    const bool tail = nb != NO;
    // 1. the diagonal block, with the tile DAG on the sub-matrix
    CholBatch b{};
    CholArgs& a = b.one;
    a.G = in.G + k0 + k0 * ld; a.ld = ld; a.T = Ts; a.KM = in.KM;
    a.diag0 = in.diag0 + k0; a.Linv = in.Linv + (k0 / T64) * T64 * T64; a.Lt = in.Lt;
    a.state = in.dag + 1; a.head = a.state + (int64_t)Ts * Ts; a.err = err; a.info = in.info;
    a.offs = tail ? in.blk_offs_tail : in.blk_offs; a.ntasks = tail ? in.blk_ntasks_tail : in.blk_ntasks;
    a.grp = kGemmGroup;
    a.col_off = k0;
    b.ntasks = a.ntasks; b.head = a.head; b.err = a.err;
    const int64_t nctr = (int64_t)Ts * Ts + 1;
    hipLaunchKernelGGL(dag_reset_kernel, dim3((unsigned)std::min<int64_t>(ceil_div(nctr, 256), 1024)), dim3(256), 0, s,
                       a.state, nctr);
    hipLaunchKernelGGL(chol_dag_kernel, dim3((unsigned)persistent_grid(chol_dag_kernel, in.tune_chol_per_cu)),
                       dim3(256), 0, s, b);
    if (m <= 0) break;
    // 2. X = L_kk^{-1}: forward solve on the identity (only the lower triangle of X is nonzero)
    SolveBatch sb{};
    SolveArgs& v = sb.one;
    v.G = a.G; v.ld = ld; v.T = Ts; v.Linv = a.Linv;
    v.In = in.blk_I; v.ldIn = NO; v.Out = in.blk_X; v.ldOut = NO;
    v.R = nb; v.Rp = nullptr; v.nrt = Ts;
    v.flags = a.head + 1; v.info = in.info; v.skip = nullptr;
    sb.ntasks = (int64_t)Ts * Ts; sb.head = v.flags + (int64_t)Ts * Ts; sb.err = a.err; sb.backward = 0;
    const int64_t nflags = (int64_t)Ts * Ts + 1;
    hipLaunchKernelGGL(dag_reset_kernel, dim3((unsigned)std::min<int64_t>(ceil_div(nflags, 256), 1024)), dim3(256), 0, s,
                       v.flags, nflags);
    hipLaunchKernelGGL((solve_dag_kernel_t<false, kSolveWaves>), dim3((unsigned)std::min<int64_t>(persistent_grid(solve_dag_kernel_t<false, kSolveWaves>, 0, 64 * kSolveWaves), sb.ntasks)),
                       dim3(64 * kSolveWaves), 0, s, sb);
    // 3. panel: L_panel = G_panel X^T (from a copy of G_panel)
    double* panel = in.G + (k0 + nb) + k0 * ld;
    hipError_t e = launch_copy_panel(panel, ld, in.blk_P, m, m, nb, s);
    if (e == hipSuccess)
      e = launch_nt_gemm(in.blk_P, m, in.blk_X, NO, panel, ld, m, nb, nb, 1.0, 0, 0, s, in.tune_gemm_tile,
                         1);   // X = L_kk^{-1} is lower triangular
    // 4. trailing lower triangle: G_22 -= L_panel L_panel^T
    if (e == hipSuccess)
      e = launch_nt_gemm(panel, ld, panel, ld, in.G + (k0 + nb) + (k0 + nb) * ld, ld, m, m, nb, -1.0, 1, 1, s,
                         in.tune_gemm_tile);
    if (e != hipSuccess) return e;
  }
  return hipGetLastError();
}

int* chol_error_flag(const Inst& in) {
  const int64_t T = in.KMp / T64;
  return in.blk_NO > 0 ? in.dag : in.dag + T * T + 1;
}

hipError_t launch_cholesky(const Inst& in, hipStream_t s, hipEvent_t after_reset) {
  if (in.blk_NO > 0) {
    const hipError_t e = launch_cholesky_blocked(in, s);
    return e != hipSuccess ? e : launch_solve_fold(in, s);
  }
  const int T = (int)(in.KMp / T64);
  // counters: state T*T, then head, err
  const int64_t nctr = (int64_t)T * T + 2;
  hipLaunchKernelGGL(dag_reset_kernel, dim3((unsigned)std::min<int64_t>(ceil_div(nctr, 256), 1024)), dim3(256),
                     0, s, in.dag, nctr);
  if (after_reset) {
    const hipError_t e = hipEventRecord(after_reset, s);
    if (e != hipSuccess) return e;
  }
  CholBatch b{};
  b.one = chol_args(in);
  b.ntasks = in.chol_ntasks; b.head = b.one.head; b.err = b.one.err;
  hipLaunchKernelGGL(chol_dag_kernel, dim3((unsigned)persistent_grid(chol_dag_kernel, in.tune_chol_per_cu)), dim3(256),
                     0, s, b);
  const hipError_t e = hipGetLastError();
  return e != hipSuccess ? e : launch_solve_fold(in, s);
}

// The folded products of the block solves: block (i, y) forms, for the
// distance d = 1 + y / 2, Mf_i = Linv_i L_{i,i-d} (y even, i >= d) or
// Mb_i = Linv_i^T L_{i+d,i}^T (y odd, i + d <= T - 1); column-major, in M
// at block (y T + i) (Mf, Mb, Mf2, Mb2).
__global__ __launch_bounds__(256) void solve_fold_kernel(const double* G, int64_t ld, const double* Linv, int T,
                                                         double* M) {
  __shared__ double As[T64 * T64];
  __shared__ double Bs[T64 * T64];
  const int i = blockIdx.x, y = blockIdx.y, dir = y & 1, dist = 1 + y / 2;
  if ((dir == 0 && i < dist) || (dir == 1 && i + dist > T - 1)) return;
  const gdouble* Lb = gp(Linv + (int64_t)i * T64 * T64);
  const int64_t i0 = (int64_t)i * T64, o = (int64_t)dist * T64;
#pragma unroll
  for (int u = 0; u < 16; ++u) {
    const int idx = threadIdx.x + 256 * u, p = idx % T64, c = idx / T64;
    if (dir == 0) {
      As[idx] = Lb[idx];                                            // A[p][c] = Linv[p][c]
      Bs[xs64(p, c)] = gp(G)[(i0 + p) + (i0 - o + c) * ld];         // B[p][c] = L_{i,i-d}[p][c]
    } else {
      As[xs64(p, c)] = Lb[idx];                                     // A[c][p] = Linv[p][c]
      Bs[idx] = gp(G)[(i0 + o + p) + (i0 + c) * ld];                // B[c][p] = L_{i+d,i}[p][c]
    }
  }
  __syncthreads();
  TileF64<T64, T64, 2, 2> acc;
  acc.zero();
  if (dir == 0) mma64_lds<false, true>(acc, As, Bs, 1.0);
  else mma64_lds<true, false>(acc, As, Bs, 1.0);
  double* Mo = M + ((int64_t)y * T + i) * T64 * T64;
  acc.for_each([&](int r, int c, double v) { Mo[r + c * T64] = v; });
}

hipError_t launch_solve_fold(const Inst& in, hipStream_t s) {
  const int T = (int)(in.KMp / T64);
  if (!in.Msol || T < 2) return hipSuccess;
  hipLaunchKernelGGL(solve_fold_kernel, dim3((unsigned)T, 4), dim3(256), 0, s, in.G, in.KMp, in.Linv, T, in.Msol);
  return hipGetLastError();
}

static SolveArgs solve_args(const Inst& in, const double* In, double* Out, int64_t R, const int* skip) {
  SolveArgs a;
  const int T = (int)(in.KMp / T64);
  a.G = in.G; a.ld = in.KMp; a.T = T; a.Linv = in.Linv;
  const int64_t bs = (int64_t)T * T64 * T64;
  a.Mf = in.Msol; a.Mb = in.Msol ? in.Msol + bs : nullptr;
  a.Mf2 = in.Msol ? in.Msol + 2 * bs : nullptr; a.Mb2 = in.Msol ? in.Msol + 3 * bs : nullptr;
  a.In = In; a.ldIn = in.KMp; a.Out = Out; a.ldOut = in.KMp;
  a.R = R; a.Rp = nullptr; a.nrt = in.nrt_max;
  a.flags = in.dag + (int64_t)T * T + 2;               // T * nrt_max flags, then head
  a.info = in.info; a.skip = skip;
  return a;
}

// The forward pass of the solve, Wk <- L^{-1} B (B = in.Y, Wk = in.B, R
// right-hand sides), on stream s while the factorization runs on another
// stream: its tasks read each L block and diagonal inverse once the
// factorization has published it.  `s` must be ordered after the reset of
// the factorization's tile states (its tasks would read the last
// factorization's states otherwise).  The error flag is its own (the last
// int of the counters).
hipError_t launch_chol_solve_fwd_concurrent(const Inst& in, int64_t R, hipStream_t s) {
  if (R <= 0) return hipSuccess;
  const int T = (int)(in.KMp / T64);
  if (in.blk_NO > 0 || !in.Lt) return hipErrorInvalidValue;
  SolveBatch b{};
  b.one = solve_args(in, in.Y, in.B, R, nullptr);
  b.one.Mf = b.one.Mb = b.one.Mf2 = b.one.Mb2 = nullptr;   // formed after the factorization
  b.one.cstate = in.dag; b.one.cT = T; b.one.Lt = in.Lt;
  b.one.nrt = (int)ceil_div(R, T64);
  b.ntasks = (int64_t)T * b.one.nrt;
  b.head = b.one.flags + (int64_t)T * in.nrt_max;
  b.err = b.head + 1;
  b.backward = 0;
  const int64_t nflags = (int64_t)T * in.nrt_max + 2;       // flags, head, err
  hipLaunchKernelGGL(dag_reset_kernel, dim3((unsigned)std::min<int64_t>(ceil_div(nflags, 256), 1024)), dim3(256), 0,
                     s, b.one.flags, nflags);
  const unsigned g = (unsigned)std::min<int64_t>(persistent_grid(solve_dag_kernel_t<true, 4>, 1), b.ntasks);
  hipLaunchKernelGGL((solve_dag_kernel_t<true, 4>), dim3(g), dim3(256), 0, s, b);
  return hipGetLastError();
}

int* chol_solve_fwd_error_flag(const Inst& in) {
  const int64_t T = in.KMp / T64;
  return in.dag + T * T + 2 + T * in.nrt_max + 1;
}

// Blocked solves for a factor from the blocked factorization, with many
// right-hand sides: per block column of NO rows, the tile-DAG solve of the
// diagonal block, then one MFMA product that applies the solved rows to all
// rows still to come:
//   forward,  blocks in order:   Z_k = L_kk^{-1} Y_k,  Y_rest -= L_rest,k Z_k   (rows below)
//   backward, blocks reversed:   Y_k = L_kk^{-T} W_k,  W_rest -= L_k,rest^T Y_k (rows above)
// so that almost all the flops run as large products instead of 64 x 64
// tile tasks.  Y (forward) and Wk (backward) are overwritten as they are
// consumed.  The diagonal-block solves use the 64 x 64 inverses and folded
// products of the whole factor, restricted to the block.
constexpr int kBlockedSolveMinTiles = 4;   // right-hand-side tiles of 64 from which the blocked solve is used

static hipError_t launch_chol_solve_blocked(const Inst& in, double* Y, int64_t ldY, int64_t R, double* Wk,
                                            int64_t ldW, hipStream_t s, const int* skip) {
  const int T = (int)(in.KMp / T64);
  const int64_t ld = in.KMp, NO = in.blk_NO, bs = (int64_t)T * T64 * T64;
  const int nrt = (int)ceil_div(R, T64);
  int* err = in.dag + (int64_t)T * T + 1;
  const int64_t nflags = (int64_t)T * in.nrt_max + 2;      // err, flags, head
  const unsigned g0 = (unsigned)persistent_grid(solve_dag_kernel_t<false, kSolveWaves>, 0, 64 * kSolveWaves);
  const int64_t nblk = ceil_div(in.KMp, NO);
  for (int pass = 0; pass < 2; ++pass) {
    for (int64_t bb = 0; bb < nblk; ++bb) {
      const int64_t blk = pass ? nblk - 1 - bb : bb;
      const int64_t k0 = blk * NO, nb = std::min<int64_t>(NO, in.KMp - k0);
      const int Ts = (int)(nb / T64);
      const int64_t t0 = k0 / T64;
      SolveBatch b{};
      SolveArgs& a = b.one;
      a.G = in.G + k0 + k0 * ld; a.ld = ld; a.T = Ts;
      a.Linv = in.Linv + t0 * T64 * T64;
      if (in.Msol) {
        a.Mf = in.Msol + t0 * T64 * T64; a.Mb = a.Mf + bs;
        a.Mf2 = a.Mf + 2 * bs; a.Mb2 = a.Mf + 3 * bs;
      }
      if (!pass) { a.In = Y + k0; a.ldIn = ldY; a.Out = Wk + k0; a.ldOut = ldW; }
      else { a.In = Wk + k0; a.ldIn = ldW; a.Out = Y + k0; a.ldOut = ldY; }
      a.R = R; a.Rp = nullptr; a.nrt = nrt;
      a.flags = err + 1; a.info = in.info; a.skip = skip;
      b.ntasks = (int64_t)Ts * nrt;
      b.head = a.flags + (int64_t)T * in.nrt_max;
      b.err = err;
      b.backward = pass;
      hipLaunchKernelGGL(dag_reset_kernel, dim3((unsigned)std::min<int64_t>(ceil_div(nflags, 256), 1024)),
                         dim3(256), 0, s, err, nflags);
      hipLaunchKernelGGL((solve_dag_kernel_t<false, kSolveWaves>), dim3((unsigned)std::min<int64_t>(g0, b.ntasks)),
                         dim3(64 * kSolveWaves), 0, s, b);
      hipError_t e;
      if (!pass) {
        // Y(k0 + nb.., :) -= L(k0 + nb.., k0..) Z_k
        const int64_t m = in.KMp - k0 - nb;
        e = launch_solve_gemm(false, in.G + (k0 + nb) + k0 * ld, ld, Wk + k0, ldW, Y + k0 + nb, ldY, m, R, nb,
                              -1.0, skip, s);
      } else {
        // W(0..k0, :) -= L(k0.., 0..k0)^T Y_k
        e = launch_solve_gemm(true, in.G + k0, ld, Y + k0, ldY, Wk, ldW, k0, R, nb, -1.0, skip, s);
      }
      if (e != hipSuccess) return e;
    }
  }
  return hipGetLastError();
}

// Y (KMp x R, ld ldY) <- G^{-1} Y; Wk (KMp x R) is work: it holds the
// forward result between the passes and is overwritten.  With first_pass =
// 1 only the backward pass runs (Wk already holds the forward result).
hipError_t launch_chol_solve(const Inst& in, double* Y, int64_t ldY, int64_t R, double* Wk, int64_t ldW,
                             hipStream_t s, const int* skip, int first_pass) {
  if (R <= 0) return hipSuccess;
  if (in.blk_NO > 0 && first_pass == 0 && ceil_div(R, T64) >= kBlockedSolveMinTiles)
    return launch_chol_solve_blocked(in, Y, ldY, R, Wk, ldW, s, skip);
  const int T = (int)(in.KMp / T64);
  SolveBatch b{};
  b.one = solve_args(in, Y, Wk, R, skip);
  b.one.ldIn = ldY; b.one.ldOut = ldW;
  b.one.nrt = (int)ceil_div(R, T64);
  b.ntasks = (int64_t)T * b.one.nrt;
  b.head = b.one.flags + (int64_t)T * in.nrt_max;
  b.err = in.dag + (int64_t)T * T + 1;                        // just before the flags
  // the error flag, the flags and the head are reset before each pass (after
  // a blocked factorization nothing else clears the error flag)
  const int64_t nflags = (int64_t)T * in.nrt_max + 2;
  const unsigned g = (unsigned)std::min<int64_t>(persistent_grid(solve_dag_kernel_t<false, kSolveWaves>, 0, 64 * kSolveWaves), b.ntasks);
  for (int pass = first_pass; pass < 2; ++pass) {
    hipLaunchKernelGGL(dag_reset_kernel, dim3((unsigned)std::min<int64_t>(ceil_div(nflags, 256), 1024)),
                       dim3(256), 0, s, b.err, nflags);
    b.backward = pass;
    if (pass == 1) {
      b.one.In = Wk; b.one.ldIn = ldW; b.one.Out = Y; b.one.ldOut = ldY;
    }
    hipLaunchKernelGGL((solve_dag_kernel_t<false, kSolveWaves>), dim3(g), dim3(64 * kSolveWaves), 0, s, b);
  }
  return hipGetLastError();
}

// ------------------------------------------------------------------ batches
// Every instance of a plan in one persistent launch: the instances' task
// lists are interleaved round by round (the diagonal and panel tasks of a
// step before its updates), largest instance first, and each instance keeps
// its own order, so the waits stay deadlock-free.
struct DagBatch {
  int count = 0;
  CholArgs* chol = nullptr; DagSeg* chol_segs = nullptr; int chol_nsegs = 0; int64_t chol_total = 0;
  SolveArgs* solve[2] = {nullptr, nullptr};   // solve into Y (initial) or into D (refinement)
  DagSeg* solve_segs = nullptr; int solve_nsegs = 0; int64_t solve_total = 0;
  int64_t* R = nullptr;                        // right-hand sides of the current apply, per instance
  int** rst_ptr = nullptr; int64_t* rst_cnt = nullptr;   // [0, count): Cholesky states, [count, 2 count): solve flags
  int64_t rst_max[2] = {0, 0};
  int* ctr = nullptr;                          // [0] Cholesky head, [1] error, [2] solve head
};

__global__ void batch_reset_kernel(int* const* ptrs, const int64_t* counts) {
  int* p = ptrs[blockIdx.y];
  const int64_t n = counts[blockIdx.y];
  for (int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (int64_t)gridDim.x * blockDim.x) p[i] = 0;
}

struct RhsPack { int first, n; int64_t v[128]; };
__global__ void set_rhs_kernel(int64_t* dst, RhsPack pk) {
  if ((int)threadIdx.x < pk.n) dst[pk.first + threadIdx.x] = pk.v[threadIdx.x];
}

template <class T>
static hipError_t upload(T** d, const std::vector<T>& h) {
  *d = nullptr;
  if (h.empty()) return hipSuccess;
  hipError_t e = hipMalloc((void**)d, sizeof(T) * h.size());
  if (e == hipSuccess) e = hipMemcpy(*d, h.data(), sizeof(T) * h.size(), hipMemcpyHostToDevice);
  return e;
}

void free_dag_batch(DagBatch* b) {
  if (!b) return;
  (void)hipFree(b->chol); (void)hipFree(b->chol_segs); (void)hipFree(b->solve[0]); (void)hipFree(b->solve[1]);
  (void)hipFree(b->solve_segs); (void)hipFree(b->R); (void)hipFree(b->rst_ptr); (void)hipFree(b->rst_cnt);
  (void)hipFree(b->ctr);
  delete b;
}

DagBatch* make_dag_batch(const std::vector<Inst>& insts) {
  DagBatch* b = new DagBatch();
  const int n = (int)insts.size();
  b->count = n;
  std::vector<int> order(n);
  for (int i = 0; i < n; ++i) order[i] = i;
  std::stable_sort(order.begin(), order.end(), [&](int x, int y) { return insts[x].KMp > insts[y].KMp; });
  std::vector<CholArgs> ch(n);
  std::vector<SolveArgs> sv0(n), sv1(n);
  std::vector<std::vector<int64_t>> offs(n);
  std::vector<int> Ts(n);
  std::vector<int*> rp(2 * n);
  std::vector<int64_t> rc(2 * n);
  int maxT = 0;
  hipError_t e = hipMalloc((void**)&b->R, sizeof(int64_t) * n);
  if (e == hipSuccess) e = hipMalloc((void**)&b->ctr, sizeof(int) * 4);
  for (int i = 0; i < n && e == hipSuccess; ++i) {
    const Inst& in = insts[i];
    Ts[i] = (int)(in.KMp / T64);
    maxT = std::max(maxT, Ts[i]);
    chol_task_offsets(Ts[i], offs[i], kGemmGroup);
    ch[i] = chol_args(in);
    sv0[i] = solve_args(in, in.Y, in.B, 0, nullptr);
    sv1[i] = solve_args(in, in.D, in.B, 0, &in.ctl->done);
    sv0[i].Rp = sv1[i].Rp = b->R + i;
    rp[i] = in.dag;
    rc[i] = (int64_t)Ts[i] * Ts[i];
    rp[n + i] = sv0[i].flags;
    rc[n + i] = (int64_t)Ts[i] * in.nrt_max;
    b->rst_max[0] = std::max(b->rst_max[0], rc[i]);
    b->rst_max[1] = std::max(b->rst_max[1], rc[n + i]);
  }
  // Cholesky segments
  std::vector<DagSeg> cs;
  int64_t g = 0;
  auto add = [&](std::vector<DagSeg>& v, int inst, int64_t lstart, int64_t cnt) {
    if (cnt <= 0) return;
    v.push_back(DagSeg{g, lstart, inst, 0});
    g += cnt;
  };
  for (int i : order) add(cs, i, 0, 1);                                      // DIAG(0)
  for (int r = 0; r + 1 < maxT; ++r) {
    for (int i : order)
      if (r + 1 < Ts[i]) add(cs, i, offs[i][r], Ts[i] - r - 1);              // DIAG(r+1), TRSM(., r)
    for (int i : order)
      if (r + 1 < Ts[i]) add(cs, i, offs[i][r] + Ts[i] - r - 1, gemm_section_count(Ts[i], r, kGemmGroup));   // GEMM(., ., r)
  }
  b->chol_total = g;
  b->chol_nsegs = (int)cs.size();
  // solve segments: block row by block row, all column tiles of an instance together
  std::vector<DagSeg> ss;
  g = 0;
  for (int st = 0; st < maxT; ++st)
    for (int i : order)
      if (st < Ts[i]) add(ss, i, (int64_t)st * insts[i].nrt_max, insts[i].nrt_max);
  b->solve_total = g;
  b->solve_nsegs = (int)ss.size();
  if (e == hipSuccess) e = upload(&b->chol, ch);
  if (e == hipSuccess) e = upload(&b->chol_segs, cs);
  if (e == hipSuccess) e = upload(&b->solve[0], sv0);
  if (e == hipSuccess) e = upload(&b->solve[1], sv1);
  if (e == hipSuccess) e = upload(&b->solve_segs, ss);
  if (e == hipSuccess) e = upload(&b->rst_ptr, rp);
  if (e == hipSuccess) e = upload(&b->rst_cnt, rc);
  if (e == hipSuccess) e = hipMemset(b->R, 0, sizeof(int64_t) * n);
  if (e != hipSuccess) {
    free_dag_batch(b);
    return nullptr;
  }
  return b;
}

int* dag_batch_error(const DagBatch* b) { return b->ctr + 1; }

hipError_t launch_cholesky_batch(const DagBatch* b, hipStream_t s, int per_cu) {
  hipLaunchKernelGGL(dag_reset_kernel, dim3(1), dim3(64), 0, s, b->ctr, (int64_t)4);
  const unsigned gx = (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(b->rst_max[0], 256), 256));
  hipLaunchKernelGGL(batch_reset_kernel, dim3(gx, (unsigned)b->count), dim3(256), 0, s, b->rst_ptr, b->rst_cnt);
  CholBatch cb{};
  cb.inst = b->chol; cb.segs = b->chol_segs; cb.nsegs = b->chol_nsegs;
  cb.ntasks = b->chol_total; cb.head = b->ctr; cb.err = b->ctr + 1;
  hipLaunchKernelGGL(chol_dag_kernel, dim3((unsigned)persistent_grid(chol_dag_kernel, per_cu)), dim3(256), 0, s, cb);
  return hipGetLastError();
}

hipError_t set_batch_rhs(const DagBatch* b, const int64_t* R, hipStream_t s) {
  for (int first = 0; first < b->count; first += 128) {
    RhsPack pk;
    pk.first = first;
    pk.n = std::min(128, b->count - first);
    for (int i = 0; i < pk.n; ++i) pk.v[i] = R[first + i];
    hipLaunchKernelGGL(set_rhs_kernel, dim3(1), dim3(128), 0, s, b->R, pk);
  }
  return hipGetLastError();
}

hipError_t launch_chol_solve_batch(const DagBatch* b, int refine, hipStream_t s) {
  SolveBatch sb{};
  sb.inst = b->solve[refine ? 1 : 0]; sb.segs = b->solve_segs; sb.nsegs = b->solve_nsegs;
  sb.ntasks = b->solve_total; sb.head = b->ctr + 2; sb.err = b->ctr + 1; sb.swap_io = 1;
  const unsigned gx = (unsigned)std::max<int64_t>(1, std::min<int64_t>(ceil_div(b->rst_max[1], 256), 256));
  const unsigned g = (unsigned)std::min<int64_t>(persistent_grid(solve_dag_kernel_t<false, kSolveWaves>, 0, 64 * kSolveWaves), b->solve_total);
  for (int pass = 0; pass < 2; ++pass) {
    hipLaunchKernelGGL(dag_reset_kernel, dim3(1), dim3(64), 0, s, b->ctr + 2, (int64_t)1);
    hipLaunchKernelGGL(batch_reset_kernel, dim3(gx, (unsigned)b->count), dim3(256), 0, s, b->rst_ptr + b->count,
                       b->rst_cnt + b->count);
    sb.backward = pass;
    hipLaunchKernelGGL((solve_dag_kernel_t<false, kSolveWaves>), dim3(g), dim3(64 * kSolveWaves), 0, s, sb);
  }
  return hipGetLastError();
}


// ------------------------------------------------- member-block inverses
// The inverse of one diagonal member block G_kk (rows and columns o..o+M of
// the symmetric Gram copy Gs) for the block-Jacobi preconditioner of CG:
// the block is copied to D (Mp x Mp, identity padding), factored by the tile
// DAG and inverted by a forward and a backward solve on the identity.
// ctr: [0] error flag, then the DAG states and head, then the solve flags and
// head (2 (Mp/64)^2 + 3 ints).
__global__ void member_block_copy_kernel(const double* __restrict__ Gs, int64_t ld, int64_t o, int64_t M, int64_t Mp,
                                         double* __restrict__ D, double* __restrict__ d0) {
  const int64_t c = blockIdx.y;
  for (int64_t r = (int64_t)blockIdx.x * blockDim.x + threadIdx.x; r < Mp; r += (int64_t)gridDim.x * blockDim.x) {
    const double v = (r < M && c < M) ? Gs[(o + r) + (o + c) * ld] : (r == c ? 1.0 : 0.0);
    D[r + c * Mp] = v;
    if (r == c) d0[r] = v;
  }
}

hipError_t launch_member_block_inverse(const double* Gs, int64_t ld, int64_t o, int64_t M, int64_t Mp, double* D,
                                       double* d0, double* Linv, int* ctr, const int64_t* offs, int64_t ntasks,
                                       const double* I, double* Wk, double* Dinv, int* info, hipStream_t s) {
  const int Tb = (int)(Mp / T64);
  hipLaunchKernelGGL(member_block_copy_kernel, dim3((unsigned)std::min<int64_t>(ceil_div(Mp, 256), 8), (unsigned)Mp),
                     dim3(256), 0, s, Gs, ld, o, M, Mp, D, d0);
  const int64_t nctr = 2 * (int64_t)Tb * Tb + 3;
  hipLaunchKernelGGL(dag_reset_kernel, dim3((unsigned)std::min<int64_t>(ceil_div(nctr, 256), 64)), dim3(256), 0, s, ctr,
                     nctr);
  CholBatch b{};
  CholArgs& a = b.one;
  a.G = D; a.ld = Mp; a.T = Tb; a.KM = M; a.diag0 = d0; a.Linv = Linv; a.Lt = nullptr;
  a.state = ctr + 1; a.head = a.state + (int64_t)Tb * Tb; a.err = ctr; a.info = info;
  a.offs = offs; a.ntasks = ntasks; a.grp = kGemmGroup; a.col_off = o;
  b.ntasks = ntasks; b.head = a.head; b.err = a.err;
  hipLaunchKernelGGL(chol_dag_kernel, dim3((unsigned)persistent_grid(chol_dag_kernel)), dim3(256), 0, s, b);
  SolveBatch sb{};
  SolveArgs& v = sb.one;
  v.G = D; v.ld = Mp; v.T = Tb; v.Linv = Linv;
  v.R = Mp; v.Rp = nullptr; v.nrt = Tb;
  v.flags = a.head + 1; v.info = info; v.skip = nullptr;
  sb.ntasks = (int64_t)Tb * Tb; sb.head = v.flags + (int64_t)Tb * Tb; sb.err = ctr;
  const int64_t nflags = (int64_t)Tb * Tb + 1;
  const unsigned g = (unsigned)std::min<int64_t>(persistent_grid(solve_dag_kernel_t<false, kSolveWaves>, 0, 64 * kSolveWaves), sb.ntasks);
  for (int pass = 0; pass < 2; ++pass) {
    hipLaunchKernelGGL(dag_reset_kernel, dim3((unsigned)std::min<int64_t>(ceil_div(nflags, 256), 64)), dim3(256), 0, s,
                       v.flags, nflags);
    sb.backward = pass;
    if (pass == 0) { v.In = I; v.ldIn = Mp; v.Out = Wk; v.ldOut = Mp; }
    else { v.In = Wk; v.ldIn = Mp; v.Out = Dinv; v.ldOut = Mp; }
    hipLaunchKernelGGL((solve_dag_kernel_t<false, kSolveWaves>), dim3(g), dim3(64 * kSolveWaves), 0, s, sb);
  }
  return hipGetLastError();
}

}  // namespace pc
