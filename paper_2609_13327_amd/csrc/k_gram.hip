// FP64 Gram of the modulated square root, assembled without forming Z.
//
// Per grid column j the n_w x K block A_j (the rows of the members in column
// j, the paper's A_m of Sec. 3.9) gives S_j = A_j^T A_j.  Because the
// localization is horizontal (equal blocks C_b, Sec. 3.6) every level shares
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
                                                           double* __restrict__ S, int64_t ldS) {
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
      if (jj < jb && j0 + jj < n_h) S[(j0 + jj) * ldS + p] = acc[jj];
  }
}

hipError_t launch_column_grams(const Inst& in, hipStream_t s) {
  int jb = CG_JB;
  while (jb > 1 && (int64_t)jb * in.K * 8 > 48 * 1024) jb /= 2;
  dim3 grid((unsigned)ceil_div(in.n_h, jb), (unsigned)ceil_div(in.P, 256));
  size_t shm = (size_t)jb * in.K * sizeof(double);
  hipLaunchKernelGGL(column_grams_kernel, grid, dim3(256), shm, s, in.E, in.ldE, in.n_h, in.n_w,
                     (int)in.K, in.P, in.pairs, jb, in.S, in.ldS);
  return hipGetLastError();
}

// -------------------------------------------------------------- FP64 Gram
// Tile: TP pairs p x 128 mode pairs q, the latter two 8 x 8 blocks of
// (m, m') (origins from the tile table; column c of block h is
// m = m0_h + c / 8, m' = m0'_h + c % 8).  Per chunk of 16 grid columns j the
// workgroup stages the S rows of its TP pairs and the 32 columns of W its
// mode pairs use; the T operand W[j,m] W[j,m'] is formed when the MFMA
// fragment is read from LDS.  Full tiles (TP = 128): four waves own 64 x 64
// quadrants (4 x 4 fragments of 16 x 16), wave column h covering block h.
// The pairs left over after the full tiles (P mod 128, when at most 32)
// form tail tiles of TP = 32: each wave owns 32 pairs x 32 mode pairs, so
// that no products of empty pair rows are formed.
// When the tiles are too few to fill the device the j range is split in two
// to four parts written to G and G2 and summed afterwards in a fixed order
// (results are reproducible), as many as keep the rounds of workgroups full.
// Workgroups are mapped so that each XCD (the hardware places workgroup b on
// XCD b mod 8) works on a contiguous range of tiles, which then share S rows
// in its L2; the tail tiles come first.
constexpr int GB = 128, GBT = 32, GKC = 24, GWC = 32;
constexpr int GWS = 36;                           // W row stride in LDS: the four row groups of a read on distinct banks
constexpr int GWH = (GKC * GWC + 255) / 256;      // W values staged per thread and chunk
static_assert(GKC <= kGramZeroRows, "the last chunk reads up to GKC - 1 rows past n_h");

template <class WS>
struct GramArgs {
  const double* S; int64_t ldS;
  WS w;
  int64_t n_h, M, P;
  const int* pairs; const int* qtiles;
  int nfull, nq, tail, split;             // full pair tiles, mode-pair tiles, tail pair tile (0 or 1)
  int64_t jlen;
  double* G; double* G2; int64_t ldG;     // part q >= 1 goes to G2 + (q - 1) ldG^2
};

// One tile of TP pairs from p0, mode-pair tile qi, contraction part `part`.
template <int TP, class WS>
__device__ __forceinline__ void gram_tile(const GramArgs<WS>& a, int part, int64_t p0, int qi, double* As0,
                                          double* Ws0) {
  constexpr int FMR = TP == GB ? 4 : 2, FNC = TP == GB ? 4 : 2;   // fragments per wave: rows, columns
  constexpr int SPR = TP / 2;                                      // threads per staged S row (two pairs each)
  constexpr int SRP = 256 / SPR, NSR = (GKC + SRP - 1) / SRP;      // S rows per pass, passes
  static_assert(GKC % 4 == 0, "chunks of whole MFMA k-steps");
  const int* qt = a.qtiles + 4 * qi;                     // (m0, m0') of block 0, then of block 1
  const int64_t jbeg = (int64_t)part * a.jlen;
  const int64_t jend = jbeg + a.jlen < a.n_h ? jbeg + a.jlen : a.n_h;
  const int nchunks = (int)((jend - jbeg + GKC - 1) / GKC);
  const int t = threadIdx.x, lane = lane_id(), w = wave_id();
  const int r = lane & 15, kq = lane >> 4;
  const int rowbase = TP == GB ? (w >> 1) * 64 : 0;      // first pair row of this wave
  const int blk = TP == GB ? (w & 1) : (w >> 1);         // mode block of this wave
  const int jbase = TP == GB ? 0 : 2 * (w & 1);          // first column fragment inside the block

  // this thread's staging slots
  const int sp = (t % SPR) * 2, srow = t / SPR;          // S: rows srow + SRP i, pairs sp, sp+1
  int wcol[GWH], wrow[GWH];
  int64_t wm_idx[GWH];
#pragma unroll
  for (int h = 0; h < GWH; ++h) {
    const int idx = t + 256 * h;
    wcol[h] = idx / GKC;
    wrow[h] = idx % GKC;
    // W columns: 0..7 m of block 0, 8..15 m' of block 0, 16..23 m of block 1, 24..31 m' of block 1
    const int wc = wcol[h] < GWC ? wcol[h] : 0;
    wm_idx[h] = (int64_t)qt[2 * (wc / 16) + ((wc % 16) >= 8 ? 1 : 0)] + (wc % 8);
  }
  // The loads are unconditional, so that the products of a chunk never wait
  // for the next chunk's loads (loads behind branches, or values selected
  // right after them, make the compiler wait for them at once): S has GKC
  // zero rows past n_h, which zero the terms of rows beyond the last; W is
  // read at clamped, valid indices (finite values: times a zero S row they
  // give zero, and out-of-range mode columns only reach unwritten outputs).
  double sv[2 * NSR], wv[GWH];
  const int64_t jlast = a.n_h - 1, mlast = a.M - 1;
  auto load = [&](int chunk) {
    const int64_t j0 = jbeg + (int64_t)chunk * GKC;
#pragma unroll
    for (int i = 0; i < NSR; ++i) {
      // (a last pass that covers rows past the chunk reads its first row again; not stored)
      const int rr = srow + SRP * i < GKC ? srow + SRP * i : 0;
      const double2 v = *reinterpret_cast<const double2*>(a.S + (j0 + rr) * a.ldS + p0 + sp);
      sv[2 * i] = v.x;
      sv[2 * i + 1] = v.y;
    }
#pragma unroll
    for (int h = 0; h < GWH; ++h) {
      const int64_t j = j0 + wrow[h];
      wv[h] = a.w(j < jlast ? j : jlast, wm_idx[h] < mlast ? wm_idx[h] : mlast);
    }
  };
  auto store = [&](int buf) {
    double* As = As0 + buf * (GKC * TP);
    double* Ws = Ws0 + buf * (GKC * GWS);
#pragma unroll
    for (int i = 0; i < NSR; ++i) {
      if (NSR * SRP > GKC && srow + SRP * i >= GKC) continue;
      As[(srow + SRP * i) * TP + sp] = sv[2 * i];
      As[(srow + SRP * i) * TP + sp + 1] = sv[2 * i + 1];
    }
#pragma unroll
    for (int h = 0; h < GWH; ++h)
      if (wcol[h] < GWC) Ws[wrow[h] * GWS + wcol[h]] = wv[h];
  };

  d4 acc[FMR][FNC];
#pragma unroll
  for (int i = 0; i < FMR; ++i)
#pragma unroll
    for (int j = 0; j < FNC; ++j) acc[i][j] = d4{0.0, 0.0, 0.0, 0.0};
  if (nchunks > 0) {
    load(0);
    store(0);
    __syncthreads();
    for (int c = 0; c < nchunks; ++c) {
      const bool more = c + 1 < nchunks;
      if (more) load(c + 1);
      const double* Ab = As0 + (c & 1) * (GKC * TP);
      const double* Wb = Ws0 + (c & 1) * (GKC * GWS);
#pragma unroll
      for (int kk = 0; kk < GKC; kk += 4) {
        const int krow = kk + kq;
        double av[FMR], bv[FNC];
#pragma unroll
        for (int i = 0; i < FMR; ++i) av[i] = Ab[krow * TP + rowbase + i * 16 + r];
        const double wmp = Wb[krow * GWS + 16 * blk + 8 + (r & 7)];                          // W[j, m']
#pragma unroll
        for (int j = 0; j < FNC; ++j)
          bv[j] = Wb[krow * GWS + 16 * blk + 2 * (jbase + j) + (r >> 3)] * wmp;              // W[j, m] W[j, m']
#pragma unroll
        for (int i = 0; i < FMR; ++i)
#pragma unroll
          for (int j = 0; j < FNC; ++j) acc[i][j] = mfma_f64(av[i], bv[j], acc[i][j]);
      }
      if (more) store((c + 1) & 1);
      __syncthreads();
    }
  }
  double* Gout = part == 0 ? a.G : a.G2 + (int64_t)(part - 1) * a.ldG * a.ldG;
#pragma unroll
  for (int i = 0; i < FMR; ++i)
#pragma unroll
    for (int j = 0; j < FNC; ++j)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const int row = rowbase + i * 16 + kq + 4 * v;   // pair
        const int c = (jbase + j) * 16 + r;              // mode pair c of block blk
        const int64_t p = p0 + row;
        if (p >= a.P) continue;
        const int64_t m = qt[2 * blk] + (c >> 3), mp = qt[2 * blk + 1] + (c & 7);
        if (mp >= a.M || m > mp) continue;
        const int64_t k = a.pairs[2 * p], kp = a.pairs[2 * p + 1];
        const double val = acc[i][j][v];
        Gout[(kp * a.M + mp) + (k * a.M + m) * a.ldG] = val;
        if (k != kp && m != mp) Gout[(kp * a.M + m) + (k * a.M + mp) * a.ldG] = val;
      }
}

template <class WS>
__global__ __launch_bounds__(256) void gram_f64_kernel(GramArgs<WS> a) {
  __shared__ double As[2 * GKC * GB];
  __shared__ double Ws[2 * GKC * GWS];
  // every XCD takes an equal share of the tail units first, then a
  // contiguous range of the full ones
  const int64_t tail_units = (int64_t)a.tail * a.nq * a.split, ntiles = (int64_t)a.nfull * a.nq;
  const int64_t tail_per = (tail_units + 7) / 8, full_per = (ntiles * a.split + 7) / 8;
  const int64_t xcd = blockIdx.x % 8, l = blockIdx.x / 8;
  if (l < tail_per) {
    const int64_t u = xcd * tail_per + l;
    if (u >= tail_units) return;
    gram_tile<GBT>(a, (int)(u / a.nq), (int64_t)a.nfull * GB, (int)(u % a.nq), As, Ws);
    return;
  }
  const int64_t v = xcd * full_per + (l - tail_per);
  if (v >= ntiles * a.split) return;
  const int part = (int)(v / ntiles), tile = (int)(v % ntiles);
  gram_tile<GB>(a, part, (int64_t)(tile / a.nq) * GB, tile % a.nq, As, Ws);
}

// Contraction parts for the untuned FP64 Gram: one when the tiles fill the
// device twice over, else the count from 2..4 that gives the fewest rounds
// of workgroups (two per compute unit) per part, i.e. the shortest time when
// every workgroup takes as long.
int gram_split_for(const Inst& in) {
  int dev = 0, cus = 0;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev);
  if (cus <= 0) cus = 256;
  const int64_t tiles = ceil_div(in.P, GB) * (int64_t)in.nq;
  const int64_t slots = 2 * (int64_t)cus;
  if (tiles >= slots || in.n_h < 4 * GKC) return 1;
  int best = 2;
  for (int parts = 3; parts <= 4; ++parts)
    if (in.n_h >= 2 * parts * GKC &&
        ceil_div(tiles * parts, slots) * best < ceil_div(tiles * best, slots) * parts)
      best = parts;
  return best;
}

int gram_parts_used(const Inst& in) {
  const int want = in.tune_gram_split > 0 ? in.tune_gram_split : gram_split_for(in);
  if (!in.G2) return 1;
  return want - 1 <= in.g2_parts ? want : 1 + in.g2_parts;
}

template <class WS>
static hipError_t run_gram_f64(const Inst& in, WS w, hipStream_t s) {
  GramArgs<WS> a;
  a.S = in.S; a.ldS = in.ldS; a.w = w;
  a.n_h = in.n_h; a.M = in.M; a.P = in.P;
  a.pairs = in.pairs; a.qtiles = in.qtiles;
  // full tiles of 128 pairs; a leftover of at most 32 pairs goes to the tail tiles
  const int64_t rest = in.P % GB;
  a.nfull = (int)(in.P / GB);
  a.tail = rest > 0 && rest <= GBT ? 1 : 0;
  if (rest > GBT) ++a.nfull;
  a.nq = in.nq;
  a.split = gram_parts_used(in);
  a.jlen = round_up(ceil_div(in.n_h, a.split), GKC);
  a.G = in.G; a.G2 = a.split > 1 ? in.G2 : nullptr; a.ldG = in.KMp;
  const int64_t grid = 8 * (ceil_div((int64_t)a.tail * a.nq * a.split, 8) + ceil_div((int64_t)a.nfull * a.nq * a.split, 8));
  hipLaunchKernelGGL(gram_f64_kernel<WS>, dim3((unsigned)grid), dim3(256), 0, s, a);
  return hipGetLastError();
}

hipError_t launch_gram_f64(const Inst& in, hipStream_t s) {
  return in.W ? run_gram_f64(in, wdense(in), s) : run_gram_f64(in, wsep(in), s);
}

// ------------------------------------ padding of the Gram and its diagonal
// Rows/cols KM..KMp-1 become the identity so the blocked factorization can
// run on whole NB blocks; diag0 keeps the pre-factorization diagonal.
__global__ void gram_pad_diag_kernel(double* G, const double* G2, int nextra, int64_t ld, int64_t KM, int64_t KMp,
                                     double* diag0) {
  int64_t c = blockIdx.x;  // column
  if (c >= KM) {
    for (int64_t r = threadIdx.x; r < KMp; r += blockDim.x) G[r + c * ld] = (r == c) ? 1.0 : 0.0;
  } else {
    // the other parts of a split Gram, in part order: lower triangle of this column
    if (nextra > 0)
      for (int64_t r = c + threadIdx.x; r < KM; r += blockDim.x) {
        double v = G[r + c * ld];
        for (int q = 0; q < nextra; ++q) v += G2[(int64_t)q * ld * ld + r + c * ld];
        G[r + c * ld] = v;
      }
    for (int64_t r = KM + threadIdx.x; r < KMp; r += blockDim.x) G[r + c * ld] = 0.0;
  }
  __syncthreads();
  if (threadIdx.x == 0) diag0[c] = (c >= KM) ? 1.0 : G[c + c * ld];
}

hipError_t launch_gram_pad_and_diag(const Inst& in, hipStream_t s) {
  const int parts = gram_parts_used(in);
  hipLaunchKernelGGL(gram_pad_diag_kernel, dim3((unsigned)in.KMp), dim3(256), 0, s, in.G,
                     (const double*)(parts > 1 ? in.G2 : nullptr), parts - 1, in.KMp, in.KM, in.KMp, in.diag0);
  return hipGetLastError();
}

}  // namespace pc
