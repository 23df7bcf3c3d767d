// C-ABI of the library: plan management and the sequencing of the kernels.
// Declarations and the contract of every entry point are in include/pcsqrt.h.
#include "pcsqrt.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdio>
#include <memory>
#include <new>
#include <string>
#include <vector>

#include "pc_internal.h"

using pc::Inst;
using pc::make_qtiles;

namespace pc {
// Mode-pair tiles of the FP64 Gram: each is two 8 x 8 blocks of (m, m')
// (block origins m0, m0'), four ints per tile.  The blocks of the triangle
// m <= m' (8-aligned) are paired along m' within a block row where they can
// be; the diagonal blocks (36 of 64 pairs valid) and the unpaired ones are
// paired with each other; an odd last block is paired with an empty one
// (origin M: every pair skipped).
std::vector<int> make_qtiles(int64_t M) {
  const int nb = (int)((M + 7) / 8);
  std::vector<int> q, rest;
  auto tile = [&](int a0, int b0, int a1, int b1) { q.push_back(a0); q.push_back(b0); q.push_back(a1); q.push_back(b1); };
  for (int a = 0; a < nb; ++a) {
    rest.push_back(a); rest.push_back(a);               // the diagonal block
    int b = a + 1;
    for (; b + 1 < nb; b += 2) tile(8 * a, 8 * b, 8 * a, 8 * b + 8);
    if (b < nb) { rest.push_back(a); rest.push_back(b); }
  }
  for (size_t u = 0; u < rest.size(); u += 4) {
    if (u + 2 < rest.size()) tile(8 * rest[u], 8 * rest[u + 1], 8 * rest[u + 2], 8 * rest[u + 3]);
    else tile(8 * rest[u], 8 * rest[u + 1], (int)M, (int)M);
  }
  return q;
}
}  // namespace pc

// A refinement that stops shrinking is accepted as converged when its last
// relative update is at most this (far below the 1e-8 accuracy target of the
// reduced-precision modes); otherwise the apply reports no convergence.
static constexpr double kStallAccept = 1e-9;

// Grams of order above this are factored by block columns of 1024, each block
// by the tile DAG (the DAG alone has one diagonal step per 64 rows on its
// critical path).  In a plan of several instances the factorizations of all
// of them form one persistent tile-DAG launch, whose chains overlap, up to
// the larger order kBatchDagUpTo.
static constexpr int64_t kBlockedAbove = 8192;
static constexpr int64_t kBatchDagUpTo = 16384;

struct pc_plan {
  std::vector<Inst> inst;
  pc_options opt;
  int device = 0;
  int* d_flag = nullptr;        // device scratch int (finiteness check)
  pc::RefineCtl* h_ctl = nullptr;   // pinned host copies of the refinement controls
  int* h_modes = nullptr;           // pinned: per-instance Gram precision for a batched low-precision launch
  int* h_status = nullptr;          // pinned host copies of each instance's pivot status and error flag,
                                    // then the error flag of a forward pass run during the factorization
  // independent instances run on internal streams (fork/join with the caller's stream)
  std::vector<hipStream_t> aux;
  hipEvent_t ev_fork = nullptr;
  std::vector<hipEvent_t> ev_join;
  // hipGraph of the apply sequence, and the arguments it was captured for
  hipStream_t cap = nullptr;
  hipGraph_t graph = nullptr;
  hipGraphExec_t gexec = nullptr;
  std::vector<int64_t> gkey;
  // hipGraph of the whole factor + apply sequence (pc_factor_apply with a graph)
  hipGraph_t fgraph = nullptr;
  hipGraphExec_t fgexec = nullptr;
  std::vector<int64_t> fgkey;
  // profiling: recorded (start, stop) event pairs per phase, and a pool
  bool profiling = false;
  std::vector<std::pair<hipEvent_t, hipEvent_t>> rec[PC_NUM_PHASES];
  std::vector<hipEvent_t> pool;
  // several instances: one persistent Cholesky launch and one solve pair for all
  pc::DagBatch* batch = nullptr;
  // several instances in reduced precision: their Grams in one launch
  pc::LowGramBatch* lowgram = nullptr;
  // factor-and-apply: the products Z^T x on their own stream during the factorization
  hipStream_t ovl = nullptr;
  hipEvent_t ev_gram = nullptr, ev_reset = nullptr, ev_ztx = nullptr;
};

namespace {

#define PC_TRY(expr)                                    \
  do {                                                  \
    hipError_t e_ = (expr);                             \
    if (e_ != hipSuccess) return PC_ERR_DEVICE;         \
  } while (0)

template <class T>
hipError_t dalloc(T** p, int64_t count) {
  *p = nullptr;
  if (count <= 0) return hipSuccess;
  return hipMalloc((void**)p, sizeof(T) * (size_t)count);
}

void free_inst(Inst& in) {
  hipFree(in.G); hipFree(in.G2); in.G2 = nullptr; in.g2_parts = 0; hipFree(in.diag0); hipFree(in.Linv); hipFree(in.Lt); in.Lt = nullptr; in.lt_tiles = 0; hipFree(in.Msol); in.Msol = nullptr; hipFree(in.S); hipFree(in.pairs);
  hipFree(in.qtiles); hipFree(in.B); hipFree(in.Y); hipFree(in.D); hipFree(in.Rres);
  hipFree(in.info); hipFree(in.ctl); hipFree(in.rhs); hipFree(in.dag);
  hipFree(in.E32); hipFree(in.W32); in.E32 = nullptr; in.W32 = nullptr;
  hipFree(in.lp_tiles); in.lp_tiles = nullptr; in.lp_ntiles = 0; hipFree(in.chol_offs);
  hipFree(in.Gs); hipFree(in.Dinv); hipFree(in.cg); hipFree(in.cgcol); hipFree(in.cg_flags);
  hipFree(in.blk_P); hipFree(in.blk_X); hipFree(in.blk_I); hipFree(in.blk_offs); hipFree(in.blk_offs_tail);
  hipFree(in.cgm_Dinv); hipFree(in.cgm_work); hipFree(in.cgm_I); hipFree(in.cgm_d0); hipFree(in.cgm_Linv);
  hipFree(in.cgm_ctr); hipFree(in.cgm_offs);
  in.cgm_Dinv = in.cgm_work = in.cgm_I = in.cgm_d0 = in.cgm_Linv = nullptr;
  in.cgm_ctr = nullptr; in.cgm_offs = nullptr;
  in.blk_P = in.blk_X = in.blk_I = nullptr; in.blk_offs = in.blk_offs_tail = nullptr;
  in.Gs = in.Dinv = in.cg = nullptr; in.cgcol = nullptr; in.cg_flags = nullptr;
  in.dag = nullptr; in.chol_offs = nullptr; in.ctl = nullptr; in.rhs = nullptr;
  in.G = in.diag0 = in.Linv = in.S = in.B = in.Y = in.D = in.Rres = nullptr;
  in.pairs = in.qtiles = in.info = nullptr;
}

void free_plan(pc_plan* p) {
  if (!p) return;
  hipDeviceSynchronize();
  for (auto& in : p->inst) free_inst(in);
  for (auto& v : p->rec)
    for (auto& e : v) { hipEventDestroy(e.first); hipEventDestroy(e.second); }
  for (auto e : p->pool) hipEventDestroy(e);
  if (p->gexec) hipGraphExecDestroy(p->gexec);
  if (p->graph) hipGraphDestroy(p->graph);
  if (p->fgexec) hipGraphExecDestroy(p->fgexec);
  if (p->fgraph) hipGraphDestroy(p->fgraph);
  if (p->cap) hipStreamDestroy(p->cap);
  if (p->ovl) hipStreamDestroy(p->ovl);
  if (p->ev_gram) hipEventDestroy(p->ev_gram);
  if (p->ev_ztx) hipEventDestroy(p->ev_ztx);
  if (p->ev_reset) hipEventDestroy(p->ev_reset);
  for (auto st : p->aux) hipStreamDestroy(st);
  if (p->ev_fork) hipEventDestroy(p->ev_fork);
  for (auto e : p->ev_join) hipEventDestroy(e);
  hipFree(p->d_flag);
  pc::free_dag_batch(p->batch);
  pc::free_lowgram_batch(p->lowgram);
  if (p->h_ctl) hipHostFree(p->h_ctl);
  if (p->h_status) hipHostFree(p->h_status);
  if (p->h_modes) hipHostFree(p->h_modes);
  delete p;
}


// Room in G2 for the contraction parts 2..parts of a split FP64 Gram.
hipError_t ensure_gram_parts(Inst& in, int parts) {
  if (parts - 1 <= in.g2_parts) return hipSuccess;
  (void)hipFree(in.G2);
  in.G2 = nullptr;
  in.g2_parts = 0;
  const hipError_t e = hipMalloc((void**)&in.G2, sizeof(double) * (size_t)(parts - 1) * (size_t)(in.KMp * in.KMp));
  if (e != hipSuccess) { in.G2 = nullptr; return e; }
  in.g2_parts = parts - 1;
  return hipSuccess;
}

// Final-L tile buffer for a tile DAG of T tile rows (T (T - 1) / 2 tiles).
hipError_t ensure_lt(Inst& in, int64_t T) {
  const int64_t need = T * (T - 1) / 2;
  if (need <= in.lt_tiles) return hipSuccess;
  (void)hipFree(in.Lt);
  in.Lt = nullptr;
  in.lt_tiles = 0;
  const hipError_t e = dalloc(&in.Lt, need * pc::NB * pc::NB);
  if (e == hipSuccess) in.lt_tiles = need;
  return e;
}

// Buffers of the blocked outer factorization with block columns of NO
// (a multiple of 64); NO = 0 frees them (tile DAG only).
pc_status alloc_blocked(Inst& in, int64_t NO) {
  (void)hipFree(in.blk_P); (void)hipFree(in.blk_X); (void)hipFree(in.blk_I);
  (void)hipFree(in.blk_offs); (void)hipFree(in.blk_offs_tail);
  in.blk_P = in.blk_X = in.blk_I = nullptr;
  in.blk_offs = in.blk_offs_tail = nullptr;
  in.blk_NO = 0;
  in.blk_ntasks = in.blk_ntasks_tail = 0;
  if (NO <= 0) return ensure_lt(in, in.KMp / pc::NB) == hipSuccess ? PC_OK : PC_ERR_OOM;
  const int64_t KMp = in.KMp;
  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t x) { if (x != hipSuccess && e == hipSuccess) e = x; };
  chk(dalloc(&in.blk_P, KMp * NO));
  chk(dalloc(&in.blk_X, NO * NO));
  chk(dalloc(&in.blk_I, NO * NO));
  chk(ensure_lt(in, NO / pc::NB));
  std::vector<int64_t> bo;
  in.blk_ntasks = pc::chol_task_offsets((int)(NO / pc::NB), bo);
  chk(dalloc(&in.blk_offs, (int64_t)bo.size()));
  if (e == hipSuccess) chk(hipMemcpy(in.blk_offs, bo.data(), sizeof(int64_t) * bo.size(), hipMemcpyHostToDevice));
  const int64_t tail = KMp % NO;
  if (tail) {
    std::vector<int64_t> bt;
    in.blk_ntasks_tail = pc::chol_task_offsets((int)(tail / pc::NB), bt);
    chk(dalloc(&in.blk_offs_tail, (int64_t)bt.size()));
    if (e == hipSuccess) chk(hipMemcpy(in.blk_offs_tail, bt.data(), sizeof(int64_t) * bt.size(), hipMemcpyHostToDevice));
  }
  if (e == hipSuccess) chk(pc::launch_identity(in.blk_I, NO, nullptr));
  if (e == hipSuccess) chk(hipDeviceSynchronize());
  if (e != hipSuccess) return (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? PC_ERR_OOM : PC_ERR_DEVICE;
  in.blk_NO = NO;
  return PC_OK;
}

pc_status alloc_inst(Inst& in, int precision, int flags, bool batched) {
  const int64_t KMp = in.KMp, nblk = KMp / pc::NB, R = std::max<int64_t>(in.max_rhs, 1);
  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t x) { if (x != hipSuccess && e == hipSuccess) e = x; };
  chk(dalloc(&in.G, KMp * KMp));
  chk(dalloc(&in.diag0, KMp));
  chk(dalloc(&in.Linv, nblk * pc::NB * pc::NB));
  chk(dalloc(&in.Msol, 4 * nblk * pc::NB * pc::NB));
  in.ldS = pc::round_up(in.P, 128);
  chk(dalloc(&in.S, (in.n_h + pc::kGramZeroRows) * in.ldS));
  chk(dalloc(&in.pairs, 2 * in.P));
  std::vector<int> qt = make_qtiles(in.M);
  in.nq = (int)(qt.size() / 4);
  chk(dalloc(&in.qtiles, (int64_t)qt.size()));
  chk(dalloc(&in.B, KMp * R));
  chk(dalloc(&in.Y, KMp * R));
  chk(dalloc(&in.D, KMp * R));
  chk(dalloc(&in.Rres, in.n * R));
  chk(dalloc(&in.info, 1));
  chk(dalloc(&in.ctl, 1));
  chk(dalloc(&in.rhs, R));
  if (precision != PC_PREC_FP64) {
    const std::vector<int> order = pc::lowgram_tile_order(in.KM, in.M);
    in.lp_ntiles = (int64_t)(order.size() / 2);
    chk(dalloc(&in.lp_tiles, (int64_t)order.size()));
    if (e == hipSuccess) chk(hipMemcpy(in.lp_tiles, order.data(), sizeof(int) * order.size(), hipMemcpyHostToDevice));
  }
  if (precision == PC_PREC_BF16_REFINE || precision == PC_PREC_BF16X3_REFINE) {
    in.ldE32 = pc::round_up(in.n, pc::kLowRowPad);
    in.ldW32 = pc::round_up(in.n_h, pc::kLowRowPad);
    chk(dalloc(&in.E32, in.ldE32 * (in.K + 1)));
    chk(dalloc(&in.W32, in.ldW32 * in.M));
    if (e == hipSuccess) chk(hipMemset(in.E32, 0, sizeof(float) * in.ldE32 * (in.K + 1)));
    if (e == hipSuccess) chk(hipMemset(in.W32, 0, sizeof(float) * in.ldW32 * in.M));
  }
  in.rhs_host.assign((size_t)R, pc::RhsCtl{});
  const int64_t T = KMp / pc::NB;
  in.nrt_max = (int)pc::ceil_div(R, pc::NB);
  // counters: Cholesky states, head, error, solve flags, solve head, and the
  // error flag of a forward pass run during the factorization; the blocked
  // factorization reuses them for a diagonal block and its inverse (2 T^2 + 3)
  chk(dalloc(&in.dag, std::max<int64_t>(T * T + 2 + T * in.nrt_max + 2, 2 * T * T + 3)));
  std::vector<int64_t> offs;
  in.chol_ntasks = pc::chol_task_offsets((int)T, offs);
  chk(dalloc(&in.chol_offs, (int64_t)offs.size()));
  if (KMp > (batched ? kBatchDagUpTo : kBlockedAbove) && e == hipSuccess) {
    const pc_status bs = alloc_blocked(in, 1024);
    if (bs != PC_OK) return bs;
  } else {
    chk(ensure_lt(in, T));
  }
  if (flags & PC_FLAG_CG_MEMBER_BLOCKS) {
    const int64_t Mp = pc::round_up(in.M, pc::NB), Tb = Mp / pc::NB;
    in.cgm_Mp = Mp;
    chk(dalloc(&in.cgm_Dinv, in.K * Mp * Mp));
    chk(dalloc(&in.cgm_work, 2 * Mp * Mp));
    chk(dalloc(&in.cgm_I, Mp * Mp));
    chk(dalloc(&in.cgm_d0, Mp));
    chk(dalloc(&in.cgm_Linv, Tb * pc::NB * pc::NB));
    chk(dalloc(&in.cgm_ctr, 2 * Tb * Tb + 3));
    std::vector<int64_t> mo;
    in.cgm_ntasks = pc::chol_task_offsets((int)Tb, mo);
    chk(dalloc(&in.cgm_offs, (int64_t)mo.size()));
    if (e == hipSuccess) chk(hipMemcpy(in.cgm_offs, mo.data(), sizeof(int64_t) * mo.size(), hipMemcpyHostToDevice));
    if (e == hipSuccess) chk(pc::launch_identity(in.cgm_I, Mp, nullptr));
    if (e == hipSuccess) chk(hipDeviceSynchronize());
  }
  if (flags & PC_FLAG_KEEP_GRAM) {
    chk(dalloc(&in.Gs, KMp * KMp));
    chk(dalloc(&in.Dinv, KMp * pc::NB));
    chk(dalloc(&in.cg, 4 * KMp * R));
    chk(dalloc(&in.cgcol, R));
    chk(dalloc(&in.cg_flags, 2));
  }
  if (e != hipSuccess) return (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? PC_ERR_OOM : PC_ERR_DEVICE;
  if (hipMemcpy(in.qtiles, qt.data(), qt.size() * sizeof(int), hipMemcpyHostToDevice) != hipSuccess)
    return PC_ERR_DEVICE;
  if (hipMemcpy(in.chol_offs, offs.data(), offs.size() * sizeof(int64_t), hipMemcpyHostToDevice) != hipSuccess)
    return PC_ERR_DEVICE;
  // padding rows of the right-hand-side buffers stay zero forever
  if (hipMemset(in.B, 0, sizeof(double) * KMp * R) != hipSuccess) return PC_ERR_DEVICE;
  // S padding columns (pairs P..ldS-1) and the rows past n_h are read by the
  // Gram tiles and must be zero
  if (hipMemset(in.S, 0, sizeof(double) * (in.n_h + pc::kGramZeroRows) * in.ldS) != hipSuccess) return PC_ERR_DEVICE;
  if (precision == PC_PREC_FP64 && pc::gram_split_for(in) > 1) {
    if (ensure_gram_parts(in, pc::gram_split_for(in)) != hipSuccess) return PC_ERR_OOM;
  }
  if (hipMemset(in.Y, 0, sizeof(double) * KMp * R) != hipSuccess) return PC_ERR_DEVICE;
  if (hipMemset(in.D, 0, sizeof(double) * KMp * R) != hipSuccess) return PC_ERR_DEVICE;
  return PC_OK;
}

bool ok_ptr(const void* ptr) { return ptr != nullptr; }

hipEvent_t take_event(pc_plan* p) {
  if (!p->pool.empty()) { hipEvent_t e = p->pool.back(); p->pool.pop_back(); return e; }
  hipEvent_t e = nullptr;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}

// Records an event pair around a phase when profiling is on.
struct PhaseTimer {
  pc_plan* p; int phase; hipStream_t s; hipEvent_t a = nullptr;
  PhaseTimer(pc_plan* p_, int ph, hipStream_t s_) : p(p_), phase(ph), s(s_) {
    if (p->profiling && (a = take_event(p))) hipEventRecord(a, s);
  }
  ~PhaseTimer() {
    if (!a) return;
    hipEvent_t b = take_event(p);
    if (!b) { p->pool.push_back(a); return; }
    hipEventRecord(b, s);
    p->rec[phase].push_back({a, b});
  }
};

hipStream_t stream_for(const pc_plan* p, size_t i, hipStream_t caller) {
  return p->aux.empty() ? caller : p->aux[i % p->aux.size()];
}

// Make the internal streams wait for the caller's stream, and back.
hipError_t fork(pc_plan* p, hipStream_t s) {
  if (p->aux.empty()) return hipSuccess;
  hipError_t e = hipEventRecord(p->ev_fork, s);
  for (auto st : p->aux)
    if (e == hipSuccess) e = hipStreamWaitEvent(st, p->ev_fork, 0);
  return e;
}

hipError_t join(pc_plan* p, hipStream_t s) {
  hipError_t e = hipSuccess;
  for (size_t j = 0; j < p->aux.size() && e == hipSuccess; ++j) {
    e = hipEventRecord(p->ev_join[j], p->aux[j]);
    if (e == hipSuccess) e = hipStreamWaitEvent(s, p->ev_join[j], 0);
  }
  return e;
}

// The Gram of one instance in its current precision (FP64 structured Gram,
// or the Gram of the rounded Z formed inside the low-precision kernel).
pc_status assemble_one(pc_plan* p, Inst& in, hipStream_t s) {
  in.factored = false;
  PC_TRY(pc::launch_fill_int(in.info, -1, 1, s));
  if (in.prec == PC_PREC_FP64) {
    { PhaseTimer t(p, PC_PHASE_COLUMN_GRAMS, s); PC_TRY(pc::launch_column_grams(in, s)); }
    { PhaseTimer t(p, PC_PHASE_GRAM, s); PC_TRY(pc::launch_gram_f64(in, s)); }
  } else {
    PhaseTimer t(p, PC_PHASE_GRAM, s);
    if (in.prec != PC_PREC_FP32_REFINE) PC_TRY(pc::launch_stage_f32(in, s));
    PC_TRY(pc::launch_gram_lowprec(in, in.prec, s));
  }
  { PhaseTimer t(p, PC_PHASE_PAD, s); PC_TRY(pc::launch_gram_pad_and_diag(in, s)); }
  return PC_OK;
}

// Grams of a batch in reduced precision: the instances of each reduced
// precision in one launch (tiles of all of them, longest contraction first),
// instances raised to FP64 by the ladder on the internal streams, then the
// padding per stream.
pc_status assemble_lowgram_batch(pc_plan* p, hipStream_t s) {
  bool used[4] = {false, false, false, false};
  for (size_t i = 0; i < p->inst.size(); ++i) {
    p->h_modes[i] = p->inst[i].prec;
    used[p->inst[i].prec] = true;
  }
  PC_TRY(pc::set_lowgram_modes(p->lowgram, p->h_modes, s));
  PC_TRY(fork(p, s));
  for (size_t i = 0; i < p->inst.size(); ++i) {
    Inst& in = p->inst[i];
    hipStream_t si = stream_for(p, i, s);
    in.factored = false;
    PC_TRY(pc::launch_fill_int(in.info, -1, 1, si));
    if (in.prec == PC_PREC_FP64) {
      PC_TRY(pc::launch_column_grams(in, si));
      PC_TRY(pc::launch_gram_f64(in, si));
    } else if (in.prec != PC_PREC_FP32_REFINE) {
      PC_TRY(pc::launch_stage_f32(in, si));
    }
  }
  PC_TRY(join(p, s));
  {
    PhaseTimer t(p, PC_PHASE_GRAM, s);
    for (int prec : {PC_PREC_BF16_REFINE, PC_PREC_BF16X3_REFINE, PC_PREC_FP32_REFINE})
      if (used[prec]) PC_TRY(pc::launch_gram_lowprec_batch(p->lowgram, prec, s));
  }
  PC_TRY(fork(p, s));
  for (size_t i = 0; i < p->inst.size(); ++i) {
    Inst& in = p->inst[i];
    hipStream_t si = stream_for(p, i, s);
    PhaseTimer t(p, PC_PHASE_PAD, si);
    PC_TRY(pc::launch_gram_pad_and_diag(in, si));
  }
  PC_TRY(join(p, s));
  return PC_OK;
}

// The precision ladder: the next, more accurate Gram after `prec`
// (bf16 -> split bf16 -> fp32 -> FP64), or -1 at the top.
int next_rung(int prec) {
  switch (prec) {
    case PC_PREC_BF16_REFINE: return PC_PREC_BF16X3_REFINE;
    case PC_PREC_BF16X3_REFINE: return PC_PREC_FP32_REFINE;
    case PC_PREC_FP32_REFINE: return PC_PREC_FP64;
    default: return -1;
  }
}

// b = Z^T x, the first right-hand side of the normal equations: with the
// reduced-precision operands the plan's flags ask for while the instance is
// on a reduced-precision rung, else FP64.
hipError_t launch_first_ztx(const pc_plan* p, const Inst& in, const double* X, int64_t ldX, int64_t R, double* B,
                            int64_t ldB, hipStream_t s) {
  const int f = p->opt.flags;
  if (in.prec != PC_PREC_FP64 && (f & (PC_FLAG_ZTX_FP32 | PC_FLAG_ZTX_BF16)))
    return pc::launch_ztx_lowprec(in, (f & PC_FLAG_ZTX_FP32) ? PC_PREC_FP32_REFINE : PC_PREC_BF16_REFINE, X, ldX,
                                  R, B, ldB, s);
  return pc::launch_ztx(in, X, ldX, R, B, ldB, s);
}

bool ladder_on(const pc_plan* p) { return !(p->opt.flags & PC_FLAG_FIXED_PRECISION); }

// The apply sequence of every instance on the streams (no host wait when
// check_every == 0; otherwise the host stops early once every instance's
// refinement is done, checking every `check_every` iterations).
pc_status enqueue_apply_batched(pc_plan* p, const double* const* X, const int64_t* ldX, const int64_t* R,
                                double* const* Y, const int64_t* ldY, hipStream_t s, int check_every);

// done_ahead: 0, or 1 when b = Z^T x is already in in.Y, or 2 when the
// forward pass of the first solve is also done (in in.B).
// force_single: the per-instance path even for a batched plan (the ladder's
// re-solve of a few instances).
pc_status enqueue_apply(pc_plan* p, const double* const* X, const int64_t* ldX, const int64_t* R,
                        double* const* Y, const int64_t* ldY, hipStream_t s, int check_every,
                        int done_ahead = 0, bool force_single = false) {
  if (p->batch && !force_single) return enqueue_apply_batched(p, X, ldX, R, Y, ldY, s, check_every);
  const size_t cnt = p->inst.size();
  const int budget = p->opt.max_refine;
  PC_TRY(fork(p, s));
  for (size_t i = 0; i < cnt; ++i) {
    Inst& in = p->inst[i];
    if (R[i] == 0) continue;
    hipStream_t si = stream_for(p, i, s);
    if (done_ahead < 1) {
      PhaseTimer t(p, PC_PHASE_ZTX, si);
      PC_TRY(launch_first_ztx(p, in, X[i], ldX[i], R[i], in.Y, in.KMp, si));
    }
    {
      PhaseTimer t(p, PC_PHASE_SOLVE, si);
      PC_TRY(pc::launch_chol_solve(in, in.Y, in.KMp, R[i], in.B, in.KMp, si, nullptr, done_ahead >= 2 ? 1 : 0));
    }
    PC_TRY(pc::launch_refine_init(in.ctl, in.rhs, R[i], budget, si));
  }
  // refinement on the least-squares residual: r = x - Z y, d = G^{-1} Z^T r, y += d;
  // converged instances skip the remaining iterations on the GPU
  std::unique_ptr<PhaseTimer> refine_timer;
  if (budget > 0) refine_timer.reset(new PhaseTimer(p, PC_PHASE_REFINE, s));
  for (int it = 1; it <= budget; ++it) {
    for (size_t i = 0; i < cnt; ++i) {
      Inst& in = p->inst[i];
      if (R[i] == 0) continue;
      hipStream_t si = stream_for(p, i, s);
      const int* skip = &in.ctl->done;
      PC_TRY(pc::launch_zy(in, in.Y, in.KMp, R[i], X[i], ldX[i], in.Rres, in.n, si, skip));
      PC_TRY(pc::launch_ztx(in, in.Rres, in.n, R[i], in.D, in.KMp, si, skip));
      PC_TRY(pc::launch_chol_solve(in, in.D, in.KMp, R[i], in.B, in.KMp, si, skip));
      PC_TRY(pc::launch_refine_update(in, in.Y, in.KMp, in.D, in.KMp, R[i], in.ctl, p->opt.tol, kStallAccept, si));
      PC_TRY(pc::launch_refine_check(in.ctl, si));
    }
    if (check_every > 0 && it % check_every == 0 && it < budget) {
      bool all = true;
      for (size_t i = 0; i < cnt; ++i) {
        if (R[i] == 0) continue;
        hipStream_t si = stream_for(p, i, s);
        PC_TRY(hipMemcpyAsync(&p->h_ctl[i], p->inst[i].ctl, sizeof(pc::RefineCtl), hipMemcpyDeviceToHost, si));
      }
      for (size_t i = 0; i < cnt; ++i)
        if (R[i] != 0) PC_TRY(hipStreamSynchronize(stream_for(p, i, s)));
      for (size_t i = 0; i < cnt; ++i)
        if (R[i] != 0 && p->h_ctl[i].done == 0) all = false;
      if (all) break;
    }
  }
  refine_timer.reset();
  {
    PhaseTimer copy_timer(p, PC_PHASE_COPYOUT, s);
    for (size_t i = 0; i < cnt; ++i) {
      Inst& in = p->inst[i];
      if (R[i] == 0) continue;
      PC_TRY(pc::launch_copy_rows(in.Y, in.KMp, Y[i], ldY[i], in.KM, in.KM, R[i], stream_for(p, i, s)));
    }
  }
  PC_TRY(join(p, s));
  return PC_OK;
}


// The apply sequence with every instance's solves in one batched launch pair:
// per-instance products on the internal streams, joined before each solve.
pc_status enqueue_apply_batched(pc_plan* p, const double* const* X, const int64_t* ldX, const int64_t* R,
                                double* const* Y, const int64_t* ldY, hipStream_t s, int check_every) {
  const size_t cnt = p->inst.size();
  const int budget = p->opt.max_refine;
  PC_TRY(fork(p, s));
  for (size_t i = 0; i < cnt; ++i) {
    Inst& in = p->inst[i];
    if (R[i] == 0) continue;
    hipStream_t si = stream_for(p, i, s);
    PhaseTimer t(p, PC_PHASE_ZTX, si);
    PC_TRY(launch_first_ztx(p, in, X[i], ldX[i], R[i], in.Y, in.KMp, si));
  }
  PC_TRY(join(p, s));
  PC_TRY(pc::set_batch_rhs(p->batch, R, s));
  { PhaseTimer t(p, PC_PHASE_SOLVE, s); PC_TRY(pc::launch_chol_solve_batch(p->batch, 0, s)); }
  PC_TRY(fork(p, s));
  for (size_t i = 0; i < cnt; ++i)
    if (R[i] != 0) PC_TRY(pc::launch_refine_init(p->inst[i].ctl, p->inst[i].rhs, R[i], budget, stream_for(p, i, s)));
  std::unique_ptr<PhaseTimer> refine_timer;
  if (budget > 0) refine_timer.reset(new PhaseTimer(p, PC_PHASE_REFINE, s));
  for (int it = 1; it <= budget; ++it) {
    for (size_t i = 0; i < cnt; ++i) {
      Inst& in = p->inst[i];
      if (R[i] == 0) continue;
      hipStream_t si = stream_for(p, i, s);
      const int* skip = &in.ctl->done;
      PC_TRY(pc::launch_zy(in, in.Y, in.KMp, R[i], X[i], ldX[i], in.Rres, in.n, si, skip));
      PC_TRY(pc::launch_ztx(in, in.Rres, in.n, R[i], in.D, in.KMp, si, skip));
    }
    PC_TRY(join(p, s));
    PC_TRY(pc::launch_chol_solve_batch(p->batch, 1, s));
    PC_TRY(fork(p, s));
    for (size_t i = 0; i < cnt; ++i) {
      Inst& in = p->inst[i];
      if (R[i] == 0) continue;
      hipStream_t si = stream_for(p, i, s);
      PC_TRY(pc::launch_refine_update(in, in.Y, in.KMp, in.D, in.KMp, R[i], in.ctl, p->opt.tol, kStallAccept, si));
      PC_TRY(pc::launch_refine_check(in.ctl, si));
    }
    if (check_every > 0 && it % check_every == 0 && it < budget) {
      for (size_t i = 0; i < cnt; ++i)
        if (R[i] != 0)
          PC_TRY(hipMemcpyAsync(&p->h_ctl[i], p->inst[i].ctl, sizeof(pc::RefineCtl), hipMemcpyDeviceToHost,
                                stream_for(p, i, s)));
      for (size_t j = 0; j < p->aux.size(); ++j) PC_TRY(hipStreamSynchronize(p->aux[j]));
      bool all = true;
      for (size_t i = 0; i < cnt; ++i)
        if (R[i] != 0 && p->h_ctl[i].done == 0) all = false;
      if (all) break;
    }
  }
  refine_timer.reset();
  {
    PhaseTimer copy_timer(p, PC_PHASE_COPYOUT, s);
    for (size_t i = 0; i < cnt; ++i) {
      Inst& in = p->inst[i];
      if (R[i] == 0) continue;
      PC_TRY(pc::launch_copy_rows(in.Y, in.KMp, Y[i], ldY[i], in.KM, in.KM, R[i], stream_for(p, i, s)));
    }
  }
  PC_TRY(join(p, s));
  return PC_OK;
}


// CG on G y = b on the plan's KMp-row buffers of one instance.  On entry
// in.Y holds the start (rows >= KM zero) when warm, b is read from Bm (KM
// rows).  Runs at most maxiter iterations, checking every 8 whether every
// column converged.  Returns the largest iteration count in *iters and
// whether every column converged in *all_ok.
pc_status run_cg(pc_plan* p, Inst& in, const double* Bm, int64_t ldB, int64_t R, bool warm, double tol,
                 int maxiter, hipStream_t s, int* iters, bool* all_ok) {
  const int64_t KMp = in.KMp, ld = KMp, T = KMp / pc::NB, mr = std::max<int64_t>(in.max_rhs, 1);
  double* r = in.cg;
  double* z = in.cg + ld * mr;
  double* pv = in.cg + 2 * ld * mr;
  double* q = in.cg + 3 * ld * mr;
  PC_TRY(pc::launch_fill_int(in.cg_flags, 0, 1, s));
  if (warm) PC_TRY(pc::launch_gram_matmul(in.Gs, KMp, in.Y, q, ld, R, s));
  PC_TRY(pc::launch_cg_start(Bm, ldB, warm ? q : nullptr, r, in.Y, ld, ld, in.KM, KMp, R, tol, in.cgcol,
                             in.cg_flags, s));
  // preconditioner: the factor of the plan's reduced-precision Gram
  // (z = Lt^{-T} Lt^{-1} r), or the inverses of the member blocks, or of the
  // 64 x 64 diagonal blocks of the FP64 Gram
  const bool factor_pre = in.prec != PC_PREC_FP64;
  auto precond = [&]() -> hipError_t {
    if (factor_pre) {
      hipError_t e = pc::launch_copy_rows(r, ld, z, ld, KMp, KMp, R, s);
      return e != hipSuccess ? e : pc::launch_chol_solve(in, z, ld, R, in.D, KMp, s);
    }
    return in.cgm_Dinv ? pc::launch_member_apply(in.cgm_Dinv, in.K, in.M, in.cgm_Mp, r, z, ld, R, s)
                       : pc::launch_bj_apply(in.Dinv, T, r, z, ld, R, s);
  };
  if (in.cgm_Dinv && !factor_pre) PC_TRY(pc::launch_zero_rows(z, ld, in.KM, KMp, R, s));   // padding rows stay zero
  PC_TRY(precond());
  PC_TRY(pc::launch_cg_dir(r, z, pv, ld, KMp, R, in.cgcol, 1, s));
  int ndone = 0;
  for (int it = 1; it <= maxiter; ++it) {
    PC_TRY(pc::launch_gram_matmul(in.Gs, KMp, pv, q, ld, R, s));
    PC_TRY(pc::launch_cg_step(pv, q, in.Y, ld, r, ld, KMp, R, tol, in.cgcol, in.cg_flags, it, s));
    if (it % 8 == 0 || it == maxiter) {
      PC_TRY(hipMemcpyAsync(&ndone, in.cg_flags, sizeof(int), hipMemcpyDeviceToHost, s));
      PC_TRY(hipStreamSynchronize(s));
      if (ndone >= R) break;
    }
    PC_TRY(precond());
    PC_TRY(pc::launch_cg_dir(r, z, pv, ld, KMp, R, in.cgcol, 0, s));
  }
  std::vector<pc::CgCol> cols((size_t)R);
  PC_TRY(hipMemcpyAsync(cols.data(), in.cgcol, sizeof(pc::CgCol) * (size_t)R, hipMemcpyDeviceToHost, s));
  PC_TRY(hipStreamSynchronize(s));
  *iters = 0;
  *all_ok = true;
  for (const auto& c : cols) {
    *iters = std::max(*iters, c.iters);
    if (c.done != 1) *all_ok = false;
  }
  (void)p;
  return PC_OK;
}


// ------------------------------------------------------------- autotuning
// Tuning cache: a text file with one line per instance shape,
//   n_h n_w K M max_rhs precision  gram_split ztx_split chol_per_cu chol_block gemm_tile
// after a first line naming the format.
const char* kTuneHeader = "pcsqrt-tune-v2";

struct TuneKey {
  int64_t n_h, n_w, K, M, rhs;
  int prec;
  bool operator==(const TuneKey& o) const {
    return n_h == o.n_h && n_w == o.n_w && K == o.K && M == o.M && rhs == o.rhs && prec == o.prec;
  }
};
struct TuneEntry { TuneKey key; int gram_split, ztx_split, chol_per_cu, chol_block, gemm_tile; };

std::vector<TuneEntry> read_tune_cache(const char* path) {
  std::vector<TuneEntry> v;
  if (!path) return v;
  FILE* f = std::fopen(path, "r");
  if (!f) return v;
  char head[64] = {0};
  if (std::fscanf(f, "%63s", head) == 1 && std::string(head) == kTuneHeader) {
    TuneEntry e;
    long long a, b, c, d, r;
    int pr, g, z, ch, cb, gt;
    while (std::fscanf(f, "%lld %lld %lld %lld %lld %d %d %d %d %d %d", &a, &b, &c, &d, &r, &pr, &g, &z, &ch, &cb,
                       &gt) == 11) {
      e.key = TuneKey{a, b, c, d, r, pr};
      e.gram_split = g; e.ztx_split = z; e.chol_per_cu = ch; e.chol_block = cb; e.gemm_tile = gt;
      v.push_back(e);
    }
  }
  std::fclose(f);
  return v;
}

bool write_tune_cache(const char* path, const std::vector<TuneEntry>& v) {
  const std::string tmp = std::string(path) + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (!f) return false;
  std::fprintf(f, "%s\n", kTuneHeader);
  for (const auto& e : v)
    std::fprintf(f, "%lld %lld %lld %lld %lld %d %d %d %d %d %d\n", (long long)e.key.n_h, (long long)e.key.n_w,
                 (long long)e.key.K, (long long)e.key.M, (long long)e.key.rhs, e.key.prec, e.gram_split, e.ztx_split,
                 e.chol_per_cu, e.chol_block, e.gemm_tile);
  const bool ok = std::fclose(f) == 0;
  return ok && std::rename(tmp.c_str(), path) == 0;
}

// Mean milliseconds of `reps` runs of fn on stream s (after one untimed run
// when `warm`).
template <class F>
pc_status time_ms(hipStream_t s, int reps, F&& fn, float* out, bool warm = true) {
  hipEvent_t a = nullptr, b = nullptr;
  if (hipEventCreate(&a) != hipSuccess || hipEventCreate(&b) != hipSuccess) return PC_ERR_DEVICE;
  pc_status st = warm ? fn() : PC_OK;
  float total = 0.f;
  for (int r = 0; r < reps && st == PC_OK; ++r) {
    if (hipEventRecord(a, s) != hipSuccess) st = PC_ERR_DEVICE;
    if (st == PC_OK) st = fn();
    if (st == PC_OK && (hipEventRecord(b, s) != hipSuccess || hipEventSynchronize(b) != hipSuccess)) st = PC_ERR_DEVICE;
    float ms = 0.f;
    if (st == PC_OK && hipEventElapsedTime(&ms, a, b) != hipSuccess) st = PC_ERR_DEVICE;
    total += ms;
  }
  (void)hipEventDestroy(a);
  (void)hipEventDestroy(b);
  *out = total / (float)std::max(reps, 1);
  return st;
}
}  // namespace

extern "C" {

const char* pc_status_string(pc_status s) {
  switch (s) {
    case PC_OK: return "ok";
    case PC_ERR_INVALID_ARG: return "invalid argument";
    case PC_ERR_SHAPE: return "invalid shape (sizes must be >= 1 and K*M <= n_h*n_w)";
    case PC_ERR_NONFINITE: return "non-finite value in E or W";
    case PC_ERR_NOT_SPD: return "Gram not positive definite: Z is rank deficient";
    case PC_ERR_NOT_FACTORED: return "plan has no valid factorization";
    case PC_ERR_NO_CONVERGENCE: return "iterative refinement did not converge";
    case PC_ERR_OOM: return "device out of memory";
    case PC_ERR_DEVICE: return "HIP runtime error";
    case PC_ERR_TOO_MANY_RHS: return "more right-hand sides than max_rhs";
    case PC_ERR_WORKSPACE: return "problem too large for the fixed workspace of the allocation-free entry point";
  }
  return "unknown status";
}

// Options as given (NULL: FP64 defaults), validated.
static pc_status checked_options(const pc_options* opt, pc_options* o) {
  *o = pc_options{PC_PREC_FP64, 0, 1e-12, 0, 0};
  if (opt) *o = *opt;
  if (o->precision < PC_PREC_FP64 || o->precision > PC_PREC_BF16X3_REFINE || o->max_refine < 0 ||
      (o->flags & ~(PC_FLAG_KEEP_GRAM | PC_FLAG_CG_MEMBER_BLOCKS | PC_FLAG_FIXED_PRECISION | PC_FLAG_ZTX_FP32 |
                    PC_FLAG_ZTX_BF16)) != 0 ||
      ((o->flags & PC_FLAG_ZTX_FP32) && (o->flags & PC_FLAG_ZTX_BF16)) ||
      !std::isfinite(o->tol))
    return PC_ERR_INVALID_ARG;
  if ((o->flags & PC_FLAG_CG_MEMBER_BLOCKS) && !(o->flags & PC_FLAG_KEEP_GRAM)) return PC_ERR_INVALID_ARG;
  if (o->tol <= 0) o->tol = 1e-12;
  return PC_OK;
}

// A plan over instances whose sizes, E and modes (dense W, or separable U and
// Phi) are set and validated: allocation, streams, batches, finiteness of
// the inputs, pair tables.
static pc_status build_plan(const std::vector<Inst>& descs, const pc_options& o, hipStream_t s, pc_plan** out) {
  const int32_t count = (int32_t)descs.size();
  pc_plan* p = new (std::nothrow) pc_plan();
  if (!p) return PC_ERR_OOM;
  p->opt = o;
  hipGetDevice(&p->device);
  pc_status st = PC_OK;
  if (hipMalloc((void**)&p->d_flag, sizeof(int)) != hipSuccess) st = PC_ERR_OOM;
  for (int32_t i = 0; i < count && st == PC_OK; ++i) {
    Inst in = descs[i];
    in.n = in.n_h * in.n_w; in.KM = in.K * in.M; in.KMp = pc::round_up(in.KM, pc::NB);
    in.P = in.K * (in.K + 1) / 2;
    in.prec = o.precision;
    p->inst.push_back(in);
    st = alloc_inst(p->inst.back(), o.precision, o.flags, count > 1);
  }
  if (st == PC_OK && hipHostMalloc((void**)&p->h_ctl, sizeof(pc::RefineCtl) * (size_t)count) != hipSuccess)
    st = PC_ERR_OOM;
  if (st == PC_OK && hipHostMalloc((void**)&p->h_status, sizeof(int) * (2 * (size_t)count + 1)) != hipSuccess)
    st = PC_ERR_OOM;
  if (st == PC_OK && hipHostMalloc((void**)&p->h_modes, sizeof(int) * (size_t)count) != hipSuccess)
    st = PC_ERR_OOM;
  if (st == PC_OK && count > 1) {
    // default-priority streams for independent instances
    const int ns = std::min<int>(count, 8);
    for (int j = 0; j < ns && st == PC_OK; ++j) {
      hipStream_t st_ = nullptr;
      hipEvent_t ev = nullptr;
      if (hipStreamCreateWithFlags(&st_, hipStreamNonBlocking) != hipSuccess ||
          hipEventCreateWithFlags(&ev, hipEventDisableTiming) != hipSuccess) st = PC_ERR_DEVICE;
      p->aux.push_back(st_);
      p->ev_join.push_back(ev);
    }
    if (st == PC_OK && hipEventCreateWithFlags(&p->ev_fork, hipEventDisableTiming) != hipSuccess) st = PC_ERR_DEVICE;
  }
  if (st == PC_OK && o.use_graph && hipStreamCreateWithFlags(&p->cap, hipStreamNonBlocking) != hipSuccess)
    st = PC_ERR_DEVICE;
  bool any_blocked = false;
  for (auto& in : p->inst) any_blocked = any_blocked || in.blk_NO > 0;
  if (st == PC_OK && count > 1 && !any_blocked && !(p->batch = pc::make_dag_batch(p->inst))) st = PC_ERR_OOM;
  if (st == PC_OK && p->batch && o.precision != PC_PREC_FP64 && !(o.flags & PC_FLAG_KEEP_GRAM) &&
      !(p->lowgram = pc::make_lowgram_batch(p->inst)))
    st = PC_ERR_OOM;
  if (st == PC_OK) {
    // finiteness of E and of the modes (W, or its factors U and Phi), then the pair tables
    int bad = 0;
    if (hipMemsetAsync(p->d_flag, 0, sizeof(int), s) != hipSuccess) st = PC_ERR_DEVICE;
    for (auto& in : p->inst) {
      if (st != PC_OK) break;
      hipError_t e = pc::launch_nonfinite_check(in.E, in.ldE, in.n, in.K, p->d_flag, s);
      if (in.W) {
        if (e == hipSuccess) e = pc::launch_nonfinite_check(in.W, in.ldW, in.n_h, in.M, p->d_flag, s);
      } else {
        if (e == hipSuccess) e = pc::launch_nonfinite_check(in.U, in.ldU, in.n_h / in.n_lon, in.M, p->d_flag, s);
        if (e == hipSuccess) e = pc::launch_nonfinite_check(in.Phi, in.ldPhi, in.n_lon, in.M, p->d_flag, s);
      }
      if (e == hipSuccess) e = pc::launch_pairs_init(in, s);
      if (e != hipSuccess) st = PC_ERR_DEVICE;
    }
    if (st == PC_OK && (hipMemcpyAsync(&bad, p->d_flag, sizeof(int), hipMemcpyDeviceToHost, s) != hipSuccess ||
                        hipStreamSynchronize(s) != hipSuccess))
      st = PC_ERR_DEVICE;
    if (st == PC_OK && bad) st = PC_ERR_NONFINITE;
  }
  if (st != PC_OK) {
    free_plan(p);
    return st;
  }
  *out = p;
  return PC_OK;
}

pc_status pc_sqrt_build(const pc_instance* inst, int32_t count, const pc_options* opt, void* stream,
                        pc_plan** out) {
  if (!out) return PC_ERR_INVALID_ARG;
  *out = nullptr;
  if (!inst || count <= 0) return PC_ERR_INVALID_ARG;
  pc_options o;
  const pc_status os = checked_options(opt, &o);
  if (os != PC_OK) return os;
  std::vector<Inst> descs;
  for (int32_t i = 0; i < count; ++i) {
    const pc_instance& a = inst[i];
    if (a.n_h < 1 || a.n_w < 1 || a.K < 1 || a.M < 1) return PC_ERR_SHAPE;
    if (a.K * a.M > a.n_h * a.n_w) return PC_ERR_SHAPE;
    if (!ok_ptr(a.E) || !ok_ptr(a.W)) return PC_ERR_INVALID_ARG;
    if (a.ldE < a.n_h * a.n_w || a.ldW < a.n_h || a.max_rhs < 0) return PC_ERR_INVALID_ARG;
    Inst in;
    in.n_h = a.n_h; in.n_w = a.n_w; in.K = a.K; in.M = a.M;
    in.E = a.E; in.ldE = a.ldE; in.W = a.W; in.ldW = a.ldW; in.max_rhs = a.max_rhs;
    descs.push_back(in);
  }
  return build_plan(descs, o, (hipStream_t)stream, out);
}

pc_status pc_sqrt_build_separable(const pc_instance_separable* inst, int32_t count, const pc_options* opt,
                                  void* stream, pc_plan** out) {
  if (!out) return PC_ERR_INVALID_ARG;
  *out = nullptr;
  if (!inst || count <= 0) return PC_ERR_INVALID_ARG;
  pc_options o;
  const pc_status os = checked_options(opt, &o);
  if (os != PC_OK) return os;
  std::vector<Inst> descs;
  for (int32_t i = 0; i < count; ++i) {
    const pc_instance_separable& a = inst[i];
    if (a.n_lat < 1 || a.n_lon < 1 || a.n_w < 1 || a.K < 1 || a.M < 1) return PC_ERR_SHAPE;
    const int64_t n_h = a.n_lat * a.n_lon;
    if (a.K * a.M > n_h * a.n_w || n_h * a.n_w >= ((int64_t)1 << 40)) return PC_ERR_SHAPE;
    if (!ok_ptr(a.E) || !ok_ptr(a.U) || !ok_ptr(a.Phi)) return PC_ERR_INVALID_ARG;
    if (a.ldE < n_h * a.n_w || a.ldU < a.n_lat || a.ldPhi < a.n_lon || a.max_rhs < 0) return PC_ERR_INVALID_ARG;
    Inst in;
    in.n_h = n_h; in.n_w = a.n_w; in.K = a.K; in.M = a.M;
    in.E = a.E; in.ldE = a.ldE; in.W = nullptr; in.ldW = 0; in.max_rhs = a.max_rhs;
    in.U = a.U; in.ldU = a.ldU; in.Phi = a.Phi; in.ldPhi = a.ldPhi; in.n_lon = a.n_lon;
    descs.push_back(in);
  }
  return build_plan(descs, o, (hipStream_t)stream, out);
}

pc_status pc_gram_assemble(pc_plan* p, void* stream) {
  if (!p) return PC_ERR_INVALID_ARG;
  hipSetDevice(p->device);
  hipStream_t s = (hipStream_t)stream;
  if (p->lowgram) return assemble_lowgram_batch(p, s);
  PC_TRY(fork(p, s));
  for (size_t i = 0; i < p->inst.size(); ++i) {
    pc_status st = assemble_one(p, p->inst[i], stream_for(p, i, s));
    if (st != PC_OK) return st;
  }
  PC_TRY(join(p, s));
  return PC_OK;
}

// The factorization of every instance on the streams; `after_gram`, if set,
// is recorded once the (single, unbatched) instance's Gram is assembled, and
// `after_reset` once its tile states are reset (unblocked factorization).
static pc_status enqueue_factor(pc_plan* p, hipStream_t s, hipEvent_t after_gram,
                                hipEvent_t after_reset = nullptr) {
  if (p->lowgram) {
    const pc_status st = assemble_lowgram_batch(p, s);
    if (st != PC_OK) return st;
  }
  PC_TRY(fork(p, s));
  for (size_t i = 0; i < p->inst.size(); ++i) {
    Inst& in = p->inst[i];
    hipStream_t si = stream_for(p, i, s);
    if (!p->lowgram) {
      const pc_status st = assemble_one(p, in, si);
      if (st != PC_OK) return st;
      if (after_gram) PC_TRY(hipEventRecord(after_gram, si));
    }
    if (in.Gs) {
      // the kept Gram is the FP64 one: a copy of G, or assembled on its own
      // when G is a reduced-precision Gram (whose factor preconditions CG)
      if (in.prec == PC_PREC_FP64) PC_TRY(pc::launch_gram_symmetrize(in, in.Gs, si));
      else PC_TRY(pc::launch_kept_fp64_gram(in, si));
      PC_TRY(pc::launch_fill_int(in.cg_flags, 0, 2, si));
      if (in.cgm_Dinv) {
        // member block-Jacobi: the inverse of every diagonal M x M block
        PC_TRY(pc::launch_fill_int(in.cg_flags + 1, -1, 1, si));
        const int64_t Mp = in.cgm_Mp;
        for (int64_t k = 0; k < in.K; ++k)
          PC_TRY(pc::launch_member_block_inverse(in.Gs, in.KMp, k * in.M, in.M, Mp, in.cgm_work, in.cgm_d0,
                                                 in.cgm_Linv, in.cgm_ctr, in.cgm_offs, in.cgm_ntasks, in.cgm_I,
                                                 in.cgm_work + Mp * Mp, in.cgm_Dinv + k * Mp * Mp, in.cg_flags + 1,
                                                 si));
      } else {
        PC_TRY(pc::launch_bj_setup(in.Gs, in.KMp, in.KMp / pc::NB, in.Dinv, in.cg_flags + 1, si));
      }
    }
    if (!p->batch) {
      PhaseTimer t(p, PC_PHASE_CHOLESKY, si);
      PC_TRY(pc::launch_cholesky(in, si, after_reset));
    }
  }
  PC_TRY(join(p, s));
  if (p->batch) {
    PhaseTimer t(p, PC_PHASE_CHOLESKY, s);
    PC_TRY(pc::launch_cholesky_batch(p->batch, s, p->inst[0].tune_chol_per_cu));
    for (const Inst& in : p->inst) PC_TRY(pc::launch_solve_fold(in, s));
  }
  return PC_OK;
}

// Copies of every instance's pivot status and error flag after the
// factorization, into pinned memory (read after a later stream sync; the
// solves reuse the error flag, so the copies go right after the factor).
static pc_status read_factor_status(pc_plan* p, hipStream_t s) {
  const size_t n = p->inst.size();
  for (size_t i = 0; i < n; ++i) {
    const Inst& in = p->inst[i];
    PC_TRY(hipMemcpyAsync(&p->h_status[i], in.info, sizeof(int), hipMemcpyDeviceToHost, s));
    PC_TRY(hipMemcpyAsync(&p->h_status[n + i], p->batch ? pc::dag_batch_error(p->batch) : pc::chol_error_flag(in),
                          sizeof(int), hipMemcpyDeviceToHost, s));
  }
  return PC_OK;
}

// The factorization's outcome from those copies (after the stream sync).
static pc_status factor_outcome(pc_plan* p, int32_t* failed_instance) {
  const size_t n = p->inst.size();
  for (size_t i = 0; i < n; ++i)
    if (p->h_status[n + i]) return PC_ERR_DEVICE;   // a bounded wait expired: the factor is not trustworthy
  pc_status st = PC_OK;
  for (size_t i = 0; i < n; ++i) {
    p->inst[i].factored = p->h_status[i] < 0;
    if (p->h_status[i] >= 0 && st == PC_OK) {
      st = PC_ERR_NOT_SPD;
      if (failed_instance) *failed_instance = (int32_t)i;
    }
  }
  return st;
}

// Pivot status of every instance after the factorization (one stream sync).
static pc_status finish_factor(pc_plan* p, hipStream_t s, int32_t* failed_instance) {
  const pc_status st = read_factor_status(p, s);
  if (st != PC_OK) return st;
  PC_TRY(hipStreamSynchronize(s));
  return factor_outcome(p, failed_instance);
}

// Whether instance i's refinement failed: any right-hand side diverging,
// or, for a Gram in reduced precision, one stalled above the acceptance
// level or out of budget.  In FP64 (the plan's precision or the ladder's
// last rung) the refinement steps are corrected semi-normal steps: a stall
// (the updates fluctuate at the attainable accuracy of the FP64 residual)
// or a spent budget is the result.
static bool refinement_failed(const pc_plan* p, size_t i) {
  const int done = p->h_ctl[i].done;
  return done == 3 || (done != 1 && p->inst[i].prec != PC_PREC_FP64);
}

// Refinement outcome of an apply: one read of every instance's control block.
static pc_status finish_apply(pc_plan* p, const int64_t* R, hipStream_t s) {
  const size_t cnt = p->inst.size();
  for (size_t i = 0; i < cnt; ++i)
    if (R[i] != 0) {
      Inst& in = p->inst[i];
      in.iters = 0; in.last_rel = 0.0; in.last_R = R[i];
      std::fill(in.rhs_host.begin(), in.rhs_host.begin() + R[i], pc::RhsCtl{1, 0, 0, 0, 0.0, 0.0});
    }
  if (p->opt.max_refine == 0) return PC_OK;
  for (size_t i = 0; i < cnt; ++i)
    if (R[i] != 0) {
      PC_TRY(hipMemcpyAsync(&p->h_ctl[i], p->inst[i].ctl, sizeof(pc::RefineCtl), hipMemcpyDeviceToHost, s));
      PC_TRY(hipMemcpyAsync(p->inst[i].rhs_host.data(), p->inst[i].rhs, sizeof(pc::RhsCtl) * (size_t)R[i],
                            hipMemcpyDeviceToHost, s));
    }
  PC_TRY(hipStreamSynchronize(s));
  pc_status st = PC_OK;
  for (size_t i = 0; i < cnt; ++i) {
    if (R[i] == 0) continue;
    p->inst[i].iters = p->h_ctl[i].iters;
    p->inst[i].last_rel = p->h_ctl[i].last;
    if (refinement_failed(p, i)) st = PC_ERR_NO_CONVERGENCE;
  }
  return st;
}

// Assemble and factor instance i alone in its current precision (after the
// ladder raised it), then read its pivot status (one stream sync).
static pc_status refactor_one(pc_plan* p, size_t i, hipStream_t s) {
  Inst& in = p->inst[i];
  const size_t n = p->inst.size();
  pc_status st = assemble_one(p, in, s);
  if (st != PC_OK) return st;
  { PhaseTimer t(p, PC_PHASE_CHOLESKY, s); PC_TRY(pc::launch_cholesky(in, s)); }
  PC_TRY(hipMemcpyAsync(&p->h_status[i], in.info, sizeof(int), hipMemcpyDeviceToHost, s));
  PC_TRY(hipMemcpyAsync(&p->h_status[n + i], pc::chol_error_flag(in), sizeof(int), hipMemcpyDeviceToHost, s));
  PC_TRY(hipStreamSynchronize(s));
  if (p->h_status[n + i]) return PC_ERR_DEVICE;
  in.factored = p->h_status[i] < 0;
  return PC_OK;
}

// The ladder at factorization time: an instance whose Gram in reduced
// precision was not positive definite is assembled and factored again in
// the next precision, up to FP64.  Returns PC_ERR_NOT_SPD (first instance in
// *failed_instance) if one still fails in FP64.
static pc_status escalate_failed_factors(pc_plan* p, hipStream_t s, int32_t* failed_instance) {
  for (size_t i = 0; i < p->inst.size(); ++i) {
    Inst& in = p->inst[i];
    while (!in.factored && ladder_on(p) && next_rung(in.prec) >= 0) {
      in.prec = next_rung(in.prec);
      const pc_status st = refactor_one(p, i, s);
      if (st != PC_OK) return st;
    }
  }
  if (failed_instance) *failed_instance = -1;
  for (size_t i = 0; i < p->inst.size(); ++i)
    if (!p->inst[i].factored) {
      if (failed_instance) *failed_instance = (int32_t)i;
      return PC_ERR_NOT_SPD;
    }
  return PC_OK;
}

// The ladder at apply time: every instance whose refinement stopped without
// converging (stalled above the acceptance level, or diverging) is refactored
// in the next precision and solved again alone, until it converges or FP64
// has been tried.  An instance whose Gram is not positive definite even in
// FP64 is left without a factor (the others go on); the call then returns
// PC_ERR_NOT_SPD.
static pc_status escalate_unconverged(pc_plan* p, const double* const* X, const int64_t* ldX, const int64_t* R,
                                      double* const* Y, const int64_t* ldY, hipStream_t s) {
  const size_t cnt = p->inst.size();
  std::vector<int64_t> R2(cnt, 0);
  std::vector<char> lost(cnt, 0);
  while (ladder_on(p)) {
    bool any = false;
    for (size_t i = 0; i < cnt; ++i) {
      R2[i] = 0;
      Inst& in = p->inst[i];
      if (R[i] == 0 || lost[i] || !refinement_failed(p, i) || next_rung(in.prec) < 0) continue;
      do {
        in.prec = next_rung(in.prec);
        const pc_status fs = refactor_one(p, i, s);
        if (fs != PC_OK) return fs;
      } while (!in.factored && next_rung(in.prec) >= 0);
      if (!in.factored) { lost[i] = 1; continue; }
      R2[i] = R[i];
      any = true;
    }
    if (!any) break;
    pc_status st = enqueue_apply(p, X, ldX, R2.data(), Y, ldY, s, p->opt.max_refine > 4 ? 2 : 0, 0, true);
    if (st != PC_OK) return st;
    st = finish_apply(p, R2.data(), s);
    if (st != PC_OK && st != PC_ERR_NO_CONVERGENCE) return st;
  }
  for (size_t i = 0; i < cnt; ++i)
    if (lost[i]) return PC_ERR_NOT_SPD;
  for (size_t i = 0; i < cnt; ++i)
    if (R[i] != 0 && refinement_failed(p, i)) return PC_ERR_NO_CONVERGENCE;
  return PC_OK;
}

pc_status pc_gram_factor(pc_plan* p, void* stream, int32_t* failed_instance) {
  if (failed_instance) *failed_instance = -1;
  if (!p) return PC_ERR_INVALID_ARG;
  hipSetDevice(p->device);
  hipStream_t s = (hipStream_t)stream;
  const pc_status st = enqueue_factor(p, s, nullptr);
  if (st != PC_OK) return st;
  const pc_status fs = finish_factor(p, s, failed_instance);
  if (fs == PC_ERR_NOT_SPD && ladder_on(p)) return escalate_failed_factors(p, s, failed_instance);
  return fs;
}

pc_status pc_left_inverse_apply(pc_plan* p, const double* const* X, const int64_t* ldX, const int64_t* R,
                                double* const* Y, const int64_t* ldY, void* stream) {
  if (!p || !X || !ldX || !R || !Y || !ldY) return PC_ERR_INVALID_ARG;
  hipSetDevice(p->device);
  hipStream_t s = (hipStream_t)stream;
  const size_t cnt = p->inst.size();
  for (size_t i = 0; i < cnt; ++i) {
    const Inst& in = p->inst[i];
    if (R[i] < 0) return PC_ERR_INVALID_ARG;
    if (R[i] == 0) continue;
    if (!in.factored) return PC_ERR_NOT_FACTORED;
    if (R[i] > in.max_rhs) return PC_ERR_TOO_MANY_RHS;
    if (!X[i] || !Y[i] || ldX[i] < in.n || ldY[i] < in.KM) return PC_ERR_INVALID_ARG;
  }
  const int budget = p->opt.max_refine;
  if (p->opt.use_graph && !p->profiling) {
    // capture once per argument set on the internal stream, then replay on `s`
    // (with phase timing on, the sequence runs eagerly: timing events are not captured)
    std::vector<int64_t> key;
    for (size_t i = 0; i < cnt; ++i) {
      key.push_back((int64_t)(intptr_t)X[i]); key.push_back(ldX[i]); key.push_back(R[i]);
      key.push_back((int64_t)(intptr_t)Y[i]); key.push_back(ldY[i]);
    }
    if (!p->gexec || key != p->gkey) {
      if (p->gexec) { hipGraphExecDestroy(p->gexec); p->gexec = nullptr; }
      if (p->graph) { hipGraphDestroy(p->graph); p->graph = nullptr; }
      PC_TRY(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal));
      pc_status st = enqueue_apply(p, X, ldX, R, Y, ldY, p->cap, 0);
      hipGraph_t g = nullptr;
      const hipError_t e = hipStreamEndCapture(p->cap, &g);
      if (st != PC_OK) { if (g) hipGraphDestroy(g); return st; }
      if (e != hipSuccess) return PC_ERR_DEVICE;
      p->graph = g;
      PC_TRY(hipGraphInstantiate(&p->gexec, g, nullptr, nullptr, 0));
      p->gkey = key;
    }
    PC_TRY(hipGraphLaunch(p->gexec, s));
  } else {
    pc_status st = enqueue_apply(p, X, ldX, R, Y, ldY, s, budget > 4 ? 2 : 0);
    if (st != PC_OK) return st;
  }
  const pc_status st = finish_apply(p, R, s);
  if (st == PC_ERR_NO_CONVERGENCE && ladder_on(p)) return escalate_unconverged(p, X, ldX, R, Y, ldY, s);
  return st;
}

// pc_factor_apply with a graph: assembly, factorization, the copies of the
// pivot statuses, Z^T x, the solves and the refinement iterations of every
// instance are captured once (per argument set and per precision of each
// instance) and replayed as ONE graph, with one stream sync after it.  All
// instances with right-hand sides are solved in the graph; one whose Gram
// turned out not to be positive definite is afterwards raised along the
// ladder and solved again outside it (its Y is discarded), or reported.
static pc_status factor_apply_graph(pc_plan* p, const double* const* X, const int64_t* ldX, const int64_t* R,
                                    double* const* Y, const int64_t* ldY, hipStream_t s, int32_t* failed_instance) {
  const size_t cnt = p->inst.size();
  std::vector<int64_t> key;
  for (size_t i = 0; i < cnt; ++i) {
    key.push_back((int64_t)(intptr_t)X[i]); key.push_back(ldX[i]); key.push_back(R[i]);
    key.push_back((int64_t)(intptr_t)Y[i]); key.push_back(ldY[i]); key.push_back(p->inst[i].prec);
  }
  if (!p->fgexec || key != p->fgkey) {
    if (p->fgexec) { hipGraphExecDestroy(p->fgexec); p->fgexec = nullptr; }
    if (p->fgraph) { hipGraphDestroy(p->fgraph); p->fgraph = nullptr; }
    PC_TRY(hipStreamBeginCapture(p->cap, hipStreamCaptureModeThreadLocal));
    pc_status st = enqueue_factor(p, p->cap, nullptr);
    if (st == PC_OK) st = read_factor_status(p, p->cap);
    if (st == PC_OK) st = enqueue_apply(p, X, ldX, R, Y, ldY, p->cap, 0);
    hipGraph_t g = nullptr;
    const hipError_t e = hipStreamEndCapture(p->cap, &g);
    if (st != PC_OK) { if (g) hipGraphDestroy(g); return st; }
    if (e != hipSuccess) return PC_ERR_DEVICE;
    p->fgraph = g;
    PC_TRY(hipGraphInstantiate(&p->fgexec, g, nullptr, nullptr, 0));
    p->fgkey = key;
  }
  PC_TRY(hipGraphLaunch(p->fgexec, s));
  PC_TRY(hipStreamSynchronize(s));
  int32_t first = -1;
  pc_status fst = factor_outcome(p, &first);
  if (fst == PC_ERR_DEVICE) return fst;
  std::vector<int64_t> R2(R, R + cnt);
  for (size_t i = 0; i < cnt; ++i)
    if (!p->inst[i].factored) R2[i] = 0;
  pc_status ast = finish_apply(p, R2.data(), s);
  if (ast == PC_ERR_NO_CONVERGENCE && ladder_on(p)) ast = escalate_unconverged(p, X, ldX, R2.data(), Y, ldY, s);
  if (ast == PC_ERR_NOT_SPD) { ast = PC_OK; fst = PC_ERR_NOT_SPD; }   // lost its factor on the ladder
  if (ast != PC_OK && ast != PC_ERR_NO_CONVERGENCE) return ast;
  if (fst == PC_ERR_NOT_SPD && ladder_on(p)) {
    std::vector<int64_t> R3(cnt, 0);
    for (size_t i = 0; i < cnt; ++i)
      if (!p->inst[i].factored) R3[i] = R[i];
    int32_t still = -1;
    const pc_status es = escalate_failed_factors(p, s, &still);
    if (es != PC_OK && es != PC_ERR_NOT_SPD) return es;
    for (size_t i = 0; i < cnt; ++i)
      if (!p->inst[i].factored) R3[i] = 0;
    const pc_status rs = enqueue_apply(p, X, ldX, R3.data(), Y, ldY, s, p->opt.max_refine > 4 ? 2 : 0, 0, true);
    if (rs != PC_OK) return rs;
    pc_status st3 = finish_apply(p, R3.data(), s);
    if (st3 == PC_ERR_NO_CONVERGENCE) st3 = escalate_unconverged(p, X, ldX, R3.data(), Y, ldY, s);
    if (st3 == PC_ERR_NOT_SPD) st3 = PC_OK;        // reported below from the factored flags
    if (st3 != PC_OK && st3 != PC_ERR_NO_CONVERGENCE) return st3;
    if (st3 == PC_ERR_NO_CONVERGENCE) ast = st3;
    fst = PC_OK;
    for (size_t i = 0; i < cnt; ++i)
      if (!p->inst[i].factored && fst == PC_OK) { fst = PC_ERR_NOT_SPD; first = (int32_t)i; }
  }
  // an instance without a factor matters only if it has right-hand sides
  if (fst == PC_ERR_NOT_SPD) {
    int32_t failed = -1;
    for (size_t i = 0; i < cnt && failed < 0; ++i)
      if (!p->inst[i].factored && R[i] > 0) failed = (int32_t)i;
    if (failed >= 0) {
      if (failed_instance) *failed_instance = failed;
      return PC_ERR_NOT_SPD;
    }
  }
  return ast;
}

pc_status pc_factor_apply(pc_plan* p, const double* const* X, const int64_t* ldX, const int64_t* R,
                          double* const* Y, const int64_t* ldY, void* stream, int32_t* failed_instance) {
  if (failed_instance) *failed_instance = -1;
  if (!p || !X || !ldX || !R || !Y || !ldY) return PC_ERR_INVALID_ARG;
  hipSetDevice(p->device);
  hipStream_t s = (hipStream_t)stream;
  const size_t cnt = p->inst.size();
  for (size_t i = 0; i < cnt; ++i) {
    const Inst& in = p->inst[i];
    if (R[i] < 0) return PC_ERR_INVALID_ARG;
    if (R[i] == 0) continue;
    if (R[i] > in.max_rhs) return PC_ERR_TOO_MANY_RHS;
    if (!X[i] || !Y[i] || ldX[i] < in.n || ldY[i] < in.KM) return PC_ERR_INVALID_ARG;
  }
  // The overlap: one unbatched instance in FP64 or with refinement, no graph
  // (the products Z^T x depend on E, W and X only, which the caller's stream
  // has made ready when the Gram is assembled), factored by the tile DAG.  A
  // blocked factorization runs serially after Z^T x instead: its persistent
  // diagonal-block kernels would wait for compute units that the products
  // hold, and its panel products leave nothing idle to fill.
  const bool overlap = cnt == 1 && R[0] > 0 && !p->batch && !p->lowgram && !p->opt.use_graph &&
                       p->inst[0].blk_NO == 0;
  // (with phase timing on, the sequence runs eagerly: timing events are not captured)
  if (p->opt.use_graph && !p->profiling) return factor_apply_graph(p, X, ldX, R, Y, ldY, s, failed_instance);
  if (!overlap) {
    // an instance that fails to factor matters only if it has right-hand sides
    int32_t first = -1;
    const pc_status st = pc_gram_factor(p, stream, &first);
    if (st != PC_OK && st != PC_ERR_NOT_SPD) return st;
    if (st == PC_ERR_NOT_SPD) {
      std::vector<int64_t> R2(R, R + cnt);
      int32_t failed = -1;
      for (size_t i = 0; i < cnt; ++i)
        if (!p->inst[i].factored) {
          if (R2[i] > 0 && failed < 0) failed = (int32_t)i;
          R2[i] = 0;
        }
      const pc_status ast = pc_left_inverse_apply(p, X, ldX, R2.data(), Y, ldY, stream);
      if (failed >= 0) {
        if (failed_instance) *failed_instance = failed;
        return PC_ERR_NOT_SPD;
      }
      return ast;
    }
    return pc_left_inverse_apply(p, X, ldX, R, Y, ldY, stream);
  }
  if (!p->ovl) {
    if (hipStreamCreateWithFlags(&p->ovl, hipStreamNonBlocking) != hipSuccess) { p->ovl = nullptr; return PC_ERR_DEVICE; }
    if (hipEventCreateWithFlags(&p->ev_gram, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev_reset, hipEventDisableTiming) != hipSuccess ||
        hipEventCreateWithFlags(&p->ev_ztx, hipEventDisableTiming) != hipSuccess)
      return PC_ERR_DEVICE;
  }
  Inst& in = p->inst[0];
  // The forward pass of the first solve also runs during an unblocked
  // factorization, behind it: its tasks wait for the L blocks they read.
  const bool fwd = in.blk_NO == 0 && in.Lt != nullptr;
  pc_status st = enqueue_factor(p, s, p->ev_gram, fwd ? p->ev_reset : nullptr);
  if (st != PC_OK) return st;
  st = read_factor_status(p, s);
  if (st != PC_OK) return st;
  PC_TRY(hipStreamWaitEvent(p->ovl, p->ev_gram, 0));
  { PhaseTimer t(p, PC_PHASE_ZTX, p->ovl); PC_TRY(launch_first_ztx(p, in, X[0], ldX[0], R[0], in.Y, in.KMp, p->ovl)); }
  if (fwd) {
    PC_TRY(hipStreamWaitEvent(p->ovl, p->ev_reset, 0));
    PhaseTimer t(p, PC_PHASE_SOLVE_ALONGSIDE, p->ovl);
    PC_TRY(pc::launch_chol_solve_fwd_concurrent(in, R[0], p->ovl));
  }
  PC_TRY(hipEventRecord(p->ev_ztx, p->ovl));
  PC_TRY(hipStreamWaitEvent(s, p->ev_ztx, 0));
  if (fwd)
    PC_TRY(hipMemcpyAsync(&p->h_status[2], pc::chol_solve_fwd_error_flag(in), sizeof(int), hipMemcpyDeviceToHost, s));
  st = enqueue_apply(p, X, ldX, R, Y, ldY, s, p->opt.max_refine > 4 ? 2 : 0, fwd ? 2 : 1);
  PC_TRY(hipStreamSynchronize(s));
  const bool fwd_err = fwd && p->h_status[2] != 0;   // read before the ladder reuses the status slots
  const pc_status fst = factor_outcome(p, failed_instance);
  if (st != PC_OK) return st;
  if (fst == PC_ERR_NOT_SPD && ladder_on(p)) {
    // the ladder: refactor in a more accurate precision, then the plain apply
    const pc_status es = escalate_failed_factors(p, s, failed_instance);
    if (es != PC_OK) return es;
    return pc_left_inverse_apply(p, X, ldX, R, Y, ldY, stream);
  }
  if (fst != PC_OK) return fst;
  if (fwd_err) return PC_ERR_DEVICE;   // a bounded wait of the forward pass expired
  const pc_status ast = finish_apply(p, R, s);
  if (ast == PC_ERR_NO_CONVERGENCE && ladder_on(p)) return escalate_unconverged(p, X, ldX, R, Y, ldY, s);
  return ast;
}

pc_status pc_query_info(const pc_plan* p, int32_t instance, int32_t* iterations, double* last_rel_update) {
  if (!p || instance < 0 || (size_t)instance >= p->inst.size()) return PC_ERR_INVALID_ARG;
  if (iterations) *iterations = p->inst[instance].iters;
  if (last_rel_update) *last_rel_update = p->inst[instance].last_rel;
  return PC_OK;
}

pc_status pc_query_rhs_info(const pc_plan* p, int32_t instance, int64_t R, pc_rhs_info* out) {
  if (!p || instance < 0 || (size_t)instance >= p->inst.size() || R < 0 || (R > 0 && !out)) return PC_ERR_INVALID_ARG;
  const Inst& in = p->inst[instance];
  if (R > in.last_R) return PC_ERR_INVALID_ARG;
  for (int64_t r = 0; r < R; ++r) {
    const pc::RhsCtl& c = in.rhs_host[(size_t)r];
    out[r].iterations = c.iters;
    out[r].state = c.state;
    out[r].last_rel_update = c.last;
  }
  return PC_OK;
}

pc_status pc_query_instance(const pc_plan* p, int32_t instance, int32_t* precision, int32_t* factored) {
  if (!p || instance < 0 || (size_t)instance >= p->inst.size()) return PC_ERR_INVALID_ARG;
  if (precision) *precision = p->inst[instance].prec;
  if (factored) *factored = p->inst[instance].factored ? 1 : 0;
  return PC_OK;
}

pc_status pc_plan_destroy(pc_plan* p) {
  free_plan(p);
  return PC_OK;
}

pc_status pc_sqrt_transpose_apply(pc_plan* p, int32_t instance, const double* X, int64_t ldX, int64_t R,
                                  double* B, int64_t ldB, void* stream) {
  if (!p || instance < 0 || (size_t)instance >= p->inst.size() || R < 0) return PC_ERR_INVALID_ARG;
  const Inst& in = p->inst[instance];
  if (R == 0) return PC_OK;
  if (!X || !B || ldX < in.n || ldB < in.KM) return PC_ERR_INVALID_ARG;
  hipSetDevice(p->device);
  PC_TRY(pc::launch_ztx(in, X, ldX, R, B, ldB, (hipStream_t)stream));
  return PC_OK;
}

pc_status pc_sqrt_transpose_apply_lowprec(pc_plan* p, int32_t instance, int32_t precision, const double* X,
                                          int64_t ldX, int64_t R, double* B, int64_t ldB, void* stream) {
  if (!p || instance < 0 || (size_t)instance >= p->inst.size() || R < 0) return PC_ERR_INVALID_ARG;
  if (precision != PC_PREC_FP32_REFINE && precision != PC_PREC_BF16_REFINE) return PC_ERR_INVALID_ARG;
  const Inst& in = p->inst[instance];
  if (R == 0) return PC_OK;
  if (!X || !B || ldX < in.n || ldB < in.KM) return PC_ERR_INVALID_ARG;
  hipSetDevice(p->device);
  PC_TRY(pc::launch_ztx_lowprec(in, precision, X, ldX, R, B, ldB, (hipStream_t)stream));
  return PC_OK;
}

pc_status pc_sqrt_apply(pc_plan* p, int32_t instance, const double* Yin, int64_t ldY, int64_t R, double* X,
                        int64_t ldX, void* stream) {
  if (!p || instance < 0 || (size_t)instance >= p->inst.size() || R < 0) return PC_ERR_INVALID_ARG;
  const Inst& in = p->inst[instance];
  if (R == 0) return PC_OK;
  if (!X || !Yin || ldX < in.n || ldY < in.KM) return PC_ERR_INVALID_ARG;
  hipSetDevice(p->device);
  PC_TRY(pc::launch_zy(in, Yin, ldY, R, nullptr, 0, X, ldX, (hipStream_t)stream));
  return PC_OK;
}

int32_t pc_selftest_task_order(int32_t T, int32_t group) {
  if (T < 1 || group > T) return -1;
  return pc::check_chol_task_order(T, group);
}

pc_status pc_profile_enable(pc_plan* p, int32_t on) {
  if (!p) return PC_ERR_INVALID_ARG;
  p->profiling = on != 0;
  return PC_OK;
}

pc_status pc_profile_read(pc_plan* p, double* total_ms, int64_t* counts) {
  if (!p) return PC_ERR_INVALID_ARG;
  hipSetDevice(p->device);
  pc_status st = PC_OK;
  for (int ph = 0; ph < PC_NUM_PHASES; ++ph) {
    double tot = 0.0;
    for (auto& e : p->rec[ph]) {
      float ms = 0.f;
      if (hipEventSynchronize(e.second) != hipSuccess || hipEventElapsedTime(&ms, e.first, e.second) != hipSuccess)
        st = PC_ERR_DEVICE;
      tot += ms;
      p->pool.push_back(e.first);
      p->pool.push_back(e.second);
    }
    if (total_ms) total_ms[ph] = tot;
    if (counts) counts[ph] = (int64_t)p->rec[ph].size();
    p->rec[ph].clear();
  }
  return st;
}

pc_status pc_gram_export(const pc_plan* p, int32_t instance, double* G, int64_t ldG, void* stream) {
  if (!p || instance < 0 || (size_t)instance >= p->inst.size() || !G) return PC_ERR_INVALID_ARG;
  const Inst& in = p->inst[instance];
  if (ldG < in.KM) return PC_ERR_INVALID_ARG;
  hipSetDevice(p->device);
  PC_TRY(pc::launch_export_lower(in.G, in.KMp, G, ldG, in.KM, (hipStream_t)stream));
  return PC_OK;
}

pc_status pc_cg_solve(pc_plan* p, int32_t instance, const double* Bm, int64_t ldB, int64_t R, double* Y,
                      int64_t ldY, double tol, int32_t maxiter, int32_t warm, int32_t* iterations, void* stream) {
  if (iterations) *iterations = 0;
  if (!p || instance < 0 || (size_t)instance >= p->inst.size() || R < 0 || maxiter < 0 || !(tol >= 0.0))
    return PC_ERR_INVALID_ARG;
  Inst& in = p->inst[instance];
  if (!in.Gs) return PC_ERR_INVALID_ARG;
  if (!in.factored) return PC_ERR_NOT_FACTORED;
  if (R == 0) return PC_OK;
  if (R > in.max_rhs) return PC_ERR_TOO_MANY_RHS;
  if (!Bm || !Y || ldB < in.KM || ldY < in.KM) return PC_ERR_INVALID_ARG;
  hipSetDevice(p->device);
  hipStream_t s = (hipStream_t)stream;
  PC_TRY(pc::launch_copy_rows(Y, ldY, in.Y, in.KMp, warm ? in.KM : 0, in.KMp, R, s));
  int it = 0;
  bool ok = false;
  pc_status st = run_cg(p, in, Bm, ldB, R, warm != 0, tol, maxiter, s, &it, &ok);
  if (st != PC_OK) return st;
  PC_TRY(pc::launch_copy_rows(in.Y, in.KMp, Y, ldY, in.KM, in.KM, R, s));
  PC_TRY(hipStreamSynchronize(s));
  if (iterations) *iterations = it;
  return ok ? PC_OK : PC_ERR_NO_CONVERGENCE;
}

pc_status pc_learned_apply(pc_plan* p, int32_t instance, pc_mlp* mlp, const double* X, int64_t ldX, int64_t R,
                           double* Y, int64_t ldY, double tol, int32_t maxiter, int32_t* iterations,
                           int32_t* fallback, void* stream) {
  if (iterations) *iterations = 0;
  if (fallback) *fallback = 0;
  if (!p || instance < 0 || (size_t)instance >= p->inst.size() || R < 0 || maxiter < 0 || !(tol >= 0.0))
    return PC_ERR_INVALID_ARG;
  Inst& in = p->inst[instance];
  if (!in.Gs) return PC_ERR_INVALID_ARG;
  if (!in.factored) return PC_ERR_NOT_FACTORED;
  if (R == 0) return PC_OK;
  if (R > in.max_rhs) return PC_ERR_TOO_MANY_RHS;
  if (!X || !Y || ldX < in.n || ldY < in.KM) return PC_ERR_INVALID_ARG;
  if (mlp && (mlp->d != in.KM || R > mlp->max_batch)) return PC_ERR_INVALID_ARG;
  hipSetDevice(p->device);
  hipStream_t s = (hipStream_t)stream;
  // b = Z^T x into the plan's right-hand-side buffer
  PC_TRY(pc::launch_ztx(in, X, ldX, R, in.B, in.KMp, s));
  // start: the network's prediction, or zero
  PC_TRY(pc::launch_copy_rows(in.Y, in.KMp, in.Y, in.KMp, 0, in.KMp, R, s));
  if (mlp) {
    pc_status st = pc_mlp_warm_start(mlp, in.B, in.KMp, R, in.Y, in.KMp, s);
    if (st != PC_OK) return st;
  }
  int it = 0;
  bool ok = false;
  pc_status st = run_cg(p, in, in.B, in.KMp, R, mlp != nullptr, tol, maxiter, s, &it, &ok);
  if (st != PC_OK) return st;
  if (!ok && in.prec == PC_PREC_FP64) {
    // the direct solve replaces the iterate
    PC_TRY(pc::launch_copy_rows(in.B, in.KMp, in.Y, in.KMp, in.KM, in.KMp, R, s));
    PC_TRY(pc::launch_chol_solve(in, in.Y, in.KMp, R, in.D, in.KMp, s));
    if (fallback) *fallback = 1;
  }
  if (!ok && in.prec != PC_PREC_FP64) {
    // the direct solve of a reduced-precision plan: its factor and FP64 refinement
    if (fallback) *fallback = 1;
    if (iterations) *iterations = it;
    const size_t cnt = p->inst.size();
    std::vector<const double*> Xs(cnt, nullptr);
    std::vector<double*> Ys(cnt, nullptr);
    std::vector<int64_t> lx(cnt, 1), ly(cnt, 1), R2(cnt, 0);
    Xs[instance] = X; Ys[instance] = Y; lx[instance] = ldX; ly[instance] = ldY; R2[instance] = R;
    st = enqueue_apply(p, Xs.data(), lx.data(), R2.data(), Ys.data(), ly.data(), s, 0, 0, true);
    if (st != PC_OK) return st;
    return finish_apply(p, R2.data(), s);
  }
  PC_TRY(pc::launch_copy_rows(in.Y, in.KMp, Y, ldY, in.KM, in.KM, R, s));
  PC_TRY(hipStreamSynchronize(s));
  if (iterations) *iterations = it;
  return PC_OK;
}

pc_status pc_autotune(pc_plan* p, const char* cache_path, int32_t use_cached, void* stream) {
  if (!p) return PC_ERR_INVALID_ARG;
  hipSetDevice(p->device);
  hipStream_t s = (hipStream_t)stream;
  std::vector<TuneEntry> cache = read_tune_cache(cache_path);
  const int prec = p->opt.precision;
  const int reps = 3;
  bool any_measured = false;
  int batch_per_cu = 0;
  for (size_t i = 0; i < p->inst.size(); ++i) {
    Inst& in = p->inst[i];
    in.factored = false;
    const TuneKey key{in.n_h, in.n_w, in.K, in.M, in.max_rhs, prec};
    const TuneEntry* hit = nullptr;
    for (const auto& e : cache)
      if (e.key == key) hit = &e;
    if (hit && use_cached) {
      in.tune_gram_split = hit->gram_split;
      in.tune_ztx_split = hit->ztx_split;
      in.tune_chol_per_cu = hit->chol_per_cu;
      in.tune_gemm_tile = hit->gemm_tile;
      if (in.blk_NO > 0 && hit->chol_block > 0 && hit->chol_block != in.blk_NO) {
        const pc_status bs = alloc_blocked(in, hit->chol_block);
        if (bs != PC_OK) return bs;
      }
      continue;
    }
    any_measured = true;
    // FP64 Gram: one to four contraction parts (the others need G2)
    in.tune_gram_split = 1;
    if (prec == PC_PREC_FP64) {
      // four parts only where the tiles are few (the large Grams fill the device)
      const int most = pc::gram_split_for(in) > 1 ? 4 : 2;
      if (ensure_gram_parts(in, most) != hipSuccess) (void)ensure_gram_parts(in, 2);
      float best = 0.f;
      int choice = 1;
      for (int c = 1; c <= most; ++c) {
        if (c - 1 > in.g2_parts) break;
        in.tune_gram_split = c;
        float ms = 0.f;
        pc_status st = time_ms(s, reps, [&]() -> pc_status {
          PC_TRY(pc::launch_column_grams(in, s));
          PC_TRY(pc::launch_gram_f64(in, s));
          PC_TRY(pc::launch_gram_pad_and_diag(in, s));
          return PC_OK;
        }, &ms);
        if (st != PC_OK) return st;
        if (c == 1 || ms < best) { best = ms; choice = c; }
      }
      in.tune_gram_split = choice;
    }
    // Z^T x at the plan's right-hand-side count, on the residual scratch
    if (in.max_rhs > 0) {
      float best = 0.f;
      int choice = 1;
      PC_TRY(hipMemsetAsync(in.Rres, 0, sizeof(double) * (size_t)(in.n * in.max_rhs), s));
      for (int c = 1; c <= 2; ++c) {
        in.tune_ztx_split = c;
        float ms = 0.f;
        pc_status st = time_ms(s, reps, [&]() -> pc_status {
          PC_TRY(pc::launch_ztx(in, in.Rres, in.n, in.max_rhs, in.D, in.KMp, s));
          return PC_OK;
        }, &ms);
        if (st != PC_OK) return st;
        if (c == 1 || ms < best) { best = ms; choice = c; }
      }
      in.tune_ztx_split = choice;
    }
    // Cholesky grid, on the assembled Gram (single-instance plans; a batch is
    // tuned as a whole below)
    in.tune_chol_per_cu = 2;
    if (!p->batch) {
      float best = 0.f;
      int choice = 2;
      for (int c = 2; c >= 1; --c) {
        in.tune_chol_per_cu = c;
        float tot = 0.f;
        for (int r = 0; r < reps; ++r) {
          pc_status st = assemble_one(p, in, s);
          if (st != PC_OK) return st;
          float ms = 0.f;
          st = time_ms(s, 1, [&]() -> pc_status { PC_TRY(pc::launch_cholesky(in, s)); return PC_OK; }, &ms, false);
          if (st != PC_OK) return st;
          tot += ms;
        }
        if (c == 2 || tot < best) { best = tot; choice = c; }
      }
      in.tune_chol_per_cu = choice;
      // blocked factorization (large Grams): block width and the tile shape
      // of its panel and trailing products, timed on one assembled Gram kept
      // in a copy (restored before each run)
      if (in.blk_NO > 0) {
        pc_status st = assemble_one(p, in, s);
        if (st != PC_OK) return st;
        double* keep = nullptr;
        const size_t bytes = sizeof(double) * (size_t)(in.KMp * in.KMp);
        const bool copy = hipMalloc((void**)&keep, bytes) == hipSuccess;
        if (copy) PC_TRY(hipMemcpyAsync(keep, in.G, bytes, hipMemcpyDeviceToDevice, s));
        float bestb = 0.f;
        int64_t bw = in.blk_NO;
        int bt = 0;
        bool first = true;
        for (int64_t w : {(int64_t)1024, (int64_t)2048}) {
          if (w >= in.KMp) continue;
          st = alloc_blocked(in, w);
          if (st != PC_OK) break;
          for (int tile : {1, 2}) {
            in.tune_gemm_tile = tile;
            float tot = 0.f;
            for (int r = 0; r < 2 && st == PC_OK; ++r) {
              if (copy) {
                if (hipMemcpyAsync(in.G, keep, bytes, hipMemcpyDeviceToDevice, s) != hipSuccess) st = PC_ERR_DEVICE;
              } else {
                st = assemble_one(p, in, s);
              }
              float ms = 0.f;
              if (st == PC_OK)
                st = time_ms(s, 1, [&]() -> pc_status { PC_TRY(pc::launch_cholesky(in, s)); return PC_OK; }, &ms,
                             false);
              tot += ms;
            }
            if (st != PC_OK) break;
            if (first || tot < bestb) { bestb = tot; bw = w; bt = tile; first = false; }
          }
          if (st != PC_OK) break;
        }
        if (copy) { (void)hipStreamSynchronize(s); (void)hipFree(keep); }
        if (st != PC_OK) return st;
        if (in.blk_NO != bw) {
          st = alloc_blocked(in, bw);
          if (st != PC_OK) return st;
        }
        in.tune_gemm_tile = bt;
      }
    }
  }
  if (p->batch && any_measured) {
    float best = 0.f;
    for (int c = 2; c >= 1; --c) {
      float tot = 0.f;
      for (int r = 0; r < reps; ++r) {
        for (auto& in : p->inst) {
          pc_status st = assemble_one(p, in, s);
          if (st != PC_OK) return st;
        }
        hipEvent_t a = nullptr, b = nullptr;
        float ms = 0.f;
        PC_TRY(hipEventCreate(&a));
        PC_TRY(hipEventCreate(&b));
        PC_TRY(hipEventRecord(a, s));
        PC_TRY(pc::launch_cholesky_batch(p->batch, s, c));
        PC_TRY(hipEventRecord(b, s));
        PC_TRY(hipEventSynchronize(b));
        PC_TRY(hipEventElapsedTime(&ms, a, b));
        (void)hipEventDestroy(a);
        (void)hipEventDestroy(b);
        tot += ms;
      }
      if (c == 2 || tot < best) { best = tot; batch_per_cu = c; }
    }
    for (auto& in : p->inst) in.tune_chol_per_cu = batch_per_cu;
  }
  // keep the second Gram part only where it was chosen
  for (auto& in : p->inst)
    if (in.G2 && in.tune_gram_split == 1) {
      PC_TRY(hipStreamSynchronize(s));
      (void)hipFree(in.G2);
      in.G2 = nullptr;
      in.g2_parts = 0;
    }
  PC_TRY(hipStreamSynchronize(s));
  if (cache_path && any_measured) {
    for (const auto& in : p->inst) {
      const TuneKey key{in.n_h, in.n_w, in.K, in.M, in.max_rhs, prec};
      TuneEntry e{key, in.tune_gram_split, in.tune_ztx_split, in.tune_chol_per_cu, (int)in.blk_NO, in.tune_gemm_tile};
      bool found = false;
      for (auto& c : cache)
        if (c.key == key) { c = e; found = true; }
      if (!found) cache.push_back(e);
    }
    if (!write_tune_cache(cache_path, cache)) return PC_ERR_INVALID_ARG;
  }
  return PC_OK;
}

pc_status pc_set_tuning(pc_plan* p, int32_t instance, int32_t gram_split, int32_t ztx_split, int32_t chol_per_cu,
                        int32_t chol_block) {
  if (!p || instance < 0 || (size_t)instance >= p->inst.size()) return PC_ERR_INVALID_ARG;
  if (gram_split < 0 || gram_split > 4 || ztx_split < 0 || ztx_split > 2 || chol_per_cu < 0 || chol_per_cu > 2)
    return PC_ERR_INVALID_ARG;
  if (chol_block < -1 || (chol_block > 0 && (chol_block < 128 || chol_block % pc::NB != 0)))
    return PC_ERR_INVALID_ARG;
  if (chol_block != 0 && p->batch) return PC_ERR_INVALID_ARG;   // a batch factors every instance in one launch
  hipSetDevice(p->device);
  Inst& in = p->inst[instance];
  if (gram_split >= 2 && p->opt.precision == PC_PREC_FP64 && ensure_gram_parts(in, gram_split) != hipSuccess)
    return PC_ERR_OOM;
  if (chol_block != 0) {
    const pc_status bs = alloc_blocked(in, chol_block > 0 ? chol_block : 0);
    if (bs != PC_OK) return bs;
  }
  in.tune_gram_split = gram_split;
  in.tune_ztx_split = ztx_split;
  in.tune_chol_per_cu = chol_per_cu;
  if (p->batch)
    for (auto& o : p->inst) o.tune_chol_per_cu = chol_per_cu;
  in.factored = false;
  return PC_OK;
}

pc_status pc_set_tile_shape(pc_plan* p, int32_t instance, int32_t gemm_tile) {
  if (!p || instance < 0 || (size_t)instance >= p->inst.size() || gemm_tile < 0 || gemm_tile > 2)
    return PC_ERR_INVALID_ARG;
  p->inst[instance].tune_gemm_tile = gemm_tile;
  p->inst[instance].factored = false;
  return PC_OK;
}

pc_status pc_query_tile_shape(const pc_plan* p, int32_t instance, int32_t* gemm_tile) {
  if (!p || instance < 0 || (size_t)instance >= p->inst.size() || !gemm_tile) return PC_ERR_INVALID_ARG;
  *gemm_tile = p->inst[instance].tune_gemm_tile;
  return PC_OK;
}

pc_status pc_query_tuning(const pc_plan* p, int32_t instance, int32_t* gram_split, int32_t* ztx_split,
                          int32_t* chol_per_cu, int32_t* chol_block) {
  if (!p || instance < 0 || (size_t)instance >= p->inst.size()) return PC_ERR_INVALID_ARG;
  const Inst& in = p->inst[instance];
  if (gram_split) *gram_split = in.tune_gram_split;
  if (ztx_split) *ztx_split = in.tune_ztx_split;
  if (chol_per_cu) *chol_per_cu = in.tune_chol_per_cu;
  if (chol_block) *chol_block = (int32_t)in.blk_NO;
  return PC_OK;
}

}  // extern "C"
