// Software-pipelined FP64 MFMA main loop shared by the GEMM-shaped kernels.
//
// A "problem" type P supplies the tile geometry and how operand chunks are
// formed; the loop double-buffers the chunks in LDS (one barrier per chunk):
//   P::BM, P::BN  workgroup tile (rows x cols), P::WM x P::WN waves (64 P::WM P::WN threads)
//   P::KC         contraction rows per chunk (multiple of 4)
//   P::LDA/LDB    LDS row strides (>= BM / BN)
//   struct Ctx    per-tile state; P::ctx(tile_index) builds it (valid=false skips)
//   ARegs/BRegs   register staging of one chunk
//   loadA/loadB(ctx, chunk, regs) global -> registers
//   storeA/storeB(regs, lds)      registers -> LDS (As[k][row], Bs[k][col])
//   epilogue(ctx, acc)            consume the accumulator tile
//   OCC (optional)                waves per SIMD the register allocation must allow
//   XA, XB (optional)             operand stored row-XOR swizzled in LDS (TileF64::mma)
#pragma once
#include "pc_common.h"

#include <type_traits>

namespace pc {

template <class P, class = void>
struct gemm_occupancy { static constexpr int value = 1; };
template <class P>
struct gemm_occupancy<P, std::void_t<decltype(P::OCC)>> { static constexpr int value = P::OCC; };
template <class P, class = void>
struct gemm_swizzle { static constexpr bool a = false, b = false; };
template <class P>
struct gemm_swizzle<P, std::void_t<decltype(P::XA)>> { static constexpr bool a = P::XA, b = P::XB; };

template <class P>
__device__ __forceinline__ void gemm_tile_f64(const P& prob, const typename P::Ctx& ctx,
                                              TileF64<P::BM, P::BN, P::WM, P::WN>& acc,
                                              double* As0, double* Bs0) {
  constexpr int ASZ = P::KC * P::LDA, BSZ = P::KC * P::LDB;
  acc.zero();
  const int nk = ctx.nchunks;
  if (nk <= 0) return;
  typename P::ARegs ar;
  typename P::BRegs br;
  prob.loadA(ctx, 0, ar);
  prob.loadB(ctx, 0, br);
  prob.storeA(ar, As0);
  prob.storeB(br, Bs0);
  __syncthreads();
  for (int c = 0; c < nk; ++c) {
    const bool more = c + 1 < nk;
    if (more) {
      prob.loadA(ctx, c + 1, ar);
      prob.loadB(ctx, c + 1, br);
    }
    acc.template mma<P::KC, P::LDA, P::LDB, gemm_swizzle<P>::a, gemm_swizzle<P>::b>(As0 + (c & 1) * ASZ,
                                                                                  Bs0 + (c & 1) * BSZ);
    if (more) {
      prob.storeA(ar, As0 + ((c + 1) & 1) * ASZ);
      prob.storeB(br, Bs0 + ((c + 1) & 1) * BSZ);
    }
    __syncthreads();
  }
}


// P::WM * P::WN waves per workgroup (64 * WM * WN threads)
template <class P>
__global__ __launch_bounds__(64 * P::WM * P::WN, gemm_occupancy<P>::value) void gemm_f64_kernel(P prob) {
  __shared__ double As[2 * P::KC * P::LDA];
  __shared__ double Bs[2 * P::KC * P::LDB];
  const typename P::Ctx ctx = prob.ctx(blockIdx.x);
  if (!ctx.valid) return;
  TileF64<P::BM, P::BN, P::WM, P::WN> acc;
  gemm_tile_f64(prob, ctx, acc, As, Bs);
  prob.epilogue(ctx, acc);
}

}  // namespace pc
