// The Hybrid covariance product in standardized variables (Sec. 2.2, eq.
// svCBKHybrid):
//     P~h v = (1 - beta_e) v + beta_e (C~ o P~e) v,   P~e = E~ E~^T,  C~ = W~ W~^T.
// By the Schur product identity the paper uses for the localized square root
// (Sec. 3.7, eq. SQRTofPCModulation), C~ o (E~ E~^T) = Z~ Z~^T with Z~ the
// columns e~_k o w~_m, so the product is two structured products with Z~,
//     b = Z~^T v,   out = (1 - beta_e) v + beta_e Z~ b,
// the second with the combination fused into its epilogue.  Neither Z~ nor
// an n~ x n~ matrix is formed.
#include <cmath>

#include "pcsqrt.h"
#include "pc_internal.h"

extern "C" pc_status pc_hybrid_apply(const pc_instance* hybrid, double beta_e, const double* V, int64_t ldV,
                                     int64_t R, double* Out, int64_t ldOut, double* work, int64_t ldwork,
                                     void* stream) {
  if (!hybrid) return PC_ERR_INVALID_ARG;
  const pc_instance& a = *hybrid;
  if (a.n_h < 1 || a.n_w < 1 || a.K < 1 || a.M < 1 || R < 0) return PC_ERR_SHAPE;
  if (!a.E || !a.W || a.ldE < a.n_h * a.n_w || a.ldW < a.n_h) return PC_ERR_INVALID_ARG;
  if (!std::isfinite(beta_e) || beta_e < 0.0 || beta_e > 1.0) return PC_ERR_INVALID_ARG;
  if (R == 0) return PC_OK;
  const int64_t n = a.n_h * a.n_w, KM = a.K * a.M;
  if (!V || !Out || !work || ldV < n || ldOut < n || ldwork < KM) return PC_ERR_INVALID_ARG;
  pc::Inst in;
  in.n_h = a.n_h; in.n_w = a.n_w; in.K = a.K; in.M = a.M;
  in.n = n; in.KM = KM; in.KMp = pc::round_up(KM, pc::NB);
  in.E = a.E; in.ldE = a.ldE; in.W = a.W; in.ldW = a.ldW;
  hipStream_t s = (hipStream_t)stream;
  if (pc::launch_ztx(in, V, ldV, R, work, ldwork, s) != hipSuccess) return PC_ERR_DEVICE;
  if (pc::launch_zy_axpby(in, work, ldwork, R, V, ldV, 1.0 - beta_e, beta_e, Out, ldOut, s) != hipSuccess)
    return PC_ERR_DEVICE;
  return PC_OK;
}
