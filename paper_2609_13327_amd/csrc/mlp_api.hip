// C-ABI of the warm-start network (contracts in include/pcsqrt.h): buffer
// management and the sequencing of the forward, backward and Adam kernels.
#include "pcsqrt.h"

#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <new>

#include "pc_internal.h"

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

void free_mlp(pc_mlp* m) {
  if (!m) return;
  (void)hipDeviceSynchronize();
  (void)hipFree(m->params); (void)hipFree(m->grads); (void)hipFree(m->m); (void)hipFree(m->v);
  (void)hipFree(m->Apre); (void)hipFree(m->H); (void)hipFree(m->Y); (void)hipFree(m->dY); (void)hipFree(m->dA);
  (void)hipFree(m->row_loss); (void)hipFree(m->loss); (void)hipFree(m->Xh); (void)hipFree(m->nrm); (void)hipFree(m->partial);
  delete m;
}

float* W1(pc_mlp* m) { return m->params; }
float* b1(pc_mlp* m) { return m->params + m->h * m->d; }
float* W2(pc_mlp* m) { return m->params + m->h * m->d + m->h; }
float* b2(pc_mlp* m) { return m->params + 2 * m->h * m->d + m->h; }


pc::MlpGemm gemm(const float* A, int64_t sam, int64_t sak, const float* B, int64_t sbn, int64_t sbk, int64_t M,
                 int64_t N, int64_t K, int mode, float* C, int64_t ldc, pc_mlp* m) {
  pc::MlpGemm g{};
  g.A = A; g.sam = sam; g.sak = sak; g.a_kcont = sak == 1 ? 1 : 0;
  g.B = B; g.sbn = sbn; g.sbk = sbk; g.b_kcont = sbk == 1 ? 1 : 0;
  g.M = M; g.N = N; g.K = K;
  g.mode = mode;
  g.C = C; g.ldc = ldc;
  g.partial = m->partial;
  g.max_splits = m->max_splits;
  g.partial_cap = (int64_t)m->max_splits * m->max_batch * std::max(m->d, m->h);
  return g;
}

// Apre = X W1^T + b1, H = gelu(Apre); Y = H W2^T + b2 (row-major, ldY)
pc_status forward(pc_mlp* m, const float* X, int64_t ldX, int64_t B, float* Y, int64_t ldY, hipStream_t s) {
  const int64_t d = m->d, h = m->h;
  pc::MlpGemm g1 = gemm(X, ldX, 1, W1(m), d, 1, B, h, d, pc::MLP_EPI_BIAS_GELU, m->Apre, h, m);
  g1.bias = b1(m);
  g1.C2 = m->H;
  PC_TRY(pc::launch_mlp_gemm(g1, m->bf16, s));
  pc::MlpGemm g2 = gemm(m->H, h, 1, W2(m), h, 1, B, d, h, pc::MLP_EPI_BIAS, Y, ldY, m);
  g2.bias = b2(m);
  PC_TRY(pc::launch_mlp_gemm(g2, m->bf16, s));
  return PC_OK;
}

// loss and gradients into m->grads (and m->loss)
pc_status gradients(pc_mlp* m, const float* X, int64_t ldX, const float* T, int64_t ldT, int64_t B, hipStream_t s) {
  const int64_t d = m->d, h = m->h;
  pc_status st = forward(m, X, ldX, B, m->Y, d, s);
  if (st != PC_OK) return st;
  PC_TRY(pc::launch_mlp_loss(m->Y, d, T, ldT, d, B, m->dY, m->row_loss, m->loss, s));
  float* gW1 = m->grads;
  float* gb1 = gW1 + h * d;
  float* gW2 = gb1 + h;
  float* gb2 = gW2 + d * h;
  // dW2 = dY^T H  (d x h)
  PC_TRY(pc::launch_mlp_gemm(gemm(m->dY, 1, d, m->H, 1, h, d, h, B, pc::MLP_EPI_STORE, gW2, h, m), m->bf16, s));
  PC_TRY(pc::launch_mlp_colsum(m->dY, d, B, d, gb2, s));
  // dA = (dY W2) * gelu'(Apre)  (B x h)
  pc::MlpGemm g = gemm(m->dY, d, 1, W2(m), 1, h, B, h, d, pc::MLP_EPI_GELU_GRAD, m->dA, h, m);
  g.aux = m->Apre;
  PC_TRY(pc::launch_mlp_gemm(g, m->bf16, s));
  // dW1 = dA^T X  (h x d)
  PC_TRY(pc::launch_mlp_gemm(gemm(m->dA, 1, h, X, 1, ldX, h, d, B, pc::MLP_EPI_STORE, gW1, d, m), m->bf16, s));
  PC_TRY(pc::launch_mlp_colsum(m->dA, h, B, h, gb1, s));
  return PC_OK;
}

bool batch_ok(const pc_mlp* m, const float* X, int64_t ldX, int64_t B) {
  return X && ldX >= m->d && B >= 1 && B <= m->max_batch;
}

}  // namespace

extern "C" {

pc_status pc_mlp_create(int64_t d, int64_t h, int64_t max_batch, int32_t operand_type, pc_mlp** out) {
  if (!out) return PC_ERR_INVALID_ARG;
  *out = nullptr;
  if (d < 1 || h < 1 || max_batch < 1) return PC_ERR_SHAPE;
  if (operand_type != PC_MLP_BF16 && operand_type != PC_MLP_FP32) return PC_ERR_INVALID_ARG;
  pc_mlp* m = new (std::nothrow) pc_mlp();
  if (!m) return PC_ERR_OOM;
  (void)hipGetDevice(&m->device);
  m->d = d; m->h = h; m->max_batch = max_batch; m->bf16 = operand_type == PC_MLP_BF16;
  m->nparams = 2 * h * d + h + d;
  hipError_t e = hipSuccess;
  auto chk = [&](hipError_t x) { if (x != hipSuccess && e == hipSuccess) e = x; };
  chk(dalloc(&m->params, m->nparams));
  chk(dalloc(&m->grads, m->nparams));
  chk(dalloc(&m->m, m->nparams));
  chk(dalloc(&m->v, m->nparams));
  chk(dalloc(&m->Apre, max_batch * h));
  chk(dalloc(&m->H, max_batch * h));
  chk(dalloc(&m->Y, max_batch * d));
  chk(dalloc(&m->dY, max_batch * d));
  chk(dalloc(&m->dA, max_batch * h));
  chk(dalloc(&m->row_loss, max_batch));
  chk(dalloc(&m->loss, 1));
  chk(dalloc(&m->Xh, max_batch * d));
  chk(dalloc(&m->nrm, max_batch));
  chk(dalloc(&m->partial, (int64_t)m->max_splits * max_batch * std::max(d, h)));
  if (e == hipSuccess) {
    chk(hipMemset(m->params, 0, sizeof(float) * (size_t)m->nparams));
    chk(hipMemset(m->m, 0, sizeof(float) * (size_t)m->nparams));
    chk(hipMemset(m->v, 0, sizeof(float) * (size_t)m->nparams));
  }
  if (e != hipSuccess) {
    free_mlp(m);
    return (e == hipErrorOutOfMemory || e == hipErrorMemoryAllocation) ? PC_ERR_OOM : PC_ERR_DEVICE;
  }
  *out = m;
  return PC_OK;
}

pc_status pc_mlp_destroy(pc_mlp* m) {
  free_mlp(m);
  return PC_OK;
}

pc_status pc_mlp_set_params(pc_mlp* m, const float* w1, const float* bb1, const float* w2, const float* bb2,
                            void* stream) {
  if (!m || !w1 || !bb1 || !w2 || !bb2) return PC_ERR_INVALID_ARG;
  (void)hipSetDevice(m->device);
  hipStream_t s = (hipStream_t)stream;
  const int64_t d = m->d, h = m->h;
  PC_TRY(hipMemcpyAsync(W1(m), w1, sizeof(float) * (size_t)(h * d), hipMemcpyDeviceToDevice, s));
  PC_TRY(hipMemcpyAsync(b1(m), bb1, sizeof(float) * (size_t)h, hipMemcpyDeviceToDevice, s));
  PC_TRY(hipMemcpyAsync(W2(m), w2, sizeof(float) * (size_t)(d * h), hipMemcpyDeviceToDevice, s));
  PC_TRY(hipMemcpyAsync(b2(m), bb2, sizeof(float) * (size_t)d, hipMemcpyDeviceToDevice, s));
  PC_TRY(hipMemsetAsync(m->m, 0, sizeof(float) * (size_t)m->nparams, s));
  PC_TRY(hipMemsetAsync(m->v, 0, sizeof(float) * (size_t)m->nparams, s));
  m->step = 0;
  return PC_OK;
}

pc_status pc_mlp_get_params(const pc_mlp* mc, float* w1, float* bb1, float* w2, float* bb2, void* stream) {
  if (!mc) return PC_ERR_INVALID_ARG;
  pc_mlp* m = const_cast<pc_mlp*>(mc);
  (void)hipSetDevice(m->device);
  hipStream_t s = (hipStream_t)stream;
  const int64_t d = m->d, h = m->h;
  if (w1) PC_TRY(hipMemcpyAsync(w1, W1(m), sizeof(float) * (size_t)(h * d), hipMemcpyDeviceToDevice, s));
  if (bb1) PC_TRY(hipMemcpyAsync(bb1, b1(m), sizeof(float) * (size_t)h, hipMemcpyDeviceToDevice, s));
  if (w2) PC_TRY(hipMemcpyAsync(w2, W2(m), sizeof(float) * (size_t)(d * h), hipMemcpyDeviceToDevice, s));
  if (bb2) PC_TRY(hipMemcpyAsync(bb2, b2(m), sizeof(float) * (size_t)d, hipMemcpyDeviceToDevice, s));
  return PC_OK;
}

pc_status pc_mlp_forward(pc_mlp* m, const float* X, int64_t ldX, int64_t B, float* Y, int64_t ldY, void* stream) {
  if (!m || !batch_ok(m, X, ldX, B) || !Y || ldY < m->d) return PC_ERR_INVALID_ARG;
  (void)hipSetDevice(m->device);
  return forward(m, X, ldX, B, Y, ldY, (hipStream_t)stream);
}

pc_status pc_mlp_gradients(pc_mlp* m, const float* X, int64_t ldX, const float* T, int64_t ldT, int64_t B,
                           float* loss, float* dW1, float* db1, float* dW2, float* db2, void* stream) {
  if (!m || !batch_ok(m, X, ldX, B) || !T || ldT < m->d) return PC_ERR_INVALID_ARG;
  (void)hipSetDevice(m->device);
  hipStream_t s = (hipStream_t)stream;
  pc_status st = gradients(m, X, ldX, T, ldT, B, s);
  if (st != PC_OK) return st;
  const int64_t d = m->d, h = m->h;
  const float* g = m->grads;
  if (loss) PC_TRY(hipMemcpyAsync(loss, m->loss, sizeof(float), hipMemcpyDeviceToDevice, s));
  if (dW1) PC_TRY(hipMemcpyAsync(dW1, g, sizeof(float) * (size_t)(h * d), hipMemcpyDeviceToDevice, s));
  if (db1) PC_TRY(hipMemcpyAsync(db1, g + h * d, sizeof(float) * (size_t)h, hipMemcpyDeviceToDevice, s));
  if (dW2) PC_TRY(hipMemcpyAsync(dW2, g + h * d + h, sizeof(float) * (size_t)(d * h), hipMemcpyDeviceToDevice, s));
  if (db2) PC_TRY(hipMemcpyAsync(db2, g + 2 * h * d + h, sizeof(float) * (size_t)d, hipMemcpyDeviceToDevice, s));
  return PC_OK;
}

pc_status pc_mlp_train_step(pc_mlp* m, const float* X, int64_t ldX, const float* T, int64_t ldT, int64_t B,
                            float lr, float* loss, void* stream) {
  if (!m || !batch_ok(m, X, ldX, B) || !T || ldT < m->d || !(lr > 0.f)) return PC_ERR_INVALID_ARG;
  (void)hipSetDevice(m->device);
  hipStream_t s = (hipStream_t)stream;
  pc_status st = gradients(m, X, ldX, T, ldT, B, s);
  if (st != PC_OK) return st;
  m->step += 1;
  const double b1c = 0.9, b2c = 0.999;
  pc::AdamCoef c;
  c.lr = lr;
  c.b1 = (float)b1c;
  c.b2 = (float)b2c;
  c.omb1 = (float)(1.0 - b1c);
  c.omb2 = (float)(1.0 - b2c);
  c.bc1 = (float)(1.0 - std::pow(b1c, (double)m->step));
  c.bc2 = (float)(1.0 - std::pow(b2c, (double)m->step));
  c.eps = 1e-8f;
  PC_TRY(pc::launch_mlp_adam(m->params, m->grads, m->m, m->v, m->nparams, c, s));
  if (loss) PC_TRY(hipMemcpyAsync(loss, m->loss, sizeof(float), hipMemcpyDeviceToDevice, s));
  return PC_OK;
}

pc_status pc_mlp_warm_start(pc_mlp* m, const double* B, int64_t ldB, int64_t R, double* Y0, int64_t ldY0,
                            void* stream) {
  if (!m || !B || !Y0 || ldB < m->d || ldY0 < m->d || R < 0 || R > m->max_batch) return PC_ERR_INVALID_ARG;
  if (R == 0) return PC_OK;
  (void)hipSetDevice(m->device);
  hipStream_t s = (hipStream_t)stream;
  const int64_t d = m->d;
  PC_TRY(pc::launch_ws_prep(B, ldB, d, R, m->Xh, d, m->nrm, s));
  pc_status st = forward(m, m->Xh, d, R, m->Y, d, s);
  if (st != PC_OK) return st;
  PC_TRY(pc::launch_ws_finish(m->Y, d, m->nrm, d, R, Y0, ldY0, s));
  return PC_OK;
}

pc_status pc_mlp_training_pairs(const double* B, int64_t ldB, const double* Y, int64_t ldY, int64_t d, int64_t N,
                                float* X, int64_t ldX, float* T, int64_t ldT, void* stream) {
  if (d < 1 || N < 0) return PC_ERR_SHAPE;
  if (N == 0) return PC_OK;
  if (!B || !Y || !X || !T || ldB < d || ldY < d || ldX < d || ldT < d) return PC_ERR_INVALID_ARG;
  PC_TRY(pc::launch_training_pairs(B, ldB, Y, ldY, d, N, X, ldX, T, ldT, (hipStream_t)stream));
  return PC_OK;
}

}  // extern "C"
