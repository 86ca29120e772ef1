// Host entry points of the warm-start network kernels (mlp.hip).
#pragma once
#include <hip/hip_runtime.h>

#include <stddef.h>

namespace pdhcg {

// GEMM epilogues
enum : int {
  EPI_F32 = 0,          // out = acc                       (FP32)
  EPI_BIAS_F32,         // out = acc + bias[n]             (FP32)
  EPI_BIAS_RELU_BF16,   // out = bf16(max(acc + bias, 0))
  EPI_MASK_BF16         // out = bf16(mask > 0 ? acc : 0)
};

struct AdamStep {
  float lr, b1, b2, eps;
  float omb1, omb2;     // 1 - b1, 1 - b2 (formed in FP64: 1 - 0.999f loses digits)
  float c1, c2;         // bias corrections 1 - b1^t, 1 - b2^t
};

// C = op(A) op(B) with the epilogue `epi`; `work` holds split-K partials
hipError_t mlp_gemm(const __bf16* A, bool ta, long lda, const __bf16* B, bool tb, long ldb, int M, int N,
                    int K, int epi, const float* bias, const __bf16* mask, float* outf, __bf16* outb,
                    float* work, size_t work_floats, hipStream_t st);
hipError_t mlp_to_bf16(const float* x, __bf16* y, long n, hipStream_t st);
// dz = bf16(scale (yhat - y)); *loss = sum (yhat - y)^2 (device scalar)
hipError_t mlp_mse_grad(const float* yhat, const float* y, __bf16* dz, long n, float scale, double* part,
                        double* loss, hipStream_t st);
hipError_t mlp_colsum(const __bf16* dz, int rows, int N, float* db, hipStream_t st);
hipError_t mlp_adam(float* w, __bf16* wb, const float* g, float* m, float* v, long n, const AdamStep& a,
                    hipStream_t st);

}  // namespace pdhcg
