// C ABI of the warm-start network (pdhcg_mlp_*): buffers, forward pass,
// training step (forward, MSE gradient, backward, Adam).
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstring>
#include <new>
#include <vector>

#include "mlp.hpp"
#include "pdhcg.h"

using namespace pdhcg;

namespace {

constexpr size_t WORK_FLOATS = (size_t)16 << 20;   // split-K partials (64 MiB)

struct Layer {
  int K = 0, N = 0;
  float* W = nullptr;     // FP32 master, K x N
  __bf16* Wb = nullptr;   // BF16 copy
  float* b = nullptr;
  float *mW = nullptr, *vW = nullptr, *mb = nullptr, *vb = nullptr;   // Adam moments
  float *dW = nullptr, *db = nullptr;                                 // last gradients
};

struct Mlp {
  std::vector<int> dims;
  int L = 0, max_batch = 0;
  hipStream_t st = nullptr;
  std::vector<Layer> layers;
  __bf16* X = nullptr;              // input, BF16
  std::vector<__bf16*> H;           // H[l], l = 1..L-1 (BF16), H[0] = X
  float* Yhat = nullptr;            // output, FP32
  __bf16* dz[2] = {nullptr, nullptr};
  float* work = nullptr;
  double* part = nullptr;           // loss partials
  double* dloss = nullptr;
  long long t = 0;                  // Adam step count
  std::vector<void*> ptrs;
  hipError_t err = hipSuccess;

  template <class T>
  T* alloc(size_t n) {
    if (err != hipSuccess) return nullptr;
    void* p = nullptr;
    err = hipMalloc(&p, std::max<size_t>(n, 1) * sizeof(T));
    if (err != hipSuccess) return nullptr;
    ptrs.push_back(p);
    return (T*)p;
  }
  void release() {
    for (void* p : ptrs) (void)hipFree(p);
    ptrs.clear();
  }
};

#define MCHK(expr)                         \
  do {                                     \
    if ((expr) != hipSuccess) return PDHCG_E_HIP; \
  } while (0)

int forward(Mlp* h, const float* x, int B) {
  MCHK(mlp_to_bf16(x, h->X, (long)B * h->dims[0], h->st));
  for (int l = 0; l < h->L; ++l) {
    Layer& ly = h->layers[l];
    const __bf16* in = l == 0 ? h->X : h->H[l];
    if (l < h->L - 1)
      MCHK(mlp_gemm(in, false, ly.K, ly.Wb, false, ly.N, B, ly.N, ly.K, EPI_BIAS_RELU_BF16, ly.b, nullptr,
                    nullptr, h->H[l + 1], h->work, WORK_FLOATS, h->st));
    else
      MCHK(mlp_gemm(in, false, ly.K, ly.Wb, false, ly.N, B, ly.N, ly.K, EPI_BIAS_F32, ly.b, nullptr, h->Yhat,
                    nullptr, h->work, WORK_FLOATS, h->st));
  }
  return PDHCG_OK;
}

}  // namespace

extern "C" {

int pdhcg_mlp_create(int32_t layers, const int32_t* dims, int32_t max_batch, void* stream, void** out) {
  if (!out) return PDHCG_E_ARG;
  *out = nullptr;
  if (layers < 1 || !dims || max_batch < 1) return PDHCG_E_ARG;
  for (int l = 0; l <= layers; ++l)
    if (dims[l] < 1) return PDHCG_E_SHAPE;
  Mlp* h = new (std::nothrow) Mlp();
  if (!h) return PDHCG_E_MEM;
  h->L = layers;
  h->dims.assign(dims, dims + layers + 1);
  h->max_batch = max_batch;
  h->st = (hipStream_t)stream;
  h->layers.resize(layers);
  int dmax = 0;
  for (int l = 0; l < layers; ++l) {
    Layer& ly = h->layers[l];
    ly.K = dims[l];
    ly.N = dims[l + 1];
    const size_t kn = (size_t)ly.K * ly.N;
    ly.W = h->alloc<float>(kn);
    ly.Wb = h->alloc<__bf16>(kn);
    ly.b = h->alloc<float>(ly.N);
    ly.mW = h->alloc<float>(kn);
    ly.vW = h->alloc<float>(kn);
    ly.mb = h->alloc<float>(ly.N);
    ly.vb = h->alloc<float>(ly.N);
    ly.dW = h->alloc<float>(kn);
    ly.db = h->alloc<float>(ly.N);
    dmax = std::max(dmax, ly.N);
  }
  h->X = h->alloc<__bf16>((size_t)max_batch * dims[0]);
  h->H.assign(layers, nullptr);
  h->H[0] = h->X;
  for (int l = 1; l < layers; ++l) h->H[l] = h->alloc<__bf16>((size_t)max_batch * dims[l]);
  h->Yhat = h->alloc<float>((size_t)max_batch * dims[layers]);
  h->dz[0] = h->alloc<__bf16>((size_t)max_batch * dmax);
  h->dz[1] = h->alloc<__bf16>((size_t)max_batch * dmax);
  h->work = h->alloc<float>(WORK_FLOATS);
  h->part = h->alloc<double>(1024);
  h->dloss = h->alloc<double>(1);
  if (h->err != hipSuccess) {
    const int rc = h->err == hipErrorOutOfMemory ? PDHCG_E_MEM : PDHCG_E_HIP;
    h->release();
    delete h;
    return rc;
  }
  for (auto& ly : h->layers) {
    const size_t kn = (size_t)ly.K * ly.N;
    if (hipMemsetAsync(ly.W, 0, kn * 4, h->st) != hipSuccess || hipMemsetAsync(ly.Wb, 0, kn * 2, h->st) != hipSuccess ||
        hipMemsetAsync(ly.b, 0, ly.N * 4, h->st) != hipSuccess || hipMemsetAsync(ly.mW, 0, kn * 4, h->st) != hipSuccess ||
        hipMemsetAsync(ly.vW, 0, kn * 4, h->st) != hipSuccess || hipMemsetAsync(ly.mb, 0, ly.N * 4, h->st) != hipSuccess ||
        hipMemsetAsync(ly.vb, 0, ly.N * 4, h->st) != hipSuccess) {
      h->release();
      delete h;
      return PDHCG_E_HIP;
    }
  }
  if (hipStreamSynchronize(h->st) != hipSuccess) {
    h->release();
    delete h;
    return PDHCG_E_HIP;
  }
  *out = h;
  return PDHCG_OK;
}

int pdhcg_mlp_set_params(void* hv, int32_t layer, const float* W, const float* b) {
  Mlp* h = (Mlp*)hv;
  if (!h || layer < 0 || layer >= h->L || !W || !b) return PDHCG_E_ARG;
  Layer& ly = h->layers[layer];
  const size_t kn = (size_t)ly.K * ly.N;
  MCHK(hipMemcpyAsync(ly.W, W, kn * 4, hipMemcpyHostToDevice, h->st));
  MCHK(hipMemcpyAsync(ly.b, b, ly.N * 4, hipMemcpyHostToDevice, h->st));
  MCHK(mlp_to_bf16(ly.W, ly.Wb, (long)kn, h->st));
  MCHK(hipMemsetAsync(ly.mW, 0, kn * 4, h->st));
  MCHK(hipMemsetAsync(ly.vW, 0, kn * 4, h->st));
  MCHK(hipMemsetAsync(ly.mb, 0, ly.N * 4, h->st));
  MCHK(hipMemsetAsync(ly.vb, 0, ly.N * 4, h->st));
  h->t = 0;
  MCHK(hipStreamSynchronize(h->st));
  return PDHCG_OK;
}

int pdhcg_mlp_get_params(void* hv, int32_t layer, float* W, float* b) {
  Mlp* h = (Mlp*)hv;
  if (!h || layer < 0 || layer >= h->L) return PDHCG_E_ARG;
  Layer& ly = h->layers[layer];
  if (W) MCHK(hipMemcpyAsync(W, ly.W, (size_t)ly.K * ly.N * 4, hipMemcpyDeviceToHost, h->st));
  if (b) MCHK(hipMemcpyAsync(b, ly.b, ly.N * 4, hipMemcpyDeviceToHost, h->st));
  MCHK(hipStreamSynchronize(h->st));
  return PDHCG_OK;
}

int pdhcg_mlp_get_grads(void* hv, int32_t layer, float* dW, float* db) {
  Mlp* h = (Mlp*)hv;
  if (!h || layer < 0 || layer >= h->L) return PDHCG_E_ARG;
  Layer& ly = h->layers[layer];
  if (dW) MCHK(hipMemcpyAsync(dW, ly.dW, (size_t)ly.K * ly.N * 4, hipMemcpyDeviceToHost, h->st));
  if (db) MCHK(hipMemcpyAsync(db, ly.db, ly.N * 4, hipMemcpyDeviceToHost, h->st));
  MCHK(hipStreamSynchronize(h->st));
  return PDHCG_OK;
}

int pdhcg_mlp_forward(void* hv, const float* x, int32_t batch, float* y) {
  Mlp* h = (Mlp*)hv;
  if (!h || !x || !y || batch < 1 || batch > h->max_batch) return PDHCG_E_ARG;
  int rc = forward(h, x, batch);
  if (rc != PDHCG_OK) return rc;
  MCHK(hipMemcpyAsync(y, h->Yhat, (size_t)batch * h->dims[h->L] * 4, hipMemcpyDeviceToDevice, h->st));
  return PDHCG_OK;
}

int pdhcg_mlp_train_step(void* hv, const float* x, const float* y, int32_t batch, const pdhcg_adam* opt,
                         double* loss) {
  Mlp* h = (Mlp*)hv;
  if (!h || !x || !y || batch < 1 || batch > h->max_batch) return PDHCG_E_ARG;
  const int B = batch, L = h->L, dL = h->dims[L];
  int rc = forward(h, x, B);
  if (rc != PDHCG_OK) return rc;
  int cur = 0;
  MCHK(mlp_mse_grad(h->Yhat, y, h->dz[cur], (long)B * dL, (float)(2.0 / ((double)B * dL)), h->part, h->dloss,
                    h->st));
  for (int l = L - 1; l >= 0; --l) {
    Layer& ly = h->layers[l];
    const __bf16* in = h->H[l];     // H_{l} of the docs: the layer's input activations
    // dW = in^T dz  (M = K_in, N = N_out, K = batch)
    MCHK(mlp_gemm(in, true, ly.K, h->dz[cur], false, ly.N, ly.K, ly.N, B, EPI_F32, nullptr, nullptr, ly.dW,
                  nullptr, h->work, WORK_FLOATS, h->st));
    MCHK(mlp_colsum(h->dz[cur], B, ly.N, ly.db, h->st));
    if (l > 0) {
      // dz_prev = (dz W^T) masked by in > 0   (M = batch, N = K_in, K = N_out)
      MCHK(mlp_gemm(h->dz[cur], false, ly.N, ly.Wb, true, ly.N, B, ly.K, ly.N, EPI_MASK_BF16, nullptr, in,
                    nullptr, h->dz[1 - cur], h->work, WORK_FLOATS, h->st));
      cur = 1 - cur;
    }
  }
  if (opt) {
    h->t += 1;
    AdamStep a;
    a.lr = (float)opt->lr;
    a.b1 = (float)opt->beta1;
    a.b2 = (float)opt->beta2;
    a.eps = (float)opt->eps;
    a.omb1 = (float)(1.0 - opt->beta1);
    a.omb2 = (float)(1.0 - opt->beta2);
    a.c1 = (float)(1.0 - std::pow(opt->beta1, (double)h->t));
    a.c2 = (float)(1.0 - std::pow(opt->beta2, (double)h->t));
    for (auto& ly : h->layers) {
      MCHK(mlp_adam(ly.W, ly.Wb, ly.dW, ly.mW, ly.vW, (long)ly.K * ly.N, a, h->st));
      MCHK(mlp_adam(ly.b, nullptr, ly.db, ly.mb, ly.vb, ly.N, a, h->st));
    }
  }
  if (loss) {
    double s = 0.0;
    MCHK(hipMemcpyAsync(&s, h->dloss, sizeof(double), hipMemcpyDeviceToHost, h->st));
    MCHK(hipStreamSynchronize(h->st));
    *loss = s / ((double)B * dL);
  }
  return PDHCG_OK;
}

void pdhcg_mlp_free(void* hv) {
  Mlp* h = (Mlp*)hv;
  if (!h) return;
  (void)hipStreamSynchronize(h->st);
  h->release();
  delete h;
}

}  // extern "C"
