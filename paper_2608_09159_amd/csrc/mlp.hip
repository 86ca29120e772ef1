// Kernels of the warm-start network: a ReLU MLP trained and evaluated with
// BF16 matrix operands on the gfx950 matrix cores (FP32 accumulation), FP32
// master weights and Adam.
//
// GEMM: C[M x N] = op(A)[M x K] * op(B)[K x N], all matrices row-major.
//   A: M x K (TA = false) or stored K x M (TA = true, used transposed)
//   B: K x N (TB = false) or stored N x K (TB = true, used transposed)
// Workgroup tile 128 x 128 x TK, four waves, each wave a 64 x 64 output block
// (2 x 2 blocks of v_mfma_f32_32x32x16_bf16, TK / 16 steps per stage).  Both
// operand tiles are staged in LDS with K contiguous (row stride padded by 8
// elements), so every lane reads its 8-element fragment with one 16-byte LDS
// load; global loads are 8-byte runs along the contiguous dimension.  Long K is split over `splits` workgroups writing FP32 partial tiles;
// a second kernel sums them in a fixed order and applies the epilogue, so
// results do not depend on scheduling.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <algorithm>

#include "mlp.hpp"

namespace pdhcg {
namespace {

typedef __bf16 bf16x8 __attribute__((ext_vector_type(8)));
typedef float f32x16 __attribute__((ext_vector_type(16)));

constexpr int TM = 128, TN = 128, TK = 64, LDK = TK + 8;
constexpr int GT = 256;   // threads per GEMM workgroup (4 waves, 2 x 2 of 64 x 64)
constexpr int VW = 4;     // elements per vector load (8 bytes)

typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));

struct GemmArgs {
  const __bf16* A;
  const __bf16* B;
  long lda, ldb;
  int M, N, K;
  int kchunk;             // K range of one split (multiple of TK)
  int epi;
  int vec_a, vec_b;       // leading dimension a multiple of VW: vector loads
  const float* bias;      // EPI_BIAS_*
  const __bf16* mask;     // EPI_MASK_BF16: M x N, ld = N
  float* outf;            // FP32 output (ld = N) or partials [splits][M][N]
  __bf16* outb;           // BF16 output (ld = N)
  int partial;            // 1: write FP32 partials of split blockIdx.z
};

__device__ __forceinline__ void epilogue(const GemmArgs& g, int m, int n, float acc) {
  const size_t o = (size_t)m * g.N + n;
  switch (g.epi) {
    case EPI_F32: g.outf[o] = acc; break;
    case EPI_BIAS_F32: g.outf[o] = acc + g.bias[n]; break;
    case EPI_BIAS_RELU_BF16: g.outb[o] = (__bf16)fmaxf(acc + g.bias[n], 0.0f); break;
    case EPI_MASK_BF16: g.outb[o] = (__bf16)((float)g.mask[o] > 0.0f ? acc : 0.0f); break;
    default: break;
  }
}

// VW consecutive elements src[0..VW) along the contiguous dimension, zero
// past `lim` (elements from the start of the run) or outside the tile
__device__ __forceinline__ bf16x4 load_run(const __bf16* src, int lim, bool vec) {
  bf16x4 v;
  if (vec && lim >= VW) {
    v = *reinterpret_cast<const bf16x4*>(src);
  } else {
    const __bf16 z = (__bf16)0.0f;
#pragma unroll
    for (int j = 0; j < VW; ++j) v[j] = j < lim ? src[j] : z;
  }
  return v;
}

// LDS column of element (row r, k): the 8-element k groups of a row are
// XOR-permuted by (r / 16) so that both the staging writes and the
// fragment reads spread over the banks (2-way and 4-way, the minimum for
// 8- and 16-byte accesses of a wave)
__device__ __forceinline__ int kswz(int r, int k) {
  return ((((k >> 3) ^ (r >> 4)) & (TK / 8 - 1)) << 3) | (k & 7);
}

// one operand tile of R rows (m or n) x TK (k), staged through registers:
// k-contiguous storage (element (r, k) at P[r * ld + k]) as VW-runs of k;
// r-contiguous storage (element (r, k) at P[k * ld + r]) as 4 x 4 blocks,
// four runs of 4 rows transposed in registers into four runs of 4 k.
constexpr int NRUN = (TM * TK / VW) / GT;   // runs of VW elements per thread
static_assert((TM / 4) * (TK / 4) / GT * 4 == NRUN, "both staging forms use NRUN runs per thread");

// global -> registers (zero outside the matrix or past kend)
template <bool KCONTIG>
__device__ __forceinline__ void stage_load(bf16x4 (&x)[NRUN], const __bf16* P, long ld, int r0, int rmax,
                                           int k0, int kend, bool vec) {
  const int tid = threadIdx.x;
  const __bf16 zero = (__bf16)0.0f;
  if (KCONTIG) {
    constexpr int RUNS = TK / VW;
#pragma unroll
    for (int q = 0; q < NRUN; ++q) {
      const int v = tid + q * GT;
      const int row = r0 + v / RUNS, k = k0 + (v % RUNS) * VW;
      if (row < rmax && k < kend) x[q] = load_run(P + (size_t)row * ld + k, kend - k, vec);
      else x[q] = bf16x4{zero, zero, zero, zero};
    }
  } else {
    constexpr int RB = TM / 4;
#pragma unroll
    for (int q = 0; q < NRUN / 4; ++q) {
      const int b = tid + q * GT;
      const int row = r0 + (b % RB) * 4, kb = k0 + (b / RB) * 4;
#pragma unroll
      for (int t = 0; t < 4; ++t) {
        const int k = kb + t;
        if (row < rmax && k < kend) x[4 * q + t] = load_run(P + (size_t)k * ld + row, rmax - row, vec);
        else x[4 * q + t] = bf16x4{zero, zero, zero, zero};
      }
    }
  }
}

// registers -> S[row][k] (swizzled k groups)
template <bool KCONTIG>
__device__ __forceinline__ void stage_store(__bf16 (*S)[LDK], const bf16x4 (&x)[NRUN]) {
  const int tid = threadIdx.x;
  if (KCONTIG) {
    constexpr int RUNS = TK / VW;
#pragma unroll
    for (int q = 0; q < NRUN; ++q) {
      const int v = tid + q * GT;
      const int r = v / RUNS, kq = (v % RUNS) * VW;
      *reinterpret_cast<bf16x4*>(&S[r][kswz(r, kq)]) = x[q];
    }
  } else {
    constexpr int RB = TM / 4;
#pragma unroll
    for (int q = 0; q < NRUN / 4; ++q) {
      const int b = tid + q * GT;
      const int rb = (b % RB) * 4, kb = (b / RB) * 4;
#pragma unroll
      for (int j = 0; j < 4; ++j)
        *reinterpret_cast<bf16x4*>(&S[rb + j][kswz(rb + j, kb)]) =
            bf16x4{x[4 * q][j], x[4 * q + 1][j], x[4 * q + 2][j], x[4 * q + 3][j]};
    }
  }
}

template <bool TA, bool TB>
__global__ __launch_bounds__(GT) void gemm_kernel(GemmArgs g) {
  __shared__ __attribute__((aligned(16))) __bf16 As[TM][LDK];
  __shared__ __attribute__((aligned(16))) __bf16 Bs[TN][LDK];
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int m0 = blockIdx.y * TM, n0 = blockIdx.x * TN;
  const int kb = blockIdx.z * g.kchunk;
  const int ke = min(g.K, kb + g.kchunk);
  const int wm = (wv >> 1) * 64, wn = (wv & 1) * 64;
  f32x16 acc[2][2] = {};
  // the next stage's global loads are in flight while this stage computes
  bf16x4 xa[NRUN], xb[NRUN];
  if (kb < ke) {
    stage_load<!TA>(xa, g.A, g.lda, m0, g.M, kb, ke, g.vec_a != 0);
    stage_load<TB>(xb, g.B, g.ldb, n0, g.N, kb, ke, g.vec_b != 0);
  }
  for (int k0 = kb; k0 < ke; k0 += TK) {
    stage_store<!TA>(As, xa);
    stage_store<TB>(Bs, xb);
    __syncthreads();
    if (k0 + TK < ke) {
      stage_load<!TA>(xa, g.A, g.lda, m0, g.M, k0 + TK, ke, g.vec_a != 0);
      stage_load<TB>(xb, g.B, g.ldb, n0, g.N, k0 + TK, ke, g.vec_b != 0);
    }
    // lane l holds row/col (l % 32), k (l / 32) * 8 + j of each 32 x 32 x 16 step
#pragma unroll
    for (int ks = 0; ks < TK; ks += 16) {
      bf16x8 a[2], b[2];
#pragma unroll
      for (int i = 0; i < 2; ++i) {
        const int ra = wm + 32 * i + (lane & 31), rb = wn + 32 * i + (lane & 31);
        a[i] = *reinterpret_cast<const bf16x8*>(&As[ra][kswz(ra, ks + (lane >> 5) * 8)]);
        b[i] = *reinterpret_cast<const bf16x8*>(&Bs[rb][kswz(rb, ks + (lane >> 5) * 8)]);
      }
#pragma unroll
      for (int i = 0; i < 2; ++i)
#pragma unroll
        for (int j = 0; j < 2; ++j) acc[i][j] = __builtin_amdgcn_mfma_f32_32x32x16_bf16(a[i], b[j], acc[i][j], 0, 0, 0);
    }
    __syncthreads();
  }
  // ---- output: acc[i][j][e] is row (e / 4) * 8 + (l / 32) * 4 + e % 4 of block
  // i, column l % 32 of block j
#pragma unroll
  for (int i = 0; i < 2; ++i)
#pragma unroll
    for (int j = 0; j < 2; ++j) {
      const int n = n0 + wn + 32 * j + (lane & 31);
#pragma unroll
      for (int e = 0; e < 16; ++e) {
        const int m = m0 + wm + 32 * i + (e >> 2) * 8 + (lane >> 5) * 4 + (e & 3);
        if (m < g.M && n < g.N) {
          if (g.partial) g.outf[((size_t)blockIdx.z * g.M + m) * g.N + n] = acc[i][j][e];
          else epilogue(g, m, n, acc[i][j][e]);
        }
      }
    }
}

// sum the split-K partials in split order, then the epilogue
__global__ __launch_bounds__(256) void splitk_reduce_kernel(GemmArgs g, const float* part, int splits) {
  const long total = (long)g.M * g.N;
  for (long o = (long)blockIdx.x * 256 + threadIdx.x; o < total; o += (long)gridDim.x * 256) {
    float s = 0.0f;
    for (int z = 0; z < splits; ++z) s += part[(size_t)z * total + o];
    epilogue(g, (int)(o / g.N), (int)(o % g.N), s);
  }
}

__global__ __launch_bounds__(256) void to_bf16_kernel(const float* x, __bf16* y, long n) {
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) y[i] = (__bf16)x[i];
}

// dZ = bf16(scale * (yhat - y)); per-block partial of sum (yhat - y)^2 in FP64
__global__ __launch_bounds__(256) void mse_grad_kernel(const float* yhat, const float* y, __bf16* dz, long n,
                                                      float scale, double* part) {
  __shared__ double red[4];
  double s = 0.0;
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
    const float d = yhat[i] - y[i];
    dz[i] = (__bf16)(scale * d);
    s += (double)d * (double)d;
  }
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) part[blockIdx.x] = red[0] + red[1] + red[2] + red[3];
}

__global__ __launch_bounds__(64) void sum_partials_kernel(const double* part, int np, double* out) {
  // lane-strided sums, then a fixed-order wave reduction (deterministic)
  double s = 0.0;
  for (int i = threadIdx.x; i < np; i += 64) s += part[i];
  for (int o = 32; o >= 1; o >>= 1) s += __shfl_xor(s, o, 64);
  if (threadIdx.x == 0) out[0] = s;
}

// db[n] = sum over rows of dz[b][n] (FP32, rows in order; 8 loads in flight)
__global__ __launch_bounds__(256) void colsum_kernel(const __bf16* dz, int rows, int N, float* db) {
  const int n = blockIdx.x * 256 + threadIdx.x;
  if (n >= N) return;
  float s = 0.0f;
  int b = 0;
  for (; b + 8 <= rows; b += 8) {
    float v[8];
#pragma unroll
    for (int j = 0; j < 8; ++j) v[j] = (float)dz[(size_t)(b + j) * N + n];
#pragma unroll
    for (int j = 0; j < 8; ++j) s += v[j];
  }
  for (; b < rows; ++b) s += (float)dz[(size_t)b * N + n];
  db[n] = s;
}

__global__ __launch_bounds__(256) void adam_kernel(float* w, __bf16* wb, const float* g, float* m, float* v,
                                                  long n, AdamStep a) {
  for (long i = (long)blockIdx.x * 256 + threadIdx.x; i < n; i += (long)gridDim.x * 256) {
    const float gi = g[i];
    const float mi = a.b1 * m[i] + a.omb1 * gi;
    const float vi = a.b2 * v[i] + a.omb2 * gi * gi;
    m[i] = mi;
    v[i] = vi;
    const float wi = w[i] - a.lr * (mi / a.c1) / (sqrtf(vi / a.c2) + a.eps);
    w[i] = wi;
    if (wb) wb[i] = (__bf16)wi;
  }
}

int grid_for(long n, int per, int cap) {
  long g = (n + per - 1) / per;
  return (int)std::max<long>(1, std::min<long>(g, cap));
}

}  // namespace

hipError_t mlp_gemm(const __bf16* A, bool ta, long lda, const __bf16* B, bool tb, long ldb, int M, int N,
                    int K, int epi, const float* bias, const __bf16* mask, float* outf, __bf16* outb,
                    float* work, size_t work_floats, hipStream_t st) {
  if (M <= 0 || N <= 0) return hipSuccess;
  GemmArgs g{};
  g.A = A;
  g.B = B;
  g.lda = lda;
  g.ldb = ldb;
  g.M = M;
  g.N = N;
  g.K = K;
  g.epi = epi;
  g.vec_a = (lda % VW == 0) ? 1 : 0;
  g.vec_b = (ldb % VW == 0) ? 1 : 0;
  g.bias = bias;
  g.mask = mask;
  g.outf = outf;
  g.outb = outb;
  const int tiles = ((M + TM - 1) / TM) * ((N + TN - 1) / TN);
  // split K while the grid stays within one round of resident workgroups
  // (three per CU) and the partials fit
  const int ksteps = std::max(1, (K + TK - 1) / TK);
  int splits = 1;
  while (tiles * splits * 2 <= 768 && splits * 2 <= ksteps &&
         (size_t)(splits * 2) * (size_t)M * (size_t)N <= work_floats)
    splits *= 2;
  const int per = (ksteps + splits - 1) / splits;
  g.kchunk = per * TK;
  splits = (ksteps + per - 1) / per;
  dim3 grid((N + TN - 1) / TN, (M + TM - 1) / TM, splits);
  if (splits > 1) {
    g.partial = 1;
    GemmArgs p = g;
    p.outf = work;
    if (!ta && !tb) hipLaunchKernelGGL((gemm_kernel<false, false>), grid, dim3(GT), 0, st, p);
    else if (!ta && tb) hipLaunchKernelGGL((gemm_kernel<false, true>), grid, dim3(GT), 0, st, p);
    else if (ta && !tb) hipLaunchKernelGGL((gemm_kernel<true, false>), grid, dim3(GT), 0, st, p);
    else hipLaunchKernelGGL((gemm_kernel<true, true>), grid, dim3(GT), 0, st, p);
    g.partial = 0;
    hipLaunchKernelGGL(splitk_reduce_kernel, dim3(grid_for((long)M * N, 256, 4096)), dim3(256), 0, st, g,
                       work, splits);
  } else {
    g.partial = 0;
    if (!ta && !tb) hipLaunchKernelGGL((gemm_kernel<false, false>), grid, dim3(GT), 0, st, g);
    else if (!ta && tb) hipLaunchKernelGGL((gemm_kernel<false, true>), grid, dim3(GT), 0, st, g);
    else if (ta && !tb) hipLaunchKernelGGL((gemm_kernel<true, false>), grid, dim3(GT), 0, st, g);
    else hipLaunchKernelGGL((gemm_kernel<true, true>), grid, dim3(GT), 0, st, g);
  }
  return hipGetLastError();
}

hipError_t mlp_to_bf16(const float* x, __bf16* y, long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(to_bf16_kernel, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, x, y, n);
  return hipGetLastError();
}

hipError_t mlp_mse_grad(const float* yhat, const float* y, __bf16* dz, long n, float scale, double* part,
                        double* loss, hipStream_t st) {
  const int grid = grid_for(n, 256, 1024);
  hipLaunchKernelGGL(mse_grad_kernel, dim3(grid), dim3(256), 0, st, yhat, y, dz, n, scale, part);
  hipLaunchKernelGGL(sum_partials_kernel, dim3(1), dim3(64), 0, st, part, grid, loss);
  return hipGetLastError();
}

hipError_t mlp_colsum(const __bf16* dz, int rows, int N, float* db, hipStream_t st) {
  hipLaunchKernelGGL(colsum_kernel, dim3((N + 255) / 256), dim3(256), 0, st, dz, rows, N, db);
  return hipGetLastError();
}

hipError_t mlp_adam(float* w, __bf16* wb, const float* g, float* m, float* v, long n, const AdamStep& a,
                    hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(adam_kernel, dim3(grid_for(n, 256, 4096)), dim3(256), 0, st, w, wb, g, m, v, n, a);
  return hipGetLastError();
}

}  // namespace pdhcg
