// Persistent solver kernels for restarted PDHG on conic QP.
//
// Work decomposition: a "team" of workgroups solves one problem.  Each
// workgroup owns a contiguous range of coordinates (never splitting a cone
// block) and a contiguous range of rows of A, balanced by work on the host,
// so every per-coordinate step -- prox, cone projections, Halpern update --
// is local to the workgroup and needs only __syncthreads.  Grid barriers
// remain only where a global reduction or a gather over all coordinates is
// needed.  Every reduction is written as one partial per workgroup and
// re-reduced by every workgroup in the same fixed order (deterministic and
// identical everywhere), so all workgroups take the same control decisions
// (inner stop, restart, termination) without a host round trip.
//
// Outer iteration (reflected-Halpern epoch, eq. stored-pdhg-candidate and
// eq. rh-update; primal-first PDHG operator eq. theory-pdhg-map):
//   P1  own coordinates: A^T y (SpMV rows of A^T), v = x + tau A^T y.
//       Diagonal Q: x~ = (v - tau c)/(1 + tau q) (eq. diagonal-q-metric)
//       projected at once (elementwise cones, then own cone blocks in the
//       metric 1 + tau q).  General Q: g0 = Q x + c + (x - v)/tau and the first
//       Jacobi step with alpha = 1 (eq. jacobi-bb-step).             | barrier
//   P3  (general Q, repeated) g = Q u + c + (u - v)/tau, BB sums.    | barrier
//   P4  projected step with alpha = <s,Js>/<s,dg>; stop when the Euclidean
//       step norm <= eps_in (eq. current-inner-step-stop).           | barrier
//       With P diagonal or absent (grids), P3 and P4 share one barrier:
//       the BB sums of the step just taken are reduced with it, since the
//       gradient is affine in u (see the inner loop).
//   R u (dense factor) partials: grids form them after each coordinate pass
//   from the stored iterate (one wave per factor row); single-workgroup
//   teams accumulate them inside the pass.
//   P6  own rows: A w_x, w_y = y + sigma (b - (2 A w_x - A x)); on non-check
//       iterations the Halpern update of x, y, A x is fused.          | barrier
//   Check iterations (k = 0 of an epoch and every check_every evaluations):
//       fixed-point error E (eq. practical-fixed-point-movement), relative KKT
//       residuals of the unscaled candidate (one A^T pass + Euclidean cone
//       projections of -s), restart rule (eq. practical-restart-rule), PID
//       primal weight (eq. pid-error, pid-weight), then restart or Halpern.
#include <hip/hip_runtime.h>

#include <stdint.h>

#include <algorithm>
#include <mutex>
#include <type_traits>

#include "common.hpp"
#include "cones.hpp"
#include "solver.hpp"

namespace pdhcg {

constexpr int BLOCK = 512;
constexpr int NWAVE = BLOCK / 64;

constexpr int ITEM_CACHE = 256;   // cone items per kind cached in LDS
constexpr int ZCAP = 1024;        // coordinates whose projection inputs/outputs can stage in LDS

struct Lds {
  double red[16][NWAVE];
  double scal[SL_COUNT];
  double ht[RMAX];       // D^ h for the Q product of the current pass
  double Dl[RMAX * RMAX];  // D^ (r x r), staged once per run
  double hw[NWAVE][RMAX];   // per-wave R^ u accumulators (single-workgroup teams)
  double hu[RMAX];       // R^ u of the current inner iterate
  double hs[RMAX];       // R^ s, s = u - u_prev (one-sync inner step)
  // this workgroup's cone-item descriptors, copied once per launch when they
  // fit (read by every projection pass)
  int wst[ITEM_CACHE], wdim[ITEM_CACHE];
  unsigned char wtype[ITEM_CACHE], weu[ITEM_CACHE];
  int lst[ITEM_CACHE];
  unsigned char ltype[ITEM_CACHE], leu[ITEM_CACHE];
  double lal[ITEM_CACHE];
  // the inner step's cone-coordinate gradient and projected point, indexed
  // from the workgroup's first coordinate (when it owns at most ZCAP)
  double gl[ZCAP], zl[ZCAP];
  Ctl C;
  int flag;
  int done;
  int pcat;
  unsigned long long plast;
  unsigned epoch;
  unsigned long long pt[PT_COUNT];   // this workgroup's phase timers
};

// phase timer: charge the time since the last mark to the current category
// and switch to `cat` (thread 0 of the timing workgroup only)
__device__ __forceinline__ void tmark(Lds& L, bool on, int cat) {
  if (on && threadIdx.x == 0) {
    const unsigned long long t = wall_clock64();
    L.pt[L.pcat] += t - L.plast;
    L.plast = t;
    L.pcat = cat;
  }
}

// ---------------------------------------------------------------------------
// grid barrier.  Every workgroup writes back its L2 (agent-scope release
// fence) and stores the barrier epoch in its own arrival word; workgroup 0
// polls all arrival words and then publishes the epoch in the release word;
// everyone else polls the release word and invalidates its L2 (agent-scope
// acquire fence).  No atomic read-modify-write, one fence pair per
// workgroup.  Waits are bounded: after `limit` ticks of the constant-rate
// wall clock the abort flag is raised and every workgroup leaves the kernel
// at its next barrier.
// ---------------------------------------------------------------------------
__device__ bool grid_sync(Barrier* bar, int G, Lds& L, unsigned long long limit) {
  __syncthreads();
  if (G == 1) return true;
  const int tid = threadIdx.x;
  if (tid == 0) L.epoch += 1u;
  __syncthreads();
  const unsigned ep = L.epoch;
  if (tid == 0) {
    __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
    __hip_atomic_store(&bar->arrive[blockIdx.x * BAR_STRIDE], ep, __ATOMIC_RELAXED,
                       __HIP_MEMORY_SCOPE_AGENT);
    L.flag = 0;
  }
  __syncthreads();
  if (blockIdx.x == 0) {
    if (tid < 64) {
      const unsigned long long t0 = wall_clock64();
      int bad = 0;
      while (true) {
        int pending = 0;
        for (int j = tid; j < G; j += 64)
          pending |= (__hip_atomic_load(&bar->arrive[j * BAR_STRIDE], __ATOMIC_RELAXED,
                                        __HIP_MEMORY_SCOPE_AGENT) != ep);
        if (__ballot(pending) == 0ull) break;
        __builtin_amdgcn_s_sleep(1);
        if (wall_clock64() - t0 > limit) { bad = 1; break; }
      }
      if (tid == 0) {
        if (bad) __hip_atomic_store(&bar->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __builtin_amdgcn_fence(__ATOMIC_ACQ_REL, "agent");
        __hip_atomic_store(&bar->gen, ep, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        L.flag = bad;
      }
    }
  } else if (tid == 0) {
    const unsigned long long t0 = wall_clock64();
    int bad = 0;
    while (__hip_atomic_load(&bar->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) != ep) {
      __builtin_amdgcn_s_sleep(1);
      if (__hip_atomic_load(&bar->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) { bad = 1; break; }
      if (wall_clock64() - t0 > limit) {
        __hip_atomic_store(&bar->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        bad = 1;
        break;
      }
    }
    __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
    L.flag = bad;
  }
  __syncthreads();
  return L.flag == 0;
}

struct GridTeam {
  Barrier* bar;
  unsigned long long limit;
  int rank, size;
  __device__ bool sync(Lds& L) const { return grid_sync(bar, size, L, limit); }
};

struct SoloTeam {
  int rank = 0, size = 1;
  __device__ bool sync(Lds&) const {
    __syncthreads();
    return true;
  }
};

// ---------------------------------------------------------------------------
// workgroup reductions into per-workgroup partials
// ---------------------------------------------------------------------------
// sum of up to 16 per-thread values over the workgroup; partial[slot * G + rank]
__device__ __forceinline__ void block_store(Lds& L, const double* v, const int* slots, int k, double* partials,
                            int G, int rank) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int i = 0; i < k; ++i) {
    double s = wave_sum(v[i]);
    if (lane == 0) L.red[i][wv] = s;
  }
  __syncthreads();
  if ((int)threadIdx.x < k) {
    double s = 0.0;
    for (int w = 0; w < NWAVE; ++w) s += L.red[threadIdx.x][w];
    partials[(size_t)slots[threadIdx.x] * G + rank] = s;
  }
  __syncthreads();
}

// the dense factor R (r x n, row-major) as read by one workgroup: from its
// LDS copy of the owned columns [c0, c0 + nl) when there is one, else from
// global memory.  Every R access of a solve is to an owned column, so a
// slice that fits in LDS turns r dependent global loads per coordinate into
// LDS reads.
template <class MV>
struct RSrc {
  const MV* g;
  long n;
  const MV* l;     // LDS slice [r][nl] or null
  long nl, c0;
  __device__ __forceinline__ MV operator()(int k, long i) const {
    return l ? l[(size_t)k * nl + (i - c0)] : g[(size_t)k * n + i];
  }
};

// Single-workgroup teams (the batch kernels, a grid of one) accumulate R v
// inside the coordinate passes: hw_clear, then hw_add per coordinate chunk
// (one wave sum per factor row, into per-wave accumulators), then hw_store
// sums the waves into the partial slots.  Grids use hw_reduce_store below.
__device__ __forceinline__ void hw_clear(Lds& L) {
  for (int i = threadIdx.x; i < NWAVE * RMAX; i += BLOCK) (&L.hw[0][0])[i] = 0.0;
  __syncthreads();
}

// wave-uniform: add R[k, i] * val (0 if !active) to the wave's accumulators
// (the product in the factor's precision, the sums in FP64)
template <class MV>
__device__ __forceinline__ void hw_add(Lds& L, const RSrc<MV>& R, int r, long i, double val, bool active) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int k = 0; k < r; ++k) {
    double t = active ? (double)(R(k, i) * (MV)val) : 0.0;
    t = wave_sum(t);
    if (lane == 0) L.hw[wv][k] += t;
  }
}

__device__ __forceinline__ void hw_store(Lds& L, int r, double* partials, int G, int rank) {
  __syncthreads();
  if ((int)threadIdx.x < r) {
    double s = 0.0;
    for (int w = 0; w < NWAVE; ++w) s += L.hw[w][threadIdx.x];
    partials[(size_t)(SL_H0 + threadIdx.x) * G + rank] = s;
  }
  __syncthreads();
}

// the workgroup's share of R v over its coordinates [c0, c1) into the
// partial slots SL_H0 + k, and with vp also R (v - vp) into SL_HS0 + k: one
// wave per sum, up to three sums per wave at a time; products in the
// factor's precision, sums in FP64.  v (and vp) were written by this
// workgroup.
template <class MV>
__device__ __forceinline__ void hw_reduce_store(Lds& L, const RSrc<MV>& R, int r, const double* v,
                                                const double* vp, long c0, long c1, double* partials, int G,
                                                int rank) {
  __syncthreads();
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int nsum = vp ? 2 * r : r;
  for (int q0 = wv; q0 < nsum; q0 += 3 * NWAVE) {
    int kk[3];
    bool dd[3], on[3];
    for (int t = 0; t < 3; ++t) {
      const int q = q0 + t * NWAVE;
      on[t] = q < nsum;
      dd[t] = on[t] && q >= r;
      kk[t] = !on[t] ? 0 : (dd[t] ? q - r : q);
    }
    double s[3] = {0.0, 0.0, 0.0};
    for (long i = c0 + lane; i < c1; i += 64) {
      const double vi = v[i];
      const double di = vp ? vi - vp[i] : 0.0;
      for (int t = 0; t < 3; ++t) s[t] += (double)(R(kk[t], i) * (MV)(dd[t] ? di : vi));
    }
    for (int t = 0; t < 3; ++t) {
      const double tot = wave_sum(s[t]);
      if (lane == 0 && on[t]) partials[(size_t)((dd[t] ? SL_HS0 : SL_H0) + kk[t]) * G + rank] = tot;
    }
  }
  __syncthreads();
}

// sum_k R[k, i] ht[k] in increasing k, accumulated in the factor's precision
template <class MV>
__device__ __forceinline__ double r_dot(const RSrc<MV>& R, int r, long i, const double* ht) {
  MV acc = 0;
  for (int k = 0; k < r; ++k) acc += R(k, i) * (MV)ht[k];
  return (double)acc;
}

// sum over the G workgroup partials of `ns` slots: one wave per slot, up to
// three slots per wave at a time with all their loads in flight together;
// slot q is read from slot_of(q), its total written to *dst_of(q)
template <class SlotFn, class DstFn>
__device__ __forceinline__ void team_reduce_g(const double* partials, int G, int ns, SlotFn slot_of,
                                              DstFn dst_of) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int q0 = wv; q0 < ns; q0 += 3 * NWAVE) {
    const int q1 = q0 + NWAVE, q2 = q0 + 2 * NWAVE;
    const double* p0 = partials + (size_t)slot_of(q0) * G;
    const double* p1 = q1 < ns ? partials + (size_t)slot_of(q1) * G : p0;
    const double* p2 = q2 < ns ? partials + (size_t)slot_of(q2) * G : p0;
    double s0 = 0.0, s1 = 0.0, s2 = 0.0;
    for (int j = lane; j < G; j += 64) {
      s0 += p0[j];
      s1 += p1[j];
      s2 += p2[j];
    }
    s0 = wave_sum(s0);
    s1 = wave_sum(s1);
    s2 = wave_sum(s2);
    if (lane == 0) {
      *dst_of(q0) = s0;
      if (q1 < ns) *dst_of(q1) = s1;
      if (q2 < ns) *dst_of(q2) = s2;
    }
  }
  __syncthreads();
}

// reduce `k` slots over the G partials into L.scal[slot]
__device__ __forceinline__ void team_reduce(Lds& L, const double* partials, int G, const int* slots, int k) {
  team_reduce_g(partials, G, k, [&](int q) { return slots[q]; }, [&](int q) { return &L.scal[slots[q]]; });
}

// the r factor slots into dst
__device__ __forceinline__ void team_reduce_h(Lds& L, const double* partials, int G, int r, double* dst) {
  team_reduce_g(partials, G, r, [&](int q) { return (int)SL_H0 + q; }, [&](int q) { return &dst[q]; });
}

// `k` scalar slots and the r factor slots in one round
__device__ __forceinline__ void team_reduce_sh(Lds& L, const double* partials, int G, const int* slots, int k,
                                               int r, double* dsth) {
  team_reduce_g(partials, G, k + r, [&](int q) { return q < k ? slots[q] : (int)SL_H0 + q - k; },
                [&](int q) { return q < k ? &L.scal[slots[q]] : &dsth[q - k]; });
}

// after a projected step of the one-sync inner loop: ||s||^2, <s, M s>,
// <s, P s> into L.scal, R u into L.hu, R s into L.hs (one round), then the
// BB denominator <s, P s> + (R s)^T D (R s) + ||s||^2 / tau into
// L.scal[SL_SDG]
__device__ __forceinline__ void team_reduce_s(Lds& L, const double* partials, int G, int r, double tau) {
  team_reduce_g(partials, G, 3 + 2 * r,
                [&](int q) {
                  return q == 0 ? (int)SL_DELTA2 : q == 1 ? (int)SL_SJS : q == 2 ? (int)SL_SPS
                       : q < 3 + r ? (int)SL_H0 + (q - 3) : (int)SL_HS0 + (q - 3 - r);
                },
                [&](int q) -> double* {
                  return q == 0 ? &L.scal[SL_DELTA2] : q == 1 ? &L.scal[SL_SJS] : q == 2 ? &L.scal[SL_SPS]
                       : q < 3 + r ? &L.hu[q - 3] : &L.hs[q - 3 - r];
                });
  if (threadIdx.x < 64) {
    const int a = threadIdx.x;
    double t = 0.0;
    if (a < r) {
      double u = 0.0;
      for (int b = 0; b < r; ++b) u += L.Dl[a * r + b] * L.hs[b];
      t = L.hs[a] * u;
    }
    t = wave_sum(t);
    if (a == 0) L.scal[SL_SDG] = L.scal[SL_SPS] + t + L.scal[SL_DELTA2] / tau;
  }
  __syncthreads();
}

// L.ht = D h
__device__ __forceinline__ void make_ht(Lds& L, const DevProblem& P, const double* h) {
  __syncthreads();
  if ((int)threadIdx.x < P.r) {
    double s = 0.0;
    for (int b = 0; b < P.r; ++b) s += L.Dl[threadIdx.x * P.r + b] * h[b];
    L.ht[threadIdx.x] = s;
  }
  __syncthreads();
}

// one CSR row times x, Lw lanes per row; products and the lane's partial
// sum in the matrix's precision (FP32 accumulate for FP32 copies)
template <class MV>
__device__ __forceinline__ double spmv_row(const int64_t* ptr, const int* col, const MV* val,
                                           const double* x, long row, int sub, int Lw, bool active) {
  MV acc = 0;
  if (active) {
    const int64_t e = ptr[row + 1];
#pragma unroll 4
    for (int64_t k = ptr[row] + sub; k < e; k += Lw) acc += val[k] * (MV)x[col[k]];
  }
  return group_sum((double)acc, Lw);
}

// rows [r0, r1) of a CSR matrix times x into out, Lw lanes per row, this
// workgroup only
// rows [r0, r1) one at a time, each by the whole workgroup: a strided pass
// of all 512 threads and a fixed-order block sum.  For rows far longer than
// the rest, which the partition puts alone on their workgroup.  Kept out of
// line: inlined into the solver it would cost registers everywhere.
template <class MV>
__device__ __noinline__ void spmv_rows_block(const int64_t* ptr, const int* col, const MV* val,
                                             const double* x, double* out, long r0, long r1) {
  __shared__ double red[NWAVE];
  for (long row = r0; row < r1; ++row) {
    MV acc = 0;
    const int64_t e = ptr[row + 1];
#pragma unroll 8
    for (int64_t k = ptr[row] + threadIdx.x; k < e; k += BLOCK) acc += val[k] * (MV)x[col[k]];
    const double sw = wave_sum((double)acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = sw;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int w = 0; w < NWAVE; ++w) t += red[w];
      out[row] = t;
    }
    __syncthreads();
  }
}

template <class MV>
__device__ __forceinline__ void spmv_range(const int64_t* ptr, const int* col, const MV* val, const double* x,
                           double* out, long r0, long r1, int Lw) {
  if (Lw >= BLOCK) {
    spmv_rows_block(ptr, col, val, x, out, r0, r1);
    return;
  }
  const int groups = BLOCK / Lw;
  const int gid = threadIdx.x / Lw, sub = threadIdx.x & (Lw - 1);
  for (long base = r0; base < r1; base += groups) {
    const long row = base + gid;
    const bool act = row < r1;
    const double s = spmv_row(ptr, col, val, x, row, sub, Lw, act);
    if (act && sub == 0) out[row] = s;
  }
}

// A^T rows of this workgroup in length classes (rows with skewed lengths):
// perm lists the workgroup's rows grouped by class, seg[c]..seg[c+1] the
// positions of class c; class c runs with kClassLanes[c] lanes per row (the
// last class with the whole workgroup), so no lane walks a row much longer
// than its neighbours'.  Each row's sum keeps the order of spmv_row.
constexpr int kClasses = 5;
__device__ constexpr int kClassLanes[kClasses] = {1, 4, 16, 64, BLOCK};

template <class MV>
__device__ __noinline__ void spmv_classes(const int64_t* ptr, const int* col, const MV* val, const double* x,
                             double* out, const int* perm, const int* seg) {
  for (int c = 0; c < kClasses; ++c) {
    const int s0 = seg[c], s1 = seg[c + 1];
    if (s0 >= s1) continue;
    const int Lw = kClassLanes[c];
    if (Lw >= BLOCK) {
      for (int q = s0; q < s1; ++q) spmv_rows_block(ptr, col, val, x, out, (long)perm[q], (long)perm[q] + 1);
      continue;
    }
    const int groups = BLOCK / Lw;
    const int gid = threadIdx.x / Lw, sub = threadIdx.x & (Lw - 1);
    for (int base = s0; base < s1; base += groups) {
      const int q = base + gid;
      const bool act = q < s1;
      const long row = act ? (long)perm[q] : 0;
      const double v = spmv_row(ptr, col, val, x, row, sub, Lw, act);
      if (act && sub == 0) out[row] = v;
    }
  }
}

// wave-uniform loop over the coordinates [c0, c1): f(i, active)
template <class F>
__device__ __forceinline__ void for_range(long c0, long c1, F f) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (long base = c0 + (long)wv * 64; base < c1; base += BLOCK) {
    const long i = base + lane;
    f(i, i < c1);
  }
}

// rows [r0, r1) with Lw lanes per row: f(row, sub, active) (wave-uniform)
template <class F>
__device__ __forceinline__ void for_rows_range(long r0, long r1, int Lw, F f) {
  const int groups = BLOCK / Lw;
  const int gid = threadIdx.x / Lw, sub = threadIdx.x & (Lw - 1);
  for (long base = r0; base < r1; base += groups) {
    const long row = base + gid;
    f(row, sub, row < r1);
  }
}

__device__ __forceinline__ double elem_proj(uint8_t ct, double z) {
  return ct == CT_NONNEG ? fmax(z, 0.0) : z;
}

// elementwise projection of coordinate i, box blocks included (a clamp to
// [l^x_i, u^x_i], the same in every diagonal metric)
__device__ __forceinline__ double elem_proj_i(const DevProblem& P, long i, uint8_t ct, double z) {
  return ct == CT_BOX ? fmin(fmax(z, P.xlo[i]), P.xhi[i]) : elem_proj(ct, z);
}

// dual candidate of row l from y_l and (A xbar)_l, xbar = 2 w_x - x
// (eq. theory-pdhg-map): y + sigma (b - A xbar) for an equality row; with
// row bounds l <= A x <= u, the proximal step of the saddle function's row
// term, sigma (Pi_[l,u](q) - q) with q = A xbar - y/sigma
__device__ __forceinline__ double dual_candidate(const DevProblem& P, long l, double yl, double axb,
                                                 double sigma) {
  if (P.rlo) {
    const double lo = P.rlo[l], hi = P.rhi[l];
    if (lo != hi) {
      const double q = axb - yl / sigma;
      return sigma * (fmin(fmax(q, lo), hi) - q);
    }
  }
  return yl + sigma * (P.b[l] - axb);
}

template <bool EXT>
__device__ __forceinline__ double eproj(const DevProblem& P, long i, uint8_t ct, double z) {
  if constexpr (EXT) return elem_proj_i(P, i, ct, z);
  else return elem_proj(ct, z);
}

template <bool EXT>
__device__ __forceinline__ double dual_cand(const DevProblem& P, long l, double yl, double axb, double sigma) {
  if constexpr (EXT) return dual_candidate(P, l, yl, axb, sigma);
  else return yl + sigma * (P.b[l] - axb);
}

// (A x)_l minus its nearest point of the row's bounds (scaled)
template <bool EXT>
__device__ __forceinline__ double row_residual(const DevProblem& P, long l, double ax) {
  if constexpr (EXT) return P.rlo ? ax - fmin(fmax(ax, P.rlo[l]), P.rhi[l]) : ax - P.b[l];
  else return ax - P.b[l];
}

// the row's term of the dual objective: b_l y_l, or with bounds
// y^+ l - y^- u (the endpoint the sign of y selects)
template <bool EXT>
__device__ __forceinline__ double row_dual_term(const DevProblem& P, long l, double y) {
  if (!EXT || !P.rlo) return P.b[l] * y;
  return y > 0.0 ? y * P.rlo[l] : (y < 0.0 ? y * P.rhi[l] : 0.0);
}

// on a box coordinate with bounds lo, hi: the set the reduced cost may take
// at a solution (R with both bounds finite, R+ with only lo, R- with only
// hi, {0} with neither), and the projection of v onto it
__device__ __forceinline__ double box_dual_proj(double lo, double hi, double v) {
  const bool lf = isfinite(lo), hf = isfinite(hi);
  return (lf && hf) ? v : (lf ? fmax(v, 0.0) : (hf ? fmin(v, 0.0) : 0.0));
}

// matrix values of the bulk sweeps (A^T y, P u, R u, A w off check
// iterations): the FP64 data or, in FP32 mode, their FP32 copies
template <class MV>
struct Bulk;
template <>
struct Bulk<double> {
  const double *A, *AT, *Pv, *R;
  __device__ explicit Bulk(const DevProblem& P) : A(P.A_val), AT(P.AT_val), Pv(P.P_val), R(P.R) {}
};
template <>
struct Bulk<float> {
  const float *A, *AT, *Pv, *R;
  __device__ explicit Bulk(const DevProblem& P) : A(P.A_valf), AT(P.AT_valf), Pv(P.P_valf), R(P.Rf) {}
};

// ---------------------------------------------------------------------------
// metric and input views for the cone items
// ---------------------------------------------------------------------------
struct MetricQ {            // m_i = a + b * qd_i   (a + b q > 0)
  const double* qd;
  double a, b;
  int unit;                 // 1: m = 1
  __device__ double operator()(long i) const { return unit ? 1.0 : a + b * qd[i]; }
};

struct BufSrc {
  const double* z;
  MetricQ M;
  long st;
  __device__ double r(int j) const { return z[st + j]; }
  __device__ double m(int j) const { return M(st + j); }
};

struct NegSrc {
  const double* z;
  long st;
  __device__ double r(int j) const { return -z[st + j]; }
  __device__ double m(int j) const { return 1.0; }
};

struct StepSrc {            // u - alpha g / d  (g indexed from gb)
  const double* u;
  const double* g;
  MetricQ M;
  double alpha;
  long st;
  long gb;
  __device__ double r(int j) const { return u[st + j] - alpha * g[st + j - gb] / M(st + j); }
  __device__ double m(int j) const { return M(st + j); }
};

// this workgroup's cone items: wave items [w0, w1) (SOC/RSOC blocks), one
// per aligned group of lg lanes (lg = 16, 32 or 64, so 4, 2 or 1 blocks per
// wave); lane items [l0, l1) (EXP/POW blocks) spread over the waves (item k
// of the workgroup goes to wave k % NWAVE)
struct Items {
  int w0, w1, l0, l1, lg;
  const Lds* cache_w = nullptr;   // LDS copies of the wave-item / lane-item
  const Lds* cache_l = nullptr;   // descriptors, or null: read them from P
};

__device__ __forceinline__ long wi_start(const DevProblem& P, const Items& I, int it) {
  return I.cache_w ? I.cache_w->wst[it - I.w0] : P.wave_start[it];
}
__device__ __forceinline__ int wi_dim(const DevProblem& P, const Items& I, int it) {
  return I.cache_w ? I.cache_w->wdim[it - I.w0] : P.wave_dim[it];
}
__device__ __forceinline__ int wi_type(const DevProblem& P, const Items& I, int it) {
  return I.cache_w ? I.cache_w->wtype[it - I.w0] : P.wave_type[it];
}
__device__ __forceinline__ bool wi_euclid(const DevProblem& P, const Items& I, int it) {
  return I.cache_w ? I.cache_w->weu[it - I.w0] != 0 : P.wave_euclid[it] != 0;
}
__device__ __forceinline__ long li_start(const DevProblem& P, const Items& I, int it) {
  return I.cache_l ? I.cache_l->lst[it - I.l0] : P.lane_start[it];
}
__device__ __forceinline__ int li_type(const DevProblem& P, const Items& I, int it) {
  return I.cache_l ? I.cache_l->ltype[it - I.l0] : P.lane_type[it];
}
__device__ __forceinline__ bool li_euclid(const DevProblem& P, const Items& I, int it) {
  return I.cache_l ? I.cache_l->leu[it - I.l0] != 0 : P.lane_euclid[it] != 0;
}
__device__ __forceinline__ double li_alpha(const DevProblem& P, const Items& I, int it) {
  return I.cache_l ? I.cache_l->lal[it - I.l0] : P.lane_alpha[it];
}

// copy the workgroup's item descriptors into L when they fit; returns the
// Items with the cache pointers set
__device__ Items cache_items(const DevProblem& P, Items I, Lds& L) {
  const int nw = I.w1 - I.w0, nl = I.l1 - I.l0;
  if (nw > 0 && nw <= ITEM_CACHE) {
    for (int k = threadIdx.x; k < nw; k += BLOCK) {
      L.wst[k] = P.wave_start[I.w0 + k];
      L.wdim[k] = P.wave_dim[I.w0 + k];
      L.wtype[k] = P.wave_type[I.w0 + k];
      L.weu[k] = P.wave_euclid[I.w0 + k];
    }
    I.cache_w = &L;
  }
  if (nl > 0 && nl <= ITEM_CACHE) {
    for (int k = threadIdx.x; k < nl; k += BLOCK) {
      L.lst[k] = P.lane_start[I.l0 + k];
      L.ltype[k] = P.lane_type[I.l0 + k];
      L.leu[k] = P.lane_euclid[I.l0 + k];
      L.lal[k] = P.lane_alpha[I.l0 + k];
    }
    I.cache_l = &L;
  }
  __syncthreads();
  return I;
}

// rescaled-cone mode (eq. scaling-induced-metric): a block of the scaled
// problem is S K with S = diag(Sx on the block), and
//   Pi^M_{S K}(r) = S Pi^{S M S}_K(S^-1 r),
// so a prox projection reads S^-1 r in the metric S M S (M = 1 when the
// caller forces the Euclidean metric) and scales the root back by S; the
// check's projection (kkt) reads the unscaled -s = -nu_c S s^ instead and
// projects it onto K itself, in the Euclidean metric
template <class Src>
struct RescSrc {
  Src s;
  const double* sx;
  double nu_c;
  long st;
  bool kkt, force;
  __device__ double r(int j) const {
    const double v = sx[st + j];
    return kkt ? s.r(j) * (nu_c * v) : s.r(j) / v;
  }
  __device__ double m(int j) const {
    const double v = sx[st + j];
    return kkt ? 1.0 : (force ? 1.0 : s.m(j)) * (v * v);
  }
};

template <class MakeSrc>
__device__ __forceinline__ void project_items_resc(const DevProblem& P, const Items& I, bool force_euclid,
                                                   MakeSrc make, double* dst, double* warm, long dbase, bool kkt) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int gpw = 64 / I.lg;
  const double* sx = P.Sx;
  for (int it = I.w0 + wv * gpw + lane / I.lg; it < I.w1; it += NWAVE * gpw) {
    const long st = wi_start(P, I, it);
    const RescSrc<decltype(make(st))> src{make(st), sx, P.nu_c, st, kkt, force_euclid};
    project_wave_item(wi_type(P, I, it), wi_dim(P, I, it), kkt, src,
                      [dst, st, dbase, sx, kkt](int j, double v) { dst[st + j - dbase] = kkt ? v : v * sx[st + j]; },
                      warm ? warm + it : nullptr, I.lg);
  }
  for (int kb = 0; I.l0 + kb < I.l1; kb += BLOCK) {
    const int it = I.l0 + kb + wv + NWAVE * lane;
    if (it >= I.l1) continue;
    const long st = li_start(P, I, it);
    const int ty = li_type(P, I, it);
    Trip o;
    if (ty == PDHCG_CONE_EXP1) {
      // one common factor (kappa X), as in the cone-preserving mode
      const auto raw = make(st);
      const bool eu = force_euclid || li_euclid(P, I, it);
      const double m0 = eu ? 1.0 : raw.m(0), m2 = eu ? 1.0 : raw.m(2);
      o = kkt ? Trip{0.0, 0.0, 0.0} : project_exp1(raw.r(0), raw.r(2), m0, m2, P.Sx[st] / P.nu_b);
    } else {
      const RescSrc<decltype(make(st))> src{make(st), sx, P.nu_c, st, kkt, force_euclid};
      const double r0 = src.r(0), r1 = src.r(1), r2 = src.r(2);
      double m0 = 1.0, m1 = 1.0, m2 = 1.0;
      if (!kkt) { m0 = src.m(0); m1 = src.m(1); m2 = src.m(2); }
      double* w = warm ? warm + P.n_wave + it : nullptr;
      o = ty == PDHCG_CONE_EXP ? project_exp(r0, r1, r2, m0, m1, m2, w)
                               : project_pow(r0, r1, r2, li_alpha(P, I, it), m0, m1, m2, w);
      if (!kkt) {
        o.a *= sx[st];
        o.b *= sx[st + 1];
        o.c *= sx[st + 2];
      }
    }
    dst[st - dbase] = o.a;
    dst[st + 1 - dbase] = o.b;
    dst[st + 2 - dbase] = o.c;
  }
  __syncthreads();
}

// warm (nullable): previous roots of the root-finding projections, one per
// item (wave items first, then lane items), read as starting points and
// overwritten with the new roots
template <bool EXT = false, class MakeSrc>
__device__ __forceinline__ void project_items(const DevProblem& P, const Items& I, bool force_euclid, MakeSrc make,
                              double* dst, double* warm, unsigned long long* ptw = nullptr, long dbase = 0,
                              bool kkt = false) {
  if constexpr (EXT) {
    if (P.resc) {
      project_items_resc(P, I, force_euclid, make, dst, warm, dbase, kkt);
      return;
    }
  }
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int gpw = 64 / I.lg;                       // groups per wave
  for (int it = I.w0 + wv * gpw + lane / I.lg; it < I.w1; it += NWAVE * gpw) {
    const long st = wi_start(P, I, it);
    auto src = make(st);
    const bool eu = force_euclid || wi_euclid(P, I, it);
    const unsigned long long t0 = ptw ? wall_clock64() : 0ull;
    project_wave_item(wi_type(P, I, it), wi_dim(P, I, it), eu, src,
                      [dst, st, dbase](int j, double v) { dst[st + j - dbase] = v; }, warm ? warm + it : nullptr,
                      I.lg);
    if (ptw && threadIdx.x == 0) {
      ptw[0] += wall_clock64() - t0;
      ptw[1] += 1;
    }
  }
  for (int kb = 0; I.l0 + kb < I.l1; kb += BLOCK) {
    const int it = I.l0 + kb + wv + NWAVE * lane;
    if (it < I.l1) {
      const long st = li_start(P, I, it);
      auto src = make(st);
      const bool eu = force_euclid || li_euclid(P, I, it);
      const double r0 = src.r(0), r1 = src.r(1), r2 = src.r(2);
      double m0 = 1.0, m1 = 1.0, m2 = 1.0;
      if (!eu) { m0 = src.m(0); m1 = src.m(1); m2 = src.m(2); }
      double* w = warm ? warm + P.n_wave + it : nullptr;
      const int ty = li_type(P, I, it);
      Trip o;
      if constexpr (EXT) {
        // fixed-middle EXP block: kappa X with kappa = S_x / nu_b of the
        // block; its KKT terms are not a projection of -s (kkt: zeros here,
        // the check takes the terms itself)
        if (ty == PDHCG_CONE_EXP1) {
          o = kkt ? Trip{0.0, 0.0, 0.0} : project_exp1(r0, r2, m0, m2, P.Sx[st] / P.nu_b);
          dst[st - dbase] = o.a;
          dst[st + 1 - dbase] = o.b;
          dst[st + 2 - dbase] = o.c;
          continue;
        }
      }
      if (ty == PDHCG_CONE_EXP) o = project_exp(r0, r1, r2, m0, m1, m2, w);
      else o = project_pow(r0, r1, r2, li_alpha(P, I, it), m0, m1, m2, w);
      dst[st - dbase] = o.a;
      dst[st + 1 - dbase] = o.b;
      dst[st + 2 - dbase] = o.c;
    }
  }
  __syncthreads();
}

// wave-uniform iteration over the coordinates of this workgroup's cone items
// (same item-to-group mapping as project_items)
template <class F>
__device__ __forceinline__ void for_item_coords(const DevProblem& P, const Items& I, F f) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int gpw = 64 / I.lg;
  const int gl = lane & (I.lg - 1);
  for (int base = I.w0 + wv * gpw; base < I.w1; base += NWAVE * gpw) {
    const int it = base + lane / I.lg;
    const bool ok = it < I.w1;
    const long st = ok ? wi_start(P, I, it) : 0;
    const int dim = ok ? wi_dim(P, I, it) : 0;
    int maxd = dim;                                  // longest block of the wave
    for (int o = 32; o >= 1; o >>= 1) maxd = max(maxd, __shfl_xor(maxd, o, 64));
    for (int jb = 0; jb < maxd; jb += I.lg) {
      const int j = jb + gl;
      f(st + j, ok && j < dim);
    }
  }
  for (int kb = 0; I.l0 + kb < I.l1; kb += BLOCK) {
    const int it = I.l0 + kb + wv + NWAVE * lane;
    const bool act = it < I.l1;
    const long st = act ? li_start(P, I, it) : 0;
    for (int j = 0; j < 3; ++j) f(st + j, act);
  }
}

// ---------------------------------------------------------------------------
// the solver core, shared by the single-problem grid kernel and the batch
// kernel
// ---------------------------------------------------------------------------
struct Own {
  long c0, c1, r0, r1;
  Items it;
  int la, lr;   // lanes per row of A^T / P (own coordinates) and of A (own rows)
  const int* atperm;   // A^T rows in length classes (null: plain ranges)
  const int* atseg;
};

// EXT: the variant with row bounds, box blocks and fixed-middle EXP blocks
// (problems without them run the variant compiled without that code, whose
// register allocation is that of the plain method)
template <bool CONES, class MV, bool EXT, class Team>
__device__ void run_solver(const Run& A, const DevProblem& P, const DevVec& V, Ctl* ctl,
                           const Team& T, Lds& L, const Own& own, bool prof) {
  const Bulk<MV> M(P);
  // LDS copy of the owned columns of R (bulk precision); the FP64 reads of
  // an FP32 run (start, checks) stay in global memory
  const long nloc = own.c1 - own.c0;
  MV* rl = nullptr;
  if (A.lds && P.r > 0 && (size_t)P.r * (size_t)nloc * sizeof(MV) <= (size_t)A.lds_bytes) {
    rl = reinterpret_cast<MV*>(A.lds);
    for (long e = threadIdx.x; e < (long)P.r * nloc; e += BLOCK)
      rl[e] = M.R[(size_t)(e / nloc) * P.n + own.c0 + e % nloc];
  }
  const RSrc<MV> RB{M.R, (long)P.n, rl, nloc, own.c0};
  const RSrc<double> R64{P.R, (long)P.n, sizeof(MV) == sizeof(double) ? reinterpret_cast<const double*>(rl) : nullptr,
                         nloc, own.c0};
  const int tid = threadIdx.x;
  const int rank = T.rank, G = T.size;
  const long n = P.n, m = P.m;
  const int r = P.r;
  const DevSettings& S = *A.S;
  const TraceBufs& TB = *A.T;
  double* part = V.partials;
  const long c0 = own.c0, c1 = own.c1, r0 = own.r0, r1 = own.r1;
  const Items IT = CONES ? cache_items(P, own.it, L) : own.it;
  // CONES = false: the variant for problems whose blocks are all FREE or R+,
  // compiled without the cone projections (far fewer registers)
  const bool has_items = CONES && ((IT.w1 > IT.w0) || (IT.l1 > IT.l0));

#define SYNC_OR_EXIT()                         \
  do {                                         \
    const int _cat = L.pcat;                   \
    tmark(L, prof, PT_BAR);                    \
    const bool _ok = T.sync(L);                \
    tmark(L, prof, _cat);                      \
    if (!_ok) {                                \
      if (rank == 0 && tid == 0) {             \
        L.C.status = PDHCG_ABORTED;            \
        *ctl = L.C;                            \
      }                                        \
      return;                                  \
    }                                          \
  } while (0)

  const MetricQ unitM{P.qd, 1.0, 0.0, 1};
#define PROJ(call)                                  \
  do {                                              \
    const int _pc = L.pcat;                         \
    tmark(L, prof, PT_PROJ);                        \
    call;                                           \
    tmark(L, prof, _pc);                            \
  } while (0)

  // single-workgroup teams (the batch kernels, a grid of one) keep the
  // in-pass R v accumulation and two synchronisations per inner step: their
  // synchronisations are workgroup barriers, and in-pass accumulation reads
  // nothing back
  constexpr bool SOLO = std::is_same<Team, SoloTeam>::value;
  const bool fuse = !SOLO && !P.q_diag && (P.p_diag || !P.P_ptr);
  // inner-step staging of the cone coordinates' gradient (one-sync step
  // only) and projected point: LDS when the workgroup owns at most ZCAP
  // coordinates, else the global g and zb
  const bool zlds = (own.c1 - own.c0) <= ZCAP;
  double* const gst = (fuse && zlds) ? L.gl : V.g;
  const long gsb = (fuse && zlds) ? own.c0 : 0;
  double* const zst = zlds ? L.zl : V.zb;
  const long zsb = zlds ? own.c0 : 0;
  // the R v partial of this workgroup after a coordinate pass that wrote v
  // (and R (v - vp) for the one-sync inner step)
  auto hw_finish = [&](const auto& R, const double* v, const double* vp) {
    if constexpr (SOLO) hw_store(L, r, part, G, rank);
    else hw_reduce_store(L, R, r, v, vp, c0, c1, part, G, rank);
  };

  for (int e = tid; e < r * r; e += BLOCK) L.Dl[e] = P.Dm[e];
  __syncthreads();

  // ------------------------------------------------------------------ init
  if (!L.C.started) {
    // x = Pi_K(x0^) (zb holds the scaled warm start or zeros); a_x = x
    if constexpr (SOLO) hw_clear(L);
    for_range(c0, c1, [&](long i, bool act) {
      bool el = act && P.ctype[i] != CT_CONE;
      double x = el ? eproj<EXT>(P, i, P.ctype[i], V.zb[i]) : 0.0;
      if (el) { V.x[i] = x; V.ax[i] = x; }
      if constexpr (SOLO) hw_add(L, R64, r, i, x, el);
    });
    if (has_items) {
      project_items<EXT>(P, IT, true, [&](long st) { return BufSrc{V.zb, unitM, st}; }, V.zb, nullptr);
      for_item_coords(P, IT, [&](long i, bool act) {
        double x = act ? V.zb[i] : 0.0;
        if (act) { V.x[i] = x; V.ax[i] = x; }
        if constexpr (SOLO) hw_add(L, R64, r, i, x, act);
      });
    }
    hw_finish(R64, V.x, nullptr);
    SYNC_OR_EXIT();
    for_rows_range(r0, r1, own.lr, [&](long row, int sub, bool act) {
      double ax = spmv_row(P.A_ptr, P.A_col, P.A_val, V.x, row, sub, own.lr, act);
      if (act && sub == 0) { V.Ax[row] = ax; V.Aa[row] = ax; V.ay[row] = V.y[row]; }
    });
    team_reduce_h(L, part, G, r, L.C.hx);
    if (tid == 0) {
      L.C.started = 1;
      if (!L.C.resume) {
        L.C.omega = P.omega0;
        L.C.eps_in = S.eps_in0;
        L.C.ktot = 0;
        L.C.inner_total = 0;
        L.C.restarts = 0;
        L.C.pid_I = 0.0;
        L.C.e_prev = 0.0;
      }
      // resume (precision switch): a restart at the given point that keeps
      // the primal weight, inner tolerance and counters
      L.C.resume = 0;
      L.C.k = 0;
      L.C.E0 = L.C.Eprev = L.C.lastE = 0.0;
    }
    __syncthreads();
    SYNC_OR_EXIT();
  }

  const bool jac = S.inner == PDHCG_INNER_JACOBI;
  // P diagonal or absent: one grid synchronisation per inner step (a sparse
  // P needs the neighbours' s for <s, P s>: two)
  const double rho = S.rho;
  const int La = own.la, Lr = own.lr;
  // averaged epochs (Alg. 1): fixed step sizes, plain PDHG steps
  // z = T(z), running Cesaro averages of x, y and A x, and at the end of
  // each epoch (or at max_iter) a restart from the average with the KKT
  // check taken on it
  const bool avg = std::is_same<MV, double>::value && S.scheme == PDHCG_SCHEME_AVG;   // FP64 only

  // KKT dual part at (X, Y) with R^ X = hX: the dual slack
  // s = Q^ X + c^ - A^T Y on own coordinates, <X, Q^ X> and ||Pi_K(-s)||^2
  // (unscaled) into the partial slots SL_XQX, SL_RD2
  auto dual_check = [&](const double* X, const double* Y, const double* hX) __attribute__((always_inline)) {
    if (own.atperm) spmv_classes(P.AT_ptr, P.AT_col, P.AT_val, Y, V.t1, own.atperm, own.atseg);
    else spmv_range(P.AT_ptr, P.AT_col, P.AT_val, Y, V.t1, c0, c1, La);
    if (!P.q_diag && P.P_ptr && !P.p_diag) spmv_range(P.P_ptr, P.P_col, P.P_val, X, V.t2, c0, c1, La);
    if (!P.q_diag) make_ht(L, P, hX);
    else __syncthreads();
    constexpr int NSL = EXT ? 3 : 2;
    double acc[NSL] = {};
    for_range(c0, c1, [&](long i, bool act) {
      if (!act) return;
      const double wi = X[i];
      double qw;
      if (P.q_diag) {
        qw = P.qd[i] * wi;
      } else {
        qw = P.p_diag ? P.Pd[i] * wi : (P.P_ptr ? V.t2[i] : 0.0);
        qw += r_dot(R64, r, i, L.ht);
      }
      const double si = qw + P.c[i] - V.t1[i];
      acc[0] += wi * qw;                               // SL_XQX
      const double so = P.nu_c * P.Sx[i] * si;
      const uint8_t ct = P.ctype[i];
      if (ct == CT_FREE) acc[1] += so * so;
      else if (ct == CT_NONNEG) { const double t = fmax(-so, 0.0); acc[1] += t * t; }
      else if (EXT && ct == CT_BOX) {
        // distance of s to the reduced cost's set, and lambda^+ l - lambda^- u
        const double lo = P.xlo[i], hi = P.xhi[i];
        const double t = so - box_dual_proj(lo, hi, so);
        acc[1] += t * t;
        const double lam = box_dual_proj(lo, hi, si);
        acc[NSL - 1] += lam > 0.0 ? lam * lo : (lam < 0.0 ? lam * hi : 0.0);   // SL_BOXD
      }
      else V.s[i] = si;
    });
    if (has_items) {
      __syncthreads();
      project_items<EXT>(P, IT, true, [&](long st) { return NegSrc{V.s, st}; }, V.zb,
                    V.warm + (P.n_wave + P.n_lane), nullptr, 0, true);
      for_item_coords(P, IT, [&](long i, bool act) {
        if (act) {
          // Pi_K(-s) of the original problem: nu_c S_x Pi_K(-s^) when the
          // block shares one factor; projected unscaled in the rescaled mode
          const double f = (EXT && P.resc) ? V.zb[i] : P.nu_c * P.Sx[i] * V.zb[i];
          acc[1] += f * f;
        }
      });
      // fixed-middle EXP blocks, with the reduced cost (a, b, c) unscaled:
      // distance to Lambda = {a <= 0, c >= 0} (the dual of the set's
      // recession cone {dz <= 0, ds = 0, dt >= 0}) and the set's support
      // term inf <lambda, x> = b + lambda_a (log(-lambda_a/lambda_c) - 1)
      for (int it = IT.l0 + tid; EXT && it < IT.l1; it += BLOCK) {
        if (li_type(P, IT, it) != PDHCG_CONE_EXP1) continue;
        const long st = li_start(P, IT, it);
        const double f = P.nu_c * P.Sx[st];
        const double a = f * V.s[st], b = f * V.s[st + 1], c = f * V.s[st + 2];
        const double la = fmin(a, 0.0), lc = fmax(c, 0.0);
        acc[1] += (a - la) * (a - la) + (c - lc) * (c - lc);
        const double term = la == 0.0 ? b : (lc == 0.0 ? -INFINITY : b + la * (log(-la / lc) - 1.0));
        acc[NSL - 1] += term / (P.nu_b * P.nu_c);
      }
    }
    const int sl[3] = {SL_XQX, SL_RD2, SL_BOXD};
    block_store(L, acc, sl, NSL, part, G, rank);
  };

  // residuals, objectives and status from the reduced slots SL_RP2, SL_RD2,
  // SL_XQX, SL_CX, SL_BY (thread 0)
  auto kkt_status = [&](Ctl& C, bool bad) __attribute__((always_inline)) {
    const double* sc = L.scal;
    const double scale = P.nu_b * P.nu_c;
    C.rel_p = sqrt(sc[SL_RP2]) / (1.0 + P.norm_b);
    C.rel_d = sqrt(sc[SL_RD2]) / (1.0 + P.norm_c);
    C.pobj = scale * (0.5 * sc[SL_XQX] + sc[SL_CX]);
    if constexpr (EXT) {
      C.dobj = scale * (sc[SL_BY] + sc[SL_BOXD] - 0.5 * sc[SL_XQX]);
      // a fixed-middle EXP reduced cost with lambda_a < 0 = lambda_c has
      // dual value -inf: no gap closure yet
      C.rel_gap = C.dobj == -INFINITY ? 1.0 : fabs(C.pobj - C.dobj) / (1.0 + fabs(C.pobj) + fabs(C.dobj));
    } else {
      C.dobj = scale * (sc[SL_BY] - 0.5 * sc[SL_XQX]);
      C.rel_gap = fabs(C.pobj - C.dobj) / (1.0 + fabs(C.pobj) + fabs(C.dobj));
    }
    if (bad || !isfinite(C.rel_p) || !isfinite(C.rel_d) || !isfinite(C.rel_gap)) {
      C.status = PDHCG_NUMERICAL;
    } else if (fmax(C.rel_p, fmax(C.rel_d, C.rel_gap)) <= S.tol) {
      C.status = PDHCG_OPTIMAL;
    } else if (A.deadline != 0ull && wall_clock64() > A.deadline) {
      C.status = PDHCG_TIME_LIMIT;
    }
  };

  while (L.C.ktot < A.stop_at && L.C.status == 0) {
    const double omega = L.C.omega;
    const double tau = P.eta / omega, sigma = P.eta * omega;
    const long long k = L.C.k;
    const long long kt1 = L.C.ktot + 1;
    const bool ep_end = avg && ((k + 1 >= (long long)S.avg_epoch) || (kt1 >= S.max_iter));
    const bool check = avg ? ep_end : ((k == 0) || (kt1 % S.check_every == 0) || (kt1 >= S.max_iter));
    const double eps_in = L.C.eps_in;
    const bool tracing = TB.cap > 0 && L.C.ktot < TB.cap;
    double* W = P.q_diag ? V.wx : V.u;   // the primal candidate w_x
    const MetricQ Mq = P.q_diag ? MetricQ{P.qd, 1.0, tau, 0}
                                : (jac ? MetricQ{P.qd, 1.0 / tau, 1.0, 0} : unitM);
    const double alpha0 = jac ? 1.0 : 1.0 / (A.qmax + 1.0 / tau);

    if (tracing) {
      const long kk = L.C.ktot;
      for (long i = c0 + tid; i < c1; i += BLOCK) TB.x[kk * n + i] = V.x[i];
      for (long l = r0 + tid; l < r1; l += BLOCK) TB.y[kk * m + l] = V.y[l];
    }

    // -------------------------------------------------------------- P1
    tmark(L, prof, PT_P1);
    if (own.atperm) spmv_classes(P.AT_ptr, P.AT_col, M.AT, V.y, V.t1, own.atperm, own.atseg);
    else spmv_range(P.AT_ptr, P.AT_col, M.AT, V.y, V.t1, c0, c1, La);
    if (!P.q_diag) {
      if (P.P_ptr && !P.p_diag) spmv_range(P.P_ptr, P.P_col, M.Pv, V.x, V.t2, c0, c1, La);
      make_ht(L, P, L.C.hx);
    } else {
      __syncthreads();
    }
    if (P.q_diag) {
      for_range(c0, c1, [&](long i, bool act) {
        if (!act) return;
        const double vi = V.x[i] + tau * V.t1[i];
        const double mi = 1.0 + tau * P.qd[i];
        const double z = (vi - tau * P.c[i]) / mi;
        if (P.ctype[i] != CT_CONE) V.wx[i] = eproj<EXT>(P, i, P.ctype[i], z);
        else V.zb[i] = z;
      });
      if (has_items) {
        __syncthreads();
        PROJ(project_items<EXT>(P, IT, false, [&](long st) { return BufSrc{V.zb, Mq, st}; }, V.wx, V.warm));
      }
    } else {
      // acc: ||s||^2, <s, M s>, <s, P s> of the first step s = u - x (the
      // last two for the one-sync inner step only)
      double acc[3] = {0.0, 0.0, 0.0};
      if constexpr (SOLO) hw_clear(L);
      for_range(c0, c1, [&](long i, bool act) {
        double un = 0.0;
        bool el = false;
        if (act) {
          const double xi = V.x[i];
          const double vi = xi + tau * V.t1[i];
          const double ru = r_dot(RB, r, i, L.ht);
          const double pu = P.p_diag ? P.Pd[i] * xi : (P.P_ptr ? V.t2[i] : 0.0);
          const double g0 = pu + ru + P.c[i] + (xi - vi) / tau;
          const double mi = Mq(i);
          const double z = xi - alpha0 * g0 / mi;
          V.v[i] = vi;
          if (!fuse) V.gp[i] = g0;
          V.up[i] = xi;
          if (P.ctype[i] != CT_CONE) {
            el = true;
            un = eproj<EXT>(P, i, P.ctype[i], z);
            V.u[i] = un;
            const double si = un - xi;
            acc[0] += si * si;
            if (fuse) {
              acc[1] += si * (mi * si);
              if (P.p_diag) acc[2] += si * (P.Pd[i] * si);
            }
          } else {
            V.zb[i] = z;
          }
        }
        if constexpr (SOLO) hw_add(L, RB, r, i, un, el);
      });
      if (has_items) {
        __syncthreads();
        PROJ(project_items<EXT>(P, IT, !jac, [&](long st) { return BufSrc{V.zb, Mq, st}; }, V.zb, V.warm));
        for_item_coords(P, IT, [&](long i, bool act) {
          double un = 0.0;
          if (act) {
            un = V.zb[i];
            V.u[i] = un;
            const double si = un - V.up[i];
            acc[0] += si * si;
            if (fuse) {
              acc[1] += si * (Mq(i) * si);
              if (P.p_diag) acc[2] += si * (P.Pd[i] * si);
            }
          }
          if constexpr (SOLO) hw_add(L, RB, r, i, un, act);
        });
      }
      const int sl[3] = {SL_DELTA2, SL_SJS, SL_SPS};
      block_store(L, acc, sl, fuse ? 3 : 1, part, G, rank);
      hw_finish(RB, V.u, fuse ? V.up : nullptr);
    }
    SYNC_OR_EXIT();

    // -------------------------------------------------------------- inner loop
    int jcount = 0;
    if (!P.q_diag) {
      // With P diagonal or absent (fuse) an inner step takes one grid
      // synchronisation: the prox gradient g(u) = P u + R^T D R u + c +
      // (u - v) / tau is affine in u, so the BB denominator
      // <s, g(u) - g(u_prev)> equals <s, P s> + (R s)^T D (R s) + ||s||^2 / tau
      // with s = u - u_prev; each projected step accumulates these sums and
      // R s beside ||s||^2 and R u, and the one reduction after it gives the
      // next step size.  Otherwise the gradient pass reduces the BB sums
      // before the step (two synchronisations).
      if (fuse) {
        team_reduce_s(L, part, G, r, tau);
      } else {
        const int sl[1] = {SL_DELTA2};
        team_reduce_sh(L, part, G, sl, 1, r, L.hu);
      }
      jcount = 1;
      bool done = (S.fixed_inner <= 0) && (sqrt(L.scal[SL_DELTA2]) <= eps_in);
      const int jmax = S.fixed_inner > 0 ? S.fixed_inner : S.j_max;
      while (!done && jcount < jmax) {
        double alpha;
        tmark(L, prof, PT_P3);
        if (fuse) {
          const double den = L.scal[SL_SDG];
          const double num = jac ? L.scal[SL_SJS] : L.scal[SL_DELTA2];
          alpha = den > 0.0 ? num / den : 1.0;
          make_ht(L, P, L.hu);
        } else {
          // ---- P3: gradient at u, BB reductions
          if (P.P_ptr && !P.p_diag) spmv_range(P.P_ptr, P.P_col, M.Pv, V.u, V.t2, c0, c1, La);
          make_ht(L, P, L.hu);
          double acc[3] = {0.0, 0.0, 0.0};
          for_range(c0, c1, [&](long i, bool act) {
            if (!act) return;
            const double ru = r_dot(RB, r, i, L.ht);
            const double ui = V.u[i];
            const double pu = P.p_diag ? P.Pd[i] * ui : (P.P_ptr ? V.t2[i] : 0.0);
            const double gc = pu + ru + P.c[i] + (ui - V.v[i]) / tau;
            const double si = ui - V.up[i];
            const double dg = gc - V.gp[i];
            const double di = Mq(i);
            acc[0] += si * (di * si);
            acc[1] += si * dg;
            acc[2] += si * si;
            V.g[i] = gc;
          });
          {
            const int sl[3] = {SL_SJS, SL_SDG, SL_SS};
            block_store(L, acc, sl, 3, part, G, rank);
          }
          SYNC_OR_EXIT();
          {
            const int sl[3] = {SL_SJS, SL_SDG, SL_SS};
            team_reduce(L, part, G, sl, 3);
          }
          const double den = L.scal[SL_SDG];
          const double num = jac ? L.scal[SL_SJS] : L.scal[SL_SS];
          alpha = den > 0.0 ? num / den : 1.0;
        }
        // ---- P4: projected step (fuse: the gradient is formed here)
        tmark(L, prof, PT_P4);
        double acc[3] = {0.0, 0.0, 0.0};
        if constexpr (SOLO) hw_clear(L);
        for_range(c0, c1, [&](long i, bool act) {
          const bool el = act && P.ctype[i] != CT_CONE;
          double un = 0.0;
          if (act && (el || fuse)) {
            const double ui = V.u[i];
            double gi;
            if (fuse) {
              const double ru = r_dot(RB, r, i, L.ht);
              const double pu = P.p_diag ? P.Pd[i] * ui : 0.0;
              gi = pu + ru + P.c[i] + (ui - V.v[i]) / tau;
              if (!el) gst[i - gsb] = gi;
            } else {
              gi = V.g[i];
            }
            if (el) {
              const double mi = Mq(i);
              un = eproj<EXT>(P, i, P.ctype[i], ui - alpha * gi / mi);
              const double si = un - ui;
              acc[0] += si * si;
              if (fuse) {
                acc[1] += si * (mi * si);
                if (P.p_diag) acc[2] += si * (P.Pd[i] * si);
              } else {
                V.gp[i] = gi;
              }
              V.up[i] = ui;
              V.u[i] = un;
            }
          }
          if constexpr (SOLO) hw_add(L, RB, r, i, un, el);
        });
        if (has_items) {
          if (fuse) __syncthreads();
          PROJ(project_items<EXT>(P, IT, !jac,
                             [&](long st) { return StepSrc{V.u, gst, Mq, alpha, st, gsb}; }, zst, V.warm,
                             prof ? &L.pt[PT_WCALL] : nullptr, zsb));
          for_item_coords(P, IT, [&](long i, bool act) {
            double un = 0.0;
            if (act) {
              un = zst[i - zsb];
              const double ui = V.u[i];
              const double si = un - ui;
              acc[0] += si * si;
              if (fuse) {
                acc[1] += si * (Mq(i) * si);
                if (P.p_diag) acc[2] += si * (P.Pd[i] * si);
              } else {
                V.gp[i] = V.g[i];
              }
              V.up[i] = ui;
              V.u[i] = un;
            }
            if constexpr (SOLO) hw_add(L, RB, r, i, un, act);
          });
        }
        {
          const int sl[3] = {SL_DELTA2, SL_SJS, SL_SPS};
          block_store(L, acc, sl, fuse ? 3 : 1, part, G, rank);
          hw_finish(RB, V.u, fuse ? V.up : nullptr);
        }
        SYNC_OR_EXIT();
        if (fuse) {
          team_reduce_s(L, part, G, r, tau);
        } else {
          const int sl[1] = {SL_DELTA2};
          team_reduce_sh(L, part, G, sl, 1, r, L.hu);
        }
        ++jcount;
        done = (S.fixed_inner <= 0) && (sqrt(L.scal[SL_DELTA2]) <= eps_in);
      }
    }

    // -------------------------------------------------------------- P6
    tmark(L, prof, PT_P6);
    const double c1h = (double)(k + 1) / (double)(k + 2);
    const double c3h = 1.0 / (double)(k + 2);
    if (avg) {
      // w_y, then z = T(z): x = w_x, y = w_y, A x = A w_x, and the running
      // averages zbar = k/(k+1) zbar + w/(k+1) (eq. theory-epoch-average);
      // at the epoch's end the state restarts from zbar, and the primal
      // residual, <b, ybar> and <c, xbar> of the check are accumulated
      const double kd = (double)k;
      double acc[4] = {0.0, 0.0, 0.0, 0.0};
      for_rows_range(r0, r1, Lr, [&](long l, int sub, bool act) {
        const double aw = spmv_row(P.A_ptr, P.A_col, M.A, W, l, sub, Lr, act);
        if (act && sub == 0) {
          const double yl = V.y[l], axl = V.Ax[l];
          const double wy = dual_cand<EXT>(P, l, yl, 2.0 * aw - axl, sigma);
          V.wy[l] = wy;
          V.Aw[l] = aw;
          if (tracing) TB.wy[L.C.ktot * m + l] = wy;
          const double yb = k == 0 ? wy : (kd / (kd + 1.0)) * V.yb[l] + wy / (kd + 1.0);
          const double axb = k == 0 ? aw : (kd / (kd + 1.0)) * V.Axb[l] + aw / (kd + 1.0);
          V.yb[l] = yb;
          V.Axb[l] = axb;
          if (ep_end) {
            V.y[l] = yb;
            V.Ax[l] = axb;
            const double rp = P.nu_b * row_residual<EXT>(P, l, axb) / P.Sy[l];
            acc[1] += rp * rp;                           // SL_RP2
            acc[2] += row_dual_term<EXT>(P, l, yb);           // SL_BY
          } else {
            V.y[l] = wy;
            V.Ax[l] = aw;
          }
        }
      });
      for_range(c0, c1, [&](long i, bool act) {
        if (!act) return;
        const double xi = V.x[i], wi = W[i];
        if (tracing) TB.wx[L.C.ktot * n + i] = wi;
        acc[0] += (wi - xi) * (wi - xi);                 // SL_XMOV2
        const double xb = k == 0 ? wi : (kd / (kd + 1.0)) * V.xb[i] + wi / (kd + 1.0);
        V.xb[i] = xb;
        if (ep_end) {
          V.x[i] = xb;
          acc[3] += P.c[i] * xb;                         // SL_CX
        } else {
          V.x[i] = wi;
        }
      });
      const int sl[4] = {SL_XMOV2, SL_RP2, SL_BY, SL_CX};
      block_store(L, acc, sl, ep_end ? 4 : 1, part, G, rank);
      SYNC_OR_EXIT();
      if (tid == 0) {
        L.C.inner_total += jcount;
        L.C.ktot = kt1;
      }
      team_reduce(L, part, G, sl, ep_end ? 4 : 1);
      if (tid == 0) {
        L.C.eps_in = fmin(L.C.eps_in, fmax(S.gamma_in * sqrt(L.scal[SL_XMOV2]) / tau, S.eps_min));
      }
      // R^ x of the new state: R^ w_x is the last inner R^ u; its running
      // average is kept beside the others
      if ((int)tid < r) {
        const double hb = k == 0 ? L.hu[tid] : (kd / (kd + 1.0)) * L.C.hxb[tid] + L.hu[tid] / (kd + 1.0);
        L.C.hxb[tid] = hb;
        L.C.hx[tid] = ep_end ? hb : L.hu[tid];
      }
      __syncthreads();
      if (!ep_end) {
        if (tid == 0) {
          L.C.k = k + 1;
          if (tracing && rank == 0) {
            double* t = TB.sc + (kt1 - 1) * 8;
            t[0] = tau; t[1] = sigma; t[2] = omega; t[3] = eps_in;
            t[4] = jcount; t[5] = 0.0; t[6] = 0.0; t[7] = 0.0;
          }
        }
        __syncthreads();
        continue;
      }
      // end of the epoch: the KKT check below runs on the new state zbar
    } else {
    {
      double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      if (check) {
        // check iterations use the FP64 data: the residuals and the restart
        // statistics of a check are exact FP64
        for_rows_range(r0, r1, Lr, [&](long l, int sub, bool act) {
          const double aw = spmv_row(P.A_ptr, P.A_col, P.A_val, W, l, sub, Lr, act);
          if (act && sub == 0) {
            const double yl = V.y[l], axl = V.Ax[l];
            const double wy = dual_cand<EXT>(P, l, yl, 2.0 * aw - axl, sigma);
            V.wy[l] = wy;
            V.Aw[l] = aw;
            if (tracing) TB.wy[L.C.ktot * m + l] = wy;
            const double dy = yl - wy;
            acc[0] += dy * dy;                           // SL_DY2
            acc[1] += (axl - aw) * dy;                   // SL_ADXDY
            const double rp = P.nu_b * row_residual<EXT>(P, l, aw) / P.Sy[l];
            acc[2] += rp * rp;                           // SL_RP2
            acc[3] += row_dual_term<EXT>(P, l, wy);           // SL_BY
            const double my = wy - V.ay[l];
            acc[4] += my * my;                           // SL_MOVY2
          }
        });
      } else {
        // the reflected-Halpern update of y and A x fused into the pass
        for_rows_range(r0, r1, Lr, [&](long l, int sub, bool act) {
          const double aw = spmv_row(P.A_ptr, P.A_col, M.A, W, l, sub, Lr, act);
          if (act && sub == 0) {
            const double yl = V.y[l], axl = V.Ax[l];
            const double wy = dual_cand<EXT>(P, l, yl, 2.0 * aw - axl, sigma);
            V.wy[l] = wy;
            V.Aw[l] = aw;
            if (tracing) TB.wy[L.C.ktot * m + l] = wy;
            V.y[l] = c1h * (2.0 * rho * wy + (1.0 - 2.0 * rho) * yl) + c3h * V.ay[l];
            V.Ax[l] = c1h * (2.0 * rho * aw + (1.0 - 2.0 * rho) * axl) + c3h * V.Aa[l];
          }
        });
      }
      if constexpr (SOLO) {
        if (!check) hw_clear(L);
      }
      for_range(c0, c1, [&](long i, bool act) {
        double xn = 0.0;
        if (act) {
          const double xi = V.x[i], wi = W[i];
          if (tracing) TB.wx[L.C.ktot * n + i] = wi;
          if (check) {
            const double dx = xi - wi;
            acc[5] += dx * dx;                           // SL_DX2
            const double mx = wi - V.ax[i];
            acc[6] += mx * mx;                           // SL_MOVX2
            acc[7] += P.c[i] * wi;                       // SL_CX
          } else {
            xn = c1h * (2.0 * rho * wi + (1.0 - 2.0 * rho) * xi) + c3h * V.ax[i];
            acc[5] += (xn - xi) * (xn - xi);             // SL_XMOV2
            V.x[i] = xn;
          }
        }
        if constexpr (SOLO) {
          if (!check) hw_add(L, RB, r, i, xn, act);
        }
      });
      if (check) {
        const int sl[8] = {SL_DY2, SL_ADXDY, SL_RP2, SL_BY, SL_MOVY2, SL_DX2, SL_MOVX2, SL_CX};
        block_store(L, acc, sl, 8, part, G, rank);
      } else {
        const int sl[1] = {SL_XMOV2};
        block_store(L, &acc[5], sl, 1, part, G, rank);
        hw_finish(RB, V.x, nullptr);
      }
    }
    SYNC_OR_EXIT();

    if (tid == 0) {
      L.C.inner_total += jcount;
      L.C.ktot = kt1;
    }
    __syncthreads();

    if (!check) {
      {
        const int sl[1] = {SL_XMOV2};
        team_reduce_sh(L, part, G, sl, 1, r, L.C.hx);
      }
      if (tid == 0) {
        L.C.eps_in = fmin(L.C.eps_in, fmax(S.gamma_in * sqrt(L.scal[SL_XMOV2]) / tau, S.eps_min));
        L.C.k = k + 1;
        if (tracing && rank == 0) {
          double* sc = TB.sc + (kt1 - 1) * 8;
          sc[0] = tau; sc[1] = sigma; sc[2] = omega; sc[3] = eps_in;
          sc[4] = jcount; sc[5] = 0.0; sc[6] = 0.0; sc[7] = 0.0;
        }
      }
      __syncthreads();
      continue;
    }
    }

    // ---------------------------------------------------------- check
    // reflected Halpern: on the candidate w (R^ w_x is the last inner R^ u;
    // diagonal Q has r = 0); averaged epochs: on the new state zbar
    tmark(L, prof, PT_CHECK);
    if (!avg) {
      const int sl[8] = {SL_DY2, SL_ADXDY, SL_RP2, SL_BY, SL_MOVY2, SL_DX2, SL_MOVX2, SL_CX};
      team_reduce(L, part, G, sl, 8);
    }
    dual_check(avg ? V.x : W, avg ? V.y : V.wy, avg ? L.C.hx : L.hu);
    SYNC_OR_EXIT();
    {
      const int sl[3] = {SL_XQX, SL_RD2, SL_BOXD};
      team_reduce(L, part, G, sl, EXT ? 3 : 2);
    }
    if (avg) {
      if (tid == 0) {
        kkt_status(L.C, false);
        L.C.k = 0;
        L.C.restarts += 1;
        if (tracing && rank == 0) {
          double* t = TB.sc + (kt1 - 1) * 8;
          t[0] = tau; t[1] = sigma; t[2] = omega; t[3] = eps_in;
          t[4] = jcount; t[5] = 1.0; t[6] = 1.0; t[7] = 0.0;
        }
      }
      __syncthreads();
      if (L.C.status != 0) break;
      continue;
    }
    if (tid == 0) {
      Ctl& C = L.C;
      const double* sc = L.scal;
      const double E2 = omega * sc[SL_DX2] + sc[SL_DY2] / omega + 2.0 * P.eta * sc[SL_ADXDY];
      const double E = sqrt(fmax(E2, 0.0));
      bool rs = false;
      if (k == 0) C.E0 = E;
      else rs = (E <= S.beta_s * C.E0) || (E <= S.beta_n * C.E0 && E > C.Eprev) ||
                ((double)(k + 1) >= S.beta_a * (double)kt1);
      C.Eprev = E;
      C.lastE = E;
      kkt_status(C, !isfinite(E));
      if (C.status == 0 && rs) {
        const double dxm = sqrt(sc[SL_MOVX2]), dym = sqrt(sc[SL_MOVY2]);
        if (dxm > 1e-12 && dym > 1e-12) {
          const double e = log(dym / (omega * dxm));
          C.pid_I = S.pid_beta_i * C.pid_I + e;
          C.omega = exp(log(omega) + S.pid_kp * e + S.pid_ki * C.pid_I + S.pid_kd * (e - C.e_prev));
          C.e_prev = e;
        }
        C.k = 0;
        C.restarts += 1;
      }
      L.done = rs ? 1 : 0;
      if (tracing && rank == 0) {
        double* t = TB.sc + (kt1 - 1) * 8;
        t[0] = tau; t[1] = sigma; t[2] = omega; t[3] = eps_in;
        t[4] = jcount; t[5] = rs ? 1.0 : 0.0; t[6] = 1.0; t[7] = E;
      }
    }
    __syncthreads();
    const bool restart = L.done != 0;
    if (L.C.status != 0) break;

    // ---------------------------------------------------------- restart or Halpern
    tmark(L, prof, PT_HALP);
    {
      double xm = 0.0;
      if constexpr (SOLO) {
        if (!restart) hw_clear(L);
      }
      for (long l = r0 + tid; l < r1; l += BLOCK) {
        const double wy = V.wy[l], aw = V.Aw[l];
        if (restart) {
          V.y[l] = wy; V.ay[l] = wy; V.Ax[l] = aw; V.Aa[l] = aw;
        } else {
          V.y[l] = c1h * (2.0 * rho * wy + (1.0 - 2.0 * rho) * V.y[l]) + c3h * V.ay[l];
          V.Ax[l] = c1h * (2.0 * rho * aw + (1.0 - 2.0 * rho) * V.Ax[l]) + c3h * V.Aa[l];
        }
      }
      for_range(c0, c1, [&](long i, bool act) {
        double xn = 0.0;
        if (act) {
          const double wi = W[i];
          if (restart) {
            V.x[i] = wi; V.ax[i] = wi;
          } else {
            const double xi = V.x[i];
            xn = c1h * (2.0 * rho * wi + (1.0 - 2.0 * rho) * xi) + c3h * V.ax[i];
            xm += (xn - xi) * (xn - xi);
            V.x[i] = xn;
          }
        }
        if constexpr (SOLO) {
          if (!restart) hw_add(L, RB, r, i, xn, act);
        }
      });
      if (!restart) {
        const int sl[1] = {SL_XMOV2};
        block_store(L, &xm, sl, 1, part, G, rank);
        hw_finish(RB, V.x, nullptr);
      }
    }
    SYNC_OR_EXIT();
    if (restart) {
      if ((int)tid < r) L.C.hx[tid] = L.hu[tid];
      __syncthreads();
    } else {
      {
        const int sl[1] = {SL_XMOV2};
        team_reduce_sh(L, part, G, sl, 1, r, L.C.hx);
      }
      if (tid == 0) {
        L.C.eps_in = fmin(L.C.eps_in, fmax(S.gamma_in * sqrt(L.scal[SL_XMOV2]) / tau, S.eps_min));
        L.C.k = k + 1;
      }
      __syncthreads();
    }
  }
#undef SYNC_OR_EXIT
#undef PROJ
}

// ---------------------------------------------------------------------------
// single-problem kernel: the whole grid is one team
// ---------------------------------------------------------------------------
template <class MV, bool SOLO, bool EXT, bool CONES = true>
__device__ void solve_body(const KArgs& A) {
  __shared__ Lds L;
  const int rank = blockIdx.x, G = gridDim.x;
  if (threadIdx.x < PT_COUNT) L.pt[threadIdx.x] = 0ull;
  if (threadIdx.x == 0) {
    L.C = *A.ctl;
    L.pcat = PT_INIT;
    L.plast = wall_clock64();
    L.epoch = __hip_atomic_load(&A.bar->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  }
  __syncthreads();
  if (L.C.status != 0) return;
  const bool prof = A.profile != 0;
  const DevProblem& P = A.P;
  Own own;
  own.c0 = P.part_c[rank];
  own.c1 = P.part_c[rank + 1];
  own.r0 = P.part_r[rank];
  own.r1 = P.part_r[rank + 1];
  own.it = Items{P.part_w[rank], P.part_w[rank + 1], P.part_l[rank], P.part_l[rank + 1],
                 (int)P.part_lanes[4 * rank + 2]};
  own.la = P.part_lanes[4 * rank + 0];
  own.lr = P.part_lanes[4 * rank + 1];
  own.atperm = P.at_perm;
  own.atseg = P.at_perm ? P.at_seg + (kClasses + 1) * rank : nullptr;
  extern __shared__ __align__(16) unsigned char dyn_lds[];
  const Run run{&A.S, &A.T, A.stop_at, A.qmax, 0ull, A.lds_bytes > 0 ? dyn_lds : nullptr, A.lds_bytes};
  if constexpr (SOLO) {
    run_solver<CONES, MV, EXT>(run, P, A.V, A.ctl, SoloTeam{}, L, own, prof);
  } else {
    GridTeam T{A.bar, A.spin_limit, rank, G};
    run_solver<CONES, MV, EXT>(run, P, A.V, A.ctl, T, L, own, prof);
  }
  tmark(L, prof, PT_INIT);
  __syncthreads();
  if (prof && threadIdx.x < PT_COUNT) A.ptimes[(size_t)rank * PT_COUNT + threadIdx.x] += L.pt[threadIdx.x];
  if (rank == 0 && threadIdx.x == 0 && L.C.status != PDHCG_ABORTED) *A.ctl = L.C;
}

__global__ __launch_bounds__(BLOCK) void solve_kernel(KArgs A) { solve_body<double, false, false>(A); }

// row bounds, boxes and fixed-middle EXP blocks
__global__ __launch_bounds__(BLOCK) void solve_kernel_ext(KArgs A) { solve_body<double, false, true>(A); }

// problems without cone blocks (FREE / R+ only, no EXT feature): compiled
// without the projection code, at 4 waves per SIMD (two workgroups per CU),
// so twice the gathers of the latency-bound products are in flight
__global__ __launch_bounds__(BLOCK, 4) void solve_kernel_lin(KArgs A) { solve_body<double, false, false, false>(A); }
// the same with row bounds and boxes (no fixed-middle EXP blocks: those are
// cone items)
__global__ __launch_bounds__(BLOCK, 4) void solve_kernel_lin_ext(KArgs A) { solve_body<double, false, true, false>(A); }

// FP32 bulk sweeps (FP32 copies of A, A^T, P, R); everything else as above
__global__ __launch_bounds__(BLOCK) void solve_kernel_f32(KArgs A) { solve_body<float, false, false>(A); }
__global__ __launch_bounds__(BLOCK) void solve_kernel_f32_ext(KArgs A) { solve_body<float, false, true>(A); }
// and without cone blocks, at two workgroups per CU like the FP64 cone-free
// kernels (the FP64 polish runs those on the same grid)
__global__ __launch_bounds__(BLOCK, 4) void solve_kernel_f32_lin(KArgs A) { solve_body<float, false, false, false>(A); }
__global__ __launch_bounds__(BLOCK, 4) void solve_kernel_f32_lin_ext(KArgs A) { solve_body<float, false, true, false>(A); }

// a grid of one workgroup: workgroup barriers and the single-workgroup
// reductions of the batch kernels (the same arithmetic as a batch solve)
__global__ __launch_bounds__(BLOCK) void solve_kernel_one(KArgs A) { solve_body<double, true, false>(A); }
__global__ __launch_bounds__(BLOCK) void solve_kernel_one_ext(KArgs A) { solve_body<double, true, true>(A); }

// ---------------------------------------------------------------------------
// setup kernels: CSR SpMV and deterministic two-pass norms (power iteration)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void spmv_kernel(const int64_t* ptr, const int* col,
                                                     const double* val, const double* x,
                                                     double* y, long rows, int Lw) {
  const int groups = BLOCK / Lw;
  const int gid = threadIdx.x / Lw, sub = threadIdx.x & (Lw - 1);
  for (long base = (long)blockIdx.x * groups; base < rows; base += (long)gridDim.x * groups) {
    const long row = base + gid;
    const bool act = row < rows;
    const double s = spmv_row(ptr, col, val, x, row, sub, Lw, act);
    if (act && sub == 0) y[row] = s;
  }
}

// rows perm[0..count) with Lw lanes each (setup products of matrices with
// skewed row lengths, one launch per length class)
__global__ __launch_bounds__(BLOCK) void spmv_perm_kernel(const int64_t* ptr, const int* col,
                                                         const double* val, const double* x, double* y,
                                                         const int* perm, long count, int Lw) {
  const int groups = BLOCK / Lw;
  const int gid = threadIdx.x / Lw, sub = threadIdx.x & (Lw - 1);
  for (long base = (long)blockIdx.x * groups; base < count; base += (long)gridDim.x * groups) {
    const long q = base + gid;
    const bool act = q < count;
    const long row = act ? (long)perm[q] : 0;
    const double s = spmv_row(ptr, col, val, x, row, sub, Lw, act);
    if (act && sub == 0) y[row] = s;
  }
}

// one workgroup per row of perm[0..count): the longest rows
__global__ __launch_bounds__(BLOCK) void spmv_perm_block_kernel(const int64_t* ptr, const int* col,
                                                               const double* val, const double* x,
                                                               double* y, const int* perm, long count) {
  for (long q = blockIdx.x; q < count; q += gridDim.x)
    spmv_rows_block(ptr, col, val, x, y, (long)perm[q], (long)perm[q] + 1);
}

__global__ __launch_bounds__(BLOCK) void sumsq_partial_kernel(const double* x, long n, double* part) {
  __shared__ double red[NWAVE];
  double s = 0.0;
  for (long i = (long)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (long)gridDim.x * BLOCK) s += x[i] * x[i];
  s = wave_sum(s);
  if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
  __syncthreads();
  if (threadIdx.x == 0) {
    double t = 0.0;
    for (int w = 0; w < NWAVE; ++w) t += red[w];
    part[blockIdx.x] = t;
  }
}

__global__ __launch_bounds__(BLOCK) void finish_norm_kernel(const double* part, int np, double* out) {
  if (threadIdx.x < 64) {
    double s = 0.0;
    for (int j = threadIdx.x; j < np; j += 64) s += part[j];
    s = wave_sum(s);
    if (threadIdx.x == 0) out[0] = sqrt(s);
  }
}

__global__ __launch_bounds__(BLOCK) void scale_kernel(double* x, long n, const double* nrm) {
  const double f = nrm[0];
  for (long i = (long)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (long)gridDim.x * BLOCK)
    x[i] = f > 0.0 ? x[i] / f : x[i];
}

__global__ __launch_bounds__(BLOCK) void fill_kernel(double* x, long n, double v) {
  for (long i = (long)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (long)gridDim.x * BLOCK) x[i] = v;
}

// ---------------------------------------------------------------------------
// caller-facing vectors on the device: warm starts into the scaled space and
// results out of it (Section "Problem Rescaling": x^ = S_x x / nu_b,
// y^ = y / (nu_c S_y)), in the caller's coordinate order (perm[j] = the
// caller's index of internal coordinate j; null: the same order)
// ---------------------------------------------------------------------------
// dst[j] = S[j] src[perm[j]] / nu (x in), or src[j] / (nu S[j]) (y in)
__global__ __launch_bounds__(BLOCK) void scale_in_kernel(const double* src, const int* perm, const double* S,
                                                         double nu, int inv, double* dst, long n) {
  for (long j = (long)blockIdx.x * BLOCK + threadIdx.x; j < n; j += (long)gridDim.x * BLOCK) {
    const double v = src[perm ? perm[j] : j];
    dst[j] = inv ? v / (nu * S[j]) : S[j] * v / nu;
  }
}

// dst[perm[j]] = nu src[j] / S[j] (x out), or nu S[j] src[j] (y out)
__global__ __launch_bounds__(BLOCK) void scale_out_kernel(const double* src, const int* perm, const double* S,
                                                          double nu, int inv, double* dst, long n) {
  for (long j = (long)blockIdx.x * BLOCK + threadIdx.x; j < n; j += (long)gridDim.x * BLOCK)
    dst[perm ? perm[j] : j] = inv ? nu * src[j] / S[j] : nu * S[j] * src[j];
}

// the factor part of Q^ w: per workgroup, partial sums of (R^ w)_k over a
// slice of the coordinates (part[blockIdx.x * r + k])
__global__ __launch_bounds__(BLOCK) void rdot_partial_kernel(const double* R, int r, long n, const double* w,
                                                             double* part) {
  __shared__ double red[NWAVE];
  for (int k = 0; k < r; ++k) {
    double acc = 0.0;
    for (long i = (long)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (long)gridDim.x * BLOCK)
      acc += R[(size_t)k * n + i] * w[i];
    acc = wave_sum(acc);
    if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = acc;
    __syncthreads();
    if (threadIdx.x == 0) {
      double t = 0.0;
      for (int q = 0; q < NWAVE; ++q) t += red[q];
      part[(size_t)blockIdx.x * r + k] = t;
    }
    __syncthreads();
  }
}

// ht = D^ (R^ w) from the partials of nb workgroups (one workgroup, fixed
// summation order)
__global__ __launch_bounds__(BLOCK) void rdot_finish_kernel(const double* part, int nb, int r, const double* D,
                                                            double* ht) {
  __shared__ double hh[RMAX];
  if ((int)threadIdx.x < r) {
    double t = 0.0;
    for (int b = 0; b < nb; ++b) t += part[(size_t)b * r + threadIdx.x];
    hh[threadIdx.x] = t;
  }
  __syncthreads();
  if ((int)threadIdx.x < r) {
    double t = 0.0;
    for (int j = 0; j < r; ++j) t += D[threadIdx.x * r + j] * hh[j];
    ht[threadIdx.x] = t;
  }
}

// the dual slack of the original problem at the unscaled (x, y) of the
// scaled candidate (w, wy): s = nu_c S_x (Q^ w + c^ - A^T wy), with
// Q^ w = diag(Q^) w (diagonal Q), or P^ w + R^T ht (ht = D^ R^ w)
__global__ __launch_bounds__(BLOCK) void dual_slack_kernel(DevProblem P, const double* w, const double* wy,
                                                           const double* ht, const int* perm, double* out) {
  const long n = P.n;
  for (long i = (long)blockIdx.x * BLOCK + threadIdx.x; i < n; i += (long)gridDim.x * BLOCK) {
    double qw;
    if (P.q_diag) {
      qw = P.qd[i] * w[i];
    } else {
      qw = 0.0;
      if (P.p_diag) qw = P.Pd[i] * w[i];
      else if (P.P_ptr)
        for (int64_t k = P.P_ptr[i]; k < P.P_ptr[i + 1]; ++k) qw += P.P_val[k] * w[P.P_col[k]];
      for (int k = 0; k < P.r; ++k) qw += P.R[(size_t)k * n + i] * ht[k];
    }
    double aty = 0.0;
    for (int64_t k = P.AT_ptr[i]; k < P.AT_ptr[i + 1]; ++k) aty += P.AT_val[k] * wy[P.AT_col[k]];
    out[perm ? perm[i] : i] = P.nu_c * P.Sx[i] * (qw + P.c[i] - aty);
  }
}

// ---------------------------------------------------------------------------
// batch kernels: independent instances, one workgroup per instance at a time
// ---------------------------------------------------------------------------
// before every batch launch: control blocks zeroed, scaled warm starts (or
// zeros) into zb and y, root warm starts unset (NaN), queue at 0
__global__ __launch_bounds__(BLOCK) void batch_reset_kernel(const InstDesc* desc, int count,
                                                           int* queue) {
  if (blockIdx.x == 0 && threadIdx.x == 0) queue[0] = 0;
  for (int i = blockIdx.x; i < count; i += gridDim.x) {
    const InstDesc& D = desc[i];
    const long n = D.P.n, m = D.P.m;
    for (long j = threadIdx.x; j < n; j += BLOCK) D.V.zb[j] = D.x0 ? D.x0[j] : 0.0;
    for (long l = threadIdx.x; l < m; l += BLOCK) D.V.y[l] = D.y0 ? D.y0[l] : 0.0;
    for (int k = threadIdx.x; k < D.n_warm; k += BLOCK) D.V.warm[k] = __builtin_nan("");
    double* c = reinterpret_cast<double*>(D.ctl);
    for (int k = threadIdx.x; k < (int)(sizeof(Ctl) / sizeof(double)); k += BLOCK) c[k] = 0.0;
  }
}

// persistent batch solve: each workgroup takes the next queue position,
// solves that instance to termination with the single-workgroup team, and
// stores its control block; instances are queued largest first
template <bool CONES, bool EXT>
__device__ void batch_body(const BatchArgs& B) {
  __shared__ Lds L;
  __shared__ int slot;
  const unsigned long long deadline = B.limit_ticks ? wall_clock64() + B.limit_ticks : 0ull;
  const bool prof = B.ptimes != nullptr;
  if (threadIdx.x < PT_COUNT) L.pt[threadIdx.x] = 0ull;
  for (;;) {
    if (threadIdx.x == 0) slot = atomicAdd(B.queue, 1);
    __syncthreads();
    const int q = __builtin_amdgcn_readfirstlane(slot);
    if (q >= B.count) break;
    const int inst = __builtin_amdgcn_readfirstlane(B.order[q]);
    const InstDesc& D = B.desc[inst];
    if (threadIdx.x == 0) {
      L.C = *D.ctl;
      L.pcat = PT_INIT;
      L.plast = wall_clock64();
      L.epoch = 0u;
    }
    __syncthreads();
    if (L.C.status == 0) {
      Own own;
      own.c0 = 0;
      own.c1 = D.P.n;
      own.r0 = 0;
      own.r1 = D.P.m;
      own.it = Items{0, D.P.n_wave, 0, D.P.n_lane, D.lg};
      own.la = D.la;
      own.lr = D.lr;
      own.atperm = nullptr;
      own.atseg = nullptr;
      const Run run{&B.S, &D.T, B.stop_at, D.qmax, deadline, nullptr, 0};
      run_solver<CONES, double, EXT>(run, D.P, D.V, D.ctl, SoloTeam{}, L, own, prof);
      tmark(L, prof, PT_INIT);
      __syncthreads();
      if (threadIdx.x == 0) *D.ctl = L.C;
    }
    __syncthreads();
  }
  if (prof && threadIdx.x < PT_COUNT) B.ptimes[(size_t)blockIdx.x * PT_COUNT + threadIdx.x] = L.pt[threadIdx.x];
}

__global__ __launch_bounds__(BLOCK) void batch_kernel(BatchArgs B) { batch_body<true, false>(B); }
__global__ __launch_bounds__(BLOCK) void batch_kernel_ext(BatchArgs B) { batch_body<true, true>(B); }

// batches without cone blocks: 4 waves per SIMD (two instances per CU)
__global__ __launch_bounds__(BLOCK, 4) void batch_kernel_lin(BatchArgs B) { batch_body<false, false>(B); }
__global__ __launch_bounds__(BLOCK, 4) void batch_kernel_lin_ext(BatchArgs B) { batch_body<false, true>(B); }

// ||A^||_2 of every instance: the power iteration of the single-problem
// setup (128 steps of A^T A from 1/sqrt(n), normalised each step), one
// workgroup per instance; out[i] = sqrt of the last norm (0 if A is empty)
__global__ __launch_bounds__(BLOCK) void batch_power_kernel(const InstDesc* desc, int count, int iters,
                                                           double* out) {
  __shared__ double red[NWAVE];
  __shared__ double nrm;
  for (int i = blockIdx.x; i < count; i += gridDim.x) {
    const DevProblem& P = desc[i].P;
    const DevVec& V = desc[i].V;
    const long n = P.n, m = P.m;
    double* z = V.v;
    double* t = V.Aw;
    double* w = V.g;
    if (m == 0 || P.A_ptr[m] == 0) {
      if (threadIdx.x == 0) out[i] = 0.0;
      continue;
    }
    const double z0 = 1.0 / sqrt((double)n);
    for (long j = threadIdx.x; j < n; j += BLOCK) z[j] = z0;
    __syncthreads();
    double lam = 0.0;
    for (int it = 0; it < iters; ++it) {
      spmv_range(P.A_ptr, P.A_col, P.A_val, z, t, 0, m, desc[i].lr);
      __syncthreads();
      spmv_range(P.AT_ptr, P.AT_col, P.AT_val, t, w, 0, n, desc[i].la);
      __syncthreads();
      double s = 0.0;
      for (long j = threadIdx.x; j < n; j += BLOCK) s += w[j] * w[j];
      s = wave_sum(s);
      if ((threadIdx.x & 63) == 0) red[threadIdx.x >> 6] = s;
      __syncthreads();
      if (threadIdx.x == 0) {
        double tot = 0.0;
        for (int k = 0; k < NWAVE; ++k) tot += red[k];
        nrm = sqrt(tot);
      }
      __syncthreads();
      const double f = nrm;
      for (long j = threadIdx.x; j < n; j += BLOCK) z[j] = f > 0.0 ? w[j] / f : w[j];
      lam = f;
      __syncthreads();
    }
    if (threadIdx.x == 0) out[i] = sqrt(lam);
    __syncthreads();
  }
}

// pack every instance's candidate (w_x, w_y) into contiguous outputs
// the result of each instance: the last PDHG candidate (reflected Halpern)
// or the state, which is the epoch average after the last restart (averaged
// epochs)
__global__ __launch_bounds__(BLOCK) void batch_gather_kernel(const InstDesc* desc, int count,
                                                            const long* offx, const long* offy,
                                                            double* ox, double* oy, int avg) {
  for (int i = blockIdx.x; i < count; i += gridDim.x) {
    const InstDesc& D = desc[i];
    const double* X = avg ? D.V.x : (D.P.q_diag ? D.V.wx : D.V.u);
    const double* Y = avg ? D.V.y : D.V.wy;
    const long n = D.P.n, m = D.P.m;
    for (long j = threadIdx.x; j < n; j += BLOCK) ox[offx[i] + j] = X[j];
    for (long l = threadIdx.x; l < m; l += BLOCK) oy[offy[i] + l] = Y[l];
  }
}

// ---------------------------------------------------------------------------
// diagnostic: a batch of blocks of one cone type projected by the solver's
// own projection routines (wave items for SOC/RSOC with a group of lg lanes
// per block, one lane per EXP/POW block, elementwise FREE/R+); blocks are
// stored one after another, dim coordinates each
// ---------------------------------------------------------------------------
struct ArrSrc {
  const double* rv;
  const double* mv;   // null: unit metric
  long st;
  __device__ double r(int j) const { return rv[st + j]; }
  __device__ double m(int j) const { return mv ? mv[st + j] : 1.0; }
};

__global__ __launch_bounds__(BLOCK) void project_kernel(int type, int dim, long count, const double* alpha,
                                                        const double* r, const double* m,
                                                        const unsigned char* euclid, double* out, int lg) {
  const long gtid = (long)blockIdx.x * BLOCK + threadIdx.x;
  const long nthr = (long)gridDim.x * BLOCK;
  if (type == PDHCG_CONE_SOC || type == PDHCG_CONE_RSOC) {
    const long ngroups = nthr / lg;
    for (long b = gtid / lg; b < count; b += ngroups) {
      const long st = b * (long)dim;
      project_wave_item(type, dim, euclid[b] != 0, ArrSrc{r, m, st},
                        [out, st](int j, double v) { out[st + j] = v; }, nullptr, lg);
    }
  } else if (type == PDHCG_CONE_EXP || type == PDHCG_CONE_POW || type == PDHCG_CONE_EXP1) {
    for (long b = gtid; b < count; b += nthr) {
      const long st = 3 * b;
      const bool eu = euclid[b] != 0;
      const double m0 = eu ? 1.0 : m[st], m1 = eu ? 1.0 : m[st + 1], m2 = eu ? 1.0 : m[st + 2];
      const Trip o = type == PDHCG_CONE_EXP ? project_exp(r[st], r[st + 1], r[st + 2], m0, m1, m2, nullptr)
                     : type == PDHCG_CONE_POW ? project_pow(r[st], r[st + 1], r[st + 2], alpha[b], m0, m1, m2,
                                                            nullptr)
                                              : project_exp1(r[st], r[st + 2], m0, m2, 1.0);
      out[st] = o.a;
      out[st + 1] = o.b;
      out[st + 2] = o.c;
    }
  } else {
    const uint8_t ct = type == PDHCG_CONE_FREE ? CT_FREE : CT_NONNEG;
    for (long i = gtid; i < count * (long)dim; i += nthr) out[i] = elem_proj(ct, r[i]);
  }
}

// ---------------------------------------------------------------------------
// host wrappers
// ---------------------------------------------------------------------------
int block_size() { return BLOCK; }

// A plain launch: the grid barrier needs every workgroup resident at once,
// so the launch is refused when the grid exceeds what the device holds
// with this kernel's registers and LDS (the barrier's waits are bounded as
// well, so a grid that cannot all be resident ends with PDHCG_ABORTED, not a
// hang).
// the solver kernel of a launch: FP32 bulk or FP64, a grid of one
// workgroup, the EXT features, problems without cone blocks
static const void* solver_kernel_for(bool fp32, bool ext, bool cones, int grid) {
  if (fp32) {
    if (ext) return cones ? (const void*)solve_kernel_f32_ext : (const void*)solve_kernel_f32_lin_ext;
    return cones ? (const void*)solve_kernel_f32 : (const void*)solve_kernel_f32_lin;
  }
  if (grid == 1) return ext ? (const void*)solve_kernel_one_ext : (const void*)solve_kernel_one;
  if (ext) return cones ? (const void*)solve_kernel_ext : (const void*)solve_kernel_lin_ext;
  return cones ? (const void*)solve_kernel : (const void*)solve_kernel_lin;
}

hipError_t launch_solve(const KArgs& args, bool fp32, int grid, hipStream_t stream) {
  KArgs a = args;
  void* params[] = {&a};
  const bool ext = args.P.ext != 0;
  const bool cones = args.P.n_wave > 0 || args.P.n_lane > 0;
  const void* k = solver_kernel_for(fp32, ext, cones, grid);
  int dev = 0, ncu = 0, per = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e == hipSuccess) e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, BLOCK, (size_t)args.lds_bytes);
  if (e != hipSuccess) return e;
  if ((long)per * (long)ncu < (long)grid) return hipErrorCooperativeLaunchTooLarge;
  return hipLaunchKernel(k, dim3(grid), dim3(BLOCK), params, (size_t)args.lds_bytes, stream);
}

hipError_t max_resident_grid_for(bool fp32, bool ext, bool cones, int lds_bytes, int* out) {
  int dev = 0, ncu = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e == hipSuccess) e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  // FP32 mode polishes in FP64 on the same grid: both kernels must fit
  int per = 0, per64 = 0;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per64, solver_kernel_for(false, ext, cones, 2), BLOCK,
                                                   (size_t)lds_bytes);
  if (e != hipSuccess) return e;
  per = per64;
  if (fp32) {
    e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, solver_kernel_for(true, ext, cones, 2), BLOCK,
                                                     (size_t)lds_bytes);
    if (e != hipSuccess) return e;
    per = std::min(per, per64);
  }
  *out = per * ncu;
  return hipSuccess;
}

hipError_t launch_spmv(const int64_t* ptr, const int* col, const double* val, const double* x,
                       double* y, long rows, int Lw, hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  long per = BLOCK / Lw;
  long grid = (rows + per - 1) / per;
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(spmv_kernel, dim3((unsigned)grid), dim3(BLOCK), 0, st, ptr, col, val, x, y,
                     rows, Lw);
  return hipGetLastError();
}

hipError_t launch_spmv_classes(const int64_t* ptr, const int* col, const double* val, const double* x,
                               double* y, const int* perm, const long* seg, hipStream_t st) {
  static const int lanes[5] = {1, 4, 16, 64, BLOCK};
  for (int c = 0; c < 5; ++c) {
    const long cnt = seg[c + 1] - seg[c];
    if (cnt <= 0) continue;
    if (lanes[c] >= BLOCK) {
      const long grid = std::min<long>(cnt, 4096);
      hipLaunchKernelGGL(spmv_perm_block_kernel, dim3((unsigned)grid), dim3(BLOCK), 0, st, ptr, col, val, x, y,
                         perm + seg[c], cnt);
    } else {
      const long per = BLOCK / lanes[c];
      const long grid = std::min<long>((cnt + per - 1) / per, 4096);
      hipLaunchKernelGGL(spmv_perm_kernel, dim3((unsigned)grid), dim3(BLOCK), 0, st, ptr, col, val, x, y,
                         perm + seg[c], cnt, lanes[c]);
    }
  }
  return hipGetLastError();
}

// nrm[0] = ||x||; part: scratch of >= 1024 doubles
hipError_t launch_norm(const double* x, long n, double* part, double* nrm, hipStream_t st) {
  int grid = (int)((n + BLOCK - 1) / BLOCK);
  if (grid > 1024) grid = 1024;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(sumsq_partial_kernel, dim3(grid), dim3(BLOCK), 0, st, x, n, part);
  hipLaunchKernelGGL(finish_norm_kernel, dim3(1), dim3(BLOCK), 0, st, part, grid, nrm);
  return hipGetLastError();
}

hipError_t launch_scale(double* x, long n, const double* nrm, hipStream_t st) {
  int grid = (int)((n + BLOCK - 1) / BLOCK);
  if (grid > 2048) grid = 2048;
  if (grid < 1) grid = 1;
  hipLaunchKernelGGL(scale_kernel, dim3(grid), dim3(BLOCK), 0, st, x, n, nrm);
  return hipGetLastError();
}

hipError_t launch_fill(double* x, long n, double v, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  int grid = (int)((n + BLOCK - 1) / BLOCK);
  if (grid > 2048) grid = 2048;
  hipLaunchKernelGGL(fill_kernel, dim3(grid), dim3(BLOCK), 0, st, x, n, v);
  return hipGetLastError();
}

static int io_grid(long n) {
  return (int)std::max<long>(1, std::min<long>((n + BLOCK - 1) / BLOCK, 2048));
}

hipError_t launch_scale_in(const double* src, const int* perm, const double* S, double nu, bool inv, double* dst,
                           long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(scale_in_kernel, dim3(io_grid(n)), dim3(BLOCK), 0, st, src, perm, S, nu, inv ? 1 : 0, dst, n);
  return hipGetLastError();
}

hipError_t launch_scale_out(const double* src, const int* perm, const double* S, double nu, bool inv, double* dst,
                            long n, hipStream_t st) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(scale_out_kernel, dim3(io_grid(n)), dim3(BLOCK), 0, st, src, perm, S, nu, inv ? 1 : 0, dst,
                     n);
  return hipGetLastError();
}

hipError_t launch_dual_slack(const DevProblem& P, const double* w, const double* wy, const int* perm, double* io,
                             double* out, hipStream_t st) {
  if (P.n <= 0) return hipSuccess;
  const double* ht = io;
  if (!P.q_diag && P.r > 0) {
    const int nb = std::min(IO_PARTS, io_grid(P.n));
    double* part = io + RMAX;
    hipLaunchKernelGGL(rdot_partial_kernel, dim3(nb), dim3(BLOCK), 0, st, P.R, P.r, (long)P.n, w, part);
    hipLaunchKernelGGL(rdot_finish_kernel, dim3(1), dim3(BLOCK), 0, st, (const double*)part, nb, P.r, P.Dm, io);
  }
  hipLaunchKernelGGL(dual_slack_kernel, dim3(io_grid(P.n)), dim3(BLOCK), 0, st, P, w, wy, ht, perm, out);
  return hipGetLastError();
}

hipError_t reset_cone_failure(hipStream_t st) {
  const unsigned zero = 0u;
  return hipMemcpyToSymbolAsync(HIP_SYMBOL(g_cone_fail_count), &zero, sizeof(zero), 0, hipMemcpyHostToDevice,
                                st);
}

hipError_t read_cone_failure(double rec[8], unsigned* count) {
  hipError_t e = hipMemcpyFromSymbol(count, HIP_SYMBOL(g_cone_fail_count), sizeof(unsigned));
  if (e != hipSuccess) return e;
  return hipMemcpyFromSymbol(rec, HIP_SYMBOL(g_cone_fail), 8 * sizeof(double));
}

// flags[b] = 1 when the metric is absent or constant on block b (the
// Euclidean formula applies, Pi^{cI} = Pi^I), else 0
__global__ __launch_bounds__(BLOCK) void euclid_flags_kernel(long count, int dim, const double* m,
                                                             unsigned char* flags) {
  for (long b = (long)blockIdx.x * BLOCK + threadIdx.x; b < count; b += (long)gridDim.x * BLOCK) {
    bool c = true;
    if (m) {
      const double* mb = m + b * (long)dim;
      for (int j = 1; j < dim; ++j) c = c && (mb[j] == mb[0]);
    }
    flags[b] = c ? 1 : 0;
  }
}

hipError_t launch_project(int type, int dim, long count, const double* alpha, const double* r,
                          const double* m, const unsigned char* euclid, double* out, hipStream_t st) {
  if (count <= 0) return hipSuccess;
  int lg = 1;
  long threads = count;
  if (type == PDHCG_CONE_SOC || type == PDHCG_CONE_RSOC) {
    // the group width the solver gives a block of this size
    lg = dim <= 17 ? 16 : (dim <= 33 ? 32 : 64);
    threads = count * lg;
  } else if (type != PDHCG_CONE_EXP && type != PDHCG_CONE_POW && type != PDHCG_CONE_EXP1) {
    threads = count * (long)dim;
  }
  const long grid = std::max<long>(1, std::min<long>((threads + BLOCK - 1) / BLOCK, 4096));
  hipLaunchKernelGGL(project_kernel, dim3((unsigned)grid), dim3(BLOCK), 0, st, type, dim, count, alpha, r, m,
                     euclid, out, lg);
  return hipGetLastError();
}

static const void* batch_kernel_for(bool cones, bool ext) {
  return cones ? (ext ? (const void*)batch_kernel_ext : (const void*)batch_kernel)
               : (ext ? (const void*)batch_kernel_lin_ext : (const void*)batch_kernel_lin);
}

int batch_grid_limit(bool cones, bool ext) {
  int dev = 0, ncu = 0, per = 0;
  if (hipGetDevice(&dev) != hipSuccess) return 256;
  if (hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess) return 256;
  const void* k = batch_kernel_for(cones, ext);
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, k, BLOCK, 0) != hipSuccess) return ncu;
  return std::max(1, per * ncu);
}

hipError_t launch_batch(const BatchArgs& args, bool cones, bool ext, int grid, hipStream_t st) {
  BatchArgs a = args;
  void* params[] = {&a};
  return hipLaunchKernel(batch_kernel_for(cones, ext), dim3(grid), dim3(BLOCK), params, 0, st);
}

hipError_t launch_batch_reset(const InstDesc* desc, int count, int* queue, hipStream_t st) {
  const int grid = std::max(1, std::min(count, 4096));
  hipLaunchKernelGGL(batch_reset_kernel, dim3(grid), dim3(BLOCK), 0, st, desc, count, queue);
  return hipGetLastError();
}

hipError_t launch_batch_power(const InstDesc* desc, int count, int iters, double* out, hipStream_t st) {
  const int grid = std::max(1, std::min(count, batch_grid_limit(false, false)));
  hipLaunchKernelGGL(batch_power_kernel, dim3(grid), dim3(BLOCK), 0, st, desc, count, iters, out);
  return hipGetLastError();
}

hipError_t launch_batch_gather(const InstDesc* desc, int count, const long* offx, const long* offy,
                               double* ox, double* oy, int avg, hipStream_t st) {
  const int grid = std::max(1, std::min(count, 4096));
  hipLaunchKernelGGL(batch_gather_kernel, dim3(grid), dim3(BLOCK), 0, st, desc, count, offx, offy, ox,
                     oy, avg);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// the allocation-free projection entry point: its per-block flags live in a
// static device array (one copy per device, held until the process ends)
// whose device address is looked up once per device
// ---------------------------------------------------------------------------
constexpr long kNoAllocMaxBlocks = 1L << 22;   // 4 MiB of flags per device
static __device__ __align__(256) unsigned char scratch[kNoAllocMaxBlocks];

namespace {
constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
void* g_scratch_ptr[kMaxDevices] = {};
}  // namespace

// device address of `scratch` on the current device (looked up on the first
// call per device; the host-side name is not a device address)
static hipError_t scratch_address(void** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (!g_scratch_ptr[dev]) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_ptr[dev] = p;
  }
  *out = g_scratch_ptr[dev];
  return hipSuccess;
}

long noalloc_max_blocks() { return kNoAllocMaxBlocks; }

}  // namespace pdhcg

extern "C" int pdhcg_project_cones_noalloc(int32_t type, int32_t dim, int64_t count, const double* alpha,
                                           const double* r, const double* metric, double* out,
                                           void* stream) {
  using namespace pdhcg;
  if (type < PDHCG_CONE_FREE || type > PDHCG_CONE_EXP1 || type == PDHCG_CONE_BOX || dim < 1 || count < 0)
    return PDHCG_E_ARG;
  if ((type == PDHCG_CONE_RSOC && dim < 2) ||
      ((type == PDHCG_CONE_EXP || type == PDHCG_CONE_POW || type == PDHCG_CONE_EXP1) && dim != 3))
    return PDHCG_E_CONE;
  if (count > kNoAllocMaxBlocks) return PDHCG_E_ARG;
  if (count == 0) return PDHCG_OK;
  if (!r || !out || (type == PDHCG_CONE_POW && !alpha)) return PDHCG_E_ARG;
  void* flags = nullptr;
  if (scratch_address(&flags) != hipSuccess) return PDHCG_E_HIP;
  hipStream_t st = (hipStream_t)stream;
  const long grid = std::max<long>(1, std::min<long>((count + BLOCK - 1) / BLOCK, 4096));
  hipLaunchKernelGGL(euclid_flags_kernel, dim3((unsigned)grid), dim3(BLOCK), 0, st, (long)count, (int)dim, metric,
                     (unsigned char*)flags);
  if (hipGetLastError() != hipSuccess) return PDHCG_E_HIP;
  if (launch_project(type, dim, (long)count, alpha, r, metric, (const unsigned char*)flags, out, st) != hipSuccess)
    return PDHCG_E_HIP;
  return PDHCG_OK;
}
