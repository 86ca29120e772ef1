// Persistent cooperative solver kernel for restarted PDHG on conic QP.
//
// One launch runs outer iterations until the next host poll point, the
// iteration limit or termination.  The workgroups of the grid form one team:
// phases are separated by a grid barrier, every reduction is written as one
// partial per workgroup and re-reduced by every workgroup in the same fixed
// order (deterministic and identical everywhere), so every workgroup takes
// the same control decisions (inner stop, restart, termination) without any
// host round trip.
//
// Outer iteration (reflected-Halpern epoch, eq. stored-pdhg-candidate and
// eq. rh-update; primal-first PDHG operator eq. theory-pdhg-map):
//   P1  coordinate pass over rows of A^T:  v = x + tau A^T y; diagonal Q:
//       x~ = (v - tau c)/(1 + tau q) (eq. diagonal-q-metric), elementwise
//       cones projected at once; general Q: g0 = Q x + c + (x - v)/tau and the
//       first Jacobi step (alpha = 1).
//   P2  cone blocks projected in the metric (wave per SOC/RSOC, lane per
//       EXP/POW).
//   P3/P4 repeated: g = Q u + c + (u - v)/tau, BB step length
//       <s, J s>/<s, dg> (eq. jacobi-bb-step), projected step; stop when the
//       Euclidean step norm <= eps_in (eq. current-inner-step-stop).
//   P6  row pass over A: A w_x, w_y = y + sigma (b - (2 A w_x - A x)); on
//       non-check iterations the Halpern update of x, y and A x is fused here.
//   Check iterations (k = 0 of an epoch and every check_every evaluations):
//       fixed-point error E (eq. practical-fixed-point-movement), restart rule
//       (eq. practical-restart-rule), relative KKT residuals of the unscaled
//       candidate, PID primal weight on restart (eq. pid-error, pid-weight).
#include <hip/hip_runtime.h>

#include <stdint.h>

#include "common.hpp"
#include "cones.hpp"
#include "solver.hpp"

namespace pdhcg {

constexpr int BLOCK = 256;
constexpr int NWAVE = BLOCK / 64;
constexpr double DEPS = 2.220446049250313e-16;

struct Lds {
  double red[16][NWAVE];
  double scal[SL_COUNT];
  double hw[NWAVE][RMAX];
  double ht[RMAX];       // D^ h for the Q product of the current pass
  double hu[RMAX];       // R^ u of the current inner iterate
  Ctl C;
  double tau, sigma, alpha, last;
  int flag;
  int done;
};

// ---------------------------------------------------------------------------
// grid barrier with a bounded wait: if a workgroup waits longer than
// `limit` ticks of the constant-rate wall clock, the abort flag is raised and
// every workgroup leaves the kernel at its next barrier.
// ---------------------------------------------------------------------------
__device__ bool grid_sync(Barrier* bar, int G, Lds& L, unsigned long long limit) {
  __syncthreads();
  if (threadIdx.x == 0) {
    int ab = 0;
    __threadfence();
    if (G > 1) {
      unsigned gen = __hip_atomic_load(&bar->gen, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
      __threadfence();
      unsigned arrived = __hip_atomic_fetch_add(&bar->count, 1u, __ATOMIC_ACQ_REL,
                                                __HIP_MEMORY_SCOPE_AGENT);
      if (arrived == (unsigned)G - 1u) {
        __hip_atomic_store(&bar->count, 0u, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        __hip_atomic_store(&bar->gen, gen + 1u, __ATOMIC_RELEASE, __HIP_MEMORY_SCOPE_AGENT);
      } else {
        unsigned long long t0 = wall_clock64();
        while (__hip_atomic_load(&bar->gen, __ATOMIC_ACQUIRE, __HIP_MEMORY_SCOPE_AGENT) == gen) {
          __builtin_amdgcn_s_sleep(1);
          if (__hip_atomic_load(&bar->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT)) break;
          if (wall_clock64() - t0 > limit) {
            __hip_atomic_store(&bar->abort, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
            break;
          }
        }
      }
      __threadfence();
      ab = __hip_atomic_load(&bar->abort, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    L.flag = ab;
  }
  __syncthreads();
  return L.flag == 0;
}

// sum of up to 16 per-thread values over the workgroup; thread 0..k-1 store
// partial[slot * G + rank]
__device__ void block_store(Lds& L, const double* v, const int* slots, int k, double* partials,
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

// R^ u accumulators (one row of partials per rank of R)
__device__ __forceinline__ void hw_clear(Lds& L, int r) {
  for (int i = threadIdx.x; i < NWAVE * RMAX; i += BLOCK) (&L.hw[0][0])[i] = 0.0;
  __syncthreads();
}

// wave-uniform: add R[k, i] * val for this lane (0 if !active)
__device__ __forceinline__ void hw_add(Lds& L, const double* R, int n, int r, long i, double val,
                                       bool active) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int k = 0; k < r; ++k) {
    double t = active ? R[(size_t)k * n + i] * val : 0.0;
    t = wave_sum(t);
    if (lane == 0) L.hw[wv][k] += t;
  }
}

__device__ void hw_store(Lds& L, int r, double* partials, int G, int rank) {
  __syncthreads();
  if ((int)threadIdx.x < r) {
    double s = 0.0;
    for (int w = 0; w < NWAVE; ++w) s += L.hw[w][threadIdx.x];
    partials[(size_t)(SL_H0 + threadIdx.x) * G + rank] = s;
  }
  __syncthreads();
}

// reduce `k` slots over the G partials into L.scal[slot]; waves share slots
__device__ void team_reduce(Lds& L, const double* partials, int G, const int* slots, int k) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int i = wv; i < k; i += NWAVE) {
    const double* p = partials + (size_t)slots[i] * G;
    double s = 0.0;
    for (int j = lane; j < G; j += 64) s += p[j];
    s = wave_sum(s);
    if (lane == 0) L.scal[slots[i]] = s;
  }
  __syncthreads();
}

__device__ void team_reduce_h(Lds& L, const double* partials, int G, int r, double* dst) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  for (int k = wv; k < r; k += NWAVE) {
    const double* p = partials + (size_t)(SL_H0 + k) * G;
    double s = 0.0;
    for (int j = lane; j < G; j += 64) s += p[j];
    s = wave_sum(s);
    if (lane == 0) dst[k] = s;
  }
  __syncthreads();
}

// L.ht = D h
__device__ void make_ht(Lds& L, const DevProblem& P, const double* h) {
  if ((int)threadIdx.x < P.r) {
    double s = 0.0;
    for (int b = 0; b < P.r; ++b) s += P.Dm[threadIdx.x * P.r + b] * h[b];
    L.ht[threadIdx.x] = s;
  }
  __syncthreads();
}

__device__ __forceinline__ double group_sum(double v, int Lw) {
  for (int o = Lw >> 1; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double spmv_row(const int64_t* ptr, const int* col, const double* val,
                                           const double* x, long row, int sub, int Lw, bool active) {
  double acc = 0.0;
  if (active) {
    const int64_t e = ptr[row + 1];
    for (int64_t k = ptr[row] + sub; k < e; k += Lw) acc += val[k] * x[col[k]];
  }
  return group_sum(acc, Lw);
}

__device__ __forceinline__ double elem_proj(uint8_t ct, double z) {
  return ct == CT_NONNEG ? fmax(z, 0.0) : z;
}

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

struct StepSrc {            // u - alpha g / d
  const double* u;
  const double* g;
  MetricQ M;
  double alpha;
  long st;
  __device__ double r(int j) const { return u[st + j] - alpha * g[st + j] / M(st + j); }
  __device__ double m(int j) const { return M(st + j); }
};

// project every SOC/RSOC (wave items) and EXP/POW (lane items) block of src
// into dst.  After it returns, dst holds the projected cone coordinates of
// the blocks this wave processed and the block-scope fence makes them
// visible to the whole workgroup.
template <class MakeSrc>
__device__ void project_cone_items(const DevProblem& P, int gw, int gwaves, bool force_euclid,
                                   MakeSrc make, double* dst) {
  const int lane = threadIdx.x & 63;
  for (int it = gw; it < P.n_wave; it += gwaves) {
    const long st = P.wave_start[it];
    const int dim = P.wave_dim[it];
    auto src = make(st);
    const bool eu = force_euclid || P.wave_euclid[it];
    project_wave_item(P.wave_type[it], dim, eu, src, [&](int j, double v) { dst[st + j] = v; });
  }
  for (long base = (long)gw * 64; base < P.n_lane; base += (long)gwaves * 64) {
    const long it = base + lane;
    if (it < P.n_lane) {
      const long st = P.lane_start[it];
      auto src = make(st);
      const bool eu = force_euclid || P.lane_euclid[it];
      double r0 = src.r(0), r1 = src.r(1), r2 = src.r(2);
      double m0 = 1.0, m1 = 1.0, m2 = 1.0;
      if (!eu) { m0 = src.m(0); m1 = src.m(1); m2 = src.m(2); }
      double o[3];
      if (P.lane_type[it] == PDHCG_CONE_EXP) project_exp(r0, r1, r2, m0, m1, m2, o);
      else project_pow(r0, r1, r2, P.lane_alpha[it], m0, m1, m2, o);
      dst[st] = o[0];
      dst[st + 1] = o[1];
      dst[st + 2] = o[2];
    }
  }
  __threadfence_block();
}

// wave-uniform iteration over the coordinates of every cone item of this wave:
// f(i, active) with i a global coordinate
template <class F>
__device__ void for_cone_coords(const DevProblem& P, int gw, int gwaves, F f) {
  const int lane = threadIdx.x & 63;
  for (int it = gw; it < P.n_wave; it += gwaves) {
    const long st = P.wave_start[it];
    const int dim = P.wave_dim[it];
    for (int jb = 0; jb < dim; jb += 64) {
      const int j = jb + lane;
      f(st + j, j < dim);
    }
  }
  for (long base = (long)gw * 64; base < P.n_lane; base += (long)gwaves * 64) {
    const long it = base + lane;
    const bool act = it < P.n_lane;
    const long st = act ? P.lane_start[it] : 0;
    for (int j = 0; j < 3; ++j) f(st + j, act);
  }
}

// wave-uniform iteration over elementwise coordinates
template <class F>
__device__ void for_elem_coords(const DevProblem& P, int gw, int gwaves, F f) {
  const int lane = threadIdx.x & 63;
  for (long base = (long)gw * 64; base < P.n; base += (long)gwaves * 64) {
    const long i = base + lane;
    const bool act = i < P.n && P.ctype[i] != CT_CONE;
    f(i, act);
  }
}

// wave-uniform iteration over rows with Lw lanes per row
template <class F>
__device__ void for_rows(long nrows, int Lw, int gw, int gwaves, F f) {
  const int lane = threadIdx.x & 63;
  const int per = 64 / Lw;
  for (long base = (long)gw * per; base < nrows; base += (long)gwaves * per) {
    const long row = base + lane / Lw;
    f(row, lane & (Lw - 1), row < nrows);
  }
}

// ---------------------------------------------------------------------------
// the kernel
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void solve_kernel(KArgs A) {
  __shared__ Lds L;
  const DevProblem& P = A.P;
  const DevVec& V = A.V;
  const DevSettings& S = A.S;
  const int tid = threadIdx.x, lane = tid & 63, wv = tid >> 6;
  const int rank = blockIdx.x, G = gridDim.x;
  const int gw = rank * NWAVE + wv, gwaves = G * NWAVE;
  const long n = P.n, m = P.m;
  const int r = P.r;
  const unsigned long long lim = A.spin_limit;
  double* part = V.partials;

  if (tid == 0) L.C = *A.ctl;
  __syncthreads();
  if (L.C.status != 0) return;

#define SYNC_OR_EXIT()                         \
  do {                                         \
    if (!grid_sync(A.bar, G, L, lim)) {        \
      if (rank == 0 && tid == 0) {             \
        L.C.status = PDHCG_ABORTED;            \
        *A.ctl = L.C;                          \
      }                                        \
      return;                                  \
    }                                          \
  } while (0)

  const bool has_cones = (P.n_wave + P.n_lane) > 0;
  const MetricQ unitM{P.qd, 1.0, 0.0, 1};

  // ------------------------------------------------------------------ init
  if (!L.C.started) {
    // x = Pi_K(x0^) (zb holds the scaled warm start or zeros); a_x = x
    hw_clear(L, r);
    for_elem_coords(P, gw, gwaves, [&](long i, bool act) {
      double x = act ? elem_proj(P.ctype[i], V.zb[i]) : 0.0;
      if (act) { V.x[i] = x; V.ax[i] = x; }
      hw_add(L, P.R, (int)n, r, i, x, act);
    });
    project_cone_items(P, gw, gwaves, true,
                       [&](long st) { return BufSrc{V.zb, unitM, st}; }, V.zb);
    for_cone_coords(P, gw, gwaves, [&](long i, bool act) {
      double x = act ? V.zb[i] : 0.0;
      if (act) { V.x[i] = x; V.ax[i] = x; }
      hw_add(L, P.R, (int)n, r, i, x, act);
    });
    hw_store(L, r, part, G, rank);
    SYNC_OR_EXIT();
    // A x, a_y = y
    for_rows(m, P.a_lanes, gw, gwaves, [&](long row, int sub, bool act) {
      double ax = spmv_row(P.A_ptr, P.A_col, P.A_val, V.x, row, sub, P.a_lanes, act);
      if (act && sub == 0) { V.Ax[row] = ax; V.Aa[row] = ax; V.ay[row] = V.y[row]; }
    });
    team_reduce_h(L, part, G, r, L.C.hx);
    if (tid == 0) {
      L.C.started = 1;
      L.C.omega = P.omega0;
      L.C.eps_in = S.eps_in0;
      L.C.k = 0;
      L.C.ktot = 0;
      L.C.inner_total = 0;
      L.C.restarts = 0;
      L.C.pid_I = 0.0;
      L.C.e_prev = 0.0;
      L.C.E0 = L.C.Eprev = L.C.lastE = 0.0;
    }
    __syncthreads();
    SYNC_OR_EXIT();
  }

  const bool jac = S.inner == PDHCG_INNER_JACOBI;
  const double rho = S.rho;

  while (L.C.ktot < A.stop_at && L.C.status == 0) {
    const double omega = L.C.omega;
    const double tau = P.eta / omega, sigma = P.eta * omega;
    const long long k = L.C.k;
    const long long kt1 = L.C.ktot + 1;
    const bool check = (k == 0) || (kt1 % S.check_every == 0) || (kt1 >= S.max_iter);
    const double eps_in = L.C.eps_in;
    const bool tracing = A.T.cap > 0 && L.C.ktot < A.T.cap;
    double* W = P.q_diag ? V.wx : V.u;   // the primal candidate w_x
    // metric of the prox: diagonal Q -> 1 + tau q; Jacobi -> q + 1/tau
    const MetricQ Mq = P.q_diag ? MetricQ{P.qd, 1.0, tau, 0}
                                : (jac ? MetricQ{P.qd, 1.0 / tau, 1.0, 0} : unitM);
    const double alpha0 = jac ? 1.0 : 1.0 / (A.qmax + 1.0 / tau);

    if (tracing) {
      const long kk = L.C.ktot;
      for (long i = (long)rank * BLOCK + tid; i < n; i += (long)G * BLOCK) A.T.x[kk * n + i] = V.x[i];
      for (long i = (long)rank * BLOCK + tid; i < m; i += (long)G * BLOCK) A.T.y[kk * m + i] = V.y[i];
    }

    // -------------------------------------------------------------- P1
    if (!P.q_diag) make_ht(L, P, L.C.hx);
    {
      double d2 = 0.0;
      if (!P.q_diag) hw_clear(L, r);
      const int La = P.at_lanes;
      for_rows(n, La, gw, gwaves, [&](long i, int sub, bool act) {
        const double aty = spmv_row(P.AT_ptr, P.AT_col, P.AT_val, V.y, i, sub, La, act);
        double xi = act ? V.x[i] : 0.0;
        const double vi = xi + tau * aty;
        if (P.q_diag) {
          if (act && sub == 0) {
            const double mi = 1.0 + tau * P.qd[i];
            const double z = (vi - tau * P.c[i]) / mi;
            if (P.ctype[i] != CT_CONE) V.wx[i] = elem_proj(P.ctype[i], z);
            else V.zb[i] = z;
          }
        } else {
          double pu = 0.0;
          if (P.P_ptr) pu = spmv_row(P.P_ptr, P.P_col, P.P_val, V.x, i, sub, La, act);
          double un = 0.0;
          bool el = false;
          if (act && sub == 0) {
            double ru = 0.0;
            for (int kk = 0; kk < r; ++kk) ru += P.R[(size_t)kk * n + i] * L.ht[kk];
            const double g0 = pu + ru + P.c[i] + (xi - vi) / tau;
            const double di = Mq(i);
            const double z = xi - alpha0 * g0 / di;
            V.v[i] = vi;
            V.gp[i] = g0;
            V.up[i] = xi;
            if (P.ctype[i] != CT_CONE) {
              el = true;
              un = elem_proj(P.ctype[i], z);
              V.u[i] = un;
              d2 += (un - xi) * (un - xi);
            } else {
              V.zb[i] = z;
            }
          }
          hw_add(L, P.R, (int)n, r, i, un, el);
        }
      });
      if (!P.q_diag) {
        const int sl[1] = {SL_DELTA2};
        block_store(L, &d2, sl, 1, part, G, rank);
        hw_store(L, r, part, G, rank);
      }
    }
    SYNC_OR_EXIT();

    // -------------------------------------------------------------- P2
    if (has_cones) {
      if (P.q_diag) {
        project_cone_items(P, gw, gwaves, false,
                           [&](long st) { return BufSrc{V.zb, Mq, st}; }, V.wx);
      } else {
        double d2 = 0.0;
        hw_clear(L, r);
        project_cone_items(P, gw, gwaves, !jac,
                           [&](long st) { return BufSrc{V.zb, Mq, st}; }, V.zb);
        for_cone_coords(P, gw, gwaves, [&](long i, bool act) {
          double un = 0.0;
          if (act) {
            un = V.zb[i];
            V.u[i] = un;
            const double dd = un - V.up[i];
            d2 += dd * dd;
          }
          hw_add(L, P.R, (int)n, r, i, un, act);
        });
        // add to the P1 partials of this workgroup (same slots)
        {
          const int sl[1] = {SL_QMAX};
          block_store(L, &d2, sl, 1, part, G, rank);
          __syncthreads();
          if (tid == 0) part[(size_t)SL_DELTA2 * G + rank] += part[(size_t)SL_QMAX * G + rank];
          __syncthreads();
          if ((int)tid < r) {
            double s = 0.0;
            for (int w = 0; w < NWAVE; ++w) s += L.hw[w][tid];
            part[(size_t)(SL_H0 + tid) * G + rank] += s;
          }
          __syncthreads();
        }
      }
      SYNC_OR_EXIT();
    }

    // -------------------------------------------------------------- inner loop
    int jcount = 0;
    if (!P.q_diag) {
      {
        const int sl[1] = {SL_DELTA2};
        team_reduce(L, part, G, sl, 1);
        team_reduce_h(L, part, G, r, L.hu);
      }
      jcount = 1;
      bool done = (S.fixed_inner <= 0) && (sqrt(L.scal[SL_DELTA2]) <= eps_in);
      const int jmax = S.fixed_inner > 0 ? S.fixed_inner : S.j_max;
      while (!done && jcount < jmax) {
        // ---- P3: gradient at u, BB reductions
        make_ht(L, P, L.hu);
        double acc[3] = {0.0, 0.0, 0.0};
        const int La = P.at_lanes;
        for_rows(n, La, gw, gwaves, [&](long i, int sub, bool act) {
          double pu = 0.0;
          if (P.P_ptr) pu = spmv_row(P.P_ptr, P.P_col, P.P_val, V.u, i, sub, La, act);
          if (act && sub == 0) {
            double ru = 0.0;
            for (int kk = 0; kk < r; ++kk) ru += P.R[(size_t)kk * n + i] * L.ht[kk];
            const double ui = V.u[i];
            const double gc = pu + ru + P.c[i] + (ui - V.v[i]) / tau;
            const double si = ui - V.up[i];
            const double dg = gc - V.gp[i];
            const double di = Mq(i);
            acc[0] += si * (di * si);
            acc[1] += si * dg;
            acc[2] += si * si;
            V.g[i] = gc;
          }
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
        const double alpha = den > 0.0 ? num / den : 1.0;
        // ---- P4: projected step
        double d2 = 0.0;
        hw_clear(L, r);
        for_elem_coords(P, gw, gwaves, [&](long i, bool act) {
          double un = 0.0;
          if (act) {
            const double ui = V.u[i];
            const double gi = V.g[i];
            un = elem_proj(P.ctype[i], ui - alpha * gi / Mq(i));
            d2 += (un - ui) * (un - ui);
            V.up[i] = ui;
            V.gp[i] = gi;
            V.u[i] = un;
          }
          hw_add(L, P.R, (int)n, r, i, un, act);
        });
        if (has_cones) {
          project_cone_items(P, gw, gwaves, !jac,
                             [&](long st) { return StepSrc{V.u, V.g, Mq, alpha, st}; }, V.zb);
          for_cone_coords(P, gw, gwaves, [&](long i, bool act) {
            double un = 0.0;
            if (act) {
              un = V.zb[i];
              const double ui = V.u[i];
              d2 += (un - ui) * (un - ui);
              V.up[i] = ui;
              V.gp[i] = V.g[i];
              V.u[i] = un;
            }
            hw_add(L, P.R, (int)n, r, i, un, act);
          });
        }
        {
          const int sl[1] = {SL_DELTA2};
          block_store(L, &d2, sl, 1, part, G, rank);
          hw_store(L, r, part, G, rank);
        }
        SYNC_OR_EXIT();
        {
          const int sl[1] = {SL_DELTA2};
          team_reduce(L, part, G, sl, 1);
          team_reduce_h(L, part, G, r, L.hu);
        }
        ++jcount;
        done = (S.fixed_inner <= 0) && (sqrt(L.scal[SL_DELTA2]) <= eps_in);
      }
    }

    // -------------------------------------------------------------- P6
    const double c1 = (double)(k + 1) / (double)(k + 2);
    const double c3 = 1.0 / (double)(k + 2);
    {
      double acc[8] = {0, 0, 0, 0, 0, 0, 0, 0};
      // rows: A w_x, dual candidate
      const int La = P.a_lanes;
      for_rows(m, La, gw, gwaves, [&](long l, int sub, bool act) {
        const double aw = spmv_row(P.A_ptr, P.A_col, P.A_val, W, l, sub, La, act);
        if (act && sub == 0) {
          const double yl = V.y[l], axl = V.Ax[l];
          const double wy = yl + sigma * (P.b[l] - (2.0 * aw - axl));
          V.wy[l] = wy;
          V.Aw[l] = aw;
          if (tracing) A.T.wy[L.C.ktot * m + l] = wy;
          if (check) {
            const double dy = yl - wy;
            acc[0] += dy * dy;                           // SL_DY2
            acc[1] += (axl - aw) * dy;                   // SL_ADXDY
            const double rp = P.nu_b * (aw - P.b[l]) / P.Sy[l];
            acc[2] += rp * rp;                           // SL_RP2
            acc[3] += P.b[l] * wy;                       // SL_BY
            const double my = wy - V.ay[l];
            acc[4] += my * my;                           // SL_MOVY2
          } else {
            V.y[l] = c1 * (2.0 * rho * wy + (1.0 - 2.0 * rho) * yl) + c3 * V.ay[l];
            V.Ax[l] = c1 * (2.0 * rho * aw + (1.0 - 2.0 * rho) * axl) + c3 * V.Aa[l];
          }
        }
      });
      // coordinates
      if (!check) hw_clear(L, r);
      for (long base = (long)gw * 64; base < n; base += (long)gwaves * 64) {
        const long i = base + lane;
        const bool act = i < n;
        double xn = 0.0;
        if (act) {
          const double xi = V.x[i], wi = W[i];
          if (tracing) A.T.wx[L.C.ktot * n + i] = wi;
          if (check) {
            const double dx = xi - wi;
            acc[5] += dx * dx;                           // SL_DX2
            const double mx = wi - V.ax[i];
            acc[6] += mx * mx;                           // SL_MOVX2
            acc[7] += P.c[i] * wi;                       // SL_CX
          } else {
            xn = c1 * (2.0 * rho * wi + (1.0 - 2.0 * rho) * xi) + c3 * V.ax[i];
            acc[5] += (xn - xi) * (xn - xi);             // SL_XMOV2 (stored below)
            V.x[i] = xn;
          }
        }
        if (!check) hw_add(L, P.R, (int)n, r, i, xn, act);
      }
      if (check) {
        const int sl[8] = {SL_DY2, SL_ADXDY, SL_RP2, SL_BY, SL_MOVY2, SL_DX2, SL_MOVX2, SL_CX};
        block_store(L, acc, sl, 8, part, G, rank);
      } else {
        const int sl[1] = {SL_XMOV2};
        block_store(L, &acc[5], sl, 1, part, G, rank);
        hw_store(L, r, part, G, rank);
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
        team_reduce(L, part, G, sl, 1);
        team_reduce_h(L, part, G, r, L.C.hx);
      }
      if (tid == 0) {
        L.C.eps_in = fmin(L.C.eps_in, fmax(S.gamma_in * sqrt(L.scal[SL_XMOV2]) / tau, S.eps_min));
        L.C.k = k + 1;
      }
      __syncthreads();
      if (tracing && rank == 0 && tid == 0) {
        double* sc = A.T.sc + (L.C.ktot - 1) * 8;
        sc[0] = tau; sc[1] = sigma; sc[2] = omega; sc[3] = eps_in;
        sc[4] = jcount; sc[5] = 0.0; sc[6] = 0.0; sc[7] = 0.0;
      }
      continue;
    }

    // ---------------------------------------------------------- check
    {
      const int sl[8] = {SL_DY2, SL_ADXDY, SL_RP2, SL_BY, SL_MOVY2, SL_DX2, SL_MOVX2, SL_CX};
      team_reduce(L, part, G, sl, 8);
    }
    // R^ w_x: for the Jacobi path it is the last inner R^ u; diagonal Q has r = 0
    // C1: dual slack s = Q w + c - A^T w_y
    {
      if (!P.q_diag) make_ht(L, P, L.hu);
      double acc[2] = {0.0, 0.0};
      const int La = P.at_lanes;
      for_rows(n, La, gw, gwaves, [&](long i, int sub, bool act) {
        const double aty = spmv_row(P.AT_ptr, P.AT_col, P.AT_val, V.wy, i, sub, La, act);
        double qw = 0.0;
        if (P.q_diag) {
          if (act) qw = P.qd[i] * W[i];
        } else {
          if (P.P_ptr) qw = spmv_row(P.P_ptr, P.P_col, P.P_val, W, i, sub, La, act);
          if (act) for (int kk = 0; kk < r; ++kk) qw += P.R[(size_t)kk * n + i] * L.ht[kk];
        }
        if (act && sub == 0) {
          const double wi = W[i];
          const double si = qw + P.c[i] - aty;
          acc[0] += wi * qw;                               // SL_XQX
          const double so = P.nu_c * P.Sx[i] * si;
          const uint8_t ct = P.ctype[i];
          if (ct == CT_FREE) acc[1] += so * so;
          else if (ct == CT_NONNEG) { const double t = fmax(-so, 0.0); acc[1] += t * t; }
          else V.s[i] = si;
        }
      });
      const int sl[2] = {SL_XQX, SL_RD2};
      block_store(L, acc, sl, 2, part, G, rank);
    }
    SYNC_OR_EXIT();
    if (has_cones) {
      double rd = 0.0;
      project_cone_items(P, gw, gwaves, true, [&](long st) { return NegSrc{V.s, st}; }, V.zb);
      for_cone_coords(P, gw, gwaves, [&](long i, bool act) {
        if (act) {
          const double f = P.nu_c * P.Sx[i] * V.zb[i];
          rd += f * f;
        }
      });
      const int sl[1] = {SL_QMAX};
      block_store(L, &rd, sl, 1, part, G, rank);
      SYNC_OR_EXIT();
    }
    {
      int sl[3] = {SL_XQX, SL_RD2, SL_QMAX};
      team_reduce(L, part, G, sl, has_cones ? 3 : 2);
    }
    bool restart = false;
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
      const double rd2 = sc[SL_RD2] + (has_cones ? sc[SL_QMAX] : 0.0);
      const double scale = P.nu_b * P.nu_c;
      C.rel_p = sqrt(sc[SL_RP2]) / (1.0 + P.norm_b);
      C.rel_d = sqrt(rd2) / (1.0 + P.norm_c);
      C.pobj = scale * (0.5 * sc[SL_XQX] + sc[SL_CX]);
      C.dobj = scale * (sc[SL_BY] - 0.5 * sc[SL_XQX]);
      C.rel_gap = fabs(C.pobj - C.dobj) / (1.0 + fabs(C.pobj) + fabs(C.dobj));
      if (!isfinite(E) || !isfinite(C.rel_p) || !isfinite(C.rel_d) || !isfinite(C.rel_gap)) {
        C.status = PDHCG_NUMERICAL;
      } else if (fmax(C.rel_p, fmax(C.rel_d, C.rel_gap)) <= S.tol) {
        C.status = PDHCG_OPTIMAL;
      }
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
        double* t = A.T.sc + (kt1 - 1) * 8;
        t[0] = tau; t[1] = sigma; t[2] = omega; t[3] = eps_in;
        t[4] = jcount; t[5] = rs ? 1.0 : 0.0; t[6] = 1.0; t[7] = E;
      }
    }
    __syncthreads();
    restart = L.done != 0;
    if (L.C.status != 0) break;

    // ---------------------------------------------------------- restart or Halpern
    {
      double xm = 0.0;
      if (!restart) hw_clear(L, r);
      for_rows(m, 1, gw, gwaves, [&](long l, int sub, bool act) {
        if (!act) return;
        const double wy = V.wy[l], aw = V.Aw[l];
        if (restart) {
          V.y[l] = wy; V.ay[l] = wy; V.Ax[l] = aw; V.Aa[l] = aw;
        } else {
          V.y[l] = c1 * (2.0 * rho * wy + (1.0 - 2.0 * rho) * V.y[l]) + c3 * V.ay[l];
          V.Ax[l] = c1 * (2.0 * rho * aw + (1.0 - 2.0 * rho) * V.Ax[l]) + c3 * V.Aa[l];
        }
      });
      for (long base = (long)gw * 64; base < n; base += (long)gwaves * 64) {
        const long i = base + lane;
        const bool act = i < n;
        double xn = 0.0;
        if (act) {
          const double wi = W[i];
          if (restart) {
            V.x[i] = wi; V.ax[i] = wi;
          } else {
            const double xi = V.x[i];
            xn = c1 * (2.0 * rho * wi + (1.0 - 2.0 * rho) * xi) + c3 * V.ax[i];
            xm += (xn - xi) * (xn - xi);
            V.x[i] = xn;
          }
        }
        if (!restart) hw_add(L, P.R, (int)n, r, i, xn, act);
      }
      if (!restart) {
        const int sl[1] = {SL_XMOV2};
        block_store(L, &xm, sl, 1, part, G, rank);
        hw_store(L, r, part, G, rank);
      }
    }
    SYNC_OR_EXIT();
    if (restart) {
      if ((int)tid < r) L.C.hx[tid] = L.hu[tid];
      __syncthreads();
    } else {
      {
        const int sl[1] = {SL_XMOV2};
        team_reduce(L, part, G, sl, 1);
        team_reduce_h(L, part, G, r, L.C.hx);
      }
      if (tid == 0) {
        L.C.eps_in = fmin(L.C.eps_in, fmax(S.gamma_in * sqrt(L.scal[SL_XMOV2]) / tau, S.eps_min));
        L.C.k = k + 1;
      }
      __syncthreads();
    }
  }
  if (rank == 0 && tid == 0) *A.ctl = L.C;
#undef SYNC_OR_EXIT
}

// ---------------------------------------------------------------------------
// setup kernels: CSR SpMV and deterministic two-pass norms (power iteration)
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(BLOCK) void spmv_kernel(const int64_t* ptr, const int* col,
                                                     const double* val, const double* x,
                                                     double* y, long rows, int Lw) {
  const int lane = threadIdx.x & 63, wv = threadIdx.x >> 6;
  const int gw = blockIdx.x * NWAVE + wv, gwaves = gridDim.x * NWAVE;
  for_rows(rows, Lw, gw, gwaves, [&](long row, int sub, bool act) {
    double s = spmv_row(ptr, col, val, x, row, sub, Lw, act);
    if (act && sub == 0) y[row] = s;
  });
  (void)lane;
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

// out[0] = sqrt(sum part); x2 = x / out[0] (if scale_out)
__global__ __launch_bounds__(BLOCK) void finish_norm_kernel(const double* part, int np, double* out) {
  double s = 0.0;
  for (int j = threadIdx.x; j < np; j += 64) s += part[j];
  if (threadIdx.x < 64) {
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
// host wrappers
// ---------------------------------------------------------------------------
int block_size() { return BLOCK; }

hipError_t launch_solve(const KArgs& args, int grid, hipStream_t stream) {
  KArgs a = args;
  void* params[] = {&a};
  return hipLaunchCooperativeKernel((const void*)solve_kernel, dim3(grid), dim3(BLOCK), params, 0,
                                    stream);
}

hipError_t max_coop_grid(int* out) {
  int dev = 0, ncu = 0, per = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  e = hipDeviceGetAttribute(&ncu, hipDeviceAttributeMultiprocessorCount, dev);
  if (e != hipSuccess) return e;
  e = hipOccupancyMaxActiveBlocksPerMultiprocessor(&per, (const void*)solve_kernel, BLOCK, 0);
  if (e != hipSuccess) return e;
  *out = per * ncu;
  return hipSuccess;
}

hipError_t launch_spmv(const int64_t* ptr, const int* col, const double* val, const double* x,
                       double* y, long rows, int Lw, hipStream_t st) {
  if (rows <= 0) return hipSuccess;
  long per = 64 / Lw * NWAVE;
  long grid = (rows + per - 1) / per;
  if (grid > 4096) grid = 4096;
  hipLaunchKernelGGL(spmv_kernel, dim3((unsigned)grid), dim3(BLOCK), 0, st, ptr, col, val, x, y,
                     rows, Lw);
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

}  // namespace pdhcg
