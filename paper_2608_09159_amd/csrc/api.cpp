// C ABI of the solver: handle management, uploads, the host driver loop.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstdlib>
#include <cstring>
#include <new>
#include <vector>

#include "common.hpp"
#include "host_setup.hpp"
#include "pdhcg.h"
#include "solver.hpp"

using namespace pdhcg;

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

struct DevBuf {
  std::vector<void*> ptrs;
  hipError_t err = hipSuccess;
  template <class T>
  T* alloc(size_t count) {
    if (err != hipSuccess) return nullptr;
    void* p = nullptr;
    size_t bytes = std::max<size_t>(count, 1) * sizeof(T);
    err = hipMalloc(&p, bytes);
    if (err != hipSuccess) return nullptr;
    ptrs.push_back(p);
    return (T*)p;
  }
  template <class T>
  T* upload(const std::vector<T>& v) {
    T* p = alloc<T>(v.size());
    if (p && !v.empty()) err = hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
    return p;
  }
  void release() {
    for (void* p : ptrs) (void)hipFree(p);
    ptrs.clear();
  }
};

struct Instance {
  HostInstance H;
  DevBuf mem;
  DevProblem P{};
  DevVec V{};
  Ctl* ctl = nullptr;
  Barrier* bar = nullptr;
  TraceBufs T{};
  double* scratch = nullptr;   // power iteration scratch
  double qmax = 0.0;
  int grid = 1;
  size_t bar_bytes = 0;
  long n_warm = 0;
};

struct Handle {
  pdhcg_settings s;
  DevSettings ds;
  std::vector<Instance*> inst;
  hipStream_t stream = nullptr;
  double setup_s = 0.0;
  unsigned long long spin_limit = 0;
};

int pow2_floor(double v) {
  int L = 1;
  while (L * 2 <= v && L < 64) L *= 2;
  return L;
}

#define HIPCHK(expr)                          \
  do {                                        \
    hipError_t _e = (expr);                   \
    if (_e != hipSuccess) {                   \
      if (h->s.verbose) std::fprintf(stderr, "pdhcg: %s failed: %s\n", #expr, hipGetErrorString(_e)); \
      return PDHCG_E_HIP;                     \
    }                                         \
  } while (0)

DevSettings to_dev(const pdhcg_settings& s) {
  DevSettings d{};
  d.tol = s.tol;
  d.max_iter = s.max_iter;
  d.check_every = s.check_every;
  d.scheme = s.scheme;
  d.rho = s.rho;
  d.avg_epoch = s.avg_epoch;
  d.inner = s.inner;
  d.fixed_inner = s.fixed_inner;
  d.j_max = s.j_max;
  d.eps_in0 = s.eps_in0;
  d.gamma_in = s.gamma_in;
  d.eps_min = s.eps_min;
  d.beta_s = s.beta_s;
  d.beta_n = s.beta_n;
  d.beta_a = s.beta_a;
  d.pid_beta_i = s.pid_beta_i;
  d.pid_kp = s.pid_kp;
  d.pid_ki = s.pid_ki;
  d.pid_kd = s.pid_kd;
  d.trace_iters = s.trace_iters;
  return d;
}

int upload_instance(Handle* h, Instance* I) {
  const HostInstance& H = I->H;
  DevBuf& B = I->mem;
  DevProblem& P = I->P;
  const long n = H.n, m = H.m;
  P.n = H.n;
  P.m = H.m;
  P.r = H.r;
  // lanes per row from the mean row length (power of two <= mean, 1..64)
  double mean_at = n > 0 ? (double)H.AT.nnz() / n : 1.0;
  double mean_p = (H.P.rows > 0 && n > 0) ? (double)H.P.nnz() / n : 0.0;
  double mean_a = m > 0 ? (double)H.A.nnz() / m : 1.0;
  P.at_lanes = h->s.lanes_at > 0 ? h->s.lanes_at : pow2_floor(std::max(mean_at, mean_p));
  P.a_lanes = h->s.lanes_a > 0 ? h->s.lanes_a : pow2_floor(mean_a);
  P.A_ptr = B.upload(H.A.ptr);
  P.A_col = B.upload(H.A.col);
  P.A_val = B.upload(H.A.val);
  P.AT_ptr = B.upload(H.AT.ptr);
  P.AT_col = B.upload(H.AT.col);
  P.AT_val = B.upload(H.AT.val);
  if (H.P.rows > 0) {
    P.P_ptr = B.upload(H.P.ptr);
    P.P_col = B.upload(H.P.col);
    P.P_val = B.upload(H.P.val);
  } else {
    P.P_ptr = nullptr;
    P.P_col = nullptr;
    P.P_val = nullptr;
  }
  P.R = H.r > 0 ? B.upload(H.R) : nullptr;
  P.Dm = H.r > 0 ? B.upload(H.D) : nullptr;
  P.b = B.upload(H.b);
  P.c = B.upload(H.c);
  P.qd = B.upload(H.qdiag);
  P.Sx = B.upload(H.Sx);
  P.Sy = B.upload(H.Sy);
  P.ctype = B.upload(H.ctype);
  P.n_wave = (int)H.wave_start.size();
  P.n_lane = (int)H.lane_start.size();
  P.wave_start = B.upload(H.wave_start);
  P.wave_dim = B.upload(H.wave_dim);
  P.wave_type = B.upload(H.wave_type);
  P.wave_euclid = B.upload(H.wave_euclid);
  P.lane_start = B.upload(H.lane_start);
  P.lane_type = B.upload(H.lane_type);
  P.lane_alpha = B.upload(H.lane_alpha);
  P.lane_euclid = B.upload(H.lane_euclid);
  P.nu_b = H.nu_b;
  P.nu_c = H.nu_c;
  P.norm_b = H.norm_b;
  P.norm_c = H.norm_c;
  P.q_diag = H.q_diag ? 1 : 0;
  I->qmax = 0.0;
  for (double q : H.qdiag) I->qmax = std::max(I->qmax, q);

  DevVec& V = I->V;
  V.x = B.alloc<double>(n);
  V.y = B.alloc<double>(m);
  V.ax = B.alloc<double>(n);
  V.ay = B.alloc<double>(m);
  V.wx = B.alloc<double>(n);
  V.wy = B.alloc<double>(m);
  V.Ax = B.alloc<double>(m);
  V.Aa = B.alloc<double>(m);
  V.Aw = B.alloc<double>(m);
  V.v = B.alloc<double>(n);
  V.u = B.alloc<double>(n);
  V.up = B.alloc<double>(n);
  V.g = B.alloc<double>(n);
  V.gp = B.alloc<double>(n);
  V.zb = B.alloc<double>(n);
  V.s = B.alloc<double>(n);
  V.t1 = B.alloc<double>(n);
  V.t2 = B.alloc<double>(n);
  I->n_warm = 2L * ((long)H.wave_start.size() + (long)H.lane_start.size());
  V.warm = B.alloc<double>(I->n_warm);
  V.xb = V.yb = V.Axb = nullptr;
  I->scratch = B.alloc<double>(2048 + 2);
  I->ctl = B.alloc<Ctl>(1);
  I->bar = nullptr;   // allocated with the grid size below
  if (h->s.trace_iters > 0) {
    long cap = h->s.trace_iters;
    I->T.cap = (int)cap;
    I->T.x = B.alloc<double>(cap * n);
    I->T.wx = B.alloc<double>(cap * n);
    I->T.y = B.alloc<double>(cap * std::max<long>(m, 1));
    I->T.wy = B.alloc<double>(cap * std::max<long>(m, 1));
    I->T.sc = B.alloc<double>(cap * 8);
  }
  if (B.err != hipSuccess) return B.err == hipErrorOutOfMemory ? PDHCG_E_MEM : PDHCG_E_HIP;

  // launch geometry
  int maxg = 1;
  HIPCHK(max_coop_grid(&maxg));
  int G = h->s.grid_dim;
  if (G <= 0) {
    long work = std::max<long>(std::max<long>(n, m), 1);
    long want = (work + (long)block_size() - 1) / (long)block_size();
    G = (int)std::min<long>(std::max<long>(want, 1), maxg);
  }
  G = std::max(1, std::min(G, maxg));
  I->grid = G;
  // ownership ranges: coordinates weighted by their share of the A^T and P
  // passes, the dense factor and the cone projections (cone blocks are never
  // split); rows by their nonzeros
  {
    std::vector<long> pc(G + 1, 0), pr(G + 1, 0);
    std::vector<int> pw(G + 1, 0), pl(G + 1, 0);
    auto split = [&](const std::vector<std::pair<long, double>>& units, long total_items,
                     std::vector<long>& out) {
      double total = 0.0;
      for (const auto& u : units) total += u.second;
      out[0] = 0;
      int kk = 1;
      double cum = 0.0;
      for (const auto& u : units) {
        cum += u.second;
        while (kk < G && cum >= total * kk / G) out[kk++] = u.first;   // u.first = end index
      }
      while (kk <= G) out[kk++] = total_items;
      out[G] = total_items;
    };
    std::vector<std::pair<long, double>> cu;
    cu.reserve(n);
    for (const auto& cb : H.cones) {
      auto wcoord = [&](long i) {
        double w = 2.0 + (double)(H.AT.ptr[i + 1] - H.AT.ptr[i]) + H.r;
        if (H.P.rows > 0) w += (double)(H.P.ptr[i + 1] - H.P.ptr[i]);
        return w;
      };
      if (cb.type == PDHCG_CONE_FREE || cb.type == PDHCG_CONE_NONNEG) {
        for (long i = cb.start; i < cb.start + cb.dim; ++i) cu.emplace_back(i + 1, wcoord(i));
      } else {
        double w = 0.0;
        for (long i = cb.start; i < cb.start + cb.dim; ++i) w += wcoord(i) + 16.0;
        if (cb.type == PDHCG_CONE_EXP || cb.type == PDHCG_CONE_POW) w += 400.0;
        cu.emplace_back((long)cb.start + cb.dim, w);
      }
    }
    split(cu, n, pc);
    std::vector<std::pair<long, double>> ru;
    ru.reserve(m);
    for (long l = 0; l < m; ++l) ru.emplace_back(l + 1, 2.0 + (double)(H.A.ptr[l + 1] - H.A.ptr[l]));
    split(ru, m, pr);
    for (int w = 0; w <= G; ++w) {
      pw[w] = (int)(std::lower_bound(H.wave_start.begin(), H.wave_start.end(), (int)std::min<long>(pc[w], n)) -
                    H.wave_start.begin());
      pl[w] = (int)(std::lower_bound(H.lane_start.begin(), H.lane_start.end(), (int)std::min<long>(pc[w], n)) -
                    H.lane_start.begin());
    }
    // lanes per row chosen per workgroup from its own rows (about two
    // nonzeros per lane), SOC/RSOC group width from its longest block
    std::vector<unsigned char> lanes(4 * (size_t)G, 1);
    auto pick = [](double mean) {
      int L = 1;
      while (L * 2 <= std::max(1.0, mean / 2.0) && L < 64) L *= 2;
      return L;
    };
    for (int w = 0; w < G; ++w) {
      long nr = pc[w + 1] - pc[w];
      double nz = 0.0;
      if (nr > 0) {
        nz = (double)(H.AT.ptr[pc[w + 1]] - H.AT.ptr[pc[w]]);
        if (H.P.rows > 0) nz = std::max(nz, (double)(H.P.ptr[pc[w + 1]] - H.P.ptr[pc[w]]));
      }
      lanes[4 * w + 0] = (unsigned char)(h->s.lanes_at > 0 ? h->s.lanes_at : pick(nr > 0 ? nz / nr : 1.0));
      long mr = pr[w + 1] - pr[w];
      double mz = mr > 0 ? (double)(H.A.ptr[pr[w + 1]] - H.A.ptr[pr[w]]) / mr : 1.0;
      lanes[4 * w + 1] = (unsigned char)(h->s.lanes_a > 0 ? h->s.lanes_a : pick(mz));
      int maxdim = 1;
      for (int it = pw[w]; it < pw[w + 1]; ++it) maxdim = std::max(maxdim, H.wave_dim[it]);
      lanes[4 * w + 2] = (unsigned char)(maxdim <= 17 ? 16 : (maxdim <= 33 ? 32 : 64));
    }
    P.part_c = B.upload(pc);
    P.part_r = B.upload(pr);
    P.part_w = B.upload(pw);
    P.part_l = B.upload(pl);
    P.part_lanes = B.upload(lanes);
  }
  V.partials = B.alloc<double>((size_t)SL_COUNT * G);
  I->bar_bytes = sizeof(Barrier) + sizeof(unsigned) * (size_t)G * BAR_STRIDE;
  I->bar = (Barrier*)B.alloc<char>(I->bar_bytes);
  if (B.err != hipSuccess) return PDHCG_E_MEM;
  return PDHCG_OK;
}

// ||A^||_2 by power iteration on A^T A from 1/sqrt(n) (fixed iteration count)
int power_norm(Handle* h, Instance* I, double* out) {
  const DevProblem& P = I->P;
  const long n = P.n, m = P.m;
  hipStream_t st = h->stream;
  double* z = I->V.v;
  double* t = I->V.Aw;
  double* w = I->V.g;
  double* part = I->scratch;
  double* nrm = I->scratch + 2048;
  HIPCHK(launch_fill(z, n, 1.0 / std::sqrt((double)n), st));
  double lam = 0.0;
  if (m == 0 || I->H.A.nnz() == 0) { *out = 0.0; return PDHCG_OK; }
  for (int it = 0; it < h->s.power_iters; ++it) {
    HIPCHK(launch_spmv(P.A_ptr, P.A_col, P.A_val, z, t, m, P.a_lanes, st));
    HIPCHK(launch_spmv(P.AT_ptr, P.AT_col, P.AT_val, t, w, n, P.at_lanes, st));
    HIPCHK(launch_norm(w, n, part, nrm, st));
    HIPCHK(hipMemcpyAsync(z, w, n * sizeof(double), hipMemcpyDeviceToDevice, st));
    HIPCHK(launch_scale(z, n, nrm, st));
  }
  HIPCHK(hipMemcpyAsync(&lam, nrm, sizeof(double), hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  *out = std::sqrt(lam);
  return PDHCG_OK;
}

void free_instance(Instance* I) {
  if (!I) return;
  I->mem.release();
  delete I;
}

}  // namespace

extern "C" {

int pdhcg_default_settings(pdhcg_settings* s) {
  if (!s) return PDHCG_E_ARG;
  std::memset(s, 0, sizeof(*s));
  s->tol = 1e-6;
  s->max_iter = 1000000;
  s->time_limit = 3600.0;
  s->check_every = 64;
  s->scheme = PDHCG_SCHEME_RH;
  s->rho = 1.0;
  s->avg_epoch = 64;
  s->inner = PDHCG_INNER_JACOBI;
  s->fixed_inner = 0;
  s->j_max = 500;
  s->eps_in0 = 1e-3;
  s->gamma_in = 5e-4;
  s->eps_min = 1e-9;
  s->beta_s = 0.2;
  s->beta_n = 0.8;
  s->beta_a = 0.36;
  s->pid_beta_i = 0.3;
  s->pid_kp = 0.99;
  s->pid_ki = 0.01;
  s->pid_kd = 0.0;
  s->scaling = 1;
  s->ruiz_iters = 10;
  s->pock_chambolle = 1;
  s->pc_alpha = 1.0;
  s->bound_objective = 1;
  s->power_iters = 128;
  s->a_norm = 0.0;
  s->omega0 = 0.0;
  s->precision = PDHCG_PREC_FP64;
  s->trace_iters = 0;
  s->host_poll = 512;
  s->stream = nullptr;
  s->verbose = 0;
  return PDHCG_OK;
}

const char* pdhcg_strerror(int code) {
  switch (code) {
    case PDHCG_OK: return "ok";
    case PDHCG_E_ARG: return "invalid argument";
    case PDHCG_E_SHAPE: return "invalid dimensions";
    case PDHCG_E_CSR: return "invalid CSR structure";
    case PDHCG_E_CONE: return "invalid cone partition";
    case PDHCG_E_NONSYM: return "P or D is not symmetric";
    case PDHCG_E_MEM: return "allocation failed";
    case PDHCG_E_HIP: return "HIP runtime error";
    case PDHCG_E_STATE: return "call not valid for this handle";
    case PDHCG_E_NOTRACE: return "no trace recorded";
    case PDHCG_OPTIMAL: return "optimal";
    case PDHCG_MAX_ITER: return "iteration limit";
    case PDHCG_TIME_LIMIT: return "time limit";
    case PDHCG_NUMERICAL: return "numerical failure";
    case PDHCG_ABORTED: return "device barrier timed out";
    default: return "unknown";
  }
}

const char* pdhcg_version(void) { return "pdhcg-mi355x 0.1 (gfx950, FP64)"; }

int pdhcg_setup(const pdhcg_problem* probs, int32_t count, const pdhcg_settings* s, void** out) {
  if (!out) return PDHCG_E_ARG;
  *out = nullptr;
  if (!probs || !s || count < 1) return PDHCG_E_ARG;
  if (count != 1) return PDHCG_E_ARG;   // batches: pdhcg_solve_batch
  if (s->tol <= 0 || s->check_every < 1 || s->j_max < 1 || s->max_iter < 0 ||
      !(s->rho >= 0.5 && s->rho <= 1.0) || s->power_iters < 0 || s->scheme != PDHCG_SCHEME_RH ||
      s->precision != PDHCG_PREC_FP64 || s->trace_iters < 0)
    return PDHCG_E_ARG;
  if (s->lanes_at < 0 || s->lanes_at > 64 || (s->lanes_at & (s->lanes_at - 1)) ||
      s->lanes_a < 0 || s->lanes_a > 64 || (s->lanes_a & (s->lanes_a - 1)))
    return PDHCG_E_ARG;
  double t0 = now_s();
  Handle* h = new (std::nothrow) Handle();
  if (!h) return PDHCG_E_MEM;
  h->s = *s;
  if (h->s.host_poll <= 0) h->s.host_poll = 512;
  h->ds = to_dev(h->s);
  h->stream = (hipStream_t)s->stream;
  // host-side validation and rescaling first: invalid input is reported
  // without touching the device
  for (int i = 0; i < count; ++i) {
    Instance* I = new (std::nothrow) Instance();
    if (!I) { pdhcg_free(h); return PDHCG_E_MEM; }
    h->inst.push_back(I);
    int rc = build_instance(probs[i], h->s, I->H);
    if (rc != PDHCG_OK) { pdhcg_free(h); return rc; }
  }
  int dev = 0, rate_khz = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess) {
    pdhcg_free(h);
    return PDHCG_E_HIP;
  }
  if (rate_khz <= 0) rate_khz = 100000;
  h->spin_limit = (unsigned long long)rate_khz * 1000ull * 4ull;   // 4 s
  for (int i = 0; i < count; ++i) {
    Instance* I = h->inst[i];
    int rc = upload_instance(h, I);
    if (rc != PDHCG_OK) { pdhcg_free(h); return rc; }
    double an = s->a_norm;
    if (!(an > 0)) {
      rc = power_norm(h, I, &an);
      if (rc != PDHCG_OK) { pdhcg_free(h); return rc; }
    }
    if (!(an > 0)) an = 1.0;   // A = 0 or no rows: the dual step is void
    I->P.eta = 0.998 / an;
    double nb = 0, nc = 0;
    for (double v : I->H.b) nb += v * v;
    for (double v : I->H.c) nc += v * v;
    nb = std::sqrt(nb);
    nc = std::sqrt(nc);
    I->P.omega0 = s->omega0 > 0 ? s->omega0 : ((nb > 1e-10 && nc > 1e-10) ? nc / nb : 1.0);
  }
  h->setup_s = now_s() - t0;
  *out = h;
  return PDHCG_OK;
}

int pdhcg_solve(void* hv, const double* x0, const double* y0, pdhcg_result* res) {
  Handle* h = (Handle*)hv;
  if (!h || !res) return PDHCG_E_ARG;
  if (h->inst.size() != 1) return PDHCG_E_STATE;
  Instance* I = h->inst[0];
  const HostInstance& H = I->H;
  const long n = H.n, m = H.m;
  hipStream_t st = h->stream;
  double t0 = now_s();
  // warm start in the scaled space: x^ = S_x x0 / nu_b, y^ = y0 / (nu_c S_y)
  std::vector<double> tmp;
  if (x0) {
    tmp.resize(n);
    for (long i = 0; i < n; ++i) tmp[i] = H.Sx[i] * x0[i] / H.nu_b;
    HIPCHK(hipMemcpyAsync(I->V.zb, tmp.data(), n * sizeof(double), hipMemcpyHostToDevice, st));
  } else {
    HIPCHK(launch_fill(I->V.zb, n, 0.0, st));
  }
  std::vector<double> tmpy;
  if (y0 && m > 0) {
    tmpy.resize(m);
    for (long l = 0; l < m; ++l) tmpy[l] = y0[l] / (H.nu_c * H.Sy[l]);
    HIPCHK(hipMemcpyAsync(I->V.y, tmpy.data(), m * sizeof(double), hipMemcpyHostToDevice, st));
  } else {
    HIPCHK(launch_fill(I->V.y, m, 0.0, st));
  }
  Ctl c0;
  std::memset(&c0, 0, sizeof(c0));
  HIPCHK(hipMemcpyAsync(I->ctl, &c0, sizeof(c0), hipMemcpyHostToDevice, st));
  HIPCHK(hipMemsetAsync(I->bar, 0, I->bar_bytes, st));
  HIPCHK(launch_fill(I->V.warm, I->n_warm, NAN, st));
  KArgs a{};
  a.P = I->P;
  a.V = I->V;
  a.S = h->ds;
  a.ctl = I->ctl;
  a.bar = I->bar;
  a.T = I->T;
  a.spin_limit = h->spin_limit;
  a.qmax = I->qmax;
  a.profile = h->s.verbose & 8 ? 1 : 0;
  unsigned long long* dpt = nullptr;
  if (a.profile) {
    HIPCHK(hipMalloc(&dpt, sizeof(unsigned long long) * PT_COUNT * I->grid));
    HIPCHK(hipMemsetAsync(dpt, 0, sizeof(unsigned long long) * PT_COUNT * I->grid, st));
  }
  a.ptimes = dpt;
  Ctl c = c0;
  int status = 0;
  const long long maxit = h->s.max_iter;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  const bool timing = h->s.time_kernels != 0;
  double ksum = 0.0;
  long long nlaunch = 0;
  if (timing) {
    HIPCHK(hipEventCreate(&ev0));
    HIPCHK(hipEventCreate(&ev1));
  }
  while (true) {
    a.stop_at = std::min<long long>(maxit, c.ktot + h->s.host_poll);
    if (timing) HIPCHK(hipEventRecord(ev0, st));
    HIPCHK(launch_solve(a, I->grid, st));
    if (timing) HIPCHK(hipEventRecord(ev1, st));
    HIPCHK(hipMemcpyAsync(&c, I->ctl, sizeof(c), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    ++nlaunch;
    if (timing) {
      float ms = 0.0f;
      HIPCHK(hipEventElapsedTime(&ms, ev0, ev1));
      ksum += ms * 1e-3;
    }
    if (c.status != 0) { status = c.status; break; }
    if (c.ktot >= maxit) { status = PDHCG_MAX_ITER; break; }
    if (now_s() - t0 > h->s.time_limit) { status = PDHCG_TIME_LIMIT; break; }
  }
  if (timing) {
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
  }
  res->kernel_s = ksum;
  res->kernel_launches = nlaunch;
  res->grid_dim = I->grid;
  res->block_dim = block_size();
  if (h->s.verbose & 8) {
    static const char* names[PT_COUNT] = {"init", "P1", "P2", "P3", "P4", "P6", "check",
                                          "halpern", "barrier", "proj", "wcall", "ncall"};
    int dev = 0, khz = 100000;
    (void)hipGetDevice(&dev);
    (void)hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
    std::vector<unsigned long long> pt((size_t)PT_COUNT * I->grid);
    (void)hipMemcpy(pt.data(), dpt, pt.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost);
    (void)hipFree(dpt);
    std::fprintf(stderr, "pdhcg phase times over %d workgroups (lanes at=%d a=%d): mean / max / argmax [ms]\n",
                 I->grid, I->P.at_lanes, I->P.a_lanes);
    for (int i = 0; i < PT_COUNT; ++i) {
      double s = 0, mx = 0;
      int am = 0;
      for (int w = 0; w < I->grid; ++w) {
        double v = pt[(size_t)w * PT_COUNT + i] / (double)khz;
        s += v;
        if (v > mx) { mx = v; am = w; }
      }
      std::fprintf(stderr, "  %-8s %10.3f %10.3f %5d\n", names[i], s / I->grid, mx, am);
    }
    if (const char* path = std::getenv("PDHCG_PROFILE_DUMP")) {
      if (FILE* f = std::fopen(path, "w")) {
        for (int w = 0; w < I->grid; ++w) {
          std::fprintf(f, "%d,%ld,%ld", w, (long)0, (long)0);
          for (int i = 0; i < PT_COUNT; ++i) std::fprintf(f, ",%.4f", pt[(size_t)w * PT_COUNT + i] / (double)khz);
          std::fprintf(f, "\n");
        }
        std::fclose(f);
      }
    }
  }
  // results (unscaled)
  const double* W = I->P.q_diag ? I->V.wx : I->V.u;
  std::vector<double> wx(n), wy(m);
  if (c.ktot > 0) {
    HIPCHK(hipMemcpyAsync(wx.data(), W, n * sizeof(double), hipMemcpyDeviceToHost, st));
    if (m > 0) HIPCHK(hipMemcpyAsync(wy.data(), I->V.wy, m * sizeof(double), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  res->status = status;
  res->iterations = c.ktot;
  res->inner_iterations = c.inner_total;
  res->restarts = c.restarts;
  res->rel_primal = c.rel_p;
  res->rel_dual = c.rel_d;
  res->rel_gap = c.rel_gap;
  res->primal_obj = c.pobj;
  res->dual_obj = c.dobj;
  res->omega = c.omega;
  res->a_norm = 0.998 / I->P.eta;
  res->setup_s = h->setup_s;
  if (res->x)
    for (long i = 0; i < n; ++i) res->x[i] = H.nu_b * wx[i] / H.Sx[i];
  if (res->y)
    for (long l = 0; l < m; ++l) res->y[l] = H.nu_c * H.Sy[l] * wy[l];
  if (res->s) {
    // s = nu_c S_x (Q^ w + c^ - A^T w_y)
    std::vector<double> q(n, 0.0);
    if (H.P.rows > 0)
      for (long i = 0; i < n; ++i)
        for (int64_t k = H.P.ptr[i]; k < H.P.ptr[i + 1]; ++k) q[i] += H.P.val[k] * wx[H.P.col[k]];
    if (H.r > 0) {
      std::vector<double> hh(H.r, 0.0), ht(H.r, 0.0);
      for (int k = 0; k < H.r; ++k)
        for (long i = 0; i < n; ++i) hh[k] += H.R[(size_t)k * n + i] * wx[i];
      for (int k = 0; k < H.r; ++k)
        for (int b = 0; b < H.r; ++b) ht[k] += H.D[k * H.r + b] * hh[b];
      for (long i = 0; i < n; ++i)
        for (int k = 0; k < H.r; ++k) q[i] += H.R[(size_t)k * n + i] * ht[k];
    }
    for (long i = 0; i < n; ++i) {
      double aty = 0.0;
      for (int64_t k = H.AT.ptr[i]; k < H.AT.ptr[i + 1]; ++k) aty += H.AT.val[k] * wy[H.AT.col[k]];
      res->s[i] = H.nu_c * H.Sx[i] * (q[i] + H.c[i] - aty);
    }
  }
  res->solve_s = now_s() - t0;
  return PDHCG_OK;
}

int pdhcg_solve_batch(void* hv, const double* const* x0s, const double* const* y0s, pdhcg_result* res) {
  (void)hv; (void)x0s; (void)y0s; (void)res;
  return PDHCG_E_STATE;
}

int pdhcg_get_trace(void* hv, int32_t inst, pdhcg_trace* t) {
  Handle* h = (Handle*)hv;
  if (!h || !t || inst < 0 || inst >= (int)h->inst.size()) return PDHCG_E_ARG;
  Instance* I = h->inst[inst];
  if (I->T.cap <= 0) return PDHCG_E_NOTRACE;
  Ctl c;
  if (hipMemcpy(&c, I->ctl, sizeof(c), hipMemcpyDeviceToHost) != hipSuccess) return PDHCG_E_HIP;
  long rec = std::min<long long>(c.ktot, I->T.cap);
  rec = std::min<long>(rec, t->count);
  const long n = I->H.n, m = I->H.m;
  auto cp = [&](double* dst, const double* src, size_t cnt) -> bool {
    if (!dst || cnt == 0) return true;
    return hipMemcpy(dst, src, cnt * sizeof(double), hipMemcpyDeviceToHost) == hipSuccess;
  };
  if (!cp(t->x, I->T.x, rec * n) || !cp(t->wx, I->T.wx, rec * n) || !cp(t->y, I->T.y, rec * m) ||
      !cp(t->wy, I->T.wy, rec * m))
    return PDHCG_E_HIP;
  std::vector<double> sc(rec * 8);
  if (!cp(sc.data(), I->T.sc, rec * 8)) return PDHCG_E_HIP;
  for (long k = 0; k < rec; ++k) {
    if (t->tau) t->tau[k] = sc[k * 8 + 0];
    if (t->sigma) t->sigma[k] = sc[k * 8 + 1];
    if (t->omega) t->omega[k] = sc[k * 8 + 2];
    if (t->eps_in) t->eps_in[k] = sc[k * 8 + 3];
    if (t->inner) t->inner[k] = (int32_t)sc[k * 8 + 4];
    if (t->restart) t->restart[k] = (int32_t)sc[k * 8 + 5];
    if (t->check) t->check[k] = (int32_t)sc[k * 8 + 6];
    if (t->E) t->E[k] = sc[k * 8 + 7];
  }
  t->count = (int32_t)rec;
  return PDHCG_OK;
}

int pdhcg_get_scaling(void* hv, int32_t inst, double* Sx, double* Sy, double* nu_b, double* nu_c,
                      double* eta, double* omega0) {
  Handle* h = (Handle*)hv;
  if (!h || inst < 0 || inst >= (int)h->inst.size()) return PDHCG_E_ARG;
  const Instance* I = h->inst[inst];
  if (Sx) std::copy(I->H.Sx.begin(), I->H.Sx.end(), Sx);
  if (Sy) std::copy(I->H.Sy.begin(), I->H.Sy.end(), Sy);
  if (nu_b) *nu_b = I->H.nu_b;
  if (nu_c) *nu_c = I->H.nu_c;
  if (eta) *eta = I->P.eta;
  if (omega0) *omega0 = I->P.omega0;
  return PDHCG_OK;
}

void pdhcg_free(void* hv) {
  Handle* h = (Handle*)hv;
  if (!h) return;
  for (Instance* I : h->inst) free_instance(I);
  delete h;
}

}  // extern "C"
