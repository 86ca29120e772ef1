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

// row bounds, box blocks, fixed-middle EXP blocks or the rescaled-cone
// mode: the kernel variant
// compiled with that code runs the instance
bool needs_ext(const HostInstance& H) {
  if (!H.rlo.empty() || !H.xlo.empty() || H.resc) return true;
  for (const ConeBlock& k : H.cones)
    if (k.type == PDHCG_CONE_EXP1) return true;
  return false;
}

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// device allocations of a handle: hipMalloc, or the caller's allocator
// (settings.dev_alloc / dev_free)
struct DevBuf {
  std::vector<void*> ptrs;
  hipError_t err = hipSuccess;
  pdhcg_alloc_fn fa = nullptr;
  pdhcg_free_fn ff = nullptr;
  void* ctx = nullptr;
  void* stream = nullptr;
  DevBuf() = default;
  DevBuf(const DevBuf&) = delete;
  DevBuf& operator=(const DevBuf&) = delete;
  ~DevBuf() { release(); }
  void use(const pdhcg_settings& s) {
    fa = s.dev_alloc;
    ff = s.dev_free;
    ctx = s.alloc_ctx;
    stream = s.stream;
  }
  void* raw(size_t bytes) {
    if (err != hipSuccess) return nullptr;
    void* p = nullptr;
    if (fa) {
      p = fa(bytes, stream, ctx);
      if (!p) err = hipErrorOutOfMemory;
    } else {
      err = hipMalloc(&p, bytes);
    }
    if (err != hipSuccess) return nullptr;
    ptrs.push_back(p);
    return p;
  }
  template <class T>
  T* alloc(size_t count) {
    return (T*)raw(std::max<size_t>(count, 1) * sizeof(T));
  }
  template <class T>
  T* upload(const std::vector<T>& v) {
    T* p = alloc<T>(v.size());
    if (p && !v.empty()) err = hipMemcpy(p, v.data(), v.size() * sizeof(T), hipMemcpyHostToDevice);
    return p;
  }
  void release() {
    for (void* p : ptrs) {
      if (ff) ff(p, stream, ctx);
      else (void)hipFree(p);
    }
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
  int lds_bytes = 0;           // dynamic LDS per workgroup for its slice of R
  int* at_cls_perm = nullptr;  // all A^T rows by length class (skewed rows; setup products)
  long at_cls_seg[6] = {0, 0, 0, 0, 0, 0};
  size_t bar_bytes = 0;
  long n_warm = 0;
  int* d_perm = nullptr;       // caller index of each internal coordinate (null: same order)
  double* io = nullptr;        // IO_DOUBLES of scratch for the dual-slack output
};

struct Batch;

}  // namespace

// the opaque handle of the C ABI
struct pdhcg_handle {
  pdhcg_settings s;
  DevSettings ds;
  std::vector<Instance*> inst;
  hipStream_t stream = nullptr;
  double setup_s = 0.0;
  unsigned long long spin_limit = 0;
  int rate_khz = 100000;
  Batch* B = nullptr;     // count > 1: the batch arena and its launch state
};

namespace {

using Handle = pdhcg_handle;

// Batch of independent instances.  All instance data lives in one device
// arena, each instance in a contiguous 256-byte aligned region; the
// descriptors (device pointers into the arena, step sizes, lane mapping) are
// an array the batch kernel indexes by instance.
struct Batch {
  int count = 0;
  DevBuf mem;
  char* arena = nullptr;
  std::vector<InstDesc> desc;
  InstDesc* d_desc = nullptr;
  int* d_queue = nullptr;
  int* d_order = nullptr;
  Ctl* d_ctl = nullptr;
  long* d_offx = nullptr;
  long* d_offy = nullptr;
  double* d_outx = nullptr;
  double* d_outy = nullptr;
  double* d_x0 = nullptr;
  double* d_y0 = nullptr;
  double* d_norm = nullptr;
  double* d_s = nullptr;          // packed dual slacks (host outputs), made on first use
  double* io = nullptr;           // IO_DOUBLES of scratch for the dual-slack output
  std::vector<long> offx, offy;   // count + 1 prefix sums of n and m
  int grid = 1;
  bool cones = false;             // some instance has SOC/RSOC/EXP/POW blocks
  bool ext = false;               // some instance has row bounds, boxes or EXP1 blocks
  int div_a = 2, div_at = 2;      // lanes-per-row rule: lanes <= mean nnz / div
  double tune_s = 0.0;
  hipStream_t cap = nullptr;      // private stream used for graph capture
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
};

// lanes per row minimising the dependent memory round trips of one
// workgroup's pass over `rows` rows of mean length `mean`: each group of rows
// costs a row-pointer load plus, per four nonzeros of a lane, a column-index
// and a gathered-value load.  With the longest row `maxlen` (default: the
// mean) one pass costs as much as that row, since the workgroup waits for
// its slowest group.
int pick_lanes(double rows, double mean, int maxL = 64, double maxlen = -1.0) {
  int best = 1;
  double bc = 1e300;
  if (maxlen < mean) maxlen = mean;
  for (int L = 1; L <= maxL; L = (L == 64 ? block_size() : 2 * L)) {
    const double passes = std::ceil(std::max(rows, 1.0) / (double)(block_size() / L));
    const double trips = std::ceil(std::max(mean, 1.0) / (4.0 * L));
    const double tmax = std::ceil(std::max(maxlen, 1.0) / (4.0 * L));
    const double cost = (passes - 1.0) * (1.0 + 2.0 * trips) + (1.0 + 2.0 * tmax) + 0.25 * std::log2((double)L);
    if (cost < bc) {
      bc = cost;
      best = L;
    }
  }
  return best;
}

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
  P.p_diag = H.p_diag ? 1 : 0;
  P.Pd = H.p_diag ? B.upload(H.pdiag) : nullptr;
  P.A_valf = P.AT_valf = P.P_valf = P.Rf = nullptr;
  if (h->s.precision == PDHCG_PREC_FP32) {
    auto f32 = [](const std::vector<double>& v) { return std::vector<float>(v.begin(), v.end()); };
    P.A_valf = B.upload(f32(H.A.val));
    P.AT_valf = B.upload(f32(H.AT.val));
    if (H.P.rows > 0) P.P_valf = B.upload(f32(H.P.val));
    if (H.r > 0) P.Rf = B.upload(f32(H.R));
  }
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
  P.rlo = H.rlo.empty() ? nullptr : B.upload(H.rlo);
  P.rhi = H.rhi.empty() ? nullptr : B.upload(H.rhi);
  P.xlo = H.xlo.empty() ? nullptr : B.upload(H.xlo);
  P.xhi = H.xhi.empty() ? nullptr : B.upload(H.xhi);
  P.ext = needs_ext(H) ? 1 : 0;
  P.resc = H.resc ? 1 : 0;
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
  if (h->s.scheme == PDHCG_SCHEME_AVG) {
    V.xb = B.alloc<double>(n);
    V.yb = B.alloc<double>(m);
    V.Axb = B.alloc<double>(m);
  }
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

  // launch geometry: at most the workgroups resident at once for the kernel
  // this solve runs (two per CU for problems without cone blocks)
  const bool fp32 = h->s.precision == PDHCG_PREC_FP32;
  const bool has_cones = !H.wave_start.empty() || !H.lane_start.empty();
  bool lin_kernel = false;    // the solve runs solve_kernel_lin(_ext) (set with the grid)
  int maxg = 1;
  HIPCHK(max_resident_grid_for(fp32, P.ext != 0, has_cones, 0, &maxg));
  int G = h->s.grid_dim;
  if (G <= 0) {
    long work = std::max<long>(std::max<long>(n, m), 1);
    // about two thirds of a workgroup's threads per row or coordinate
    // (measured: more, smaller workgroups shorten every latency-bound phase)
    const long per = std::max(1L, (long)block_size() * 2 / 3);
    long want = (work + per - 1) / per;
    G = (int)std::min<long>(std::max<long>(want, 1), maxg);
  }
  G = std::max(1, std::min(G, maxg));
  I->grid = G;
  lin_kernel = !has_cones && G > 1;
  // ownership ranges: coordinates weighted by their share of the A^T and P
  // passes, the dense factor and the cone projections (cone blocks are never
  // split); rows by their nonzeros
  {
    std::vector<long> pc(G + 1, 0), pr(G + 1, 0);
    std::vector<int> pw(G + 1, 0), pl(G + 1, 0);
    // split into G contiguous ranges.  A unit flagged heavy (it holds a row
    // far longer than the rest) gets a workgroup of its own, so its lanes are
    // chosen for it alone; the other workgroups are shared among the light
    // segments between heavy units in proportion to their weight (at least
    // one per nonempty segment), and each segment is cut by cumulative
    // weight.  Without heavy units this is the plain cumulative split.
    // units of kind kHeadKind: the head of a degree order (below)
    const signed char kind_head = 100;
    auto split = [&](const std::vector<std::pair<long, double>>& units, const std::vector<char>& heavy_u,
                     const std::vector<signed char>& kind_u, long total_items, std::vector<long>& out) {
      struct Seg { size_t a, b; bool heavy; double w; int k; };
      std::vector<Seg> segs;
      double wlight = 0.0;
      for (size_t i = 0; i < units.size();) {
        if (heavy_u[i]) {
          segs.push_back({i, i + 1, true, units[i].second, 1});
          ++i;
          continue;
        }
        size_t j = i;
        double w = 0.0;
        while (j < units.size() && !heavy_u[j] && kind_u[j] == kind_u[i]) w += units[j++].second;
        segs.push_back({i, j, false, w, 0});
        wlight += w;
        i = j;
      }
      int nheavy = 0, nlight = 0;
      for (const auto& s : segs) (s.heavy ? nheavy : nlight) += 1;
      int avail = G - nheavy;
      // head segments (kind_head) are packed in order: a new workgroup
      // whenever the next unit would overflow the average light share, so a
      // head workgroup holds at most that share or a single unit; their
      // workgroup counts come from the packing, the other light segments
      // share the rest
      const double cap = avail > 0 ? wlight / avail : 0.0;
      auto pack = [&](const Seg& sg, std::vector<long>* cuts) {
        int bins = 1;
        double cur = 0.0;
        for (size_t u = sg.a; u < sg.b; ++u) {
          if (cur > 0.0 && cur + units[u].second > cap) {
            if (cuts) cuts->push_back(units[u - 1].first);
            ++bins;
            cur = 0.0;
          }
          cur += units[u].second;
        }
        return bins;
      };
      int khead = 0, nhead = 0;
      double whead = 0.0;
      for (auto& sg : segs)
        if (!sg.heavy && kind_u[sg.a] == kind_head) {
          sg.k = pack(sg, nullptr);
          khead += sg.k;
          whead += sg.w;
          ++nhead;
        }
      if ((nheavy == 0 && nlight <= 1) || avail < nlight || avail - khead < nlight - nhead) {
        // plain cumulative split (also the fallback when there are too many
        // heavy units for dedicated workgroups)
        double total = 0.0;
        for (const auto& u : units) total += u.second;
        out[0] = 0;
        int kk = 1;
        double cum = 0.0;
        for (const auto& u : units) {
          cum += u.second;
          while (kk < G && cum >= total * kk / G) out[kk++] = u.first;
        }
        while (kk <= G) out[kk++] = total_items;
        out[G] = total_items;
        return;
      }
      // proportional shares with at least one workgroup per light segment
      const int avail_p = avail - khead;
      const double wlight_p = wlight - whead;
      auto is_head = [&](const Seg& sg) { return !sg.heavy && kind_u[sg.a] == kind_head; };
      int given = 0;
      for (auto& s : segs)
        if (!s.heavy && !is_head(s)) {
          s.k = std::max(1, (int)std::floor(avail_p * s.w / std::max(wlight_p, 1e-300)));
          given += s.k;
        }
      while (given > avail_p) {        // take back from the largest shares
        Seg* big = nullptr;
        for (auto& s : segs)
          if (!s.heavy && !is_head(s) && s.k > 1 && (!big || s.w / s.k < big->w / big->k)) big = &s;
        if (!big) break;
        big->k -= 1;
        given -= 1;
      }
      while (given < avail_p) {        // hand out the rest to the heaviest per workgroup
        Seg* big = nullptr;
        for (auto& s : segs)
          if (!s.heavy && !is_head(s) && (!big || s.w / s.k > big->w / big->k)) big = &s;
        if (!big) break;
        big->k += 1;
        given += 1;
      }
      int kk = 0;
      out[0] = 0;
      for (const auto& s : segs) {
        const long seg_end = units[s.b - 1].first;
        if (s.heavy || s.k == 1) {
          out[++kk] = seg_end;
          continue;
        }
        if (is_head(s)) {
          std::vector<long> cuts;
          pack(s, &cuts);
          for (long c : cuts) out[++kk] = c;
          out[++kk] = seg_end;
          continue;
        }
        double cum = 0.0;
        int made = 0;
        for (size_t u = s.a; u < s.b && made < s.k - 1; ++u) {
          cum += units[u].second;
          while (made < s.k - 1 && cum >= s.w * (made + 1) / s.k) {
            out[++kk] = units[u].first;
            ++made;
          }
        }
        while (made < s.k - 1) {
          out[++kk] = seg_end;
          ++made;
        }
        out[++kk] = seg_end;
      }
      while (kk < G) out[++kk] = total_items;
      out[G] = total_items;
    };
    std::vector<std::pair<long, double>> cu;
    std::vector<char> cheavy;
    // unit kinds: elementwise coordinates, or the cone type; a workgroup's
    // range never spans two kinds, so no workgroup runs two kinds of
    // projection (or mixes SOC and RSOC group widths) one after the other
    std::vector<signed char> ckind;
    cu.reserve(n);
    cheavy.reserve(n);
    ckind.reserve(n);
    // heavy: a unit with an A^T or P row of at least 4096 nonzeros and over
    // half a workgroup's share of the total weight (flags set below, once
    // the total is known).  Lighter long rows share a workgroup with other
    // coordinates and run in the A^T length classes; a dedicated workgroup
    // holds one coordinate's P and elementwise work, so below that size it
    // idles through the inner loop (measured on the large sparse QP: 60 of
    // 256 workgroups dedicated at 5% of a share waited at the grid barriers
    // for a third of the solve)
    std::vector<double> unit_nz;
    unit_nz.reserve(n);
    auto rownz = [&](long i) {
      double z = (double)(H.AT.ptr[i + 1] - H.AT.ptr[i]);
      if (H.P.rows > 0) z = std::max(z, (double)(H.P.ptr[i + 1] - H.P.ptr[i]));
      return z;
    };
    // per-coordinate work of one outer iteration: the A^T row once, the
    // elementwise work, P row (unless P is diagonal) and factor columns
    // once per prox step (about fq of them for a general Q).  With a
    // sparse P the inner loop's P products dominate and run in phases of
    // their own, so the A^T row, read in the one phase per iteration that
    // precedes them, counts 1/fq of its nonzeros: ownership leans towards
    // the inner loop's work (measured on the large sparse QP, whose
    // power-law A^T rows otherwise give the slack columns' workgroups 28%
    // more P rows in every inner step)
    const double fq = H.q_diag ? 1.0 : 3.0;
    const bool sparse_p = H.P.rows > 0 && !H.p_diag;
    const double at_w = sparse_p ? 1.0 / fq : 1.0;
    auto wcoord = [&](long i) {
      double w = fq * (2.0 + H.r) + at_w * (double)(H.AT.ptr[i + 1] - H.AT.ptr[i]);
      if (sparse_p) w += fq * (double)(H.P.ptr[i + 1] - H.P.ptr[i]);
      return w;
    };
    // the head of a degree order (its longest A^T rows) is a segment of its
    // own, cut by the work of the A^T phase (A^T row and P row), in the
    // units of the other coordinates' weight: each head workgroup gets an
    // average workgroup's share of that phase, and no other workgroup
    // carries a long A^T row beside a full share of P rows
    double lam_head = 0.0;
    if (H.head > 0 && sparse_p) {
      double sw = 0.0, sz = 0.0;
      for (long i = H.head; i < n; ++i) {
        sw += wcoord(i);
        sz += (double)(H.AT.ptr[i + 1] - H.AT.ptr[i]) + (double)(H.P.ptr[i + 1] - H.P.ptr[i]);
      }
      lam_head = sz > 0.0 ? sw / sz : 0.0;
    }
    auto whead = [&](long i) {
      if (!sparse_p) return wcoord(i);
      return lam_head * ((double)(H.AT.ptr[i + 1] - H.AT.ptr[i]) + (double)(H.P.ptr[i + 1] - H.P.ptr[i]));
    };
    const signed char kHeadKind = kind_head;
    for (const auto& cb : H.cones) {
      if (cb.type == PDHCG_CONE_FREE || cb.type == PDHCG_CONE_NONNEG || cb.type == PDHCG_CONE_BOX) {
        for (long i = cb.start; i < cb.start + cb.dim; ++i) {
          const bool hd = i < H.head;
          cu.emplace_back(i + 1, hd ? whead(i) : wcoord(i));
          unit_nz.push_back(rownz(i));
          ckind.push_back(hd ? kHeadKind : 0);
        }
      } else {
        double w = 0.0, zmax = 0.0;
        for (long i = cb.start; i < cb.start + cb.dim; ++i) {
          w += wcoord(i) + 26.0 * fq;
          zmax = std::max(zmax, rownz(i));
        }
        if (cb.type == PDHCG_CONE_EXP) w += 180.0 * fq;
        if (cb.type == PDHCG_CONE_POW) w += 320.0 * fq;
        cu.emplace_back((long)cb.start + cb.dim, w);
        unit_nz.push_back(zmax);
        ckind.push_back((signed char)(1 + cb.type));
      }
    }
    {
      double wtot = 0.0;
      for (const auto& u : cu) wtot += u.second;
      const double heavy_nz = std::max(4096.0, 0.5 * wtot / G);
      for (double z : unit_nz) cheavy.push_back(z > heavy_nz);
    }
    // with many alternating kinds the kind boundaries would fragment the
    // split: keep them only while there are few kind runs
    auto few_runs = [&](std::vector<signed char>& kind) {
      int runs = 0;
      for (size_t i = 0; i < kind.size(); ++i) runs += (i == 0 || kind[i] != kind[i - 1]) ? 1 : 0;
      if (runs > std::max(1, G / 8)) std::fill(kind.begin(), kind.end(), (signed char)0);
    };
    few_runs(ckind);
    split(cu, cheavy, ckind, n, pc);
    // rows: weighted by their nonzeros; a workgroup's rows share one length
    // class (<= 16, 64, 256, 1024 nonzeros, longer) while the classes come in
    // few runs, so the lanes per row chosen from the mean fit every row
    std::vector<std::pair<long, double>> ru;
    std::vector<signed char> rkind(m);
    ru.reserve(m);
    for (long l = 0; l < m; ++l) {
      const long z = H.A.ptr[l + 1] - H.A.ptr[l];
      ru.emplace_back(l + 1, 2.0 + (double)z);
      rkind[l] = (signed char)(z <= 16 ? 0 : (z <= 64 ? 1 : (z <= 256 ? 2 : (z <= 1024 ? 3 : 4))));
    }
    few_runs(rkind);
    split(ru, std::vector<char>(ru.size(), 0), rkind, m, pr);
    for (int w = 0; w <= G; ++w) {
      pw[w] = (int)(std::lower_bound(H.wave_start.begin(), H.wave_start.end(), (int)std::min<long>(pc[w], n)) -
                    H.wave_start.begin());
      pl[w] = (int)(std::lower_bound(H.lane_start.begin(), H.lane_start.end(), (int)std::min<long>(pc[w], n)) -
                    H.lane_start.begin());
    }
    // skewed A^T row lengths (some row of a workgroup more than 16 times its
    // mean and longer than 64): A^T rows then run in length classes (below)
    bool at_classes = false;
    for (int w = 0; w < G && !at_classes; ++w) {
      const long nr = pc[w + 1] - pc[w];
      if (nr <= 0) continue;
      const double mean = (double)(H.AT.ptr[pc[w + 1]] - H.AT.ptr[pc[w]]) / nr;
      for (long i = pc[w]; i < pc[w + 1]; ++i) {
        const double z = (double)(H.AT.ptr[i + 1] - H.AT.ptr[i]);
        if (z > 64.0 && z > 16.0 * mean) { at_classes = true; break; }
      }
    }
    at_classes = at_classes && h->s.lanes_at <= 0;
    // lanes per row chosen per workgroup from its own rows (about two
    // nonzeros per lane; the longest row priced in, of A^T only when A^T
    // does not run in length classes), SOC/RSOC group width from its longest
    // block
    std::vector<unsigned short> lanes(4 * (size_t)G, 1);
    for (int w = 0; w < G; ++w) {
      long nr = pc[w + 1] - pc[w];
      double nz = 0.0, zmax = 0.0;
      if (nr > 0) {
        // with A^T in length classes the workgroup's lanes serve its P rows
        // (and the setup products) only
        const double pnz = H.P.rows > 0 ? (double)(H.P.ptr[pc[w + 1]] - H.P.ptr[pc[w]]) : 0.0;
        nz = (double)(H.AT.ptr[pc[w + 1]] - H.AT.ptr[pc[w]]);
        if (H.P.rows > 0) nz = at_classes ? pnz : std::max(nz, pnz);
        for (long i = pc[w]; i < pc[w + 1]; ++i) {
          double z = H.P.rows > 0 ? (double)(H.P.ptr[i + 1] - H.P.ptr[i]) : 0.0;
          if (!at_classes) z = std::max(z, (double)(H.AT.ptr[i + 1] - H.AT.ptr[i]));
          zmax = std::max(zmax, z);
        }
      }
      lanes[4 * w + 0] = (unsigned short)(h->s.lanes_at > 0 ? h->s.lanes_at
                                                          : pick_lanes((double)nr, nr > 0 ? nz / nr : 1.0,
                                                                       block_size(), zmax));
      long mr = pr[w + 1] - pr[w];
      double mz = mr > 0 ? (double)(H.A.ptr[pr[w + 1]] - H.A.ptr[pr[w]]) / mr : 1.0, mmax = 0.0;
      for (long l = pr[w]; l < pr[w + 1]; ++l) mmax = std::max(mmax, (double)(H.A.ptr[l + 1] - H.A.ptr[l]));
      int la_rows = pick_lanes((double)mr, mz, 64, mmax);
      // the cone-free kernel keeps twice the waves in flight: rows of a few
      // nonzeros gain from two lanes even where the round-trip model sees
      // the extra passes (measured on the large sparse QP: the solve 8%
      // faster; the same floor for its P rows of three nonzeros was 2%
      // slower)
      if (lin_kernel && mz >= 4.0) la_rows = std::max(la_rows, 2);
      lanes[4 * w + 1] = (unsigned short)(h->s.lanes_a > 0 ? h->s.lanes_a : la_rows);
      int maxdim = 1;
      for (int it = pw[w]; it < pw[w + 1]; ++it) maxdim = std::max(maxdim, H.wave_dim[it]);
      lanes[4 * w + 2] = (unsigned short)(maxdim <= 17 ? 16 : (maxdim <= 33 ? 32 : 64));
    }
    // the owned columns of R in LDS when the largest slice fits in 64 KiB
    long maxloc = 0;
    for (int w = 0; w < G; ++w) maxloc = std::max(maxloc, pc[w + 1] - pc[w]);
    const size_t rbytes = (size_t)H.r * (size_t)maxloc * sizeof(double);
    I->lds_bytes = (H.r > 0 && rbytes <= (size_t)64 * 1024) ? (int)rbytes : 0;
    if (I->lds_bytes > 0) {
      // the slice must not cost the grid its residency
      int mg = 0;
      HIPCHK(max_resident_grid_for(fp32, P.ext != 0, has_cones, I->lds_bytes, &mg));
      if (mg < G) I->lds_bytes = 0;
    }
    // skewed A^T row lengths (some row of a workgroup more than 16 times its
    // mean and longer than 64): order each workgroup's rows by length class
    // (<= 16, 64, 256, 1024 nonzeros, longer), run with 1, 4, 16, 64 and 512
    // lanes per row
    P.at_perm = nullptr;
    P.at_seg = nullptr;
    {
      if (at_classes) {
        constexpr int NC = 5;
        std::vector<int> perm(n), seg((size_t)(NC + 1) * G);
        for (int w = 0; w < G; ++w) {
          std::vector<std::vector<int>> cls(NC);
          for (long i = pc[w]; i < pc[w + 1]; ++i) {
            const long z = H.AT.ptr[i + 1] - H.AT.ptr[i];
            const int c = z <= 16 ? 0 : (z <= 64 ? 1 : (z <= 256 ? 2 : (z <= 1024 ? 3 : 4)));
            cls[c].push_back((int)i);
          }
          long pos = pc[w];
          for (int c = 0; c < NC; ++c) {
            seg[(size_t)(NC + 1) * w + c] = (int)pos;
            for (int i : cls[c]) perm[pos++] = i;
          }
          seg[(size_t)(NC + 1) * w + NC] = (int)pos;
        }
        P.at_perm = B.upload(perm);
        P.at_seg = B.upload(seg);
      }
    }
    // the same length classes over all of A^T for the setup products
    if (P.at_perm) {
      std::vector<std::vector<int>> cls(5);
      for (long i = 0; i < n; ++i) {
        const long z = H.AT.ptr[i + 1] - H.AT.ptr[i];
        cls[z <= 16 ? 0 : (z <= 64 ? 1 : (z <= 256 ? 2 : (z <= 1024 ? 3 : 4)))].push_back((int)i);
      }
      std::vector<int> all;
      all.reserve(n);
      for (int c = 0; c < 5; ++c) {
        I->at_cls_seg[c] = (long)all.size();
        all.insert(all.end(), cls[c].begin(), cls[c].end());
      }
      I->at_cls_seg[5] = (long)all.size();
      I->at_cls_perm = B.upload(all);
    }
    P.part_c = B.upload(pc);
    P.part_r = B.upload(pr);
    P.part_w = B.upload(pw);
    P.part_l = B.upload(pl);
    P.part_lanes = B.upload(lanes);
    if (const char* path = std::getenv("PDHCG_PARTITION_DUMP")) {
      // one line per workgroup: coordinate range, row range, lanes per A^T
      // row, per A row, SOC group width
      if (FILE* f = std::fopen(path, "w")) {
        for (int w = 0; w < G; ++w)
          std::fprintf(f, "%d %ld %ld %ld %ld %d %d %d\n", w, pc[w], pc[w + 1], pr[w], pr[w + 1], lanes[4 * w],
                       lanes[4 * w + 1], lanes[4 * w + 2]);
        std::fclose(f);
      }
    }
  }
  V.partials = B.alloc<double>((size_t)SL_COUNT * G);
  I->bar_bytes = sizeof(Barrier) + sizeof(unsigned) * (size_t)G * BAR_STRIDE;
  I->bar = (Barrier*)B.alloc<char>(I->bar_bytes);
  I->d_perm = H.perm.empty() ? nullptr : B.upload(H.perm);
  I->io = B.alloc<double>(IO_DOUBLES);
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
    if (I->at_cls_perm)
      HIPCHK(launch_spmv_classes(P.AT_ptr, P.AT_col, P.AT_val, t, w, I->at_cls_perm, I->at_cls_seg, st));
    else
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

// per-workgroup phase timers (settings.verbose & 8): summary on stderr, and
// one CSV line per workgroup into $PDHCG_PROFILE_DUMP when set
void report_phases(const unsigned long long* dpt, int grid) {
  static const char* names[PT_COUNT] = {"init", "P1", "P2", "P3", "P4", "P6", "check",
                                        "halpern", "barrier", "proj", "wcall", "ncall"};
  int dev = 0, khz = 100000;
  (void)hipGetDevice(&dev);
  (void)hipDeviceGetAttribute(&khz, hipDeviceAttributeWallClockRate, dev);
  std::vector<unsigned long long> pt((size_t)PT_COUNT * grid);
  (void)hipMemcpy(pt.data(), dpt, pt.size() * sizeof(unsigned long long), hipMemcpyDeviceToHost);
  std::fprintf(stderr, "pdhcg phase times over %d workgroups: mean / max / argmax [ms]\n", grid);
  for (int i = 0; i < PT_COUNT; ++i) {
    double s = 0, mx = 0;
    int am = 0;
    for (int w = 0; w < grid; ++w) {
      double v = pt[(size_t)w * PT_COUNT + i] / (double)khz;
      s += v;
      if (v > mx) { mx = v; am = w; }
    }
    std::fprintf(stderr, "  %-8s %10.3f %10.3f %5d\n", names[i], s / grid, mx, am);
  }
  if (const char* path = std::getenv("PDHCG_PROFILE_DUMP")) {
    if (FILE* f = std::fopen(path, "w")) {
      for (int w = 0; w < grid; ++w) {
        std::fprintf(f, "%d", w);
        for (int i = 0; i < PT_COUNT; ++i) std::fprintf(f, ",%.4f", pt[(size_t)w * PT_COUNT + i] / (double)khz);
        std::fprintf(f, "\n");
      }
      std::fclose(f);
    }
  }
}

// a host copy of a problem whose arrays are device memory
// (settings.memory_kind = PDHCG_MEM_DEVICE); setup then proceeds as for host
// input
struct HostMirror {
  std::vector<int64_t> arp, prp;
  std::vector<int32_t> acol, pcol, ctype, cstart, cdim;
  std::vector<double> aval, b, c, pval, R, D, calpha, rlo, rhi, xlo, xhi;
  pdhcg_problem p{};
};

template <class T>
int d2h(const T* src, int64_t count, std::vector<T>& dst, const T** out) {
  *out = nullptr;
  if (!src) return PDHCG_OK;
  if (count < 0) return PDHCG_E_SHAPE;
  dst.resize((size_t)std::max<int64_t>(count, 1));
  if (count > 0 && hipMemcpy(dst.data(), src, (size_t)count * sizeof(T), hipMemcpyDeviceToHost) != hipSuccess)
    return PDHCG_E_HIP;
  *out = dst.data();
  return PDHCG_OK;
}

int mirror_problem(const pdhcg_problem& d, HostMirror& M) {
  M.p = d;
  const int64_t n = d.n, m = d.m, r = d.r;
  if (n < 1 || m < 0 || r < 0 || d.nblocks < 0) return PDHCG_E_SHAPE;
  constexpr int64_t kMaxNnz = (int64_t)1 << 36;
  int rc = d2h(d.A_rowptr, m + 1, M.arp, &M.p.A_rowptr);
  const int64_t nnz = (rc == PDHCG_OK && M.p.A_rowptr) ? M.arp[m] : 0;
  if (nnz < 0 || nnz > kMaxNnz) return PDHCG_E_CSR;
  if (rc == PDHCG_OK) rc = d2h(d.A_col, nnz, M.acol, &M.p.A_col);
  if (rc == PDHCG_OK) rc = d2h(d.A_val, nnz, M.aval, &M.p.A_val);
  if (rc == PDHCG_OK) rc = d2h(d.b, m, M.b, &M.p.b);
  if (rc == PDHCG_OK) rc = d2h(d.c, n, M.c, &M.p.c);
  if (rc == PDHCG_OK) rc = d2h(d.P_rowptr, n + 1, M.prp, &M.p.P_rowptr);
  const int64_t pnnz = (rc == PDHCG_OK && M.p.P_rowptr) ? M.prp[n] : 0;
  if (pnnz < 0 || pnnz > kMaxNnz) return PDHCG_E_CSR;
  if (rc == PDHCG_OK) rc = d2h(d.P_col, pnnz, M.pcol, &M.p.P_col);
  if (rc == PDHCG_OK) rc = d2h(d.P_val, pnnz, M.pval, &M.p.P_val);
  if (rc == PDHCG_OK) rc = d2h(d.R, r * n, M.R, &M.p.R);
  if (rc == PDHCG_OK) rc = d2h(d.D, r * r, M.D, &M.p.D);
  if (rc == PDHCG_OK) rc = d2h(d.cone_type, (int64_t)d.nblocks, M.ctype, &M.p.cone_type);
  if (rc == PDHCG_OK) rc = d2h(d.cone_start, (int64_t)d.nblocks, M.cstart, &M.p.cone_start);
  if (rc == PDHCG_OK) rc = d2h(d.cone_dim, (int64_t)d.nblocks, M.cdim, &M.p.cone_dim);
  if (rc == PDHCG_OK) rc = d2h(d.cone_alpha, (int64_t)d.nblocks, M.calpha, &M.p.cone_alpha);
  if (rc == PDHCG_OK) rc = d2h(d.row_lo, m, M.rlo, &M.p.row_lo);
  if (rc == PDHCG_OK) rc = d2h(d.row_hi, m, M.rhi, &M.p.row_hi);
  if (rc == PDHCG_OK) rc = d2h(d.x_lo, n, M.xlo, &M.p.x_lo);
  if (rc == PDHCG_OK) rc = d2h(d.x_hi, n, M.xhi, &M.p.x_hi);
  return rc;
}

// counters of one solved instance and, with host outputs (wx, wy non-null:
// the scaled candidate on the host), the unscaled x and y; the dual slack
// and device outputs are written by the io kernels
void finish_result(const HostInstance& H, const Ctl& c, int status, const double* wx, const double* wy,
                   double eta, double setup_s, pdhcg_result* res) {
  const long n = H.n, m = H.m;
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
  res->a_norm = 0.998 / eta;
  res->setup_s = setup_s;
  const bool pm = !H.perm.empty();   // internal coordinate j is the caller's perm[j]
  if (res->x && wx)
    for (long i = 0; i < n; ++i) res->x[pm ? H.perm[i] : i] = H.nu_b * wx[i] / H.Sx[i];
  if (res->y && wy)
    for (long l = 0; l < m; ++l) res->y[l] = H.nu_c * H.Sy[l] * wy[l];
}

// outputs of one instance from its scaled candidate (W, Wy) on the device:
// with device outputs x, y and s straight into the caller's buffers; with
// host outputs s through the staging vector `stage` (n doubles), x and y
// being unscaled on the host by finish_result
hipError_t device_outputs(const DevProblem& P, const int* perm, double* io, const double* W, const double* Wy,
                          bool dev, double* stage, pdhcg_result* res, hipStream_t st) {
  hipError_t e = hipSuccess;
  if (dev) {
    if (res->x) e = launch_scale_out(W, perm, P.Sx, P.nu_b, true, res->x, P.n, st);
    if (e == hipSuccess && res->y) e = launch_scale_out(Wy, nullptr, P.Sy, P.nu_c, false, res->y, P.m, st);
    if (e == hipSuccess && res->s) e = launch_dual_slack(P, W, Wy, perm, io, res->s, st);
    return e;
  }
  if (res->s) {
    e = launch_dual_slack(P, W, Wy, perm, io, stage, st);
    if (e == hipSuccess) e = hipMemcpyAsync(res->s, stage, (size_t)P.n * sizeof(double), hipMemcpyDeviceToHost, st);
  }
  return e;
}

// carves one instance's region of the batch arena: `put` places a host
// array (copied into the staging image when there is one), `take` reserves
// device space; offsets are 256-byte aligned
struct Carve {
  size_t off = 0;
  char* stage = nullptr;      // host image of the region (null: sizing pass)
  uintptr_t dev = 0;          // device address of the region
  template <class T>
  T* take(size_t count) {
    off = (off + 255) & ~(size_t)255;
    T* p = (T*)(dev + off);
    off += std::max<size_t>(count, 1) * sizeof(T);
    return p;
  }
  template <class T>
  T* put(const std::vector<T>& v) {
    const size_t o = (off + 255) & ~(size_t)255;
    T* p = take<T>(v.size());
    if (stage && !v.empty()) std::memcpy(stage + o, v.data(), v.size() * sizeof(T));
    return p;
  }
};

void carve_instance(const HostInstance& H, int trace_cap, bool avg, Carve& c, InstDesc& D) {
  const long n = H.n, m = H.m;
  DevProblem& P = D.P;
  P = DevProblem{};
  P.n = H.n;
  P.m = H.m;
  P.r = H.r;
  P.A_ptr = c.put(H.A.ptr);
  P.A_col = c.put(H.A.col);
  P.A_val = c.put(H.A.val);
  P.AT_ptr = c.put(H.AT.ptr);
  P.AT_col = c.put(H.AT.col);
  P.AT_val = c.put(H.AT.val);
  if (H.P.rows > 0) {
    P.P_ptr = c.put(H.P.ptr);
    P.P_col = c.put(H.P.col);
    P.P_val = c.put(H.P.val);
  }
  P.R = H.r > 0 ? c.put(H.R) : nullptr;
  P.Dm = H.r > 0 ? c.put(H.D) : nullptr;
  P.p_diag = H.p_diag ? 1 : 0;
  P.Pd = H.p_diag ? c.put(H.pdiag) : nullptr;
  P.b = c.put(H.b);
  P.c = c.put(H.c);
  P.qd = c.put(H.qdiag);
  P.Sx = c.put(H.Sx);
  P.Sy = c.put(H.Sy);
  P.ctype = c.put(H.ctype);
  P.n_wave = (int)H.wave_start.size();
  P.n_lane = (int)H.lane_start.size();
  P.wave_start = c.put(H.wave_start);
  P.wave_dim = c.put(H.wave_dim);
  P.wave_type = c.put(H.wave_type);
  P.wave_euclid = c.put(H.wave_euclid);
  P.lane_start = c.put(H.lane_start);
  P.lane_type = c.put(H.lane_type);
  P.lane_alpha = c.put(H.lane_alpha);
  P.lane_euclid = c.put(H.lane_euclid);
  P.nu_b = H.nu_b;
  P.nu_c = H.nu_c;
  P.norm_b = H.norm_b;
  P.norm_c = H.norm_c;
  P.q_diag = H.q_diag ? 1 : 0;
  P.rlo = H.rlo.empty() ? nullptr : c.put(H.rlo);
  P.rhi = H.rhi.empty() ? nullptr : c.put(H.rhi);
  P.xlo = H.xlo.empty() ? nullptr : c.put(H.xlo);
  P.xhi = H.xhi.empty() ? nullptr : c.put(H.xhi);
  P.ext = needs_ext(H) ? 1 : 0;
  P.resc = H.resc ? 1 : 0;
  D.perm = H.perm.empty() ? nullptr : c.put(H.perm);
  DevVec& V = D.V;
  V = DevVec{};
  V.x = c.take<double>(n);
  V.y = c.take<double>(m);
  V.ax = c.take<double>(n);
  V.ay = c.take<double>(m);
  V.wx = c.take<double>(n);
  V.wy = c.take<double>(m);
  V.Ax = c.take<double>(m);
  V.Aa = c.take<double>(m);
  V.Aw = c.take<double>(m);
  V.v = c.take<double>(n);
  V.u = c.take<double>(n);
  V.up = c.take<double>(n);
  V.g = c.take<double>(n);
  V.gp = c.take<double>(n);
  V.zb = c.take<double>(n);
  V.s = c.take<double>(n);
  V.t1 = c.take<double>(n);
  V.t2 = c.take<double>(n);
  D.n_warm = 2 * (P.n_wave + P.n_lane);
  V.warm = c.take<double>(D.n_warm);
  if (avg) {
    V.xb = c.take<double>(n);
    V.yb = c.take<double>(m);
    V.Axb = c.take<double>(m);
  }
  V.partials = c.take<double>(SL_COUNT);
  D.T = TraceBufs{};
  if (trace_cap > 0) {
    D.T.cap = trace_cap;
    D.T.x = c.take<double>((size_t)trace_cap * n);
    D.T.wx = c.take<double>((size_t)trace_cap * n);
    D.T.y = c.take<double>((size_t)trace_cap * std::max<long>(m, 1));
    D.T.wy = c.take<double>((size_t)trace_cap * std::max<long>(m, 1));
    D.T.sc = c.take<double>((size_t)trace_cap * 8);
  }
  D.qmax = 0.0;
  for (double q : H.qdiag) D.qmax = std::max(D.qmax, q);
  int maxdim = 1;
  for (int d : H.wave_dim) maxdim = std::max(maxdim, d);
  D.lg = maxdim <= 17 ? 16 : (maxdim <= 33 ? 32 : 64);
  D.x0 = nullptr;
  D.y0 = nullptr;
}

// lanes per row for rows of mean length `mean`: a power of two <= mean/div;
// div = 0 selects the round-trip model of the single-problem path (with the
// whole instance on one workgroup)
int lanes_rule(double rows, double mean, int div, double maxlen = -1.0) {
  if (div <= 0) return pick_lanes(rows, mean, 64, maxlen);
  int L = 1;
  while (L * 2 <= std::max(1.0, mean / div) && L < 64) L *= 2;
  return L;
}

void set_lanes(Handle* h, int div_a, int div_at) {
  Batch* B = h->B;
  for (int i = 0; i < B->count; ++i) {
    const HostInstance& H = h->inst[i]->H;
    int64_t nz_at = H.AT.nnz();
    if (H.P.rows > 0) nz_at = std::max<int64_t>(nz_at, H.P.nnz());
    const double mat = H.n > 0 ? (double)nz_at / H.n : 1.0;
    const double ma = H.m > 0 ? (double)H.A.nnz() / H.m : 1.0;
    // longest rows, as the single-solve partition prices them
    double zat = 0.0, za = 0.0;
    for (long j = 0; j < H.n; ++j) {
      double z = (double)(H.AT.ptr[j + 1] - H.AT.ptr[j]);
      if (H.P.rows > 0) z = std::max(z, (double)(H.P.ptr[j + 1] - H.P.ptr[j]));
      zat = std::max(zat, z);
    }
    for (long l = 0; l < H.m; ++l) za = std::max(za, (double)(H.A.ptr[l + 1] - H.A.ptr[l]));
    B->desc[i].la = h->s.lanes_at > 0 ? h->s.lanes_at : lanes_rule((double)H.n, mat, div_at, zat);
    B->desc[i].lr = h->s.lanes_a > 0 ? h->s.lanes_a : lanes_rule((double)H.m, ma, div_a, za);
  }
  B->div_a = div_a;
  B->div_at = div_at;
}

int upload_desc(Handle* h, hipStream_t st) {
  Batch* B = h->B;
  HIPCHK(hipMemcpyAsync(B->d_desc, B->desc.data(), sizeof(InstDesc) * B->count, hipMemcpyHostToDevice, st));
  return PDHCG_OK;
}

BatchArgs batch_args(Handle* h, long long stop_at) {
  Batch* B = h->B;
  BatchArgs a{};
  a.desc = B->d_desc;
  a.count = B->count;
  a.order = B->d_order;
  a.queue = B->d_queue;
  a.S = h->ds;
  a.stop_at = stop_at;
  const double lim = h->s.time_limit;
  a.limit_ticks = (lim > 0 && lim < 1e9) ? (unsigned long long)(lim * 1e3 * h->rate_khz) : 0ull;
  return a;
}

int setup_batch(Handle* h) {
  Batch* B = h->B;
  const int count = B->count;
  const int cap = h->s.trace_iters;
  hipStream_t st = h->stream;
  B->desc.assign(count, InstDesc{});
  // region sizes, then one arena, then the staged images in chunks
  std::vector<size_t> base(count + 1, 0);
  for (int i = 0; i < count; ++i) {
    Carve c;
    InstDesc tmp{};
    carve_instance(h->inst[i]->H, cap, h->s.scheme == PDHCG_SCHEME_AVG, c, tmp);
    base[i + 1] = base[i] + ((c.off + 255) & ~(size_t)255);
  }
  B->arena = B->mem.alloc<char>(base[count]);
  B->io = B->mem.alloc<double>(IO_DOUBLES);
  if (B->mem.err != hipSuccess) return B->mem.err == hipErrorOutOfMemory ? PDHCG_E_MEM : PDHCG_E_HIP;
  {
    std::vector<char> stage;
    int first = 0;
    const size_t chunk = (size_t)64 << 20;
    auto flush = [&](int upto) -> int {
      if (stage.empty()) return PDHCG_OK;
      HIPCHK(hipMemcpy(B->arena + base[first], stage.data(), stage.size(), hipMemcpyHostToDevice));
      stage.clear();
      first = upto;
      return PDHCG_OK;
    };
    for (int i = 0; i < count; ++i) {
      const size_t sz = base[i + 1] - base[i];
      if (!stage.empty() && stage.size() + sz > chunk) {
        int rc = flush(i);
        if (rc != PDHCG_OK) return rc;
      }
      const size_t o = stage.size();
      stage.resize(o + sz, 0);
      Carve c;
      c.stage = stage.data() + o;
      c.dev = (uintptr_t)(B->arena + base[i]);
      carve_instance(h->inst[i]->H, cap, h->s.scheme == PDHCG_SCHEME_AVG, c, B->desc[i]);
    }
    int rc = flush(count);
    if (rc != PDHCG_OK) return rc;
  }
  // control blocks, queue, order (largest first), packed outputs
  B->d_ctl = B->mem.alloc<Ctl>(count);
  B->d_desc = B->mem.alloc<InstDesc>(count);
  B->d_queue = B->mem.alloc<int>(1);
  B->d_norm = B->mem.alloc<double>(count);
  B->offx.assign(count + 1, 0);
  B->offy.assign(count + 1, 0);
  for (int i = 0; i < count; ++i) {
    B->offx[i + 1] = B->offx[i] + h->inst[i]->H.n;
    B->offy[i + 1] = B->offy[i] + h->inst[i]->H.m;
    B->desc[i].ctl = B->d_ctl + i;
  }
  B->d_offx = B->mem.upload(B->offx);
  B->d_offy = B->mem.upload(B->offy);
  B->d_outx = B->mem.alloc<double>(B->offx[count]);
  B->d_outy = B->mem.alloc<double>(B->offy[count]);
  std::vector<int> order(count);
  std::vector<double> work(count);
  for (int i = 0; i < count; ++i) {
    const HostInstance& H = h->inst[i]->H;
    order[i] = i;
    work[i] = (double)H.n * (4.0 + H.r) + 2.0 * (double)H.A.nnz() + (double)H.P.nnz() +
              32.0 * (double)(H.wave_start.size() + H.lane_start.size());
  }
  std::stable_sort(order.begin(), order.end(), [&](int a, int b) { return work[a] > work[b]; });
  B->d_order = B->mem.upload(order);
  if (B->mem.err != hipSuccess) return B->mem.err == hipErrorOutOfMemory ? PDHCG_E_MEM : PDHCG_E_HIP;
  for (int i = 0; i < count; ++i) {
    const HostInstance& H = h->inst[i]->H;
    if (!H.wave_start.empty() || !H.lane_start.empty()) B->cones = true;
    if (needs_ext(H)) B->ext = true;
  }
  const int lim = batch_grid_limit(B->cones, B->ext);
  B->grid = h->s.grid_dim > 0 ? std::min(h->s.grid_dim, lim) : lim;
  B->grid = std::max(1, std::min(B->grid, count));

  // step sizes: power iteration per instance with the default lane rule
  set_lanes(h, 0, 0);
  int rc = upload_desc(h, st);
  if (rc != PDHCG_OK) return rc;
  std::vector<double> an(count, h->s.a_norm);
  if (!(h->s.a_norm > 0)) {
    HIPCHK(launch_batch_power(B->d_desc, count, h->s.power_iters, B->d_norm, st));
    HIPCHK(hipMemcpyAsync(an.data(), B->d_norm, sizeof(double) * count, hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
  }
  for (int i = 0; i < count; ++i) {
    const HostInstance& H = h->inst[i]->H;
    double a_n = an[i];
    if (!(a_n > 0)) a_n = 1.0;
    B->desc[i].P.eta = 0.998 / a_n;
    double nb = 0, nc = 0;
    for (double v : H.b) nb += v * v;
    for (double v : H.c) nc += v * v;
    nb = std::sqrt(nb);
    nc = std::sqrt(nc);
    B->desc[i].P.omega0 = h->s.omega0 > 0 ? h->s.omega0 : ((nb > 1e-10 && nc > 1e-10) ? nc / nb : 1.0);
    h->inst[i]->P = B->desc[i].P;
  }
  // autotuner: time a fixed number of outer iterations of the whole batch
  // under each candidate lanes-per-row rule and keep the fastest
  if (h->s.autotune && h->s.lanes_a <= 0 && h->s.lanes_at <= 0) {
    const double t0 = now_s();
    const int it = h->s.tune_iters > 0 ? h->s.tune_iters : 64;
    hipEvent_t e0, e1;
    HIPCHK(hipEventCreate(&e0));
    HIPCHK(hipEventCreate(&e1));
    float best = 3.4e38f;
    int bda = 0, bdat = 0;
    const int divs_a[] = {0, 1, 2, 4, 8, 16};   // 0: the round-trip model
    const int divs_at[] = {0, 1, 2, 4};
    for (int pass = 0; pass < 2; ++pass) {     // pass 0 warms caches and code
      for (int da : divs_a) {
        for (int dat : divs_at) {
          set_lanes(h, da, dat);
          rc = upload_desc(h, st);
          if (rc != PDHCG_OK) return rc;
          HIPCHK(launch_batch_reset(B->d_desc, count, B->d_queue, st));
          HIPCHK(hipEventRecord(e0, st));
          HIPCHK(launch_batch(batch_args(h, it), B->cones, B->ext, B->grid, st));
          HIPCHK(hipEventRecord(e1, st));
          HIPCHK(hipEventSynchronize(e1));
          float ms = 0.0f;
          HIPCHK(hipEventElapsedTime(&ms, e0, e1));
          if (pass == 1 && ms < best) {
            best = ms;
            bda = da;
            bdat = dat;
          }
          if (pass == 0) break;
        }
        if (pass == 0) break;
      }
    }
    (void)hipEventDestroy(e0);
    (void)hipEventDestroy(e1);
    set_lanes(h, bda, bdat);
    B->tune_s = now_s() - t0;
    if (h->s.verbose)
      std::fprintf(stderr, "pdhcg: batch autotune: lanes rule A/%d, A^T/%d (%.3f ms per probe)\n", bda, bdat,
                   best);
  }
  rc = upload_desc(h, st);
  if (rc != PDHCG_OK) return rc;
  HIPCHK(hipStreamSynchronize(st));
  return PDHCG_OK;
}

int capture_batch(Handle* h) {
  Batch* B = h->B;
  if (B->exec) return PDHCG_OK;
  if (!B->cap) HIPCHK(hipStreamCreateWithFlags(&B->cap, hipStreamNonBlocking));
  HIPCHK(hipStreamBeginCapture(B->cap, hipStreamCaptureModeThreadLocal));
  hipError_t e = launch_batch_reset(B->d_desc, B->count, B->d_queue, B->cap);
  if (e == hipSuccess) e = launch_batch(batch_args(h, h->s.max_iter), B->cones, B->ext, B->grid, B->cap);
  if (e == hipSuccess)
    e = launch_batch_gather(B->d_desc, B->count, B->d_offx, B->d_offy, B->d_outx, B->d_outy,
                            h->s.scheme == PDHCG_SCHEME_AVG ? 1 : 0, B->cap);
  hipGraph_t g = nullptr;
  hipError_t e2 = hipStreamEndCapture(B->cap, &g);
  if (e != hipSuccess || e2 != hipSuccess) {
    if (g) (void)hipGraphDestroy(g);
    return PDHCG_E_HIP;
  }
  B->graph = g;
  HIPCHK(hipGraphInstantiate(&B->exec, g, nullptr, nullptr, 0));
  return PDHCG_OK;
}

void free_batch(Batch* B) {
  if (!B) return;
  if (B->exec) (void)hipGraphExecDestroy(B->exec);
  if (B->graph) (void)hipGraphDestroy(B->graph);
  if (B->cap) (void)hipStreamDestroy(B->cap);
  B->mem.release();
  delete B;
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
  s->time_kernels = 0;
  s->autotune = 1;
  s->tune_iters = 64;
  s->fp32_tol = 0.0;
  s->interleave = PDHCG_ORDER_AUTO;
  s->cone_scaling = PDHCG_SCALE_BLOCK;
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

int pdhcg_setup(const pdhcg_problem* probs, int32_t count, const pdhcg_settings* s, pdhcg_handle** out) {
  if (!out) return PDHCG_E_ARG;
  *out = nullptr;
  if (!probs || !s || count < 1) return PDHCG_E_ARG;
  if (s->tol <= 0 || s->check_every < 1 || s->j_max < 1 || s->max_iter < 0 ||
      !(s->rho >= 0.5 && s->rho <= 1.0) || s->power_iters < 0 ||
      (s->scheme != PDHCG_SCHEME_RH && s->scheme != PDHCG_SCHEME_AVG) ||
      (s->scheme == PDHCG_SCHEME_AVG && (s->avg_epoch < 1 || s->precision != PDHCG_PREC_FP64)) ||
      (s->precision != PDHCG_PREC_FP64 && s->precision != PDHCG_PREC_FP32) || s->trace_iters < 0 ||
      (s->cone_scaling != PDHCG_SCALE_BLOCK && s->cone_scaling != PDHCG_SCALE_CONE) ||
      s->interleave < PDHCG_ORDER_CALLER || s->interleave > PDHCG_ORDER_DEGREE)
    return PDHCG_E_ARG;
  if (count > 1 && s->precision != PDHCG_PREC_FP64) return PDHCG_E_ARG;   // batches are FP64
  if ((s->memory_kind != PDHCG_MEM_HOST && s->memory_kind != PDHCG_MEM_DEVICE) ||
      (s->dev_alloc == nullptr) != (s->dev_free == nullptr))
    return PDHCG_E_ARG;
  // device-resident problem arrays: validated and rescaled from a host copy
  std::vector<HostMirror> mirror;
  if (s->memory_kind == PDHCG_MEM_DEVICE) {
    mirror.resize(count);
    for (int i = 0; i < count; ++i) {
      int rc = mirror_problem(probs[i], mirror[i]);
      if (rc != PDHCG_OK) return rc;
    }
  }
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
    I->mem.use(h->s);
    h->inst.push_back(I);
    int rc = build_instance(mirror.empty() ? probs[i] : mirror[i].p, h->s, I->H);
    if (rc != PDHCG_OK) { pdhcg_free(h); return rc; }
  }
  int dev = 0, rate_khz = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&rate_khz, hipDeviceAttributeWallClockRate, dev) != hipSuccess) {
    pdhcg_free(h);
    return PDHCG_E_HIP;
  }
  if (rate_khz <= 0) rate_khz = 100000;
  h->rate_khz = rate_khz;
  h->spin_limit = (unsigned long long)rate_khz * 1000ull * 4ull;   // 4 s
  if (count > 1) {
    h->B = new (std::nothrow) Batch();
    if (!h->B) { pdhcg_free(h); return PDHCG_E_MEM; }
    h->B->mem.use(h->s);
    h->B->count = count;
    int rc = setup_batch(h);
    if (rc != PDHCG_OK) { pdhcg_free(h); return rc; }
    h->setup_s = now_s() - t0;
    *out = h;
    return PDHCG_OK;
  }
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

int pdhcg_solve(pdhcg_handle* h, const double* x0, const double* y0, pdhcg_result* res) {
  if (!h || !res) return PDHCG_E_ARG;
  if (h->inst.size() != 1 || h->B) return PDHCG_E_STATE;
  Instance* I = h->inst[0];
  const HostInstance& H = I->H;
  const long n = H.n, m = H.m;
  hipStream_t st = h->stream;
  double t0 = now_s();
  // warm start in the scaled space: x^ = S_x x0 / nu_b, y^ = y0 / (nu_c S_y)
  const bool dev = h->s.memory_kind == PDHCG_MEM_DEVICE;
  std::vector<double> tmp;
  if (x0 && dev) {
    HIPCHK(launch_scale_in(x0, I->d_perm, I->P.Sx, H.nu_b, false, I->V.zb, n, st));
  } else if (x0) {
    tmp.resize(n);
    for (long i = 0; i < n; ++i) tmp[i] = H.Sx[i] * x0[H.perm.empty() ? i : H.perm[i]] / H.nu_b;
    HIPCHK(hipMemcpyAsync(I->V.zb, tmp.data(), n * sizeof(double), hipMemcpyHostToDevice, st));
  } else {
    HIPCHK(launch_fill(I->V.zb, n, 0.0, st));
  }
  std::vector<double> tmpy;
  if (y0 && m > 0 && dev) {
    HIPCHK(launch_scale_in(y0, nullptr, I->P.Sy, H.nu_c, true, I->V.y, m, st));
  } else if (y0 && m > 0) {
    tmpy.resize(m);
    for (long l = 0; l < m; ++l) tmpy[l] = y0[l] / (H.nu_c * H.Sy[l]);
    HIPCHK(hipMemcpyAsync(I->V.y, tmpy.data(), m * sizeof(double), hipMemcpyHostToDevice, st));
  } else {
    HIPCHK(launch_fill(I->V.y, m, 0.0, st));
  }
  Ctl c0;
  std::memset(&c0, 0, sizeof(c0));
  HIPCHK(reset_cone_failure(st));
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
  a.lds_bytes = I->lds_bytes;
  a.profile = h->s.verbose & 8 ? 1 : 0;
  unsigned long long* dpt = nullptr;
  DevBuf tbuf;                  // phase timers (settings.verbose & 8)
  tbuf.use(h->s);
  if (a.profile) {
    dpt = tbuf.alloc<unsigned long long>((size_t)PT_COUNT * I->grid);
    if (tbuf.err != hipSuccess) return PDHCG_E_MEM;
    HIPCHK(hipMemsetAsync(dpt, 0, sizeof(unsigned long long) * PT_COUNT * I->grid, st));
  }
  a.ptimes = dpt;
  Ctl c = c0;
  int status = 0;
  const long long maxit = h->s.max_iter;
  // FP32 mode: FP32 bulk sweeps until the looser tolerance fp32_tol, then an
  // FP64 polish restarted at that candidate (same primal weight, inner
  // tolerance and counters) down to tol
  bool phase32 = h->s.precision == PDHCG_PREC_FP32;
  const double tol32 = std::max(h->s.tol, h->s.fp32_tol > 0 ? h->s.fp32_tol : 10.0 * h->s.tol);
  if (phase32) a.S.tol = tol32;
  long long switch_at = -1;
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
    HIPCHK(launch_solve(a, phase32, I->grid, st));
    if (timing) HIPCHK(hipEventRecord(ev1, st));
    HIPCHK(hipMemcpyAsync(&c, I->ctl, sizeof(c), hipMemcpyDeviceToHost, st));
    HIPCHK(hipStreamSynchronize(st));
    ++nlaunch;
    if (timing) {
      float ms = 0.0f;
      HIPCHK(hipEventElapsedTime(&ms, ev0, ev1));
      ksum += ms * 1e-3;
    }
    if (c.status == PDHCG_OPTIMAL && phase32 && tol32 > h->s.tol) {
      // precision switch: the FP64 run re-initialises from (zb, y) = the
      // FP32 phase's candidate (w_x, w_y)
      const double* Wd = I->P.q_diag ? I->V.wx : I->V.u;
      HIPCHK(hipMemcpyAsync(I->V.zb, Wd, n * sizeof(double), hipMemcpyDeviceToDevice, st));
      if (m > 0) HIPCHK(hipMemcpyAsync(I->V.y, I->V.wy, m * sizeof(double), hipMemcpyDeviceToDevice, st));
      c.status = 0;
      c.started = 0;
      c.resume = 1;
      HIPCHK(hipMemcpyAsync(I->ctl, &c, sizeof(c), hipMemcpyHostToDevice, st));
      HIPCHK(hipStreamSynchronize(st));
      phase32 = false;
      a.S.tol = h->s.tol;
      switch_at = c.ktot;
      if (c.ktot >= maxit) { status = PDHCG_MAX_ITER; break; }
      continue;
    }
    if (h->s.verbose & 1) {
      // progress of long solves (stderr, at most every 5 s)
      static thread_local double last_print = 0.0;
      const double tn = now_s();
      if (tn - last_print >= 5.0 || c.status != 0) {
        last_print = tn;
        std::fprintf(stderr, "pdhcg: %lld it, %lld inner, %lld restarts, rel_p %.2e rel_d %.2e gap %.2e, %.1f s\n",
                     (long long)c.ktot, (long long)c.inner_total, (long long)c.restarts, c.rel_p, c.rel_d,
                     c.rel_gap, tn - t0);
      }
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
  res->polish_iterations = switch_at >= 0 ? c.ktot - switch_at : 0;
  if (h->s.verbose & 8) {
    report_phases(dpt, I->grid);
    tbuf.release();
  }
  // results (unscaled): the last PDHG candidate, or for averaged epochs the
  // state, which is the epoch average after the last restart
  const bool avg = h->s.scheme == PDHCG_SCHEME_AVG;
  const double* W = avg ? I->V.x : (I->P.q_diag ? I->V.wx : I->V.u);
  const double* Wy = avg ? I->V.y : I->V.wy;
  if (c.ktot == 0) {   // no evaluation yet: the zero point
    HIPCHK(launch_fill(I->V.t1, n, 0.0, st));
    HIPCHK(launch_fill(I->V.Aw, m, 0.0, st));
    W = I->V.t1;
    Wy = I->V.Aw;
  }
  HIPCHK(device_outputs(I->P, I->d_perm, I->io, W, Wy, dev, I->V.t2, res, st));
  std::vector<double> wx, wy;
  if (!dev && (res->x || res->y)) {
    wx.resize(n);
    wy.resize(std::max<long>(m, 1));
    HIPCHK(hipMemcpyAsync(wx.data(), W, n * sizeof(double), hipMemcpyDeviceToHost, st));
    if (m > 0) HIPCHK(hipMemcpyAsync(wy.data(), Wy, m * sizeof(double), hipMemcpyDeviceToHost, st));
  }
  HIPCHK(hipStreamSynchronize(st));
  finish_result(H, c, status, wx.empty() ? nullptr : wx.data(), wx.empty() ? nullptr : wy.data(), I->P.eta,
                h->setup_s, res);
  res->solve_s = now_s() - t0;
  return PDHCG_OK;
}

int pdhcg_solve_batch(pdhcg_handle* h, const double* const* x0s, const double* const* y0s, pdhcg_result* res) {
  if (!h || !res) return PDHCG_E_ARG;
  if (!h->B) return pdhcg_solve(h, x0s ? x0s[0] : nullptr, y0s ? y0s[0] : nullptr, res);
  Batch* B = h->B;
  const int count = B->count;
  hipStream_t st = h->stream;
  const double t0 = now_s();
  // warm starts: scaled on the host into packed buffers; the reset node of
  // the graph copies them into each instance's zb / y
  bool dirty = false;
  const bool dev = h->s.memory_kind == PDHCG_MEM_DEVICE;
  std::vector<double> px, py;
  if (x0s && !dev) px.assign(std::max<long>(B->offx[count], 1), 0.0);
  if (y0s && !dev) py.assign(std::max<long>(B->offy[count], 1), 0.0);
  if (x0s && !B->d_x0) B->d_x0 = B->mem.alloc<double>(B->offx[count]);
  if (y0s && !B->d_y0) B->d_y0 = B->mem.alloc<double>(std::max<long>(B->offy[count], 1));
  if (B->mem.err != hipSuccess) return PDHCG_E_MEM;
  for (int i = 0; i < count; ++i) {
    const HostInstance& H = h->inst[i]->H;
    const double* x0 = x0s ? x0s[i] : nullptr;
    const double* y0 = y0s ? y0s[i] : nullptr;
    const DevProblem& P = B->desc[i].P;
    if (x0 && dev)
      HIPCHK(launch_scale_in(x0, B->desc[i].perm, P.Sx, H.nu_b, false, B->d_x0 + B->offx[i], H.n, st));
    else if (x0)
      for (long j = 0; j < H.n; ++j) px[B->offx[i] + j] = H.Sx[j] * x0[H.perm.empty() ? j : H.perm[j]] / H.nu_b;
    if (y0 && dev)
      HIPCHK(launch_scale_in(y0, nullptr, P.Sy, H.nu_c, true, B->d_y0 + B->offy[i], H.m, st));
    else if (y0)
      for (long l = 0; l < H.m; ++l) py[B->offy[i] + l] = y0[l] / (H.nu_c * H.Sy[l]);
    const double* want_x = x0 ? B->d_x0 + B->offx[i] : nullptr;
    const double* want_y = (y0 && H.m > 0) ? B->d_y0 + B->offy[i] : nullptr;
    if (B->desc[i].x0 != want_x || B->desc[i].y0 != want_y) {
      B->desc[i].x0 = want_x;
      B->desc[i].y0 = want_y;
      dirty = true;
    }
  }
  if (x0s && !dev)
    HIPCHK(hipMemcpyAsync(B->d_x0, px.data(), sizeof(double) * B->offx[count], hipMemcpyHostToDevice, st));
  if (y0s && !dev && B->offy[count] > 0)
    HIPCHK(hipMemcpyAsync(B->d_y0, py.data(), sizeof(double) * B->offy[count], hipMemcpyHostToDevice, st));
  if (dirty) {
    int rc = upload_desc(h, st);
    if (rc != PDHCG_OK) return rc;
  }
  int rc = capture_batch(h);
  if (rc != PDHCG_OK) return rc;
  HIPCHK(reset_cone_failure(st));
  const bool timing = h->s.time_kernels != 0;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  if (timing) {
    HIPCHK(hipEventCreate(&ev0));
    HIPCHK(hipEventCreate(&ev1));
    HIPCHK(hipEventRecord(ev0, st));
  }
  unsigned long long* dpt = nullptr;
  DevBuf tbuf;                  // phase timers (settings.verbose & 8)
  tbuf.use(h->s);
  if (h->s.verbose & 8) {
    // profiled run: a direct launch with phase timers instead of the graph
    dpt = tbuf.alloc<unsigned long long>((size_t)PT_COUNT * B->grid);
    if (tbuf.err != hipSuccess) return PDHCG_E_MEM;
    BatchArgs pa = batch_args(h, h->s.max_iter);
    pa.ptimes = dpt;
    HIPCHK(launch_batch_reset(B->d_desc, B->count, B->d_queue, st));
    HIPCHK(launch_batch(pa, B->cones, B->ext, B->grid, st));
    HIPCHK(launch_batch_gather(B->d_desc, B->count, B->d_offx, B->d_offy, B->d_outx, B->d_outy,
                               h->s.scheme == PDHCG_SCHEME_AVG ? 1 : 0, st));
  } else {
    HIPCHK(hipGraphLaunch(B->exec, st));
  }
  if (timing) HIPCHK(hipEventRecord(ev1, st));
  std::vector<Ctl> ctl(count);
  HIPCHK(hipMemcpyAsync(ctl.data(), B->d_ctl, sizeof(Ctl) * count, hipMemcpyDeviceToHost, st));
  HIPCHK(hipStreamSynchronize(st));
  // candidates of instances stopped before their first evaluation: the zero
  // point; then the device outputs (dual slacks through d_s for host
  // outputs)
  bool want_s = false;
  for (int i = 0; i < count; ++i) {
    if (ctl[i].ktot == 0) {
      HIPCHK(launch_fill(B->d_outx + B->offx[i], h->inst[i]->H.n, 0.0, st));
      HIPCHK(launch_fill(B->d_outy + B->offy[i], h->inst[i]->H.m, 0.0, st));
    }
    want_s = want_s || res[i].s;
  }
  if (want_s && !dev && !B->d_s) {
    B->d_s = B->mem.alloc<double>(B->offx[count]);
    if (B->mem.err != hipSuccess) return PDHCG_E_MEM;
  }
  for (int i = 0; i < count; ++i)
    HIPCHK(device_outputs(B->desc[i].P, B->desc[i].perm, B->io, B->d_outx + B->offx[i], B->d_outy + B->offy[i],
                          dev, B->d_s ? B->d_s + B->offx[i] : nullptr, &res[i], st));
  std::vector<double> ox, oy;
  if (!dev) {
    ox.resize(std::max<long>(B->offx[count], 1));
    oy.resize(std::max<long>(B->offy[count], 1));
    HIPCHK(hipMemcpyAsync(ox.data(), B->d_outx, sizeof(double) * B->offx[count], hipMemcpyDeviceToHost, st));
    if (B->offy[count] > 0)
      HIPCHK(hipMemcpyAsync(oy.data(), B->d_outy, sizeof(double) * B->offy[count], hipMemcpyDeviceToHost, st));
  }
  HIPCHK(hipStreamSynchronize(st));
  double ks = 0.0;
  if (timing) {
    float ms = 0.0f;
    HIPCHK(hipEventElapsedTime(&ms, ev0, ev1));
    ks = ms * 1e-3;
    (void)hipEventDestroy(ev0);
    (void)hipEventDestroy(ev1);
  }
  if (dpt) {
    report_phases(dpt, B->grid);
    tbuf.release();
  }
  for (int i = 0; i < count; ++i) {
    const HostInstance& H = h->inst[i]->H;
    const Ctl& c = ctl[i];
    int status = c.status;
    if (status == 0) status = c.ktot >= h->s.max_iter ? PDHCG_MAX_ITER : PDHCG_TIME_LIMIT;
    const double* wx = dev ? nullptr : ox.data() + B->offx[i];
    const double* wy = dev ? nullptr : oy.data() + B->offy[i];
    finish_result(H, c, status, wx, wy, B->desc[i].P.eta, h->setup_s, &res[i]);
    res[i].kernel_s = i == 0 ? ks : 0.0;
    res[i].kernel_launches = i == 0 ? 1 : 0;
    res[i].grid_dim = B->grid;
    res[i].block_dim = block_size();
  }
  const double dt = now_s() - t0;
  for (int i = 0; i < count; ++i) res[i].solve_s = dt;
  return PDHCG_OK;
}


int pdhcg_last_cone_failure(double* rec, int64_t* count) {
  if (!rec || !count) return PDHCG_E_ARG;
  unsigned cnt = 0;
  if (read_cone_failure(rec, &cnt) != hipSuccess) return PDHCG_E_HIP;
  *count = cnt;
  if (cnt == 0)
    for (int i = 0; i < 8; ++i) rec[i] = 0.0;
  return PDHCG_OK;
}

int pdhcg_project_cones(int32_t type, int32_t dim, int64_t count, const double* alpha, const double* r,
                        const double* metric, double* out) {
  if (type < PDHCG_CONE_FREE || type > PDHCG_CONE_EXP1 || type == PDHCG_CONE_BOX || dim < 1 || count < 0)
    return PDHCG_E_ARG;
  if ((type == PDHCG_CONE_RSOC && dim < 2) ||
      ((type == PDHCG_CONE_EXP || type == PDHCG_CONE_POW || type == PDHCG_CONE_EXP1) && dim != 3))
    return PDHCG_E_CONE;
  if (count == 0) return PDHCG_OK;
  if (!r || !out || (type == PDHCG_CONE_POW && !alpha)) return PDHCG_E_ARG;
  const size_t len = (size_t)count * (size_t)dim;
  std::vector<unsigned char> eu((size_t)count, 1);
  if (metric) {
    for (size_t i = 0; i < len; ++i)
      if (!(metric[i] > 0.0) || !std::isfinite(metric[i])) return PDHCG_E_ARG;
    // a metric that is constant on a block takes the Euclidean formula, as in
    // the solver (Pi^{cI} = Pi^I)
    for (int64_t b = 0; b < count; ++b) {
      const double* mb = metric + (size_t)b * dim;
      bool c = true;
      for (int j = 1; j < dim; ++j) c = c && (mb[j] == mb[0]);
      eu[(size_t)b] = c ? 1 : 0;
    }
  }
  if (type == PDHCG_CONE_POW)
    for (int64_t b = 0; b < count; ++b)
      if (!(alpha[b] > 0.0 && alpha[b] < 1.0)) return PDHCG_E_CONE;
  DevBuf B;
  double* d_r = B.alloc<double>(len);
  double* d_o = B.alloc<double>(len);
  double* d_m = metric ? B.alloc<double>(len) : nullptr;
  double* d_a = type == PDHCG_CONE_POW ? B.alloc<double>((size_t)count) : nullptr;
  unsigned char* d_e = B.alloc<unsigned char>((size_t)count);
  if (B.err != hipSuccess) {
    B.release();
    return PDHCG_E_MEM;
  }
  hipError_t e = hipMemcpy(d_r, r, len * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess && d_m) e = hipMemcpy(d_m, metric, len * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess && d_a) e = hipMemcpy(d_a, alpha, (size_t)count * sizeof(double), hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(d_e, eu.data(), (size_t)count, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = launch_project(type, dim, (long)count, d_a, d_r, d_m, d_e, d_o, nullptr);
  if (e == hipSuccess) e = hipMemcpy(out, d_o, len * sizeof(double), hipMemcpyDeviceToHost);
  B.release();
  return e == hipSuccess ? PDHCG_OK : PDHCG_E_HIP;
}

int pdhcg_get_trace(pdhcg_handle* h, int32_t inst, pdhcg_trace* t) {
  if (!h || !t || inst < 0 || inst >= (int)h->inst.size()) return PDHCG_E_ARG;
  Instance* I = h->inst[inst];
  const TraceBufs& T = h->B ? h->B->desc[inst].T : I->T;
  const Ctl* dctl = h->B ? h->B->desc[inst].ctl : I->ctl;
  if (T.cap <= 0) return PDHCG_E_NOTRACE;
  Ctl c;
  if (hipMemcpy(&c, dctl, sizeof(c), hipMemcpyDeviceToHost) != hipSuccess) return PDHCG_E_HIP;
  long rec = std::min<long long>(c.ktot, T.cap);
  rec = std::min<long>(rec, t->count);
  const long n = I->H.n, m = I->H.m;
  auto cp = [&](double* dst, const double* src, size_t cnt) -> bool {
    if (!dst || cnt == 0) return true;
    return hipMemcpy(dst, src, cnt * sizeof(double), hipMemcpyDeviceToHost) == hipSuccess;
  };
  if (!cp(t->x, T.x, rec * n) || !cp(t->wx, T.wx, rec * n) || !cp(t->y, T.y, rec * m) ||
      !cp(t->wy, T.wy, rec * m))
    return PDHCG_E_HIP;
  if (!I->H.perm.empty()) {   // primal slices back to the caller's order
    std::vector<double> row(n);
    for (double* base : {t->x, t->wx}) {
      if (!base) continue;
      for (long k = 0; k < rec; ++k) {
        double* v = base + (size_t)k * n;
        for (long j = 0; j < n; ++j) row[I->H.perm[j]] = v[j];
        std::copy(row.begin(), row.end(), v);
      }
    }
  }
  std::vector<double> sc(rec * 8);
  if (!cp(sc.data(), T.sc, rec * 8)) return PDHCG_E_HIP;
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

int pdhcg_get_scaling(pdhcg_handle* h, int32_t inst, double* Sx, double* Sy, double* nu_b, double* nu_c,
                      double* eta, double* omega0) {
  if (!h || inst < 0 || inst >= (int)h->inst.size()) return PDHCG_E_ARG;
  const Instance* I = h->inst[inst];
  if (Sx)
    for (size_t j = 0; j < I->H.Sx.size(); ++j) Sx[I->H.perm.empty() ? j : (size_t)I->H.perm[j]] = I->H.Sx[j];
  if (Sy) std::copy(I->H.Sy.begin(), I->H.Sy.end(), Sy);
  if (nu_b) *nu_b = I->H.nu_b;
  if (nu_c) *nu_c = I->H.nu_c;
  if (eta) *eta = I->P.eta;
  if (omega0) *omega0 = I->P.omega0;
  return PDHCG_OK;
}

void pdhcg_free(pdhcg_handle* h) {
  if (!h) return;
  free_batch(h->B);
  for (Instance* I : h->inst) free_instance(I);
  delete h;
}

}  // extern "C"
