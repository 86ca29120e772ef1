// Device-side projections onto the cones of the paper's Appendix C, in the
// Euclidean norm and in the diagonal M-norm of eq. metric-block-projection.
//
// Work mapping on CDNA: one 64-lane wavefront per SOC / RSOC block (each lane
// owns coordinates lane, lane+64, ...; reductions are xor butterflies, whose
// result is bitwise identical in every lane, so control flow stays
// wave-uniform), one lane per 3-dimensional EXP / POW block.
//
//  SOC, metric (eq. soc-metric-projection): the secular equation in lambda is
//    solved in the shifted variable delta = |m_t - lambda| through
//    psi(delta) = delta ||v(delta)|| - m_t |r_t|, which is increasing, equal
//    to -m_t|r_t| at 0 and positive at the far end of the bracket, and whose
//    root is computed to full relative precision by safeguarded Newton.
//  RSOC: mapped to an SOC.  With s' = sqrt(m_s) s, t' = sqrt(m_t) t,
//    q = sqrt(m_s m_t), n = (s' - t')/sqrt2, p = (s' + t')/sqrt2 and
//    v' = sqrt(q) v, the set ||v||^2 <= 2 s t, s,t >= 0 becomes the SOC
//    ||(v', n)|| <= p with metric (m_v/q, 1; 1).  With m = 1 this is the
//    rotation U of eq. rsoc-via-soc.  The root lies below or above q/2 in the
//    xi of eq. rsoc-metric-projection exactly when p > 0 or p < 0.
//  EXP (eq. exp-metric-projection): the root of h_M on the set of ratios
//    rho whose ray is visible from r and carries eta_M > 0, bisected on the
//    cancellation-free H = h_M * Den; special cases as printed.
//  POW: bisection of Prop. power-cone-bisection on g_M over (0, R) with the
//    stable quadratic root of eq. power-cone-stable-quadratic-root.
#pragma once
#include <hip/hip_runtime.h>

#include <math.h>

namespace pdhcg {

#ifdef PDHCG_COUNT_ITERS
__device__ unsigned long long pdhcg_soc_evals;
#endif

// Cross-lane reductions on DPP: quad permutations (xor 1, xor 2), row half
// mirror (pairs lane i with 7-i), row mirror (i with 15-i), a 32-lane
// swizzle (xor 16) and the two half-wave readlanes.  Every step adds a value
// to its partner's with the operands merely swapped, so all lanes of a group
// finish with bitwise identical sums and control flow that depends on them
// stays uniform.
template <int CTRL>
__device__ __forceinline__ double dpp_d(double v) {
  const int lo = __builtin_amdgcn_update_dpp(0, __double2loint(v), CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_update_dpp(0, __double2hiint(v), CTRL, 0xF, 0xF, false);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double swz_xor16(double v) {
  const int lo = __builtin_amdgcn_ds_swizzle(__double2loint(v), 0x401F);
  const int hi = __builtin_amdgcn_ds_swizzle(__double2hiint(v), 0x401F);
  return __hiloint2double(hi, lo);
}

__device__ __forceinline__ double readlane_d(double v, int l) {
  const int lo = __builtin_amdgcn_readlane(__double2loint(v), l);
  const int hi = __builtin_amdgcn_readlane(__double2hiint(v), l);
  return __hiloint2double(hi, lo);
}

// sum over aligned groups of Lw lanes (Lw a power of two <= 64); every lane
// of the wave must call it with the same Lw
__device__ __forceinline__ double group_sum(double v, int Lw) {
  if (Lw >= 2) v += dpp_d<0xB1>(v);
  if (Lw >= 4) v += dpp_d<0x4E>(v);
  if (Lw >= 8) v += dpp_d<0x141>(v);
  if (Lw >= 16) v += dpp_d<0x140>(v);
  if (Lw >= 32) v += swz_xor16(v);
  if (Lw >= 64) v = readlane_d(v, 0) + readlane_d(v, 32);
  return v;
}

__device__ __forceinline__ double wave_sum(double v) {
  v += dpp_d<0xB1>(v);
  v += dpp_d<0x4E>(v);
  v += dpp_d<0x141>(v);
  v += dpp_d<0x140>(v);
  v += swz_xor16(v);
  return readlane_d(v, 0) + readlane_d(v, 32);
}

// ---------------------------------------------------------------------------
// SOC on one wavefront
// ---------------------------------------------------------------------------
// result parameters: kind 0 keep, 1 zero, 2 Euclidean boundary
// (v = fac * r_v, t = tval), 3 metric boundary (v_j = m_j r_j/(m_j + lam),
// t = tval)
struct SocSol {
  int kind;
  double lam, fac, tval;
};

template <class In>
__device__ SocSol soc_wave_solve(const In& in, bool euclid, double* warm, int Lg) {
  const int lane = threadIdx.x & (Lg - 1);
  const double rt = in.rt(), mt = in.mt();
  const int dv = in.dimv();
  // blocks of up to Lg + 1 coordinates keep (r_j, m_j) in one register pair per lane
  const bool small = dv <= Lg;
  double rr = 0.0, mm = 1.0;
  if (small && lane < dv) {
    rr = in.rv(lane);
    mm = in.mv(lane);
  }
  double nv2 = 0.0, nmv2 = 0.0;
  if (small) {
    nv2 = rr * rr;
    nmv2 = (mm * rr) * (mm * rr);
  } else {
    for (int j = lane; j < dv; j += Lg) {
      double r = in.rv(j);
      double mr = in.mv(j) * r;
      nv2 += r * r;
      nmv2 += mr * mr;
    }
  }
  nv2 = group_sum(nv2, Lg);
  const double a = sqrt(nv2);
  SocSol out{0, 0.0, 0.0, 0.0};
  if (a <= rt) return out;
  if (euclid) {
    if (a <= -rt) { out.kind = 1; return out; }
    out.kind = 2;
    out.fac = (a + rt) / (2.0 * a);
    out.tval = 0.5 * (a + rt);
    return out;
  }
  nmv2 = group_sum(nmv2, Lg);
  if (sqrt(nmv2) <= -mt * rt) { out.kind = 1; return out; }
  out.kind = 3;
  if (rt == 0.0) {                      // singular case lam = m_t
    double s2 = 0.0;
    if (small) {
      const double vj = mm * rr / (mm + mt);
      s2 = vj * vj;
    } else {
      for (int j = lane; j < dv; j += Lg) {
        double m = in.mv(j);
        double vj = m * in.rv(j) / (m + mt);
        s2 += vj * vj;
      }
    }
    out.lam = mt;
    out.tval = sqrt(group_sum(s2, Lg));
    return out;
  }
  const double sg = rt > 0.0 ? 1.0 : -1.0;
  const double art = fabs(rt);
  auto eval = [&](double d, double& psi, double& dpsi) {
#ifdef PDHCG_COUNT_ITERS
    if (lane == 0 && blockIdx.x == 0) atomicAdd(&pdhcg_soc_evals, 1ull);
#endif
    double s2 = 0.0, s3 = 0.0;
    const double base = mt - sg * d;
    if (small) {
      const double inv = 1.0 / (mm + base);
      const double vj = mm * rr * inv;
      s2 = vj * vj;
      s3 = s2 * inv;
    } else {
      for (int j = lane; j < dv; j += Lg) {
        double m = in.mv(j);
        const double inv = 1.0 / (m + base);
        double vj = m * in.rv(j) * inv;
        s2 += vj * vj;
        s3 += vj * vj * inv;
      }
    }
    s2 = group_sum(s2, Lg);
    s3 = group_sum(s3, Lg);
    double nv = sqrt(s2);
    psi = d * nv - mt * art;
    dpsi = nv + (nv > 0.0 ? d * sg * s3 / nv : 0.0);
  };
  // psi is increasing; for r_t > 0 it is convex on (0, m_t), for r_t < 0
  // concave on (0, inf).  Newton from either side therefore overshoots at most
  // once (to the right of the root for r_t > 0, where hi = m_t bounds it; to
  // the left for r_t < 0, where lo bounds it) and needs no upper bracket for
  // r_t < 0.  Steps leaving the bracket fall back to bisection / doubling.
  double lo = 0.0, hi = sg > 0.0 ? mt : INFINITY, psi, dpsi;
  // start: the previous root of this block, else the Euclidean estimate
  // t = (||r_v|| + r_t)/2 (t = m_t |r_t| / delta), else the middle
  double d = sg > 0.0 ? 0.5 * mt : mt;
  {
    const double w0 = warm ? *warm : NAN;
    const double tE = 0.5 * (a + rt);
    if (w0 > lo && w0 < hi) d = w0;
    else if (tE > 0.0 && mt * art / tE > lo && mt * art / tE < hi) d = mt * art / tE;
  }
  for (int it = 0; it < 400; ++it) {
    eval(d, psi, dpsi);
    if (psi < 0.0) lo = d; else hi = d;
    if (psi == 0.0) break;
    double dn = d - psi / dpsi;
    // converged: the Newton correction is below the resolution of d (tested
    // before the bracket test, since a converged step may land on the
    // bracket end it has just set)
    if (fabs(dn - d) <= 4.0 * 2.220446049250313e-16 * d) {
      d = dn;
      break;
    }
    if (!(dn > lo && dn < hi)) dn = isfinite(hi) ? 0.5 * (lo + hi) : 2.0 * fmax(d, lo);
    if (isfinite(hi) && hi - lo <= 4.0 * 2.220446049250313e-16 * hi) {
      d = dn;
      break;
    }
    d = dn;
  }
  if (warm && lane == 0) *warm = d;
  out.lam = mt - sg * d;
  out.tval = mt * art / d;
  return out;
}

__device__ __forceinline__ double soc_out_v(const SocSol& s, double r, double m) {
  switch (s.kind) {
    case 0: return r;
    case 1: return 0.0;
    case 2: return s.fac * r;
    default: return m * r / (m + s.lam);
  }
}

__device__ __forceinline__ double soc_out_t(const SocSol& s, double rt) {
  return s.kind == 0 ? rt : (s.kind == 1 ? 0.0 : s.tval);
}

// Input views.  Src provides r(j) (pre-projection value) and m(j) (metric)
// for block-local coordinates j.
template <class Src>
struct SocView {
  const Src& src;
  int dim;
  __device__ int dimv() const { return dim - 1; }
  __device__ double rv(int j) const { return src.r(j); }
  __device__ double mv(int j) const { return src.m(j); }
  __device__ double rt() const { return src.r(dim - 1); }
  __device__ double mt() const { return src.m(dim - 1); }
};

template <class Src>
struct RsocView {
  const Src& src;
  int dim;
  double q, sq, rn, rp;   // q = sqrt(ms mt), sq = sqrt(q)
  __device__ int dimv() const { return dim - 1; }
  __device__ double rv(int j) const { return j < dim - 2 ? sq * src.r(j) : rn; }
  __device__ double mv(int j) const { return j < dim - 2 ? src.m(j) / q : 1.0; }
  __device__ double rt() const { return rp; }
  __device__ double mt() const { return 1.0; }
};

// Project block [0, dim) of Src onto SOC (type 2) or RSOC (type 3) with an
// aligned group of Lg lanes (16, 32 or 64); the result for local coordinate j
// is delivered to sink(j, value).  Every lane of the group must call this
// with identical arguments; other groups of the wave may work on other
// blocks (all reductions stay inside the group).  warm (nullable)
// holds the previous root of this block and receives the new one.
template <class Src, class Sink>
__device__ __noinline__ void project_wave_item(int type, int dim, bool euclid, Src src, Sink sink,
                                               double* warm, int Lg) {
  const int lane = threadIdx.x & (Lg - 1);
  if (type == 2) {
    SocView<Src> view{src, dim};
    SocSol s = soc_wave_solve(view, euclid, warm, Lg);
    for (int j = lane; j < dim - 1; j += Lg) sink(j, soc_out_v(s, src.r(j), src.m(j)));
    if (lane == ((dim - 1) & (Lg - 1))) sink(dim - 1, soc_out_t(s, src.r(dim - 1)));
    return;
  }
  // RSOC
  const double rs = src.r(dim - 2), rtt = src.r(dim - 1);
  double ms = 1.0, mtt = 1.0;
  if (!euclid) { ms = src.m(dim - 2); mtt = src.m(dim - 1); }
  const double sms = sqrt(ms), smt = sqrt(mtt);
  const double q = sms * smt;
  const double h = 0.70710678118654752440;
  RsocView<Src> view{src, dim, q, sqrt(q), (sms * rs - smt * rtt) * h, (sms * rs + smt * rtt) * h};
  SocSol s = soc_wave_solve(view, euclid, warm, Lg);
  for (int j = lane; j < dim - 2; j += Lg) {
    double vp = soc_out_v(s, view.rv(j), view.mv(j));
    sink(j, s.kind == 0 ? src.r(j) : vp / view.sq);
  }
  if (lane == 0) {
    double nout = soc_out_v(s, view.rn, 1.0);
    double pout = soc_out_t(s, view.rp);
    double so, to;
    if (s.kind == 0) { so = rs; to = rtt; }
    else {
      so = (pout + nout) * h / sms;
      to = (pout - nout) * h / smt;
    }
    sink(dim - 2, so);
    sink(dim - 1, to);
  }
}

// ---------------------------------------------------------------------------
// EXP on one lane
// ---------------------------------------------------------------------------
__device__ __forceinline__ bool exp_in_cone(double r, double s, double t) {
  if (s > 0.0) {
    double q = r / s;
    if (q > 709.0) return false;
    return s * exp(q) <= t;
  }
  if (s == 0.0) return r <= 0.0 && t >= 0.0;
  return false;
}

// dual cone cl{(a, b, c): a < 0, -a e^{b/a} <= e c}
__device__ __forceinline__ bool exp_in_dual(double a, double b, double c) {
  if (a < 0.0) {
    double q = b / a;
    if (q > 709.0) return false;
    return -a * exp(q) <= 2.718281828459045235 * c;
  }
  if (a == 0.0) return b >= 0.0 && c >= 0.0;
  return false;
}

struct ExpData {
  double r0, s0, t0, mr, ms, mt;
};

// sign-carrying H = h_M * Den (scaled by e^{-2 rho} for rho > 0), and the
// point eta (rho, 1, e^rho)
__device__ __forceinline__ double exp_H(const ExpData& e, double rho) {
  if (rho > 0.0) {
    double em = exp(-rho);
    double em2 = em * em;
    return e.mt * (e.mr * e.r0 * (rho - 1.0) + e.ms * e.s0)
         - e.mt * e.t0 * em * (e.mr * rho * (rho - 1.0) + e.ms)
         + e.mr * e.ms * (rho * e.s0 - e.r0) * em2;
  }
  double x = exp(rho);
  return e.mt * x * x * (e.mr * e.r0 * (rho - 1.0) + e.ms * e.s0)
       - e.mt * e.t0 * x * (e.mr * rho * (rho - 1.0) + e.ms)
       + e.mr * e.ms * (rho * e.s0 - e.r0);
}

__device__ __forceinline__ void exp_point(const ExpData& e, double rho, double out[3]) {
  double eta, eta_e;
  if (rho > 0.0) {
    double em = exp(-rho);
    double em2 = em * em;
    double num = e.mr * rho * e.r0 * em2 + e.ms * e.s0 * em2 + e.mt * e.t0 * em;
    double den = e.mr * rho * rho * em2 + e.ms * em2 + e.mt;
    eta = num / den;
    eta_e = (e.mr * rho * e.r0 * em + e.ms * e.s0 * em + e.mt * e.t0) / den;
  } else {
    double x = exp(rho);
    double num = e.mr * rho * e.r0 + e.ms * e.s0 + e.mt * x * e.t0;
    double den = e.mr * rho * rho + e.ms + e.mt * x * x;
    eta = num / den;
    eta_e = eta * x;
  }
  out[0] = eta * rho;
  out[1] = eta;
  out[2] = eta_e;
}

// psi(rho) - t0 with psi(rho) = e^rho (r0 + (1 - rho) s0); sign only for rho > 700
__device__ __forceinline__ double exp_vis(const ExpData& e, double rho) {
  double f = e.r0 + (1.0 - rho) * e.s0;
  if (rho > 700.0) return f > 0.0 ? INFINITY : (f < 0.0 ? -INFINITY : -e.t0);
  return exp(rho) * f - e.t0;
}

// N(rho) = m_r rho r0 + m_s s0 + m_t t0 e^rho (numerator of eta)
__device__ __forceinline__ double exp_N(const ExpData& e, double rho) {
  if (rho > 700.0) {
    if (e.t0 != 0.0) return e.t0 > 0.0 ? INFINITY : -INFINITY;
    return e.mr * rho * e.r0 + e.ms * e.s0;
  }
  return e.mr * rho * e.r0 + e.ms * e.s0 + e.mt * e.t0 * exp(rho);
}

constexpr double RHO_LIM = 1.0e100;

// H and dH/drho (both divided by e^{2 rho} for rho > 0)
__device__ __forceinline__ void exp_H_d(const ExpData& e, double rho, double& H, double& dH) {
  const double A = e.mr * e.r0 * (rho - 1.0) + e.ms * e.s0;
  const double B = e.mr * rho * (rho - 1.0) + e.ms;
  const double Cc = rho * e.s0 - e.r0;
  const double dB = e.mr * (2.0 * rho - 1.0);
  if (rho > 0.0) {
    const double em = exp(-rho), em2 = em * em;
    H = e.mt * A - e.mt * e.t0 * em * B + e.mr * e.ms * Cc * em2;
    dH = e.mt * e.mr * e.r0 - e.mt * e.t0 * em * (dB - B) + e.mr * e.ms * em2 * (e.s0 - 2.0 * Cc);
  } else {
    const double x = exp(rho), x2 = x * x;
    H = e.mt * x2 * A - e.mt * e.t0 * x * B + e.mr * e.ms * Cc;
    dH = e.mt * x2 * (2.0 * A + e.mr * e.r0) - e.mt * e.t0 * x * (B + dB) + e.mr * e.ms * e.s0;
  }
}

// f(kind, rho) and its derivative: 0 -> H (scaled), 1 -> vis, 2 -> N
__device__ __forceinline__ double exp_f(const ExpData& e, int kind, double rho) {
  return kind == 0 ? exp_H(e, rho) : (kind == 1 ? exp_vis(e, rho) : exp_N(e, rho));
}

__device__ __forceinline__ double exp_df(const ExpData& e, int kind, double rho) {
  if (kind == 0) {
    double H, dH;
    exp_H_d(e, rho, H, dH);
    return dH;
  }
  if (rho > 700.0) return NAN;
  const double x = exp(rho);
  return kind == 1 ? x * (e.r0 - rho * e.s0) : e.mr * e.r0 + e.mt * e.t0 * x;
}

// sign change of f on [lo, hi] (`inc`: negative at lo): Newton steps inside
// the bracket, bisection when a step leaves it or stalls
__device__ double exp_bisect(const ExpData& e, int kind, double lo, double hi, bool inc) {
  double x = 0.5 * (lo + hi);
  double prev = INFINITY;
  for (int it = 0; it < 3000; ++it) {
    if (!(lo < hi) || hi - lo <= 8.881784197001252e-16 * fmax(1.0, fabs(x))) break;
    const double v = exp_f(e, kind, x);
    if (v == 0.0) return x;
    if ((v < 0.0) == inc) lo = x; else hi = x;
    const double dv = exp_df(e, kind, x);
    double xn = (isfinite(dv) && dv != 0.0) ? x - v / dv : NAN;
    if (fabs(xn - x) <= 4.0 * 2.220446049250313e-16 * fmax(1.0, fabs(x))) return xn;   // converged
    const double mid = 0.5 * (lo + hi);
    if (!(xn > lo && xn < hi) || fabs(xn - x) > 0.5 * prev) xn = mid;
    prev = fabs(xn - x);
    x = xn;
  }
  return 0.5 * (lo + hi);
}

// walk from x0 in direction dir with doubling steps until f has the wanted
// sign; returns the point or the limit (+-RHO_LIM)
__device__ double exp_walk(const ExpData& e, int kind, double x0, double dir, bool want_pos) {
  double step = 1.0;
  for (int it = 0; it < 400; ++it) {
    double x = x0 + dir * step;
    if (dir > 0.0 ? x >= RHO_LIM : x <= -RHO_LIM) return dir * RHO_LIM;
    double v = exp_f(e, kind, x);
    if ((v > 0.0) == want_pos) return x;
    step *= 2.0;
  }
  return dir * RHO_LIM;
}

struct Ival {
  double lo, hi;
};

// components of the visible set {rho: psi(rho) > t0}; at most 2
__device__ int exp_visible(const ExpData& e, Ival out[2]) {
  const double inf = INFINITY;
  if (e.s0 > 0.0) {
    double rm = e.r0 / e.s0;
    double b = exp_bisect(e, 1, rm, exp_walk(e, 1, rm, 1.0, false), false);
    if (e.t0 > 0.0) {
      double a = exp_bisect(e, 1, exp_walk(e, 1, rm, -1.0, false), rm, true);
      out[0] = {a, b};
    } else {
      out[0] = {-inf, b};
    }
    return 1;
  }
  if (e.s0 == 0.0) {
    out[0] = e.t0 > 0.0 ? Ival{log(e.t0 / e.r0), inf} : Ival{-inf, inf};
    return 1;
  }
  double rm = e.r0 / e.s0;
  double b = exp_bisect(e, 1, rm, exp_walk(e, 1, rm, 1.0, true), true);
  if (e.t0 >= 0.0) { out[0] = {b, inf}; return 1; }
  if (exp_vis(e, rm) >= 0.0) { out[0] = {-inf, inf}; return 1; }
  double a = exp_bisect(e, 1, exp_walk(e, 1, rm, -1.0, true), rm, false);
  out[0] = {-inf, a};
  out[1] = {b, inf};
  return 2;
}

// components of {rho: N(rho) > 0}; at most 2
__device__ int exp_positive(const ExpData& e, Ival out[2]) {
  const double inf = INFINITY;
  if (e.t0 == 0.0) {
    if (e.r0 > 0.0) { out[0] = {-e.ms * e.s0 / (e.mr * e.r0), inf}; return 1; }
    if (e.r0 < 0.0) { out[0] = {-inf, -e.ms * e.s0 / (e.mr * e.r0)}; return 1; }
    if (e.s0 > 0.0) { out[0] = {-inf, inf}; return 1; }
    return 0;
  }
  if (e.t0 < 0.0) {
    if (e.r0 <= 0.0) {
      if (e.r0 == 0.0) {
        if (e.s0 <= 0.0) return 0;
        out[0] = {-inf, log(e.ms * e.s0 / (-e.mt * e.t0))};
        return 1;
      }
      double hi = exp_walk(e, 2, 0.0, 1.0, false);
      double lo = exp_walk(e, 2, 0.0, -1.0, true);
      if (exp_N(e, lo) <= 0.0) return 0;
      out[0] = {-inf, exp_bisect(e, 2, lo, hi, false)};
      return 1;
    }
    double xm = log(e.mr * e.r0 / (-e.mt * e.t0));
    if (exp_N(e, xm) <= 0.0) return 0;
    double a = exp_bisect(e, 2, exp_walk(e, 2, xm, -1.0, false), xm, true);
    double b = exp_bisect(e, 2, xm, exp_walk(e, 2, xm, 1.0, false), false);
    out[0] = {a, b};
    return 1;
  }
  if (e.r0 >= 0.0) {
    if (e.r0 == 0.0) {
      out[0] = e.s0 >= 0.0 ? Ival{-inf, inf} : Ival{log(-e.ms * e.s0 / (e.mt * e.t0)), inf};
      return 1;
    }
    double lo = exp_walk(e, 2, 0.0, -1.0, false);
    if (exp_N(e, lo) > 0.0) { out[0] = {-inf, inf}; return 1; }
    out[0] = {exp_bisect(e, 2, lo, exp_walk(e, 2, 0.0, 1.0, true), true), inf};
    return 1;
  }
  double xm = log(e.mr * e.r0 / (-e.mt * e.t0));
  if (exp_N(e, xm) > 0.0) { out[0] = {-inf, inf}; return 1; }
  double a = exp_bisect(e, 2, exp_walk(e, 2, xm, -1.0, true), xm, false);
  double b = exp_bisect(e, 2, xm, exp_walk(e, 2, xm, 1.0, true), true);
  out[0] = {-inf, a};
  out[1] = {b, inf};
  return 2;
}

// Newton on H from rho0.  A root at which eta_M > 0 (N > 0) and the ray is
// visible from r (psi > t0) is the projection (the normal M(r - u) then
// points outward, so u satisfies the projection's optimality conditions);
// anything else is rejected and the caller falls back to the bracket search.
__device__ bool exp_newton(const ExpData& e, double rho, double out[3], double* warm) {
  for (int it = 0; it < 60; ++it) {
    double H, dH;
    exp_H_d(e, rho, H, dH);
    if (!(dH != 0.0) || !isfinite(H) || !isfinite(dH)) return false;
    double step = H / dH;
    const double cap = fmax(2.0, 0.5 * fabs(rho));
    if (step > cap) step = cap;
    if (step < -cap) step = -cap;
    const double rn = rho - step;
    if (fabs(rn - rho) <= 4.0 * 2.220446049250313e-16 * fmax(1.0, fabs(rho))) {
      rho = rn;
      if (!(exp_N(e, rho) > 0.0) || !(exp_vis(e, rho) > 0.0)) return false;
      exp_point(e, rho, out);
      if (!(out[1] >= 0.0 && isfinite(out[0]) && isfinite(out[2]))) return false;
      if (warm) *warm = rho;
      return true;
    }
    rho = rn;
    if (fabs(rho) > 700.0) return false;
  }
  return false;
}

// diagnostics: the inputs of the first cone projection of a solve whose
// root-finding failed, and the number of failures (read by the host with
// pdhcg_last_cone_failure; reset before every solve)
__device__ double g_cone_fail[8];
__device__ unsigned int g_cone_fail_count;

__device__ void note_cone_failure(int type, double a, double b, double c, double ma, double mb, double mc,
                                  double al) {
  if (atomicAdd(&g_cone_fail_count, 1u) == 0u) {
    g_cone_fail[0] = (double)type;
    g_cone_fail[1] = a;
    g_cone_fail[2] = b;
    g_cone_fail[3] = c;
    g_cone_fail[4] = ma;
    g_cone_fail[5] = mb;
    g_cone_fail[6] = mc;
    g_cone_fail[7] = al;
  }
}

__device__ __forceinline__ void project_exp_body(double r0, double s0, double t0, double mr, double ms,
                                                 double mt, double out[3], double* warm) {
  if (exp_in_cone(r0, s0, t0)) { out[0] = r0; out[1] = s0; out[2] = t0; return; }
  if (exp_in_dual(-mr * r0, -ms * s0, -mt * t0)) { out[0] = out[1] = out[2] = 0.0; return; }
  if (r0 <= 0.0 && s0 <= 0.0) { out[0] = r0; out[1] = 0.0; out[2] = fmax(t0, 0.0); return; }
  ExpData e{r0, s0, t0, mr, ms, mt};
  {
    // start: the previous root of this block, else the ratio of r itself when
    // s0 > 0, else the boundary ratio log(t0 / r0) of the t-r face
    double rho0 = 0.0;
    if (s0 > 0.0) rho0 = fmin(fmax(r0 / s0, -50.0), 50.0);
    else if (t0 > 0.0 && r0 > 0.0) rho0 = fmin(fmax(log(t0 / r0), -50.0), 50.0);
    double rho_w = warm ? *warm : NAN;
    if (isfinite(rho_w) && exp_newton(e, rho_w, out, warm)) return;
    if (exp_newton(e, rho0, out, warm)) return;
  }
  Ival V[2], Np[2];
  int nv = exp_visible(e, V);
  int nn = exp_positive(e, Np);
  double fallback = NAN;
  for (int i = 0; i < nv; ++i)
    for (int j = 0; j < nn; ++j) {
      double lo = fmax(V[i].lo, Np[j].lo), hi = fmin(V[i].hi, Np[j].hi);
      if (!(lo < hi)) continue;
      bool lfin = isfinite(lo), hfin = isfinite(hi);
      if (!lfin && !hfin) {
        if (exp_H(e, 0.0) < 0.0) { lo = 0.0; hi = exp_walk(e, 0, 0.0, 1.0, true); }
        else { hi = 0.0; lo = exp_walk(e, 0, 0.0, -1.0, false); }
      } else if (!lfin) {
        if (!(exp_H(e, hi) > 0.0)) continue;
        lo = exp_walk(e, 0, hi, -1.0, false);
      } else if (!hfin) {
        if (!(exp_H(e, lo) < 0.0)) continue;
        hi = exp_walk(e, 0, lo, 1.0, true);
      } else if (!(exp_H(e, lo) < 0.0 && exp_H(e, hi) > 0.0)) {
        continue;
      }
      if (fabs(lo) >= RHO_LIM || fabs(hi) >= RHO_LIM) {
        if (isnan(fallback)) fallback = fabs(lo) >= RHO_LIM ? lo : hi;
        continue;
      }
      double rho = exp_bisect(e, 0, lo, hi, true);
      exp_point(e, rho, out);
      if (out[1] >= 0.0) {
        if (warm) *warm = rho;
        return;
      }
    }
  if (!isnan(fallback)) {
    exp_point(e, fallback, out);
    if (out[1] >= 0.0) return;
  }
  {
    // no admissible root survives in floating point: when -M r lies within
    // rounding of the boundary of K^* (the dual slack of a solved block sits
    // there), the projection is 0 to rounding, since |Pi(r)| = dist(r, -K^*)
    const double a = -mr * r0, b = -ms * s0, c = -mt * t0;
    if (a < 0.0) {
      const double lhs = -a * exp(b / a), rhs = 2.718281828459045 * c;
      if (lhs - rhs <= 1e-12 * (fabs(lhs) + fabs(rhs))) {
        out[0] = out[1] = out[2] = 0.0;
        return;
      }
    }
  }
  note_cone_failure(PDHCG_CONE_EXP, r0, s0, t0, mr, ms, mt, 0.0);
  out[0] = out[1] = out[2] = NAN;   // reported as a numerical failure
}

// ---------------------------------------------------------------------------
// POW on one lane
// ---------------------------------------------------------------------------
__device__ __forceinline__ double pow_qroot(double s, double c) {
  double d = sqrt(s * s + 4.0 * c);
  return s >= 0.0 ? 0.5 * (s + d) : 2.0 * c / (d - s);
}

__device__ __forceinline__ void project_pow_body(double x, double y, double z, double al, double mx, double my,
                                                 double mz, double out[3], double* warm) {
  if (z == 0.0) { out[0] = fmax(x, 0.0); out[1] = fmax(y, 0.0); out[2] = 0.0; return; }
  if (x >= 0.0 && y >= 0.0 && pow(x, al) * pow(y, 1.0 - al) >= fabs(z)) {
    out[0] = x; out[1] = y; out[2] = z; return;
  }
  {
    double p = -mx * x, q = -my * y, w = -mz * z;
    if (p >= 0.0 && q >= 0.0 && pow(p / al, al) * pow(q / (1.0 - al), 1.0 - al) >= fabs(w)) {
      out[0] = out[1] = out[2] = 0.0;
      return;
    }
  }
  const double R = fabs(z);
  const double cx = al * mz / mx, cy = (1.0 - al) * mz / my;
  // g_M is positive left of its unique root in (0, R) and negative right of
  // it; Newton steps are taken inside the sign bracket, bisection otherwise.
  double lo = 0.0, hi = R;
  const double tol = 1e-15 * fmax(1.0, R);
  double rho = 0.5 * R;
  if (warm && *warm > 0.0 && *warm < R) rho = *warm;
  for (int it = 0; it < 3000 && hi - lo > tol; ++it) {
    const double w = rho * (R - rho), dw = R - 2.0 * rho;
    const double xv = pow_qroot(x, cx * w), yv = pow_qroot(y, cy * w);
    double g, dg = 0.0;
    if (xv > 0.0 && yv > 0.0) {
      g = al * log(xv) + (1.0 - al) * log(yv) - log(rho);
      const double dx = cx * dw / (2.0 * xv - x), dy = cy * dw / (2.0 * yv - y);
      dg = al * dx / xv + (1.0 - al) * dy / yv - 1.0 / rho;
    } else {
      g = -INFINITY;
    }
    if (g > 0.0) lo = rho;
    else if (g < 0.0) hi = rho;
    else { lo = hi = rho; break; }
    double rn = (isfinite(g) && dg < 0.0) ? rho - g / dg : 0.5 * (lo + hi);
    if (fabs(rn - rho) <= 2.220446049250313e-16 * rho) { lo = hi = rn; break; }   // converged
    if (!(rn > lo && rn < hi)) rn = 0.5 * (lo + hi);
    rho = rn;
  }
  rho = 0.5 * (lo + hi);
  if (warm) *warm = rho;
  const double w = rho * (R - rho);
  out[0] = pow_qroot(x, cx * w);
  out[1] = pow_qroot(y, cy * w);
  out[2] = copysign(rho, z);
}

// ---------------------------------------------------------------------------
// EXP block with the middle coordinate fixed at one, on one lane: the point
// (z0, ., t0) projected onto {(z, 1, t): e^z <= t} in the metric (mz, ., mt).
// Outside the set the projection is (z, 1, e^z) at the root of
// f(z) = mz (z - z0) + mt (e^z - t0) e^z (stationarity on the boundary with
// multiplier mt (e^z - t0) >= 0); f increases where e^z >= t0, is positive
// at z0 and negative at log t0 (t0 > 0) or far enough below z0.  Safeguarded
// Newton inside the sign bracket.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double exp1_f(double z, double z0, double t0, double mz, double mt, double& df) {
  const double ez = exp(z);
  df = mz + mt * ez * (2.0 * ez - t0);
  return mz * (z - z0) + mt * (ez - t0) * ez;
}

__device__ __forceinline__ void project_exp1_body(double z0, double t0, double mz, double mt, double out[3]) {
  out[1] = 1.0;
  if (z0 <= 709.0 && exp(z0) <= t0) { out[0] = z0; out[2] = t0; return; }
  double hi = fmin(z0, 709.0), lo, d;
  if (t0 > 0.0) {
    lo = fmin(log(t0), hi);
  } else {
    double step = 1.0;
    lo = hi - step;
    while (exp1_f(lo, z0, t0, mz, mt, d) >= 0.0 && step < 1e300) {
      step *= 2.0;
      lo = hi - step;
    }
  }
  // at the root mz (z0 - z) = mt (e^z - t0) e^z >= mt (e^z - t0+)^2 with
  // z >= lo, so e^z <= t0+ + sqrt((mz/mt)(z0 - lo)): a tight upper end (from
  // z0 itself Newton would creep down by about 1/2 per step where the
  // e^(2z) term dominates)
  hi = fmin(hi, log(fmax(t0, 0.0) + sqrt((mz / mt) * (z0 - lo))));
  if (hi < lo) hi = lo;
  double z = hi;
  const double tol = 1e-15 * fmax(1.0, fabs(hi));
  for (int it = 0; it < 2000 && hi - lo > tol; ++it) {
    const double fz = exp1_f(z, z0, t0, mz, mt, d);
    if (fz > 0.0) hi = z;
    else if (fz < 0.0) lo = z;
    else { lo = hi = z; break; }
    double zn = (d > 0.0) ? z - fz / d : 0.5 * (lo + hi);
    if (fabs(zn - z) <= 2.220446049250313e-16 * fmax(1.0, fabs(z))) { lo = hi = zn; break; }   // converged
    if (!(zn > lo && zn < hi)) zn = 0.5 * (lo + hi);
    z = zn;
  }
  z = 0.5 * (lo + hi);
  out[0] = z;
  out[2] = exp(z);
}

// Out-of-line entry points (one copy of each root-finder in the code, kept
// apart from the register allocation of the solver loop); the projected
// point comes back in registers, not through the caller's stack.
struct Trip {
  double a, b, c;
};

__device__ __noinline__ Trip project_exp(double r0, double s0, double t0, double mr, double ms, double mt,
                                         double* warm) {
  double o[3];
  project_exp_body(r0, s0, t0, mr, ms, mt, o, warm);
  return Trip{o[0], o[1], o[2]};
}

__device__ __noinline__ Trip project_pow(double x, double y, double z, double al, double mx, double my,
                                         double mz, double* warm) {
  double o[3];
  project_pow_body(x, y, z, al, mx, my, mz, o, warm);
  return Trip{o[0], o[1], o[2]};
}

// the fixed-middle EXP block kappa X in scaled coordinates (kappa the
// block's common scale): kappa Pi^M_X(r / kappa)
__device__ __forceinline__ Trip project_exp1(double z0, double t0, double mz, double mt, double kappa) {
  double o[3];
  project_exp1_body(z0 / kappa, t0 / kappa, mz, mt, o);
  return Trip{kappa * o[0], kappa * o[1], kappa * o[2]};
}

}  // namespace pdhcg
