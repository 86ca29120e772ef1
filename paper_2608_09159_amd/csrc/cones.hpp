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

__device__ __forceinline__ double wave_sum(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v += __shfl_xor(v, o, 64);
  return v;
}

__device__ __forceinline__ double wave_max(double v) {
#pragma unroll
  for (int o = 32; o > 0; o >>= 1) v = fmax(v, __shfl_xor(v, o, 64));
  return v;
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
__device__ SocSol soc_wave_solve(const In& in, bool euclid) {
  const int lane = threadIdx.x & 63;
  const double rt = in.rt(), mt = in.mt();
  const int dv = in.dimv();
  double nv2 = 0.0, nmv2 = 0.0;
  for (int j = lane; j < dv; j += 64) {
    double r = in.rv(j);
    double mr = in.mv(j) * r;
    nv2 += r * r;
    nmv2 += mr * mr;
  }
  nv2 = wave_sum(nv2);
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
  nmv2 = wave_sum(nmv2);
  if (sqrt(nmv2) <= -mt * rt) { out.kind = 1; return out; }
  out.kind = 3;
  if (rt == 0.0) {                      // singular case lam = m_t
    double s2 = 0.0;
    for (int j = lane; j < dv; j += 64) {
      double m = in.mv(j);
      double vj = m * in.rv(j) / (m + mt);
      s2 += vj * vj;
    }
    out.lam = mt;
    out.tval = sqrt(wave_sum(s2));
    return out;
  }
  const double sg = rt > 0.0 ? 1.0 : -1.0;
  const double art = fabs(rt);
  auto eval = [&](double d, double& psi, double& dpsi) {
    double s2 = 0.0, s3 = 0.0;
    const double base = mt - sg * d;
    for (int j = lane; j < dv; j += 64) {
      double m = in.mv(j);
      double den = m + base;
      double vj = m * in.rv(j) / den;
      s2 += vj * vj;
      s3 += vj * vj / den;
    }
    s2 = wave_sum(s2);
    s3 = wave_sum(s3);
    double nv = sqrt(s2);
    psi = d * nv - mt * art;
    dpsi = nv + (nv > 0.0 ? d * sg * s3 / nv : 0.0);
  };
  double lo = 0.0, hi = mt, psi, dpsi;
  if (sg < 0.0) {
    for (int it = 0; it < 2100; ++it) {
      eval(hi, psi, dpsi);
      if (psi > 0.0) break;
      lo = hi;
      hi *= 2.0;
    }
  }
  double d = 0.5 * (lo + hi);
  for (int it = 0; it < 300; ++it) {
    eval(d, psi, dpsi);
    if (psi < 0.0) lo = d; else hi = d;
    if (psi == 0.0) break;
    double dn = d - psi / dpsi;
    if (!(dn > lo && dn < hi)) dn = 0.5 * (lo + hi);
    if (fabs(dn - d) <= 4.0 * 2.220446049250313e-16 * d || hi - lo <= 4.0 * 2.220446049250313e-16 * hi) {
      d = dn;
      break;
    }
    d = dn;
  }
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

// Project block [0, dim) of Src onto SOC (type 2) or RSOC (type 3); the
// result for local coordinate j is delivered to sink(j, value).  Every lane
// of the wave must call this with identical arguments.
template <class Src, class Sink>
__device__ void project_wave_item(int type, int dim, bool euclid, const Src& src, Sink sink) {
  const int lane = threadIdx.x & 63;
  if (type == 2) {
    SocView<Src> view{src, dim};
    SocSol s = soc_wave_solve(view, euclid);
    for (int j = lane; j < dim - 1; j += 64) sink(j, soc_out_v(s, src.r(j), src.m(j)));
    if (lane == ((dim - 1) & 63)) sink(dim - 1, soc_out_t(s, src.r(dim - 1)));
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
  SocSol s = soc_wave_solve(view, euclid);
  for (int j = lane; j < dim - 2; j += 64) {
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

// f(kind, rho): 0 -> H, 1 -> vis, 2 -> N
__device__ __forceinline__ double exp_f(const ExpData& e, int kind, double rho) {
  return kind == 0 ? exp_H(e, rho) : (kind == 1 ? exp_vis(e, rho) : exp_N(e, rho));
}

// bisection for a sign change of f on [lo, hi]; `inc` means negative at lo
__device__ double exp_bisect(const ExpData& e, int kind, double lo, double hi, bool inc) {
  for (int it = 0; it < 3000; ++it) {
    double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi || hi - lo <= 8.881784197001252e-16 * fmax(1.0, fabs(mid))) break;
    double v = exp_f(e, kind, mid);
    if ((v < 0.0) == inc) lo = mid; else hi = mid;
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

__device__ __noinline__ void project_exp(double r0, double s0, double t0, double mr, double ms, double mt,
                            double out[3]) {
  if (exp_in_cone(r0, s0, t0)) { out[0] = r0; out[1] = s0; out[2] = t0; return; }
  if (exp_in_dual(-mr * r0, -ms * s0, -mt * t0)) { out[0] = out[1] = out[2] = 0.0; return; }
  if (r0 <= 0.0 && s0 <= 0.0) { out[0] = r0; out[1] = 0.0; out[2] = fmax(t0, 0.0); return; }
  ExpData e{r0, s0, t0, mr, ms, mt};
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
      if (out[1] >= 0.0) return;
    }
  if (!isnan(fallback)) {
    exp_point(e, fallback, out);
    if (out[1] >= 0.0) return;
  }
  out[0] = out[1] = out[2] = NAN;   // reported as a numerical failure
}

// ---------------------------------------------------------------------------
// POW on one lane
// ---------------------------------------------------------------------------
__device__ __forceinline__ double pow_qroot(double s, double c) {
  double d = sqrt(s * s + 4.0 * c);
  return s >= 0.0 ? 0.5 * (s + d) : 2.0 * c / (d - s);
}

__device__ __noinline__ void project_pow(double x, double y, double z, double al, double mx, double my,
                            double mz, double out[3]) {
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
  double lo = 0.0, hi = R;
  const double tol = 1e-15 * fmax(1.0, R);
  for (int it = 0; it < 3000 && hi - lo > tol; ++it) {
    double mid = 0.5 * (lo + hi);
    double w = mid * (R - mid);
    double xv = pow_qroot(x, cx * w), yv = pow_qroot(y, cy * w);
    double g = (xv > 0.0 && yv > 0.0) ? al * log(xv) + (1.0 - al) * log(yv) - log(mid) : -INFINITY;
    if (g > 0.0) lo = mid;
    else if (g < 0.0) hi = mid;
    else { lo = hi = mid; break; }
  }
  const double rho = 0.5 * (lo + hi);
  const double w = rho * (R - rho);
  out[0] = pow_qroot(x, cx * w);
  out[1] = pow_qroot(y, cy * w);
  out[2] = copysign(rho, z);
}

}  // namespace pdhcg
