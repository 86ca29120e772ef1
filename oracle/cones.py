"""Projections onto the cones of the paper's Appendix C, in the Euclidean norm
and in the diagonal M-norm of eq. metric-block-projection,
    Pi^M_C(r) = argmin_{u in C} 1/2 ||u - r||_M^2,   M = diag(m) > 0.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Coordinate order (Section "Practical Implementation", the cone list):
    SOC   (v, t)      ||v|| <= t
    RSOC  (v, s, t)   ||v||^2 <= 2 s t,  s, t >= 0
    EXP   (r, s, t)   cl{ s > 0, s exp(r/s) <= t }
    POW   (x, y, z)   x, y >= 0,  x^a y^(1-a) >= |z|

Pins (tests/test_oracle_cones.py): the KKT characterisation of Pi^M_K
(u in K, M(u - r) in K*, <u, M(u - r)> = 0) on random and adversarial inputs;
M = cI reduces to the Euclidean projection; the closed forms printed in
Appendix C (box/R+, SOC, RSOC through the rotation U, the SOC r_t = 0 case,
the RSOC singular case, the EXP r0 <= 0, s0 <= 0 case, the POW r_z = 0 case);
POW with alpha = 1/2 against the RSOC M-norm projection; brute force over
boundary points for tiny inputs; the EXP closest-point fallback (used only
where the root bracket degenerates, next to the polar cone) against the root
method on generic inputs, and near-polar inputs projecting to ~0.

Membership tests are exact floating-point comparisons; the projection is
continuous, so a borderline decision changes the result only at rounding
level.
"""
from __future__ import annotations

import math

import numpy as np

EPS = 2.0 ** -52
E_CONST = math.e
RHO_MAX = 1.0e100     # search range for the EXP ratio rho = r/s; rho^2 stays
RHO_MIN = -1.0e100    # finite and e^{-rho} underflows gracefully


# ----------------------------------------------------------------------------
# membership and dual cones
# ----------------------------------------------------------------------------
def in_soc(u):
    u = np.asarray(u, dtype=float)
    return bool(np.linalg.norm(u[:-1]) <= u[-1])


def in_rsoc(u):
    u = np.asarray(u, dtype=float)
    v, s, t = u[:-2], u[-2], u[-1]
    return bool(s >= 0 and t >= 0 and float(v @ v) <= 2.0 * s * t)


def in_exp(u):
    r, s, t = (float(a) for a in u)
    if s > 0:
        q = r / s
        if q > 709.0:
            return False
        return s * math.exp(q) <= t
    if s == 0:
        return r <= 0 and t >= 0
    return False


def in_exp_dual(u):
    """K_exp^* = cl{(a, b, c): a < 0, -a exp(b/a) <= e c}; derived from the
    EXP cone definition of the implementation section (the paper does not
    print it): its boundary rays are -grad(s e^{r/s} - t) at boundary rays of
    K_exp."""
    a, b, c = (float(x) for x in u)
    if a < 0:
        q = b / a
        if q > 709.0:
            return False
        return -a * math.exp(q) <= E_CONST * c
    if a == 0:
        return b >= 0 and c >= 0
    return False


def in_pow(u, alpha):
    x, y, z = (float(a) for a in u)
    if x < 0 or y < 0:
        return False
    return (x ** alpha) * (y ** (1.0 - alpha)) >= abs(z)


def in_pow_dual(u, alpha):
    """Dual power cone as printed in Appendix C (three-dimensional power
    cone subsection)."""
    p, q, w = (float(a) for a in u)
    if p < 0 or q < 0:
        return False
    return (p / alpha) ** alpha * (q / (1.0 - alpha)) ** (1.0 - alpha) >= abs(w)


def in_cone(kind, u, alpha=0.0):
    if kind == "free":
        return True
    if kind == "nonneg":
        return bool(np.all(np.asarray(u) >= 0))
    if kind == "soc":
        return in_soc(u)
    if kind == "rsoc":
        return in_rsoc(u)
    if kind == "exp":
        return in_exp(u)
    if kind == "pow":
        return in_pow(u, alpha)
    raise ValueError(kind)


def in_dual_cone(kind, u, alpha=0.0):
    """SOC and RSOC are self-dual; the free cone's dual is {0}."""
    if kind == "free":
        return bool(np.all(np.asarray(u) == 0))
    if kind in ("nonneg", "soc", "rsoc"):
        return in_cone(kind, u, alpha)
    if kind == "exp":
        return in_exp_dual(u)
    if kind == "pow":
        return in_pow_dual(u, alpha)
    raise ValueError(kind)


# ----------------------------------------------------------------------------
# SOC
# ----------------------------------------------------------------------------
def soc_euclid(R):
    """Closed form of eq. soc-euclidean-projection, row-wise on R (k x d)."""
    R = np.atleast_2d(np.asarray(R, dtype=float))
    V, T = R[:, :-1], R[:, -1]
    a = np.linalg.norm(V, axis=1)
    out = np.zeros_like(R)
    keep = a <= T
    out[keep] = R[keep]
    mid = ~keep & ~(a <= -T)
    if np.any(mid):
        f = 0.5 * (a[mid] + T[mid])
        out[mid, :-1] = (f / a[mid])[:, None] * V[mid]
        out[mid, -1] = f
    return out


def _bisect_increasing(fun, lo, hi, active, max_iter=2200):
    """Vectorised bisection for the sign change of functions that are
    negative near ``lo`` and positive near ``hi``; stops at full relative
    precision of the abscissa."""
    lo = lo.copy()
    hi = hi.copy()
    act = active.copy()
    for _ in range(max_iter):
        if not np.any(act):
            break
        mid = 0.5 * (lo + hi)
        done = (mid <= lo) | (mid >= hi) | (hi - lo <= 4.0 * EPS * np.abs(hi))
        act &= ~done
        if not np.any(act):
            break
        f = fun(mid, act)
        neg = act & (f < 0)
        pos = act & ~(f < 0)
        lo[neg] = mid[neg]
        hi[pos] = mid[pos]
    return 0.5 * (lo + hi)


def soc_metric(R, Mt):
    """M-norm SOC projection through the secular equation of
    eq. soc-metric-projection: v_i = m_i r_i/(m_i + lam), t = m_t r_t/(m_t - lam),
    ||v||^2 = t^2, with lam in (0, m_t) if r_t > 0 and in (m_t, inf) if r_t < 0;
    r_t = 0 is the singular case lam = m_t.

    The root is located by bisection on the distance delta = |m_t - lam| > 0
    (same root, shifted coordinate), using the sign of ||v|| - t, which equals
    the sign of ||v||^2 - t^2; the upper end for r_t < 0 is found by doubling
    from lam = 2 m_t."""
    R = np.atleast_2d(np.asarray(R, dtype=float))
    Mt = np.broadcast_to(np.atleast_2d(np.asarray(Mt, dtype=float)), R.shape)
    V, T = R[:, :-1], R[:, -1]
    MV, MT = Mt[:, :-1], Mt[:, -1]
    out = np.zeros_like(R)
    inK = np.linalg.norm(V, axis=1) <= T
    zero = ~inK & (np.linalg.norm(MV * V, axis=1) <= -MT * T)
    sing = ~inK & ~zero & (T == 0)
    hard = ~inK & ~zero & ~sing
    out[inK] = R[inK]
    if np.any(sing):
        vv = MV[sing] * V[sing] / (MV[sing] + MT[sing][:, None])
        out[sing, :-1] = vv
        out[sing, -1] = np.linalg.norm(vv, axis=1)
    if np.any(hard):
        Vh, Th, MVh, MTh = V[hard], T[hard], MV[hard], MT[hard]
        sg = np.where(Th > 0, 1.0, -1.0)
        absT = np.abs(Th)

        def side(delta, act):
            lam = MTh - sg * delta
            vv = MVh * Vh / (MVh + lam[:, None])
            return np.linalg.norm(vv, axis=1) - MTh * absT / delta

        lo = np.zeros_like(Th)
        hi = MTh.copy()
        act = sg < 0
        for _ in range(2100):
            if not np.any(act):
                break
            f = side(hi, act)
            grow = act & ~(f > 0)
            hi[grow] *= 2.0
            act = grow
        delta = _bisect_increasing(side, lo, hi, np.ones_like(Th, dtype=bool))
        lam = MTh - sg * delta
        out[hard, :-1] = MVh * Vh / (MVh + lam[:, None])
        out[hard, -1] = MTh * absT / delta
    return out


# ----------------------------------------------------------------------------
# RSOC
# ----------------------------------------------------------------------------
def rsoc_euclid(R):
    """eq. rsoc-via-soc: Pi = U^{-1} Pi_soc(U r), with
    U(v, s, t) = ((v, (s - t)/sqrt2), (s + t)/sqrt2)."""
    R = np.atleast_2d(np.asarray(R, dtype=float))
    h = 1.0 / math.sqrt(2.0)
    W = np.empty_like(R)
    W[:, :-2] = R[:, :-2]
    W[:, -2] = (R[:, -2] - R[:, -1]) * h
    W[:, -1] = (R[:, -2] + R[:, -1]) * h
    P = soc_euclid(W)
    out = np.empty_like(R)
    out[:, :-2] = P[:, :-2]
    out[:, -2] = (P[:, -1] + P[:, -2]) * h
    out[:, -1] = (P[:, -1] - P[:, -2]) * h
    return out


def rsoc_metric(R, Mt):
    """M-norm RSOC projection through the xi-system of
    eq. rsoc-metric-projection:
        v_i = m_i r_i / (m_i + 2 xi),
        [m_s, -2xi; -2xi, m_t] [s; t] = [m_s r_s; m_t r_t],
        ||v||^2 = 2 s t.
    The 2x2 system is singular at 2 xi = q = sqrt(m_s m_t); when its right-hand
    side is consistent (sqrt(m_s) r_s + sqrt(m_t) r_t = 0) the explicit
    solution eq. rsoc-metric-singular-projection applies.  Otherwise the root
    lies on one side of q/2 (the subsection's closing paragraph); the side is
    fixed by the sign of kappa = sqrt(m_s) r_s + sqrt(m_t) r_t: as 2 xi -> q
    both s and t tend to +inf from the side on which the 2x2 determinant has
    the sign of kappa, so phi = ||v||^2 - 2 s t -> -inf there, while phi > 0 at
    xi = 0 (kappa > 0) and phi*xi^2 > 0 as xi -> inf (kappa < 0, outside the
    zero-projection case).  Bisection on delta = |xi - q/2|."""
    R = np.atleast_2d(np.asarray(R, dtype=float))
    Mt = np.broadcast_to(np.atleast_2d(np.asarray(Mt, dtype=float)), R.shape)
    V, S, T = R[:, :-2], R[:, -2], R[:, -1]
    MV, MS, MT = Mt[:, :-2], Mt[:, -2], Mt[:, -1]
    out = np.zeros_like(R)
    inK = (S >= 0) & (T >= 0) & (np.einsum("ij,ij->i", V, V) <= 2.0 * S * T)
    MVV = MV * V
    zero = ~inK & (MS * S <= 0) & (MT * T <= 0) & (
        np.einsum("ij,ij->i", MVV, MVV) <= 2.0 * (MS * S) * (MT * T))
    sqs, sqt = np.sqrt(MS), np.sqrt(MT)
    kappa = sqs * S + sqt * T
    sing = ~inK & ~zero & (kappa == 0)
    hard = ~inK & ~zero & ~sing
    out[inK] = R[inK]
    if np.any(sing):
        q = np.sqrt(MS[sing] * MT[sing])
        dl = sqs[sing] * S[sing]
        vv = MV[sing] * V[sing] / (MV[sing] + q[:, None])
        chi = np.sqrt(dl * dl + 2.0 * q * np.einsum("ij,ij->i", vv, vv))
        out[sing, :-2] = vv
        out[sing, -2] = (dl + chi) / (2.0 * sqs[sing])
        out[sing, -1] = (-dl + chi) / (2.0 * sqt[sing])
    if np.any(hard):
        Vh, Sh, Th = V[hard], S[hard], T[hard]
        MVh, MSh, MTh = MV[hard], MS[hard], MT[hard]
        q = np.sqrt(MSh * MTh)
        up = kappa[hard] < 0          # root on the side xi > q/2

        def xi_of(delta):
            return np.where(up, 0.5 * q + delta, 0.5 * q - delta)

        def st_of(delta):
            xi = xi_of(delta)
            # det = m_s m_t - 4 xi^2 = (q - 2xi)(q + 2xi), q - 2xi = -/+ 2 delta
            det = np.where(up, -2.0 * delta, 2.0 * delta) * (q + 2.0 * xi)
            s = MTh * (MSh * Sh + 2.0 * xi * Th) / det
            t = MSh * (MTh * Th + 2.0 * xi * Sh) / det
            return xi, s, t

        def phi(delta, act):
            xi, s, t = st_of(delta)
            vv = MVh * Vh / (MVh + 2.0 * xi[:, None])
            return np.einsum("ij,ij->i", vv, vv) - 2.0 * s * t

        lo = np.zeros_like(q)
        hi = 0.5 * q
        act = up.copy()
        for _ in range(2100):
            if not np.any(act):
                break
            f = phi(hi, act)
            grow = act & ~(f > 0)
            hi[grow] *= 2.0
            act = grow
        delta = _bisect_increasing(phi, lo, hi, np.ones_like(q, dtype=bool))
        xi, s, t = st_of(delta)
        out[hard, :-2] = MVh * Vh / (MVh + 2.0 * xi[:, None])
        out[hard, -2] = s
        out[hard, -1] = t
    return out


# ----------------------------------------------------------------------------
# EXP
# ----------------------------------------------------------------------------
def _exp_eta_h(rho, r0, s0, t0, mr, ms, mt):
    """eta_M(rho) and the sign-carrying H(rho) = h_M(rho) * Den(rho) of
    eq. exp-metric-projection, where Den = m_r rho^2 + m_s + m_t e^{2 rho} > 0.
    Expanding h_M Den = N Den'/2 - N' Den (N the numerator of eta_M) the
    m_r^2 rho^2 r0 and m_t^2 e^{3 rho} t0 terms cancel exactly, leaving
        H = m_t e^{2rho} (m_r r0 (rho - 1) + m_s s0)
            - m_t t0 e^{rho} (m_r rho (rho - 1) + m_s) + m_r m_s (rho s0 - r0),
    which is evaluated without cancellation.  For rho > 0 everything is
    divided by e^{2 rho} (same eta, same sign of H).  Returns
    (eta, H_scaled, e^{rho} eta)."""
    if rho > 0:
        em = math.exp(-rho)
        em2 = em * em
        num = mr * rho * r0 * em2 + ms * s0 * em2 + mt * t0 * em
        den = mr * rho * rho * em2 + ms * em2 + mt
        eta = num / den
        H = (mt * (mr * r0 * (rho - 1.0) + ms * s0)
             - mt * t0 * em * (mr * rho * (rho - 1.0) + ms)
             + mr * ms * (rho * s0 - r0) * em2)
        eta_e = (mr * rho * r0 * em + ms * s0 * em + mt * t0) / den
        return eta, H, eta_e
    e = math.exp(rho)
    num = mr * rho * r0 + ms * s0 + mt * e * t0
    den = mr * rho * rho + ms + mt * e * e
    eta = num / den
    H = (mt * e * e * (mr * r0 * (rho - 1.0) + ms * s0)
         - mt * t0 * e * (mr * rho * (rho - 1.0) + ms)
         + mr * ms * (rho * s0 - r0))
    return eta, H, eta * e


def _exp_psi(rho, r0, s0):
    """psi(rho) = <(r0, s0, .), grad> part: e^rho (r0 + (1 - rho) s0); the ray
    with ratio rho is visible from r iff psi(rho) > t0."""
    f = r0 + (1.0 - rho) * s0
    if rho > 700.0:
        return math.copysign(math.inf, f) if f != 0 else 0.0
    return math.exp(rho) * f


def _bisect_scalar(f, lo, hi, increasing=True, max_iter=3000):
    """Scalar bisection for the sign change of f on [lo, hi]."""
    for _ in range(max_iter):
        mid = 0.5 * (lo + hi)
        if mid <= lo or mid >= hi or hi - lo <= 4.0 * EPS * max(1.0, abs(mid)):
            break
        v = f(mid)
        if (v < 0) == increasing:
            lo = mid
        else:
            hi = mid
    return 0.5 * (lo + hi)


def _step_out(f, start, direction, want_positive, limit):
    """Walk from ``start`` in ``direction`` with doubling steps until
    f(x) has the wanted sign; returns x (clamped at ``limit``)."""
    step = 1.0
    x = start
    for _ in range(4000):
        x = start + direction * step
        if (direction > 0 and x >= limit) or (direction < 0 and x <= limit):
            return limit
        v = f(x)
        if (v > 0) == want_positive:
            return x
        step *= 2.0
    return limit


def _exp_visible_components(r0, s0, t0):
    """Components of V = {rho : psi(rho) > t0}, the ratios rho = r/s of the
    boundary rays of K_exp that are visible from r (<r, grad g> > 0 with
    g = s e^{r/s} - t).  The metric projection lies on a visible ray because
    M(r - u) = mu grad g with mu > 0 gives <r, grad g> = mu ||grad g||^2_{M^-1}.
    Returns a list of (lo, hi) with infinite ends allowed."""
    inf = math.inf

    def psi_minus_t(x):
        return _exp_psi(x, r0, s0) - t0

    if s0 > 0:
        rm = r0 / s0                    # maximiser of psi, psi(rm) > t0
        hi_far = _step_out(psi_minus_t, rm, +1.0, False, RHO_MAX)
        b = _bisect_scalar(psi_minus_t, rm, hi_far, increasing=False)
        if t0 > 0:
            lo_far = _step_out(psi_minus_t, rm, -1.0, False, RHO_MIN)
            a = _bisect_scalar(psi_minus_t, lo_far, rm, increasing=True)
            return [(a, b)]
        return [(-inf, b)]
    if s0 == 0:                         # here r0 > 0
        if t0 > 0:
            return [(math.log(t0 / r0), inf)]
        return [(-inf, inf)]
    # s0 < 0, r0 > 0: psi has its minimum at rm = r0/s0 < 0, psi(rm) < 0
    rm = r0 / s0
    hi_far = _step_out(psi_minus_t, rm, +1.0, True, RHO_MAX)
    b = _bisect_scalar(psi_minus_t, rm, hi_far, increasing=True)
    if t0 >= 0:
        return [(b, inf)]
    if _exp_psi(rm, r0, s0) >= t0:
        return [(-inf, inf)]
    lo_far = _step_out(psi_minus_t, rm, -1.0, True, RHO_MIN)
    a = _bisect_scalar(psi_minus_t, lo_far, rm, increasing=False)
    return [(-inf, a), (b, inf)]


def _exp_positive_components(r0, s0, t0, mr, ms, mt):
    """Components of {rho : N(rho) > 0}, N = m_r rho r0 + m_s s0 + m_t t0 e^rho
    the numerator of eta_M: the rays on which the nearest point to r is not
    the origin.  N is linear (t0 = 0), concave (t0 < 0) or convex (t0 > 0),
    so the set has at most two components."""
    inf = math.inf

    def N(x):
        if x > 700.0:
            return math.copysign(math.inf, t0) if t0 != 0 else mr * x * r0 + ms * s0
        return mr * x * r0 + ms * s0 + mt * t0 * math.exp(x)

    def root_between(lo, hi, increasing):
        return _bisect_scalar(N, lo, hi, increasing=increasing)

    if t0 == 0:
        if r0 > 0:
            return [(-ms * s0 / (mr * r0), inf)]
        if r0 < 0:
            return [(-inf, -ms * s0 / (mr * r0))]
        return [(-inf, inf)] if s0 > 0 else []
    if t0 < 0:
        if r0 <= 0:                      # N decreasing
            if r0 == 0 and s0 <= 0:
                return []
            if r0 == 0:
                return [(-inf, math.log(ms * s0 / (-mt * t0)))]
            hi = _step_out(N, 0.0, +1.0, False, RHO_MAX)
            lo = _step_out(N, 0.0, -1.0, True, RHO_MIN)
            if N(lo) <= 0:
                return []
            return [(-inf, root_between(lo, hi, False))]
        xm = math.log(mr * r0 / (-mt * t0))   # maximiser
        if N(xm) <= 0:
            return []
        a = root_between(_step_out(N, xm, -1.0, False, RHO_MIN), xm, True)
        b = root_between(xm, _step_out(N, xm, +1.0, False, RHO_MAX), False)
        return [(a, b)]
    # t0 > 0: convex
    if r0 >= 0:                          # N increasing
        if r0 == 0:
            return [(-inf, inf)] if s0 >= 0 else [(math.log(-ms * s0 / (mt * t0)), inf)]
        lo = _step_out(N, 0.0, -1.0, False, RHO_MIN)
        if N(lo) > 0:
            return [(-inf, inf)]
        return [(root_between(lo, _step_out(N, 0.0, +1.0, True, RHO_MAX), True), inf)]
    xm = math.log(mr * r0 / (-mt * t0))       # minimiser (r0 < 0)
    if N(xm) > 0:
        return [(-inf, inf)]
    a = root_between(_step_out(N, xm, -1.0, True, RHO_MIN), xm, False)
    b = root_between(xm, _step_out(N, xm, +1.0, True, RHO_MAX), True)
    return [(-inf, a), (b, inf)]


def _intersect(A, B):
    out = []
    for a0, a1 in A:
        for b0, b1 in B:
            lo, hi = max(a0, b0), min(a1, b1)
            if lo < hi:
                out.append((lo, hi))
    return out


def exp_metric_one(r, m=(1.0, 1.0, 1.0)):
    """Pi^M onto K_exp for one block (Appendix C, exponential-cone
    subsection).

    Cases in order: r in K -> r;  -M r in K^* -> 0;  r0 <= 0 and s0 <= 0 ->
    (r0, 0, max(t0, 0));  otherwise the smooth-boundary point
    eta_M(rho)(rho, 1, e^rho) at the admissible root of h_M.

    Bracket (the paper defers it to PDCS): a root of h_M is a stationary
    point of the M-cosine c(rho) = N/sqrt(Den) between r and the ray
    (rho, 1, e^rho) (c' = -h_M/sqrt(Den)), i.e. M(r - u) is normal to the
    boundary at u = eta_M(rho)(rho, 1, e^rho).  It is the projection iff
    eta_M > 0 (N > 0) and the normal points outward (the ray is visible from
    r, psi(rho) > t0).  On the set V ∩ {N > 0} the stationary point is
    therefore unique, and it is a maximum of c, so on the component holding it
    h_M changes sign from - to +; at an end where N = 0, h_M = -N' has the
    right sign automatically.  Each component is searched for such a bracket
    and bisected."""
    r0, s0, t0 = (float(a) for a in r)
    mr, ms, mt = (float(a) for a in m)
    if in_exp((r0, s0, t0)):
        return np.array([r0, s0, t0])
    if in_exp_dual((-mr * r0, -ms * s0, -mt * t0)):
        return np.zeros(3)
    if r0 <= 0 and s0 <= 0:
        return np.array([r0, 0.0, max(t0, 0.0)])

    def hfun(x):
        return _exp_eta_h(x, r0, s0, t0, mr, ms, mt)[1]

    def point(x):
        eta, _, eta_e = _exp_eta_h(x, r0, s0, t0, mr, ms, mt)
        return np.array([eta * x, eta, eta_e])

    fallback = []
    comps = _intersect(_exp_visible_components(r0, s0, t0),
                       _exp_positive_components(r0, s0, t0, mr, ms, mt))
    for lo, hi in comps:
        lo_f = lo if math.isfinite(lo) else None
        hi_f = hi if math.isfinite(hi) else None
        if lo_f is None and hi_f is None:
            x0 = 0.0
            if hfun(x0) < 0:
                lo_f, hi_f = x0, _step_out(hfun, x0, +1.0, True, RHO_MAX)
            else:
                lo_f, hi_f = _step_out(hfun, x0, -1.0, False, RHO_MIN), x0
        elif lo_f is None:
            if not hfun(hi_f) > 0:
                continue
            lo_f = _step_out(hfun, hi_f, -1.0, False, RHO_MIN)
        elif hi_f is None:
            if not hfun(lo_f) < 0:
                continue
            hi_f = _step_out(hfun, lo_f, +1.0, True, RHO_MAX)
        elif not (hfun(lo_f) < 0 and hfun(hi_f) > 0):
            continue
        if lo_f in (RHO_MIN, RHO_MAX) or hi_f in (RHO_MIN, RHO_MAX):
            # no sign change inside the search range: keep the range end as a
            # limiting candidate (the root, if any, lies beyond |rho| = 1e100)
            fallback.append(lo_f if lo_f in (RHO_MIN, RHO_MAX) else hi_f)
            continue
        u = point(_bisect_scalar(hfun, lo_f, hi_f))
        if u[1] >= 0:                  # eta > 0; it may underflow to 0 for rho >~ 745
            return u
    for x in fallback:
        u = point(x)
        if u[1] >= 0:
            return u
    # No admissible sign change survives in floating point: r lies within
    # rounding of the polar cone (Pi(r) ~ 0) or of the ray family's ends.
    # Fall back to the definition of the projection (closest point of K).
    return exp_closest_direct(r0, s0, t0, mr, ms, mt)


def exp_closest_direct(r0, s0, t0, mr=1.0, ms=1.0, mt=1.0):
    """Closest point of K_exp to r in the diagonal M-norm: r itself when
    r is in K, else by direct comparison of the pieces of the cone's
    boundary: the apex 0, the face
    {(a, 0, b): a <= 0, b >= 0} (its M-projection clamps componentwise), and
    the rays (rho, 1, e^rho), whose M-projection is eta(rho) (rho, 1, e^rho)
    with eta = <r, d>_M / |d|_M^2 when positive.  The ray parameter is
    located on a grid (uniform on [-60, 60], logarithmic tails to 1e12) and
    refined by golden-section search on the distance.  Used where the root
    bracket of h_M degenerates; accurate to about sqrt(eps) in rho."""
    vals = (r0, s0, t0, mr, ms, mt)
    if not all(math.isfinite(v) for v in vals):
        raise FloatingPointError(f"exp projection: non-finite input {vals}")

    if in_exp((r0, s0, t0)):
        return np.array([r0, s0, t0])

    def dist2(u):
        return mr * (u[0] - r0) ** 2 + ms * (u[1] - s0) ** 2 + mt * (u[2] - t0) ** 2

    def ray_point(x):
        eta, _, eta_e = _exp_eta_h(x, r0, s0, t0, mr, ms, mt)
        if not eta > 0:
            return None
        return np.array([eta * x, eta, eta_e])

    best = np.zeros(3)
    face = np.array([min(r0, 0.0), 0.0, max(t0, 0.0)])
    if dist2(face) < dist2(best):
        best = face
    tails = np.logspace(math.log10(60.0), 12.0, 200)
    grid = np.concatenate([-tails[::-1], np.linspace(-60.0, 60.0, 4801), tails])
    d_grid = np.full(grid.size, np.inf)
    for k, x in enumerate(grid):
        u = ray_point(float(x))
        if u is not None:
            d_grid[k] = dist2(u)
    k = int(np.argmin(d_grid))
    if math.isfinite(d_grid[k]):
        lo, hi = float(grid[max(k - 1, 0)]), float(grid[min(k + 1, grid.size - 1)])
        g = (math.sqrt(5.0) - 1.0) / 2.0

        def f(x):
            u = ray_point(x)
            return dist2(u) if u is not None else math.inf
        a, b = lo, hi
        c, d = b - g * (b - a), a + g * (b - a)
        fc, fd = f(c), f(d)
        for _ in range(200):
            if fc <= fd:
                b, d, fd = d, c, fc
                c = b - g * (b - a)
                fc = f(c)
            else:
                a, c, fc = c, d, fd
                d = a + g * (b - a)
                fd = f(d)
        for x in (c, d, float(grid[k])):
            u = ray_point(x)
            if u is not None and dist2(u) < dist2(best):
                best = u
    return best


# ----------------------------------------------------------------------------
# EXP block with the middle coordinate fixed at one
# ----------------------------------------------------------------------------
def exp1_metric_one(r, m=(1.0, 1.0, 1.0)):
    """Pi^M onto X = {(z, s, t): s = 1, e^z <= t}, the exponential-cone block
    whose middle coordinate is fixed at one (Section "Large-Scale Fisher
    Equilibrium"): s = 1, and (z, t) is r's (z, t) when e^z0 <= t0, else the
    point (z, e^z) where m_z (z - z0) + m_t (e^z - t0) e^z = 0 (stationarity
    of m_z (z - z0)^2 + m_t (t - t0)^2 on t = e^z, with the multiplier
    m_t (t - t0) >= 0).  That function is increasing where e^z >= t0 and
    positive at z0; its root is bisected between z0 and a point where it is
    negative (log t0 when t0 > 0, else found by stepping down)."""
    z0, _, t0 = (float(a) for a in r)
    mz, _, mt = (float(a) for a in m)
    if z0 <= 709.0 and math.exp(z0) <= t0:
        return np.array([z0, 1.0, t0])

    def f(z):
        ez = math.exp(z)
        return mz * (z - z0) + mt * (ez - t0) * ez

    hi = min(z0, 709.0)
    if t0 > 0:
        lo = min(math.log(t0), hi)
    else:
        step = 1.0
        lo = hi - step
        while f(lo) >= 0:
            step *= 2.0
            lo = hi - step
    z = _bisect_scalar(f, lo, hi, increasing=True)
    return np.array([z, 1.0, math.exp(z)])


def exp1_dual_terms(a, b, c):
    """For the reduced cost (a, b, c) of an exp1 block: its projection
    (min(a, 0), b, max(c, 0)) onto Lambda = {a <= 0, c >= 0} (the dual of
    the set's recession cone {dz <= 0, ds = 0, dt >= 0}) and the infimum
    over the set of <lambda, x> = b + lambda_a (log(-lambda_a/lambda_c) - 1)
    (b when lambda_a = 0; -inf when lambda_a < 0 = lambda_c)."""
    la, lc = min(a, 0.0), max(c, 0.0)
    if la == 0.0:
        term = b
    elif lc == 0.0:
        term = -math.inf
    else:
        term = b + la * (math.log(-la / lc) - 1.0)
    return (la, b, lc), term


# ----------------------------------------------------------------------------
# POW
# ----------------------------------------------------------------------------
def _qroot(s, c):
    """Cancellation-free positive root of u^2 - s u - c = 0
    (eq. power-cone-stable-quadratic-root)."""
    d = math.sqrt(s * s + 4.0 * c)
    if s >= 0:
        return 0.5 * (s + d)
    return 2.0 * c / (d - s)


def pow_metric_one(r, alpha, m=(1.0, 1.0, 1.0), eps_bis=1e-15):
    """Pi^M onto K_pow^alpha for one block: the r_z = 0 formula, the
    membership and zero-projection tests, then the bisection of
    Prop. power-cone-bisection on g_M over (0, R), R = |r_z|, stopping when
    rho_U - rho_L <= eps_bis max(1, R) and returning the midpoint
    (eq. power-metric-projection-recovery)."""
    x, y, z = (float(a) for a in r)
    mx, my, mz = (float(a) for a in m)
    a = float(alpha)
    if z == 0:
        return np.array([max(x, 0.0), max(y, 0.0), 0.0])
    if in_pow((x, y, z), a):
        return np.array([x, y, z])
    if in_pow_dual((-mx * x, -my * y, -mz * z), a):
        return np.zeros(3)
    Rz = abs(z)
    cx = a * mz / mx
    cy = (1.0 - a) * mz / my

    def xm(rho):
        return _qroot(x, cx * rho * (Rz - rho))

    def ym(rho):
        return _qroot(y, cy * rho * (Rz - rho))

    def g(rho):
        xv, yv = xm(rho), ym(rho)
        if xv <= 0 or yv <= 0:
            return -math.inf
        return a * math.log(xv) + (1.0 - a) * math.log(yv) - math.log(rho)

    lo, hi = 0.0, Rz
    tol = eps_bis * max(1.0, Rz)
    for _ in range(3000):
        if hi - lo <= tol:
            break
        mid = 0.5 * (lo + hi)
        gm = g(mid)
        if gm > 0:
            lo = mid
        elif gm < 0:
            hi = mid
        else:
            lo = hi = mid
            break
    rho = 0.5 * (lo + hi)
    return np.array([xm(rho), ym(rho), math.copysign(rho, z)])


# ----------------------------------------------------------------------------
# product-cone projection
# ----------------------------------------------------------------------------
class Projector:
    """Pi^M_K for K = product of blocks, grouped by (type, dim) so that SOC
    and RSOC blocks are projected in vectorised batches.

    ``project(r, m=None, euclid=None)``: m is the diagonal of M (length n)
    or None (Euclidean).  ``euclid`` is a boolean per block; True selects the
    Euclidean formula (valid when m is constant on the block, since
    Pi^{cI} = Pi^I).  Box blocks [lo_i, hi_i] (the box set of
    eq. solver-input) clamp, in any diagonal metric; lo and hi have length n
    and are read at the box coordinates.

    cone_scale (length n, positive; rescaled-cone mode of Section "Problem
    Rescaling"): each SOC, RSOC, EXP and POW block j is the scaled set S_j K_j
    with S_j = diag(cone_scale on the block).  Substituting w = S_j u in
    min_{w in S_j K_j} ||w - r||_M^2 gives
        Pi^M_{S_j K_j}(r) = S_j Pi^{S_j M S_j}_{K_j}(S_j^-1 r),
    the metric form of eq. scaling-induced-metric; the block is projected
    that way, always with the metric routines (S_j M S_j is diagonal and in
    general not constant on the block, so ``euclid`` does not apply)."""

    def __init__(self, cones, n, lo=None, hi=None, kappa=None, cone_scale=None):
        self.cones = list(cones)
        self.n = n
        self.groups = {}
        self.cone_scale = None
        if cone_scale is not None:
            self.cone_scale = np.asarray(cone_scale, dtype=float)
            sc = [np.arange(st, st + d) for kind, st, d, al in self.cones
                  if kind in ("soc", "rsoc", "exp", "pow")]
            self.scaled_idx = np.concatenate(sc) if sc else np.zeros(0, dtype=np.int64)
        # exp1 blocks in scaled coordinates: the set kappa X with kappa the
        # block's (common) scale factor; 1 in the original coordinates
        self.kappa = None if kappa is None else np.asarray(kappa, dtype=float)
        box = [np.arange(st, st + d) for kind, st, d, al in self.cones if kind == "box"]
        self.box_idx = np.concatenate(box) if box else np.zeros(0, dtype=np.int64)
        if self.box_idx.size:
            self.box_lo = np.asarray(lo, dtype=float)[self.box_idx]
            self.box_hi = np.asarray(hi, dtype=float)[self.box_idx]
        for bi, (kind, st, d, al) in enumerate(self.cones):
            if kind in ("soc", "rsoc"):
                self.groups.setdefault((kind, d), []).append(bi)
        self.free_idx = []
        self.nonneg_idx = []
        for kind, st, d, al in self.cones:
            if kind == "free":
                self.free_idx.append(np.arange(st, st + d))
            elif kind == "nonneg":
                self.nonneg_idx.append(np.arange(st, st + d))
        self.nonneg_idx = (np.concatenate(self.nonneg_idx) if self.nonneg_idx
                           else np.zeros(0, dtype=np.int64))

    def const_blocks(self, q):
        """True for blocks on which the vector q is constant (exactly)."""
        out = np.zeros(len(self.cones), dtype=bool)
        for bi, (kind, st, d, al) in enumerate(self.cones):
            seg = q[st:st + d]
            out[bi] = bool(np.all(seg == seg[0]))
        return out

    def project(self, r, m=None, euclid=None):
        r = np.asarray(r, dtype=float)
        if self.cone_scale is not None and self.scaled_idx.size:
            idx = self.scaled_idx
            s = self.cone_scale
            if euclid is None:
                euclid = np.ones(len(self.cones), dtype=bool) if m is None else \
                    np.zeros(len(self.cones), dtype=bool)
            base = np.ones(self.n) if m is None else np.array(m, dtype=float)
            for bi, (kind, st, d, al) in enumerate(self.cones):
                if euclid[bi]:
                    base[st:st + d] = 1.0
            r2 = r.copy()
            r2[idx] = r[idx] / s[idx]
            m2 = base.copy()
            m2[idx] = base[idx] * s[idx] * s[idx]
            out = self._project(r2, m2, np.where(
                [k in ("soc", "rsoc", "exp", "pow") for k, _, _, _ in self.cones], False, euclid))
            res = self._project(r, m, euclid)
            res[idx] = s[idx] * out[idx]
            return res
        return self._project(r, m, euclid)

    def _project(self, r, m=None, euclid=None):
        r = np.asarray(r, dtype=float)
        out = r.copy()
        if self.nonneg_idx.size:
            out[self.nonneg_idx] = np.maximum(r[self.nonneg_idx], 0.0)
        if self.box_idx.size:
            out[self.box_idx] = np.minimum(np.maximum(r[self.box_idx], self.box_lo), self.box_hi)
        if euclid is None:
            euclid = np.ones(len(self.cones), dtype=bool) if m is None else \
                np.zeros(len(self.cones), dtype=bool)
        for (kind, d), blist in self.groups.items():
            blist = np.asarray(blist)
            starts = np.array([self.cones[b][1] for b in blist])
            idx = starts[:, None] + np.arange(d)[None, :]
            eu = euclid[blist]
            if np.any(eu):
                Rb = r[idx[eu]]
                out[idx[eu]] = soc_euclid(Rb) if kind == "soc" else rsoc_euclid(Rb)
            if np.any(~eu):
                Rb = r[idx[~eu]]
                Mb = m[idx[~eu]]
                out[idx[~eu]] = soc_metric(Rb, Mb) if kind == "soc" else rsoc_metric(Rb, Mb)
        for bi, (kind, st, d, al) in enumerate(self.cones):
            if kind not in ("exp", "pow", "exp1"):
                continue
            mm = (1.0, 1.0, 1.0) if (euclid[bi] or m is None) else m[st:st + 3]
            if kind == "exp":
                out[st:st + 3] = exp_metric_one(r[st:st + 3], mm)
            elif kind == "exp1":
                k = 1.0 if self.kappa is None else float(self.kappa[st])
                out[st:st + 3] = k * exp1_metric_one(r[st:st + 3] / k, mm)
            else:
                out[st:st + 3] = pow_metric_one(r[st:st + 3], al, mm)
        return out


def project_euclid(r, cones):
    """Euclidean Pi_K (convenience wrapper)."""
    return Projector(cones, len(r)).project(r)
