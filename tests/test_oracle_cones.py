"""Pins for the oracle's cone projections (Appendix C of the paper).

A metric projection u = Pi^M_K(r) is characterised uniquely by
    u in K,   M(u - r) in K^*,   <u, M(u - r)> = 0,
so these tests check that triple (with tolerances written here, not the
oracle's exact membership tests), the printed closed forms, M = cI against
the Euclidean formula, POW(1/2) against RSOC, and brute-force minimisation on
tiny inputs.
"""
import math

import numpy as np
import pytest
from scipy.optimize import minimize

from oracle import cones as C

RNG = np.random.default_rng(12345)


# ---------------------------------------------------------------------------
# tolerant membership written for the tests
# ---------------------------------------------------------------------------
def soc_gap(u):           # <= 0 inside
    return np.linalg.norm(u[:-1]) - u[-1]


def rsoc_gap(u):
    v, s, t = u[:-2], u[-2], u[-1]
    return max(v @ v - 2 * s * t, -s, -t)


def exp_gap(u, scale):
    r, s, t = u
    if s > 1e-300:
        if r / s > 700:
            return math.inf
        return s * math.exp(r / s) - t
    return max(r, -t, -s) if s >= -1e-12 * scale else -s


def expd_gap(u, scale):
    a, b, c = u
    if a < -1e-300:
        q = b / a
        if q > 700:
            return math.inf
        return -a * math.exp(q) - math.e * c
    return max(a, -b, -c)


def pow_gap(u, al):
    x, y, z = u
    if x < 0 or y < 0:
        return max(-x, -y)
    return abs(z) - x ** al * y ** (1 - al)


def powd_gap(u, al):
    p, q, w = u
    if p < 0 or q < 0:
        return max(-p, -q)
    return abs(w) - (p / al) ** al * (q / (1 - al)) ** (1 - al)


INTERIOR = {"soc": lambda d: np.r_[np.zeros(d - 1), 1.0],
            "rsoc": lambda d: np.r_[np.zeros(d - 2), 1.0, 1.0],
            "exp": lambda d: np.array([-1.0, 1.0, 1.0]),
            "pow": lambda d: np.array([1.0, 1.0, 0.0])}


def check_kkt(kind, r, u, m, alpha=0.0, tol=1e-8):
    """u in K and M(u - r) in K^* up to a shift of size tol*scale along a
    direction interior to the cone (a distance test that stays well posed
    near the boundary), and <u, M(u - r)> = 0."""
    scale = max(1.0, np.abs(r).max())
    g = m * (u - r)                       # M(u - r) must lie in K^*
    gs = scale * max(1.0, m.max())
    e = INTERIOR[kind](len(r))
    up = u + tol * scale * e
    gp = g + tol * gs * e
    if kind == "soc":
        pg, dg = soc_gap(up), soc_gap(gp)
    elif kind == "rsoc":
        pg, dg = rsoc_gap(up), rsoc_gap(gp)
    elif kind == "exp":
        pg, dg = exp_gap(up, scale), expd_gap(gp, gs)
    elif kind == "pow":
        pg, dg = pow_gap(up, alpha), powd_gap(gp, alpha)
    else:
        raise ValueError(kind)
    assert pg <= 0, (kind, r, u, m, "primal", pg)
    assert dg <= 0, (kind, r, u, m, "dual", dg)
    assert abs(u @ g) <= tol * scale * gs, (kind, r, u, m, "compl", u @ g)


def random_vectors(d, k, rng):
    out = []
    for i in range(k):
        sc = 10.0 ** rng.uniform(-3, 3) if i % 3 == 0 else 1.0
        out.append(sc * rng.standard_normal(d))
    return out


def random_metric(d, rng):
    return 10.0 ** rng.uniform(-1.5, 1.5, size=d)


# ---------------------------------------------------------------------------
# R+ and box: closed form
# ---------------------------------------------------------------------------
def test_nonneg_closed_form():
    r = RNG.standard_normal(50)
    P = C.Projector([("nonneg", 0, 50, 0.0)], 50)
    np.testing.assert_array_equal(P.project(r), np.maximum(r, 0))
    np.testing.assert_array_equal(P.project(r, random_metric(50, RNG)), np.maximum(r, 0))


def test_free_is_identity():
    r = RNG.standard_normal(7)
    P = C.Projector([("free", 0, 7, 0.0)], 7)
    np.testing.assert_array_equal(P.project(r), r)


# ---------------------------------------------------------------------------
# SOC
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("d", [2, 3, 5, 20])
def test_soc_euclid_kkt(d):
    for r in random_vectors(d, 60, RNG):
        u = C.soc_euclid(r)[0]
        check_kkt("soc", r, u, np.ones(d))


@pytest.mark.parametrize("d", [2, 3, 5, 20])
def test_soc_metric_kkt(d):
    for r in random_vectors(d, 60, RNG):
        m = random_metric(d, RNG)
        u = C.soc_metric(r, m)[0]
        check_kkt("soc", r, u, m)


def test_soc_metric_constant_equals_euclid():
    for r in random_vectors(6, 80, RNG):
        c = 10.0 ** RNG.uniform(-2, 2)
        np.testing.assert_allclose(C.soc_metric(r, np.full(6, c))[0], C.soc_euclid(r)[0],
                                   rtol=1e-12, atol=1e-12 * np.abs(r).max())


def test_soc_singular_rt_zero():
    """r_t = 0: lam = m_t, v_i = m_i r_i/(m_i + m_t), t = ||v|| (Appendix C)."""
    for _ in range(30):
        r = RNG.standard_normal(5)
        r[-1] = 0.0
        m = random_metric(5, RNG)
        u = C.soc_metric(r, m)[0]
        v = m[:-1] * r[:-1] / (m[:-1] + m[-1])
        np.testing.assert_allclose(u[:-1], v, rtol=1e-14)
        np.testing.assert_allclose(u[-1], np.linalg.norm(v), rtol=1e-14)
        check_kkt("soc", r, u, m)


def test_soc_adversarial():
    m = np.array([1e-3, 1.0, 1e3, 1.0])
    cases = [np.array([1.0, 0, 0, 1e-12]), np.array([1.0, 1.0, 1.0, -1e-12]),
             np.array([1e-9, 0, 0, 1.0]), np.array([1.0, 2.0, 3.0, -3.7]),
             np.array([0, 0, 0, -1.0]), np.array([1e6, -1e6, 1e-6, 1.0])]
    for r in cases:
        check_kkt("soc", r, C.soc_metric(r, m)[0], m)
        check_kkt("soc", r, C.soc_euclid(r)[0], np.ones(4))


# ---------------------------------------------------------------------------
# RSOC
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("d", [3, 4, 10])
def test_rsoc_euclid_kkt(d):
    for r in random_vectors(d, 60, RNG):
        check_kkt("rsoc", r, C.rsoc_euclid(r)[0], np.ones(d))


@pytest.mark.parametrize("d", [3, 4, 10])
def test_rsoc_metric_kkt(d):
    for r in random_vectors(d, 80, RNG):
        m = random_metric(d, RNG)
        check_kkt("rsoc", r, C.rsoc_metric(r, m)[0], m)


def test_rsoc_metric_constant_equals_euclid():
    for r in random_vectors(5, 80, RNG):
        c = 10.0 ** RNG.uniform(-2, 2)
        np.testing.assert_allclose(C.rsoc_metric(r, np.full(5, c))[0], C.rsoc_euclid(r)[0],
                                   rtol=1e-10, atol=1e-11 * np.abs(r).max())


def test_rsoc_singular_consistent_case():
    """sqrt(m_s) r_s + sqrt(m_t) r_t = 0: explicit solution of Appendix C."""
    for _ in range(40):
        m = random_metric(5, RNG)
        r = RNG.standard_normal(5)
        r[-1] = -math.sqrt(m[-2]) * r[-2] / math.sqrt(m[-1])
        if math.sqrt(m[-2]) * r[-2] + math.sqrt(m[-1]) * r[-1] != 0.0:
            continue
        u = C.rsoc_metric(r, m)[0]
        check_kkt("rsoc", r, u, m)
        assert abs(u[:-2] @ u[:-2] - 2 * u[-2] * u[-1]) <= 1e-12 * max(1, u @ u)


def test_rsoc_both_branches_hit():
    """Roots on both sides of q/2 occur and are valid."""
    lower = upper = 0
    for r in random_vectors(4, 200, RNG):
        m = random_metric(4, RNG)
        kappa = math.sqrt(m[-2]) * r[-2] + math.sqrt(m[-1]) * r[-1]
        u = C.rsoc_metric(r, m)[0]
        check_kkt("rsoc", r, u, m)
        if not C.in_rsoc(r) and np.any(u != 0):
            lower += kappa > 0
            upper += kappa < 0
    assert lower > 5 and upper > 5


# ---------------------------------------------------------------------------
# EXP
# ---------------------------------------------------------------------------
def exp_inputs(rng, k):
    out = []
    for i in range(k):
        r = rng.standard_normal(3)
        if i % 4 == 1:
            r *= 10.0 ** rng.uniform(-4, 4)
        if i % 7 == 3:
            r[1] = abs(r[1]) * 1e-6
        if i % 11 == 5:
            r[0] = abs(r[0]) * 50
        out.append(r)
    return out


def test_exp_euclid_kkt():
    for r in exp_inputs(RNG, 300):
        check_kkt("exp", r, C.exp_metric_one(r), np.ones(3), tol=1e-7)


def test_exp_metric_kkt():
    for r in exp_inputs(RNG, 300):
        m = random_metric(3, RNG)
        check_kkt("exp", r, C.exp_metric_one(r, m), m, tol=1e-7)


def test_exp_special_cases():
    """r0 <= 0 and s0 <= 0 (outside K and -Mr outside K^*) give
    (r0, 0, max(t0, 0)) in both metrics (Appendix C)."""
    for _ in range(50):
        r = np.array([-abs(RNG.standard_normal()), -abs(RNG.standard_normal()),
                      RNG.standard_normal()])
        m = random_metric(3, RNG)
        u = C.exp_metric_one(r, m)
        if C.in_exp_dual(-m * r):
            np.testing.assert_array_equal(u, 0)
        else:
            np.testing.assert_array_equal(u, [r[0], 0.0, max(r[2], 0.0)])
            check_kkt("exp", r, u, m)


def test_exp_constant_metric():
    for r in exp_inputs(RNG, 100):
        c = 10.0 ** RNG.uniform(-2, 2)
        np.testing.assert_allclose(C.exp_metric_one(r, (c, c, c)), C.exp_metric_one(r),
                                   rtol=1e-9, atol=1e-11 * np.abs(r).max())


def _brute_exp(r, m):
    """Minimise ||u - r||_M over the boundary eta(rho, 1, e^rho), the face
    {(a, 0, b): a <= 0, b >= 0} and the origin, by a dense grid plus
    Nelder-Mead refinement."""
    best = (0.5 * np.sum(m * r * r), np.zeros(3))
    # face
    a = min(r[0], 0.0)
    b = max(r[2], 0.0)
    u = np.array([a, 0.0, b])
    best = min(best, (0.5 * np.sum(m * (u - r) ** 2), u), key=lambda z: z[0])

    def f(p):
        rho, le = p
        eta = math.exp(min(le, 50))
        if rho > 40:
            return 1e300
        u = eta * np.array([rho, 1.0, math.exp(rho)])
        return 0.5 * np.sum(m * (u - r) ** 2)

    grid = [(f((rho, le)), rho, le) for rho in np.linspace(-20, 20, 161)
            for le in np.linspace(-12, 6, 73)]
    grid.sort()
    for val, rho, le in grid[:6]:
        res = minimize(f, [rho, le], method="Nelder-Mead",
                       options=dict(xatol=1e-12, fatol=1e-15, maxiter=4000))
        if res.fun < best[0]:
            rho, le = res.x
            eta = math.exp(le)
            best = (res.fun, eta * np.array([rho, 1.0, math.exp(rho)]))
    return best


def test_exp_brute_force():
    rng = np.random.default_rng(7)
    for _ in range(25):
        r = rng.standard_normal(3)
        m = random_metric(3, rng)
        u = C.exp_metric_one(r, m)
        du = 0.5 * np.sum(m * (u - r) ** 2)
        bval, bu = _brute_exp(r, m)
        assert du <= bval + 1e-9 * max(1.0, bval), (r, m, u, bu)


def test_exp_direct_closest_point_agrees():
    """The closest-point fallback (direct search over the boundary pieces)
    and the root-of-h_M method agree on generic inputs, inside and outside K,
    in both metrics."""
    rng = np.random.default_rng(8)
    for r in exp_inputs(rng, 150):
        m = random_metric(3, rng)
        a = C.exp_metric_one(r, m)
        b = C.exp_closest_direct(*r, *m)
        assert np.linalg.norm(a - b) <= 1e-7 * max(1.0, np.linalg.norm(r)), (r, m, a, b)


def test_exp_near_polar_boundary():
    """Inputs within rounding of the polar cone -K^* (as the dual slack of a
    solved EXP block is) project to (nearly) zero and satisfy the KKT
    characterisation; the bracket of h_M degenerates there."""
    rng = np.random.default_rng(9)
    cases = [(np.array([1.22744381, 0.97589908, -1.0]), np.ones(3))]
    for i in range(60):
        a = -abs(rng.standard_normal()) * 10.0 ** rng.uniform(-2, 2)
        b = rng.standard_normal() * abs(a)
        c = -a * math.exp(b / a) / math.e               # (a, b, c) on the boundary of K^*
        m = np.ones(3) if i % 2 else random_metric(3, rng)
        # -M r on the boundary of K^*, up to relative 1e-13
        r = -np.array([a, b, c]) / m * (1.0 + 1e-13 * rng.standard_normal(3))
        cases.append((r, m))
    for r, m in cases:
        u = C.exp_metric_one(r, m)
        assert np.linalg.norm(u) <= 1e-9 * np.linalg.norm(r), (r, m, u)
        check_kkt("exp", r, u, m, tol=1e-7)


# ---------------------------------------------------------------------------
# POW
# ---------------------------------------------------------------------------
def test_pow_kkt():
    for i, r in enumerate(random_vectors(3, 300, RNG)):
        al = RNG.uniform(0.05, 0.95)
        m = random_metric(3, RNG) if i % 2 else np.ones(3)
        check_kkt("pow", r, C.pow_metric_one(r, al, m), m, al, tol=1e-8)


def test_pow_rz_zero():
    for _ in range(20):
        r = RNG.standard_normal(3)
        r[2] = 0.0
        u = C.pow_metric_one(r, 0.3, random_metric(3, RNG))
        np.testing.assert_array_equal(u, [max(r[0], 0), max(r[1], 0), 0.0])


def test_pow_half_equals_rsoc():
    """K_pow^{1/2} = {x, y >= 0, xy >= z^2} is the image of RSOC(3) under
    (v, s, t) -> (s, t, v/sqrt2); the M-norm projection with (m_x, m_y, m_z)
    maps to the RSOC projection with metric (m_z/2, m_x, m_y)."""
    for _ in range(150):
        r = RNG.standard_normal(3) * 10.0 ** RNG.uniform(-2, 2)
        m = random_metric(3, RNG)
        u = C.pow_metric_one(r, 0.5, m)
        rr = np.array([math.sqrt(2) * r[2], r[0], r[1]])
        mm = np.array([m[2] / 2, m[0], m[1]])
        w = C.rsoc_metric(rr, mm)[0]
        np.testing.assert_allclose(u, [w[1], w[2], w[0] / math.sqrt(2)],
                                   rtol=1e-9, atol=1e-11 * np.abs(r).max())


# ---------------------------------------------------------------------------
# generic brute force for SOC / RSOC / POW on tiny inputs
# ---------------------------------------------------------------------------
def _brute_generic(cons, r, m, x0s):
    best = None
    for x0 in x0s:
        res = minimize(lambda u: 0.5 * np.sum(m * (u - r) ** 2), x0,
                       jac=lambda u: m * (u - r), constraints=cons, method="SLSQP",
                       options=dict(ftol=1e-14, maxiter=500))
        feas = all(cn["fun"](res.x) >= -1e-9 for cn in cons)
        if feas and (best is None or res.fun < best):
            best = res.fun
    return best


def test_brute_force_soc_rsoc_pow():
    rng = np.random.default_rng(99)
    for _ in range(15):
        r = rng.standard_normal(3)
        m = random_metric(3, rng)
        starts = [np.array([0.0, 0.0, 1.0]), np.abs(r) + 0.1, np.array([1.0, 1.0, 0.0])]
        u = C.soc_metric(r, m)[0]
        b = _brute_generic([{"type": "ineq", "fun": lambda w: w[2] ** 2 - w[0] ** 2 - w[1] ** 2},
                            {"type": "ineq", "fun": lambda w: w[2]}], r, m, starts)
        assert b is not None
        assert 0.5 * np.sum(m * (u - r) ** 2) <= b + 1e-8
        u = C.rsoc_metric(r, m)[0]
        b = _brute_generic([{"type": "ineq", "fun": lambda w: 2 * w[1] * w[2] - w[0] ** 2},
                            {"type": "ineq", "fun": lambda w: w[1]},
                            {"type": "ineq", "fun": lambda w: w[2]}], r, m, starts)
        assert b is not None
        assert 0.5 * np.sum(m * (u - r) ** 2) <= b + 1e-8
        al = rng.uniform(0.2, 0.8)
        u = C.pow_metric_one(r, al, m)
        b = _brute_generic([{"type": "ineq",
                             "fun": lambda w: np.maximum(w[0], 0) ** al
                             * np.maximum(w[1], 0) ** (1 - al) - abs(w[2])},
                            {"type": "ineq", "fun": lambda w: w[0]},
                            {"type": "ineq", "fun": lambda w: w[1]}],
                           r, m, [np.array([1.0, 1.0, 0.0]), np.abs(r) + 0.5])
        if b is not None:
            assert 0.5 * np.sum(m * (u - r) ** 2) <= b + 1e-8


def test_projector_groups_match_single_calls():
    cones = [("soc", 0, 4, 0.0), ("rsoc", 4, 3, 0.0), ("soc", 7, 4, 0.0),
             ("exp", 11, 3, 0.0), ("pow", 14, 3, 0.35), ("nonneg", 17, 3, 0.0)]
    r = RNG.standard_normal(20)
    m = random_metric(20, RNG)
    P = C.Projector(cones, 20)
    out = P.project(r, m, np.zeros(len(cones), dtype=bool))
    np.testing.assert_allclose(out[0:4], C.soc_metric(r[0:4], m[0:4])[0])
    np.testing.assert_allclose(out[4:7], C.rsoc_metric(r[4:7], m[4:7])[0])
    np.testing.assert_allclose(out[7:11], C.soc_metric(r[7:11], m[7:11])[0])
    np.testing.assert_allclose(out[11:14], C.exp_metric_one(r[11:14], m[11:14]))
    np.testing.assert_allclose(out[14:17], C.pow_metric_one(r[14:17], 0.35, m[14:17]))
    np.testing.assert_array_equal(out[17:], np.maximum(r[17:], 0))


# ---------------------------------------------------------------------------
# exponential block with the middle coordinate fixed at one (Fisher form)
# ---------------------------------------------------------------------------
def _exp1_inputs(rng, n=400):
    R = rng.standard_normal((n, 3)) * 10.0 ** rng.uniform(-1, 1, (n, 1))
    R[: n // 4, 2] = -np.abs(R[: n // 4, 2])          # t0 <= 0
    R[n // 4: n // 2, 2] = np.exp(R[n // 4: n // 2, 0]) * rng.uniform(1, 2, n // 4)   # inside
    return R


def test_exp1_projection_kkt():
    """u = Pi^M_X(r) for X = {(z, 1, t): e^z <= t}: u in X, and M(r - u) is a
    normal of X at u: zero in (z, t) inside, else (lam e^z, ., -lam) with
    lam >= 0 (the s entry is free: s is fixed)."""
    from oracle import cones as OC
    rng = np.random.default_rng(51)
    R = _exp1_inputs(rng)
    M = 10.0 ** rng.uniform(-1, 1, R.shape)
    for r, m in zip(R, M):
        u = OC.exp1_metric_one(r, m)
        assert u[1] == 1.0 and math.exp(u[0]) <= u[2] * (1 + 1e-14)
        gz, gt = m[0] * (r[0] - u[0]), m[2] * (r[2] - u[2])
        if math.exp(r[0]) <= r[2]:
            assert u[0] == r[0] and u[2] == r[2]
        else:
            lam = -gt
            assert lam >= -1e-12 * max(1, abs(gt))
            assert gz == pytest.approx(lam * math.exp(u[0]), rel=1e-9, abs=1e-12)


def test_exp1_projection_brute_force():
    """Against a dense search over the boundary z (and the point itself when
    it is inside) in the metric distance."""
    from oracle import cones as OC
    rng = np.random.default_rng(52)
    R = _exp1_inputs(rng, 60)
    M = 10.0 ** rng.uniform(-1, 1, R.shape)
    for r, m in zip(R, M):
        u = OC.exp1_metric_one(r, m)
        zs = np.linspace(u[0] - 3, u[0] + 3, 200001)
        d = m[0] * (zs - r[0]) ** 2 + m[2] * (np.exp(zs) - r[2]) ** 2
        best = float(d.min())
        du = m[0] * (u[0] - r[0]) ** 2 + m[2] * (u[2] - r[2]) ** 2
        if math.exp(r[0]) > r[2]:
            assert du <= best * (1 + 1e-9) + 1e-15


def test_exp1_support_term_brute_force():
    """inf over X of <lambda, x> for lambda in Lambda = {a <= 0, c >= 0}:
    b + a (log(-a/c) - 1), against a grid over the boundary."""
    from oracle import cones as OC
    rng = np.random.default_rng(53)
    for _ in range(50):
        a, b, c = -rng.uniform(0.1, 3), rng.standard_normal(), rng.uniform(0.1, 3)
        lam, term = OC.exp1_dual_terms(a, b, c)
        assert lam == (a, b, c)
        zs = np.linspace(-20, 10, 300001)
        grid = b + float(np.min(a * zs + c * np.exp(zs)))
        # the grid (spacing 1e-4) misses the minimum by O(c e^z spacing^2)
        assert term <= grid + 1e-12 and grid - term <= 1e-7 * (1 + abs(term))
    assert OC.exp1_dual_terms(0.5, 1.5, 2.0)[1] == 1.5           # lambda_a = 0: z -> -inf
    assert OC.exp1_dual_terms(-1.0, 0.0, -1.0)[1] == -math.inf   # lambda_c = 0 < -lambda_a
