"""Pins for the oracle's rescaled-cone mode (Section "Problem Rescaling",
eq. cone-scaling-candidates, eq. scaling-induced-metric).

* The block projection onto a scaled cone S K in a diagonal metric M is
  characterised, like any metric projection onto a closed convex cone, by
      w in S K,   M(w - r) in (S K)^* = S^-1 K^*,   <w, M(w - r)> = 0;
  the tests check that triple written on w itself (membership of S^-1 w in K
  and of S M (w - r) in K^*, with the tolerant tests of test_oracle_cones),
  and brute-force minimisation over S K on tiny SOC and RSOC inputs with the
  constraints written on w.
* The factors of the rescaled-cone mode are those of the same problem with
  every cone block relabelled as free coordinates (the coordinatewise rule,
  itself pinned by the worked examples in test_oracle_pins).
* A whole solve in the rescaled-cone mode reaches the solution of the
  cone-preserving mode (the scaling changes the path, not the answer)."""
import numpy as np
import pytest
from scipy.optimize import minimize

from instances import synth
from oracle import pdhg, scaling
from oracle.cones import Projector
from test_oracle_cones import check_kkt


def _scaled_case(kind, rng, d):
    s = 10.0 ** rng.uniform(-1.0, 1.0, size=d)
    m = 10.0 ** rng.uniform(-1.0, 1.0, size=d)
    r = rng.standard_normal(d) * (10.0 ** rng.uniform(-1, 1))
    return s, m, r


@pytest.mark.parametrize("kind,d", [("soc", 5), ("rsoc", 4), ("exp", 3), ("pow", 3)])
@pytest.mark.parametrize("metric", [True, False])
def test_rescaled_projection_kkt(kind, d, metric):
    rng = np.random.default_rng({"soc": 1, "rsoc": 2, "exp": 3, "pow": 4}[kind] + 10 * metric)
    for _ in range(40):
        s, m, r = _scaled_case(kind, rng, d)
        al = float(rng.uniform(0.2, 0.8)) if kind == "pow" else 0.0
        P = Projector([(kind, 0, d, al)], d, cone_scale=s)
        if metric:
            w = P.project(r, m, np.array([False]))
        else:
            w = P.project(r)
            m = np.ones(d)
        # u = S^-1 w in K, S M (w - r) in K^*, <w, M (w - r)> = 0: the triple
        # of check_kkt for the point u, the input S^-1 r and the metric S M S
        check_kkt(kind, r / s, w / s, m * s * s, alpha=al, tol=1e-7)


def test_rescaled_euclid_flag_uses_scale_only():
    """A block flagged Euclidean (constant metric) is still projected in the
    metric S^2 in the rescaled-cone mode: the result equals the projection
    with M = 1 and differs from the plain Euclidean projection onto K."""
    rng = np.random.default_rng(7)
    s, m, r = _scaled_case("soc", rng, 4)
    P = Projector([("soc", 0, 4, 0.0)], 4, cone_scale=s)
    w1 = P.project(r, np.full(4, 3.0), np.array([True]))
    w2 = P.project(r)
    np.testing.assert_allclose(w1, w2, rtol=1e-13, atol=1e-15)
    w0 = Projector([("soc", 0, 4, 0.0)], 4).project(r)
    assert np.max(np.abs(w0 - w2)) > 1e-3


def _boundary_min(wmap, r, m, rng):
    """min over the boundary of a 3-dimensional scaled cone, given as the
    image of R^2 under wmap, by Nelder-Mead from a grid of starts."""
    f = lambda p: 0.5 * np.sum(m * (wmap(p) - r) ** 2)
    best = f(np.zeros(2))
    for a in np.linspace(-3, 3, 4):
        for b in np.linspace(-3, 3, 4):
            res = minimize(f, np.array([a, b]), method="Nelder-Mead",
                           options=dict(xatol=1e-11, fatol=1e-14, maxiter=2000))
            best = min(best, res.fun)
    return best


def test_rescaled_brute_force_soc_rsoc():
    """min 1/2 ||w - r||_M^2 over S K: either r lies in S K, or the minimum is
    on the boundary of S K, parametrised directly (SOC: (s_0 a, s_1 b,
    s_2 sqrt(a^2 + b^2)); RSOC: (s_0 sqrt(2) p q, s_1 p^2, s_2 q^2))."""
    rng = np.random.default_rng(21)
    for _ in range(12):
        s, m, r = _scaled_case("soc", rng, 3)
        u = r / s
        w = Projector([("soc", 0, 3, 0.0)], 3, cone_scale=s).project(r, m, np.array([False]))
        if np.hypot(u[0], u[1]) <= u[2]:
            np.testing.assert_allclose(w, r, rtol=1e-12, atol=1e-14)
        else:
            b = _boundary_min(lambda p: np.array([s[0] * p[0], s[1] * p[1], s[2] * np.hypot(p[0], p[1])]),
                              r, m, rng)
            assert 0.5 * np.sum(m * (w - r) ** 2) <= b + 1e-9 * (1.0 + b)
        w = Projector([("rsoc", 0, 3, 0.0)], 3, cone_scale=s).project(r, m, np.array([False]))
        if u[1] >= 0 and u[2] >= 0 and u[0] ** 2 <= 2 * u[1] * u[2]:
            np.testing.assert_allclose(w, r, rtol=1e-12, atol=1e-14)
        else:
            b = _boundary_min(lambda p: np.array([s[0] * np.sqrt(2) * p[0] * p[1], s[1] * p[0] ** 2,
                                                  s[2] * p[1] ** 2]), r, m, rng)
            assert 0.5 * np.sum(m * (w - r) ** 2) <= b + 1e-9 * (1.0 + b)


def test_rescaled_factors_are_coordinatewise():
    p = synth.tiny_mixed(3)
    sr = scaling.scale_problem(p, cone_mode="rescaled")
    free = [("free", st, d, 0.0) for kind, st, d, al in p.cones]
    q = synth.Problem(n=p.n, m=p.m, A=p.A, b=p.b, c=p.c, P=p.P, R=p.R, D=p.D, cones=free, name="free")
    sf = scaling.scale_problem(q)
    np.testing.assert_array_equal(sr.Sx, sf.Sx)
    np.testing.assert_array_equal(sr.Sy, sf.Sy)
    sb = scaling.scale_problem(p)
    for kind, st, d, al in p.cones:
        if kind in ("soc", "rsoc", "exp", "pow"):
            assert np.all(sb.Sx[st:st + d] == sb.Sx[st])          # one factor per block
            assert np.ptp(sr.Sx[st:st + d]) > 0                   # coordinatewise


def test_rescaled_exp1_blocks_keep_one_factor():
    p = synth.fisher(seed=1, n_buyers=12, n_goods=6, density=0.5, graph_seed=1, dist="paper", middle="fixed")
    sr = scaling.scale_problem(p, cone_mode="rescaled")
    for kind, st, d, al in p.cones:
        if kind == "exp1":
            assert np.all(sr.Sx[st:st + d] == sr.Sx[st])


def test_rescaled_mode_reaches_the_same_solution():
    p = synth.tiny_mixed(4)
    rb = pdhg.solve(p, pdhg.Settings(tol=1e-9))
    rr = pdhg.solve(p, pdhg.Settings(tol=1e-9, cone_scaling="rescaled"))
    assert rb.status == rr.status == "OPTIMAL"
    assert rr.kkt["primal_obj"] == pytest.approx(rb.kkt["primal_obj"], rel=1e-6, abs=1e-7)
    np.testing.assert_allclose(rr.x, rb.x, atol=2e-5)
    # the mode is active: the two runs follow different paths
    tb = pdhg.solve(p, pdhg.Settings(trace_iters=2, max_iter=2))
    tr = pdhg.solve(p, pdhg.Settings(trace_iters=2, max_iter=2, cone_scaling="rescaled"))
    assert np.max(np.abs(tb.trace[1]["wx"] - tr.trace[1]["wx"])) > 1e-6
