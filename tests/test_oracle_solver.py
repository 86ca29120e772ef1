"""Pins for the oracle's setup, proximal step, PDHG operator, restart metric,
Halpern epochs and whole solves.  Every expected value comes from a textbook
definition, an identity printed in the paper, or brute force; none comes
from the oracle itself or from the HIP library."""
import itertools
import json
import math
import os

import numpy as np
import pytest
import scipy.sparse as sp

from instances import synth
from oracle import pdhg, scaling
from oracle.cones import Projector

HERE = os.path.dirname(os.path.abspath(__file__))


# ---------------------------------------------------------------------------
# helpers written for the tests
# ---------------------------------------------------------------------------
def dense_Q(p):
    Q = np.zeros((p.n, p.n))
    if p.P is not None:
        Q += p.P.toarray()
    if p.R is not None:
        Q += p.R.T @ p.D @ p.R
    return Q


def active_set_qp(H, g, A=None, b=None):
    """min 1/2 u'Hu + g'u  s.t. A u = b, u >= 0, by enumerating the zero set
    (tiny n only)."""
    n = len(g)
    best = None
    for k in range(n + 1):
        for Z in itertools.combinations(range(n), k):
            F = [i for i in range(n) if i not in Z]
            nf = len(F)
            mA = 0 if A is None else A.shape[0]
            K = np.zeros((nf + mA, nf + mA))
            rhs = np.zeros(nf + mA)
            K[:nf, :nf] = H[np.ix_(F, F)]
            rhs[:nf] = -g[F]
            if mA:
                K[:nf, nf:] = -A[:, F].T
                K[nf:, :nf] = A[:, F]
                rhs[nf:] = b
            try:
                sol = np.linalg.lstsq(K, rhs, rcond=None)[0]
            except np.linalg.LinAlgError:
                continue
            u = np.zeros(n)
            u[F] = sol[:nf]
            if np.any(u < -1e-10) or np.linalg.norm(K @ sol - rhs) > 1e-8:
                continue
            if mA and np.linalg.norm(A @ u - b) > 1e-8:
                continue
            y = sol[nf:] if mA else np.zeros(0)
            s = H @ u + g - (A.T @ y if mA else 0)
            if np.any(s[list(Z)] < -1e-9):
                continue
            val = 0.5 * u @ H @ u + g @ u
            if best is None or val < best[0]:
                best = (val, np.maximum(u, 0), y)
    return best


# ---------------------------------------------------------------------------
# defaults (Table practical-defaults)
# ---------------------------------------------------------------------------
def test_defaults_match_paper_table():
    gold = json.load(open(os.path.join(HERE, "golden", "practical_defaults.json")))
    st = pdhg.Settings()
    for key in ("ruiz_iters", "pc_alpha", "eps_in0", "gamma_in", "eps_min", "rho",
                "beta_s", "beta_n", "beta_a", "pid_beta_i", "pid_kp", "pid_ki", "pid_kd"):
        assert getattr(st, key) == gold[key], key
    assert st.bound_objective is gold["bound_objective"]
    assert (st.inner == "jacobi") is gold["jacobi"]
    p = synth.tiny_qp(0)
    S = pdhg.setup(p)
    assert S.eta == pytest.approx(gold["eta_factor"] / S.a_norm, rel=1e-15)


# ---------------------------------------------------------------------------
# setup: power iteration, scaling
# ---------------------------------------------------------------------------
def test_power_norm_matches_svd():
    rng = np.random.default_rng(3)
    U, _ = np.linalg.qr(rng.standard_normal((30, 30)))
    V, _ = np.linalg.qr(rng.standard_normal((50, 50)))
    s = np.linspace(1, 3, 30)
    s[0] = 6.0
    A = U @ np.diag(s) @ V[:30]
    assert pdhg.power_norm(sp.csr_matrix(A), 128) == pytest.approx(
        np.linalg.svd(A, compute_uv=False)[0], rel=1e-12)


def test_scaling_roundtrip_and_structure():
    p = synth.tiny_mixed(2)
    sc = scaling.scale_problem(p)
    x = np.random.default_rng(0).standard_normal(p.n)
    y = np.random.default_rng(1).standard_normal(p.m)
    np.testing.assert_allclose(sc.unscale_x(sc.scale_x(x)), x, rtol=1e-14)
    np.testing.assert_allclose(sc.unscale_y(sc.scale_y(y)), y, rtol=1e-14)
    # A^ = S_y A S_x^-1 / (no nu): check the defining relation entrywise
    Ad = p.A.toarray()
    np.testing.assert_allclose(sc.A.toarray(), sc.Sy[:, None] * Ad / sc.Sx[None, :], rtol=1e-13)
    # cone blocks get one common factor (cone-preserving mode)
    for kind, st, d, al in p.cones:
        if kind not in ("free", "nonneg"):
            assert np.all(sc.Sx[st:st + d] == sc.Sx[st])
    # the objective of x^ equals the original objective / (nu_b nu_c)
    Q = dense_Q(p)
    xh = sc.scale_x(x)
    Qh = (sc.P.toarray() if sc.P is not None else 0) + sc.R.T @ sc.D @ sc.R
    f_orig = 0.5 * x @ Q @ x + p.c @ x
    f_hat = 0.5 * xh @ Qh @ xh + sc.c @ xh
    assert f_hat == pytest.approx(f_orig / (sc.nu_b * sc.nu_c), rel=1e-12)
    np.testing.assert_allclose(sc.A @ xh - sc.b, sc.Sy * (p.A @ x - p.b) / sc.nu_b,
                               rtol=1e-12, atol=1e-14)


def test_ruiz_equilibrates():
    p = synth.tiny_qp(1)
    sc = scaling.scale_problem(p, ruiz_iters=30, pock_chambolle=False,
                               bound_objective=False)
    absA = abs(sc.A)
    colmax = np.asarray(absA.max(axis=0).todense()).ravel()
    np.testing.assert_allclose(colmax[colmax > 0], 1.0, atol=1e-3)   # empty columns stay 0
    np.testing.assert_allclose(np.asarray(absA.max(axis=1).todense()).ravel(), 1.0, atol=1e-3)


# ---------------------------------------------------------------------------
# proximal step
# ---------------------------------------------------------------------------
def test_diag_prox_nonneg_textbook():
    """diag Q on R+: argmin_{u>=0} 1/2 q u^2 + c u + (u - v)^2/(2 tau) is
    max(0, (v - tau c)/(1 + tau q))."""
    p = synth.tiny_nonneg_qp(0, n=10, diag_only=True)
    S = pdhg.setup(p)
    rng = np.random.default_rng(5)
    v = rng.standard_normal(p.n)
    tau = 0.37
    u, j, _ = pdhg.prox(S, v, np.zeros(p.n), tau, 1e-9)
    q = S.q.diag
    np.testing.assert_allclose(u, np.maximum(0, (v - tau * S.sc.c) / (1 + tau * q)), rtol=1e-15)
    assert j == 0


@pytest.mark.parametrize("inner", ["jacobi", "euclid"])
def test_jbb_prox_matches_active_set(inner):
    p = synth.tiny_nonneg_qp(4, n=7)
    S = pdhg.setup(p, pdhg.Settings(inner=inner, j_max=20000))
    Qh = dense_Q(type(p)(n=p.n, m=p.m, A=S.sc.A, b=S.sc.b, c=S.sc.c, P=S.sc.P,
                         cones=p.cones))
    rng = np.random.default_rng(8)
    v = rng.standard_normal(p.n)
    tau = 0.8
    u, j, _ = pdhg.prox(S, v, np.abs(v), tau, 1e-13)
    val, ustar, _ = active_set_qp(Qh + np.eye(p.n) / tau, S.sc.c - v / tau)
    np.testing.assert_allclose(u, ustar, atol=1e-9)


def test_pg_contraction_to_prox_point():
    """Prop. fixed-pg-work: projected gradient with eta_PG = 2/(L+mu) contracts
    towards the prox point at rate rho_PG; the oracle's converged prox point
    must be that fixed point."""
    p = synth.tiny_nonneg_qp(6, n=9)
    S = pdhg.setup(p, pdhg.Settings(j_max=20000))
    Qh = S.sc.P.toarray()
    tau = 0.5
    Hm = Qh + np.eye(p.n) / tau
    ev = np.linalg.eigvalsh(Hm)
    L, mu = ev[-1], ev[0]
    eta_pg = 2 / (L + mu)
    rho_pg = (L - mu) / (L + mu)
    v = np.random.default_rng(1).standard_normal(p.n)
    pstar, _, _ = pdhg.prox(S, v, np.zeros(p.n), tau, 1e-14)
    u0 = np.random.default_rng(2).uniform(0, 1, p.n)
    u = u0.copy()
    for J in range(1, 30):
        u = np.maximum(u - eta_pg * (Hm @ u + S.sc.c - v / tau), 0)
        assert np.linalg.norm(u - pstar) <= rho_pg ** J * np.linalg.norm(u0 - pstar) + 1e-12


# ---------------------------------------------------------------------------
# PDHG operator identities
# ---------------------------------------------------------------------------
def _pdhg_setup_diag():
    p = synth.tiny_mixed(3, lowrank=False)
    S = pdhg.setup(p)
    return p, S


def test_resolvent_identity_dual_part():
    """A(x - w_x) + sigma^-1 (y - w_y) = A w_x - b (proof of Lemma
    one-step-energy, dual step)."""
    p, S = _pdhg_setup_diag()
    rng = np.random.default_rng(0)
    x, y = rng.standard_normal(p.n), rng.standard_normal(p.m)
    tau, sigma = S.eta / 1.3, S.eta * 1.3
    wx, wy, _ = pdhg.pdhg_step(S, x, y, tau, sigma, 1e-9)
    A = S.sc.A
    np.testing.assert_allclose(A @ (x - wx) + (y - wy) / sigma, A @ wx - S.sc.b,
                               rtol=1e-11, atol=1e-12)


def test_resolvent_identity_primal_part():
    """tau^-1 (x - w_x) + A^T (y - w_y) - (Q w_x + c - A^T w_y) lies in the
    normal cone N_K(w_x) (eq. pdhg-residual-kkt, primal row)."""
    p, S = _pdhg_setup_diag()
    rng = np.random.default_rng(1)
    x, y = rng.standard_normal(p.n), rng.standard_normal(p.m)
    tau, sigma = S.eta / 0.7, S.eta * 0.7
    wx, wy, _ = pdhg.pdhg_step(S, x, y, tau, sigma, 1e-9)
    A = S.sc.A
    r = (x - wx) / tau + A.T @ (y - wy) - (S.q(wx) + S.sc.c - A.T @ wy)
    # r in N_K(wx)  <=>  wx in K, -r in K^*, <wx, r> = 0  <=>  wx = Pi_K(wx + r)
    np.testing.assert_allclose(Projector(p.cones, p.n).project(wx + r), wx, atol=1e-9)


def _metric_norm2(S, dx, dy, tau, sigma):
    A = S.sc.A
    return dx @ dx / tau + dy @ dy / sigma + 2 * dy @ (A @ dx)


def test_firm_nonexpansive():
    """T is firmly nonexpansive in the metric M_n (exact prox)."""
    p, S = _pdhg_setup_diag()
    rng = np.random.default_rng(2)
    tau, sigma = S.eta / 0.9, S.eta * 0.9
    for _ in range(20):
        z1 = (rng.standard_normal(p.n), rng.standard_normal(p.m))
        z2 = (rng.standard_normal(p.n), rng.standard_normal(p.m))
        t1 = pdhg.pdhg_step(S, *z1, tau, sigma, 1e-9)
        t2 = pdhg.pdhg_step(S, *z2, tau, sigma, 1e-9)
        dtx, dty = t1[0] - t2[0], t1[1] - t2[1]
        dzx, dzy = z1[0] - z2[0], z1[1] - z2[1]
        A = S.sc.A
        lhs = _metric_norm2(S, dtx, dty, tau, sigma)
        inner = dtx @ dzx / tau + dty @ dzy / sigma + dty @ (A @ dzx) + dzy @ (A @ dtx)
        assert lhs <= inner + 1e-9 * max(1, abs(inner))


def test_restart_metric_is_scaled_M_norm():
    """E^2 = omega||dx||^2 + ||dy||^2/omega + 2 eta <A dx, dy> equals
    eta ||z - Tz||^2_{M_n} with tau = eta/omega, sigma = eta omega."""
    p, S = _pdhg_setup_diag()
    rng = np.random.default_rng(4)
    omega = 1.7
    tau, sigma = S.eta / omega, S.eta * omega
    dx, dy = rng.standard_normal(p.n), rng.standard_normal(p.m)
    E2 = omega * dx @ dx + dy @ dy / omega + 2 * S.eta * (S.sc.A @ dx) @ dy
    Ad = S.sc.A.toarray()
    M = np.block([[np.eye(p.n) / tau, Ad.T], [Ad, np.eye(p.m) / sigma]])
    z = np.concatenate([dx, dy])
    assert E2 == pytest.approx(S.eta * z @ M @ z, rel=1e-12)
    assert np.linalg.eigvalsh(M)[0] > 0


def test_halpern_residual_decay():
    """R(h^k) <= ||a - z*||_M / (rho (k+1)) (eq. rh-residual-decay), exact
    prox, fixed step sizes, one epoch."""
    p, S = _pdhg_setup_diag()
    st = pdhg.Settings(tol=1e-12, max_iter=200000)
    ref = pdhg.solve(p, st, S=S)
    assert ref.status == "OPTIMAL"
    zs = (S.sc.scale_x(ref.x), S.sc.scale_y(ref.y))
    omega = 1.0
    tau, sigma = S.eta / omega, S.eta * omega
    rng = np.random.default_rng(6)
    for rho in (0.5, 1.0):
        a = (rng.standard_normal(p.n), rng.standard_normal(p.m))
        h = (a[0].copy(), a[1].copy())
        da = math.sqrt(_metric_norm2(S, a[0] - zs[0], a[1] - zs[1], tau, sigma))
        for k in range(60):
            w = pdhg.pdhg_step(S, *h, tau, sigma, 1e-9)
            if k >= 1:
                res = math.sqrt(_metric_norm2(S, h[0] - w[0], h[1] - w[1], tau, sigma))
                assert res <= da / (rho * (k + 1)) * (1 + 1e-6) + 1e-9
            c1 = (k + 1) / (k + 2)
            h = (c1 * (2 * rho * w[0] + (1 - 2 * rho) * h[0]) + a[0] / (k + 2),
                 c1 * (2 * rho * w[1] + (1 - 2 * rho) * h[1]) + a[1] / (k + 2))


def test_fejer_monotone_plain_pdhg():
    """Lemma one-step-energy: ||z^{k+1} - z*||_P <= ||z^k - z*||_P."""
    p, S = _pdhg_setup_diag()
    ref = pdhg.solve(p, pdhg.Settings(tol=1e-12, max_iter=200000), S=S)
    zs = (S.sc.scale_x(ref.x), S.sc.scale_y(ref.y))
    tau = sigma = S.eta
    rng = np.random.default_rng(9)
    z = (rng.standard_normal(p.n), rng.standard_normal(p.m))
    prev = math.inf
    for _ in range(80):
        d = math.sqrt(_metric_norm2(S, z[0] - zs[0], z[1] - zs[1], tau, sigma))
        assert d <= prev * (1 + 1e-9) + 1e-12
        prev = d
        w = pdhg.pdhg_step(S, *z, tau, sigma, 1e-9)
        z = (w[0], w[1])


# ---------------------------------------------------------------------------
# whole solves
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_free_qp_matches_kkt_solve(seed):
    p = synth.tiny_free_qp(seed)
    Q = dense_Q(p)
    Ad = p.A.toarray()
    K = np.block([[Q, -Ad.T], [Ad, np.zeros((p.m, p.m))]])
    sol = np.linalg.solve(K, np.concatenate([-p.c, p.b]))
    r = pdhg.solve(p, pdhg.Settings(tol=1e-8))
    assert r.status == "OPTIMAL"
    np.testing.assert_allclose(r.x, sol[:p.n], rtol=1e-5, atol=1e-6)
    np.testing.assert_allclose(r.y, sol[p.n:], rtol=1e-5, atol=1e-6)


@pytest.mark.parametrize("seed,diag", [(0, False), (1, False), (2, True), (3, True)])
def test_nonneg_qp_matches_active_set(seed, diag):
    p = synth.tiny_nonneg_qp(seed, n=8, m=3, diag_only=diag)
    val, ustar, ystar = active_set_qp(dense_Q(p), p.c, p.A.toarray(), p.b)
    r = pdhg.solve(p, pdhg.Settings(tol=1e-8))
    assert r.status == "OPTIMAL"
    np.testing.assert_allclose(r.x, ustar, atol=1e-5)
    assert r.kkt["primal_obj"] == pytest.approx(val, rel=1e-6, abs=1e-7)


def test_kkt_invariant_to_scaling():
    p = synth.tiny_mixed(5)
    r1 = pdhg.solve(p, pdhg.Settings(tol=1e-8))
    r2 = pdhg.solve(p, pdhg.Settings(tol=1e-8, scaling=False))
    assert r1.status == r2.status == "OPTIMAL"
    assert r1.kkt["primal_obj"] == pytest.approx(r2.kkt["primal_obj"], rel=1e-5, abs=1e-6)
    np.testing.assert_allclose(r1.x, r2.x, atol=1e-4)


def test_mixed_solution_satisfies_kkt():
    """The returned point satisfies eq. kkt-cqp to the tolerance, checked
    blockwise with the textbook cone definitions."""
    p = synth.tiny_mixed(6)
    r = pdhg.solve(p, pdhg.Settings(tol=1e-9))
    assert r.status == "OPTIMAL"
    x, y = r.x, r.y
    assert np.linalg.norm(p.A @ x - p.b) <= 1e-7 * (1 + np.linalg.norm(p.b))
    s = dense_Q(p) @ x + p.c - p.A.T @ y
    assert abs(x @ s) <= 1e-6 * (1 + abs(x @ dense_Q(p) @ x))
    for kind, st, d, al in p.cones:
        xb = x[st:st + d]
        if kind == "nonneg":
            assert xb.min() >= 0
        elif kind == "soc":
            assert np.linalg.norm(xb[:-1]) <= xb[-1] + 1e-12
        elif kind == "rsoc":
            assert xb[:-2] @ xb[:-2] <= 2 * xb[-2] * xb[-1] + 1e-12
        elif kind == "exp":
            assert xb[1] >= 0 and xb[1] * math.exp(xb[0] / max(xb[1], 1e-300)) <= xb[2] * (1 + 1e-12) + 1e-14
        elif kind == "pow":
            assert xb[0] ** al * xb[1] ** (1 - al) >= abs(xb[2]) * (1 - 1e-12) - 1e-14


def test_avg_scheme_converges():
    p = synth.tiny_nonneg_qp(2, n=8, m=3, diag_only=True)
    r = pdhg.solve(p, pdhg.Settings(scheme="avg", tol=1e-6, max_iter=200000))
    assert r.status == "OPTIMAL"
    val, ustar, _ = active_set_qp(dense_Q(p), p.c, p.A.toarray(), p.b)
    assert r.kkt["primal_obj"] == pytest.approx(val, rel=1e-4, abs=1e-5)


def test_status_limits():
    p = synth.tiny_qp(0)
    r = pdhg.solve(p, pdhg.Settings(max_iter=10))
    assert r.status == "MAX_ITER" and r.iterations == 10


def test_fisher_small_solves():
    """Small Fisher market: with the saddle function <y, b - Ax> of
    eq. saddle and a minimisation objective, the equilibrium prices are the
    negated duals of the supply rows; they must be nonnegative, and each
    buyer's spending (prices . allocation + retained money) must equal its
    budget (Eisenberg-Gale optimality)."""
    p = synth.fisher(seed=1, n_buyers=30, n_goods=12, density=0.3)
    r = pdhg.solve(p, pdhg.Settings(tol=1e-7, max_iter=200000))
    assert r.status == "OPTIMAL"
    prices = -r.y[:12]
    assert prices.min() >= -1e-5
    bi, gj = p.meta["graph"]
    e = bi.size
    spend = np.bincount(bi, weights=prices[gj] * r.x[:e], minlength=30) + r.x[e:e + 30]
    np.testing.assert_allclose(spend, p.meta["w"], rtol=1e-3, atol=1e-3)


def test_fisher_fixed_middle_equals_row_form():
    """The Fisher market with exponential blocks whose middle coordinate is
    fixed at one by the set and with an explicit row s_i = 1 are the same
    problem: equal optimal objective and equilibrium prices."""
    ps = [synth.fisher(seed=1, n_buyers=40, n_goods=16, density=0.3, graph_seed=1, dist="paper", middle=m)
          for m in ("row", "fixed")]
    rs = [pdhg.solve(p, pdhg.Settings(tol=1e-8, max_iter=400000)) for p in ps]
    assert rs[0].status == rs[1].status == "OPTIMAL"
    assert rs[1].kkt["primal_obj"] == pytest.approx(rs[0].kkt["primal_obj"], rel=1e-6)
    np.testing.assert_allclose(-rs[1].y[:16], -rs[0].y[:16], rtol=1e-4, atol=1e-6)
