"""GPU parity: the HIP library (through the C ABI) against the CPU oracle.

Iterate parity: the first 50 outer iterations (Halpern state and PDHG
candidate, scaled space) agree to 1e-10 relative in the max norm of each
vector, with identical inner-step counts, check and restart decisions.
Final parity: objective and the three relative KKT residuals agree to 1e-6
(absolute difference of the relative residuals, relative difference of the
objective).  Full-size instances are checked on a few iterations and, after
a full solve, by recomputing the KKT residuals of the returned point on the
CPU."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import paper_2608_09159_amd as G
from instances import Problem, synth
from oracle import pdhg

pytestmark = pytest.mark.gpu

ITER_TOL = 1e-10
FINAL_TOL = 1e-6


def _rel(a, b):
    scale = max(float(np.max(np.abs(b))) if b.size else 0.0, 1e-300)
    return float(np.max(np.abs(a - b))) / scale if b.size else 0.0


def oracle_settings(**kw):
    st = pdhg.Settings()
    for k, v in kw.items():
        setattr(st, k, v)
    return st


def trace_parity(prob, iters=50, check_every=4, x0=None, y0=None, **kw):
    okw = {k: v for k, v in kw.items() if k not in ("grid_dim", "lanes_at", "lanes_a")}
    print(f"[parity] {prob.name} n={prob.n} m={prob.m} iters={iters} {kw}", flush=True)
    h = G.setup(prob, trace_iters=iters, check_every=check_every, max_iter=iters, **kw)
    try:
        g = h.solve(x0, y0)
        tr = h.trace(iters)
    finally:
        h.free()
    o = pdhg.solve(prob, oracle_settings(trace_iters=iters, check_every=check_every,
                                         max_iter=iters, **okw), x0=x0, y0=y0)
    assert tr["count"] == len(o.trace), (tr["count"], len(o.trace))
    last = tr["count"] - 1
    for k, ot in enumerate(o.trace):
        for key in ("x", "y", "wx", "wy"):
            err = _rel(tr[key][k], ot[key])
            assert err <= ITER_TOL, (prob.name, k, key, err)
        for key in ("tau", "sigma", "omega", "eps_in"):
            assert tr[key][k] == pytest.approx(ot[key], rel=ITER_TOL), (prob.name, k, key)
        assert tr["inner"][k] == ot["inner"], (prob.name, k, "inner")
        if k < last or o.status == "OPTIMAL":
            assert bool(tr["check"][k]) == bool(ot["check"]), (prob.name, k, "check")
            assert bool(tr["restart"][k]) == bool(ot["restart"]), (prob.name, k, "restart")
            if ot["check"]:
                assert tr["E"][k] == pytest.approx(ot["E"], rel=1e-9, abs=1e-300)
    return g, o


def final_parity(prob, **kw):
    print(f"[final] {prob.name} n={prob.n} m={prob.m} {kw}", flush=True)
    g = G.solve(prob, **kw)
    okw = {k: v for k, v in kw.items() if k not in ("grid_dim", "lanes_at", "lanes_a")}
    o = pdhg.solve(prob, oracle_settings(**okw))
    assert g["status"] == o.status
    for key in ("rel_primal", "rel_dual", "rel_gap"):
        assert abs(g[key] - o.kkt[key]) <= FINAL_TOL, (key, g[key], o.kkt[key])
    for key in ("primal_obj", "dual_obj"):
        assert abs(g[key] - o.kkt[key]) <= FINAL_TOL * max(1.0, abs(o.kkt[key])), key
    return g, o


def recheck_kkt(prob, g, tol):
    """Residuals of the returned point recomputed on the CPU agree with the
    library's own and meet the tolerance."""
    k = pdhg.kkt_residuals(prob, g["x"], g["y"])
    for key in ("rel_primal", "rel_dual", "rel_gap"):
        assert k[key] <= tol * 1.001, (key, k[key])
        assert abs(k[key] - g[key]) <= 1e-8, (key, k[key], g[key])


# ---------------------------------------------------------------------------
# small instances: 50-iteration parity
# ---------------------------------------------------------------------------
SMALL = [
    ("tiny_qp", lambda: synth.tiny_qp(0)),
    ("tiny_qp_s3", lambda: synth.tiny_qp(3)),
    ("tiny_mixed", lambda: synth.tiny_mixed(0)),
    ("tiny_mixed_diag", lambda: synth.tiny_mixed(1, lowrank=False)),
    ("tiny_mixed_noq", lambda: synth.tiny_mixed(2, with_q=False)),
    ("tiny_free", lambda: synth.tiny_free_qp(1)),
    ("mixed_cone_1k", lambda: synth.mixed_cone_scaled(seed=0, scale=0.01)),
    ("mixed_cone_shuffled", lambda: synth.mixed_cone_scaled(seed=1, scale=0.005, shuffle_blocks=True)),
    ("fisher_60x30", lambda: synth.fisher(seed=3, n_buyers=60, n_goods=30, density=0.2)),
    ("portfolio", lambda: synth.portfolio(1_000_007, n_assets=120, n_factors=7)),
]


@pytest.mark.parametrize("name,make", SMALL, ids=[s[0] for s in SMALL])
def test_iterate_parity_small(name, make):
    trace_parity(make())


@pytest.mark.parametrize("grid", [2, 7])
def test_iterate_parity_multi_workgroup(grid):
    """Several workgroups on a small problem: exercises the grid barrier and
    the cross-workgroup reductions."""
    trace_parity(synth.mixed_cone_scaled(seed=4, scale=0.02), grid_dim=grid)
    trace_parity(synth.tiny_qp(1), grid_dim=grid, lanes_at=4, lanes_a=2)


@pytest.mark.parametrize("lanes", [1, 2, 16, 64])
def test_iterate_parity_lane_mappings(lanes):
    trace_parity(synth.fisher(seed=5, n_buyers=40, n_goods=25, density=0.3), iters=30,
                 lanes_at=lanes, lanes_a=lanes, grid_dim=3)


def edge_cone_problem(seed=0, m=9):
    """Blocks that stress the work mapping: an SOC longer than one wavefront,
    an RSOC without v part, a 1-dimensional SOC, power cones with extreme
    exponents, free coordinates."""
    rng = np.random.default_rng(seed)
    spec = [("soc", 150, 0.0), ("rsoc", 2, 0.0), ("soc", 1, 0.0), ("pow", 3, 0.05),
            ("pow", 3, 0.95), ("exp", 3, 0.0), ("rsoc", 70, 0.0), ("free", 3, 0.0),
            ("nonneg", 5, 0.0)]
    cones, st = [], 0
    for kind, d, al in spec:
        cones.append((kind, st, d, al))
        st += d
    n = st
    A = sp.random(m, n, density=0.3, random_state=rng, data_rvs=rng.standard_normal, format="csr")
    x0 = synth._interior_point(rng, n, cones)
    P = sp.diags(rng.uniform(0.1, 1.0, size=n)).tocsr()
    R = rng.standard_normal((3, n)) / math.sqrt(n)
    return Problem(n=n, m=m, A=A, b=A @ x0, c=rng.standard_normal(n), P=P, R=R, D=np.eye(3),
                   cones=cones, name="edge_cones")


def test_iterate_parity_edge_cones():
    trace_parity(edge_cone_problem())
    trace_parity(edge_cone_problem(1), grid_dim=3)


def test_iterate_parity_no_rows():
    """m = 0: minimise 1/2 x'Qx + c'x over K (the dual step is void)."""
    p = synth.tiny_mixed(4)
    q = Problem(n=p.n, m=0, A=sp.csr_matrix((0, p.n)), b=np.zeros(0), c=p.c, P=p.P, R=p.R,
                D=p.D, cones=p.cones, name="no_rows")
    trace_parity(q, iters=30)


@pytest.mark.parametrize("opt", [dict(inner="euclid"), dict(fixed_inner=3), dict(rho=0.5),
                                 dict(scaling=False), dict(check_every=1)])
def test_iterate_parity_options(opt):
    o = dict(opt)
    ce = o.pop("check_every", 4)
    trace_parity(synth.mixed_cone_scaled(seed=2, scale=0.006), check_every=ce, **o)


def test_iterate_parity_warm_start():
    p = synth.tiny_mixed(0)
    rng = np.random.default_rng(0)
    trace_parity(p, x0=rng.standard_normal(p.n), y0=rng.standard_normal(p.m))


# ---------------------------------------------------------------------------
# whole solves
# ---------------------------------------------------------------------------
@pytest.mark.parametrize("seed", [0, 1, 2])
def test_final_parity_tiny_qp(seed):
    g, o = final_parity(synth.tiny_qp(seed))
    assert g["iterations"] == o.iterations
    recheck_kkt(synth.tiny_qp(seed), g, 1e-6)


def test_final_parity_mixed():
    p = synth.mixed_cone_scaled(seed=0, scale=0.004)
    g, o = final_parity(p, max_iter=100000)
    recheck_kkt(p, g, 1e-6)


def test_final_parity_fisher():
    p = synth.fisher(seed=7, n_buyers=50, n_goods=20, density=0.25)
    g, o = final_parity(p, max_iter=200000)
    recheck_kkt(p, g, 1e-6)


def test_status_max_iter_and_determinism():
    p = synth.mixed_cone_scaled(seed=3, scale=0.01)
    a = G.solve(p, max_iter=77, grid_dim=5)
    b = G.solve(p, max_iter=77, grid_dim=5)
    assert a["status"] == "MAX_ITER" and a["iterations"] == 77
    assert np.array_equal(a["x"], b["x"]) and np.array_equal(a["y"], b["y"])


def test_dual_slack_output():
    p = synth.tiny_mixed(0)
    g = G.solve(p, want_s=True)
    Q = p.P.toarray() + p.R.T @ p.D @ p.R
    s = Q @ g["x"] + p.c - p.A.T @ g["y"]
    np.testing.assert_allclose(g["s"], s, rtol=1e-9, atol=1e-12)


# ---------------------------------------------------------------------------
# full-size instances (the benchmark shapes), launch configuration of bench.py
# ---------------------------------------------------------------------------
def test_full_size_mixed_cone_first_iterations():
    p = synth.mixed_cone(seed=0)
    trace_parity(p, iters=3, check_every=64)


def test_full_size_fisher_first_iterations():
    p = synth.fisher(seed=1_000_001)
    trace_parity(p, iters=3, check_every=64)


def test_full_size_tiny_qp_config_solve():
    p = synth.tiny_qp(0)
    g = G.solve(p)
    recheck_kkt(p, g, 1e-6)
