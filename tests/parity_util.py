"""Shared parity helpers of the GPU tests: library results against the CPU
oracle (iterate traces, final residuals, KKT rechecks) and a problem whose
cone blocks stress the work mapping."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

import paper_2608_09159_amd as G
from instances import Problem, synth
from oracle import pdhg

ITER_TOL = 1e-10
FINAL_OBJ_TOL = 1e-8
FINAL_RES_RTOL = 1e-3
FINAL_XY_TOL = 1e-7


def _rel(a, b):
    scale = max(float(np.max(np.abs(b))) if b.size else 0.0, 1e-300)
    return float(np.max(np.abs(a - b))) / scale if b.size else 0.0


def oracle_settings(**kw):
    st = pdhg.Settings()
    for k, v in kw.items():
        setattr(st, k, v)
    return st


def trace_parity(prob, iters=50, check_every=4, x0=None, y0=None, **kw):
    okw = {k: v for k, v in kw.items() if k not in ("grid_dim", "lanes_at", "lanes_a", "interleave")}
    print(f"[parity] {prob.name} n={prob.n} m={prob.m} iters={iters} {kw}", flush=True)
    h = G.setup(prob, trace_iters=iters, check_every=check_every, max_iter=iters, **kw)
    try:
        g = h.solve(x0, y0)
        tr = h.trace(iters)
    finally:
        h.free()
    o = pdhg.solve(prob, oracle_settings(trace_iters=iters, check_every=check_every,
                                         max_iter=iters, **okw), x0=x0, y0=y0)
    assert_trace_matches(prob.name, tr, o)
    return g, o


def assert_trace_matches(name, tr, o):
    """Library trace `tr` against the oracle result `o`, iteration by
    iteration (the inner-step counts, check and restart decisions exactly)."""
    prob_name = name
    assert tr["count"] == len(o.trace), (tr["count"], len(o.trace))
    for k, ot in enumerate(o.trace):
        for key in ("x", "y", "wx", "wy"):
            err = _rel(tr[key][k], ot[key])
            assert err <= ITER_TOL, (prob_name, k, key, err)
        for key in ("tau", "sigma", "omega", "eps_in"):
            assert tr[key][k] == pytest.approx(ot[key], rel=ITER_TOL), (prob_name, k, key)
        assert tr["inner"][k] == ot["inner"], (prob_name, k, "inner")
        assert bool(tr["check"][k]) == bool(ot["check"]), (prob_name, k, "check")
        assert bool(tr["restart"][k]) == bool(ot["restart"]), (prob_name, k, "restart")
        if ot["check"] and ot["E"] is not None:
            assert tr["E"][k] == pytest.approx(ot["E"], rel=1e-9, abs=1e-300)


def final_parity(prob, **kw):
    print(f"[final] {prob.name} n={prob.n} m={prob.m} {kw}", flush=True)
    g = G.solve(prob, **kw)
    okw = {k: v for k, v in kw.items() if k not in ("grid_dim", "lanes_at", "lanes_a", "interleave")}
    o = pdhg.solve(prob, oracle_settings(**okw))
    assert_final_matches(g, o)
    return g, o


def assert_final_matches(g, o, same_path=True, inner_slack=0):
    """A library result `g` against the oracle result `o`.

    Always: the same status; the objectives within 1e-8 relative; each
    relative KKT residual within 1e-3 of the oracle's value relative to it
    (floor 1e-11: the residuals are themselves ~tol, so rounding differences
    of the iterates show up in their low digits).  With same_path (the
    default), the two runs took the same discrete decisions: equal outer,
    inner and restart counts, and the returned x and y agree to 1e-7 relative
    in the max norm.  inner_slack allows that many inner steps of
    difference: an inner stop test (||du|| <= eps_in) that falls within
    rounding of its threshold can end one side's inner loop a step earlier
    without changing any outer decision."""
    assert g["status"] == o.status, (g["status"], o.status)
    if same_path:
        assert g["iterations"] == o.iterations, ("iterations", g["iterations"], o.iterations)
        assert g["restarts"] == o.restarts, ("restarts", g["restarts"], o.restarts)
        assert abs(g["inner_iterations"] - o.inner_iterations) <= inner_slack, \
            ("inner", g["inner_iterations"], o.inner_iterations)
        for key, ov in (("x", o.x), ("y", o.y)):
            err = _rel(g[key], ov)
            assert err <= FINAL_XY_TOL, (key, err)
    for key in ("primal_obj", "dual_obj"):
        assert abs(g[key] - o.kkt[key]) <= FINAL_OBJ_TOL * max(1.0, abs(o.kkt[key])), \
            (key, g[key], o.kkt[key])
    for key in ("rel_primal", "rel_dual", "rel_gap"):
        assert abs(g[key] - o.kkt[key]) <= FINAL_RES_RTOL * o.kkt[key] + 1e-11, \
            (key, g[key], o.kkt[key])


def recheck_kkt(prob, g, tol):
    """Residuals of the returned point recomputed on the CPU agree with the
    library's own and meet the tolerance."""
    k = pdhg.kkt_residuals(prob, g["x"], g["y"])
    for key in ("rel_primal", "rel_dual", "rel_gap"):
        assert k[key] <= tol * 1.001, (key, k[key])
        assert abs(k[key] - g[key]) <= 1e-8, (key, k[key], g[key])


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


def degree_order_rule(p, ranges=512):
    """The device order of PDHCG_ORDER_DEGREE recomputed from its stated
    rule: columns by their count of nonzeros in A, longest first (ties in the
    caller's order); the head (counts >= max(4096, (nnz(A) + nnz(P)) / 512 /
    8)) in that order; then the rest dealt in turn to the 512 ranges less
    the head's workgroups (head rows packed in order up to a 1/512 share of
    the A^T and P nonzeros)."""
    deg = np.bincount(p.A.indices, minlength=p.n)
    pnz = np.diff(p.P.tocsr().indptr) if p.P is not None else np.zeros(p.n, dtype=np.int64)
    order = np.argsort(-deg, kind="stable")
    share = (p.A.nnz + (p.P.nnz if p.P is not None else 0)) / ranges
    head = int(np.sum(deg >= max(4096.0, share / 8.0)))
    bins, cur = 0, 0.0
    for i in order[:head]:
        z = float(deg[i] + pnz[i])
        if cur > 0.0 and cur + z > share:
            bins, cur = bins + 1, 0.0
        cur += z
    bins += head > 0
    rest = order[head:]
    R = max(1, min(max(ranges - bins, 1), rest.size))
    return np.concatenate([order[:head]] + [rest[r::R] for r in range(R)]), head
