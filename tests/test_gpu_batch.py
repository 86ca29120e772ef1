"""GPU parity of the batched solve (pdhcg_solve_batch): many independent
instances in one persistent launch, one workgroup per instance, each with its
own step sizes, primal weight, restarts and inner tolerance.

* Iterate parity: every instance of a heterogeneous batch (portfolio QPs,
  tiny QPs, every cone type, a Fisher market, an instance without rows)
  matches the oracle's first 50 iterations to 1e-10, as single solves do.
* Final parity: status, residuals and objectives of every instance match the
  oracle's whole solve to 1e-6.
* Equivalence: with the same step size and lane mapping, an instance solved
  in a batch and solved alone through pdhcg_solve (one workgroup) produce
  bit-identical results, with and without warm starts.
* The portfolio batch of the benchmark (4096 instances) solves to 1e-6 with
  residuals rechecked on the CPU, and a sample matches the oracle.
"""
import numpy as np
import pytest
import scipy.sparse as sp

import paper_2608_09159_amd as G
from instances import Problem, synth
from oracle import pdhg
from parity_util import (assert_final_matches, assert_trace_matches, edge_cone_problem,
                         oracle_settings, recheck_kkt)

pytestmark = pytest.mark.gpu


def no_rows(seed):
    p = synth.tiny_mixed(seed)
    return Problem(n=p.n, m=0, A=sp.csr_matrix((0, p.n)), b=np.zeros(0), c=p.c, P=p.P, R=p.R,
                   D=p.D, cones=p.cones, name="no_rows")


def mixed_batch():
    ps = [synth.portfolio(1_000_000 + i, n_assets=na, n_factors=k)
          for i, (na, k) in enumerate([(60, 5), (200, 12), (35, 20), (120, 7), (700, 9)])]
    ps += [synth.tiny_qp(0), synth.tiny_mixed(0), synth.tiny_mixed(1, lowrank=False),
           synth.tiny_mixed(2, with_q=False), synth.fisher(seed=3, n_buyers=60, n_goods=30, density=0.2),
           edge_cone_problem(2), no_rows(5), synth.tiny_free_qp(3)]
    return ps


def test_batch_iterate_parity():
    ps = mixed_batch()
    iters = 50
    print(f"[batch trace] {len(ps)} instances", flush=True)
    h = G.setup_batch(ps, trace_iters=iters, check_every=4, max_iter=iters)
    try:
        res = h.solve()
        traces = [h.trace(iters, inst=i) for i in range(len(ps))]
    finally:
        h.free()
    for i, p in enumerate(ps):
        print(f"  [{i}] {p.name} n={p.n} m={p.m} status={res[i]['status']}", flush=True)
        o = pdhg.solve(p, oracle_settings(trace_iters=iters, check_every=4, max_iter=iters))
        assert_trace_matches(f"{p.name}#{i}", traces[i], o)


def test_batch_final_parity():
    ps = mixed_batch()
    print(f"[batch final] {len(ps)} instances", flush=True)
    h = G.setup_batch(ps, max_iter=200000)
    try:
        res = h.solve()
    finally:
        h.free()
    for i, p in enumerate(ps):
        o = pdhg.solve(p, oracle_settings(max_iter=200000))
        print(f"  [{i}] {p.name} gpu {res[i]['iterations']} it, oracle {o.iterations} it", flush=True)
        assert_final_matches(res[i], o)
        recheck_kkt(p, res[i], 1e-6)


def test_batch_step_sizes_per_instance():
    """Each instance gets its own ||A||_2 from the batched power iteration,
    equal to the oracle's power iteration on the same scaled matrix."""
    ps = mixed_batch()
    h = G.setup_batch(ps, max_iter=1)
    try:
        etas = [h.scaling(i)["eta"] for i in range(len(ps))]
    finally:
        h.free()
    for i, p in enumerate(ps):
        S = pdhg.setup(p, pdhg.Settings())
        assert etas[i] == pytest.approx(S.eta, rel=1e-12), (i, p.name)
    assert len({round(e, 12) for e in etas}) > 5


def _single_vs_batch(ps, x0s=None, y0s=None):
    kw = dict(a_norm=1.0, autotune=0, max_iter=20000)
    h = G.setup_batch(ps, **kw)
    try:
        res = h.solve(x0s, y0s)
    finally:
        h.free()
    for i, p in enumerate(ps):
        # alone on one workgroup, as each instance of the batch is
        g = G.solve(p, x0=None if x0s is None else x0s[i], y0=None if y0s is None else y0s[i],
                    grid_dim=1, **kw)
        print(f"  [{i}] {p.name}: batch {res[i]['iterations']} it, single {g['iterations']} it",
              flush=True)
        assert res[i]["status"] == g["status"]
        assert res[i]["iterations"] == g["iterations"]
        assert res[i]["inner_iterations"] == g["inner_iterations"]
        assert np.array_equal(res[i]["x"], g["x"]), i
        assert np.array_equal(res[i]["y"], g["y"]), i


def test_batch_equals_single_solves():
    ps = [synth.portfolio(1_000_100 + i, n_assets=na) for i, na in enumerate([80, 300, 450])]
    ps += [synth.tiny_qp(2), synth.tiny_mixed(3), synth.fisher(seed=4, n_buyers=40, n_goods=20,
                                                               density=0.25)]
    print(f"[batch vs single] {len(ps)} instances", flush=True)
    _single_vs_batch(ps)


def test_batch_without_cones_equals_single_solves():
    """A batch whose blocks are all R+ runs the cone-free kernel variant; its
    results are still bit-identical to single solves."""
    ps = [synth.portfolio(1_000_500 + i, n_assets=na) for i, na in enumerate([90, 250, 480, 60])]
    ps.append(synth.tiny_qp(5))
    print(f"[batch lin vs single] {len(ps)} instances", flush=True)
    _single_vs_batch(ps)


def test_batch_warm_start_equals_single():
    ps = [synth.tiny_mixed(6), synth.portfolio(1_000_200, n_assets=150), synth.tiny_qp(4)]
    rng = np.random.default_rng(11)
    x0s = [rng.standard_normal(ps[0].n), None, np.abs(rng.standard_normal(ps[2].n))]
    y0s = [rng.standard_normal(ps[0].m), rng.standard_normal(ps[1].m), None]
    print("[batch warm] 3 instances", flush=True)
    _single_vs_batch(ps, x0s, y0s)


def test_batch_repeated_solves_identical():
    """The graph replays: a second and third solve of the same batch give the
    same result, cold after warm included."""
    ps = [synth.portfolio(1_000_300 + i) for i in range(6)]
    h = G.setup_batch(ps, autotune=0)
    try:
        a = h.solve()
        b = h.solve(x0s=[r["x"] for r in a], y0s=[r["y"] for r in a])
        c = h.solve()
    finally:
        h.free()
    for ra, rb, rc in zip(a, b, c):
        assert ra["status"] == "OPTIMAL" and rb["status"] == "OPTIMAL"
        assert rb["iterations"] <= ra["iterations"]
        assert rc["iterations"] == ra["iterations"]
        assert np.array_equal(rc["x"], ra["x"]) and np.array_equal(rc["y"], ra["y"])


def test_batch_max_iter_status():
    ps = [synth.portfolio(1_000_400 + i, n_assets=200) for i in range(4)]
    h = G.setup_batch(ps, max_iter=7, autotune=0)
    try:
        res = h.solve()
    finally:
        h.free()
    for r in res:
        assert r["status"] == "MAX_ITER" and r["iterations"] == 7


def test_full_size_portfolio_batch():
    """The benchmark batch: 4096 portfolio QPs (n ~ U{50..2000}), autotuned
    lane mapping, one graph launch."""
    ps = synth.portfolio_batch(4096)
    print(f"[batch 4096] sum n = {sum(p.n for p in ps)}", flush=True)
    h = G.setup_batch(ps)
    try:
        res = h.solve()
    finally:
        h.free()
    st = [r["status"] for r in res]
    assert st.count("OPTIMAL") == len(ps), {s: st.count(s) for s in set(st)}
    rng = np.random.default_rng(0)
    for i in rng.choice(len(ps), size=16, replace=False):
        recheck_kkt(ps[i], res[i], 1e-6)
    for i in (0, 1, 2):
        o = pdhg.solve(ps[i], oracle_settings())
        print(f"  [{i}] n={ps[i].n} gpu {res[i]['iterations']} it, {res[i]['inner_iterations']} inner, "
              f"oracle {o.iterations} it, {o.inner_iterations} inner", flush=True)
        # instance 0 (n = 1380) once ended 2 of 6141 inner steps apart with
        # the same outer iterations and restarts
        assert_final_matches(res[i], o, inner_slack=4)
