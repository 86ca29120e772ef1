"""GPU parity at the benchmark shapes, in the launch configuration bench.py
times (default settings: automatic grid, check every 64 iterations).

* mixed-cone SOCP/QCQP, n = 1e5, m = 5e4: the first 50 outer iterations
  element by element (check every 4 iterations, so restarts and primal
  weight updates happen inside the window), and a whole solve to 1e-6 with
  the same status, outer / inner / restart counts, iterate and objective as
  the oracle.
* Fisher market 1000 x 500 (exponential cones): the first 50 iterations.
* large sparse QP family (power-law column degrees, R+ slack columns) at
  n = 6e4: a whole solve to 1e-6 with the oracle's counts (thousands of
  outer iterations through the heavy-row workgroups and the A^T length
  classes), and at n = 1e6 the first 20 iterations; both again in the
  degree order (PDHCG_ORDER_DEGREE), which the default settings pick for
  the family at n = 1e7.

The oracle runs in this process; each test prints what it runs before it
starts (the oracle's part takes up to about a minute)."""
import time

import numpy as np
import pytest

import paper_2608_09159_amd as G
from instances import synth
from oracle import pdhg
from parity_util import assert_final_matches, oracle_settings, recheck_kkt, trace_parity

pytestmark = pytest.mark.gpu


def _final(prob, **kw):
    print(f"[final] {prob.name} n={prob.n} m={prob.m} {kw}", flush=True)
    g = G.solve(prob, **kw)
    print(f"  gpu {g['status']} {g['iterations']} it, {g['inner_iterations']} inner, "
          f"{g['restarts']} restarts, {g['solve_s']:.3f} s", flush=True)
    t = time.perf_counter()
    o = pdhg.solve(prob, oracle_settings(**{k: v for k, v in kw.items() if k != "interleave"}))
    print(f"  oracle {o.status} {o.iterations} it, {o.inner_iterations} inner, "
          f"{o.restarts} restarts, {time.perf_counter() - t:.1f} s", flush=True)
    assert_final_matches(g, o)
    recheck_kkt(prob, g, kw.get("tol", 1e-6))
    return g, o


@pytest.mark.timeout(300)
def test_mixed_cone_full_size_50_iterations():
    trace_parity(synth.mixed_cone(seed=0), iters=50, check_every=4)


@pytest.mark.timeout(300)
def test_mixed_cone_full_size_final():
    _final(synth.mixed_cone(seed=0))


@pytest.mark.timeout(300)
def test_fisher_full_size_50_iterations():
    trace_parity(synth.fisher(seed=1_000_001), iters=50, check_every=4)


@pytest.mark.timeout(300)
def test_large_sparse_qp_family_final():
    _final(synth.large_sparse_qp(seed=1, n=60_000, m=30_000))


@pytest.mark.timeout(300)
def test_large_sparse_qp_1e6_first_iterations():
    trace_parity(synth.large_sparse_qp(seed=2, n=1_000_000, m=500_000), iters=20, check_every=4)


@pytest.mark.timeout(300)
def test_large_sparse_qp_family_final_degree_order():
    _final(synth.large_sparse_qp(seed=1, n=60_000, m=30_000), interleave="degree")


@pytest.mark.timeout(300)
def test_large_sparse_qp_1e6_degree_order_first_iterations():
    trace_parity(synth.large_sparse_qp(seed=2, n=1_000_000, m=500_000), iters=20, check_every=4,
                 interleave="degree")
