"""GPU parity of the implementation form (eq. solver-input): two-sided row
bounds and box blocks, through the C ABI against the oracle.  Iterates of
the first 50 iterations to 1e-10 (single workgroup, several workgroups,
diagonal, low-rank and zero Q, averaged epochs, with and without cone blocks:
the cone-free instances run the cone-free kernel), whole solves with equal
counts, and a batch mixing bounded and equality instances."""
import numpy as np
import pytest

import paper_2608_09159_amd as G
from instances import synth
from oracle import pdhg
from parity_util import (assert_final_matches, assert_trace_matches, oracle_settings, recheck_kkt,
                         trace_parity)

pytestmark = pytest.mark.gpu

CASES = [
    ("lowrank", lambda: synth.bounded_qp(0), {}),
    ("diag", lambda: synth.bounded_qp(1, q="diag"), {}),
    ("lp", lambda: synth.bounded_qp(2, q=None), {}),
    ("lowrank_grid5", lambda: synth.bounded_qp(4), {"grid_dim": 5}),
    ("large_grid", lambda: synth.bounded_qp(3, n_box=3000, n_cone_soc=40, n_exp=20, m=1500, density=0.004), {}),
    ("avg", lambda: synth.bounded_qp(5, q="diag"), {"scheme": "avg", "avg_epoch": 8}),
    # without cone blocks: the cone-free kernel with the implementation form
    ("cone_free_grid4", lambda: synth.bounded_qp(9, n_cone_soc=0, n_exp=0), {"grid_dim": 4}),
    ("cone_free_lp_large", lambda: synth.bounded_qp(10, n_box=3000, n_cone_soc=0, n_exp=0, m=1500,
                                                     density=0.004, q=None), {}),
]


@pytest.mark.parametrize("name,make,kw", CASES, ids=[c[0] for c in CASES])
def test_bounded_iterate_parity(name, make, kw):
    trace_parity(make(), iters=50, **kw)


@pytest.mark.parametrize("name,make", [
    ("lowrank", lambda: synth.bounded_qp(0)),
    ("lp", lambda: synth.bounded_qp(2, q=None)),
    ("large", lambda: synth.bounded_qp(3, n_box=3000, n_cone_soc=40, n_exp=20, m=1500, density=0.004)),
    ("cone_free_large", lambda: synth.bounded_qp(11, n_box=3000, n_cone_soc=0, n_exp=0, m=1500, density=0.004)),
])
def test_bounded_final_parity(name, make):
    p = make()
    print(f"[bounded final] {p.name}", flush=True)
    g = G.solve(p, max_iter=100000)
    o = pdhg.solve(p, oracle_settings(max_iter=100000))
    print(f"  gpu {g['status']} {g['iterations']} it, oracle {o.status} {o.iterations} it", flush=True)
    assert g["status"] == "OPTIMAL"
    assert_final_matches(g, o)
    recheck_kkt(p, g, 1e-6)
    # the returned point keeps every box bound (clamped in the scaled space,
    # so to rounding of the unscaling)
    box = [st for k, st, d, a in p.cones if k == "box"]
    for k, st, d, a in p.cones:
        if k == "box":
            x, lo, hi = g["x"][st:st + d], p.x_lo[st:st + d], p.x_hi[st:st + d]
            slack = 4e-16 * np.maximum(1.0, np.abs(x))
            assert np.all(x >= lo - slack) and np.all(x <= hi + slack)
    assert box


def test_bounded_batch_matches_single_and_oracle():
    ps = [synth.bounded_qp(6), synth.tiny_qp(1), synth.bounded_qp(7, q=None), synth.tiny_mixed(2)]
    iters = 40
    h = G.setup_batch(ps, trace_iters=iters, max_iter=iters, check_every=4)
    try:
        h.solve()
        traces = [h.trace(iters, inst=i) for i in range(len(ps))]
    finally:
        h.free()
    for i, p in enumerate(ps):
        o = pdhg.solve(p, oracle_settings(trace_iters=iters, check_every=4, max_iter=iters))
        assert_trace_matches(f"{p.name}#{i}", traces[i], o)


def test_bounded_warm_start_and_dual_slack():
    p = synth.bounded_qp(8)
    rng = np.random.default_rng(3)
    trace_parity(p, iters=30, x0=rng.standard_normal(p.n), y0=rng.standard_normal(p.m))
