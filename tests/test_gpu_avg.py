"""GPU parity of the restarted averaged PDHG iteration (Alg. 1: fixed step
sizes, plain PDHG steps, Cesaro average of each epoch, restart from the
average, termination tested on it) against the oracle's averaged scheme:
iterates, step sizes, inner tolerances and epoch ends over the first 50
iterations to 1e-10, and whole solves with equal counts."""
import numpy as np
import pytest

import paper_2608_09159_amd as G
from instances import synth
from oracle import pdhg
from parity_util import assert_final_matches, assert_trace_matches, oracle_settings, recheck_kkt, trace_parity

pytestmark = pytest.mark.gpu

CASES = [
    ("tiny_qp", lambda: synth.tiny_qp(0), {}),
    ("tiny_mixed", lambda: synth.tiny_mixed(0), {}),
    ("tiny_mixed_diag_grid3", lambda: synth.tiny_mixed(1, lowrank=False), {"grid_dim": 3}),
    ("mixed_cone_2k_grid7", lambda: synth.mixed_cone_scaled(seed=4, scale=0.02), {"grid_dim": 7}),
    ("fisher_60x30", lambda: synth.fisher(seed=3, n_buyers=60, n_goods=30, density=0.2), {}),
    ("portfolio", lambda: synth.portfolio(1_000_007, n_assets=120, n_factors=7), {}),
]


@pytest.mark.parametrize("name,make,kw", CASES, ids=[c[0] for c in CASES])
def test_avg_iterate_parity(name, make, kw):
    trace_parity(make(), iters=50, scheme="avg", avg_epoch=8, **kw)


def test_avg_iterate_parity_epoch_one_and_max_iter_mid_epoch():
    """T = 1 (every step restarts from itself) and a run cut by max_iter in
    the middle of an epoch (the partial average is the restart point)."""
    trace_parity(synth.tiny_mixed(2, with_q=False), iters=20, scheme="avg", avg_epoch=1)
    trace_parity(synth.tiny_qp(1), iters=29, scheme="avg", avg_epoch=8)


@pytest.mark.parametrize("name,make,T", [
    ("nonneg_diag", lambda: synth.tiny_nonneg_qp(2, n=8, m=3, diag_only=True), 16),
    ("tiny_mixed_noq", lambda: synth.tiny_mixed(2, with_q=False), 32),
])
def test_avg_final_parity(name, make, T):
    p = make()
    kw = dict(scheme="avg", avg_epoch=T, max_iter=200000)
    print(f"[avg final] {p.name} T={T}", flush=True)
    g = G.solve(p, **kw)
    o = pdhg.solve(p, oracle_settings(**kw))
    print(f"  gpu {g['status']} {g['iterations']} it, oracle {o.status} {o.iterations} it", flush=True)
    assert g["status"] == "OPTIMAL"
    assert_final_matches(g, o)
    recheck_kkt(p, g, 1e-6)


def test_avg_batch_matches_oracle():
    """The batch kernels (one workgroup per instance) run the same averaged
    epochs: each instance's trace matches the oracle."""
    ps = [synth.tiny_qp(2), synth.tiny_mixed(3), synth.portfolio(1_000_011, n_assets=90, n_factors=5)]
    iters = 40
    h = G.setup_batch(ps, scheme="avg", avg_epoch=8, trace_iters=iters, max_iter=iters, check_every=4)
    try:
        h.solve()
        traces = [h.trace(iters, inst=i) for i in range(len(ps))]
    finally:
        h.free()
    for i, p in enumerate(ps):
        o = pdhg.solve(p, oracle_settings(scheme="avg", avg_epoch=8, trace_iters=iters, max_iter=iters,
                                          check_every=4))
        assert_trace_matches(f"{p.name}#{i}", traces[i], o)


def test_avg_rejects_fp32():
    with pytest.raises(RuntimeError):
        G.setup(synth.tiny_qp(0), scheme="avg", precision="fp32")
