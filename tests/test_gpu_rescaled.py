"""GPU parity of the rescaled-cone scaling mode (cone_scaling = "rescaled",
Section "Problem Rescaling", eq. scaling-induced-metric): coordinatewise
factors on the SOC, RSOC, EXP and POW blocks, each block projected onto
S_j K_j through the metric S_j M S_j.

Iterates against the oracle's trace (relative 1e-10 over 50 iterations),
whole solves with the oracle's counts, the prox in both inner metrics, a
batch, and the device answer against the cone-preserving mode's."""
import numpy as np
import pytest

import paper_2608_09159_amd as G
from instances import synth
from oracle import pdhg
from parity_util import (assert_final_matches, assert_trace_matches, edge_cone_problem, final_parity,
                         oracle_settings, recheck_kkt, trace_parity)

pytestmark = pytest.mark.gpu

RESC = dict(cone_scaling="rescaled")


@pytest.mark.parametrize("make", [lambda: synth.tiny_mixed(4), lambda: synth.tiny_mixed(2, with_q=False),
                                  lambda: synth.tiny_mixed(6, lowrank=False), lambda: edge_cone_problem(1),
                                  lambda: synth.mixed_cone_scaled(seed=3, scale=0.02)],
                         ids=["lowrank", "noq", "diag", "edge", "mixed_small"])
def test_rescaled_iterate_parity(make):
    trace_parity(make(), iters=50, check_every=4, **RESC)


@pytest.mark.parametrize("grid", [3, 16])
def test_rescaled_iterate_parity_grids(grid):
    trace_parity(synth.mixed_cone_scaled(seed=5, scale=0.02), iters=40, check_every=4, grid_dim=grid, **RESC)


def test_rescaled_iterate_parity_euclid_inner():
    """Projected BB in the Euclidean metric: the cone blocks still carry the
    metric S_j^2."""
    trace_parity(synth.tiny_mixed(7), iters=40, check_every=4, inner="euclid", **RESC)


def test_rescaled_iterate_parity_fisher_fixed_middle():
    """EXP1 blocks keep one common factor beside rescaled R+ coordinates."""
    p = synth.fisher(seed=1, n_buyers=60, n_goods=24, density=0.25, graph_seed=1, dist="paper", middle="fixed")
    trace_parity(p, iters=40, check_every=4, **RESC)


@pytest.mark.parametrize("make", [lambda: synth.tiny_mixed(4), lambda: synth.tiny_mixed(5, lowrank=False)],
                         ids=["lowrank", "diag"])
def test_rescaled_final_parity(make):
    p = make()
    g, o = final_parity(p, tol=1e-7, **RESC)
    recheck_kkt(p, g, 1e-7)


def test_rescaled_matches_block_mode_answer():
    """The scaling changes the path, not the answer."""
    p = synth.mixed_cone_scaled(seed=2, scale=0.02)
    gb = G.solve(p, tol=1e-8)
    gr = G.solve(p, tol=1e-8, **RESC)
    print(f"[rescaled vs block] block {gb['iterations']} it, rescaled {gr['iterations']} it", flush=True)
    assert gb["status"] == gr["status"] == "OPTIMAL"
    assert gr["primal_obj"] == pytest.approx(gb["primal_obj"], rel=1e-6, abs=1e-8)
    recheck_kkt(p, gr, 1e-8)


def test_rescaled_batch_parity():
    ps = [synth.tiny_mixed(4), edge_cone_problem(2), synth.tiny_qp(1)]
    iters = 40
    h = G.setup_batch(ps, trace_iters=iters, check_every=4, max_iter=iters, **RESC)
    try:
        h.solve()
        traces = [h.trace(iters, inst=i) for i in range(len(ps))]
    finally:
        h.free()
    for i, p in enumerate(ps):
        print(f"  [{i}] {p.name}", flush=True)
        o = pdhg.solve(p, oracle_settings(trace_iters=iters, check_every=4, max_iter=iters, **RESC))
        assert_trace_matches(f"{p.name}#{i}", traces[i], o)
