"""GPU parity on Fisher markets of the paper's recipe (valuations and
budgets U[0.1, 1.1], supplies 0.2 n) in the paper's representation, the
exponential blocks (z_i, 1, t_i) with the middle coordinate fixed at one:
a small member iterate by iterate and to the end against the oracle (and
the explicit-row form once), and the paper's n = 1000 shape (400 goods,
density 0.2) over 50 iterations and through a whole solve rechecked on the
CPU, with the equilibrium conditions of the market."""
import numpy as np
import pytest

import paper_2608_09159_amd as G
from instances import synth
from oracle import pdhg
from parity_util import assert_final_matches, oracle_settings, recheck_kkt, trace_parity

pytestmark = pytest.mark.gpu


def _small(middle="fixed"):
    return synth.fisher(seed=1, n_buyers=60, n_goods=24, density=0.25, graph_seed=1, dist="paper",
                        middle=middle)


@pytest.mark.parametrize("middle", ["fixed", "row"])
def test_fisher_paper_small_iterates(middle):
    trace_parity(_small(middle), iters=50, check_every=4)


@pytest.mark.parametrize("middle,kw", [("fixed", {}), ("fixed", {"grid_dim": 3}), ("row", {})])
def test_fisher_paper_small_final(middle, kw):
    p = _small(middle)
    g = G.solve(p, max_iter=200000, **kw)
    o = pdhg.solve(p, oracle_settings(max_iter=200000))
    print(f"[fisher paper small {middle}] gpu {g['iterations']} it, oracle {o.iterations} it", flush=True)
    assert g["status"] == "OPTIMAL"
    assert_final_matches(g, o)


def _equilibrium(p, g):
    """Prices (negated duals of the supply rows) are nonnegative and each
    buyer spends its budget (prices . allocation + retained money)."""
    m_goods = p.meta["n_goods"]
    prices = -g["y"][:m_goods]
    assert prices.min() >= -1e-6 * max(1.0, prices.max())
    bi, gj = p.meta["graph"]
    e = bi.size
    nb = p.meta["n_buyers"]
    spend = np.bincount(bi, weights=prices[gj] * g["x"][:e], minlength=nb) + g["x"][e:e + nb]
    np.testing.assert_allclose(spend, p.meta["w"], rtol=1e-3, atol=1e-3)


@pytest.mark.timeout(300)
def test_fisher_paper_1000_buyers():
    p = synth.fisher_paper(1000)
    trace_parity(p, iters=50, check_every=4)
    g = G.solve(p)
    print(f"[fisher paper 1000] {g['status']} {g['iterations']} it {g['solve_s']:.3f} s", flush=True)
    assert g["status"] == "OPTIMAL"
    recheck_kkt(p, g, 1e-6)
    _equilibrium(p, g)
