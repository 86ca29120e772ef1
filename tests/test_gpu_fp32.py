"""GPU checks of the FP32-bulk mode (settings.precision = fp32): FP32 copies
of A, A^T, P and R for the bulk sweeps, FP64 iterates, reductions, restart
and KKT checks, then an FP64 polish to the requested tolerance.

Parity status: the FP32 phase has no exact reference (the oracle is FP64),
so its iterates are reported against the FP64 oracle with a bound written
here (error report, parity unpinned).  The polished results reach the
tolerance: KKT residuals of the returned point, recomputed on the CPU in
FP64, within 1e-6, the same status as the oracle, and objectives within
1e-5 relative of the oracle's (two different 1e-6-accurate points; their
objectives may differ by a few times the gap tolerance)."""
import numpy as np
import pytest

import paper_2608_09159_amd as G
from instances import synth
from oracle import pdhg
from parity_util import oracle_settings, recheck_kkt

pytestmark = pytest.mark.gpu


def _rel(a, b):
    return float(np.max(np.abs(a - b))) / max(float(np.max(np.abs(b))), 1e-300)


@pytest.mark.parametrize("make,grid", [(lambda: synth.mixed_cone_scaled(seed=0, scale=0.01), 0),
                                       (lambda: synth.tiny_qp(1), 0),
                                       (lambda: synth.fisher(seed=3, n_buyers=60, n_goods=30, density=0.2), 0),
                                       (lambda: synth.large_sparse_qp(seed=1, n=60_000, m=30_000), 0),
                                       (lambda: synth.bounded_qp(9, n_cone_soc=0, n_exp=0), 4)],
                         ids=["mixed_cone_1k", "tiny_qp", "fisher_60x30", "large_sparse_qp_60k",
                              "cone_free_bounded_grid4"])
def test_fp32_first_iterations_error_report(make, grid):
    """First 20 iterations (fixed inner count, one check) of the FP32 phase
    against the FP64 oracle: relative error of every iterate below 1e-4
    (cone-free problems on several workgroups run the FP32 cone-free
    kernels)."""
    p = make()
    iters = 20
    kw = dict(trace_iters=iters, max_iter=iters, check_every=64, fixed_inner=3)
    h = G.setup(p, precision="fp32", grid_dim=grid, **kw)
    try:
        h.solve()
        tr = h.trace(iters)
    finally:
        h.free()
    o = pdhg.solve(p, oracle_settings(**kw))
    worst = 0.0
    for k, ot in enumerate(o.trace):
        for key in ("x", "y", "wx", "wy"):
            worst = max(worst, _rel(tr[key][k], ot[key]))
    print(f"[fp32] {p.name}: max relative iterate error over {iters} iterations = {worst:.3e}",
          flush=True)
    assert worst <= 1e-4


@pytest.mark.parametrize("make,grid", [(lambda: synth.mixed_cone_scaled(seed=0, scale=0.004), 0),
                                       (lambda: synth.tiny_qp(0), 0),
                                       (lambda: synth.fisher(seed=7, n_buyers=50, n_goods=20, density=0.25), 0),
                                       (lambda: synth.bounded_qp(12, n_cone_soc=0, n_exp=0), 4)],
                         ids=["mixed_cone", "tiny_qp", "fisher", "cone_free_bounded_grid4"])
def test_fp32_polished_solve_matches_oracle(make, grid):
    p = make()
    g = G.solve(p, precision="fp32", fp32_tol=1e-4, max_iter=200000, grid_dim=grid)
    o = pdhg.solve(p, oracle_settings(max_iter=200000))
    dx = np.linalg.norm(g["x"] - o.x) / max(np.linalg.norm(o.x), 1e-300)
    print(f"[fp32] {p.name}: {g['iterations']} it ({g['polish_iterations']} FP64 polish), "
          f"oracle {o.iterations} it, |dx|/|x| = {dx:.3e}, "
          f"dobj = {abs(g['primal_obj'] - o.kkt['primal_obj']):.3e}", flush=True)
    assert g["polish_iterations"] > 0
    assert g["status"] == o.status == "OPTIMAL"
    for key in ("primal_obj", "dual_obj"):
        assert abs(g[key] - o.kkt[key]) <= 1e-5 * max(1.0, abs(o.kkt[key])), key
    recheck_kkt(p, g, 1e-6)


def test_fp32_without_polish_when_tolerances_meet():
    """fp32_tol <= tol: the FP32 phase alone runs to tol (no polish)."""
    p = synth.tiny_qp(2)
    g = G.solve(p, precision="fp32", fp32_tol=1e-6)
    assert g["polish_iterations"] == 0
    if g["status"] == "OPTIMAL":
        recheck_kkt(p, g, 1e-6)


def test_fp32_full_size_mixed_cone():
    """The benchmark instance in FP32 mode reaches 1e-6 relative KKT (checked
    on the CPU in FP64); error of x against the FP64 GPU solve reported."""
    p = synth.mixed_cone(seed=0)
    g32 = G.solve(p, precision="fp32")
    g64 = G.solve(p)
    dx = np.linalg.norm(g32["x"] - g64["x"]) / np.linalg.norm(g64["x"])
    print(f"[fp32] mixed_cone: fp32 {g32['iterations']} it ({g32['polish_iterations']} polish), "
          f"fp64 {g64['iterations']} it, |dx|/|x| = {dx:.3e}", flush=True)
    assert g32["status"] == "OPTIMAL"
    recheck_kkt(p, g32, 1e-6)
    assert abs(g32["primal_obj"] - g64["primal_obj"]) <= 1e-5 * max(1.0, abs(g64["primal_obj"]))
