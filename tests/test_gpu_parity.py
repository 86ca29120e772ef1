"""GPU parity: the HIP library (through the C ABI) against the CPU oracle.

Iterate parity: the first 50 outer iterations (Halpern state and PDHG
candidate, scaled space) agree to 1e-10 relative in the max norm of each
vector, with identical inner-step counts, check and restart decisions.
Final parity: objective and the three relative KKT residuals agree to 1e-6
(absolute difference of the relative residuals, relative difference of the
objective).  Full-size instances are checked on a few iterations and, after
a full solve, by recomputing the KKT residuals of the returned point on the
CPU."""
import numpy as np
import pytest
import scipy.sparse as sp

import paper_2608_09159_amd as G
from instances import Problem, synth
from parity_util import degree_order_rule, edge_cone_problem, final_parity, recheck_kkt, trace_parity

pytestmark = pytest.mark.gpu


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


def test_iterate_parity_skewed_columns():
    """Power-law column degrees (the large sparse QP family at n = 60,000):
    the longest A^T rows get workgroups of their own (whole-workgroup rows)
    and the others run in length classes."""
    trace_parity(synth.large_sparse_qp(seed=1, n=60_000, m=30_000), iters=20)


def _partition_dump(prob, tmp_path, **kw):
    """Set up `prob` with the partition dump on; returns the rows
    (workgroup, c0, c1, r0, r1, lanes_at, lanes_a, group width)."""
    import os
    path = str(tmp_path / "partition.txt")
    os.environ["PDHCG_PARTITION_DUMP"] = path
    try:
        G.setup(prob, **kw).free()
    finally:
        del os.environ["PDHCG_PARTITION_DUMP"]
    return np.loadtxt(path, dtype=np.int64, ndmin=2)


def test_iterate_parity_kind_partition(tmp_path):
    """Many workgroups on the mixed-cone family: each cone kind (SOC, RSOC,
    EXP, POW, R+) gets workgroups of its own (checked on the partition), and
    the iterates still match the oracle (one-sync inner steps across 48
    workgroups)."""
    p = synth.mixed_cone_scaled(seed=6, scale=0.02)
    part = _partition_dump(p, tmp_path, grid_dim=48)
    kind = np.zeros(p.n, dtype=int)
    codes = {"free": 0, "nonneg": 0, "soc": 1, "rsoc": 2, "exp": 3, "pow": 4}
    for c in p.cones:
        kind[c[1]:c[1] + c[2]] = codes[c[0]]
    for w, c0, c1 in part[:, :3]:
        if c1 > c0:
            assert len(set(kind[c0:c1])) == 1, (w, c0, c1)
    trace_parity(p, grid_dim=48, iters=30)


def test_iterate_parity_row_classes(tmp_path):
    """Rows ordered by length (long rows first): each workgroup's rows stay in
    one length class, and the iterates match the oracle."""
    q = synth.mixed_cone_scaled(seed=7, scale=0.02)
    lens = np.diff(q.A.indptr)
    order = np.argsort(-lens, kind="stable")
    p = Problem(n=q.n, m=q.m, A=q.A[order].tocsr(), b=q.b[order], c=q.c, P=q.P, R=q.R, D=q.D,
                cones=q.cones, name="mixed_cone_rows_by_length")
    plens = np.diff(p.A.indptr)
    cls = np.digitize(plens, [16.5, 64.5, 256.5, 1024.5])
    assert len(set(cls)) >= 2
    part = _partition_dump(p, tmp_path, grid_dim=24)
    for w, r0, r1 in part[:, [0, 3, 4]]:
        if r1 > r0:
            assert len(set(cls[r0:r1])) == 1, (w, r0, r1)
    trace_parity(p, grid_dim=24, iters=30)


def test_partition_long_rows_share_workgroups(tmp_path):
    """Large sparse QP family at n = 1e6 (power-law A^T rows, sparse P): a
    workgroup of its own only for a row above half a workgroup's share of the
    coordinate weight (fq (2 + r) + nnz(A^T row) / fq + fq nnz(P row), fq = 3),
    so every other workgroup holds P rows, within 1.4x of the mean.  (The
    same instance's iterates are compared with the oracle in
    test_gpu_parity_full.test_large_sparse_qp_1e6_first_iterations.)"""
    p = synth.large_sparse_qp(seed=2, n=1_000_000, m=500_000)
    part = _partition_dump(p, tmp_path)
    atn = np.diff(p.A.tocsc().indptr).astype(float)
    pn = np.diff(p.P.tocsr().indptr).astype(float)
    G = len(part)
    w = 3.0 * 2.0 + atn / 3.0 + 3.0 * pn
    heavy = max(4096.0, 0.5 * w.sum() / G)
    pw = []
    for _, c0, c1 in part[:, [0, 1, 2]]:
        if c1 - c0 == 1:
            assert max(atn[c0], pn[c0]) > heavy, (c0, atn[c0], heavy)
        pw.append(pn[c0:c1].sum())
    pw = np.array(pw)
    print(f"[partition] G={G} dedicated={(part[:, 2] - part[:, 1] == 1).sum()} "
          f"P nnz per workgroup max/mean {pw.max() / pw.mean():.3f}", flush=True)
    assert pw.max() <= 1.4 * pw.mean()


def test_partition_degree_order(tmp_path):
    """Degree order on the large sparse QP family at n = 1e6: the head of
    long A^T rows gets workgroups of its own, each a single row or a run of
    head rows packed up to the average workgroup's A^T-phase nonzeros (A^T
    row plus P row); the dealt rest gives every other workgroup the same P
    nonzeros within 1.1x of the mean (the caller's order, with its block of
    slack columns, allows 1.4x), and A^T-phase nonzeros within 1.5x (the cut
    balances the weight, in which an A^T nonzero counts 1/3)."""
    p = synth.large_sparse_qp(seed=2, n=1_000_000, m=500_000)
    perm, head = degree_order_rule(p)
    part = _partition_dump(p, tmp_path, interleave="degree")
    atn = np.diff(p.A.tocsc().indptr)[perm].astype(float)
    pn = np.diff(p.P.tocsr().indptr)[perm].astype(float)
    ph = atn + pn
    c0, c1 = part[:, 1], part[:, 2]
    in_head = c1 <= head
    assert head > 0 and in_head.any()
    assert np.all(in_head | (c0 >= head))               # no workgroup mixes head and rest
    ph_w = np.array([ph[a:b].sum() for a, b in zip(c0, c1)])
    pn_w = np.array([pn[a:b].sum() for a, b in zip(c0, c1)])
    rest = ~in_head & (c1 > c0)
    mean_ph = ph_w[rest].mean()
    for a, b, z in zip(c0[in_head], c1[in_head], ph_w[in_head]):
        assert b - a == 1 or z <= 1.05 * mean_ph, (a, b, z, mean_ph)
    print(f"[degree partition] head {head} rows on {in_head.sum()} workgroups; rest: P nnz max/mean "
          f"{pn_w[rest].max() / pn_w[rest].mean():.3f}, A^T-phase max/mean {ph_w[rest].max() / mean_ph:.3f}",
          flush=True)
    assert pn_w[rest].max() <= 1.1 * pn_w[rest].mean()
    assert ph_w[rest].max() <= 1.5 * mean_ph


def test_iterate_parity_degree_order():
    """The degree order renumbers the coordinates of a cone-free problem on
    the device; warm starts, iterates and outputs stay in the caller's
    order and match the oracle."""
    p = synth.large_sparse_qp(seed=1, n=60_000, m=30_000)
    rng = np.random.default_rng(3)
    trace_parity(p, iters=20, interleave="degree", x0=np.abs(rng.standard_normal(p.n)),
                 y0=rng.standard_normal(p.m))


def test_setup_is_deterministic():
    """The host setup runs its row loops on several threads (maxima by
    atomic updates, transposes by column ranges); two setups of the same
    instance in the degree order give bit-identical scalings, step sizes and
    iterates."""
    p = synth.large_sparse_qp(seed=2, n=1_000_000, m=500_000)
    out = []
    for _ in range(2):
        h = G.setup(p, max_iter=16, check_every=4, interleave="degree")
        try:
            out.append((h.scaling(), h.solve()))
        finally:
            h.free()
    (sa, ra), (sb, rb) = out
    for key in ("Sx", "Sy"):
        assert np.array_equal(sa[key], sb[key]), key
    for key in ("nu_b", "nu_c", "eta", "omega0"):
        assert sa[key] == sb[key], key
    for key in ("x", "y"):
        assert np.array_equal(ra[key], rb[key]), key


def test_iterate_parity_degree_order_mixed_types():
    """The degree order forced on a cone-free problem that mixes box, R+ and
    free coordinates with two-sided rows and a low-rank Q: each coordinate
    keeps its type (runs of one type become blocks) and its box bounds, and
    warm starts, iterates and outputs stay in the caller's order."""
    p = synth.bounded_qp(seed=3)
    cones = [(k if k in ("box", "nonneg", "free") else "free", st, d, 0.0) for k, st, d, al in p.cones]
    q = Problem(n=p.n, m=p.m, A=p.A, b=p.b, c=p.c, P=p.P, R=p.R, D=p.D, cones=cones, row_lo=p.row_lo,
                row_hi=p.row_hi, x_lo=p.x_lo, x_hi=p.x_hi, name="bounded_cone_free")
    rng = np.random.default_rng(4)
    trace_parity(q, iters=30, interleave="degree", grid_dim=4, x0=rng.standard_normal(q.n),
                 y0=rng.standard_normal(q.m))


def test_degree_order_keeps_cone_problems_in_caller_order():
    """Problems with cone blocks are left in the caller's order by the
    degree setting (the order is for cone-free problems only)."""
    trace_parity(synth.tiny_mixed(4), iters=20, interleave="degree")


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


def test_iterate_parity_interleaved_order():
    """interleave = 1 renumbers the coordinates on the device (cone blocks
    spread among the R+ coordinates); iterates, traces and warm starts are
    still in the caller's order."""
    p = synth.mixed_cone_scaled(seed=5, scale=0.01)
    trace_parity(p, interleave=1, grid_dim=4)
    rng = np.random.default_rng(1)
    q = synth.tiny_mixed(3)
    trace_parity(q, interleave=1, x0=rng.standard_normal(q.n), y0=rng.standard_normal(q.m))


def test_dual_slack_output_interleaved():
    p = synth.tiny_mixed(0)
    g = G.solve(p, want_s=True, interleave=1)
    Q = p.P.toarray() + p.R.T @ p.D @ p.R
    s = Q @ g["x"] + p.c - p.A.T @ g["y"]
    np.testing.assert_allclose(g["s"], s, rtol=1e-9, atol=1e-12)


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


@pytest.mark.parametrize("seed", [26, 31, 41])
def test_fisher_dual_slack_near_polar(seed):
    """Fisher instances whose solved exponential-cone dual slacks sit within
    rounding of the dual cone's boundary: the KKT projection of -s returns
    ~0 there, and the solve reaches the tolerance (these seeds once ended
    in a numerical failure)."""
    p = synth.fisher(seed=seed)
    g = G.solve(p)
    cnt, rec = G.last_cone_failure()
    assert cnt == 0, rec
    assert g["status"] == "OPTIMAL"
    recheck_kkt(p, g, 1e-6)


def test_full_size_tiny_qp_config_solve():
    p = synth.tiny_qp(0)
    g = G.solve(p)
    recheck_kkt(p, g, 1e-6)
