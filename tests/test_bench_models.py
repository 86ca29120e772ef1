"""The byte models behind the bench line's roofline figures (CPU only).

Each count is rebuilt here by hand from its definition for small shapes
where every term can be listed: the solver kernel's algorithmic bytes per
outer iteration (per-pass reads and writes), the training step's HBM bytes
and the working-set footprint."""
import numpy as np
import scipy.sparse as sp

import bench
from instances import Problem


def _lp(n=10, m=4, nnz_per_row=3, seed=0):
    rng = np.random.default_rng(seed)
    rows = np.repeat(np.arange(m), nnz_per_row)
    cols = np.concatenate([rng.choice(n, nnz_per_row, replace=False) for _ in range(m)])
    A = sp.csr_matrix((rng.standard_normal(rows.size), (rows, cols)), shape=(m, n))
    return Problem(n=n, m=m, A=A, b=np.ones(m), c=np.ones(n), cones=[("nonneg", 0, n, 0.0)], name="lp")


def test_bytes_model_diagonal_q_by_hand():
    """Q = 0, R+ only: one A^T product, the elementwise prox, one A product
    with the dual and Halpern updates per outer iteration, and a check."""
    p = _lp()
    n, m, z = p.n, p.m, p.A.nnz
    at = 12 * z + 8 * (n + 1) + 8 * m        # values + int32 columns, row pointers, gathered y
    a = 12 * z + 8 * (m + 1) + 8 * n         # same for A with gathered w_x
    per_iter = at + 33 * n + (a + 72 * m + 32 * n)
    check = at + 73 * n + 40 * m
    assert bench.bytes_model(p, 5, 0, 2) == 5 * per_iter + 2 * check


def test_bytes_model_inner_steps_scale_with_p_and_factor():
    """General Q = P + R^T R: every inner step after the first reads P and
    the factor twice (R u and R^T h) on top of its vector traffic."""
    p = _lp(seed=1)
    n, m = p.n, p.m
    P = sp.csr_matrix(np.eye(n) + np.diag(np.ones(n - 1), 1) + np.diag(np.ones(n - 1), -1))
    r = 3
    q = Problem(n=n, m=m, A=p.A, b=p.b, c=p.c, P=P, R=np.ones((r, n)), D=np.eye(r), cones=p.cones, name="qp")
    base = bench.bytes_model(q, 4, 4, 0)                       # no step beyond the first
    more = bench.bytes_model(q, 4, 10, 0)                      # six further steps
    step = 12 * P.nnz + 8 * (n + 1) + 8 * n + 16 * r * n + 121 * n
    assert more - base == 6 * step


def test_mlp_step_bytes_counts_adam_and_layers():
    dims, B = [6, 4, 5], 2
    by = bench.mlp_step_bytes(dims, B)
    params = 6 * 4 + 4 + 4 * 5 + 5
    fwd = (2 * B * 6 + 2 * 6 * 4 + 2 * B * 4) + (2 * B * 4 + 2 * 4 * 5 + 4 * B * 5)
    loss = 4 * B * 5 * 2 + 2 * B * 5
    bwd_last = (2 * B * 4 + 2 * B * 5 + 4 * 4 * 5) + (2 * B * 5 + 4 * 5) \
        + (2 * B * 5 + 2 * 4 * 5 + 2 * B * 4 + 2 * B * 4)
    bwd_first = (2 * B * 6 + 2 * B * 4 + 4 * 6 * 4) + (2 * B * 4 + 4 * 4)
    inp = 4 * B * 6 + 2 * B * 6
    assert by == inp + fwd + loss + bwd_last + bwd_first + 30 * params
    # the full warm-start network: the Adam state dominates
    full = bench.mlp_step_bytes([51000, 512, 512, 56500], 256)
    assert 2.4e9 < full < 2.6e9


def test_footprint_bytes():
    p = _lp()
    fb = bench.footprint_bytes(p)
    assert fb == 24 * p.A.nnz + 8 * (p.m + 1) + 8 * (p.n + 1) + 8 * (17 * p.n + 8 * p.m)


def test_method_bytes_model_by_hand():
    """The method's bytes: 24 nnz(A) + 60n + 116m per outer iteration, 32n
    for a diagonal prox or 12 nnz(P) + 16rn + 92n per inner step, and per
    check one A^T product (12 nnz(A) + 20n + 8m) and one Q product
    (12 nnz(P) + 16rn + 16n)."""
    p = _lp()
    n, m, z = p.n, p.m, p.A.nnz
    assert bench.method_bytes_model(p, 7, 0, 3) == 7 * (24 * z + 60 * n + 116 * m + 32 * n) \
        + 3 * (12 * z + 20 * n + 8 * m + 16 * n)
    P = sp.csr_matrix(np.eye(n) + np.diag(np.ones(n - 1), 1) + np.diag(np.ones(n - 1), -1))
    r = 2
    q = Problem(n=n, m=m, A=p.A, b=p.b, c=p.c, P=P, R=np.ones((r, n)), D=np.eye(r), cones=p.cones, name="qp")
    assert bench.method_bytes_model(q, 4, 11, 2) == 4 * (24 * z + 60 * n + 116 * m) \
        + 11 * (12 * P.nnz + 16 * r * n + 92 * n) + 2 * (12 * z + 20 * n + 8 * m + 12 * P.nnz + 16 * r * n + 16 * n)
