"""Seeded synthetic instances shaped like the paper's workloads.

The paper measures on public benchmark sets (Maros-Meszaros, Mittelmann
QP/QCQP/SOCP, LIBSVM Lasso) that are not available here; the families below
stand in for them in shape only (sizes, sparsity, cone mix, structure).  All
randomness comes from ``numpy.random.default_rng(seed)``.

Families
--------
tiny_qp          n=200, m=100 sparse QP over the nonnegative orthant.
mixed_cone       SOC/RSOC/EXP/POW/R+ mix with Q = diag + low-rank factor
                 (QCQP/SOCP-like; full size n=1e5, m=5e4).
large_sparse_qp  n=1e7, m=5e6 sparse QP with power-law column degrees and
                 inequality rows encoded by R+ slack columns.
portfolio        factor-model portfolio QPs with budget and sector caps
                 (batched family, one seed per instance).
fisher           quasilinear Fisher market in exponential-cone form
                 (Section "Large-Scale Fisher Equilibrium", eq. fisher-conic).
tiny_free_qp / tiny_nonneg_qp / tiny_mixed
                 small families for whole-solve pins.
bounded_qp       the implementation form: two-sided, one-sided, equality
                 and free rows, box coordinates with finite and one-sided
                 bounds, with R+, free, SOC and EXP blocks.
"""
from __future__ import annotations

import math

import numpy as np
import scipy.sparse as sp

from .problem import Problem


# ----------------------------------------------------------------------------
# helpers (data drawing only)
# ----------------------------------------------------------------------------
def _random_rows(rng, m, n, row_nnz, col_sampler=None):
    """CSR pattern with the requested nnz per row (duplicates dropped)."""
    row_nnz = np.asarray(row_nnz, dtype=np.int64)
    rows = np.repeat(np.arange(m, dtype=np.int64), row_nnz)
    if col_sampler is None:
        cols = rng.integers(0, n, size=rows.size, dtype=np.int64)
    else:
        cols = col_sampler(rows.size)
    key = np.unique(rows * n + cols)
    rows = key // n
    cols = key % n
    return rows, cols


def _interior_point(rng, n, cones):
    """A point strictly inside K (recipe of the mixed-cone family)."""
    x = np.abs(rng.standard_normal(n)) + 0.1
    for kind, st, d, al in cones:
        if kind == "free":
            x[st:st + d] = rng.standard_normal(d)
        elif kind == "nonneg":
            x[st:st + d] = np.abs(rng.standard_normal(d)) + 0.1
        elif kind == "soc":
            v = rng.standard_normal(d - 1)
            x[st:st + d - 1] = v
            x[st + d - 1] = np.linalg.norm(v) + abs(rng.standard_normal()) + 0.1
        elif kind == "rsoc":
            v = rng.standard_normal(d - 2)
            x[st:st + d - 2] = v
            h = np.linalg.norm(v) / math.sqrt(2.0) + abs(rng.standard_normal()) + 0.1
            x[st + d - 2] = h
            x[st + d - 1] = h
        elif kind == "exp":
            s = abs(rng.standard_normal()) + 0.1
            r = s * rng.standard_normal()
            t = s * math.exp(r / s) + abs(rng.standard_normal()) + 0.1
            x[st:st + 3] = (r, s, t)
        elif kind == "pow":
            a = rng.uniform(0.5, 2.0)
            b = rng.uniform(0.5, 2.0)
            z = 0.9 * rng.uniform(-1.0, 1.0) * a ** al * b ** (1.0 - al)
            x[st:st + 3] = (a, b, z)
    return x


# ----------------------------------------------------------------------------
# tiny QP over R+  (n=200, m=100)
# ----------------------------------------------------------------------------
def tiny_qp(seed=0, n=200, m=100, a_density=0.05, b_density=0.02):
    """A: m x n at 5% density N(0,1) (resampled until every row is nonempty
    and A has full row rank); Q = B^T B + 1e-2 I with B n x n at 2% density;
    x0 = |N(0,1)|, b = A x0, c ~ N(0,1), K = R+^n."""
    rng = np.random.default_rng(seed)
    while True:
        A = sp.random(m, n, density=a_density, random_state=rng,
                      data_rvs=rng.standard_normal, format="csr")
        if np.all(np.diff(A.indptr) > 0) and np.linalg.matrix_rank(A.toarray()) == m:
            break
    B = sp.random(n, n, density=b_density, random_state=rng,
                  data_rvs=rng.standard_normal, format="csr")
    P = (B.T @ B + 1e-2 * sp.identity(n)).tocsr()
    x0 = np.abs(rng.standard_normal(n))
    b = A @ x0
    c = rng.standard_normal(n)
    return Problem(n=n, m=m, A=A, b=b, c=c, P=P,
                   cones=[("nonneg", 0, n, 0.0)], name=f"tiny_qp[{seed}]",
                   meta={"x_feas": x0})


# ----------------------------------------------------------------------------
# mixed-cone SOCP/QCQP-like family
# ----------------------------------------------------------------------------
def mixed_cone(seed=0, n=100_000, m=50_000, n_soc=2000, soc_dim=20,
               n_rsoc=1000, rsoc_dim=10, n_exp=500, n_pow=500, rank=10,
               row_nnz_mean=20.0, shuffle_blocks=False):
    """Rows: nnz ~ max(1, Poisson(20)), columns uniform, values N(0,1).
    Q = diag(U(0.1,1)) + F F^T with F n x rank, entries N(0, 1/n)
    (std 1/sqrt(n)); passed as P = diag, R = F^T, D = I.
    Cones (contiguous by type): SOC(soc_dim) x n_soc, RSOC(rsoc_dim) x n_rsoc,
    EXP x n_exp, POW x n_pow (alpha ~ U(0.2,0.8)), R+ for the rest.
    b = A x0 for a strictly interior x0; c ~ N(0,1)."""
    rng = np.random.default_rng(seed)
    used = n_soc * soc_dim + n_rsoc * rsoc_dim + 3 * (n_exp + n_pow)
    if used > n:
        raise ValueError("cone blocks exceed n")
    blocks = ([("soc", soc_dim)] * n_soc + [("rsoc", rsoc_dim)] * n_rsoc +
              [("exp", 3)] * n_exp + [("pow", 3)] * n_pow)
    if shuffle_blocks:
        order = rng.permutation(len(blocks))
        blocks = [blocks[i] for i in order]
    cones = []
    st = 0
    for kind, d in blocks:
        al = float(rng.uniform(0.2, 0.8)) if kind == "pow" else 0.0
        cones.append((kind, st, d, al))
        st += d
    if st < n:
        cones.append(("nonneg", st, n - st, 0.0))
    k = np.maximum(1, rng.poisson(row_nnz_mean, size=m))
    k = np.minimum(k, n)
    rows, cols = _random_rows(rng, m, n, k)
    vals = rng.standard_normal(rows.size)
    A = sp.csr_matrix((vals, (rows, cols)), shape=(m, n))
    qd = rng.uniform(0.1, 1.0, size=n)
    F = rng.standard_normal((n, rank)) / math.sqrt(n)
    x0 = _interior_point(rng, n, cones)
    b = A @ x0
    c = rng.standard_normal(n)
    return Problem(n=n, m=m, A=A, b=b, c=c, P=sp.diags(qd).tocsr(),
                   R=np.ascontiguousarray(F.T), D=np.eye(rank), cones=cones,
                   name=f"mixed_cone[n={n},m={m},seed={seed}]",
                   meta={"x_feas": x0})


def mixed_cone_scaled(seed=0, scale=0.02, **kw):
    """The mixed-cone family with every count multiplied by ``scale``
    (at least one block of each cone type)."""
    n = max(200, int(round(100_000 * scale)))
    m = max(50, int(round(50_000 * scale)))
    args = dict(n=n, m=m,
                n_soc=max(1, int(round(2000 * scale))),
                n_rsoc=max(1, int(round(1000 * scale))),
                n_exp=max(1, int(round(500 * scale))),
                n_pow=max(1, int(round(500 * scale))))
    args.update(kw)
    return mixed_cone(seed=seed, **args)


# ----------------------------------------------------------------------------
# large sparse QP with power-law column degrees
# ----------------------------------------------------------------------------
def large_sparse_qp(seed=0, n=10_000_000, m=5_000_000, slack_frac=0.1,
                    row_nnz_extra=9.0, q_pairs=None, power=0.8):
    """n R+ columns, m rows.  Structural rows have 1 + Poisson(9) entries with
    columns drawn from p_j ~ (j+1)^-0.8 over a random permutation of the
    structural columns; values N(0,1).  A fraction ``slack_frac`` of the
    columns are slack columns with a single +1 in distinct rows (those rows
    are inequalities a^T x <= b).  Q has ``q_pairs`` symmetric off-diagonal
    pairs with values 0.1 N(0,1) plus a diagonal sum_j |Q_ij| + U(0.01,0.1)
    (strictly diagonally dominant).  x0 = |N(0,1)|, b = A x0, c ~ N(0,1)."""
    rng = np.random.default_rng(seed)
    n_slack = min(int(round(slack_frac * n)), m)
    n_struct = n - n_slack
    if q_pairs is None:
        q_pairs = n
    perm = rng.permutation(n_struct)
    top = (n_struct + 1.0) ** (1.0 - power) - 1.0

    def sampler(size):
        u = rng.random(size)
        j = np.floor((u * top + 1.0) ** (1.0 / (1.0 - power)) - 1.0).astype(np.int64)
        np.clip(j, 0, n_struct - 1, out=j)
        return perm[j]

    k = 1 + rng.poisson(row_nnz_extra, size=m)
    rows, cols = _random_rows(rng, m, n_struct, k, col_sampler=sampler)
    vals = rng.standard_normal(rows.size)
    srow = rng.choice(m, size=n_slack, replace=False)
    rows = np.concatenate([rows, srow])
    cols = np.concatenate([cols, n_struct + np.arange(n_slack)])
    vals = np.concatenate([vals, np.ones(n_slack)])
    A = sp.csr_matrix((vals, (rows, cols)), shape=(m, n))
    # Q: symmetric off-diagonal pairs + dominant diagonal
    qi = rng.integers(0, n, size=q_pairs)
    qj = rng.integers(0, n, size=q_pairs)
    keep = qi != qj
    qi, qj = qi[keep], qj[keep]
    qv = 0.1 * rng.standard_normal(qi.size)
    off = sp.coo_matrix((np.concatenate([qv, qv]),
                         (np.concatenate([qi, qj]), np.concatenate([qj, qi]))),
                        shape=(n, n)).tocsr()
    off.sum_duplicates()
    diag = np.asarray(abs(off).sum(axis=1)).ravel() + rng.uniform(0.01, 0.1, size=n)
    P = (off + sp.diags(diag)).tocsr()
    P.sort_indices()
    x0 = np.abs(rng.standard_normal(n))
    b = A @ x0
    c = rng.standard_normal(n)
    return Problem(n=n, m=m, A=A, b=b, c=c, P=P, cones=[("nonneg", 0, n, 0.0)],
                   name=f"large_sparse_qp[n={n},m={m},seed={seed}]",
                   meta={"x_feas": x0, "n_slack": n_slack})


# ----------------------------------------------------------------------------
# batched portfolio QPs
# ----------------------------------------------------------------------------
def portfolio(seed, n_assets=None, n_factors=None, n_sectors=10, cap=0.3):
    """One factor-model portfolio QP.  n ~ U{50..2000}, k ~ U{5..20},
    F ~ N(0, 0.1^2) (n x k), D ~ U(0.01, 0.1); Q = F F^T + diag(D) passed as
    P = diag(D), R = F^T, D = I.  c = -mu, mu ~ N(0.05, 0.02^2).  Rows: the
    budget sum(x) = 1 and, per sector S_k, sum_{i in S_k} x_i + s_k = cap.
    Variables x in R+^n and sector slacks s in R+^10."""
    rng = np.random.default_rng(seed)
    na = int(rng.integers(50, 2001)) if n_assets is None else int(n_assets)
    k = int(rng.integers(5, 21)) if n_factors is None else int(n_factors)
    F = 0.1 * rng.standard_normal((na, k))
    Dg = rng.uniform(0.01, 0.1, size=na)
    mu = rng.normal(0.05, 0.02, size=na)
    sector = rng.integers(0, n_sectors, size=na)
    n = na + n_sectors
    m = 1 + n_sectors
    rows = [np.zeros(na, dtype=np.int64), 1 + sector, 1 + np.arange(n_sectors)]
    cols = [np.arange(na), np.arange(na), na + np.arange(n_sectors)]
    A = sp.csr_matrix((np.ones(2 * na + n_sectors),
                       (np.concatenate(rows), np.concatenate(cols))), shape=(m, n))
    b = np.concatenate([[1.0], np.full(n_sectors, cap)])
    c = np.concatenate([-mu, np.zeros(n_sectors)])
    P = sp.diags(np.concatenate([Dg, np.zeros(n_sectors)])).tocsr()
    R = np.zeros((k, n))
    R[:, :na] = F.T
    return Problem(n=n, m=m, A=A, b=b, c=c, P=P, R=R, D=np.eye(k),
                   cones=[("nonneg", 0, n, 0.0)], name=f"portfolio[{seed}]",
                   meta={"n_assets": na, "n_factors": k})


def portfolio_batch(count=4096, base_seed=1_000_000, **kw):
    return [portfolio(base_seed + i, **kw) for i in range(count)]


# ----------------------------------------------------------------------------
# quasilinear Fisher market, exponential-cone form (eq. fisher-conic)
# ----------------------------------------------------------------------------
def fisher_graph(n_buyers=1000, n_goods=500, density=0.1, seed=0):
    """Valuation graph: each (buyer, good) pair is an edge with probability
    ``density``; every buyer and every good gets at least one edge.  Above
    1e8 pairs the edges are drawn in O(edges) memory: the gaps between
    successive edges in row-major pair order are geometric(density), which
    gives the same distribution as independent draws per pair."""
    rng = np.random.default_rng(seed)
    if n_buyers * n_goods <= 100_000_000:
        mask = rng.random((n_buyers, n_goods)) < density
        for i in np.where(~mask.any(axis=1))[0]:
            mask[i, rng.integers(n_goods)] = True
        for j in np.where(~mask.any(axis=0))[0]:
            mask[rng.integers(n_buyers), j] = True
        bi, gj = np.nonzero(mask)
        return bi.astype(np.int64), gj.astype(np.int64)
    total = n_buyers * n_goods
    chunks, pos = [], -1
    while pos < total:
        gaps = rng.geometric(density, size=max(1_000_000, int(1.05 * density * (total - pos))))
        cand = pos + np.cumsum(gaps)
        pos = int(cand[-1])
        chunks.append(cand[cand < total])
    cells = np.concatenate(chunks)
    bi, gj = cells // n_goods, cells % n_goods
    extra = []
    miss_b = np.setdiff1d(np.arange(n_buyers), bi)
    extra += [ib * n_goods + rng.integers(n_goods) for ib in miss_b]
    miss_g = np.setdiff1d(np.arange(n_goods), gj)
    extra += [rng.integers(n_buyers) * n_goods + jg for jg in miss_g]
    if extra:
        cells = np.unique(np.concatenate([cells, np.asarray(extra, dtype=np.int64)]))
        bi, gj = cells // n_goods, cells % n_goods
    return bi.astype(np.int64), gj.astype(np.int64)


# the paper's Fisher instance shapes: buyers -> (goods, density)
FISHER_PAPER_SHAPES = {1_000: (400, 0.20), 10_000: (4_000, 0.02), 100_000: (4_000, 0.02),
                       1_000_000: (4_000, 0.02), 10_000_000: (4_000, 0.01)}


def fisher_paper(n_buyers=1_000, seed=1, middle="fixed"):
    """A Fisher market of the paper's experiment: goods and valuation
    density by the buyer count (FISHER_PAPER_SHAPES), valuations and
    budgets U[0.1, 1.1], supplies 0.2 n, seed 1 (graph and values drawn with
    numpy's generator, so the instance matches the paper's in shape only)."""
    goods, rho = FISHER_PAPER_SHAPES[n_buyers]
    return fisher(seed=seed, n_buyers=n_buyers, n_goods=goods, density=rho, graph_seed=seed,
                  dist="paper", middle=middle)


def fisher(seed=1, n_buyers=1000, n_goods=500, density=0.1, graph_seed=0,
           dist="lognormal", graph=None, middle="row", spread=None, base_seed=0):
    """Fisher market in the exponential-cone form of eq. fisher-conic with the
    middle exponential-cone coordinate held at one by an explicit row.

    Variables (in order): allocations x_e on the edges (R+), retained money
    delta_i (R+), and per buyer an exponential-cone block (z_i, s_i, t_i).
    Rows: supply sum_i x_ij = b_j; t_i - sum_j u_ij x_ij - delta_i = 0;
    s_i = 1.  Objective sum_i (delta_i - w_i z_i); Q = 0.

    dist="lognormal": u_ij ~ lognormal(0,1), w_i ~ lognormal(0,0.5), b_j = 1.
    dist="paper":     u_ij, w_i ~ U[0.1, 1.1], b_j = 0.2 n (the paper's
                      Fisher experiment recipe).
    spread (lognormal only): the instance is a perturbation of the base
                      market drawn from `base_seed`, u = u0 exp(spread g),
                      w = w0 exp(spread g') with g, g' ~ N(0,1) from `seed`
                      (a family whose solution moves smoothly with its
                      parameters).
    middle="row":     (z_i, s_i, t_i) in an exponential-cone block and a row
                      s_i = 1 (m + 2n rows);
    middle="fixed":   the block (z_i, 1, t_i) with its middle coordinate fixed
                      at one by the set itself (kind "exp1"), as the paper
                      stores it (m + n rows)."""
    if graph is None:
        graph = fisher_graph(n_buyers, n_goods, density, graph_seed)
    bi, gj = graph
    e = bi.size
    rng = np.random.default_rng(seed)
    if dist == "lognormal" and spread is not None:
        base = np.random.default_rng(base_seed)
        u = base.lognormal(0.0, 1.0, size=e) * np.exp(spread * rng.standard_normal(e))
        w = base.lognormal(0.0, 0.5, size=n_buyers) * np.exp(spread * rng.standard_normal(n_buyers))
        supply = np.ones(n_goods)
    elif dist == "lognormal":
        u = rng.lognormal(0.0, 1.0, size=e)
        w = rng.lognormal(0.0, 0.5, size=n_buyers)
        supply = np.ones(n_goods)
    elif dist == "paper":
        u = rng.uniform(0.1, 1.1, size=e)
        w = rng.uniform(0.1, 1.1, size=n_buyers)
        supply = np.full(n_goods, 0.2 * n_buyers)
    else:
        raise ValueError(dist)
    nb = n_buyers
    fixed = middle == "fixed"
    n = e + 4 * nb
    m = n_goods + (1 if fixed else 2) * nb
    off_d = e
    off_c = e + nb
    zi = off_c + 3 * np.arange(nb)
    rows = [gj,                                    # supply rows
            n_goods + bi,                          # t-definition rows (-u x)
            n_goods + np.arange(nb),               # (-delta)
            n_goods + np.arange(nb)]               # (+t)
    cols = [np.arange(e), np.arange(e), off_d + np.arange(nb), zi + 2]
    vals = [np.ones(e), -u, -np.ones(nb), np.ones(nb)]
    if not fixed:
        rows.append(n_goods + nb + np.arange(nb))  # s_i = 1
        cols.append(zi + 1)
        vals.append(np.ones(nb))
    A = sp.csr_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(m, n))
    b = np.concatenate([supply, np.zeros(nb)] + ([] if fixed else [np.ones(nb)]))
    c = np.zeros(n)
    c[off_d:off_d + nb] = 1.0
    c[zi] = -w
    kind = "exp1" if fixed else "exp"
    cones = [("nonneg", 0, e + nb, 0.0)] + [(kind, int(z), 3, 0.0) for z in zi]
    return Problem(n=n, m=m, A=A, b=b, c=c, cones=cones,
                   name=f"fisher[{n_buyers}x{n_goods},seed={seed}{',fixed' if fixed else ''}]",
                   meta={"u": u, "w": w, "graph": graph, "n_buyers": nb,
                         "n_goods": n_goods, "edges": e})


# ----------------------------------------------------------------------------
# tiny families for whole-solve pins
# ----------------------------------------------------------------------------
def tiny_free_qp(seed=0, n=8, m=3):
    """Equality-constrained strongly convex QP over free variables."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n))
    B = rng.standard_normal((n, n))
    P = B.T @ B / n + 0.5 * np.eye(n)
    b = rng.standard_normal(m)
    c = rng.standard_normal(n)
    return Problem(n=n, m=m, A=sp.csr_matrix(A), b=b, c=c, P=sp.csr_matrix(P),
                   cones=[("free", 0, n, 0.0)], name=f"tiny_free_qp[{seed}]")


def tiny_nonneg_qp(seed=0, n=8, m=3, diag_only=False):
    """Small QP over R+ with a feasible interior point."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n))
    if diag_only:
        P = np.diag(rng.uniform(0.1, 2.0, size=n))
    else:
        B = rng.standard_normal((n, n))
        P = B.T @ B / n + 0.1 * np.eye(n)
    x0 = rng.uniform(0.2, 1.5, size=n)
    b = A @ x0
    c = rng.standard_normal(n)
    return Problem(n=n, m=m, A=sp.csr_matrix(A), b=b, c=c, P=sp.csr_matrix(P),
                   cones=[("nonneg", 0, n, 0.0)], name=f"tiny_nonneg_qp[{seed}]",
                   meta={"x_feas": x0})


def tiny_mixed(seed=0, m=12, with_q=True, lowrank=True):
    """One block of every cone type plus a few R+ and free coordinates."""
    rng = np.random.default_rng(seed)
    spec = [("soc", 5), ("rsoc", 4), ("exp", 3), ("pow", 3), ("nonneg", 4), ("free", 2)]
    cones = []
    st = 0
    for kind, d in spec:
        al = float(rng.uniform(0.2, 0.8)) if kind == "pow" else 0.0
        cones.append((kind, st, d, al))
        st += d
    n = st
    A = sp.random(m, n, density=0.5, random_state=rng, data_rvs=rng.standard_normal,
                  format="csr")
    A = A + sp.csr_matrix((np.ones(m), (np.arange(m), np.arange(m) % n)), shape=(m, n))
    x0 = _interior_point(rng, n, cones)
    b = A @ x0
    c = rng.standard_normal(n)
    P = R = D = None
    if with_q:
        P = sp.diags(rng.uniform(0.1, 1.0, size=n)).tocsr()
        if lowrank:
            R = rng.standard_normal((2, n)) / math.sqrt(n)
            D = np.eye(2)
    return Problem(n=n, m=m, A=A, b=b, c=c, P=P, R=R, D=D, cones=cones,
                   name=f"tiny_mixed[{seed}]", meta={"x_feas": x0})


# ----------------------------------------------------------------------------
# implementation form: row bounds and box blocks
# ----------------------------------------------------------------------------
def bounded_qp(seed=0, n_box=40, n_cone_soc=2, n_exp=1, m=30, density=0.2, q="lowrank"):
    """Rows l <= A x <= u of five kinds around a strictly interior point
    (range, equality, lower only, upper only, free, in a seeded mix); box
    coordinates with finite, lower-only and upper-only bounds; a nonnegative
    block, a free block, SOC(5) blocks and EXP blocks.  q: None (Q = 0),
    "diag" or "lowrank" (diag + rank-2 factor).  Costs on the coordinates
    that are unbounded in one direction point towards the bound."""
    rng = np.random.default_rng(seed)
    cones = []
    st = 0
    cones.append(("box", st, n_box, 0.0)); st += n_box
    cones.append(("nonneg", st, 6, 0.0)); st += 6
    cones.append(("free", st, 3, 0.0)); st += 3
    for _ in range(n_cone_soc):
        cones.append(("soc", st, 5, 0.0)); st += 5
    for _ in range(n_exp):
        cones.append(("exp", st, 3, 0.0)); st += 3
    n = st
    A = sp.random(m, n, density=density, random_state=rng, data_rvs=rng.standard_normal, format="csr")
    # every free coordinate appears in an equality or two-sided row
    A = (A + sp.csr_matrix((np.ones(3), ([0, 1, 2], [n_box + 6, n_box + 7, n_box + 8])), shape=(m, n))).tocsr()
    x0 = _interior_point(rng, n, cones)
    x0[:n_box] = rng.uniform(0.2, 0.8, n_box)
    ax = A @ x0
    kinds = rng.choice(["range", "eq", "lo", "hi", "free"], size=m, p=[0.4, 0.2, 0.15, 0.15, 0.1])
    kinds[:3] = ["eq", "range", "eq"]
    lo = np.empty(m)
    hi = np.empty(m)
    for j, k in enumerate(kinds):
        a, b = rng.uniform(0.05, 1.0, 2)
        lo[j], hi[j] = {"range": (ax[j] - a, ax[j] + b), "eq": (ax[j], ax[j]), "lo": (ax[j] - a, np.inf),
                        "hi": (-np.inf, ax[j] + b), "free": (-np.inf, np.inf)}[k]
    xlo = np.full(n, -np.inf)
    xhi = np.full(n, np.inf)
    third = n_box // 3
    xlo[:n_box] = x0[:n_box] - rng.uniform(0.1, 0.6, n_box)
    xhi[:third] = x0[:third] + rng.uniform(0.1, 0.6, third)            # finite box
    # [third, 2 third): lower only; [2 third, n_box): upper only
    xhi[2 * third:n_box] = x0[2 * third:n_box] + rng.uniform(0.1, 0.6, n_box - 2 * third)
    xlo[2 * third:n_box] = -np.inf
    c = rng.standard_normal(n)
    c[third:2 * third] = np.abs(c[third:2 * third]) + 0.1
    c[2 * third:n_box] = -np.abs(c[2 * third:n_box]) - 0.1
    c[n_box:n_box + 6] = np.abs(c[n_box:n_box + 6]) + 0.1
    P = R = D = None
    if q in ("diag", "lowrank"):
        P = sp.diags(rng.uniform(0.1, 1.0, size=n)).tocsr()
    if q == "lowrank":
        R = rng.standard_normal((2, n)) / math.sqrt(n)
        D = np.eye(2)
    b = np.where(lo == hi, lo, 0.0)
    return Problem(n=n, m=m, A=A, b=b, c=c, P=P, R=R, D=D, cones=cones, row_lo=lo, row_hi=hi,
                   x_lo=xlo, x_hi=xhi, name=f"bounded_qp[{seed},n={n},m={m},q={q}]",
                   meta={"x_feas": x0, "row_kinds": kinds})
