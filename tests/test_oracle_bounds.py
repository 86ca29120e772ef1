"""Pins of the oracle's implementation form (eq. solver-input): two-sided row
bounds l <= A x <= u and box blocks.  None of the expected values comes
from the oracle: the dual step is checked against the definition of the
proximal step by a one-dimensional search per row, bounded LPs against
scipy's HiGHS (linprog) and a boxed QP against active-set enumeration, and
the KKT residual definitions at HiGHS's own primal-dual solution."""
import itertools
import math

import numpy as np
import pytest
import scipy.sparse as sp
from scipy.optimize import linprog

from instances import Problem
from oracle import pdhg

INF = math.inf


def bounded_instance(seed, n=12, m=7, with_q=False, rng_scale=1.0):
    """Rows of every kind (range, equality, lower only, upper only, free)
    around a feasible point; coordinates in box blocks with finite, lower-
    only and upper-only bounds, a nonnegative block and a free block."""
    rng = np.random.default_rng(seed)
    A = rng.standard_normal((m, n))
    A[rng.random((m, n)) < 0.3] = 0.0
    xf = rng.uniform(0.2, 0.8, n)
    ax = A @ xf
    kinds = ["range", "eq", "lo", "hi", "free"] + ["range"] * (m - 5)
    lo = np.empty(m)
    hi = np.empty(m)
    for j, k in enumerate(kinds):
        a, b = rng.uniform(0.05, 1.0, 2) * rng_scale
        lo[j], hi[j] = {"range": (ax[j] - a, ax[j] + b), "eq": (ax[j], ax[j]),
                        "lo": (ax[j] - a, INF), "hi": (-INF, ax[j] + b), "free": (-INF, INF)}[k]
    xlo = np.full(n, -INF)
    xhi = np.full(n, INF)
    # coordinates 0-5 box [finite, finite], 6-7 box [l, inf), 8 box (-inf, u],
    # 9-10 nonneg, 11 free
    xlo[:6], xhi[:6] = xf[:6] - rng.uniform(0.1, 0.5, 6), xf[:6] + rng.uniform(0.1, 0.5, 6)
    xlo[6:8] = xf[6:8] - 0.3
    xhi[8] = xf[8] + 0.3
    cones = [("box", 0, 9, 0.0), ("nonneg", 9, 2, 0.0), ("free", 11, 1, 0.0)]
    c = rng.standard_normal(n)
    # bounded below on the unbounded directions: costs that push towards the
    # finite ends, and the free coordinate tied by the rows
    c[6:8] = np.abs(c[6:8]) + 0.1
    c[8] = -abs(c[8]) - 0.1
    c[9:11] = np.abs(c[9:11]) + 0.1
    A[0, 11] = A[1, 11] = 1.0
    P = None
    if with_q:
        B = rng.standard_normal((n, n)) / math.sqrt(n)
        P = sp.csr_matrix(B.T @ B + 0.05 * np.eye(n))
    return Problem(n=n, m=m, A=sp.csr_matrix(A), b=np.zeros(m), c=c, P=P, cones=cones,
                   row_lo=lo, row_hi=hi, x_lo=xlo, x_hi=xhi, name=f"bounded[{seed}]",
                   meta={"x_feas": xf})


def _phi(t, axb, lo, hi, y, sigma):
    """The dual proximal objective of one row: t (A xbar) + sup_{b in [lo, hi]}
    (-t b) + (t - y)^2 / (2 sigma)."""
    if t > 0:
        sup = -t * lo if math.isfinite(lo) else INF
    elif t < 0:
        sup = -t * hi if math.isfinite(hi) else INF
    else:
        sup = 0.0
    return t * axb + sup + (t - y) ** 2 / (2 * sigma)


def _golden_min(f, a, b, iters=200):
    g = (math.sqrt(5) - 1) / 2
    c, d = b - g * (b - a), a + g * (b - a)
    fc, fd = f(c), f(d)
    for _ in range(iters):
        if fc <= fd:
            b, d, fd = d, c, fc
            c = b - g * (b - a)
            fc = f(c)
        else:
            a, c, fc = c, d, fd
            d = a + g * (b - a)
            fd = f(d)
    return 0.5 * (a + b)


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_dual_step_is_the_proximal_step(seed):
    """w_y minimises, row by row, the dual proximal objective of the saddle
    function with A x in [l, u] (a convex function of one variable, located
    here by golden-section search on a wide bracket)."""
    p = bounded_instance(seed)
    S = pdhg.setup(p)
    rng = np.random.default_rng(10 + seed)
    x = S.proj.project(rng.standard_normal(p.n))
    y = 3.0 * rng.standard_normal(p.m)
    tau, sigma = S.eta / 0.8, S.eta * 0.8
    wx, wy, _ = pdhg.pdhg_step(S, x, y, tau, sigma, 1e-12)
    axb = S.sc.A @ (2 * wx - x)
    for j in range(p.m):
        if not (math.isfinite(S.sc.lo[j]) or math.isfinite(S.sc.hi[j])):
            assert wy[j] == 0.0       # a free row: sup_b (-t b) is infinite for every t != 0
            continue
        f = lambda t: _phi(t, axb[j], S.sc.lo[j], S.sc.hi[j], y[j], sigma)
        span = 10.0 * (1.0 + abs(y[j]) + sigma * abs(axb[j]))
        t = _golden_min(f, -span, span)
        assert wy[j] == pytest.approx(t, abs=1e-7 * (1 + abs(t))), (j, wy[j], t)
        assert f(wy[j]) <= f(t) + 1e-12 * (1 + abs(f(t)))


def _highs(p):
    """The LP with scipy's HiGHS: rows split into A_ub / A_eq."""
    A = p.A.toarray()
    lo, hi = p.row_lo, p.row_hi
    eq = lo == hi
    ub_rows, ub_rhs = [], []
    for j in range(p.m):
        if eq[j]:
            continue
        if math.isfinite(hi[j]):
            ub_rows.append(A[j]); ub_rhs.append(hi[j])
        if math.isfinite(lo[j]):
            ub_rows.append(-A[j]); ub_rhs.append(-lo[j])
    bounds = []
    for i in range(p.n):
        kind = [k for k, st, d, al in p.cones if st <= i < st + d][0]
        if kind == "box":
            bounds.append((None if not math.isfinite(p.x_lo[i]) else p.x_lo[i],
                           None if not math.isfinite(p.x_hi[i]) else p.x_hi[i]))
        elif kind == "nonneg":
            bounds.append((0, None))
        else:
            bounds.append((None, None))
    r = linprog(p.c, A_ub=np.array(ub_rows), b_ub=np.array(ub_rhs), A_eq=A[eq], b_eq=lo[eq],
                bounds=bounds, method="highs")
    assert r.status == 0, r.message
    # y in the convention of the saddle function (y >= 0 on an active lower
    # bound, <= 0 on an active upper bound): the objective's sensitivity to
    # each row's bound
    y = np.zeros(p.m)
    k = 0
    for j in range(p.m):
        if eq[j]:
            continue
        if math.isfinite(hi[j]):
            y[j] += r.ineqlin.marginals[k]; k += 1
        if math.isfinite(lo[j]):
            y[j] -= r.ineqlin.marginals[k]; k += 1
    y[eq] = r.eqlin.marginals
    return r, y


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_kkt_residuals_vanish_at_highs_solution(seed):
    """The residual and dual-objective definitions (row bounds, box dual
    sets) give ~0 at HiGHS's own primal-dual solution."""
    p = bounded_instance(seed)
    r, y = _highs(p)
    k = pdhg.kkt_residuals(p, r.x, y)
    assert k["rel_primal"] <= 1e-9
    assert k["rel_dual"] <= 1e-9
    assert k["rel_gap"] <= 1e-9
    assert k["primal_obj"] == pytest.approx(r.fun, rel=1e-9, abs=1e-9)


@pytest.mark.parametrize("seed", [0, 1, 2, 3])
def test_bounded_lp_matches_highs(seed):
    p = bounded_instance(seed)
    r, y = _highs(p)
    o = pdhg.solve(p, pdhg.Settings(tol=1e-9, max_iter=400000))
    assert o.status == "OPTIMAL"
    assert o.kkt["primal_obj"] == pytest.approx(r.fun, rel=1e-6, abs=1e-6)
    # every row and box bound holds up to the tolerance
    ax = p.A @ o.x
    assert np.all(ax >= p.row_lo - 1e-6) and np.all(ax <= p.row_hi + 1e-6)
    box = np.arange(9)
    assert np.all(o.x[box] >= p.x_lo[box] - 1e-12) and np.all(o.x[box] <= p.x_hi[box] + 1e-12)


def _active_set_bounded_qp(H, g, A, lo, hi, xlo, xhi):
    """min 1/2 u'Hu + g'u s.t. lo <= A u <= hi, xlo <= u <= xhi by enumerating
    which bound each coordinate and row sits at (tiny sizes only)."""
    n, m = len(g), A.shape[0]
    best = None
    copts = [(None,)] + [(k,) for k in ("lo", "hi")]
    for cs in itertools.product(("free", "lo", "hi"), repeat=n):
        if any((c == "lo" and not math.isfinite(xlo[i])) or (c == "hi" and not math.isfinite(xhi[i]))
               for i, c in enumerate(cs)):
            continue
        for rs in itertools.product(("off", "lo", "hi"), repeat=m):
            if any((c == "lo" and not math.isfinite(lo[j])) or (c == "hi" and not math.isfinite(hi[j]))
                   for j, c in enumerate(rs)):
                continue
            F = [i for i in range(n) if cs[i] == "free"]
            fixed = np.array([xlo[i] if cs[i] == "lo" else (xhi[i] if cs[i] == "hi" else 0.0)
                              for i in range(n)])
            act = [j for j in range(m) if rs[j] != "off"]
            rhs_rows = np.array([lo[j] if rs[j] == "lo" else hi[j] for j in act])
            nf, na = len(F), len(act)
            K = np.zeros((nf + na, nf + na))
            rhs = np.zeros(nf + na)
            K[:nf, :nf] = H[np.ix_(F, F)]
            rhs[:nf] = -(g[F] + H[np.ix_(F, range(n))] @ fixed)
            if na:
                Aa = A[np.ix_(act, F)]
                K[:nf, nf:] = -Aa.T
                K[nf:, :nf] = Aa
                rhs[nf:] = rhs_rows - A[np.ix_(act, range(n))] @ fixed
            try:
                sol = np.linalg.solve(K, rhs)
            except np.linalg.LinAlgError:
                continue
            u = fixed.copy()
            u[F] = sol[:nf]
            if np.any(u < xlo - 1e-9) or np.any(u > xhi + 1e-9):
                continue
            au = A @ u
            if np.any(au < lo - 1e-9) or np.any(au > hi + 1e-9):
                continue
            val = 0.5 * u @ H @ u + g @ u
            if best is None or val < best[0] - 1e-12:
                best = (val, u)
    return best


@pytest.mark.parametrize("seed", [0, 1, 2])
def test_bounded_qp_matches_active_set(seed):
    """A strongly convex QP with range rows and box blocks: the oracle's
    solution equals the minimiser found by enumerating active bounds (the
    feasible stationary point of least objective)."""
    rng = np.random.default_rng(100 + seed)
    n, m = 5, 2
    A = rng.standard_normal((m, n))
    xf = rng.uniform(0.2, 0.8, n)
    ax = A @ xf
    lo = ax - rng.uniform(0.05, 0.3, m)
    hi = ax + rng.uniform(0.05, 0.3, m)
    xlo = xf - rng.uniform(0.1, 0.4, n)
    xhi = xf + rng.uniform(0.1, 0.4, n)
    xhi[4] = INF
    B = rng.standard_normal((n, n))
    H = B.T @ B / n + 0.1 * np.eye(n)
    g = 2.0 * rng.standard_normal(n)
    p = Problem(n=n, m=m, A=sp.csr_matrix(A), b=np.zeros(m), c=g, P=sp.csr_matrix(H),
                cones=[("box", 0, n, 0.0)], row_lo=lo, row_hi=hi, x_lo=xlo, x_hi=xhi)
    val, ustar = _active_set_bounded_qp(H, g, A, lo, hi, xlo, xhi)
    o = pdhg.solve(p, pdhg.Settings(tol=1e-10, max_iter=400000))
    assert o.status == "OPTIMAL"
    np.testing.assert_allclose(o.x, ustar, atol=1e-6)
    assert o.kkt["primal_obj"] == pytest.approx(val, rel=1e-7, abs=1e-8)


def test_bound_objective_with_row_bounds_worked_example():
    """Scaling off except bound-objective, rows 3 <= a1'x <= 3 and
    -inf <= a2'x <= 4: the combined bounds are (3, 4), so nu_b = 5 + 1 = 6;
    row and box bounds are divided by it (box [-12, 6] -> [-2, 1], the
    infinite endpoint stays infinite)."""
    A = sp.csr_matrix(np.array([[1.0, 1.0, 0.0], [0.0, 1.0, 1.0]]))
    p = Problem(n=3, m=2, A=A, b=np.zeros(2), c=np.array([0.0, 3.0, 4.0]),
                cones=[("box", 0, 2, 0.0), ("nonneg", 2, 1, 0.0)],
                row_lo=np.array([3.0, -INF]), row_hi=np.array([3.0, 4.0]),
                x_lo=np.array([-12.0, 6.0, 0.0]), x_hi=np.array([6.0, INF, 0.0]))
    from oracle import scaling
    sc = scaling.scale_problem(p, ruiz_iters=0, pock_chambolle=False, bound_objective=True)
    assert sc.nu_b == 6.0 and sc.nu_c == 6.0
    np.testing.assert_array_equal(sc.lo, [0.5, -INF])
    np.testing.assert_array_equal(sc.hi, [0.5, 4.0 / 6.0])
    np.testing.assert_array_equal(sc.xlo[:2], [-2.0, 1.0])
    np.testing.assert_array_equal(sc.xhi[:2], [1.0, INF])
