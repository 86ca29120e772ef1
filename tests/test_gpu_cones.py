"""GPU parity of the cone projections (Appendix C): the device routines the
solver uses, called through the diagnostic entry pdhcg_project_cones, against
the oracle's projections, element by element, on >= 1e5 blocks per cone type
and metric.  The inputs mix generic points over many scales with every
special case of the appendix: SOC r_t = 0, the RSOC singular case
kappa = sqrt(m_s) r_s + sqrt(m_t) r_t = 0, EXP with r0 <= 0 and s0 <= 0, POW
r_z = 0, points inside the cone and inside the polar cone, points within
rounding of either boundary (the EXP near-polar fallback included), near the
apex, and POW exponents close to 0 and 1.

Tolerance: |device - oracle| <= 1e-9 * max(1, ||r||_inf) per block (the
projections are 1-Lipschitz in the M-norm and both sides solve their roots to
~1e-15 relative; the EXP closest-point fallback of the oracle is accurate to
sqrt(eps) in the ray parameter, but there the projection itself is within
rounding of zero)."""
import math

import numpy as np
import pytest

import paper_2608_09159_amd as G
from oracle import cones as OC

pytestmark = pytest.mark.gpu

TOL = 1e-9
N_BIG = 100_000


def _scales(rng, n, lo=-3.0, hi=3.0):
    return 10.0 ** rng.uniform(lo, hi, size=n)


def _metric(rng, shape, const_frac=0.1):
    M = 10.0 ** rng.uniform(-1.0, 1.0, size=shape)
    k = int(const_frac * shape[0])
    M[:k] = M[:k, :1]                      # constant on the block: Euclidean formula
    return M


def _compare(name, dev, ref, R):
    assert np.all(np.isfinite(dev)), (name, "non-finite device output",
                                      R[~np.all(np.isfinite(dev), axis=1)][:3])
    scale = np.maximum(1.0, np.max(np.abs(R), axis=1))
    err = np.max(np.abs(dev - ref), axis=1) / scale
    worst = int(np.argmax(err))
    print(f"[cones] {name}: {R.shape[0]} blocks, max scaled error {err[worst]:.2e}", flush=True)
    assert err[worst] <= TOL, (name, worst, R[worst], dev[worst], ref[worst])


# ---------------------------------------------------------------------------
# SOC (v, t) and RSOC (v, s, t)
# ---------------------------------------------------------------------------
def soc_inputs(rng, n, d, M):
    """Rows of several kinds (the metric M of the same shape, or None)."""
    R = rng.standard_normal((n, d)) * _scales(rng, n)[:, None]
    k = n // 10
    idx = rng.permutation(n)
    parts = np.array_split(idx, 10)
    v = R[:, :-1]
    nv = np.linalg.norm(v, axis=1)
    # inside the cone
    R[parts[0], -1] = nv[parts[0]] * (1.0 + rng.uniform(0, 2, size=parts[0].size))
    # inside the polar cone -M^-1 K (SOC is self-dual)
    if d > 1:
        mv = np.ones((n, d - 1)) if M is None else M[:, :-1]
        mt = np.ones(n) if M is None else M[:, -1]
        p = parts[1]
        R[p, -1] = -np.linalg.norm(mv[p] * v[p], axis=1) / mt[p] * (1.0 + rng.uniform(0, 2, p.size))
    # r_t = 0 exactly
    R[parts[2], -1] = 0.0
    # on the boundary within rounding
    R[parts[3], -1] = nv[parts[3]] * (1.0 + rng.choice([-1, 1], parts[3].size) * 1e-15)
    # near the apex
    R[parts[4]] *= 1e-12
    # large scale
    R[parts[5]] *= 1e12
    # t much larger or much smaller than ||v|| in magnitude
    R[parts[6], -1] = -nv[parts[6]] * 1e-9
    R[parts[7], :-1] *= 1e-9
    return R


def rsoc_inputs(rng, n, d, M):
    R = rng.standard_normal((n, d)) * _scales(rng, n)[:, None]
    parts = np.array_split(rng.permutation(n), 10)
    v = R[:, :-2]
    vv = np.einsum("ij,ij->i", v, v)
    # inside: s, t > 0 with ||v||^2 <= 2 s t
    p = parts[0]
    s = np.abs(R[p, -2]) + 1e-3
    R[p, -2] = s
    R[p, -1] = vv[p] / (2 * s) * (1 + rng.uniform(0, 2, p.size)) + 1e-3
    # kappa = 0 exactly: equal metric on s and t, r_t = -r_s
    p = parts[1]
    R[p, -1] = -R[p, -2]
    if M is not None:
        M[p, -1] = M[p, -2]
    # s = t = 0
    R[parts[2], -2:] = 0.0
    # v = 0
    R[parts[3], :-2] = 0.0
    # near apex / large
    R[parts[4]] *= 1e-12
    R[parts[5]] *= 1e12
    # boundary within rounding
    p = parts[6]
    s = np.abs(R[p, -2]) + 1e-3
    R[p, -2] = s
    R[p, -1] = vv[p] / (2 * s) * (1 + rng.choice([-1, 1], p.size) * 1e-15)
    # polar side: both scalars negative and large
    p = parts[7]
    R[p, -2] = -np.abs(R[p, -2]) * 10
    R[p, -1] = -np.abs(R[p, -1]) * 10
    return R


SOC_DIMS = [(1, 2000), (2, 10000), (3, 20000), (5, 10000), (17, 20000), (20, 40000),
            (33, 5000), (70, 2000), (150, 1000)]
RSOC_DIMS = [(2, 10000), (3, 20000), (10, 50000), (18, 10000), (40, 10000), (70, 2000)]


@pytest.mark.parametrize("metric", [False, True], ids=["euclid", "metric"])
def test_soc_projection_parity(metric):
    rng = np.random.default_rng(101 + metric)
    total = 0
    for d, n in SOC_DIMS:
        M = _metric(rng, (n, d)) if metric else None
        R = soc_inputs(rng, n, d, M)
        dev = G.project_cones("soc", R, M)
        ref = OC.soc_metric(R, M) if metric else OC.soc_euclid(R)
        _compare(f"soc d={d} {'metric' if metric else 'euclid'}", dev, ref, R)
        total += n
    assert total >= N_BIG


@pytest.mark.parametrize("metric", [False, True], ids=["euclid", "metric"])
def test_rsoc_projection_parity(metric):
    rng = np.random.default_rng(201 + metric)
    total = 0
    for d, n in RSOC_DIMS:
        M = _metric(rng, (n, d)) if metric else None
        R = rsoc_inputs(rng, n, d, M)
        dev = G.project_cones("rsoc", R, M)
        ref = OC.rsoc_metric(R, M) if metric else OC.rsoc_euclid(R)
        _compare(f"rsoc d={d} {'metric' if metric else 'euclid'}", dev, ref, R)
        total += n
    assert total >= N_BIG


# ---------------------------------------------------------------------------
# EXP (r, s, t): K* = {(u, v, w): u < 0, -u e^{v/u} <= e w} u {(0, v, w): v, w >= 0}
# ---------------------------------------------------------------------------
def exp_inputs(rng, n, M):
    R = rng.standard_normal((n, 3)) * _scales(rng, n, -2, 2)[:, None]
    m = np.ones((n, 3)) if M is None else M
    parts = np.array_split(rng.permutation(n), 12)
    # r0 <= 0 and s0 <= 0
    p = parts[0]
    R[p, 0] = -np.abs(R[p, 0])
    R[p, 1] = -np.abs(R[p, 1])
    R[parts[1][: parts[1].size // 4], 1] = 0.0
    # inside: s > 0, t >= s e^{r/s}
    p = parts[2]
    s = np.abs(R[p, 1]) + 1e-3
    q = rng.uniform(-5, 5, p.size)
    R[p, 0] = s * q
    R[p, 1] = s
    R[p, 2] = s * np.exp(q) * (1 + rng.uniform(0, 1, p.size))
    # inside the polar cone -M^-1 K*
    p = parts[3]
    a = np.abs(R[p, 0]) + 1e-3
    vv = rng.standard_normal(p.size) * a
    w = a * np.exp(-vv / a - 1.0) * (1 + rng.uniform(0, 1, p.size))
    D = np.stack([-a, vv, w], axis=1)
    R[p] = -D / m[p]
    # within rounding of the polar cone's boundary (the near-polar fallback)
    p = parts[4][:400]
    a = np.abs(R[p, 0]) + 1e-3
    vv = rng.standard_normal(p.size) * a
    w = a * np.exp(-vv / a - 1.0) * (1 + rng.choice([-1, 1], p.size) * 1e-14)
    D = np.stack([-a, vv, w], axis=1)
    R[p] = -D / m[p]
    # within rounding of the cone's boundary
    p = parts[5]
    s = np.abs(R[p, 1]) + 1e-3
    q = rng.uniform(-5, 5, p.size)
    R[p, 0] = s * q
    R[p, 1] = s
    R[p, 2] = s * np.exp(q) * (1 + rng.choice([-1, 1], p.size) * 1e-15)
    # large ratios r/s and s = 0 with r > 0
    p = parts[6]
    R[p, 1] = np.abs(R[p, 1]) * 1e-3
    p = parts[7]
    R[p, 1] = 0.0
    R[p, 0] = np.abs(R[p, 0])
    # near apex, large scale
    R[parts[8]] *= 1e-10
    R[parts[9]] *= 1e8
    return R


@pytest.mark.parametrize("metric", [False, True], ids=["euclid", "metric"])
def test_exp_projection_parity(metric):
    rng = np.random.default_rng(301 + metric)
    n = N_BIG
    M = _metric(rng, (n, 3)) if metric else None
    R = exp_inputs(rng, n, M)
    dev = G.project_cones("exp", R, M)
    ref = np.empty_like(R)
    for i in range(n):
        mm = (1.0, 1.0, 1.0) if M is None else M[i]
        ref[i] = OC.exp_metric_one(R[i], mm)
    _compare(f"exp {'metric' if metric else 'euclid'}", dev, ref, R)


# ---------------------------------------------------------------------------
# POW(alpha) (x, y, z); dual printed in the appendix:
# (p/alpha)^alpha (q/(1-alpha))^(1-alpha) >= |w|, p, q >= 0
# ---------------------------------------------------------------------------
def pow_inputs(rng, n, M):
    R = rng.standard_normal((n, 3)) * _scales(rng, n, -2, 2)[:, None]
    al = rng.uniform(0.02, 0.98, n)
    m = np.ones((n, 3)) if M is None else M
    parts = np.array_split(rng.permutation(n), 10)
    al[parts[0]] = rng.choice([0.01, 0.05, 0.5, 0.95, 0.99], parts[0].size)
    R[parts[1], 2] = 0.0                                  # r_z = 0
    p = parts[2]                                          # inside
    x, y = np.abs(R[p, 0]) + 1e-3, np.abs(R[p, 1]) + 1e-3
    R[p, 0], R[p, 1] = x, y
    R[p, 2] = x ** al[p] * y ** (1 - al[p]) * rng.uniform(-1, 1, p.size)
    p = parts[3]                                          # inside the polar cone
    pp, qq = np.abs(R[p, 0]) + 1e-3, np.abs(R[p, 1]) + 1e-3
    ww = (pp / al[p]) ** al[p] * (qq / (1 - al[p])) ** (1 - al[p]) * rng.uniform(-1, 1, p.size)
    R[p] = -np.stack([pp, qq, ww], axis=1) / m[p]
    p = parts[4]                                          # boundary within rounding
    x, y = np.abs(R[p, 0]) + 1e-3, np.abs(R[p, 1]) + 1e-3
    R[p, 0], R[p, 1] = x, y
    R[p, 2] = x ** al[p] * y ** (1 - al[p]) * (1 + rng.choice([-1, 1], p.size) * 1e-15)
    R[parts[5], 0] = -np.abs(R[parts[5], 0])              # one negative base
    R[parts[6]] *= 1e-10
    R[parts[7]] *= 1e8
    return R, al


@pytest.mark.parametrize("metric", [False, True], ids=["euclid", "metric"])
def test_pow_projection_parity(metric):
    rng = np.random.default_rng(401 + metric)
    n = N_BIG
    M = _metric(rng, (n, 3)) if metric else None
    R, al = pow_inputs(rng, n, M)
    dev = G.project_cones("pow", R, M, al)
    ref = np.empty_like(R)
    for i in range(n):
        mm = (1.0, 1.0, 1.0) if M is None else M[i]
        ref[i] = OC.pow_metric_one(R[i], al[i], mm)
    _compare(f"pow {'metric' if metric else 'euclid'}", dev, ref, R)


def test_elementwise_projection():
    rng = np.random.default_rng(5)
    R = rng.standard_normal((1000, 4))
    np.testing.assert_array_equal(G.project_cones("free", R), R)
    np.testing.assert_array_equal(G.project_cones("nonneg", R), np.maximum(R, 0.0))


@pytest.mark.parametrize("metric", [False, True], ids=["euclid", "metric"])
def test_exp1_projection_parity(metric):
    """Exponential block with the middle coordinate fixed at one: points
    inside, with t0 <= 0, near the boundary, at large and small scales."""
    rng = np.random.default_rng(501 + metric)
    n = N_BIG
    R = rng.standard_normal((n, 3)) * _scales(rng, n, -1, 1)[:, None]
    parts = np.array_split(rng.permutation(n), 6)
    R[parts[0], 2] = -np.abs(R[parts[0], 2])
    R[parts[1], 2] = np.exp(R[parts[1], 0]) * rng.uniform(1, 2, parts[1].size)
    R[parts[2], 2] = np.exp(R[parts[2], 0]) * (1 + rng.choice([-1, 1], parts[2].size) * 1e-15)
    R[parts[3], 0] *= 5.0
    R[parts[4], 2] *= 1e6
    # far outside: z0 up to ~700 with t0 of either sign (where the e^(2z)
    # term dominates the stationarity function)
    p5 = parts[5]
    R[p5, 0] = rng.uniform(20.0, 700.0, p5.size)
    R[p5, 2] = rng.standard_normal(p5.size) * 10.0 ** rng.uniform(-1, 3, p5.size)
    M = _metric(rng, (n, 3)) if metric else None
    dev = G.project_cones("exp1", R, M)
    ref = np.empty_like(R)
    for i in range(n):
        ref[i] = OC.exp1_metric_one(R[i], (1.0, 1.0, 1.0) if M is None else M[i])
    _compare(f"exp1 {'metric' if metric else 'euclid'}", dev, ref, R)
