"""Pins of the oracle parts that whole-solve tests cannot see: the rescaling
factors, the restart / primal-weight / inner-tolerance bookkeeping, and the
averaged epochs of Alg. 1.

Every expected value below is derived by hand (the derivation is in each
docstring) or from an inequality the paper proves; none is computed by the
oracle.  Each test is written so that a plausible slip in the oracle (a
missing square root, block mean for block max or RMS, swapped exponents, an
inverted PID error, the wrong E_{n,k-1}, an off-by-one in K_tot, the wrong
iterate in the inner-tolerance rule, restarting from the last iterate
instead of the epoch average) makes it fail."""
import math

import numpy as np
import pytest
import scipy.sparse as sp

from instances import Problem, synth
from oracle import pdhg, scaling
from oracle.cones import Projector


def _prob(A, cones, b=None, c=None):
    A = sp.csr_matrix(np.asarray(A, dtype=float))
    m, n = A.shape
    return Problem(n=n, m=m, A=A, b=np.ones(m) if b is None else np.asarray(b, float),
                   c=np.ones(n) if c is None else np.asarray(c, float), cones=cones)


CONES_SOC3_RP2 = [("soc", 0, 3, 0.0), ("nonneg", 3, 2, 0.0)]


# ---------------------------------------------------------------------------
# Section "Problem Rescaling": eq. problem-rescaling, eq. cone-scaling-candidates,
# eq. cone-preserving-scaling
# ---------------------------------------------------------------------------
def test_ruiz_pass_worked_example():
    """One Ruiz pass on a 3x5 matrix whose columns 0-2 form one SOC(3) block
    and columns 3-4 are R+:

        A = [[16, 0, 0,  4, 0],
             [ 0, 4, 0,  0, 1],
             [ 0, 0, 1, 16, 0]]

    Row candidates sqrt(max_i |A_li|) = (sqrt16, sqrt4, sqrt16) = (4, 2, 4).
    Column candidates sqrt(max_l |A_li|) = (4, 2, 1, 4, 1); the SOC block takes
    their maximum (cone-preserving Ruiz): (4, 4, 4, 4, 1).
    A~_li = A_li / (dr_l dc_i):
        [[1, 0, 0, 1/4, 0], [0, 1/2, 0, 0, 1/2], [0, 0, 1/16, 1, 0]],
    S_y = 1/dr = (1/4, 1/2, 1/4), S_x = dc = (4, 4, 4, 4, 1).
    (A block mean would give 7/3 on the block; no square root 16.)"""
    A = [[16, 0, 0, 4, 0], [0, 4, 0, 0, 1], [0, 0, 1, 16, 0]]
    sc = scaling.scale_problem(_prob(A, CONES_SOC3_RP2), ruiz_iters=1,
                               pock_chambolle=False, bound_objective=False)
    np.testing.assert_array_equal(sc.Sx, [4, 4, 4, 4, 1])
    np.testing.assert_array_equal(sc.Sy, [0.25, 0.5, 0.25])
    np.testing.assert_array_equal(sc.A.toarray(), [[1, 0, 0, 0.25, 0], [0, 0.5, 0, 0, 0.5],
                                                   [0, 0, 1 / 16, 1, 0]])


def test_two_ruiz_passes_compose():
    """A second pass acts on A~ of the first: row maxima of A~ above are
    (1, 1/2, 1) -> row factors (1, 1/sqrt2, 1); column maxima (1, 1/2, 1/16,
    1, 1/2) -> candidates (1, 1/sqrt2, 1/4, 1, 1/sqrt2), block max 1 on the
    SOC block -> (1, 1, 1, 1, 1/sqrt2).  Accumulated: S_x = (4, 4, 4, 4,
    1/sqrt2), S_y = (1/4, sqrt2/2, 1/4)."""
    A = [[16, 0, 0, 4, 0], [0, 4, 0, 0, 1], [0, 0, 1, 16, 0]]
    sc = scaling.scale_problem(_prob(A, CONES_SOC3_RP2), ruiz_iters=2,
                               pock_chambolle=False, bound_objective=False)
    r2 = math.sqrt(2.0)
    np.testing.assert_allclose(sc.Sx, [4, 4, 4, 4, 1 / r2], rtol=1e-15)
    np.testing.assert_allclose(sc.Sy, [0.25, r2 / 2, 0.25], rtol=1e-15)


def test_pock_chambolle_pass_worked_example_alpha1():
    """One Pock-Chambolle pass (alpha = 1) on a 4x5 matrix, SOC(3) on columns
    0-2, R+ on 3-4:

        A = [[ 1,  0, 0,  0,  0],
             [-1,  3, 0,  0,  0],
             [ 0, -1, 6, -9,  0],
             [ 0,  0, 0,  0, 16]]

    Column candidates sqrt(sum_l |A_li|^(2-alpha)) = sqrt(2, 4, 6, 9, 16); the
    SOC block takes the root mean square of its candidates,
    sqrt((2 + 4 + 6)/3) = 2, so dc = (2, 2, 2, 3, 4).  Row factors
    sqrt(sum_i |A_li|^alpha) = sqrt(1, 4, 16, 16) = (1, 2, 4, 4).
    A~ = [[1/2, 0, 0, 0, 0], [-1/4, 3/4, 0, 0, 0], [0, -1/8, 3/4, -3/4, 0],
          [0, 0, 0, 0, 1]].
    (A block max would give sqrt6, a block mean of the candidates
    (sqrt2 + 2 + sqrt6)/3.)"""
    A = [[1, 0, 0, 0, 0], [-1, 3, 0, 0, 0], [0, -1, 6, -9, 0], [0, 0, 0, 0, 16]]
    sc = scaling.scale_problem(_prob(A, CONES_SOC3_RP2), ruiz_iters=0, pc_alpha=1.0,
                               pock_chambolle=True, bound_objective=False)
    np.testing.assert_array_equal(sc.Sx, [2, 2, 2, 3, 4])
    np.testing.assert_array_equal(sc.Sy, [1, 0.5, 0.25, 0.25])
    np.testing.assert_array_equal(sc.A.toarray(), [[0.5, 0, 0, 0, 0], [-0.25, 0.75, 0, 0, 0],
                                                   [0, -0.125, 0.75, -0.75, 0], [0, 0, 0, 0, 1]])


def test_pock_chambolle_pass_worked_example_alpha2():
    """alpha = 2 separates the two exponents: columns use
    sum_l |A_li|^0 (the nonzero count), rows sum_i |A_li|^2.

        A = [[1, 2, 2, 0, 4],
             [2, 1, 2, 0, 4],
             [2, 2, 1, 0, 4],
             [2, 2, 2, 2, 3]]

    Column counts (4, 4, 4, 1, 4) -> candidates (2, 2, 2, 1, 2), block RMS 2.
    Row 2-norms: sqrt(1+4+4+16) = sqrt(4+1+4+16) = sqrt(4+4+1+16) =
    sqrt(4+4+4+4+9) = 5.  (Swapped exponents would give the column 2-norms
    and sqrt of the row counts.)"""
    A = [[1, 2, 2, 0, 4], [2, 1, 2, 0, 4], [2, 2, 1, 0, 4], [2, 2, 2, 2, 3]]
    sc = scaling.scale_problem(_prob(A, CONES_SOC3_RP2), ruiz_iters=0, pc_alpha=2.0,
                               pock_chambolle=True, bound_objective=False)
    np.testing.assert_array_equal(sc.Sx, [2, 2, 2, 1, 2])
    np.testing.assert_array_equal(sc.Sy, [0.2, 0.2, 0.2, 0.2])


def test_bound_objective_worked_example():
    """Scaling off except bound-objective: nu_b = ||b|| + 1 = ||(3, 4)|| + 1 = 6,
    nu_c = ||(0, 12, 0, 5, 0)|| + 1 = 14; b^ = b/6, c^ = c/14, and the
    quadratic is multiplied by nu_b/nu_c = 3/7 (diag P = (7, 14, 21, 28, 35)
    becomes (3, 6, 9, 12, 15))."""
    A = [[1, 0, 0, 1, 0], [0, 1, 1, 0, 1]]
    p = _prob(A, CONES_SOC3_RP2, b=[3, 4], c=[0, 12, 0, 5, 0])
    p.P = sp.diags([7.0, 14, 21, 28, 35]).tocsr()
    sc = scaling.scale_problem(p, ruiz_iters=0, pock_chambolle=False, bound_objective=True)
    assert sc.nu_b == 6.0 and sc.nu_c == 14.0
    np.testing.assert_allclose(sc.b, [0.5, 4 / 6], rtol=1e-15)
    np.testing.assert_allclose(sc.c, [0, 12 / 14, 0, 5 / 14, 0], rtol=1e-15)
    np.testing.assert_allclose(sc.P.diagonal(), [3, 6, 9, 12, 15], rtol=1e-15)


def test_ruiz_then_pock_chambolle_order():
    """Ruiz passes come first and Pock-Chambolle acts on their output: on the
    Ruiz example, after its one pass A~ = [[1,0,0,1/4,0],[0,1/2,0,0,1/2],
    [0,0,1/16,1,0]]; PC (alpha = 1) then has column sums (1, 1/2, 1/16, 5/4,
    1/2) -> block RMS sqrt((1 + 1/2 + 1/16)/3) = sqrt(25/48) on the SOC
    block, sqrt(5/4), sqrt(1/2) on R+; row sums (5/4, 1, 17/16)."""
    A = [[16, 0, 0, 4, 0], [0, 4, 0, 0, 1], [0, 0, 1, 16, 0]]
    sc = scaling.scale_problem(_prob(A, CONES_SOC3_RP2), ruiz_iters=1, pc_alpha=1.0,
                               pock_chambolle=True, bound_objective=False)
    blk = math.sqrt(25 / 48)
    np.testing.assert_allclose(sc.Sx, [4 * blk, 4 * blk, 4 * blk, 4 * math.sqrt(1.25),
                                       math.sqrt(0.5)], rtol=1e-15)
    np.testing.assert_allclose(sc.Sy, [0.25 / math.sqrt(1.25), 0.5, 0.25 / math.sqrt(17 / 16)],
                               rtol=1e-15)


# ---------------------------------------------------------------------------
# eq. practical-restart-rule, eq. pid-error, eq. pid-weight,
# eq. monotone-primal-inner-tol, eq. rh-update: trace consistency
# ---------------------------------------------------------------------------
def _metric_E(A, tau, sigma, eta, dx, dy):
    """E = sqrt(eta * ||(dx, dy)||^2_M) with the dense preconditioner
    M = [[I/tau, A^T], [A, I/sigma]] (eq. theory-preconditioner); eta times
    this norm is eq. practical-fixed-point-movement."""
    Ad = A.toarray()
    n, m = Ad.shape[1], Ad.shape[0]
    M = np.block([[np.eye(n) / tau, Ad.T], [Ad, np.eye(m) / sigma]])
    z = np.concatenate([dx, dy])
    return math.sqrt(max(eta * float(z @ M @ z), 0.0))


def check_restart_trace(S, tr, st):
    """Replays the decisions of a reflected-Halpern trace from its raw
    iterates in the paper's notation and returns the count of each restart
    trigger.  Epoch n starts at the entry after a restart; k counts the
    evaluations of the epoch; K_tot = (entry index) + 1."""
    eta, A = S.eta, S.sc.A
    kinds = dict(sufficient=0, necessary=0, artificial=0, pid=0)
    start = 0                       # entry at which the current epoch started
    E0 = Eprev = None
    I_prev = e_prev = 0.0
    for j, t in enumerate(tr):
        k = j - start
        ktot = j + 1
        assert t["tau"] == pytest.approx(eta / t["omega"], rel=1e-15)
        assert t["sigma"] == pytest.approx(eta * t["omega"], rel=1e-15)
        check = k == 0 or ktot % st.check_every == 0 or ktot == st.max_iter
        assert bool(t["check"]) == check, j
        restart = False
        if check:
            E = _metric_E(A, t["tau"], t["sigma"], eta, t["x"] - t["wx"], t["y"] - t["wy"])
            assert t["E"] == pytest.approx(E, rel=1e-9), j
            if k == 0:
                E0 = E
            else:
                suff = E <= st.beta_s * E0
                nec = E <= st.beta_n * E0 and E > Eprev
                art = (k + 1) >= st.beta_a * ktot   # evaluations of the epoch vs in total
                restart = suff or nec or art
                if restart:
                    kinds["sufficient" if suff else ("necessary" if nec else "artificial")] += 1
            Eprev = E
        assert bool(t["restart"]) == restart, j
        if j + 1 == len(tr):
            break
        nxt = tr[j + 1]
        anchor_x, anchor_y = tr[start]["x"], tr[start]["y"]
        if restart:
            np.testing.assert_array_equal(nxt["x"], t["wx"])
            np.testing.assert_array_equal(nxt["y"], t["wy"])
            dxm = np.linalg.norm(t["wx"] - anchor_x)
            dym = np.linalg.norm(t["wy"] - anchor_y)
            om = t["omega"]
            if dxm > 1e-12 and dym > 1e-12:
                e = math.log(dym / (om * dxm))
                I_n = st.pid_beta_i * I_prev + e
                om_next = math.exp(math.log(om) + st.pid_kp * e + st.pid_ki * I_n
                                   + st.pid_kd * (e - e_prev))
                I_prev, e_prev = I_n, e
                kinds["pid"] += 1
            else:
                om_next = om
            assert nxt["omega"] == pytest.approx(om_next, rel=1e-13), j
            assert nxt["eps_in"] == t["eps_in"], j       # inherited across the restart
            start = j + 1
        else:
            c1, c3 = (k + 1) / (k + 2), 1.0 / (k + 2)
            rho = st.rho
            np.testing.assert_allclose(
                nxt["x"], c1 * (2 * rho * t["wx"] + (1 - 2 * rho) * t["x"]) + c3 * anchor_x,
                rtol=1e-13, atol=1e-15)
            np.testing.assert_allclose(
                nxt["y"], c1 * (2 * rho * t["wy"] + (1 - 2 * rho) * t["y"]) + c3 * anchor_y,
                rtol=1e-13, atol=1e-15)
            assert nxt["omega"] == t["omega"], j
            eps = min(t["eps_in"], max(st.gamma_in * np.linalg.norm(nxt["x"] - t["x"]) / t["tau"],
                                       st.eps_min))
            assert nxt["eps_in"] == pytest.approx(eps, rel=1e-12), j
    return kinds


@pytest.mark.parametrize("make,check_every", [
    (lambda: synth.tiny_qp(1), 4),
    (lambda: synth.tiny_mixed(4), 2),
])
def test_restart_pid_inner_tolerance_trace(make, check_every):
    """Every check flag, E value, restart decision (with its trigger), primal
    weight update, restart point, Halpern step and inner tolerance of a long
    oracle trace follows from the raw iterates and the paper's rules; the
    run contains restarts of all three kinds and several PID updates
    (with check_every = 2 the epoch's previous checked E is two evaluations
    back)."""
    p = make()
    iters = 700
    st = pdhg.Settings(trace_iters=iters, max_iter=iters, check_every=check_every, tol=1e-14)
    S = pdhg.setup(p, st)
    r = pdhg.solve(p, st, S=S)
    assert len(r.trace) >= 300
    kinds = check_restart_trace(S, r.trace, st)
    assert kinds["pid"] >= 3, kinds
    assert min(kinds["sufficient"], kinds["necessary"], kinds["artificial"]) >= 1, kinds


# ---------------------------------------------------------------------------
# Alg. 1 (restarted averaged PDHG): ergodic gap bound of the epoch average
# ---------------------------------------------------------------------------
def _lagrangian(S, x, y):
    """L(x, y) = 1/2 <x, Q x> + <c, x> + <y, b - A x> (eq. saddle), scaled data."""
    return 0.5 * float(x @ S.q(x)) + float(S.sc.c @ x) + float(y @ (S.sc.b - S.sc.A @ x))


def _gap(S, z, zh):
    """Q(z, zh) = L(x, yh) - L(xh, y) (eq. ordinary-duality-gap)."""
    return _lagrangian(S, z[0], zh[1]) - _lagrangian(S, zh[0], z[1])


def _pnorm2(S, tau, sigma, dx, dy):
    A = S.sc.A
    return float(dx @ dx) / tau + float(dy @ dy) / sigma + 2.0 * float(dy @ (A @ dx))


def _comparison_points(S, p, z0, z1, zb, T, tau, sigma, rng, zstar):
    """Points of K x Y: the solution, random points projected onto K, points
    near the epoch start and the epoch's first iterate, and two points that
    make the bound tight for the tested point zb: the dual point
    y0 + T sigma (b - A xb) with x = x0 (the maximiser of the bound's
    difference over y, which the telescoped dual updates control only for
    the average) and the primal point Pi_K(x0 - T tau (Q x0 + c - A^T yb))
    with y = y0."""
    proj = Projector(p.cones, p.n)
    sc = S.sc
    pts = [zstar,
           (z0[0], z0[1] + T * sigma * (sc.b - sc.A @ zb[0])),
           (proj.project(z0[0] - T * tau * (S.q(z0[0]) + sc.c - sc.A.T @ zb[1])), z0[1])]
    for _ in range(12):
        pts.append((proj.project(rng.standard_normal(p.n)), rng.standard_normal(p.m)))
    for base in (z0, z1):
        for scale in (1e-3, 1e-2, 1e-1):
            pts.append((proj.project(base[0] + scale * rng.standard_normal(p.n)),
                        base[1] + scale * rng.standard_normal(p.m)))
    return pts


@pytest.mark.parametrize("make,T", [
    (lambda: synth.tiny_mixed(3, lowrank=False), 1),
    (lambda: synth.tiny_mixed(3, lowrank=False), 6),
    (lambda: synth.tiny_mixed(2, with_q=False), 16),
    (lambda: synth.tiny_nonneg_qp(2, n=8, m=3, diag_only=True), 5),
])
def test_avg_epoch_ergodic_gap_bound(make, T):
    """Prop. one-epoch-estimates (eq. ordinary-gap-rate): with exact proximal
    steps (diagonal Q) and fixed tau, sigma, the point an epoch restarts from
    satisfies Q(zbar^{n,T}, zh) <= ||z^{n,0} - zh||_P^2 / (2T) for every zh in
    K x Y.  The restart points are read from the oracle's trace of Alg. 1
    (the state at the first evaluation of the next epoch)."""
    p = make()
    epochs = 4
    st = pdhg.Settings(scheme="avg", avg_epoch=T, trace_iters=epochs * T + 1,
                       max_iter=epochs * T + 1, tol=1e-16)
    S = pdhg.setup(p, st)
    assert S.q.is_diag
    ref = pdhg.solve(p, pdhg.Settings(tol=1e-11, max_iter=200000), S=pdhg.setup(p))
    zstar = (S.sc.scale_x(ref.x), S.sc.scale_y(ref.y))
    r = pdhg.solve(p, st, S=S)
    tr = r.trace
    tau, sigma = tr[0]["tau"], tr[0]["sigma"]
    rng = np.random.default_rng(11)
    worst = -np.inf
    for n in range(epochs):
        t0 = tr[n * T]
        z0 = (t0["x"], t0["y"])
        z1 = (t0["wx"], t0["wy"])
        zb = (tr[(n + 1) * T]["x"], tr[(n + 1) * T]["y"])    # restart point of the next epoch
        for zh in _comparison_points(S, p, z0, z1, zb, T, tau, sigma, rng, zstar):
            lhs = _gap(S, zb, zh)
            rhs = _pnorm2(S, tau, sigma, z0[0] - zh[0], z0[1] - zh[1]) / (2.0 * T)
            assert lhs <= rhs + 1e-10 * (1.0 + abs(rhs)), (n, lhs, rhs)
            worst = max(worst, lhs - rhs)
    # the averaged primal point stays in K (convexity), exactly up to rounding
    proj = Projector(p.cones, p.n)
    for n in range(1, epochs + 1):
        xb = tr[n * T]["x"]
        np.testing.assert_allclose(proj.project(xb), xb, atol=1e-12)
