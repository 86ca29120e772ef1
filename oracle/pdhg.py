"""Restarted PDHG for conic convex QP, written from the paper step by step in
plain NumPy/SciPy float64.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Passages followed
-----------------
* PDHG operator, primal first (eq. theory-pdhg-map):
      p = prox_{tau F}(x + tau A^T y),  q = y + sigma (b - A(2p - x)).
* Proximal subproblem (eq. prox-subproblem) with v = x + tau A^T y:
  - diagonal Q: one metric projection, M = I + tau Q,
    x~ = M^-1 (v - tau c)  (eq. diagonal-q-metric);
  - general Q: Jacobi-preconditioned projected Barzilai-Borwein
    (eq. jacobi-inner-metric, eq. jacobi-bb-step) with the Euclidean stop test
    (eq. current-inner-step-stop); "euclid" selects plain projected BB1
    (eq. bb-inner-gradient, eq. bb-step).
* Reflected-Halpern epochs (eq. stored-pdhg-candidate, eq. rh-update,
  eq. restart-output) with reflection rho.
* Restarted averaged epochs (Alg. 1, eq. theory-epoch-average).
* Adaptive inner tolerance (eq. monotone-primal-inner-tol).
* Step sizes tau = eta/omega, sigma = eta omega, eta = 0.998/||A||_2
  (eq. practical-stepsizes); PID primal weight (eq. pid-error, pid-weight).
* Adaptive restart (eq. practical-fixed-point-movement,
  eq. practical-restart-rule); defaults of Table practical-defaults.
* Termination on the unscaled candidate: relative KKT residuals of the
  optimality conditions eq. kkt-cqp.
* Implementation form (eq. solver-input): row bounds l <= A x <= u and box
  blocks.  The paper states the form, not the dual step; written from the
  saddle function with the row constraint A x in B = [l, u], the dual
  candidate is w_y = sigma (Pi_B(q) - q) with q = A(2 w_x - x) - y/sigma,
  which is y + sigma (b - A(2 w_x - x)) when l = u = b (equality rows use
  that form); boxes clamp in the prox.
* Exponential blocks with the middle coordinate fixed at one ("exp1", the
  Fisher experiment's representation): projection onto {(z, 1, t): e^z <= t}
  scaled to the block's coordinates; KKT terms from the set's recession
  cone and support function (exp1_dual_terms).

Readings where the paper is silent (each also listed in the design doc):
* ||A||_2 by 128 power iterations on A^T A from 1/sqrt(n) (overridable);
  a zero estimate (A = 0 or no rows) is replaced by 1;
* omega_0 = ||c^||/||b^|| when both exceed 1e-10, else 1 (overridable);
* start z = (Pi_X(x0^), y0^), x0^ = 0 without a warm start (0 lies in every
  cone but not necessarily in a box); the inner solve starts at the Halpern
  primal state x; first inner step uses alpha = 1 (Jacobi) or
  1/max(diag Q^ + 1/tau) (Euclidean); J_max = 500;
* checks at k = 0 of each epoch (defines E_0), whenever the global
  iteration count is a multiple of check_every, and at the last allowed
  evaluation (max_iter), so the reported residuals are a check's; artificial
  restart when
  (k+1) >= beta_a K_tot, K_tot counting the current evaluation; E_{n,k-1} is
  the previous checked E of the epoch;
* PID: skipped when either movement is <= 1e-12; integral and previous error
  start at zero;
* a restart replaces the Halpern update of that iteration and restarts from
  the candidate; the inner tolerance is kept across restarts;
* relative KKT: rel_p = ||Ax - b||/(1 + ||b||),
  rel_d = ||Pi_K(-s)||/(1 + ||c||) with s = Qx + c - A^T y (= dist(s, K^*)),
  rel_gap = |P - D|/(1 + |P| + |D|), P = x'Qx/2 + c'x, D = b'y - x'Qx/2;
* the metric of a cone block is treated as constant (Euclidean formula) when
  diag(Q^) is constant on it.

Parity status: every step above is pinned by tests/test_oracle_*.py against
closed forms, invariants or brute force.  The restart, primal-weight and
inner-tolerance bookkeeping is pinned by replaying long traces against the
paper's rules with the restart metric recomputed from the dense
preconditioner (tests/test_oracle_pins.py); the averaged scheme's restart
points by the ergodic gap bound of Prop. one-epoch-estimates.
"""
from __future__ import annotations

import math
import time
from dataclasses import dataclass, field, asdict
from typing import Optional

import numpy as np
import scipy.sparse as sp

from .cones import Projector, exp1_dual_terms
from .scaling import scale_problem


@dataclass
class Settings:
    tol: float = 1e-6
    max_iter: int = 100_000
    time_limit: float = 3600.0
    check_every: int = 64
    scheme: str = "rh"            # "rh" (reflected Halpern) or "avg" (Alg. 1)
    rho: float = 1.0              # reflection coefficient
    avg_epoch: int = 64           # T of Alg. 1
    inner: str = "jacobi"         # "jacobi" | "euclid"
    fixed_inner: int = 0          # >0: exactly that many inner steps
    j_max: int = 500
    eps_in0: float = 1e-3
    gamma_in: float = 5e-4
    eps_min: float = 1e-9
    beta_s: float = 0.2
    beta_n: float = 0.8
    beta_a: float = 0.36
    pid_beta_i: float = 0.3
    pid_kp: float = 0.99
    pid_ki: float = 0.01
    pid_kd: float = 0.0
    ruiz_iters: int = 10
    pc_alpha: float = 1.0
    pock_chambolle: bool = True
    bound_objective: bool = True
    scaling: bool = True
    cone_scaling: str = "block"   # "block" (cone-preserving) | "rescaled" (rescaled-cone)
    power_iters: int = 128
    a_norm: float = 0.0           # >0 overrides the power iteration
    omega0: float = 0.0           # >0 overrides the initial primal weight
    trace_iters: int = 0


def power_norm(A, iters=128):
    """sigma_max(A) by power iteration on A^T A from 1/sqrt(n) * ones."""
    n = A.shape[1]
    z = np.full(n, 1.0 / math.sqrt(n))
    lam = 0.0
    for _ in range(iters):
        w = A.T @ (A @ z)
        lam = float(np.linalg.norm(w))
        if lam == 0.0:
            break
        z = w / lam
    return math.sqrt(lam)


class QOp:
    """Q^ u = P^ u + R^T (D^ (R^ u)) without materialising Q."""

    def __init__(self, P, R, D, n):
        self.P, self.R, self.D, self.n = P, R, D, n
        d = np.zeros(n)
        if P is not None:
            d += P.diagonal()
        if R is not None:
            d += np.einsum("ai,ab,bi->i", R, D, R)
        self.diag = d
        self.is_diag = R is None and (P is None or _is_diagonal(P))

    def __call__(self, u):
        out = np.zeros(self.n)
        if self.P is not None:
            out += self.P @ u
        if self.R is not None:
            out += self.R.T @ (self.D @ (self.R @ u))
        return out


def _is_diagonal(P):
    P = sp.coo_matrix(P)
    return bool(np.all(P.row == P.col))


def _signed_bound_dot(v, lo, hi):
    """sum_j (v_j^+ lo_j - v_j^- hi_j), taking only the endpoints that a
    nonzero part of v selects (the others may be infinite)."""
    pos = v > 0
    neg = v < 0
    return float(v[pos] @ lo[pos]) + float(v[neg] @ hi[neg])


def box_dual_part(s, lo, hi):
    """For box coordinates with bounds lo, hi: lambda = the projection of the
    reduced cost s onto the set it may take at a solution (R when both
    bounds are finite, R+ with only lo, R- with only hi, {0} with neither),
    so dist(s, that set) = |s - lambda|."""
    lf, hf = np.isfinite(lo), np.isfinite(hi)
    lam = np.where(lf & hf, s, np.where(lf, np.maximum(s, 0.0),
                                        np.where(hf, np.minimum(s, 0.0), 0.0)))
    return lam


def kkt_residuals(prob, x, y, proj=None):
    """Relative KKT residuals of the original problem (eq. kkt-cqp) at (x, y).

    With row bounds the primal residual is the distance of A x to [l, u] and
    the dual objective takes sum(y^+ l - y^- u) in place of <b, y>; on box
    coordinates the dual residual is the distance of s to the set the
    reduced cost may take (box_dual_part) and the dual objective gains
    sum(lambda^+ l^x - lambda^- u^x).  The normaliser of the primal residual
    is 1 + ||combined bounds|| (||b|| for equalities)."""
    from .scaling import combined_bounds
    if proj is None:
        proj = Projector(prob.cones, prob.n, prob.x_lo, prob.x_hi)
    Qx = np.zeros(prob.n)
    if prob.P is not None:
        Qx += prob.P @ x
    if prob.R is not None:
        Qx += prob.R.T @ (prob.D @ (prob.R @ x))
    Ax = prob.A @ x
    if prob.row_lo is None:
        rpv = Ax - prob.b
        bnorm = float(np.linalg.norm(prob.b))
        by = float(prob.b @ y)
    else:
        rpv = Ax - np.minimum(np.maximum(Ax, prob.row_lo), prob.row_hi)
        bnorm = float(np.linalg.norm(combined_bounds(prob.row_lo, prob.row_hi)))
        by = _signed_bound_dot(y, prob.row_lo, prob.row_hi)
    rp = float(np.linalg.norm(rpv)) / (1.0 + bnorm)
    s = Qx + prob.c - prob.A.T @ y
    dres = proj.project(-s)
    boxterm = 0.0
    if proj.box_idx.size:
        sb = s[proj.box_idx]
        lam = box_dual_part(sb, proj.box_lo, proj.box_hi)
        dres[proj.box_idx] = sb - lam
        boxterm = _signed_bound_dot(lam, proj.box_lo, proj.box_hi)
    for kind, st, d, al in prob.cones:
        if kind == "exp1":           # fixed-middle exponential blocks
            lam, term = exp1_dual_terms(*s[st:st + 3])
            dres[st:st + 3] = s[st:st + 3] - np.array(lam)
            boxterm += term
    rd = float(np.linalg.norm(dres)) / (1.0 + float(np.linalg.norm(prob.c)))
    xqx = float(x @ Qx)
    pobj = 0.5 * xqx + float(prob.c @ x)
    dobj = by + boxterm - 0.5 * xqx
    # an exp1 reduced cost with lambda_a < 0 = lambda_c has dual value -inf
    gap = abs(pobj - dobj) / (1.0 + abs(pobj) + abs(dobj)) if math.isfinite(dobj) else 1.0
    return dict(rel_primal=rp, rel_dual=rd, rel_gap=gap, primal_obj=pobj, dual_obj=dobj)


@dataclass
class Setup:
    prob: object
    st: Settings
    sc: object
    q: QOp
    proj: Projector
    euclid_blocks: np.ndarray
    a_norm: float
    eta: float
    omega0: float
    kproj: Projector = None     # original-space projector (bounds unscaled) for the checks


def setup(prob, st: Settings = None):
    st = st or Settings()
    sc = scale_problem(prob, ruiz_iters=st.ruiz_iters, pc_alpha=st.pc_alpha,
                       pock_chambolle=st.pock_chambolle,
                       bound_objective=st.bound_objective, enabled=st.scaling,
                       cone_mode=st.cone_scaling)
    q = QOp(sc.P, sc.R, sc.D, prob.n)
    # rescaled-cone mode: a cone block of the scaled problem is S_j K_j
    # (S_x / nu_b differs from S_x by a positive scalar, which leaves a cone
    # unchanged)
    proj = Projector(prob.cones, prob.n, sc.xlo, sc.xhi, kappa=sc.Sx / sc.nu_b,
                     cone_scale=sc.Sx if st.cone_scaling == "rescaled" else None)
    euclid_blocks = proj.const_blocks(q.diag)
    a_norm = st.a_norm if st.a_norm > 0 else power_norm(sc.A, st.power_iters)
    if not a_norm > 0:       # A = 0 or no rows: any step size keeps tau sigma ||A||^2 < 1
        a_norm = 1.0
    eta = 0.998 / a_norm
    nb, nc = float(np.linalg.norm(sc.b)), float(np.linalg.norm(sc.c))
    if st.omega0 > 0:
        om = st.omega0
    elif nb > 1e-10 and nc > 1e-10:
        om = nc / nb
    else:
        om = 1.0
    kproj = Projector(prob.cones, prob.n, prob.x_lo, prob.x_hi)
    return Setup(prob=prob, st=st, sc=sc, q=q, proj=proj, euclid_blocks=euclid_blocks,
                 a_norm=a_norm, eta=eta, omega0=om, kproj=kproj)


# ----------------------------------------------------------------------------
# proximal step
# ----------------------------------------------------------------------------
def prox(S: Setup, v, x, tau, eps_in):
    """Returns (p, inner_steps, last_step_norm)."""
    sc, q, st = S.sc, S.q, S.st
    if q.is_diag:
        mvec = 1.0 + tau * q.diag                       # eq. diagonal-q-metric
        xt = (v - tau * sc.c) / mvec
        return S.proj.project(xt, mvec, S.euclid_blocks), 0, 0.0

    def grad(u):                                        # eq. bb-inner-gradient
        return q(u) + sc.c + (u - v) / tau

    jac = st.inner == "jacobi"
    if jac:
        d = q.diag + 1.0 / tau                          # eq. jacobi-inner-metric
        eu = S.euclid_blocks
        alpha0 = 1.0
    else:
        d = np.ones(S.prob.n)
        eu = np.ones(len(S.prob.cones), dtype=bool)
        alpha0 = 1.0 / float(np.max(q.diag + 1.0 / tau))
    fixed = st.fixed_inner
    jmax = fixed if fixed > 0 else st.j_max
    up = x
    gp = grad(up)
    u = S.proj.project(up - alpha0 * gp / d, d, eu)
    j = 1
    last = float(np.linalg.norm(u - up))
    if fixed <= 0 and last <= eps_in:
        return u, j, last
    while j < jmax:
        gc = grad(u)
        s = u - up
        dg = gc - gp
        den = float(s @ dg)
        alpha = float(s @ (d * s)) / den if den > 0 else 1.0   # eq. jacobi-bb-step
        un = S.proj.project(u - alpha * gc / d, d, eu)
        j += 1
        delta = un - u
        up, gp, u = u, gc, un
        last = float(np.linalg.norm(delta))
        if fixed <= 0 and last <= eps_in:                # eq. current-inner-step-stop
            break
    return u, j, last


def pdhg_step(S: Setup, x, y, tau, sigma, eps_in):
    """One evaluation of the PDHG operator T(x, y) -> (w_x, w_y)."""
    sc = S.sc
    v = x + tau * (sc.A.T @ y)
    wx, nin, _ = prox(S, v, x, tau, eps_in)
    ax = sc.A @ (2.0 * wx - x)
    if sc.lo is None:
        wy = y + sigma * (sc.b - ax)
    else:
        q = ax - y / sigma
        wy = sigma * (np.minimum(np.maximum(q, sc.lo), sc.hi) - q)
        eq = sc.lo == sc.hi
        wy[eq] = y[eq] + sigma * (sc.lo[eq] - ax[eq])
    return wx, wy, nin


# ----------------------------------------------------------------------------
# solver
# ----------------------------------------------------------------------------
@dataclass
class Result:
    status: str
    iterations: int
    inner_iterations: int
    restarts: int
    x: np.ndarray
    y: np.ndarray
    kkt: dict
    solve_s: float
    trace: list = field(default_factory=list)
    omega: float = 0.0
    a_norm: float = 0.0


def solve(prob, st: Settings = None, x0=None, y0=None, S: Setup = None):
    st = st or Settings()
    if S is None:
        S = setup(prob, st)
    if st.scheme == "avg":
        return _solve_avg(S, x0, y0)
    sc = S.sc
    t0 = time.perf_counter()
    n, m = prob.n, prob.m
    x = S.proj.project(sc.scale_x(x0) if x0 is not None else np.zeros(n))
    y = sc.scale_y(y0) if y0 is not None else np.zeros(m)
    ax, ay = x.copy(), y.copy()
    k = 0
    ktot = 0
    inner_tot = 0
    restarts = 0
    eps_in = st.eps_in0
    omega = S.omega0
    pid_i = 0.0
    e_prev = 0.0
    E0 = Eprev = 0.0
    eta = S.eta
    rho = st.rho
    trace = []
    kkt = None
    status = "MAX_ITER"
    wx, wy = x, y
    while ktot < st.max_iter:
        tau = eta / omega
        sigma = eta * omega
        wx, wy, nin = pdhg_step(S, x, y, tau, sigma, eps_in)
        inner_tot += nin
        ktot += 1
        restart = False
        check = (k == 0) or (ktot % st.check_every == 0) or (ktot >= st.max_iter)
        E = None
        if check:
            dx = x - wx
            dy = y - wy
            E2 = omega * float(dx @ dx) + float(dy @ dy) / omega \
                + 2.0 * eta * float((sc.A @ dx) @ dy)
            E = math.sqrt(max(E2, 0.0))
            if k == 0:
                E0 = E
            else:
                restart = (E <= st.beta_s * E0) or \
                          (E <= st.beta_n * E0 and E > Eprev) or \
                          (k + 1 >= st.beta_a * ktot)
            Eprev = E
            kkt = kkt_residuals(prob, sc.unscale_x(wx), sc.unscale_y(wy), S.kproj)
        if len(trace) < st.trace_iters:
            trace.append(dict(x=x.copy(), y=y.copy(), wx=wx.copy(), wy=wy.copy(),
                              tau=tau, sigma=sigma, omega=omega, inner=nin,
                              eps_in=eps_in, k=k, check=check, E=E, restart=restart))
        if check and max(kkt["rel_primal"], kkt["rel_dual"], kkt["rel_gap"]) <= st.tol:
            status = "OPTIMAL"
            break
        if time.perf_counter() - t0 > st.time_limit:
            status = "TIME_LIMIT"
            break
        if restart:
            ddx = float(np.linalg.norm(wx - ax))
            ddy = float(np.linalg.norm(wy - ay))
            if ddx > 1e-12 and ddy > 1e-12:              # eq. pid-error, pid-weight
                e = math.log(ddy / (omega * ddx))
                pid_i = st.pid_beta_i * pid_i + e
                omega = math.exp(math.log(omega) + st.pid_kp * e + st.pid_ki * pid_i
                                 + st.pid_kd * (e - e_prev))
                e_prev = e
            x, y = wx.copy(), wy.copy()
            ax, ay = wx.copy(), wy.copy()
            k = 0
            restarts += 1
        else:                                            # eq. rh-update
            c1 = (k + 1.0) / (k + 2.0)
            c3 = 1.0 / (k + 2.0)
            xn = c1 * (2.0 * rho * wx + (1.0 - 2.0 * rho) * x) + c3 * ax
            yn = c1 * (2.0 * rho * wy + (1.0 - 2.0 * rho) * y) + c3 * ay
            eps_in = min(eps_in, max(st.gamma_in * float(np.linalg.norm(xn - x)) / tau,
                                     st.eps_min))        # eq. monotone-primal-inner-tol
            x, y = xn, yn
            k += 1
    if kkt is None or status == "MAX_ITER":
        kkt = kkt_residuals(prob, sc.unscale_x(wx), sc.unscale_y(wy), S.kproj)
    return Result(status=status, iterations=ktot, inner_iterations=inner_tot,
                  restarts=restarts, x=sc.unscale_x(wx), y=sc.unscale_y(wy), kkt=kkt,
                  solve_s=time.perf_counter() - t0, trace=trace, omega=omega,
                  a_norm=S.a_norm)


def _solve_avg(S: Setup, x0, y0):
    """Alg. 1: fixed tau, sigma; epochs of T steps; restart from the Cesaro
    average (eq. theory-epoch-average); termination tested on the epoch
    average at each restart.  The inner tolerance follows the same adaptive
    rule, driven by the movement of consecutive PDHG iterates."""
    st, sc, prob = S.st, S.sc, S.prob
    t0 = time.perf_counter()
    x = S.proj.project(sc.scale_x(x0) if x0 is not None else np.zeros(prob.n))
    y = sc.scale_y(y0) if y0 is not None else np.zeros(prob.m)
    tau = S.eta / S.omega0
    sigma = S.eta * S.omega0
    eps_in = st.eps_in0
    ktot = inner_tot = restarts = 0
    trace = []
    status = "MAX_ITER"
    xb, yb = x.copy(), y.copy()
    kkt = None
    while ktot < st.max_iter:
        xb = np.zeros_like(x)
        yb = np.zeros_like(y)
        for k in range(st.avg_epoch):
            wx, wy, nin = pdhg_step(S, x, y, tau, sigma, eps_in)
            inner_tot += nin
            ktot += 1
            if len(trace) < st.trace_iters:
                end = k + 1 == st.avg_epoch or ktot >= st.max_iter   # restart and check follow
                trace.append(dict(x=x.copy(), y=y.copy(), wx=wx.copy(), wy=wy.copy(),
                                  tau=tau, sigma=sigma, omega=S.omega0, inner=nin,
                                  eps_in=eps_in, k=k, check=end, restart=end, E=None))
            eps_in = min(eps_in, max(st.gamma_in * float(np.linalg.norm(wx - x)) / tau,
                                     st.eps_min))
            xb = (k / (k + 1.0)) * xb + wx / (k + 1.0)
            yb = (k / (k + 1.0)) * yb + wy / (k + 1.0)
            x, y = wx, wy
            if ktot >= st.max_iter:
                break
        x, y = xb.copy(), yb.copy()
        restarts += 1
        kkt = kkt_residuals(prob, sc.unscale_x(xb), sc.unscale_y(yb), S.kproj)
        if max(kkt["rel_primal"], kkt["rel_dual"], kkt["rel_gap"]) <= st.tol:
            status = "OPTIMAL"
            break
        if time.perf_counter() - t0 > st.time_limit:
            status = "TIME_LIMIT"
            break
    return Result(status=status, iterations=ktot, inner_iterations=inner_tot,
                  restarts=restarts, x=sc.unscale_x(xb), y=sc.unscale_y(yb), kkt=kkt,
                  solve_s=time.perf_counter() - t0, trace=trace, omega=S.omega0,
                  a_norm=S.a_norm)
