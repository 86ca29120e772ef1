"""Problem rescaling of the paper's Section "Problem Rescaling"
(eq. problem-rescaling, eq. cone-scaling-candidates,
eq. cone-preserving-scaling) with the defaults of Table practical-defaults:
10 Ruiz passes, one Pock-Chambolle pass with alpha = 1, cone-preserving block
scaling, bound-objective rescaling enabled.

TEST INFRASTRUCTURE ONLY (see the package docstring).

Readings where the paper is silent:
* rows use the same coordinatewise rule as columns: Ruiz row factor
  sqrt(max_i |A_li|), Pock-Chambolle row factor sqrt(sum_i |A_li|^alpha)
  (the Pock-Chambolle pairing of exponents alpha / 2 - alpha);
* a zero row or column gets the factor 1;
* the Pock-Chambolle sums run over the stored nonzeros of A~, so an exponent
  of zero (alpha = 0 for rows, alpha = 2 for columns) counts them;
* order: Ruiz passes, then Pock-Chambolle, then bound-objective;
* bound-objective constants: nu_b = ||b~|| + 1, nu_c = ||c~|| + 1,
  b^ = b~/nu_b, c^ = c~/nu_c and Q^ = (nu_b/nu_c) Q~, which keeps the
  objective of x^ = x~/nu_b equal to the scaled objective divided by
  nu_b nu_c;
* the candidates of eq. cone-scaling-candidates involve A only.

With x~ = S_x x, A~ = S_y A S_x^-1, Q~ = S_x^-1 Q S_x^-1, c~ = S_x^-1 c,
b~ = S_y b; an original solution is recovered as x = nu_b S_x^-1 x^,
y = nu_c S_y y^.

Implementation form (eq. solver-input): row bounds scale with their rows,
l~ = S_y l, u~ = S_y u, box bounds with their coordinates, l^x~ = S_x l^x,
and both are divided by nu_b with b; box coordinates take coordinatewise
factors like R+ and free ones.  With row bounds, nu_b is built from the
combined bound of each row (its value for an equality, else the larger
finite endpoint in magnitude, 0 when neither is finite): "the bound data" of
the bound-objective rescaling.

Rescaled-cone mode (cone_mode="rescaled"): the candidates of
eq. cone-scaling-candidates stay coordinatewise on SOC, RSOC, EXP and POW
blocks too, so a block becomes S_j K_j with S_j the block's slice of S_x
(projected through eq. scaling-induced-metric, see cones.Projector).
Reading: fixed-middle exp1 blocks keep one common factor in both modes, since
their set is not a cone and S_j X is not a scaled copy of X.

Pins: hand-derived worked examples of one and two Ruiz passes, of a
Pock-Chambolle pass with alpha = 1 and alpha = 2, of Ruiz followed by
Pock-Chambolle and of the bound-objective constants
(tests/test_oracle_pins.py); unscale(scale(.)) is the identity, the unscaled
KKT residuals of a solve do not depend on the scaling, and after the Ruiz
passes every row and column infinity-norm is close to one
(tests/test_oracle_solver.py).
"""
from __future__ import annotations

from dataclasses import dataclass
from typing import Optional

import numpy as np
import scipy.sparse as sp


@dataclass
class Scaled:
    A: sp.csr_matrix
    b: np.ndarray
    c: np.ndarray
    P: Optional[sp.csr_matrix]
    R: Optional[np.ndarray]
    D: Optional[np.ndarray]
    Sx: np.ndarray
    Sy: np.ndarray
    nu_b: float
    nu_c: float
    lo: Optional[np.ndarray] = None    # scaled row bounds (None: A x = b)
    hi: Optional[np.ndarray] = None
    xlo: Optional[np.ndarray] = None   # scaled box bounds (length n)
    xhi: Optional[np.ndarray] = None

    def unscale_x(self, xh):
        return self.nu_b * xh / self.Sx

    def unscale_y(self, yh):
        return self.nu_c * self.Sy * yh

    def scale_x(self, x):
        return self.Sx * x / self.nu_b

    def scale_y(self, y):
        return y / (self.Sy * self.nu_c)


def _cone_blocks(cones, cone_mode="block"):
    """Blocks whose coordinates share one factor: every non-elementwise block
    in the cone-preserving mode, only the exp1 blocks in the rescaled-cone
    mode (one common factor keeps the set's shape, so a scaled exp1 block is
    kappa X with kappa = S_x / nu_b)."""
    if cone_mode == "rescaled":
        return [(st, d) for kind, st, d, al in cones if kind == "exp1"]
    return [(st, d) for kind, st, d, al in cones if kind not in ("free", "nonneg", "box")]


def combined_bounds(lo, hi):
    """Per row: the value of an equality, else the larger finite endpoint in
    magnitude (0 when neither endpoint is finite)."""
    flo = np.where(np.isfinite(lo), np.abs(lo), 0.0)
    fhi = np.where(np.isfinite(hi), np.abs(hi), 0.0)
    return np.where(lo == hi, lo, np.maximum(flo, fhi))


def _apply(A, row, col):
    return sp.diags(1.0 / row) @ A @ sp.diags(1.0 / col)


def _abs_power_sums(A, e):
    """(row sums, column sums) of |A_li|^e over the nonzeros of A."""
    B = abs(A).tocsr()
    B.eliminate_zeros()
    B.data = B.data ** e
    return (np.asarray(B.sum(axis=1)).ravel(), np.asarray(B.sum(axis=0)).ravel())


def scale_problem(prob, ruiz_iters=10, pc_alpha=1.0, pock_chambolle=True,
                  bound_objective=True, enabled=True, cone_mode="block"):
    if cone_mode not in ("block", "rescaled"):
        raise ValueError(cone_mode)
    A = sp.csr_matrix(prob.A, dtype=float, copy=True)
    m, n = A.shape
    Sx = np.ones(n)
    Sy = np.ones(m)
    blocks = _cone_blocks(prob.cones, cone_mode)
    if enabled and m > 0:        # no rows: every factor is 1
        for _ in range(ruiz_iters):
            absA = abs(A)
            col = np.sqrt(np.asarray(absA.max(axis=0).todense()).ravel())
            row = np.sqrt(np.asarray(absA.max(axis=1).todense()).ravel())
            for st, d in blocks:          # eq. cone-preserving-scaling (Ruiz)
                col[st:st + d] = col[st:st + d].max()
            col[col == 0] = 1.0
            row[row == 0] = 1.0
            A = _apply(A, row, col).tocsr()
            Sy = Sy / row
            Sx = Sx * col
        if pock_chambolle:
            col = np.sqrt(_abs_power_sums(A, 2.0 - pc_alpha)[1])
            row = np.sqrt(_abs_power_sums(A, pc_alpha)[0])
            for st, d in blocks:          # eq. cone-preserving-scaling (PC: RMS)
                col[st:st + d] = np.sqrt(np.mean(col[st:st + d] ** 2))
            col[col == 0] = 1.0
            row[row == 0] = 1.0
            A = _apply(A, row, col).tocsr()
            Sy = Sy / row
            Sx = Sx * col
    c = prob.c / Sx
    b = prob.b * Sy
    lo = hi = xlo = xhi = None
    if prob.row_lo is not None:
        lo = prob.row_lo * Sy
        hi = prob.row_hi * Sy
        b = combined_bounds(lo, hi)
    if prob.x_lo is not None:
        xlo = prob.x_lo * Sx
        xhi = prob.x_hi * Sx
    P = None
    if prob.P is not None:
        P = (sp.diags(1.0 / Sx) @ prob.P @ sp.diags(1.0 / Sx)).tocsr()
    R = None if prob.R is None else prob.R / Sx[None, :]
    D = None if prob.D is None else prob.D.copy()
    nu_b = nu_c = 1.0
    if enabled and bound_objective:
        nu_b = float(np.linalg.norm(b)) + 1.0
        nu_c = float(np.linalg.norm(c)) + 1.0
    b = b / nu_b
    c = c / nu_c
    if lo is not None:
        lo, hi = lo / nu_b, hi / nu_b
    if xlo is not None:
        xlo, xhi = xlo / nu_b, xhi / nu_b
    if P is not None:
        P = (P * (nu_b / nu_c)).tocsr()
    if D is not None:
        D = D * (nu_b / nu_c)
    A.sort_indices()
    return Scaled(A=A, b=b, c=c, P=P, R=R, D=D, Sx=Sx, Sy=Sy, nu_b=nu_b, nu_c=nu_c,
                  lo=lo, hi=hi, xlo=xlo, xhi=xhi)
