"""Plain container for a conic convex QP

    minimise 1/2 <x, Q x> + <c, x>   subject to  A x = b,  x in K,

the problem statement of the paper's introduction (eq. cqp), with the
structured quadratic Q = P + R^T D R of its implementation section and K a
Cartesian product of blocks from the cone list of the same section: free,
nonnegative, second-order (v, t), rotated second-order (v, s, t),
exponential (r, s, t) and 3-D power (x, y, z) with exponent alpha.

The implementation form of the same section (eq. solver-input) is covered
by the optional fields: row bounds row_lo <= A x <= row_hi (when given they
replace A x = b; infinite entries are absent bounds, equal entries
equalities) and box blocks x_i in [x_lo_i, x_hi_i] (blocks of kind "box";
x_lo / x_hi have length n and are read at the box coordinates only).  Blocks
of kind "exp1" are exponential-cone blocks (z, s, t) with the middle
coordinate fixed at one, {(z, 1, t): e^z <= t}, as in the Fisher experiment.

The container holds data only; it performs no solver arithmetic.
"""
from __future__ import annotations

from dataclasses import dataclass, field
from typing import List, Optional, Tuple

import numpy as np
import scipy.sparse as sp

CONE_TYPES = ("free", "nonneg", "soc", "rsoc", "exp", "pow", "box", "exp1")


@dataclass
class Problem:
    n: int
    m: int
    A: sp.csr_matrix                   # m x n
    b: np.ndarray                      # m
    c: np.ndarray                      # n
    cones: List[Tuple[str, int, int, float]]   # (type, start, dim, alpha)
    P: Optional[sp.csr_matrix] = None  # n x n symmetric, full storage
    R: Optional[np.ndarray] = None     # r x n, row-major
    D: Optional[np.ndarray] = None     # r x r symmetric
    name: str = ""
    meta: dict = field(default_factory=dict)
    row_lo: Optional[np.ndarray] = None   # m, with row_hi: row_lo <= A x <= row_hi
    row_hi: Optional[np.ndarray] = None
    x_lo: Optional[np.ndarray] = None     # n, bounds of the box blocks
    x_hi: Optional[np.ndarray] = None

    def __post_init__(self):
        self.A = sp.csr_matrix(self.A, dtype=np.float64)
        self.A.sort_indices()
        self.b = np.ascontiguousarray(self.b, dtype=np.float64)
        self.c = np.ascontiguousarray(self.c, dtype=np.float64)
        if self.P is not None:
            self.P = sp.csr_matrix(self.P, dtype=np.float64)
            self.P.sort_indices()
        for f in ("row_lo", "row_hi", "x_lo", "x_hi"):
            v = getattr(self, f)
            if v is not None:
                setattr(self, f, np.ascontiguousarray(v, dtype=np.float64))
        if self.R is not None:
            self.R = np.ascontiguousarray(self.R, dtype=np.float64)
            if self.D is None:
                self.D = np.eye(self.R.shape[0])
            self.D = np.ascontiguousarray(self.D, dtype=np.float64)

    @property
    def rank_r(self) -> int:
        return 0 if self.R is None else int(self.R.shape[0])

    @property
    def has_row_bounds(self) -> bool:
        return self.row_lo is not None
