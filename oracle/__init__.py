"""Plain, slow FP64 CPU oracle of the restarted PDHG method for conic convex
QP (PDHCG-CQP, arXiv 2608.09159).

TEST INFRASTRUCTURE ONLY.  This package exists to check the HIP library; it
is imported by the tests, by the smoke check and by the benchmark's CPU
baseline leg, and by nothing else.  It shares no code with the library: it
reads ``instances.Problem`` data and computes everything itself in NumPy /
SciPy float64, following the paper's text step by step.

Modules
-------
cones    Euclidean and diagonal-metric projections onto the cones of
         Appendix C, membership and dual-cone tests.
scaling  Ruiz / Pock-Chambolle / cone-preserving / bound-objective rescaling
         (Section "Problem Rescaling").
pdhg     power iteration, proximal step (diagonal-Q metric projection and
         Jacobi projected Barzilai-Borwein), reflected-Halpern epochs,
         adaptive restart, PID primal weight, averaged epochs (Alg. 1),
         relative KKT residuals.

Parity status of each part is listed at the top of each module.
"""
from . import cones, scaling, pdhg  # noqa: F401
