"""Seeded synthetic problem generators shared by the tests, the benchmark and
the warm-start data pipeline.

This package only draws random problem data (matrices, vectors, cone
partitions).  It contains none of the solver's arithmetic: no scaling, no
projection, no PDHG step.  Both the CPU oracle (through the tests) and the
HIP library (through the Python binding) consume the same ``Problem``
objects, so neither side depends on the other.
"""
from .problem import Problem, CONE_TYPES
from . import synth

__all__ = ["Problem", "CONE_TYPES", "synth"]
