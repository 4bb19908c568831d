"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This package produces phase-space points (RAMBO + cuts), helicities,
colour-flow labels and the continuous colour / polarization variables.  It
contains none of the matrix-element arithmetic: the oracle and the HIP
library both consume what it writes and neither is imported here.
"""
from .rng import splitmix64_uniform, mix64
from .rambo import (
    SQRT_S_DEFAULT,
    make_events,
    rambo_massless,
    passes_cuts,
    workload,
    mixed_counts,
    mixed_workload,
)
from .continuous import continuous_states

__all__ = [
    "splitmix64_uniform",
    "mix64",
    "SQRT_S_DEFAULT",
    "make_events",
    "rambo_massless",
    "passes_cuts",
    "workload",
    "mixed_counts",
    "mixed_workload",
    "continuous_states",
]
