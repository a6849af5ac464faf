"""Seeded synthetic inputs shared by the oracle, the tests and the bench.

This package only draws random numbers.  It holds none of the search
method's arithmetic (no distances, no ordering, no pruning), so the CPU
oracle and the GPU path can both consume its output without sharing any
method code.
"""
from .gen import (  # noqa: F401
    Mixture,
    isotropic_mixture,
    skewed_mixture,
    anisotropic_unit_mixture,
    integer_grid,
    standard_normal,
    KERNEL_STUDY_N,
    KERNEL_STUDY_D,
    KERNEL_STUDY_BLOCKS,
    workload,
    WORKLOADS,
)
