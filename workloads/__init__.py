"""Seeded synthetic workloads for band-Lanczos block MINRES.

This package holds only input construction (sparse matrices, right-hand
sides).  It contains none of the solver's arithmetic, so that the CPU oracle,
the tests, the benchmark and the GPU library can all draw the same inputs
without sharing any solver code.
"""
from .gen import (  # noqa: F401
    Csr,
    laplacian,
    random_symmetric,
    rhs_normal,
    rhs_stress,
    rhs_e1_ae1,
    rhs_near_copy,
    permuted,
    redblack_order,
    rhs_near_e1_ae1,
    diag_positions,
    with_diagonal_shift,
    ThetaProblem,
    theta_problem,
    WORKLOADS,
    workload,
)
