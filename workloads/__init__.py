"""Seeded synthetic inputs shared by the oracle, the tests and the benchmark.

This module builds problems, nothing else: counter-based random numbers,
the sparse SPD operators that stand in for the paper's PDE/FE matrices,
exact solutions and right-hand sides.  It holds none of the preconditioner's
or the solver's arithmetic, so both the FP64 oracle and the GPU path can take
their inputs from here without sharing any code of the method.
"""

from .rng import splitmix64, uniform, normal, exponential
from .grids import (
    stencil5_csr,
    stencil7_csr,
    stencil7_nnz,
    stencil7_bounds,
    stencil5_eigenvalues,
    harmonic27_kappa,
    harmonic27_csr,
    csr_diagonal,
    rhs_from_solution,
)
from .elasticity import q1_reference_stiffness, elasticity_q1_moduli, elasticity_q1_csr
from .serving import KINDS, serving_trace

__all__ = [
    "splitmix64",
    "uniform",
    "normal",
    "exponential",
    "stencil5_csr",
    "stencil7_csr",
    "stencil7_nnz",
    "stencil7_bounds",
    "stencil5_eigenvalues",
    "harmonic27_kappa",
    "harmonic27_csr",
    "csr_diagonal",
    "rhs_from_solution",
    "q1_reference_stiffness",
    "elasticity_q1_moduli",
    "elasticity_q1_csr",
    "KINDS",
    "serving_trace",
]
