"""FP64 CPU oracle for Newton-Chebyshev preconditioned CG.

TEST INFRASTRUCTURE ONLY: the test suite, the smoke check and the benchmark's
CPU-baseline leg are its only users.  The GPU library never imports it.
``oracle.nc`` is the numpy/scipy oracle; ``oracle.omp`` binds the C/OpenMP one
(nc_omp.c), which computes the same PCG with the rows split over host threads.
"""

from .nc import (
    ChebScalars,
    CountingOperator,
    NCResult,
    NotSPD,
    PCGResult,
    block_jacobi_factor,
    chebyshev_apply,
    chebyshev_scalars,
    cluster_indicator,
    csr,
    dacg_smallest,
    hotelling_step,
    jacobi_scale,
    lanczos_extremes,
    nc_apply_unscaled,
    nc_apply_second_level,
    nc_pcg,
    nc_pcg_second_level,
    newton_apply,
    newton_zetas,
    pcg,
    power_method,
    preconditioned_spectrum,
    second_level_operator,
)

__all__ = [
    "ChebScalars",
    "CountingOperator",
    "NCResult",
    "NotSPD",
    "PCGResult",
    "block_jacobi_factor",
    "chebyshev_apply",
    "chebyshev_scalars",
    "cluster_indicator",
    "csr",
    "dacg_smallest",
    "hotelling_step",
    "jacobi_scale",
    "lanczos_extremes",
    "nc_apply_unscaled",
    "nc_apply_second_level",
    "nc_pcg",
    "nc_pcg_second_level",
    "newton_apply",
    "newton_zetas",
    "pcg",
    "power_method",
    "preconditioned_spectrum",
    "second_level_operator",
]
