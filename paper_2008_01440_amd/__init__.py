"""Newton-Chebyshev polynomial-preconditioned CG on AMD MI355X.

Thin Python binding of the C ABI in include/pcheb.h (libpcheb.so, built from
csrc/ by build.py).  The functions keep the C names; they only marshal
arguments.  Device memory and streams come from PyTorch: vectors are float64
CUDA tensors and the default stream is torch's current stream.  Every
computation runs in the HIP library; importing this package does not need a
GPU, but calling it without the built library raises.
"""

from ._abi import (
    PCG_FLEXIBLE,
    PCG_NO_GRAPH,
    PCG_REFRESH,
    PCG_TIME_KERNELS,
    PCG_X0_GIVEN,
    PchebError,
    Group,
    Handle,
    Operator,
    STATUS,
    Server,
    TorchCachingAllocator,
    library_path,
    load_library,
    pcg_solve,
    pcg_solve_group,
    pcheb_apply,
    pcheb_destroy,
    pcheb_estimate_bounds,
    pcheb_estimate_bounds_noalloc,
    pcheb_estimate_bounds_pdacg,
    pcheb_fill_uniform,
    pcheb_footprint_bytes,
    pcheb_group_apply,
    pcheb_group_create,
    pcheb_group_destroy,
    pcheb_last_error,
    pcheb_matvec,
    pcheb_set_allocator,
    pcheb_setup,
)

__all__ = [
    "PCG_FLEXIBLE",
    "PCG_NO_GRAPH",
    "PCG_REFRESH",
    "PCG_TIME_KERNELS",
    "PCG_X0_GIVEN",
    "PchebError",
    "Group",
    "Handle",
    "Operator",
    "STATUS",
    "Server",
    "TorchCachingAllocator",
    "library_path",
    "load_library",
    "pcg_solve",
    "pcg_solve_group",
    "pcheb_apply",
    "pcheb_destroy",
    "pcheb_estimate_bounds",
    "pcheb_estimate_bounds_noalloc",
    "pcheb_estimate_bounds_pdacg",
    "pcheb_fill_uniform",
    "pcheb_footprint_bytes",
    "pcheb_group_apply",
    "pcheb_group_create",
    "pcheb_group_destroy",
    "pcheb_last_error",
    "pcheb_matvec",
    "pcheb_set_allocator",
    "pcheb_setup",
]
