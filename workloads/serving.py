"""A seeded request trace for the solve server: Poisson arrivals of solves on
cubic grids of random size with the 7-point Laplacian or the 27-point
harmonic-mean lognormal operator.

Requests with the same (stencil, N) use the same coefficient seed, so they can
share one resident operator; every request has its own right-hand-side seed."""

import numpy as np

from .rng import exponential, splitmix64

KINDS = ("stencil7", "stencil27h")


def serving_trace(n_requests: int = 2000, rate: float = 50.0, seed: int = 3, n_lo: int = 32, n_hi: int = 160):
    """Returns a dict of arrays, one entry per request in arrival order:
    t (arrival time in seconds from 0), N (grid edge), kind (index into KINDS),
    coeff_seed (lognormal field seed, per (kind, N)) and rhs_seed.

    Gaps are exponential with the given rate (stream `seed`); N is uniform on
    [n_lo, n_hi] (stream seed + 1, word modulo the range, bias < 2^-56) and the
    stencil a fair coin (stream seed + 2, top bit)."""
    if n_requests < 0 or not rate > 0 or n_lo < 1 or n_hi < n_lo:
        raise ValueError("need n_requests >= 0, rate > 0 and 1 <= n_lo <= n_hi")
    t = np.cumsum(exponential(seed, n_requests, rate)) if rate != np.inf else np.zeros(n_requests)
    N = n_lo + (splitmix64(seed + 1, n_requests) % np.uint64(n_hi - n_lo + 1)).astype(np.int64)
    kind = (splitmix64(seed + 2, n_requests) >> np.uint64(63)).astype(np.int64)
    coeff_seed = 1_000_000 + 1000 * N + kind
    rhs_seed = 2_000_000 + np.arange(n_requests, dtype=np.int64)
    return {"t": t, "N": N, "kind": kind, "coeff_seed": coeff_seed, "rhs_seed": rhs_seed}
