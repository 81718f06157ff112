"""Counter-based SplitMix64 random numbers (Steele, Lea & Flood, OOPSLA 2014).

Element i of a stream with seed s is mix(s + (i + 1) * 0x9E3779B97F4A7C15), where
mix is the SplitMix64 finaliser.  Because every element is a pure function of
(seed, index), streams are reproducible, can be generated in any order and in
vectorised form, and a C implementation of the same definition produces the
same bits.
"""

import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, n: int, offset: int = 0) -> np.ndarray:
    """Return elements offset .. offset+n-1 of the SplitMix64 stream of `seed`."""
    i = np.arange(offset + 1, offset + n + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + i * _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def _unit(seed: int, n: int, offset: int = 0) -> np.ndarray:
    """Doubles in [0, 1): the top 53 bits of each SplitMix64 word times 2^-53."""
    return (splitmix64(seed, n, offset) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def uniform(seed: int, n: int, lo: float = 0.0, hi: float = 1.0) -> np.ndarray:
    """n i.i.d. U[lo, hi) doubles from the stream of `seed`."""
    return lo + (hi - lo) * _unit(seed, n)


def normal(seed: int, n: int) -> np.ndarray:
    """n i.i.d. N(0, 1) doubles by the Box–Muller transform.

    Element i uses stream words 2i and 2i+1 of `seed`."""
    u = _unit(seed, 2 * n)
    u1 = 1.0 - u[0::2]  # (0, 1], so the logarithm is finite
    u2 = u[1::2]
    return np.sqrt(-2.0 * np.log(u1)) * np.cos(2.0 * np.pi * u2)


def exponential(seed: int, n: int, rate: float) -> np.ndarray:
    """n i.i.d. exponential gaps with the given rate (inverse-CDF method)."""
    return -np.log(1.0 - _unit(seed, n)) / rate
