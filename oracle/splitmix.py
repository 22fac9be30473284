"""SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014; the 64-bit finaliser as published by Vigna).

The solver's pseudo-random choices (MIS priorities, power-iteration and
Lanczos start vectors) are all ``splitmix64(x)`` of a counter ``x``: one
generator step from state ``x``:

    z = x + 0x9E3779B97F4A7C15
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB
    return z ^ (z >> 31)          (all arithmetic modulo 2^64)
"""
import numpy as np

_GAMMA = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(x):
    """Vectorised SplitMix64 output for state(s) ``x`` (uint64 array)."""
    z = np.asarray(x, dtype=np.uint64).copy()
    with np.errstate(over="ignore"):
        z = z + _GAMMA
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def unit_centered(x):
    """splitmix64(x) / 2^64 - 1/2 as FP64 (used for start vectors)."""
    return splitmix64(x).astype(np.float64) / 18446744073709551616.0 - 0.5
