"""Counter-based SplitMix64 start vector (oracle side, test infrastructure).

SplitMix64 is the published generator of Steele, Lea and Flood (OOPSLA 2014) in
the form popularised by Vigna: state advance by the golden-ratio increment
0x9E3779B97F4A7C15, then the 64-bit finaliser
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
  z = (z ^ (z >> 27)) * 0x94D049BB133111EB
  z =  z ^ (z >> 31).
Element k of the stream with seed s uses the state s + (k + 1) * increment, so
any element can be computed independently.  The top 53 bits give a double in
[0, 1), mapped to [-1, 1).  The paper does not fix the Lanczos start vector;
this is the reading used on both sides.
"""
from __future__ import annotations

import numpy as np

_GOLDEN = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB
_MASK = (1 << 64) - 1


def splitmix64_scalar(seed, k):
    z = (seed + (k + 1) * _GOLDEN) & _MASK
    z = ((z ^ (z >> 30)) * _M1) & _MASK
    z = ((z ^ (z >> 27)) * _M2) & _MASK
    return z ^ (z >> 31)


def splitmix64(seed, n):
    """First n outputs of the stream as uint64 (vectorised, wrap-around arithmetic)."""
    with np.errstate(over="ignore"):
        k = np.arange(1, n + 1, dtype=np.uint64)
        z = np.uint64(seed & _MASK) + k * np.uint64(_GOLDEN)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(_M1)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(_M2)
        z = z ^ (z >> np.uint64(31))
    return z


def uniform_pm1(seed, n):
    """Doubles in [-1, 1): 2 * (z >> 11) * 2**-53 - 1."""
    z = splitmix64(seed, n)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53) * 2.0 - 1.0


def start_vector(seed, n):
    v = uniform_pm1(seed, n)
    return v / np.linalg.norm(v)
