"""SplitMix64 (Steele, Lea, Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014; finaliser constants as published by Vigna) used as
a counter-based generator: value i is the (i+1)-th output of SplitMix64
started from state ``seed``.  It draws the start vector of the lambda_max
estimate (Sec. 3.1), which the library draws with its own implementation of
the same published generator.
"""
import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed, count):
    """uint64 array: output i = mix(seed + (i+1) * golden) (mod 2^64)."""
    i = np.arange(1, count + 1, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed) + i * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def uniform_pm1(seed, count):
    """Uniform doubles in [-1, 1): 2 * (top 53 bits) * 2^-53 - 1."""
    z = splitmix64(seed, count)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -52) - 1.0
