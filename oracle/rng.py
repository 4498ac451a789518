"""SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014), used as a counter-based generator.

Output j of stream `seed` is the SplitMix64 mixing function applied to
seed + (j + 1) * 0x9E3779B97F4A7C15 (mod 2^64).  A uniform double on [-1, 1)
is formed from the top 53 bits: ((z >> 11) * 2^-53) * 2 - 1, which is exact
in binary64, so any faithful implementation reproduces these values bit for
bit.  The paper does not say how the power iteration is started; this start
vector is a choice of this project.
"""
import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, count: int) -> np.ndarray:
    """The first `count` outputs of stream `seed` as uint64."""
    with np.errstate(over="ignore"):
        j = np.arange(1, count + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + j * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform_pm1(seed: int, count: int) -> np.ndarray:
    z = splitmix64(seed, count)
    u = (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    return u * 2.0 - 1.0
