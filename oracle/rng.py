"""Counter-based random stream (SplitMix64, Steele, Lea & Flood, OOPSLA 2014).

Entry j of stream s for seed t is splitmix64(t * 2^40 + s * 2^24 + j) mapped
to a double in [-0.5, 0.5) from its top 53 bits.  The GPU path implements
the same published generator on its own side; the two never share code.
"""
import numpy as np

_M64 = (1 << 64) - 1


def splitmix64(x: np.ndarray) -> np.ndarray:
    x = (x.astype(np.uint64) + np.uint64(0x9E3779B97F4A7C15))
    z = x
    z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
    return z ^ (z >> np.uint64(31))


def stream(seed: int, s: int, count: int) -> np.ndarray:
    base = (int(seed) << 40) + (int(s) << 24)
    with np.errstate(over="ignore"):
        key = np.uint64(base & _M64) + np.arange(count, dtype=np.uint64)
        z = splitmix64(key)
    return (z >> np.uint64(11)).astype(np.float64) * (2.0 ** -53) - 0.5
