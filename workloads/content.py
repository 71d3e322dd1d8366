"""Byte content of memory pools: the SplitMix64 stream.

Pool byte ``i`` under seed ``seed`` is byte ``i & 7`` (little-endian) of the
``(i >> 3)``-th output of a SplitMix64 generator whose state starts at
``seed`` (Steele, Lea & Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014): the state advances by the golden gamma
0x9E3779B97F4A7C15 before each output, and an output is the state passed
through the variant-13 finaliser (shift 30, multiply 0xBF58476D1CE4E5B9,
shift 27, multiply 0x94D049BB133111EB, shift 31).  Output ``k`` therefore
depends only on ``seed + (k + 1) * gamma``, which lets any window of a pool
be generated on its own -- the device fill kernel computes the same function
independently.
"""
import numpy as np

GAMMA = np.uint64(0x9E3779B97F4A7C15)
M1 = np.uint64(0xBF58476D1CE4E5B9)
M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, k0: int, count: int) -> np.ndarray:
    """Outputs k0 .. k0+count-1 (0-based) of the stream seeded with ``seed``."""
    k = np.arange(k0, k0 + count, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + (k + np.uint64(1)) * GAMMA
        z = (z ^ (z >> np.uint64(30))) * M1
        z = (z ^ (z >> np.uint64(27))) * M2
        z = z ^ (z >> np.uint64(31))
    return z


def content(seed: int, start: int, length: int) -> np.ndarray:
    """Bytes [start, start+length) of the pool filled under ``seed``."""
    if length <= 0:
        return np.zeros(0, dtype=np.uint8)
    w0 = start >> 3
    w1 = (start + length + 7) >> 3
    words = splitmix64(seed, w0, w1 - w0)
    b = words.astype("<u8").view(np.uint8)
    off = start - (w0 << 3)
    return b[off:off + length].copy()
