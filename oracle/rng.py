"""SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014), the counter-based generator behind the PMIS weights
and the seeded start vectors.

Output k of the stream seeded with s is mix(s + (k+1) * GAMMA), with
mix(z) = z3 where
    z1 = (z  ^ (z  >> 30)) * 0xBF58476D1CE4E5B9
    z2 = (z1 ^ (z1 >> 27)) * 0x94D049BB133111EB
    z3 =  z2 ^ (z2 >> 31)
and all arithmetic modulo 2^64.
"""
import numpy as np

GAMMA = 0x9E3779B97F4A7C15
M64 = (1 << 64) - 1


def splitmix64_scalar(seed: int, k: int) -> int:
    """Plain-integer definition, one output at a time."""
    z = (seed + (k + 1) * GAMMA) & M64
    z = ((z ^ (z >> 30)) * 0xBF58476D1CE4E5B9) & M64
    z = ((z ^ (z >> 27)) * 0x94D049BB133111EB) & M64
    return z ^ (z >> 31)


def splitmix64(seed: int, k):
    """Vectorised form (numpy uint64 arithmetic wraps modulo 2^64)."""
    with np.errstate(over="ignore"):
        k = np.asarray(k, dtype=np.uint64)
        z = np.uint64(seed & M64) + (k + np.uint64(1)) * np.uint64(GAMMA)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        return z ^ (z >> np.uint64(31))


def pmis_hash40(seed: int, level: int, idx):
    """40-bit PMIS weight of point idx on a level: the top 40 bits of output
    k = level * 2^40 + idx of the stream seeded with ``seed``."""
    k = (np.uint64(level) << np.uint64(40)) | np.asarray(idx, dtype=np.uint64)
    return splitmix64(seed, k) >> np.uint64(24)


def uniform_pm1(seed: int, stream: int, n: int):
    """n doubles in [-1, 1): 53 top bits of outputs k = stream*2^40 + i."""
    k = (np.uint64(stream) << np.uint64(40)) | np.arange(n, dtype=np.uint64)
    u = (splitmix64(seed, k) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return 2.0 * u - 1.0
