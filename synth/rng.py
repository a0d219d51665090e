"""SplitMix64 counter streams (Steele, Lea, Flood 2014), vectorised with numpy.

Word i (i = 0, 1, ...) of the stream keyed by `seed` is
    z = seed + (i + 1) * 0x9E3779B97F4A7C15   (mod 2^64)
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9
    z = (z ^ (z >> 27)) * 0x94D049BB133111EB
    z ^ (z >> 31)
so any slice of the stream can be produced without generating its prefix.
"""
import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed, start, count):
    """Words [start, start+count) of the SplitMix64 stream keyed by `seed` (uint64 array)."""
    i = np.arange(start + 1, start + 1 + count, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + i * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def stream_seed(seed, tag):
    """Derive an independent stream key from (seed, tag) by one SplitMix64 step."""
    return int(splitmix64((seed ^ (tag * 0xD1B54A32D192ED03)) & 0xFFFFFFFFFFFFFFFF, 0, 1)[0])


def uniforms(seed, start, count):
    """Uniform doubles in (0, 1): the top 53 bits of each word, offset by half an ulp."""
    w = splitmix64(seed, start, count)
    return ((w >> np.uint64(11)).astype(np.float64) + 0.5) * (2.0 ** -53)


def normals(seed, start, count):
    """Standard normal pairs by the Box-Muller transform: `count` pairs from 2*count uniforms.

    Returns two float64 arrays (a, b) of length `count`.
    """
    u = uniforms(seed, 2 * start, 2 * count)
    u1, u2 = u[0::2], u[1::2]
    r = np.sqrt(-2.0 * np.log(u1))
    t = 2.0 * np.pi * u2
    return r * np.cos(t), r * np.sin(t)
