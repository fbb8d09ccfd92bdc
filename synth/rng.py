"""Counter-based random numbers for the synthetic inputs.

Every random draw is a pure function of (seed, tag, spin, k1, k2, element index),
so any block of any tensor can be regenerated on its own, in any order, on the
host or elsewhere.  The mixer is SplitMix64 (Steele, Lea & Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014): additive Weyl step
0x9E3779B97F4A7C15 followed by the xor-shift-multiply finaliser.

Uniforms take the top 53 bits of a 64-bit output; normals use the Box-Muller
transform on two uniforms taken from consecutive counters.
"""
from __future__ import annotations

import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)

# tensor tags
TAG_F = 1
TAG_S = 2
TAG_V = 3
TAG_DRAW = 4
TAG_P = 5
TAG_G = 6


def _mix(z: np.ndarray) -> np.ndarray:
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        return z ^ (z >> np.uint64(31))


def splitmix64(x) -> np.ndarray:
    """SplitMix64 output for state x (one Weyl step, then the finaliser)."""
    x = np.asarray(x, dtype=np.uint64)
    with np.errstate(over="ignore"):
        return _mix(x + _GOLDEN)


def stream_key(seed: int, tag: int, *fields: int) -> np.uint64:
    """Fold (seed, tag, fields...) into one 64-bit stream key."""
    h = splitmix64(np.uint64(seed & 0xFFFFFFFFFFFFFFFF))
    for f in (tag,) + tuple(fields):
        h = splitmix64(h ^ np.uint64(int(f) & 0xFFFFFFFFFFFFFFFF))
    return np.uint64(h)


def uniforms(key: np.uint64, start: int, count: int) -> np.ndarray:
    """count uniforms in [0, 1) from counters start .. start+count-1 of stream key."""
    idx = np.arange(start, start + count, dtype=np.uint64)
    with np.errstate(over="ignore"):
        u = splitmix64(idx + key * np.uint64(1))
    return (u >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)


def normals(key: np.uint64, count: int) -> np.ndarray:
    """count standard normals (Box-Muller, cosine branch) from stream key."""
    u = uniforms(key, 0, 2 * count).reshape(count, 2)
    r = np.sqrt(-2.0 * np.log1p(-u[:, 0]))
    return r * np.cos(2.0 * np.pi * u[:, 1])


def complex_normals(key: np.uint64, shape) -> np.ndarray:
    """Complex Gaussian with Re and Im each N(0, 1/2), so E|z|^2 = 1."""
    n = int(np.prod(shape))
    g = normals(key, 2 * n).reshape(n, 2)
    z = (g[:, 0] + 1j * g[:, 1]) * np.sqrt(0.5)
    return z.reshape(shape)
