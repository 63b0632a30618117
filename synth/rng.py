"""Counter-based random numbers for the synthetic inputs.

Every draw is a pure function of (seed, stream, event, draw), so a sample is
reproducible, independent of batching and of thread count.  The mixing
function is the SplitMix64 finaliser (Steele, Lea, Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014); its 64-bit output x is mapped to
the open interval (0, 1) as ((x >> 11) + 0.5) * 2**-53.
"""
import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(z):
    """SplitMix64 output function applied elementwise to a uint64 array."""
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def _key(seed, stream, event, draw):
    with np.errstate(over="ignore"):
        h = splitmix64(np.uint64(seed) + _GOLDEN * np.uint64(stream + 1))
        h = splitmix64(h + _GOLDEN * (np.asarray(event, dtype=np.uint64) + np.uint64(1)))
        h = splitmix64(h + _GOLDEN * (np.asarray(draw, dtype=np.uint64) + np.uint64(1)))
    return h


def uniform(seed, stream, event, draw):
    """Uniform deviates in (0, 1), float64, broadcast over `event` and `draw`."""
    x = _key(int(seed), int(stream), event, draw)
    return ((x >> np.uint64(11)).astype(np.float64) + 0.5) * (2.0 ** -53)
