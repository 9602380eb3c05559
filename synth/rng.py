"""Counter-based random numbers: SplitMix64 (Steele, Lea and Flood, "Fast
splittable pseudorandom number generators", OOPSLA 2014), evaluated on a
counter so that any element of any stream can be drawn independently and in
any order, vectorised with numpy.

A stream is keyed by (seed, stream id); element i of the stream is the
SplitMix64 output function applied to  seed*GOLDEN + (stream << 40) + i + 1
(all arithmetic mod 2**64).  Doubles take the top 53 bits.
"""
import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed: int, stream: int, index) -> np.ndarray:
    """64-bit outputs for counters `index` (int or array) of stream `stream`."""
    idx = np.asarray(index, dtype=np.uint64)
    with np.errstate(over="ignore"):
        base = (np.uint64(seed & 0xFFFFFFFFFFFFFFFF) * _GOLDEN
                + (np.uint64(stream & 0xFFFFFF) << np.uint64(40)))
        z = (base + idx + np.uint64(1)) * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


def uniform01(seed: int, stream: int, n: int, offset: int = 0) -> np.ndarray:
    """n doubles uniform on [0, 1) from elements offset..offset+n-1 of a stream."""
    z = splitmix64(seed, stream, np.arange(offset, offset + n, dtype=np.uint64))
    return (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
