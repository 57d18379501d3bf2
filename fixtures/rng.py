"""Counter-based random numbers for the seeded synthetic inputs.

The generator is splitmix64 (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014) evaluated at counter values
1, 2, 3, ... for a given 64-bit seed, so a stream does not depend on the numpy
version or on how draws are batched.  Uniforms take the top 53 bits; normals
use the Box-Muller transform on consecutive uniform pairs.

This module holds no arithmetic of the method; it only turns seeds into
numbers.
"""
import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def splitmix64(seed, n, offset=0):
    """Return n uint64 outputs of splitmix64 for counters offset+1 .. offset+n."""
    with np.errstate(over="ignore"):
        ctr = np.arange(offset + 1, offset + n + 1, dtype=np.uint64)
        z = np.uint64(seed & 0xFFFFFFFFFFFFFFFF) + ctr * _GOLDEN
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
        z = z ^ (z >> np.uint64(31))
    return z


class Stream:
    """A sequential view of one splitmix64 stream."""

    def __init__(self, seed):
        self.seed = int(seed)
        self.pos = 0

    def bits(self, n):
        out = splitmix64(self.seed, n, self.pos)
        self.pos += n
        return out

    def uniform(self, n, lo=0.0, hi=1.0):
        u = (self.bits(n) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
        return lo + (hi - lo) * u

    def normal(self, n):
        m = (n + 1) // 2
        u1 = self.uniform(m)
        u2 = self.uniform(m)
        r = np.sqrt(-2.0 * np.log1p(-u1))
        th = 2.0 * np.pi * u2
        z = np.empty(2 * m)
        z[0::2] = r * np.cos(th)
        z[1::2] = r * np.sin(th)
        return z[:n]

    def signs(self, n):
        return np.where((self.bits(n) >> np.uint64(63)) == 0, 1.0, -1.0)
