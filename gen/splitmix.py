"""Counter-based SplitMix64 random stream (Steele, Lea and Flood, "Fast splittable
pseudorandom number generators", OOPSLA 2014).

Value i of stream (seed, tag) is the SplitMix64 finaliser applied to
key + (i + 1) * golden, where key itself is the finaliser of seed mixed with
the tag.  Every draw is a pure function of (seed, tag, i), so any slice of a
stream can be regenerated independently and both consumers of the generated
inputs see identical numbers.  Doubles are formed from the top 53 bits.
"""
import numpy as np

GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix(z):
    z = np.asarray(z, dtype=np.uint64)
    z = (z ^ (z >> np.uint64(30))) * _M1
    z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def _key(seed, tag):
    s = np.array([seed & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64)
    t = np.array([tag & 0xFFFFFFFFFFFFFFFF], dtype=np.uint64)
    return _mix(_mix(s) ^ (t * GOLDEN))[0]


def bits(seed, tag, n, start=0):
    """n raw 64-bit draws of stream (seed, tag), counters start .. start+n-1."""
    i = np.arange(start + 1, start + n + 1, dtype=np.uint64)
    return _mix(_key(seed, tag) + i * GOLDEN)


def uniform(seed, tag, n, lo=0.0, hi=1.0, start=0):
    """n doubles uniform on [lo, hi)."""
    u = (bits(seed, tag, n, start) >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return lo + (hi - lo) * u


def normal(seed, tag, n, mean=0.0, sigma=1.0):
    """n standard-normal doubles by the Box-Muller transform of two uniform streams."""
    u1 = uniform(seed, tag, n)
    u2 = uniform(seed, tag ^ 0x5A5A5A5A, n)
    r = np.sqrt(-2.0 * np.log1p(-u1))          # 1-u1 is in (0, 1]
    return mean + sigma * r * np.cos(2.0 * np.pi * u2)
