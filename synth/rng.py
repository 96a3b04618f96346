"""Counter-based uniform random numbers for the seeded synthetic inputs.

SplitMix64 (Steele, Lea and Flood, "Fast splittable pseudorandom number
generators", OOPSLA 2014): the state advances by the golden-ratio increment
0x9E3779B97F4A7C15 and each state is passed through the published 64-bit
finaliser (xor-shift 30, multiply 0xBF58476D1CE4E5B9, xor-shift 27, multiply
0x94D049BB133111EB, xor-shift 31).  Here the state of draw ``c`` of stream
``(seed, stream)`` is ``base + (c + 1) * golden`` with
``base = mix(mix(seed) ^ (stream * golden))``, so any draw can be computed
on its own from its counter: generation is order-free and vectorised.

This module only produces input data; it holds none of the method's
arithmetic.
"""
import numpy as np

_GOLDEN = np.uint64(0x9E3779B97F4A7C15)
_M1 = np.uint64(0xBF58476D1CE4E5B9)
_M2 = np.uint64(0x94D049BB133111EB)


def _mix(z):
    z = np.asarray(z, dtype=np.uint64)
    with np.errstate(over="ignore"):
        z = (z ^ (z >> np.uint64(30))) * _M1
        z = (z ^ (z >> np.uint64(27))) * _M2
    return z ^ (z >> np.uint64(31))


def stream_base(seed: int, stream: int) -> np.uint64:
    with np.errstate(over="ignore"):
        s = _mix(np.uint64(seed & 0xFFFFFFFFFFFFFFFF))
        return _mix(s ^ (np.uint64(stream) * _GOLDEN))


def u64(seed: int, stream: int, counter) -> np.ndarray:
    """Raw 64-bit outputs for the given counters (any integer array)."""
    base = stream_base(seed, stream)
    c = np.asarray(counter, dtype=np.uint64)
    with np.errstate(over="ignore"):
        state = base + (c + np.uint64(1)) * _GOLDEN
    return _mix(state)


def uniform(seed: int, stream: int, counter) -> np.ndarray:
    """Doubles in [0, 1) with 53 random bits."""
    return (u64(seed, stream, counter) >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)


def uniform_range(seed, stream, counter, lo, hi) -> np.ndarray:
    return lo + (hi - lo) * uniform(seed, stream, counter)
