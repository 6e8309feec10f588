"""SplitMix64 (Steele, Lea & Flood, "Fast splittable pseudorandom number generators",
OOPSLA 2014), written from its published definition.

The generator is not part of the paper; it is the convention by which the coupling
draws of Eq. (1) and the Haar states of the supplement's typicality estimator are
made reproducible.  The oracle and the library each implement it independently.

Definition: the state advances by the odd constant GAMMA; the output is the state
passed through a bijective finaliser (xor-shift 30, multiply, xor-shift 27,
multiply, xor-shift 31), all modulo 2^64.
"""
import numpy as np

MASK64 = (1 << 64) - 1
GAMMA = 0x9E3779B97F4A7C15
_M1 = 0xBF58476D1CE4E5B9
_M2 = 0x94D049BB133111EB


def mix(z: int) -> int:
    """The SplitMix64 output finaliser applied to one 64-bit integer."""
    z &= MASK64
    z = ((z ^ (z >> 30)) * _M1) & MASK64
    z = ((z ^ (z >> 27)) * _M2) & MASK64
    return z ^ (z >> 31)


def mix_array(z: np.ndarray) -> np.ndarray:
    """Vectorised finaliser over a uint64 array (numpy integer arithmetic wraps mod 2^64)."""
    z = np.asarray(z, dtype=np.uint64)
    z = (z ^ (z >> np.uint64(30))) * np.uint64(_M1)
    z = (z ^ (z >> np.uint64(27))) * np.uint64(_M2)
    return z ^ (z >> np.uint64(31))


class SplitMix64:
    """Sequential stream: state += GAMMA, return mix(state)."""

    def __init__(self, seed: int):
        self.state = seed & MASK64

    def next(self) -> int:
        self.state = (self.state + GAMMA) & MASK64
        return mix(self.state)


def unit_open0(r: int) -> float:
    """Uniform double in (0, 1]: ((r >> 11) + 1) * 2^-53."""
    return float((r >> 11) + 1) * (2.0 ** -53)


def unit_open1(r: int) -> float:
    """Uniform double in [0, 1): (r >> 11) * 2^-53."""
    return float(r >> 11) * (2.0 ** -53)
