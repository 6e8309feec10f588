"""Counter-based Haar-random states for the typicality estimator of the supplement
(a Haar-random state is drawn, evolved, and its overlap taken).

Amplitude n of the full 2^(N/2)-dimensional space (parity qubit most significant,
so n < 2^L is the U block and n >= 2^L the D block) is a standard complex Gaussian
made by Box-Muller from two SplitMix64 outputs of counters:

    base = mix(state_seed + (v+1) GAMMA)
    w1 = mix(base + (2n+1) GAMMA),  w2 = mix(base + (2n+2) GAMMA)
    u1 = ((w1 >> 11) + 1) 2^-53,    u2 = (w2 >> 11) 2^-53
    psi_n = sqrt(-2 ln u1) (cos 2 pi u2 + i sin 2 pi u2)

and the vector is normalised in float64.  A normalised complex Gaussian vector is
Haar distributed on the unit sphere.  ``v`` numbers independent vectors.
"""
import numpy as np

from .splitmix import GAMMA, MASK64, mix, mix_array


def raw_amplitudes(state_seed: int, v: int, idx: np.ndarray) -> np.ndarray:
    """Unnormalised amplitudes at full-space indices ``idx`` (uint64 array)."""
    base = mix((state_seed + (v + 1) * GAMMA) & MASK64)
    n = np.asarray(idx, dtype=np.uint64)
    g = np.uint64(GAMMA)
    b = np.uint64(base)
    w1 = mix_array(b + (n * np.uint64(2) + np.uint64(1)) * g)
    w2 = mix_array(b + (n * np.uint64(2) + np.uint64(2)) * g)
    u1 = ((w1 >> np.uint64(11)) + np.uint64(1)).astype(np.float64) * (2.0 ** -53)
    u2 = (w2 >> np.uint64(11)).astype(np.float64) * (2.0 ** -53)
    r = np.sqrt(-2.0 * np.log(u1))
    ang = 2.0 * np.pi * u2
    return r * np.cos(ang) + 1j * (r * np.sin(ang))


def haar_state(N: int, state_seed: int, v: int = 0) -> np.ndarray:
    """Normalised full-space state (complex128), N small enough to hold it."""
    d = 1 << (N // 2)
    psi = raw_amplitudes(state_seed, v, np.arange(d, dtype=np.uint64))
    return psi / np.sqrt(np.sum(psi.real ** 2 + psi.imag ** 2))


def raw_norm2(N: int, state_seed: int, v: int = 0, chunk: int = 1 << 22) -> float:
    """sum |raw amplitude|^2 over the full space, in chunks (for large N)."""
    d = 1 << (N // 2)
    s = 0.0
    for lo in range(0, d, chunk):
        a = raw_amplitudes(state_seed, v, np.arange(lo, min(d, lo + chunk), dtype=np.uint64))
        s += float(np.sum(a.real ** 2 + a.imag ** 2))
    return s
