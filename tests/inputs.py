"""Seeded synthetic inputs shared by the oracle side and the library side of the tests.

Holds no arithmetic of the method: only random vectors and index samples."""
import numpy as np


def complex_vector(n: int, seed: int, nvec: int = 1, dtype=np.complex128) -> np.ndarray:
    """nvec standard complex Gaussian vectors of length n (shape (nvec, n))."""
    rng = np.random.default_rng(seed)
    re = rng.standard_normal((nvec, n))
    im = rng.standard_normal((nvec, n))
    return (re + 1j * im).astype(dtype)


def row_sample(n: int, count: int, seed: int) -> np.ndarray:
    """Sorted distinct row indices in [0, n), always including 0 and n-1 (uint64)."""
    rng = np.random.default_rng(seed)
    count = min(count, n)
    r = rng.choice(n, size=count, replace=False) if n > count else np.arange(n)
    r = np.unique(np.concatenate([r, [0, n - 1]]))
    return r.astype(np.uint64)
