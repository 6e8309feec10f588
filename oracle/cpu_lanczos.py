"""Plain CPU matrix-free comparator (oracle/cpu_lanczos.c): complex128 apply of a block
Hamiltonian given as Pauli strings, and Lanczos steps, with OpenMP over amplitudes.

Test and benchmark infrastructure only: it is timed beside the GPU library and checked
against the oracle's row-by-row products; it shares no code with the library.  The shared
object is compiled from the C source with gcc when missing or older than the source.
"""
import ctypes as ct
import os
import subprocess

import numpy as np

from . import pauli

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "cpu_lanczos.c")
_LIB = os.path.join(_HERE, "libcpu_lanczos.so")
_lib = None


def build():
    subprocess.run(["gcc", "-O2", "-fopenmp", "-shared", "-fPIC", _SRC, "-o", _LIB, "-lm"], check=True)


def _load():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB) or os.path.getmtime(_LIB) < os.path.getmtime(_SRC):
            build()
        lib = ct.CDLL(_LIB)
        u64p, dp = ct.POINTER(ct.c_uint64), ct.POINTER(ct.c_double)
        lib.cpu_apply.argtypes = [ct.c_int, ct.c_int, u64p, u64p, dp, dp, ct.c_void_p, ct.c_void_p]
        lib.cpu_apply.restype = None
        lib.cpu_lanczos.argtypes = [ct.c_int, ct.c_int, u64p, u64p, dp, dp, ct.c_void_p, ct.c_int, dp, dp, dp]
        lib.cpu_lanczos.restype = ct.c_int
        _lib = lib
    return _lib


def xz_terms(terms):
    """[(labels, coefficient)] -> (x masks, z masks, coefficients) with each term equal to
    c X^x Z^z (the i^p of pauli.to_xz folded into c)."""
    xs, zs, cs = [], [], []
    for labels, c in terms:
        x, z, p = pauli.to_xz(labels)
        xs.append(x)
        zs.append(z)
        cs.append(complex(c) * (1j ** p))
    return (np.array(xs, dtype=np.uint64), np.array(zs, dtype=np.uint64), np.array(cs, dtype=np.complex128))


def _args(xzc):
    xs, zs, cs = xzc
    cre = np.ascontiguousarray(cs.real)
    cim = np.ascontiguousarray(cs.imag)
    u64p, dp = ct.POINTER(ct.c_uint64), ct.POINTER(ct.c_double)
    return (len(xs), xs.ctypes.data_as(u64p), zs.ctypes.data_as(u64p), cre.ctypes.data_as(dp),
            cim.ctypes.data_as(dp), (xs, zs, cre, cim))


def apply(L: int, xzc, v: np.ndarray) -> np.ndarray:
    lib = _load()
    v = np.ascontiguousarray(v, dtype=np.complex128)
    assert v.size == 1 << L
    y = np.empty_like(v)
    K, xp, zp, rp, ip, keep = _args(xzc)
    lib.cpu_apply(L, K, xp, zp, rp, ip, v.ctypes.data, y.ctypes.data)
    return y


def lanczos(L: int, xzc, v0: np.ndarray, steps: int):
    """Returns (alpha, beta, apply_seconds, total_seconds, threads)."""
    lib = _load()
    v0 = np.ascontiguousarray(v0, dtype=np.complex128)
    assert v0.size == 1 << L
    a, b, sec = np.zeros(steps), np.zeros(steps), np.zeros(2)
    dp = ct.POINTER(ct.c_double)
    K, xp, zp, rp, ip, keep = _args(xzc)
    thr = lib.cpu_lanczos(L, K, xp, zp, rp, ip, v0.ctypes.data, steps, a.ctypes.data_as(dp), b.ctypes.data_as(dp),
                          sec.ctypes.data_as(dp))
    if thr < 0:
        raise MemoryError("cpu_lanczos: host allocation failed")
    return a, b, float(sec[0]), float(sec[1]), thr
