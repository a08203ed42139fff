"""Oracle: build and load the plain C/OpenMP direct correlation (FP64).

Test infrastructure only: the test suite, the smoke check and the
benchmark's CPU-baseline leg use it.  ``build()`` compiles
``fdas_oracle.c`` with gcc into ``_fdas_oracle.so`` next to it.
"""
from __future__ import annotations

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "fdas_oracle.c")
_LIB = os.path.join(_HERE, "_fdas_oracle.so")
_lib = None


def build(force: bool = True) -> str:
    """Compile the C oracle (gcc -O2 -fopenmp, strict IEEE FP64: no fast-math)."""
    if force or not os.path.exists(_LIB):
        tmp = _LIB + f".tmp{os.getpid()}"
        subprocess.run(["gcc", "-O2", "-fopenmp", "-fPIC", "-shared", "-std=c99",
                        "-o", tmp, _SRC, "-lm"], check=True)
        os.replace(tmp, _LIB)
    return _LIB


def lib():
    global _lib
    if _lib is None:
        if not os.path.exists(_LIB):
            build()
        L = ctypes.CDLL(_LIB)
        d, i64, i32 = ctypes.c_void_p, ctypes.c_int64, ctypes.c_int
        L.oracle_num_threads.restype = ctypes.c_int
        L.oracle_power.argtypes = [d, i64, d, i32, i32, i64, i64, d]
        L.oracle_power_points.argtypes = [d, i64, d, i32, i32, d, d, i64, d]
        L.oracle_correlate.argtypes = [d, i64, d, i32, i32, d]
        L.oracle_grads.argtypes = [d, i64, d, i32, i32, d, d, d]
        L.oracle_grads.restype = ctypes.c_int
        L.oracle_grad_spec_points.argtypes = [d, i64, d, i32, i32, d, d, i64, d]
        L.oracle_interbin_points.argtypes = [d, i64, d, i32, i32, d, d, i64, d]
        _lib = L
    return _lib


def _c128(x):
    return np.ascontiguousarray(x, dtype=np.complex128)


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def num_threads() -> int:
    return int(lib().oracle_num_threads())


def power(A, T, r_lo: int = 0, r_hi: int | None = None) -> np.ndarray:
    """P[K][r_hi - r_lo] for columns [r_lo, r_hi) (default: all N)."""
    A, T = _c128(A), _c128(T)
    K, M = T.shape
    N = len(A)
    r_hi = N if r_hi is None else r_hi
    out = np.empty((K, r_hi - r_lo), dtype=np.float64)
    lib().oracle_power(_p(A), N, _p(T), K, M, r_lo, r_hi, _p(out))
    return out


def power_points(A, T, zi, ri) -> np.ndarray:
    """P at sampled points (zi[p], ri[p])."""
    A, T = _c128(A), _c128(T)
    K, M = T.shape
    zi = np.ascontiguousarray(zi, dtype=np.int32)
    ri = np.ascontiguousarray(ri, dtype=np.int64)
    out = np.empty(len(zi), dtype=np.float64)
    lib().oracle_power_points(_p(A), len(A), _p(T), K, M, _p(zi), _p(ri), len(zi), _p(out))
    return out


def interbin_points(A, T, zi, ci) -> np.ndarray:
    """Interbinned plane ([K][2N] layout) at sampled (zi[p], column ci[p])."""
    A, T = _c128(A), _c128(T)
    K, M = T.shape
    zi = np.ascontiguousarray(zi, dtype=np.int32)
    ci = np.ascontiguousarray(ci, dtype=np.int64)
    out = np.empty(len(zi), dtype=np.float64)
    lib().oracle_interbin_points(_p(A), len(A), _p(T), K, M, _p(zi), _p(ci), len(zi), _p(out))
    return out


def correlate(A, T) -> np.ndarray:
    A, T = _c128(A), _c128(T)
    K, M = T.shape
    out = np.empty((K, len(A)), dtype=np.complex128)
    lib().oracle_correlate(_p(A), len(A), _p(T), K, M, _p(out))
    return out


def grad_spec_points(A, T, w, ks) -> np.ndarray:
    """grad_A at the sampled bins ks (complex128), each from its defining sum."""
    A, T = _c128(A), _c128(T)
    K, M = T.shape
    w = np.ascontiguousarray(w, dtype=np.float32)
    assert w.shape == (K, len(A))
    ks = np.ascontiguousarray(ks, dtype=np.int64)
    out = np.empty(len(ks), dtype=np.complex128)
    lib().oracle_grad_spec_points(_p(A), len(A), _p(T), K, M, _p(w), _p(ks), len(ks), _p(out))
    return out


def grads(A, T, w):
    """(grad_A [N], grad_T [K][M]) complex128 for Lw = sum w P."""
    A, T = _c128(A), _c128(T)
    K, M = T.shape
    w = np.ascontiguousarray(w, dtype=np.float32)
    assert w.shape == (K, len(A))
    gA = np.empty(len(A), dtype=np.complex128)
    gT = np.empty((K, M), dtype=np.complex128)
    rc = lib().oracle_grads(_p(A), len(A), _p(T), K, M, _p(w), _p(gA), _p(gT))
    if rc != 0:
        raise MemoryError("oracle_grads: allocation failed")
    return gA, gT
