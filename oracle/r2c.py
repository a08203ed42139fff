"""Oracle for the real-to-complex front end (test infrastructure only).

The input time series is an array of n FP32 samples that is taken to the
Fourier domain with a real-to-complex transform before the correlations
(Sec. 3 processing steps, Sec. 4.1).  Its plain definition is the
unnormalised DFT of the real samples at the non-negative frequencies,

    A[k] = scale * sum_{t=0}^{n-1} x[t] exp(-2 pi i k t / n),  k = 0 .. n/2,

i.e. n/2 + 1 complex bins (the Nyquist bin included), as a library
real-to-complex FFT returns them.

``dft`` evaluates that sum literally in FP64 (O(n^2), small n only).
``spectrum`` is the same definition computed with numpy's FFT as a single
library step, in FP64, for sizes the literal sum cannot reach.
"""
from __future__ import annotations

import numpy as np


def dft(x, scale: float = 1.0) -> np.ndarray:
    """Literal sum over t for every k in [0, n/2] (complex128)."""
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    k = np.arange(n // 2 + 1, dtype=np.int64)
    t = np.arange(n, dtype=np.int64)
    # exact integer phase index (k t mod n) before scaling, so the twiddles
    # carry no accumulated argument error
    ph = (k[:, None] * t[None, :]) % n
    W = np.exp(-2j * np.pi * ph / n)
    return scale * (W @ x)


def spectrum(x, scale: float = 1.0) -> np.ndarray:
    """The same bins via numpy's real FFT in FP64 (complex128)."""
    x = np.asarray(x, dtype=np.float64)
    return scale * np.fft.rfft(x)


def dft_points(x, ks, scale: float = 1.0) -> np.ndarray:
    """The literal sum at the selected bins ks only (complex128), O(n) per
    bin, for sampled checks at sizes where the full literal sum is out of
    reach."""
    x = np.asarray(x, dtype=np.float64)
    n = len(x)
    t = np.arange(n, dtype=np.int64)
    out = np.empty(len(ks), dtype=np.complex128)
    for i, k in enumerate(np.asarray(ks, dtype=np.int64)):
        ph = (k * t) % n
        out[i] = np.dot(np.exp(-2j * np.pi * ph / n), x)
    return scale * out
