"""Oracle: direct FP64 correlation, power plane and gradients (numpy).

Test infrastructure only.  The correlation technique (Sec. 2, eq. 23)
recovers the response at bin r by correlating the M bins around r with the
complex-conjugated template.  The paper prints the sum with garbled limits;
the reading used here (taps j in [0, M) at bin offsets e_j = j - M/2, the
spectrum taken as zero outside [0, N)) is

    Y[z][r] = sum_j A[r + e_j] * conj(T[z][j]),   P[z][r] = |Y[z][r]|^2,

for every r in [0, N).  The overlap-save FFT evaluation (Sec. 3, Fig. 1) is
a fast way of computing exactly this sum; the oracle evaluates the sum
itself, with no FFT, no blocking and no reordering.

Gradients of the loss  Lw = sum_{z,r} w[z][r] P[z][r]  (not in the paper;
written from the definition above, in PyTorch's complex convention
grad = dLw/dRe + i dLw/dIm):
    g[z][r]      = 2 w[z][r] Y[z][r]
    grad_A[k]    = sum_z sum_j T[z][j] g[z][k - e_j]      (g = 0 outside [0, N))
    grad_T[z][j] = sum_r conj(g[z][r]) A[r + e_j]
"""
from __future__ import annotations

import numpy as np


def _padded(A: np.ndarray, M: int) -> np.ndarray:
    """A placed at offset M/2 of a zero array of length N + M, so that
    A[r + e_j] = pad[r + j] for every r in [0, N) and j in [0, M)."""
    N = len(A)
    pad = np.zeros(N + M, dtype=np.complex128)
    pad[M // 2:M // 2 + N] = A
    return pad


def correlate(A, T) -> np.ndarray:
    """Complex correlation Y[K][N] (complex128)."""
    A = np.asarray(A, dtype=np.complex128)
    T = np.asarray(T, dtype=np.complex128)
    K, M = T.shape
    N = len(A)
    pad = _padded(A, M)
    Y = np.zeros((K, N), dtype=np.complex128)
    for j in range(M):
        Y += np.conj(T[:, j])[:, None] * pad[j:j + N][None, :]
    return Y


def power(A, T) -> np.ndarray:
    """f-fdot power plane P[K][N] = |Y|^2 (float64)."""
    Y = correlate(A, T)
    return Y.real ** 2 + Y.imag ** 2


def loss(A, T, w) -> float:
    """Lw = sum w * P."""
    return float(np.sum(np.asarray(w, dtype=np.float64) * power(A, T)))


def grads(A, T, w):
    """(grad_A [N], grad_T [K][M]) of Lw, complex128, PyTorch convention."""
    A = np.asarray(A, dtype=np.complex128)
    T = np.asarray(T, dtype=np.complex128)
    w = np.asarray(w, dtype=np.float64)
    K, M = T.shape
    N = len(A)
    g = 2.0 * w * correlate(A, T)
    # gpad[:, M + r] = g[:, r]; then g[:, k - e_j] = gpad[:, k + M + M/2 - j]
    gpad = np.zeros((K, N + 2 * M), dtype=np.complex128)
    gpad[:, M:M + N] = g
    gA = np.zeros(N, dtype=np.complex128)
    for j in range(M):
        start = M + M // 2 - j
        gA += (T[:, j][:, None] * gpad[:, start:start + N]).sum(axis=0)
    pad = _padded(A, M)
    gT = np.zeros((K, M), dtype=np.complex128)
    gc = np.conj(g)
    for j in range(M):
        gT[:, j] = gc @ pad[j:j + N]
    return gA, gT


def interbinned_power(A, T) -> np.ndarray:
    """Power plane with interbinning (Sec. 3, eq. f-interp), P2[K][2N]:
    column 2r is |Y[r]|^2 and column 2r+1 the half-bin estimate
    |(pi/4)(Y[r] - Y[r+1])|^2, where Y[N] is the same correlation sum one bin
    past the end (the spectrum is zero outside [0, N))."""
    A = np.asarray(A, dtype=np.complex128)
    N = len(A)
    Y = correlate(np.concatenate([A, [0.0]]), T)          # Y[:, 0..N]
    P2 = np.empty((Y.shape[0], 2 * N), dtype=np.float64)
    P2[:, 0::2] = np.abs(Y[:, :N]) ** 2
    P2[:, 1::2] = np.abs((np.pi / 4) * (Y[:, :N] - Y[:, 1:N + 1])) ** 2
    return P2


def fourier_interpolated_power(A, zmax: float, dz: float, M: int) -> np.ndarray:
    """Two-bin Fourier interpolation (Sec. 3, the alternative to eq.
    f-interp: templates and signal at doubled resolution), P2[K][2N]:
    column 2r is |Y[r]|^2 with the M-tap templates, and column 2r+1 the
    matched-filter response at the half bin r + 1/2 over the M bins centred
    there, k in [r - M/2 + 1, r + M/2]:
        Y_half[z][r] = sum_k A[k] conj(R(r + 1/2 - k, z)),
    the spectrum zero outside [0, N).  Templates from the closed form."""
    from . import templates as ot
    A = np.asarray(A, dtype=np.complex128)
    N = len(A)
    T = ot.templates(zmax, dz, M)
    zs = ot.z_grid(zmax, dz)
    P2 = np.empty((len(zs), 2 * N), dtype=np.float64)
    P2[:, 0::2] = power(A, T)
    # k = r - M/2 + 1 + i, i in [0, M): offset q = r + 1/2 - k = M/2 - 1/2 - i
    q = M / 2 - 0.5 - np.arange(M, dtype=np.float64)
    pad = np.zeros(N + M, dtype=np.complex128)
    pad[M // 2 - 1:M // 2 - 1 + N] = A            # pad[r + i] = A[r - M/2 + 1 + i]
    for zi, z in enumerate(zs):
        w = np.conj(ot.response(q, z))
        Y = np.zeros(N, dtype=np.complex128)
        for i in range(M):
            Y += w[i] * pad[i:i + N]
        P2[zi, 1::2] = Y.real ** 2 + Y.imag ** 2
    return P2


def fourier_half_points(A, zmax: float, dz: float, M: int, zi, ri) -> np.ndarray:
    """The half-bin column |Y_half[z][r]|^2 of fourier_interpolated_power at
    the sampled (template index, bin) pairs, each from its defining sum."""
    from . import templates as ot
    A = np.asarray(A, dtype=np.complex128)
    N = len(A)
    zs = ot.z_grid(zmax, dz)
    q = M / 2 - 0.5 - np.arange(M, dtype=np.float64)
    W = np.conj(np.stack([ot.response(q, z) for z in zs]))          # [K][M]
    pad = np.zeros(N + M, dtype=np.complex128)
    pad[M // 2 - 1:M // 2 - 1 + N] = A
    zi = np.asarray(zi, dtype=np.int64)
    ri = np.asarray(ri, dtype=np.int64)
    idx = ri[:, None] + np.arange(M)[None, :]
    Y = np.sum(W[zi] * pad[idx], axis=1)
    return Y.real ** 2 + Y.imag ** 2
