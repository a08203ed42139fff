"""Oracle for harmonic summing and candidate selection on the f-fdot plane.

TEST INFRASTRUCTURE ONLY (see the package header).

The paper names both steps without giving formulas (Sec. 3: the correlated
power is compared with a precomputed threshold to find candidates; a pulsed
signal spreads its power over harmonics, so the powers of the harmonics are
added to that of the fundamental before the search for peaks; both steps
lie outside the paper's measured path, Sec. 3 and Sec. 7).  Readings used here:

Harmonic sum.  A constant-fdot signal at frequency bin r and drift z (Sec. 2:
r = f T, z = fdot T^2) has its h-th harmonic at (h r, h z).  For a plane
P[K][N] over rows z_k = (k - c) dz, c = (K - 1)/2, and columns r = 0..N-1,
the H-fold sum at the fundamental (k, r) is

    S_H[k][r] = sum_{h=1}^{H} P[c + h (k - c)][h r],

defined where every harmonic lies on the plane: h r < N and |h (k - c)| <= c
for all h <= H, i.e. r in [0, ceil(N/H)) and k in [c - floor(c/H),
c + floor(c/H)].  Harmonics of grid points are grid points, so no
interpolation is involved.  S_H is stored as [K_H][N_H] with K_H =
2 floor(c/H) + 1 rows (row k - c + floor(c/H)) and N_H = ceil(N/H) columns.
The sum runs in FP32 in the order h = 1, 2, ..., H (the decisions below are
taken on these FP32 values, so both sides must form them identically);
``harmonic_sum_f64`` gives the FP64 value for tolerance checks.

Candidates.  A candidate of fold H is a point (k, r) of S_H whose value
exceeds the threshold and is >= each of its (up to 8) neighbours inside the
fold's domain (a peak of summed power).  The set is unique; ties on a
plateau yield every tied maximum.
"""
from __future__ import annotations

import numpy as np


def fold_shape(N: int, K: int, H: int):
    """(K_H, N_H): rows and columns of the H-fold sum of a [K][N] plane."""
    if K < 1 or K % 2 == 0 or H < 1 or N < 0:
        raise ValueError("K must be odd and positive, H >= 1, N >= 0")
    c = (K - 1) // 2
    return 2 * (c // H) + 1, -(-N // H)


def _harmonic_index(N: int, K: int, H: int, h: int):
    """Row and column indices of harmonic h for every fundamental point of
    the H-fold domain (broadcastable arrays)."""
    c = (K - 1) // 2
    KH, NH = fold_shape(N, K, H)
    k = c - c // H + np.arange(KH)
    r = np.arange(NH)
    return (c + h * (k - c))[:, None], (h * r)[None, :]


def harmonic_sum(P, H: int) -> np.ndarray:
    """S_H as FP32, summed in the order h = 1..H."""
    P = np.asarray(P, dtype=np.float32)
    K, N = P.shape
    KH, NH = fold_shape(N, K, H)
    S = np.zeros((KH, NH), dtype=np.float32)
    for h in range(1, H + 1):
        rows, cols = _harmonic_index(N, K, H, h)
        S = S + P[rows, cols]
    return S


def harmonic_sum_f64(P, H: int) -> np.ndarray:
    """S_H with the same terms summed in FP64."""
    P = np.asarray(P, dtype=np.float64)
    K, N = P.shape
    KH, NH = fold_shape(N, K, H)
    S = np.zeros((KH, NH), dtype=np.float64)
    for h in range(1, H + 1):
        rows, cols = _harmonic_index(N, K, H, h)
        S += P[rows, cols]
    return S


def peaks(S, threshold: float) -> np.ndarray:
    """Candidates of one fold: (row, column) pairs of S (its own indices),
    sorted by row then column, where S > threshold and S >= every
    neighbour inside S."""
    S = np.asarray(S, dtype=np.float32)
    KH, NH = S.shape
    if KH == 0 or NH == 0:
        return np.zeros((0, 2), dtype=np.int64)
    pad = np.full((KH + 2, NH + 2), -np.inf, dtype=np.float32)
    pad[1:-1, 1:-1] = S
    ok = S > np.float32(threshold)
    for dk in (-1, 0, 1):
        for dr in (-1, 0, 1):
            if dk == 0 and dr == 0:
                continue
            ok &= S >= pad[1 + dk:1 + dk + KH, 1 + dr:1 + dr + NH]
    k, r = np.nonzero(ok)
    return np.stack([k, r], axis=1).astype(np.int64)
