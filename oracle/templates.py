"""Oracle: acceleration templates, FP64 (test infrastructure only).

The template for trial frequency derivative z is the predicted normalised
Fourier response of a unit-amplitude constant-fdot signal (Sec. 2, the text
around eq. 23; the paper cites the closed form rather than printing it).
Written out from the definition of the DFT coefficient (Sec. 4.2, eq. DFT,
in its continuous limit): a signal that sits at bin r at mid-observation and
drifts by z bins over the observation (eq. 22),

    x(u) = exp(i 2 pi [r u + z (u^2 - u)/2]),  u = t/T in [0, 1),

has response at bin k

    R(q, z) = int_0^1 exp(i 2 pi [q u + z (u^2 - u)/2]) du,   q = r - k.

Closed form (complete the square, substitute t = sqrt(2z) (u + q'/z)):
    z = 0 : R = (exp(i 2 pi q) - 1) / (i 2 pi q),  R(0, 0) = 1
    z > 0 : q' = q - z/2,  s = sqrt(2/z)
            R = exp(-i pi q'^2/z) / sqrt(2z) *
                [C(s(q'+z)) - C(s q') + i (S(s(q'+z)) - S(s q'))]
    z < 0 : R(q, z) = conj R(-q, -z)
with C, S the Fresnel integrals int_0^x cos/sin(pi t^2/2) dt, taken from
scipy.special.fresnel (a library primitive standing in for one step).

Tap j of an M-tap template sits at bin offset e_j = j - M/2 (j in [0, M)),
and T[z][j] = R(e_j, z).  Readings of the paper (which is silent or
ambiguous on these): mid-observation frequency reference, time origin at the
first sample (the DFT indexes from n = 0), no renormalisation of truncated
taps, and the z grid z_k = -zmax + k dz ascending.
"""
from __future__ import annotations

import numpy as np
from scipy.special import fresnel


def response(q, z: float) -> np.ndarray:
    """R(q, z) in FP64 for an array of (possibly fractional) offsets q."""
    q = np.asarray(q, dtype=np.float64)
    z = float(z)
    if z < 0.0:
        return np.conj(response(-q, -z))
    if z == 0.0:
        out = np.ones(q.shape, dtype=np.complex128)
        nz = q != 0.0
        qq = q[nz]
        out[nz] = (np.exp(2j * np.pi * qq) - 1.0) / (2j * np.pi * qq)
        return out
    qp = q - 0.5 * z
    s = np.sqrt(2.0 / z)
    s1, c1 = fresnel(s * qp)
    s2, c2 = fresnel(s * (qp + z))
    return np.exp(-1j * np.pi * qp * qp / z) / np.sqrt(2.0 * z) * ((c2 - c1) + 1j * (s2 - s1))


def z_grid(zmax: float, dz: float) -> np.ndarray:
    """Trial z values -zmax, -zmax+dz, ..., +zmax (ascending rows)."""
    K = int(round(2.0 * zmax / dz)) + 1
    return -zmax + dz * np.arange(K, dtype=np.float64)


def tap_offsets(M: int) -> np.ndarray:
    """Bin offset e_j = j - M/2 of tap j."""
    return np.arange(M, dtype=np.float64) - M // 2


def templates(zmax: float, dz: float, M: int) -> np.ndarray:
    """Template bank T[K][M] (complex128): T[k][j] = R(j - M/2, z_k)."""
    e = tap_offsets(M)
    return np.stack([response(e, z) for z in z_grid(zmax, dz)])
