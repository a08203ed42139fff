"""Pins for the oracle's two-bin Fourier interpolation (Sec. 3: the more
accurate alternative to interbinning, templates and signal at doubled
resolution).  The half-bin columns are checked against literal loops, the
closed-form energy of the truncated half-bin response (z = 0: sum of
1/(pi q)^2 over the half-integer offsets in the window), quadrature of the
response for z != 0, an independent time-domain chirp, and the integer
columns against the plain plane."""
import numpy as np
import pytest

import fdas_synth as syn
from oracle import direct
from oracle import templates as ot
from tests.quadrature import response_quadrature


def test_literal_loops():
    N, M, zmax = 40, 8, 4.0
    A = syn.random_spectrum(3, N).astype(np.complex128)
    P2 = direct.fourier_interpolated_power(A, zmax, 2.0, M)
    for zi, z in enumerate(ot.z_grid(zmax, 2.0)):
        for r in range(N):
            s = 0j
            for k in range(r - M // 2 + 1, r + M // 2 + 1):
                if 0 <= k < N:
                    s += A[k] * np.conj(ot.response(np.array([r + 0.5 - k]), z)[0])
            assert abs(P2[zi, 2 * r + 1] - abs(s) ** 2) < 1e-12


def test_integer_columns_are_the_plain_plane():
    A = syn.random_spectrum(4, 300).astype(np.complex128)
    P2 = direct.fourier_interpolated_power(A, 6.0, 2.0, 32)
    assert np.max(np.abs(P2[:, 0::2] - direct.power(A, ot.templates(6.0, 2.0, 32)))) < 1e-12


@pytest.mark.parametrize("M", [8, 64, 256])
def test_half_bin_z0_energy_closed_form(M):
    # a z = 0 signal at k0 + 1/2: Y_half = a * sum |R(q, 0)|^2 over the M
    # half-integer offsets q = +-1/2, ..., +-(M-1)/2, with |R(q, 0)| = 1/(pi |q|)
    N, k0, a = 600, 300, 1.5 - 2.0j
    A = a * ot.response(k0 + 0.5 - np.arange(N, dtype=np.float64), 0.0)
    P2 = direct.fourier_interpolated_power(A, 0.0, 2.0, M)
    q = np.arange(M) - M / 2 + 0.5
    E = np.sum(1.0 / (np.pi * q) ** 2)
    assert abs(P2[0, 2 * k0 + 1] - abs(a) ** 2 * E ** 2) < 1e-12 * abs(a) ** 2
    assert E > 1.0 - 4.0 / (np.pi ** 2 * M) - 1e-3


@pytest.mark.parametrize("z0", [8.0, -14.0])
def test_half_bin_accelerated_energy_by_quadrature(z0):
    N, k0, M = 800, 400, 64
    A = ot.response(k0 + 0.5 - np.arange(N, dtype=np.float64), z0)
    P2 = direct.fourier_interpolated_power(A, 20.0, 2.0, M)
    zi = int(np.argmin(np.abs(ot.z_grid(20.0, 2.0) - z0)))
    q = M / 2 - 0.5 - np.arange(M, dtype=np.float64)
    E = np.sum(np.abs(response_quadrature(q, z0)) ** 2)
    assert abs(P2[zi, 2 * k0 + 1] - E ** 2) < 1e-9


def test_time_domain_chirp_at_a_half_bin():
    N, M = 8192, 128
    r0, z0 = 3000.5, 12.0
    A = syn.chirp_spectrum(N, [(np.sqrt(50.0), 0.0, r0, z0)])
    P2 = direct.fourier_interpolated_power(A, 20.0, 2.0, M)
    zz, cc = np.unravel_index(np.argmax(P2), P2.shape)
    assert ot.z_grid(20.0, 2.0)[zz] == z0 and cc == 2 * 3000 + 1
    assert abs(P2[zz, cc] / 50.0 - 1.0) < 1e-2


def test_points_match_full_plane():
    A = syn.random_spectrum(8, 700).astype(np.complex128)
    P2 = direct.fourier_interpolated_power(A, 10.0, 2.0, 64)
    rng = np.random.default_rng(2)
    zi = rng.integers(0, P2.shape[0], 500)
    ri = np.concatenate([rng.integers(0, 700, 494), [0, 1, 2, 697, 698, 699]])
    got = direct.fourier_half_points(A, 10.0, 2.0, 64, zi, ri)
    assert np.max(np.abs(got - P2[zi, 2 * ri + 1])) < 1e-12 * np.max(P2)
