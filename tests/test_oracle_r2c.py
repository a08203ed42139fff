"""Pins for the real-to-complex front end oracle (Sec. 4.1).

The literal sum is checked against closed forms (impulse, constant, a
cosine on a bin, a sine between bins, an alternating sequence), Parseval's
identity for a real series, linearity, and a time shift; the FFT route is
checked against the literal sum.
"""
import numpy as np
import pytest

from oracle import r2c


def _series(seed, n):
    return np.random.default_rng(seed).normal(size=n)


def test_impulse_is_flat():
    n = 64
    x = np.zeros(n)
    x[0] = 2.5
    assert np.max(np.abs(r2c.dft(x) - 2.5)) < 1e-12


def test_shifted_impulse_is_a_phase_ramp():
    n, t0 = 96, 7
    x = np.zeros(n)
    x[t0] = 1.0
    k = np.arange(n // 2 + 1)
    assert np.max(np.abs(r2c.dft(x) - np.exp(-2j * np.pi * k * t0 / n))) < 1e-12


def test_constant_goes_to_dc():
    n = 50
    A = r2c.dft(np.full(n, 0.75))
    assert abs(A[0] - 0.75 * n) < 1e-12 and np.max(np.abs(A[1:])) < 1e-12


@pytest.mark.parametrize("k0", [1, 5, 31])
def test_cosine_on_a_bin(k0):
    # x = cos(2 pi k0 t / n + phi)  ->  A[k0] = (n/2) e^{i phi}, zero elsewhere
    n, phi = 64, 0.4
    t = np.arange(n)
    A = r2c.dft(np.cos(2 * np.pi * k0 * t / n + phi))
    ref = np.zeros(n // 2 + 1, dtype=complex)
    ref[k0] = 0.5 * n * np.exp(1j * phi)
    assert np.max(np.abs(A - ref)) < 1e-11


def test_alternating_sequence_goes_to_nyquist():
    n = 40
    A = r2c.dft((-1.0) ** np.arange(n))
    ref = np.zeros(n // 2 + 1, dtype=complex)
    ref[n // 2] = n
    assert np.max(np.abs(A - ref)) < 1e-11


def test_sine_between_bins_closed_form():
    # x = e^{i 2 pi f t/n} summed: geometric series; take the real part via
    # (e^{+} + e^{-})/2 so the series is real
    n, f = 128, 10.5
    t = np.arange(n)
    x = np.cos(2 * np.pi * f * t / n)
    k = np.arange(n // 2 + 1)

    def geo(d):                      # sum_t e^{i 2 pi d t / n}
        return (1 - np.exp(2j * np.pi * d)) / (1 - np.exp(2j * np.pi * d / n))

    ref = 0.5 * (geo(f - k) + geo(-f - k))
    assert np.max(np.abs(r2c.dft(x) - ref)) < 1e-10


def test_parseval_for_real_series():
    # sum x^2 = (1/n) (|A_0|^2 + 2 sum_{0<k<n/2} |A_k|^2 + |A_{n/2}|^2), n even
    n = 200
    x = _series(1, n)
    A = r2c.dft(x)
    e = (abs(A[0]) ** 2 + 2 * np.sum(np.abs(A[1:-1]) ** 2) + abs(A[-1]) ** 2) / n
    assert abs(e - np.sum(x * x)) < 1e-10 * np.sum(x * x)


def test_linearity_and_scale():
    n = 60
    x, y = _series(2, n), _series(3, n)
    lhs = r2c.dft(2.0 * x - 3.0 * y, scale=0.5)
    rhs = 0.5 * (2.0 * r2c.dft(x) - 3.0 * r2c.dft(y))
    assert np.max(np.abs(lhs - rhs)) < 1e-11


def test_circular_time_shift():
    n, d = 80, 13
    x = _series(4, n)
    k = np.arange(n // 2 + 1)
    assert np.max(np.abs(r2c.dft(np.roll(x, d)) - np.exp(-2j * np.pi * k * d / n) * r2c.dft(x))) < 1e-10


@pytest.mark.parametrize("n", [2, 16, 250, 1024])
def test_fft_route_matches_literal_sum(n):
    x = _series(n, n)
    a, b = r2c.spectrum(x, scale=0.25), r2c.dft(x, scale=0.25)
    assert np.max(np.abs(a - b)) < 1e-12 * max(1.0, np.max(np.abs(b)))


def test_dft_points_match_literal_sum():
    n = 512
    x = _series(9, n)
    ks = np.array([0, 1, 17, 255, 256])
    assert np.max(np.abs(r2c.dft_points(x, ks, 0.5) - r2c.dft(x, 0.5)[ks])) < 1e-10
