"""Pins for the oracle's correlation and power plane (Sec. 2 eq. 23, Sec. 3).

Each check compares the oracle with something it does not compute itself:
the identity template, injected signals against the textbook sinc^2 limit,
a time-domain chirp route, linearity (parallelogram law), the +/-z
symmetry, shift equivariance, noise statistics, brute-force overlap-save
with explicit DFT matrices (the paper's own method, Fig. 1), and literal
loops.  The C/OpenMP oracle is checked against the numpy one.
"""
import numpy as np
import pytest

import fdas_synth as syn
from oracle import direct, native
from oracle import templates as ot


def _rand(seed, n):
    return syn.random_spectrum(seed, n).astype(np.complex128)


def test_z0_reproduces_input_power():
    A = _rand(1, 3000)
    T = ot.templates(6.0, 2.0, 32)
    P = direct.power(A, T)
    assert np.max(np.abs(P[3] - np.abs(A) ** 2)) < 1e-12 * np.max(np.abs(A) ** 2) + 1e-14


def _injected(N, r0, z0, amp=1.0, phase=0.3):
    k = np.arange(N, dtype=np.float64)
    return amp * np.exp(1j * phase) * ot.response(r0 - k, z0)


@pytest.mark.parametrize("delta", [0.0, 0.3, 0.5, 0.7])
@pytest.mark.parametrize("z0", [0.0, 8.0, -14.0])
def test_injected_signal_peak_vs_sinc2_limit(delta, z0):
    # A_k = a R(r0 - k, z0): the matched filter at (round(r0), z0) recovers
    # |a|^2 |sum_e R(delta - e) conj R(-e)|^2, which tends (M -> inf, by
    # Parseval) to |a|^2 sinc^2(pi delta) -- the scalloping curve.
    N, M = 4096, 256
    r0 = 2000 + delta
    A = _injected(N, r0, z0, amp=np.sqrt(50.0))
    T = ot.templates(20.0, 2.0, M)
    zs = ot.z_grid(20.0, 2.0)
    P = direct.power(A, T)
    kz = int(np.argmin(np.abs(zs - z0)))
    limit = 50.0 * (np.sinc(delta) ** 2)
    peak_r = int(np.argmax(P[kz]))
    assert peak_r in (2000, 2001)
    assert abs(peak_r - r0) <= 0.5 + 1e-9           # within half a bin (Sec. 5.2)
    assert abs(P[kz, 2000] - limit) < 2e-3 * 50.0   # M = 256 truncation
    # the true template wins over its neighbours one z step away
    zz, rr = np.unravel_index(np.argmax(P), P.shape)
    assert abs(zs[zz] - z0) <= 2.0 and abs(rr - r0) <= 1.0


def test_config1_peak_power_vs_limit():
    # On the workload-1 grid (M = 64) the truncated sum falls 3.4e-5 |a|^2
    # short of the limit sinc^2(0.3 pi) = 0.7368397.
    N, M = 1 << 14, 64
    A = _injected(N, 8000.3, 8.0, amp=1.0, phase=0.0)
    T = ot.templates(20.0, 2.0, M)
    P = direct.power(A, T)
    val = P[14, 8000]
    assert abs(np.sinc(0.3) ** 2 - 0.7368397) < 1e-7
    assert 0.7366 < val < np.sinc(0.3) ** 2


def test_time_domain_chirp_route():
    # Independent of the closed form: synthesise the chirp in the time
    # domain and FFT it.  The on-grid peak recovers ~|a|^2 at the injected
    # (r, z), and the drift direction/origin conventions must agree.
    N, M = 8192, 128
    for r0, z0 in [(3000.0, 12.0), (5000.0, -30.0), (1234.0, 0.0)]:
        A = syn.chirp_spectrum(N, [(np.sqrt(50.0), 0.0, r0, z0)])
        T = ot.templates(40.0, 2.0, M)
        zs = ot.z_grid(40.0, 2.0)
        P = direct.power(A, T)
        zz, rr = np.unravel_index(np.argmax(P), P.shape)
        assert zs[zz] == z0 and rr == int(r0)
        assert abs(P[zz, rr] / 50.0 - 1.0) < 5e-3


def test_parallelogram_law():
    A, B = _rand(2, 1500), _rand(3, 1500)
    T = syn.random_taps(4, 3, 16).astype(np.complex128)
    lhs = direct.power(A + B, T) + direct.power(A - B, T)
    rhs = 2 * direct.power(A, T) + 2 * direct.power(B, T)
    assert np.max(np.abs(lhs - rhs)) < 1e-11 * np.max(rhs)


def test_minus_z_is_plus_z_of_conjugate():
    A = _rand(5, 2000)
    T = ot.templates(30.0, 2.0, 64)
    P = direct.power(A, T)
    Pc = direct.power(np.conj(A), T)
    assert np.max(np.abs(P[::-1] - Pc)) < 1e-10 * np.max(P)


def test_shift_equivariance():
    A = _rand(6, 3000)
    T = syn.random_taps(7, 2, 32).astype(np.complex128)
    d = 37
    As = np.zeros_like(A)
    As[d:] = A[:-d]
    P, Ps = direct.power(A, T), direct.power(As, T)
    assert np.max(np.abs(Ps[:, 100 + d:2800] - P[:, 100:2800 - d])) < 1e-12 * np.max(P)


def test_noise_mean_power_is_template_energy():
    A = _rand(8, 1 << 17)
    T = ot.templates(40.0, 20.0, 128)
    P = direct.power(A, T)
    energy = np.sum(np.abs(T) ** 2, axis=1)
    mean = P[:, 128:-128].mean(axis=1)
    # exponential-ish statistics over ~1.3e5 correlated samples: a few %
    assert np.max(np.abs(mean / energy - 1.0)) < 0.05


def _overlap_save_dft(A, T, L):
    """The paper's overlap-save (Sec. 3, Fig. 1) with explicit O(L^2) DFT
    matrices: the filter's halves sit at the two ends of an L-array (centred
    on bin 0, zeros strictly between M/2 and L-M/2+1), windows overlap their
    neighbours by M/2 at each end with zero padding before the start, and
    the M contaminated edge outputs of each window are dropped."""
    K, M = T.shape
    N = len(A)
    B = L - M
    n = np.arange(L)
    F = np.exp(-2j * np.pi * np.outer(n, n) / L)
    Finv = np.conj(F)                      # IDFT printed without 1/L (Sec. 4.2)
    out = np.zeros((K, N), dtype=np.complex128)
    for z in range(K):
        h = np.zeros(L, dtype=np.complex128)
        for j in range(M):
            h[(M // 2 - j) % L] = np.conj(T[z, j])
        assert np.all(h[M // 2 + 1:L - M // 2 + 1] == 0)
        Hf = F @ h
        for s in range(-(-N // B)):
            start = s * B - M // 2
            a = np.zeros(L, dtype=np.complex128)
            for t in range(L):
                if 0 <= start + t < N:
                    a[t] = A[start + t]
            y = (Finv @ ((F @ a) * Hf)) / L
            for u in range(B):
                if s * B + u < N:
                    out[z, s * B + u] = y[u + M // 2]
    return out


@pytest.mark.parametrize("N,L,M", [(300, 64, 16), (97, 32, 8), (64, 64, 16), (5, 16, 4)])
def test_brute_force_overlap_save(N, L, M):
    A = _rand(9, N)
    T = syn.random_taps(10, 3, M).astype(np.complex128)
    Y = direct.correlate(A, T)
    Yos = _overlap_save_dft(A, T, L)
    assert np.max(np.abs(Y - Yos)) < 1e-12 * max(1.0, np.max(np.abs(Y)))


def test_literal_loops():
    A = _rand(11, 23)
    T = syn.random_taps(12, 2, 6).astype(np.complex128)
    K, M = T.shape
    Y = direct.correlate(A, T)
    for z in range(K):
        for r in range(len(A)):
            s = 0j
            for j in range(M):
                k = r + j - M // 2
                if 0 <= k < len(A):
                    s += A[k] * T[z, j].conjugate()
            assert abs(Y[z, r] - s) < 1e-14


def test_c_oracle_matches_numpy_oracle():
    A = _rand(13, 5000)
    T = ot.templates(10.0, 2.0, 64)
    P = direct.power(A, T)
    Pc = native.power(A, T)
    assert np.max(np.abs(P - Pc)) < 1e-12 * np.max(P)
    Pw = native.power(A, T, 1000, 1234)
    assert np.max(np.abs(Pw - P[:, 1000:1234])) < 1e-12 * np.max(P)
    rng = np.random.default_rng(0)
    zi = rng.integers(0, T.shape[0], 500)
    ri = rng.integers(0, len(A), 500)
    assert np.max(np.abs(native.power_points(A, T, zi, ri) - P[zi, ri])) < 1e-12 * np.max(P)
    Yc = native.correlate(A, T)
    assert np.max(np.abs(Yc - direct.correlate(A, T))) < 1e-12 * np.sqrt(np.max(P))
