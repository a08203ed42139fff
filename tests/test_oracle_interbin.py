"""Pins for the oracle's interbinned plane (Sec. 3, eq. f-interp)."""
import os

import numpy as np

import fdas_synth as syn
from oracle import direct, native
from oracle import templates as ot

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


def test_half_bin_signal_is_recovered_exactly():
    # z = 0 template is a delta, so Y = A; a z = 0 signal midway between
    # bins k0 and k0+1 has A_k0 = a 2i/pi and A_k0+1 = -a 2i/pi, and the
    # half-bin estimate (pi/4)(A_k0 - A_k0+1) has modulus exactly |a|.
    N, k0, a = 400, 200, 3.0 + 4.0j
    k = np.arange(N, dtype=np.float64)
    A = a * ot.response(k0 + 0.5 - k, 0.0)
    T = ot.templates(0.0, 2.0, 64)
    P2 = direct.interbinned_power(A, T)
    assert abs(P2[0, 2 * k0 + 1] - abs(a) ** 2) < 1e-12 * abs(a) ** 2
    assert abs(P2[0, 2 * k0] - abs(a) ** 2 * 4 / np.pi ** 2) < 1e-12 * abs(a) ** 2


def test_paper_maximum_losses():
    rows = {r.split()[0]: r.split()[1:] for r in open(os.path.join(GOLDEN, "interbinning_loss.txt"))
            if r.strip() and not r.startswith("#")}
    d = np.linspace(0.0, 1.0, 4001)
    N, k0 = 256, 100
    k = np.arange(N, dtype=np.float64)
    T = ot.templates(0.0, 2.0, 2)           # identity template: P2 from the spectrum itself
    plain_best, ib_best = [], []
    for dd in d:
        A = ot.response(k0 + dd - k, 0.0)
        P2 = direct.interbinned_power(A, T)[0]
        plain_best.append(np.sqrt(P2[0::2].max()))
        ib_best.append(np.sqrt(P2.max()))
    for name, best in (("plain", plain_best), ("interbinned", ib_best)):
        pct, digits = rows[name]
        loss = 100.0 * (1.0 - min(best))
        nd = int(digits)
        assert float(f"{loss:.{nd}g}") == float(pct), (name, loss)


def test_interbin_columns_by_literal_definition():
    A = syn.random_spectrum(3, 50).astype(np.complex128)
    T = syn.random_taps(4, 2, 8).astype(np.complex128)
    P2 = direct.interbinned_power(A, T)
    K, M = T.shape
    N = len(A)

    def y(z, r):
        s = 0j
        for j in range(M):
            kk = r + j - M // 2
            if 0 <= kk < N:
                s += A[kk] * np.conj(T[z, j])
        return s

    for z in range(K):
        for r in range(N):
            assert abs(P2[z, 2 * r] - abs(y(z, r)) ** 2) < 1e-12
            h = (np.pi / 4) * (y(z, r) - y(z, r + 1))
            assert abs(P2[z, 2 * r + 1] - abs(h) ** 2) < 1e-12


def test_c_interbin_points_match_numpy():
    A = syn.random_spectrum(5, 3000).astype(np.complex128)
    T = ot.templates(10.0, 2.0, 64)
    P2 = direct.interbinned_power(A, T)
    rng = np.random.default_rng(1)
    zi = rng.integers(0, T.shape[0], 3000)
    ci = np.concatenate([rng.integers(0, 6000, 2990), [0, 1, 5998, 5999, 2, 3, 4, 5, 6, 7]])
    got = native.interbin_points(A, T, zi, ci)
    assert np.max(np.abs(got - P2[zi, ci])) < 1e-12 * np.max(P2)
