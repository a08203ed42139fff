"""Pins for the harmonic-sum and candidate oracle (Sec. 3: harmonic summing,
threshold and peak search; readings in oracle/harmonic.py).

Closed forms on planes linear in r and z fix which rows and columns are
summed and how many terms; a planted harmonic comb must sum to its total at
its fundamental; flipping the z axis commutes with the sum; the fold domain
is the largest on which every harmonic exists.  Candidate selection is
pinned on planes whose peaks are known by construction (checkerboard,
plateau, diagonal neighbour, monotone ramp).  Mutants of the oracle with
plausible slips each fail at least one pin, while the oracle passes all.
"""
import numpy as np
import pytest

from oracle import harmonic as oh

FOLDS = (1, 2, 4, 8, 16)


def _ramp(K, N, a, b, d):
    c = (K - 1) // 2
    k = np.arange(K)[:, None]
    r = np.arange(N)[None, :]
    return (a * r + b * (k - c) + d).astype(np.float32)


# ---- pins as predicates --------------------------------------------------------


def pin_ramp(hsum):
    """P = a r + b (k - c) + d (small integers, exact in FP32) gives
    S_H = (a r + b (k - c)) H (H + 1)/2 + d H on the fold's domain."""
    for K, N in ((41, 300), (85, 1000), (201, 777)):
        c = (K - 1) // 2
        P = _ramp(K, N, 3, 5, 7)
        for H in FOLDS:
            try:
                S = hsum(P, H)
            except IndexError:
                return False
            KH, NH = oh.fold_shape(N, K, H)
            if S.shape != (KH, NH):
                return False
            k = (c - c // H + np.arange(KH))[:, None]
            r = np.arange(NH)[None, :]
            ref = (3 * r + 5 * (k - c)) * (H * (H + 1) // 2) + 7 * H
            if not np.array_equal(S, ref.astype(np.float32)):
                return False
    return True


def pin_identity(hsum):
    P = np.random.default_rng(1).random((21, 500), dtype=np.float32)
    return np.array_equal(hsum(P, 1), P)


def pin_comb(hsum):
    """Harmonics h = 1..8 of a fundamental (k0, r0) planted with power h
    (zeros elsewhere): S_H at (k0, r0) is sum_{h <= H} h, and the 8-fold sum
    peaks there (any other point collects a proper subset of the comb)."""
    K, N = 85, 4096
    c = (K - 1) // 2
    for k0, r0 in ((c + 3, 250), (c - 5, 301), (c, 77)):
        P = np.zeros((K, N), dtype=np.float32)
        for h in range(1, 9):
            P[c + h * (k0 - c), h * r0] = h
        for H in (1, 2, 4, 8):
            S = hsum(P, H)
            if S[k0 - (c - c // H), r0] != H * (H + 1) // 2:
                return False
        kk, rr = np.unravel_index(np.argmax(S), S.shape)
        if (kk + c - c // 8, rr) != (k0, r0):
            return False
    return True


def pin_flip(hsum):
    """Reversing the z axis of the plane reverses the rows of every fold."""
    P = np.random.default_rng(2).random((61, 640), dtype=np.float32)
    return all(np.array_equal(hsum(P[::-1], H), hsum(P, H)[::-1]) for H in FOLDS)


def pin_checkerboard(find):
    """On a 0/1 checkerboard every 1 equals its diagonal neighbours and
    exceeds its others: all of them, and only they, are peaks."""
    K, N = 9, 12
    P = ((np.arange(K)[:, None] + np.arange(N)[None, :]) % 2).astype(np.float32)
    got = find(P, 0.5)
    ref = np.argwhere(P > 0.5)
    return np.array_equal(got, ref)


def pin_local_structure(find):
    """A plateau of two equal maxima gives both; a point whose diagonal
    neighbour is larger is not a peak; values at the threshold are not
    candidates; edges and corners count."""
    P = np.zeros((6, 8), dtype=np.float32)
    P[2, 3] = P[2, 4] = 5.0          # plateau
    P[4, 6], P[5, 7] = 3.0, 4.0      # diagonal neighbour larger
    P[0, 0] = 2.0                    # corner
    P[5, 0] = 1.0                    # exactly at the threshold
    got = {tuple(x) for x in find(P, 1.0)}
    return got == {(2, 3), (2, 4), (5, 7), (0, 0)}


def pin_monotone(find):
    """A strictly increasing ramp has its only peak at the far corner."""
    P = _ramp(7, 9, 1, 10, 0)
    got = find(P, -1e9)
    return len(got) == 1 and tuple(got[0]) == (6, 8)


PINS_SUM = (pin_ramp, pin_identity, pin_comb, pin_flip)
PINS_PEAK = (pin_checkerboard, pin_local_structure, pin_monotone)


# ---- the oracle passes every pin -----------------------------------------------


@pytest.mark.parametrize("pin", PINS_SUM, ids=lambda p: p.__name__)
def test_sum_oracle_passes(pin):
    assert pin(oh.harmonic_sum)


@pytest.mark.parametrize("pin", PINS_PEAK, ids=lambda p: p.__name__)
def test_peak_oracle_passes(pin):
    assert pin(oh.peaks)


def test_fold_domain_is_the_largest_valid_one():
    for N in (1, 2, 15, 16, 17, 1000, 4097):
        for K in (1, 3, 21, 85, 201):
            c = (K - 1) // 2
            for H in FOLDS:
                KH, NH = oh.fold_shape(N, K, H)
                assert H * (NH - 1) <= N - 1 < H * NH       # h r < N for all h <= H
                half = (KH - 1) // 2
                assert H * half <= c < H * (half + 1)       # |h (k - c)| <= c


def test_fp32_sum_tracks_the_fp64_sum():
    P = np.random.default_rng(3).exponential(size=(85, 5000)).astype(np.float32)
    for H in FOLDS:
        a, b = oh.harmonic_sum(P, H), oh.harmonic_sum_f64(P, H)
        assert np.max(np.abs(a - b) / b) < 4e-7 * H


def test_noise_sums_have_gamma_moments():
    # unit-mean exponential powers (|A|^2 of N(0,1/2) complex noise): the
    # H-fold sum has mean H and variance H
    P = np.random.default_rng(4).exponential(size=(201, 20000)).astype(np.float32)
    for H in (2, 4, 8):
        S = oh.harmonic_sum_f64(P, H)
        n = S.size
        assert abs(S.mean() - H) < 6 * np.sqrt(H / n)
        assert abs(S.var() / H - 1) < 0.05


# ---- mutants: each fails some pin ----------------------------------------------


def _sum_rows_times_k(P, H):
    # harmonic rows at h k instead of c + h (k - c)
    K, N = P.shape
    c = (K - 1) // 2
    KH, NH = oh.fold_shape(N, K, H)
    k = (c - c // H + np.arange(KH))[:, None]
    r = np.arange(NH)[None, :]
    S = np.zeros((KH, NH), np.float32)
    for h in range(1, H + 1):
        S = S + P[np.minimum(h * k, K - 1), h * r]
    return S


def _sum_z_unscaled(P, H):
    # harmonics taken at the fundamental's template row
    K, N = P.shape
    c = (K - 1) // 2
    KH, NH = oh.fold_shape(N, K, H)
    k = (c - c // H + np.arange(KH))[:, None]
    r = np.arange(NH)[None, :]
    S = np.zeros((KH, NH), np.float32)
    for h in range(1, H + 1):
        S = S + P[k + 0 * r, h * r]
    return S


def _sum_from_h0(P, H):
    # h = 0 .. H-1
    K, N = P.shape
    c = (K - 1) // 2
    KH, NH = oh.fold_shape(N, K, H)
    k = (c - c // H + np.arange(KH))[:, None]
    r = np.arange(NH)[None, :]
    S = np.zeros((KH, NH), np.float32)
    for h in range(0, H):
        S = S + P[c + h * (k - c), h * r]
    return S


def _sum_domain_from_row0(P, H):
    # fold rows counted from row 0 of the plane instead of centred on z = 0
    K, N = P.shape
    c = (K - 1) // 2
    KH, NH = oh.fold_shape(N, K, H)
    k = np.arange(KH)[:, None]
    r = np.arange(NH)[None, :]
    S = np.zeros((KH, NH), np.float32)
    for h in range(1, H + 1):
        S = S + P[np.clip(c + h * (k - c), 0, K - 1), h * r]
    return S


def _peaks_strict(S, thr):
    S = np.asarray(S, np.float32)
    pad = np.full((S.shape[0] + 2, S.shape[1] + 2), -np.inf, np.float32)
    pad[1:-1, 1:-1] = S
    ok = S > thr
    for dk in (-1, 0, 1):
        for dr in (-1, 0, 1):
            if dk or dr:
                ok &= S > pad[1 + dk:1 + dk + S.shape[0], 1 + dr:1 + dr + S.shape[1]]
    return np.argwhere(ok)


def _peaks_four_neighbours(S, thr):
    S = np.asarray(S, np.float32)
    pad = np.full((S.shape[0] + 2, S.shape[1] + 2), -np.inf, np.float32)
    pad[1:-1, 1:-1] = S
    ok = S > thr
    for dk, dr in ((-1, 0), (1, 0), (0, -1), (0, 1)):
        ok &= S >= pad[1 + dk:1 + dk + S.shape[0], 1 + dr:1 + dr + S.shape[1]]
    return np.argwhere(ok)


def _peaks_threshold_inclusive(S, thr):
    S = np.asarray(S, np.float32)
    pad = np.full((S.shape[0] + 2, S.shape[1] + 2), -np.inf, np.float32)
    pad[1:-1, 1:-1] = S
    ok = S >= thr
    for dk in (-1, 0, 1):
        for dr in (-1, 0, 1):
            if dk or dr:
                ok &= S >= pad[1 + dk:1 + dk + S.shape[0], 1 + dr:1 + dr + S.shape[1]]
    return np.argwhere(ok)


@pytest.mark.parametrize("mutant", [_sum_rows_times_k, _sum_z_unscaled, _sum_from_h0,
                                    _sum_domain_from_row0], ids=lambda m: m.__name__)
def test_sum_mutant_fails_a_pin(mutant):
    assert not all(pin(mutant) for pin in PINS_SUM)


@pytest.mark.parametrize("mutant", [_peaks_strict, _peaks_four_neighbours,
                                     _peaks_threshold_inclusive],
                         ids=lambda m: m.__name__)
def test_peak_mutant_fails_a_pin(mutant):
    assert not all(pin(mutant) for pin in PINS_PEAK)
