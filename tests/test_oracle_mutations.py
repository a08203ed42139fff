"""Mutation checks for the oracle's pins.

Each mutant below is the oracle with one plausible mistake planted in it
(here, on the CPU): a dropped conjugate, a window off by one bin, reflected
taps, the wrong sign of the chirp phase, a symmetric time origin, the
frequency referenced to the start of the observation, a wrong interbinning
sign, factor or neighbour, slips in the adjoint, and a wrong exponent sign or
time origin in the real-to-complex transform.  For each, at least one
of the pins that guard the oracle must fail, while the oracle itself passes
all of them -- so the pins can tell these mistakes from the method.
"""
import numpy as np
import pytest

import fdas_synth as syn
from oracle import direct, r2c
from oracle import templates as ot
from tests.quadrature import response_quadrature

# ---- pins as predicates (the same checks as the oracle's own tests) ----------


def pin_chirp(power, templates):
    """Time-domain chirps: the plane's maximum sits at the injected (r, z)
    and recovers ~|a|^2 there (Sec. 2 signal model, Sec. 3)."""
    N, M = 8192, 128
    for r0, z0 in [(3000.0, 12.0), (5000.0, -30.0), (1234.0, 0.0)]:
        A = syn.chirp_spectrum(N, [(np.sqrt(50.0), 0.0, r0, z0)])
        P = power(A, templates(40.0, 2.0, M))
        zz, rr = np.unravel_index(np.argmax(P), P.shape)
        if not (ot.z_grid(40.0, 2.0)[zz] == z0 and rr == int(r0)
                and abs(P[zz, rr] / 50.0 - 1.0) < 5e-3):
            return False
    return True


def pin_quadrature(response):
    """Closed form against quadrature of the defining integral."""
    q = np.arange(-40.0, 41.0)
    for z in (-20.0, -2.0, 0.0, 6.0, 30.0):
        if np.max(np.abs(response(q, z) - response_quadrature(q, z))) > 1e-10:
            return False
    return True


def pin_half_bin(interbinned_power):
    """A z = 0 signal midway between two bins is recovered exactly at the
    interbinned column, and the bin itself shows 4/pi^2 of it (Sec. 3)."""
    N, k0, a = 400, 200, 3.0 + 4.0j
    A = a * ot.response(k0 + 0.5 - np.arange(N, dtype=np.float64), 0.0)
    P2 = interbinned_power(A, ot.templates(0.0, 2.0, 64))
    return (abs(P2[0, 2 * k0 + 1] - abs(a) ** 2) < 1e-12 * abs(a) ** 2
            and abs(P2[0, 2 * k0] - abs(a) ** 2 * 4 / np.pi ** 2) < 1e-12 * abs(a) ** 2)


def _fd(f, x, h=1.0):
    g = np.zeros_like(x)
    flat, gf = x.reshape(-1), g.reshape(-1)
    for i in range(flat.size):
        for unit in (1.0, 1j):
            xp, xm = flat.copy(), flat.copy()
            xp[i] += unit * h
            xm[i] -= unit * h
            gf[i] += unit * (f(xp.reshape(x.shape)) - f(xm.reshape(x.shape))) / (2 * h)
    return g


def pin_finite_differences(grads):
    """Both gradients against central differences of the loss (exact for a
    quadratic form)."""
    rng = np.random.default_rng(0)
    N, K, M = 30, 2, 6
    A = (rng.normal(size=N) + 1j * rng.normal(size=N)) / np.sqrt(2)
    T = (rng.normal(size=(K, M)) + 1j * rng.normal(size=(K, M))) / np.sqrt(2 * M)
    w = rng.random((K, N))
    gA, gT = grads(A, T, w)
    fA = _fd(lambda a: direct.loss(a, T, w), A)
    fT = _fd(lambda t: direct.loss(A, t, w), T)
    return (np.max(np.abs(gA - fA)) < 1e-9 * np.max(np.abs(fA))
            and np.max(np.abs(gT - fT)) < 1e-9 * np.max(np.abs(fT)))


# ---- mutants ---------------------------------------------------------------------


def _power_with(correlate):
    return lambda A, T: np.abs(correlate(A, T)) ** 2


def corr_dropped_conj(A, T):
    return direct.correlate(A, np.conj(T))


def corr_window_off_by_one(A, T):
    A = np.asarray(A, dtype=np.complex128)
    return direct.correlate(np.concatenate([A[1:], [0.0]]), T)


def corr_reflected_taps(A, T):
    return direct.correlate(A, np.asarray(T)[:, ::-1])


def response_phase_sign(q, z):
    return np.conj(ot.response(q, z))


def response_symmetric_origin(q, z):
    q = np.asarray(q, dtype=np.float64)
    return ot.response(q, z) * np.exp(1j * np.pi * q)


def response_start_reference(q, z):
    return ot.response(np.asarray(q, dtype=np.float64) + 0.5 * z, z)


def _templates_with(response):
    def templates(zmax, dz, M):
        e = ot.tap_offsets(M)
        return np.stack([response(e, z) for z in ot.z_grid(zmax, dz)])
    return templates


def _ib(half):
    def interbinned_power(A, T):
        A = np.asarray(A, dtype=np.complex128)
        N = len(A)
        Y = direct.correlate(np.concatenate([[0.0], A, [0.0]]), T)   # Y[:, r + 1] = Y_r
        P2 = np.empty((Y.shape[0], 2 * N))
        P2[:, 0::2] = np.abs(Y[:, 1:N + 1]) ** 2
        P2[:, 1::2] = half(Y[:, 1:N + 1], Y[:, 2:N + 2], Y[:, 0:N])
        return P2
    return interbinned_power


ib_sign = _ib(lambda y, yn, yp: np.abs((np.pi / 4) * (y + yn)) ** 2)
ib_no_factor = _ib(lambda y, yn, yp: np.abs(y - yn) ** 2)
ib_left_neighbour = _ib(lambda y, yn, yp: np.abs((np.pi / 4) * (y - yp)) ** 2)


def grads_conj_taps_in_adjoint(A, T, w):
    gA, _ = direct.grads(A, np.conj(T), w)
    _, gT = direct.grads(A, T, w)
    return gA, gT


def grads_missing_factor_two(A, T, w):
    gA, gT = direct.grads(A, T, w)
    return gA / 2, gT / 2


def grads_unconjugated_taps_gradient(A, T, w):
    gA, gT = direct.grads(A, T, w)
    return gA, np.conj(gT)


def pin_r2c(dft):
    """Real-to-complex transform: a shifted impulse gives the phase ramp and
    a cosine on bin k0 gives (n/2) e^{i phi} at k0 (closed forms)."""
    n, t0, k0, phi = 64, 5, 9, 0.4
    x = np.zeros(n)
    x[t0] = 1.0
    k = np.arange(n // 2 + 1)
    ok = np.max(np.abs(dft(x) - np.exp(-2j * np.pi * k * t0 / n))) < 1e-12
    t = np.arange(n)
    ref = np.zeros(n // 2 + 1, dtype=complex)
    ref[k0] = 0.5 * n * np.exp(1j * phi)
    return ok and np.max(np.abs(dft(np.cos(2 * np.pi * k0 * t / n + phi)) - ref)) < 1e-11


def r2c_wrong_exponent_sign(x):
    return np.conj(r2c.dft(x))


def r2c_time_index_from_one(x):
    return r2c.dft(np.roll(np.asarray(x, dtype=np.float64), 1))


def pin_fourier2(fi):
    """Half-bin column of the two-bin interpolation: an accelerated signal at
    k0 + 1/2 gives (sum over the window of |R(q, z0)|^2)^2, by quadrature."""
    N, k0, M, z0 = 300, 150, 32, 8.0
    A = ot.response(k0 + 0.5 - np.arange(N, dtype=np.float64), z0)
    P2 = fi(A, 10.0, 2.0, M)
    zi = int(np.argmin(np.abs(ot.z_grid(10.0, 2.0) - z0)))
    q = M / 2 - 0.5 - np.arange(M, dtype=np.float64)
    E = np.sum(np.abs(response_quadrature(q, z0)) ** 2)
    return abs(P2[zi, 2 * k0 + 1] - E ** 2) < 1e-9


def fourier2_reversed_offset(A, zmax, dz, M):
    # the half-bin response taken at k - r - 1/2 instead of r + 1/2 - k
    A = np.asarray(A, dtype=np.complex128)
    return direct.fourier_interpolated_power(np.conj(A[::-1]), zmax, dz, M)[:, ::-1]


def fourier2_window_off_by_one(A, zmax, dz, M):
    A = np.asarray(A, dtype=np.complex128)
    P2 = direct.fourier_interpolated_power(A, zmax, dz, M)
    P2[:, 1::2] = np.roll(P2[:, 1::2], 1, axis=1)
    return P2


MUTANTS = {
    "fourier2 offset sign": lambda: pin_fourier2(fourier2_reversed_offset),
    "fourier2 window shift": lambda: pin_fourier2(fourier2_window_off_by_one),
    "r2c exponent sign": lambda: pin_r2c(r2c_wrong_exponent_sign),
    "r2c time origin": lambda: pin_r2c(r2c_time_index_from_one),
    "dropped conj": lambda: pin_chirp(_power_with(corr_dropped_conj), ot.templates),
    "window off by one": lambda: pin_chirp(_power_with(corr_window_off_by_one), ot.templates),
    "reflected taps": lambda: pin_chirp(_power_with(corr_reflected_taps), ot.templates),
    "chirp phase sign": lambda: (pin_quadrature(response_phase_sign)
                                 and pin_chirp(direct.power, _templates_with(response_phase_sign))),
    "symmetric time origin": lambda: (
        pin_quadrature(response_symmetric_origin)
        and pin_chirp(direct.power, _templates_with(response_symmetric_origin))),
    "start-of-observation reference": lambda: (
        pin_quadrature(response_start_reference)
        and pin_chirp(direct.power, _templates_with(response_start_reference))),
    "interbinning sign": lambda: pin_half_bin(ib_sign),
    "interbinning factor": lambda: pin_half_bin(ib_no_factor),
    "interbinning neighbour": lambda: pin_half_bin(ib_left_neighbour),
    "adjoint with conj(T)": lambda: pin_finite_differences(grads_conj_taps_in_adjoint),
    "adjoint missing factor 2": lambda: pin_finite_differences(grads_missing_factor_two),
    "taps gradient conjugated": lambda: pin_finite_differences(grads_unconjugated_taps_gradient),
}


def test_oracle_passes_every_pin():
    assert pin_chirp(direct.power, ot.templates)
    assert pin_quadrature(ot.response)
    assert pin_half_bin(direct.interbinned_power)
    assert pin_half_bin(_ib(lambda y, yn, yp: np.abs((np.pi / 4) * (y - yn)) ** 2))
    assert pin_finite_differences(direct.grads)
    assert pin_r2c(r2c.dft)
    assert pin_fourier2(direct.fourier_interpolated_power)


@pytest.mark.parametrize("name", sorted(MUTANTS))
def test_pins_reject_mutant(name):
    assert not MUTANTS[name](), name
