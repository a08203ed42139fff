"""Seeded synthetic spectra shaped like the paper's workloads.

This module only draws random numbers and synthesises test signals.  It holds
none of the correlation arithmetic: it is shared by the FP64 oracle (tests,
CPU baseline) and the GPU path's tests and benchmark so that both see the
same input bytes.

Signal model (Sec. 2, eq. 22): a constant frequency-derivative signal whose
frequency drifts by ``z`` Fourier bins over the observation and sits at bin
``r`` at mid-observation,

    x(u) = a * exp(i*(phi + 2*pi*(r*u + z*(u*u - u)/2))),   u = n/N in [0, 1).

The spectrum of such a signal is obtained here the way a telescope pipeline
would get it: the complex time series is synthesised sample by sample and
Fourier transformed (numpy's FFT, divided by N so that an on-bin sinusoid of
amplitude a gives amplitude a).  Noise is complex white Gaussian with
E|A_k|^2 = 1, i.e. a normalised spectrum (Sec. 3 describes normalisation as
a step before the correlation).

Workloads (seed = workload number, numpy PCG64):
  1  one 2^16-bin spectrum, one signal r0=20000.3, z0=+8, |a|^2=50, phase 0;
     21 templates (z=-20..20 step 2), 64 taps, segment 512.
  2  one 2^21-bin spectrum, 16 signals r~U[1e4,2e6], z~U[-80,80], no two
     within 2M bins; 85 templates (z=-84..84 step 2), 256 taps, segment
     2048 or 4096.
  3  256 ragged spectra, N_b log-uniform in [2^18, 2^21], one signal each
     (r~U[0.05,0.95]*N_b, z~U[-60,60]); 85 templates x 256 taps.
  4  one 2^20-bin spectrum, one signal r=524288.4, z=20; 85 templates x 128
     taps, segment 512; loss weights w~U(0,1) of shape [K][N].

Also: random spectra and taps for edge cases, real time series (optionally
with a pulsed signal: harmonics h r0, h z0 of one constant-fdot signal) for
the real-to-complex front end, and unit-mean exponential power planes for
the steps that consume the plane.
  5  64 ragged spectra, N_b log-uniform in [2^21, 2^22], 4 signals each with
     z~U[-190,190]; 201 templates x 512 taps, segment 8192.

Draw order within a spectrum: noise real parts, noise imaginary parts, then
signal parameters.  For ragged workloads the lengths are drawn first from the
workload's stream; spectrum b then draws from its own stream, seeded with
(workload number, b), so spectra can be generated in parallel.
"""
from __future__ import annotations

import math
import os
from concurrent.futures import ThreadPoolExecutor
from dataclasses import dataclass, field

import numpy as np

AMP2 = 50.0  # |a|^2 of every injected signal: peak ~50x the mean noise power


@dataclass
class Workload:
    """One workload: spectra (complex64), search grid and segment length."""
    number: int
    spectra: list            # list of np.complex64 arrays
    zmax: float
    dz: float
    M: int
    L: int
    signals: list = field(default_factory=list)   # per spectrum: [(a, phi, r, z)]
    name: str = ""

    @property
    def K(self) -> int:
        return int(round(2 * self.zmax / self.dz)) + 1

    @property
    def lengths(self) -> np.ndarray:
        return np.array([len(s) for s in self.spectra], dtype=np.int64)

    def packed(self):
        """Concatenated spectra and int64 offsets[nspec+1]."""
        lens = self.lengths
        off = np.zeros(len(lens) + 1, dtype=np.int64)
        np.cumsum(lens, out=off[1:])
        return np.concatenate(self.spectra).astype(np.complex64), off


def noise(rng: np.random.Generator, n: int) -> np.ndarray:
    """Complex white noise with Re, Im ~ N(0, 1/2) (E|A|^2 = 1), complex128."""
    re = rng.normal(0.0, math.sqrt(0.5), n)
    im = rng.normal(0.0, math.sqrt(0.5), n)
    return re + 1j * im


def chirp_spectrum(n: int, signals) -> np.ndarray:
    """Spectrum (n bins) of a sum of constant-fdot complex sinusoids.

    ``signals`` is an iterable of (a, phi, r, z).  The time series is built
    sample by sample in FP64 and transformed with numpy's FFT / n.
    """
    u = np.arange(n, dtype=np.float64) / n
    x = np.zeros(n, dtype=np.complex128)
    quad = u * u - u
    for a, phi, r, z in signals:
        cycles = r * u + 0.5 * z * quad
        # reduce to [0,1) cycles before scaling by 2*pi to keep the phase exact
        cycles -= np.floor(cycles)
        x += a * np.exp(1j * (phi + 2.0 * np.pi * cycles))
    return np.fft.fft(x) / n


def _spectrum(rng, n, signals_fn):
    base = noise(rng, n)
    sigs = signals_fn(rng, n)
    if sigs:
        base = base + chirp_spectrum(n, sigs)
    return base.astype(np.complex64), sigs


def _separated(rng, count, lo, hi, min_sep, zlo, zhi, amp):
    """Draw ``count`` signals with r~U[lo,hi], z~U[zlo,zhi], phase~U(0,2pi),
    redrawing r until no two lie within ``min_sep`` bins."""
    rs = []
    while len(rs) < count:
        r = rng.uniform(lo, hi)
        if all(abs(r - q) >= min_sep for q in rs):
            rs.append(r)
    out = []
    for r in rs:
        z = rng.uniform(zlo, zhi)
        phi = rng.uniform(0.0, 2.0 * np.pi)
        out.append((amp, phi, r, z))
    return out


_RAGGED = {3: (256, 18, 21), 5: (64, 21, 22)}   # count, log2 of the length range


def _ragged_lengths(rng, number):
    count, lo, hi = _RAGGED[number]
    lens = np.floor(np.exp(rng.uniform(lo * math.log(2), hi * math.log(2), count)))
    return lens.astype(np.int64)


def ragged_lengths(number: int) -> np.ndarray:
    """The spectrum lengths of ragged workload 3 or 5 (the first draws of its
    stream), without synthesising the spectra."""
    return _ragged_lengths(np.random.default_rng(number), number)


def workload(number: int, L: int | None = None, nspec: int | None = None,
             length_scale: float = 1.0) -> Workload:
    """Build workload ``number`` (1..5).

    ``L`` overrides the segment length, ``nspec`` truncates ragged workloads
    to their first spectra (same draws), ``length_scale`` shrinks ragged
    lengths for quick tests (lengths are drawn first, then scaled).
    """
    rng = np.random.default_rng(number)
    amp = math.sqrt(AMP2)
    if number == 1:
        spec, sigs = _spectrum(rng, 1 << 16, lambda g, n: [(amp, 0.0, 20000.3, 8.0)])
        return Workload(1, [spec], 20.0, 2.0, 64, L or 512, [sigs],
                        "2^16 bins, 21 templates x 64 taps, segment 512")
    if number == 2:
        M = 256
        spec, sigs = _spectrum(rng, 1 << 21, lambda g, n: _separated(
            g, 16, 1e4, 2e6, 2 * M, -80.0, 80.0, amp))
        return Workload(2, [spec], 84.0, 2.0, M, L or 2048, [sigs],
                        "2^21 bins, 85 templates x 256 taps")
    if number in (3, 5):
        if number == 3:
            zr, nsig, zmax, M, Ld = 60.0, 1, 84.0, 256, 2048
        else:
            zr, nsig, zmax, M, Ld = 190.0, 4, 200.0, 512, 8192
        lens = _ragged_lengths(rng, number)
        if nspec is not None:
            lens = lens[:nspec]
        if length_scale != 1.0:
            lens = np.maximum((lens * length_scale).astype(np.int64), 1)
        def one(b, nb, nsig=nsig, zr=zr, M=M):
            g = np.random.default_rng([number, b])

            def sig_fn(g, n):
                if nsig == 1:
                    r = g.uniform(0.05, 0.95) * n
                    z = g.uniform(-zr, zr)
                    return [(amp, g.uniform(0.0, 2.0 * np.pi), r, z)]
                return _separated(g, nsig, 0.05 * n, 0.95 * n, 2 * M, -zr, zr, amp)

            return _spectrum(g, int(nb), sig_fn)

        workers = max(1, min(16, os.cpu_count() or 1))
        with ThreadPoolExecutor(max_workers=workers) as ex:
            done = list(ex.map(lambda bn: one(*bn), enumerate(lens)))
        specs = [d[0] for d in done]
        allsigs = [d[1] for d in done]
        name = (f"{len(specs)} ragged spectra, {int(2*zmax/2)+1} templates x {M} taps")
        return Workload(number, specs, zmax, 2.0, M, L or Ld, allsigs, name)
    if number == 4:
        spec, sigs = _spectrum(rng, 1 << 20, lambda g, n: [(amp, g.uniform(0, 2 * np.pi),
                                                            524288.4, 20.0)])
        return Workload(4, [spec], 84.0, 2.0, 128, L or 512, [sigs],
                        "2^20 bins, 85 templates x 128 taps, segment 512")
    raise ValueError(f"unknown workload {number}")


def time_series(seed: int, n: int, signals=(), sigma: float = 1.0,
                dtype=np.float32) -> np.ndarray:
    """A real time series of n samples for the real-to-complex front end:
    white Gaussian noise of standard deviation sigma plus real
    constant-fdot sinusoids a*cos(phi + 2*pi*(r*u + z*(u*u - u)/2)),
    u = t/n, from the same signal model as the spectra above.  ``signals``
    is an iterable of (a, phi, r, z); r is the mid-observation bin."""
    rng = np.random.default_rng(seed)
    x = rng.normal(0.0, sigma, n)
    u = np.arange(n, dtype=np.float64) / n
    quad = u * u - u
    for a, phi, r, z in signals:
        cycles = r * u + 0.5 * z * quad
        cycles -= np.floor(cycles)
        x += a * np.cos(phi + 2.0 * np.pi * cycles)
    return x.astype(dtype)


def loss_weights(number: int, K: int, n: int) -> np.ndarray:
    """Loss weights w ~ U(0,1), float32 [K][n], drawn from their own stream
    (seed 1000 + workload number) so the spectrum draws are unaffected."""
    rng = np.random.default_rng(1000 + number)
    return rng.random((K, n), dtype=np.float32)


def random_spectrum(seed: int, n: int, dtype=np.complex64) -> np.ndarray:
    """Plain complex white noise (E|A|^2 = 1) for edge-case tests."""
    rng = np.random.default_rng(seed)
    return noise(rng, n).astype(dtype)


def random_taps(seed: int, K: int, M: int) -> np.ndarray:
    """Arbitrary complex taps (not templates) for bank-independent tests."""
    rng = np.random.default_rng(seed)
    return (noise(rng, K * M) / math.sqrt(M)).reshape(K, M).astype(np.complex64)


def random_plane(seed: int, K: int, n: int) -> np.ndarray:
    """A [K][n] float32 power plane of unit-mean exponential values (the
    power statistics of normalised complex Gaussian noise), for tests and
    timings of the steps that consume the plane."""
    rng = np.random.default_rng([seed, K, n])
    return rng.exponential(size=(K, n)).astype(np.float32)


def pulsed_series(seed: int, n: int, r0: float, z0: float, harmonics: int, amp: float,
                  sigma: float = 1.0) -> np.ndarray:
    """Noise plus a pulsed constant-fdot signal: a sum of real sinusoids at
    the harmonics h = 1..harmonics of (r0, z0), i.e. at (h r0, h z0), each
    of amplitude amp and a seeded phase (a pulse train narrow enough that
    its first harmonics carry equal power)."""
    rng = np.random.default_rng([seed, 7])
    sig = [(amp, rng.uniform(0, 2 * np.pi), h * r0, h * z0) for h in range(1, harmonics + 1)]
    return time_series(seed, n, sig, sigma)
