"""The HIP kernel sources, compiled for the CPU emulation in tests/emu (each
workgroup runs as host threads with a barrier for __syncthreads), driven
through the same C ABI with host arrays and checked against the FP64 oracle.

This checks the kernels' indexing, masking, batching and adjoint data flow
where no GPU is present.  It says nothing about GPU execution; the GPU parity
tests (tests/test_gpu_*.py) do that.
"""
import ctypes
import os

import numpy as np
import pytest

import fdas_synth as syn
from oracle import native
from oracle import templates as ot

HERE = os.path.dirname(os.path.abspath(__file__))
TOL = 1e-5


@pytest.fixture(scope="module")
def emu():
    from tests.emu import build_emu
    path = build_emu.build()
    L = ctypes.CDLL(path)
    return L


def _p(a):
    return a.ctypes.data_as(ctypes.c_void_p)


def _bank(emu, taps, L):
    K, M = taps.shape
    taps = np.ascontiguousarray(taps, dtype=np.complex64)
    bank = np.zeros((K + 1) * L, dtype=np.complex64)
    assert emu.fdas_prepare_bank(_p(taps), K, M, L, _p(bank), None) == 0
    return bank


GUARD = 1 << 14      # floats of sentinel on each side of an output buffer
SENTINEL = np.float32(-12345.0)


def _guarded(shape):
    """An output array (NaN-filled, so unwritten outputs fail the comparison)
    inside a larger buffer whose margins hold a sentinel: any store outside
    the array, before or after it, shows up in the margins."""
    n = int(np.prod(shape))
    buf = np.full(n + 2 * GUARD, SENTINEL, dtype=np.float32)
    buf[GUARD:GUARD + n] = np.nan
    return buf, buf[GUARD:GUARD + n].reshape(shape)


def _check_guards(buf, arr):
    n = arr.size
    assert np.all(buf[:GUARD] == SENTINEL) and np.all(buf[GUARD + n:] == SENTINEL)


def _rel(got, ref):
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


@pytest.mark.parametrize("L,M,N,grid", [(256, 32, 1000, 0), (512, 64, 449, 2), (2048, 256, 3900, 0),
                                        (256, 128, 300, 1), (1024, 2, 2000, 7), (512, 64, 2000, 40)])
def test_emulated_forward_vs_oracle(emu, L, M, N, grid):
    K = 3
    A = syn.random_spectrum(L + N, N)
    taps = syn.random_taps(M + K, K, M)
    bank = _bank(emu, taps, L)
    buf, plane = _guarded((K, N))
    assert emu.fdas_correlate_ex(_p(A), ctypes.c_int64(N), _p(bank), K, M, L, _p(plane),
                                 grid, None) == 0
    _check_guards(buf, plane)
    assert _rel(plane, native.power(A, taps)) < TOL


@pytest.mark.parametrize("seed", range(6))
def test_emulated_forward_random_shapes(emu, seed):
    # seeded random geometry: segment length, even tap count up to L/2,
    # spectrum length (ragged tail, sometimes shorter than one segment),
    # template count and persistent grid; the plane against the oracle
    rng = np.random.default_rng(seed + 500)
    L = int(rng.choice([256, 512, 1024, 2048]))
    M = 2 * int(rng.integers(1, L // 4 + 1))
    N = int(rng.integers(1, 3 * (L - M) + 7))
    K = int(rng.integers(1, 6))
    grid = int(rng.integers(0, 9))
    A = syn.random_spectrum(seed + 900, N)
    taps = syn.random_taps(seed + 901, K, M)
    bank = _bank(emu, taps, L)
    buf, plane = _guarded((K, N))
    assert emu.fdas_correlate_ex(_p(A), ctypes.c_int64(N), _p(bank), K, M, L, _p(plane),
                                 grid, None) == 0, (L, M, N, K, grid)
    _check_guards(buf, plane)
    assert _rel(plane, native.power(A, taps)) < TOL, (L, M, N, K, grid)


def test_emulated_templates_forward_workload1_slice(emu):
    # the library's own templates and bank on a 4000-bin slice of workload 1
    w = syn.workload(1)
    A = np.ascontiguousarray(w.spectra[0][18000:22000])
    K, M, L = w.K, w.M, w.L
    taps = np.zeros((K, M), dtype=np.complex64)
    bank = np.zeros((K + 1) * L, dtype=np.complex64)
    assert emu.fdas_make_templates(ctypes.c_double(w.zmax), ctypes.c_double(w.dz), M, L,
                                   _p(taps), _p(bank), None) == 0
    plane = np.zeros((K, len(A)), dtype=np.float32)
    assert emu.fdas_correlate(_p(A), ctypes.c_int64(len(A)), _p(bank), K, M, L, _p(plane), None) == 0
    ref = native.power(A, ot.templates(w.zmax, w.dz, M))
    assert _rel(plane, ref) < TOL
    zz, rr = np.unravel_index(np.argmax(plane), plane.shape)
    assert (zz, rr) == (14, 2000)        # z = +8, r = 20000 - 18000


def test_emulated_batched_equals_plain(emu):
    L, M, K = 512, 64, 3
    lens = [700, 0, 1, 448, 1203, 5]
    taps = syn.random_taps(7, K, M)
    bank = _bank(emu, taps, L)
    specs = [syn.random_spectrum(10 + i, n) for i, n in enumerate(lens)]
    packed = np.concatenate(specs).astype(np.complex64)
    offs = np.zeros(len(lens) + 1, dtype=np.int64)
    offs[1:] = np.cumsum(lens)
    buf, planes = _guarded((K * offs[-1],))
    emu.fdas_batched_workspace_bytes.restype = ctypes.c_size_t
    wsb = emu.fdas_batched_workspace_bytes(len(lens))
    ws = np.zeros(wsb, dtype=np.uint8)
    for grid in (0, 1, 5, 13):
        planes[:] = np.nan
        assert emu.fdas_correlate_batched_ex(_p(packed), _p(offs), len(lens),
                                             ctypes.c_int64(int(offs[-1])), _p(bank), K, M, L,
                                             _p(planes), 0, grid, _p(ws), ctypes.c_size_t(wsb),
                                             None) == 0
        _check_guards(buf, planes)
        for b, n in enumerate(lens):
            if n == 0:
                continue
            view = planes[K * offs[b]:K * offs[b + 1]].reshape(K, n)
            one = np.zeros((K, n), dtype=np.float32)
            assert emu.fdas_correlate(_p(specs[b]), ctypes.c_int64(n), _p(bank), K, M, L,
                                      _p(one), None) == 0
            assert np.array_equal(view, one), b
            assert _rel(view, native.power(specs[b], taps)) < TOL


def test_emulated_batched_noalloc_equals_workspace_call(emu):
    # the allocation-free entry point (its segment prefix in the library's
    # device array) against the workspace form, twice in a row, the second
    # batch smaller: no state carries over between calls
    L, M, K = 512, 64, 3
    taps = syn.random_taps(11, K, M)
    bank = _bank(emu, taps, L)
    emu.fdas_batched_workspace_bytes.restype = ctypes.c_size_t
    for call, lens in enumerate(([700, 0, 1, 448, 1203, 5], [97, 449])):
        specs = [syn.random_spectrum(30 + 10 * call + i, n) for i, n in enumerate(lens)]
        packed = np.concatenate(specs).astype(np.complex64)
        offs = np.zeros(len(lens) + 1, dtype=np.int64)
        offs[1:] = np.cumsum(lens)
        tot = int(offs[-1])
        wsb = emu.fdas_batched_workspace_bytes(len(lens))
        ws = np.zeros(wsb, dtype=np.uint8)
        ref = np.zeros(K * tot, dtype=np.float32)
        assert emu.fdas_correlate_batched_ex(_p(packed), _p(offs), len(lens), ctypes.c_int64(tot),
                                             _p(bank), K, M, L, _p(ref), 0, 0, _p(ws),
                                             ctypes.c_size_t(wsb), None) == 0
        buf, got = _guarded((K * tot,))
        assert emu.fdas_correlate_batched_noalloc(_p(packed), _p(offs), len(lens),
                                                  ctypes.c_int64(tot), _p(bank), K, M, L,
                                                  _p(got), None) == 0
        _check_guards(buf, got)
        assert np.array_equal(got, ref), call
    # past the fixed array: rejected before any launch
    big = 65537
    offs = np.zeros(big + 1, dtype=np.int64)
    planes = np.zeros(1, dtype=np.float32)
    spec = np.zeros(1, dtype=np.complex64)
    assert emu.fdas_correlate_batched_noalloc(_p(spec), _p(offs), big, ctypes.c_int64(0),
                                              _p(bank), K, M, L, _p(planes), None) != 0

@pytest.mark.parametrize("L,E", [(1024, 8), (2048, 8), (1024, 16), (8192, 8), (4096, 8)])
def test_emulated_batched_values_per_lane(emu, L, E):
    # the other lane geometry of the batched kernel: same plane up to FP32
    # rounding, every element written, nothing outside the buffer
    M, K = 256, 3
    lens = [1900, 1, 770, 0, 2600]
    taps = syn.random_taps(L + E, K, M)
    bank = _bank(emu, taps, L)
    specs = [syn.random_spectrum(40 + i, n) for i, n in enumerate(lens)]
    packed = np.concatenate(specs).astype(np.complex64)
    offs = np.zeros(len(lens) + 1, dtype=np.int64)
    offs[1:] = np.cumsum(lens)
    buf, planes = _guarded((K * offs[-1],))
    emu.fdas_batched_workspace_bytes.restype = ctypes.c_size_t
    wsb = emu.fdas_batched_workspace_bytes(len(lens))
    ws = np.zeros(wsb, dtype=np.uint8)
    assert emu.fdas_correlate_batched_ex(_p(packed), _p(offs), len(lens),
                                         ctypes.c_int64(int(offs[-1])), _p(bank), K, M, L,
                                         _p(planes), E, 0, _p(ws), ctypes.c_size_t(wsb),
                                         None) == 0
    _check_guards(buf, planes)
    for b, n in enumerate(lens):
        if n:
            view = planes[K * offs[b]:K * offs[b + 1]].reshape(K, n)
            assert _rel(view, native.power(specs[b], taps)) < TOL, b


def test_emulated_batched_offsets_clamped_to_capacity(emu):
    # offsets the device reads past the caller's capacity: the spectra are
    # cut at the capacity, nothing is written beyond K * capacity floats
    L, M, K = 512, 64, 2
    lens = [300, 500]
    taps = syn.random_taps(3, K, M)
    bank = _bank(emu, taps, L)
    packed = syn.random_spectrum(4, sum(lens))
    cap = 600
    offs = np.array([0, 300, 5000], dtype=np.int64)
    buf, planes = _guarded((K * cap,))
    wsb = emu.fdas_batched_workspace_bytes(2)
    ws = np.zeros(wsb, dtype=np.uint8)
    assert emu.fdas_correlate_batched_ex(_p(packed), _p(offs), 2, ctypes.c_int64(cap), _p(bank),
                                         K, M, L, _p(planes), 0, 0, _p(ws),
                                         ctypes.c_size_t(wsb), None) == 0
    _check_guards(buf, planes)
    second = planes[K * 300:K * 600].reshape(K, 300)
    assert _rel(second, native.power(packed[300:600], taps)) < TOL


@pytest.mark.parametrize("L,M,zchunk", [(512, 128, 2), (256, 32, 1), (1024, 64, 3), (512, 64, 0)])
def test_emulated_backward_batched(emu, L, M, zchunk):
    # the batched adjoint: each spectrum's gradient bitwise the single-spectrum
    # call's with the same template chunking, the taps gradient the batch sum,
    # both against the oracle; empty and one-bin spectra included
    K = 3
    lens = [700, 0, 1, 2 * (L - M) + 5, 97]
    taps = syn.random_taps(L + M, K, M)
    bank = _bank(emu, taps, L)
    specs = [syn.random_spectrum(60 + i, n) for i, n in enumerate(lens)]
    packed = np.concatenate(specs).astype(np.complex64)
    offs = np.zeros(len(lens) + 1, dtype=np.int64)
    offs[1:] = np.cumsum(lens)
    tot = int(offs[-1])
    rng = np.random.default_rng(L + M)
    ws_ = [rng.random((K, n), dtype=np.float32) for n in lens]
    wpk = np.concatenate([w.reshape(-1) for w in ws_]).astype(np.float32)
    emu.fdas_backward_batched_workspace_bytes.restype = ctypes.c_size_t
    wsb = emu.fdas_backward_batched_workspace_bytes(ctypes.c_int64(tot), len(lens), K, M, L,
                                                    zchunk, 3)
    ws = np.zeros(wsb + 256, dtype=np.uint8)
    wsp = ctypes.c_void_p((ws.ctypes.data + 255) & ~255)
    gbuf, gA = _guarded((2 * tot,))            # complex64 as float pairs
    gT = np.full((K, M), np.nan, dtype=np.complex64)
    assert emu.fdas_correlate_backward_batched(_p(packed), _p(offs), len(lens),
                                               ctypes.c_int64(tot), _p(bank), K, M, L, _p(wpk),
                                               _p(gA), _p(gT), zchunk, wsp, ctypes.c_size_t(wsb),
                                               None) == 0
    _check_guards(gbuf, gA)
    gA = gA.view(np.complex64)
    emu.fdas_backward_workspace_bytes.restype = ctypes.c_size_t
    sumT = np.zeros((K, M), dtype=np.complex128)
    for b, n in enumerate(lens):
        if n == 0:
            continue
        # the batch's default chunking is the single call's only when given
        zc = zchunk if zchunk else K
        w1 = emu.fdas_backward_workspace_bytes(ctypes.c_int64(n), K, M, L, zc)
        ws1 = np.zeros(w1 + 256, dtype=np.uint8)
        p1 = ctypes.c_void_p((ws1.ctypes.data + 255) & ~255)
        a1 = np.full(n, np.nan, dtype=np.complex64)
        t1 = np.full((K, M), np.nan, dtype=np.complex64)
        assert emu.fdas_correlate_backward_ex(_p(specs[b]), ctypes.c_int64(n), _p(bank), K, M, L,
                                              _p(ws_[b]), _p(a1), _p(t1), zc, p1,
                                              ctypes.c_size_t(w1), None) == 0
        if zchunk:
            assert np.array_equal(gA[offs[b]:offs[b + 1]], a1), b
        rA, rT = native.grads(specs[b], taps, ws_[b])
        assert _rel(gA[offs[b]:offs[b + 1]], rA) < TOL, b
        sumT += rT
    assert _rel(gT, sumT) < TOL
    # spectra gradient alone: same values
    gA2 = np.full(tot, np.nan, dtype=np.complex64)
    assert emu.fdas_correlate_backward_batched(_p(packed), _p(offs), len(lens),
                                               ctypes.c_int64(tot), _p(bank), K, M, L, _p(wpk),
                                               _p(gA2), None, zchunk, wsp, ctypes.c_size_t(wsb),
                                               None) == 0
    assert np.allclose(gA2, gA, rtol=0, atol=1e-6 * np.max(np.abs(gA)))


def test_emulated_backward_batched_empty_batch(emu):
    # no spectra: zero gradients, every output written
    K, M, L, cap = 2, 64, 512, 50
    taps = syn.random_taps(1, K, M)
    bank = _bank(emu, taps, L)
    offs = np.zeros(1, dtype=np.int64)
    wsb = emu.fdas_backward_batched_workspace_bytes(ctypes.c_int64(cap), 0, K, M, L, 0, 3)
    ws = np.zeros(wsb + 256, dtype=np.uint8)
    wsp = ctypes.c_void_p((ws.ctypes.data + 255) & ~255)
    spec = np.zeros(cap, dtype=np.complex64)
    w = np.zeros(K * cap, dtype=np.float32)
    gA = np.full(cap, np.nan, dtype=np.complex64)
    gT = np.full((K, M), np.nan, dtype=np.complex64)
    assert emu.fdas_correlate_backward_batched(_p(spec), _p(offs), 0, ctypes.c_int64(cap),
                                               _p(bank), K, M, L, _p(w), _p(gA), _p(gT), 0, wsp,
                                               ctypes.c_size_t(wsb), None) == 0
    assert np.all(gA == 0) and np.all(gT == 0)


# (256, 32, 29131): 131 windows, so the taps-gradient reduction runs in two
# window chunks
# M = L/4 at 8 values per lane puts M/2 on exactly one lane slot at each end
# (512/128, 1024/256, 2048/512): the kernels specialised for those edge slots
# M/2 = T (512/128, 256/128) runs the windows in groups of three that share
# one taps transform per template: 2, 7, 5 and 8 windows leave groups of 2,
# 1, 2 and 2 at the end
@pytest.mark.parametrize("L,M,N", [(256, 32, 900), (512, 128, 600), (2048, 256, 2500),
                                   (256, 32, 29131), (1024, 256, 1500), (2048, 512, 2600),
                                   (512, 128, 2500), (512, 128, 1700), (256, 128, 1000)])
def test_emulated_backward_vs_oracle(emu, L, M, N):
    K = 3
    A = syn.random_spectrum(3 * L, N)
    taps = syn.random_taps(5 * M, K, M)
    w = np.random.default_rng(N).random((K, N), dtype=np.float32)
    bank = _bank(emu, taps, L)
    emu.fdas_backward_workspace_bytes.restype = ctypes.c_size_t
    wsb = emu.fdas_backward_workspace_bytes(ctypes.c_int64(N), K, M, L, 0)
    ws = np.zeros(wsb + 256, dtype=np.uint8)
    wsp = ctypes.c_void_p((ws.ctypes.data + 255) & ~255)
    gA = np.full(N, np.nan, dtype=np.complex64)
    gT = np.full((K, M), np.nan, dtype=np.complex64)
    assert emu.fdas_correlate_backward(_p(A), ctypes.c_int64(N), _p(bank), K, M, L, _p(w),
                                       _p(gA), _p(gT), wsp, ctypes.c_size_t(wsb), None) == 0
    rA, rT = native.grads(A, taps, w)
    assert _rel(gA, rA) < TOL
    assert _rel(gT, rT) < TOL
    # the spectrum gradient alone (the kernel specialised without the taps
    # transform) is bitwise the one computed beside the taps gradient
    gA2 = np.full(N, np.nan, dtype=np.complex64)
    assert emu.fdas_correlate_backward(_p(A), ctypes.c_int64(N), _p(bank), K, M, L, _p(w),
                                       _p(gA2), None, wsp, ctypes.c_size_t(wsb), None) == 0
    assert np.array_equal(gA2, gA)


# 2048/256 and 2048/512 leave one and two lane slots at each end without
# valid outputs (the kernels skip them at compile time)
# lane 63's neighbour: a lane rotation in one wave (L <= 1024), LDS slots
# behind a barrier with several waves (2048, 4096; over many templates,
# segments and workgroup ranges)
@pytest.mark.parametrize("L,M,N,grid", [(256, 32, 1000, 0), (512, 64, 449, 3), (2048, 256, 1793, 0),
                                        (256, 2, 37, 0), (2048, 512, 3100, 2),
                                        (1024, 128, 2000, 2), (2048, 128, 4000, 3),
                                        (4096, 256, 5000, 2)])
def test_emulated_interbin_vs_oracle(emu, L, M, N, grid):
    from oracle import direct
    K = 3
    A = syn.random_spectrum(7 * L + N, N)
    taps = syn.random_taps(M + 2 * K, K, M)
    bank = _bank(emu, taps, L)
    buf, plane2 = _guarded((K, 2 * N))
    assert emu.fdas_correlate_interbin_ex(_p(A), ctypes.c_int64(N), _p(bank), K, M, L,
                                          _p(plane2), grid, None) == 0
    _check_guards(buf, plane2)
    assert _rel(plane2, direct.interbinned_power(A, taps)) < TOL


@pytest.mark.parametrize("log2n", [13, 14, 15, 16, 17, 18])
def test_emulated_r2c_vs_oracle(emu, log2n):
    # plans: 2^12 complex points -> radix bits (6, 6) with the separate split
    # kernel; 2^13 .. 2^17 -> (7, 6), (7, 7), (8, 7), (8, 8), (6, 6, 5) with
    # the split inside the last pass, so every radix 32..256 runs as a first,
    # a middle and a fused last pass
    from oracle import r2c
    n = 1 << log2n
    x = syn.time_series(log2n, n, [(0.3, 0.2, n / 7 + 0.4, 11.0)])
    emu.fdas_r2c_workspace_bytes.restype = ctypes.c_size_t
    wsb = emu.fdas_r2c_workspace_bytes(ctypes.c_int64(n))
    assert wsb > 0
    ws = np.zeros(wsb + 256, dtype=np.uint8)
    wsp = ctypes.c_void_p((ws.ctypes.data + 255) & ~255)
    buf, spec = _guarded((n + 2,))            # n/2 + 1 complex values as float pairs
    scale = 1.0 / np.sqrt(n)
    assert emu.fdas_r2c(_p(x), ctypes.c_int64(n), ctypes.c_float(scale), _p(spec), wsp,
                        ctypes.c_size_t(wsb), None) == 0
    _check_guards(buf, spec)
    got = spec.view(np.complex64).astype(np.complex128)
    ref = r2c.spectrum(x, scale)
    assert np.max(np.abs(got - ref)) < TOL * np.max(np.abs(ref))
    assert np.linalg.norm(got - ref) < 1e-6 * np.linalg.norm(ref)


@pytest.mark.parametrize("log2n", [13, 14, 17])
def test_emulated_r2c_batched_equals_single(emu, log2n):
    # three series in one launch per pass (the separate split at 2^13, the
    # fused last pass above): each series' bins bitwise those of fdas_r2c,
    # nothing written outside the batch's spectra
    n, S = 1 << log2n, 3
    xs = np.stack([syn.time_series(100 * log2n + b, n, [(0.5, 0.1 * b, n / 5 + b, 3.0 * b)])
                   for b in range(S)])
    emu.fdas_r2c_batched_workspace_bytes.restype = ctypes.c_size_t
    emu.fdas_r2c_workspace_bytes.restype = ctypes.c_size_t
    wsb = emu.fdas_r2c_batched_workspace_bytes(ctypes.c_int64(n), S)
    assert wsb == S * (n // 2) * 8
    ws = np.zeros(wsb + 256, dtype=np.uint8)
    wsp = ctypes.c_void_p((ws.ctypes.data + 255) & ~255)
    buf, spec = _guarded((S, n + 2))
    assert emu.fdas_r2c_batched(_p(xs), ctypes.c_int64(n), S, ctypes.c_float(0.5), _p(spec), wsp,
                                ctypes.c_size_t(wsb), None) == 0
    _check_guards(buf, spec)
    w1 = emu.fdas_r2c_workspace_bytes(ctypes.c_int64(n))
    for b in range(S):
        one = np.zeros(n + 2, dtype=np.float32)
        x = np.ascontiguousarray(xs[b])
        assert emu.fdas_r2c(_p(x), ctypes.c_int64(n), ctypes.c_float(0.5), _p(one), wsp,
                            ctypes.c_size_t(w1), None) == 0
        assert np.array_equal(one, spec[b]), b


@pytest.mark.parametrize("L,M,N,zmax", [(512, 64, 1500, 10.0), (2048, 256, 3900, 6.0),
                                        (256, 2, 300, 0.0)])
def test_emulated_symmetric_bank(emu, L, M, N, zmax):
    # templates from the closed form (which has T_{-z} = conj T_z), the bank
    # holding only z >= 0: the plane must match the full bank's and the oracle
    taps = ot.templates(zmax, 2.0, M).astype(np.complex64)
    K = taps.shape[0]
    A = syn.random_spectrum(N + 11, N)
    full = _bank(emu, taps, L)
    emu.fdas_bank_sym_elems.restype = ctypes.c_int64
    sym = np.zeros(emu.fdas_bank_sym_elems(K, L), dtype=np.complex64)
    assert emu.fdas_prepare_bank_sym(_p(taps), K, M, L, _p(sym), None) == 0
    c = (K - 1) // 2
    assert np.array_equal(sym[:-L], full[c * L:K * L])       # rows z >= 0
    assert np.array_equal(sym[-L:], full[K * L:])            # twiddle row
    buf, plane = _guarded((K, N))
    assert emu.fdas_correlate_sym_ex(_p(A), ctypes.c_int64(N), _p(sym), K, M, L, _p(plane), 0,
                                     None) == 0
    _check_guards(buf, plane)
    ref = native.power(A, taps)
    assert _rel(plane, ref) < TOL
    one = np.zeros((K, N), dtype=np.float32)
    assert emu.fdas_correlate(_p(A), ctypes.c_int64(N), _p(full), K, M, L, _p(one), None) == 0
    assert _rel(plane, one) < TOL
    # other grids split the (segment, template) items elsewhere, so workgroup
    # ranges start, end and cross the first stored row (z = 0) at other
    # templates: the plane is the same bit for bit
    for grid in (1, 2, 5, 13):
        again = np.zeros((K, N), dtype=np.float32)
        assert emu.fdas_correlate_sym_ex(_p(A), ctypes.c_int64(N), _p(sym), K, M, L, _p(again),
                                         grid, None) == 0
        assert np.array_equal(again, plane), grid


@pytest.mark.parametrize("L,M,N,zmax", [(512, 64, 1500, 10.0), (2048, 256, 3900, 6.0),
                                        (256, 2, 300, 2.0), (1024, 126, 777, 4.0)])
def test_emulated_fourier2(emu, L, M, N, zmax):
    from oracle import direct
    A = syn.random_spectrum(N + 23, N)
    taps = ot.templates(zmax, 2.0, M).astype(np.complex64)
    K = taps.shape[0]
    bank = _bank(emu, taps, L)
    taps_h = np.zeros(K * (M + 2), dtype=np.complex64)
    bank_h = np.zeros((K + 1) * L, dtype=np.complex64)
    assert emu.fdas_make_templates_half(ctypes.c_double(zmax), ctypes.c_double(2.0), M, L,
                                        _p(taps_h), _p(bank_h), None) == 0
    buf, plane2 = _guarded((K, 2 * N))
    assert emu.fdas_correlate_fourier2_ex(_p(A), ctypes.c_int64(N), _p(bank), _p(bank_h), K, M, L,
                                          _p(plane2), 0, None) == 0
    _check_guards(buf, plane2)
    ref = direct.fourier_interpolated_power(A, zmax, 2.0, M)
    assert _rel(plane2, ref) < TOL


def _emu_sum(emu, P, H, prev=None):
    K, N = P.shape
    kh, nh = ctypes.c_int(), ctypes.c_int64()
    assert emu.fdas_harmonic_shape(ctypes.c_int64(N), K, H, ctypes.byref(kh),
                                   ctypes.byref(nh)) == 0
    buf, S = _guarded((kh.value, nh.value))
    assert emu.fdas_harmonic_sum(_p(P), ctypes.c_int64(N), K, H,
                                 _p(prev) if prev is not None else None, _p(S), None) == 0
    _check_guards(buf, S)
    return S.copy()


@pytest.mark.parametrize("K,N", [(21, 300), (1, 37), (85, 1021), (7, 1)])
def test_emulated_harmonic_sums_bitwise(emu, K, N):
    # the FP32 sums in the order h = 1..H match the oracle bit for bit, built
    # from scratch or on the previous fold
    from oracle import harmonic as oh
    P = syn.random_plane(5, K, N)
    prev = P
    for H in (1, 2, 4, 8, 16, 32):
        ref = oh.harmonic_sum(P, H)
        scratch = _emu_sum(emu, P, H)
        assert np.array_equal(scratch, ref), H
        if H >= 2:
            chained = _emu_sum(emu, P, H, prev if H > 2 else None)
            assert np.array_equal(chained, ref), H
            prev = chained


def _emu_candidates(emu, S_src, P, H, thr, capacity):
    K, N = P.shape
    out = np.zeros(max(capacity, 1) * 2 + 2 * 64, dtype=np.int64)   # 16-byte records + margins
    out[:] = -7
    view = out[64:64 + 2 * max(capacity, 1)]
    count = np.full(1, 12345, dtype=np.uint32)
    assert emu.fdas_find_candidates(_p(S_src), ctypes.c_int64(N), K, H, ctypes.c_float(thr),
                                    _p(view), capacity, _p(count), None) == 0
    assert np.all(out[:64] == -7) and np.all(out[64 + 2 * max(capacity, 1):] == -7)
    rec = view.view(np.dtype([("r", "<i8"), ("row", "<i4"), ("power", "<f4")]))
    return int(count[0]), rec[:min(int(count[0]), capacity)]


@pytest.mark.parametrize("H", [1, 2, 8])
def test_emulated_candidates_vs_oracle(emu, H):
    from oracle import harmonic as oh
    K, N = 41, 700
    P = syn.random_plane(6, K, N)
    S = oh.harmonic_sum(P, H)
    thr = float(np.quantile(S, 0.97))
    ref = oh.peaks(S, thr)
    c = (K - 1) // 2
    row0 = c - (S.shape[0] - 1) // 2
    n, rec = _emu_candidates(emu, S, P, H, thr, 10000)
    assert n == len(ref) > 0
    got = sorted(zip(rec["row"] - row0, rec["r"]))
    assert got == sorted(map(tuple, ref.tolist()))
    assert np.array_equal(np.sort(rec["power"]), np.sort(S[ref[:, 0], ref[:, 1]]))
    # a capacity below the count: the count stays exact, only that many are written
    n2, rec2 = _emu_candidates(emu, S, P, H, thr, 5)
    assert n2 == n and len(rec2) == 5
    assert set(zip(rec2["row"] - row0, rec2["r"])) <= set(map(tuple, ref.tolist()))
    # nothing above an unreachable threshold
    n3, _ = _emu_candidates(emu, S, P, H, float(S.max()) + 1.0, 10)
    assert n3 == 0
    # count only: capacity 0 and no output buffer
    count = np.full(1, 99, dtype=np.uint32)
    assert emu.fdas_find_candidates(_p(S), ctypes.c_int64(N), K, H, ctypes.c_float(thr), None, 0,
                                    _p(count), None) == 0
    assert int(count[0]) == n


def test_emulated_batched_harmonic_sums_and_candidates(emu):
    # ragged spectra (one empty, one single-bin) packed as correlate_batched
    # lays out its planes; folds chained in one launch each; bitwise equal to
    # the oracle per spectrum, candidates equal to the per-spectrum peak sets
    from oracle import harmonic as oh
    K = 21
    lens = [300, 0, 1, 97, 130]
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    planes = [syn.random_plane(30 + b, K, n) for b, n in enumerate(lens)]
    flat = np.concatenate([p.reshape(-1) for p in planes]).astype(np.float32)
    nspec = len(lens)
    emu.fdas_harmonic_batched_workspace_bytes.restype = ctypes.c_size_t
    wsb = emu.fdas_harmonic_batched_workspace_bytes(nspec)
    ws = np.zeros(wsb // 8 + 1, dtype=np.int64)
    prev = None
    c = (K - 1) // 2
    for H in (2, 4, 8):
        KH = 2 * (c // H) + 1
        pre = np.concatenate([[0], np.cumsum([(n + H - 1) // H for n in lens])]).astype(np.int64)
        buf, S = _guarded((KH * int(pre[-1]),))
        assert emu.fdas_harmonic_sum_batched(_p(flat), _p(offs), nspec, K, H,
                                             _p(prev) if prev is not None else None, _p(S),
                                             _p(ws), ctypes.c_size_t(wsb), None) == 0
        _check_guards(buf, S)
        S = S.copy()
        for b, n in enumerate(lens):
            got = S[KH * pre[b]:KH * pre[b + 1]].reshape(KH, -1)
            assert np.array_equal(got, oh.harmonic_sum(planes[b], H)), (H, b)
        prev = S
        if H == 4:
            thr = float(np.quantile(S, 0.9))
            out = np.zeros(2 * 4096, dtype=np.int64)
            count = np.zeros(1, dtype=np.uint32)
            assert emu.fdas_find_candidates_batched(_p(S), _p(offs), nspec, K, H,
                                                    ctypes.c_float(thr), _p(out), 4096,
                                                    _p(count), _p(ws), ctypes.c_size_t(wsb),
                                                    None) == 0
            rec = out.view(np.dtype([("r", "<i8"), ("row", "<i4"), ("power", "<f4")]))
            rec = rec[:int(count[0])]
            got = sorted((int(r), int(row)) for r, row in zip(rec["r"], rec["row"]))
            want = []
            row0 = c - (KH - 1) // 2
            for b in range(nspec):
                for k, r in oh.peaks(S[KH * pre[b]:KH * pre[b + 1]].reshape(KH, -1), thr):
                    want.append((int(offs[b] + r), int(row0 + k)))
            assert got == sorted(want) and len(want) > 0


@pytest.mark.parametrize("n", [0, 3, 4, 1027, 4096 * 256 + 5])
def test_stream_probes(emu, n):
    """The streaming write fills exactly n floats (tails included) and the
    read's partial sums add up to the buffer's sum, with the partials of
    workgroups not launched set to zero."""
    P = 2048
    buf, arr = _guarded((n,))
    assert emu.fdas_stream_write(_p(arr) if n else None, ctypes.c_int64(n), ctypes.c_float(1.5),
                                 None) == 0
    _check_guards(buf, arr)
    assert np.all(arr == np.float32(1.5))
    vals = np.arange(n, dtype=np.float32) % 7      # small integers: every sum is exact
    sums = np.full(P, np.nan, dtype=np.float32)
    assert emu.fdas_stream_read(_p(vals) if n else None, ctypes.c_int64(n), _p(sums), None) == 0
    assert np.all(np.isfinite(sums))
    assert float(sums.astype(np.float64).sum()) == float(vals.astype(np.float64).sum())

