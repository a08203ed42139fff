"""C-ABI checks that need no GPU: the library loads, exports every symbol
declared in include/fdas.h, rejects bad arguments with a status before any
HIP call, and its host FP64 template math agrees with the oracle."""
import ctypes
import os
import re

import numpy as np
import pytest

from paper_1804_05335_amd import _lib
from oracle import templates as ot
from tests.quadrature import response_quadrature

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared_symbols():
    names = set()
    for hdr in os.listdir(os.path.join(ROOT, "include")):
        if hdr.endswith(".h"):
            text = open(os.path.join(ROOT, "include", hdr)).read()
            text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
            names |= set(re.findall(r"\b(fdas_[a-z0-9_]+)\s*\(", text))
    return names


def test_library_exports_every_declared_symbol():
    L = _lib.lib()
    declared = _declared_symbols()
    assert "fdas_correlate" in declared and "fdas_prepare_bank" in declared
    for name in declared:
        assert hasattr(L, name), name
    bound = {n for n, _, _ in _lib.SIGNATURES}
    assert declared == bound


def test_status_strings_and_version():
    assert _lib.fdas_version().startswith("fdas-gfx950")
    for st in range(5):
        assert _lib.status_string(st)
    assert _lib.status_string(99) == "unknown status"


def test_num_templates():
    assert _lib.fdas_num_templates(84.0, 2.0) == 85
    assert _lib.fdas_num_templates(20.0, 2.0) == 21
    assert _lib.fdas_num_templates(0.0, 2.0) == 1
    assert _lib.fdas_num_templates(200.0, 2.0) == 201
    for zmax, dz in [(3.0, 2.0), (-2.0, 2.0), (4.0, 0.0), (float("nan"), 1.0)]:
        with pytest.raises(_lib.FdasError) as e:
            _lib.fdas_num_templates(zmax, dz)
        assert e.value.status == _lib.FDAS_INVALID_ARG
    with pytest.raises(_lib.FdasError) as e:
        _lib.fdas_num_templates(5000.0, 1.0)
    assert e.value.status == _lib.FDAS_UNSUPPORTED


@pytest.mark.parametrize("z", [0.0, 2.0, -2.0, 8.0, -84.0, 200.0, 33.3])
def test_product_response_matches_oracle(z):
    q = np.concatenate([np.arange(-300, 301, 7.0), [0.5, -0.25, 12.75, 0.0]])
    got = np.array([_lib.fdas_template_response(float(x), z) for x in q])
    ref = ot.response(q, z)
    assert np.max(np.abs(got - ref)) < 1e-11


@pytest.mark.parametrize("z", [1e-4, -3e-3, 0.05])
def test_product_response_small_z_vs_quadrature(z):
    # For |z| << 1 the oracle's route multiplies by exp(-i pi q'^2/z) with a
    # phase of ~1e9 rad and loses digits; the library's route has no large
    # phase.  Check it against direct quadrature instead.
    q = np.array([-300.0, -17.0, -1.0, 0.0, 0.5, 1.0, 40.0, 255.0])
    got = np.array([_lib.fdas_template_response(float(x), z) for x in q])
    assert np.max(np.abs(got - response_quadrature(q, z))) < 1e-12


@pytest.mark.parametrize("zmax,M", [(20.0, 64), (84.0, 256), (84.0, 128), (200.0, 512)])
def test_product_templates_match_oracle(zmax, M):
    T = _lib.fdas_make_templates_host(zmax, 2.0, M)
    ref = ot.templates(zmax, 2.0, M)
    assert T.shape == ref.shape and T.dtype == np.complex64
    # FP64 values rounded once to FP32
    assert np.max(np.abs(T - ref)) <= 6e-8 * np.max(np.abs(ref))
    assert np.array_equal(T, ref.astype(np.complex64)) or \
        np.max(np.abs(T - ref.astype(np.complex64))) < 1e-7


def _fake(addr):
    return ctypes.c_void_p(addr)


def test_validation_happens_before_any_device_call():
    L = _lib.lib()
    sp, bk, pl = _fake(0x1000), _fake(0x2000), _fake(0x3000)
    cases = [
        # (N, K, M, L, expected)
        (1000, 85, 256, 3000, _lib.FDAS_UNSUPPORTED),      # L not a power of two
        (1000, 85, 256, 128, _lib.FDAS_UNSUPPORTED),       # L too small
        (1000, 85, 256, 16384, _lib.FDAS_UNSUPPORTED),     # L too large
        (1000, 85, 255, 2048, _lib.FDAS_UNSUPPORTED),      # M odd
        (1000, 85, 2048, 2048, _lib.FDAS_UNSUPPORTED),     # M > L/2
        (1000, 85, 0, 2048, _lib.FDAS_UNSUPPORTED),        # M < 2
        (1000, 0, 256, 2048, _lib.FDAS_UNSUPPORTED),       # K < 1
        (-1, 85, 256, 2048, _lib.FDAS_INVALID_ARG),        # N < 0
        ((1 << 32) + 1, 85, 256, 2048, _lib.FDAS_INVALID_ARG),
    ]
    for N, K, M, Ls, want in cases:
        assert L.fdas_correlate(sp, N, bk, K, M, Ls, pl, None) == want, (N, K, M, Ls)
        assert L.fdas_last_error()
    # null and misaligned pointers
    assert L.fdas_correlate(None, 1000, bk, 85, 256, 2048, pl, None) == _lib.FDAS_INVALID_ARG
    assert L.fdas_correlate(_fake(0x1004), 1000, bk, 85, 256, 2048, pl, None) == _lib.FDAS_INVALID_ARG
    assert L.fdas_correlate(sp, 1000, _fake(0x2008), 85, 256, 2048, pl, None) == _lib.FDAS_INVALID_ARG
    assert L.fdas_correlate(sp, 1000, bk, 85, 256, 2048, _fake(0x3002), None) == _lib.FDAS_INVALID_ARG
    assert L.fdas_correlate_ex(sp, 1000, bk, 85, 256, 2048, pl, (1 << 20) + 1, None) == _lib.FDAS_INVALID_ARG
    assert L.fdas_correlate_ex(sp, 1000, bk, 85, 256, 2048, pl, -1, None) == _lib.FDAS_INVALID_ARG
    # batched and backward validation
    ws = _fake(0x4000)
    cap = 1 << 20
    assert L.fdas_correlate_batched(sp, _fake(0x5000), 0, cap, None, 85, 256, 2048, None, None, 0, None) == _lib.FDAS_OK
    assert L.fdas_correlate_batched(sp, _fake(0x5000), -1, cap, bk, 85, 256, 2048, pl, ws, 1 << 20, None) == _lib.FDAS_INVALID_ARG
    assert L.fdas_correlate_batched(sp, _fake(0x5000), 4, cap, bk, 85, 256, 2048, pl, ws, 8, None) == _lib.FDAS_WORKSPACE_TOO_SMALL
    assert L.fdas_correlate_batched(sp, _fake(0x5004), 4, cap, bk, 85, 256, 2048, pl, ws, 1 << 20, None) == _lib.FDAS_INVALID_ARG
    assert L.fdas_correlate_batched(sp, None, 4, cap, bk, 85, 256, 2048, pl, ws, 1 << 20, None) == _lib.FDAS_INVALID_ARG
    assert L.fdas_correlate_batched(sp, _fake(0x5000), 4, cap, bk, 85, 256, 1000, pl, ws, 1 << 20, None) == _lib.FDAS_UNSUPPORTED
    # capacity outside [0, 2^40]
    assert L.fdas_correlate_batched(sp, _fake(0x5000), 4, -1, bk, 85, 256, 2048, pl, ws, 1 << 20, None) == _lib.FDAS_INVALID_ARG
    assert L.fdas_correlate_batched(sp, _fake(0x5000), 4, (1 << 40) + 1, bk, 85, 256, 2048, pl, ws, 1 << 20, None) == _lib.FDAS_INVALID_ARG
    # values per lane: 8 and 16 from L = 1024 on, else only the default
    bx = L.fdas_correlate_batched_ex
    assert bx(sp, _fake(0x5000), 4, cap, bk, 85, 256, 2048, pl, 4, 0, ws, 1 << 20, None) == _lib.FDAS_UNSUPPORTED
    assert bx(sp, _fake(0x5000), 4, cap, bk, 85, 128, 512, pl, 16, 0, ws, 1 << 20, None) == _lib.FDAS_UNSUPPORTED
    assert bx(sp, _fake(0x5000), 0, cap, bk, 85, 256, 2048, pl, 8, 0, ws, 1 << 20, None) == _lib.FDAS_OK
    assert bx(sp, _fake(0x5000), 0, cap, bk, 85, 256, 8192, pl, 16, 0, ws, 1 << 20, None) == _lib.FDAS_OK
    assert bx(sp, _fake(0x5000), 4, cap, bk, 85, 256, 2048, pl, 0, -1, ws, 1 << 20, None) == _lib.FDAS_INVALID_ARG
    # allocation-free batched call: the fixed maximum batch and the usual checks, before any launch
    na = L.fdas_correlate_batched_noalloc
    assert na(sp, _fake(0x5000), 0, cap, None, 85, 256, 2048, None, None) == _lib.FDAS_OK
    assert na(sp, _fake(0x5000), 65537, cap, bk, 85, 256, 2048, pl, None) == _lib.FDAS_INVALID_ARG
    assert b"allocation-free" in L.fdas_last_error()
    assert na(sp, _fake(0x5000), -1, cap, bk, 85, 256, 2048, pl, None) == _lib.FDAS_INVALID_ARG
    assert na(sp, _fake(0x5004), 4, cap, bk, 85, 256, 2048, pl, None) == _lib.FDAS_INVALID_ARG
    assert na(sp, None, 4, cap, bk, 85, 256, 2048, pl, None) == _lib.FDAS_INVALID_ARG
    assert na(sp, _fake(0x5000), 4, cap, bk, 85, 256, 1000, pl, None) == _lib.FDAS_UNSUPPORTED
    assert na(sp, _fake(0x5000), 4, -1, bk, 85, 256, 2048, pl, None) == _lib.FDAS_INVALID_ARG
    assert _lib.NOALLOC_MAX_SPECTRA == 65536
    # LDS bank probe: arguments checked before any launch
    lp = L.fdas_lds_probe
    assert lp(_fake(0x7000), 3, 16, 1, _fake(0x7100), _fake(0x7200), None) == _lib.FDAS_INVALID_ARG
    assert lp(_fake(0x7000), 0, 0, 1, _fake(0x7100), _fake(0x7200), None) == _lib.FDAS_INVALID_ARG
    assert lp(_fake(0x7000), 1, 16, 0, _fake(0x7100), _fake(0x7200), None) == _lib.FDAS_INVALID_ARG
    assert lp(None, 1, 16, 1, _fake(0x7100), _fake(0x7200), None) == _lib.FDAS_INVALID_ARG
    assert lp(_fake(0x7000), 1, 16, 1, _fake(0x7104), _fake(0x7200), None) == _lib.FDAS_INVALID_ARG
    # batched adjoint: workspace by the gradients wanted, validation first
    wb = L.fdas_backward_batched_workspace_bytes
    both, only_s, only_t = wb(cap, 4, 9, 128, 2048, 0, 3), wb(cap, 4, 9, 128, 2048, 0, 1), wb(cap, 4, 9, 128, 2048, 0, 2)
    assert both > max(only_s, only_t) > 0 and both % 256 == 0
    assert wb(cap, 4, 9, 128, 2048, 0, 4) == 0 and wb(-1, 4, 9, 128, 2048, 0, 3) == 0
    assert wb(cap, 4, 9, 2048, 2048, 0, 3) == 0 and wb(cap, 4, 9, 128, 2048, 10, 3) == 0
    bb = L.fdas_correlate_backward_batched
    assert bb(sp, _fake(0x5000), 4, cap, bk, 9, 128, 2048, pl, None, None, 0, ws, 0, None) == _lib.FDAS_OK
    assert bb(sp, _fake(0x5000), 4, cap, bk, 9, 128, 2048, pl, sp, None, 0, ws, only_s - 256, None) == _lib.FDAS_WORKSPACE_TOO_SMALL
    assert bb(sp, _fake(0x5000), 4, cap, bk, 9, 128, 2048, pl, sp, sp, 0, ws, only_s, None) == _lib.FDAS_WORKSPACE_TOO_SMALL
    assert bb(sp, None, 4, cap, bk, 9, 128, 2048, pl, sp, None, 0, ws, both, None) == _lib.FDAS_INVALID_ARG
    assert bb(sp, _fake(0x5000), 4, cap, bk, 9, 128, 2048, pl, sp, None, 0, _fake(0x4010), both, None) == _lib.FDAS_INVALID_ARG
    assert bb(sp, _fake(0x5000), 4, cap, bk, 9, 128, 2048, pl, sp, None, 11, ws, both, None) == _lib.FDAS_INVALID_ARG
    assert bb(sp, _fake(0x5000), -1, cap, bk, 9, 128, 2048, pl, sp, None, 0, ws, both, None) == _lib.FDAS_INVALID_ARG
    assert bb(sp, _fake(0x5000), 4, cap, bk, 9, 128, 1000, pl, sp, None, 0, ws, both, None) == _lib.FDAS_UNSUPPORTED
    wsb = L.fdas_backward_workspace_bytes(4096, 9, 128, 2048, 0)
    assert wsb > 0 and wsb % 256 == 0
    assert L.fdas_backward_workspace_bytes(4096, 9, 2048, 2048, 0) == 0
    assert L.fdas_correlate_backward(sp, 4096, bk, 9, 128, 2048, pl, sp, None, ws, wsb - 256, None) == _lib.FDAS_WORKSPACE_TOO_SMALL
    assert L.fdas_correlate_backward(sp, 4096, bk, 9, 128, 2048, pl, None, None, ws, wsb, None) == _lib.FDAS_OK
    assert L.fdas_correlate_backward(sp, 4096, bk, 9, 128, 2048, pl, sp, None, _fake(0x4010), wsb, None) == _lib.FDAS_INVALID_ARG
    assert L.fdas_correlate_backward(sp, 4096, bk, 9, 2048, 2048, pl, sp, None, ws, wsb, None) == _lib.FDAS_UNSUPPORTED
    assert L.fdas_correlate_backward(None, 4096, bk, 9, 128, 2048, pl, sp, None, ws, wsb, None) == _lib.FDAS_INVALID_ARG
    # N = 0 is a no-op that touches nothing, even with NULL buffers
    assert L.fdas_correlate(None, 0, None, 85, 256, 2048, None, None) == _lib.FDAS_OK
    # bank preparation
    assert L.fdas_prepare_bank(None, 85, 256, 2048, bk, None) == _lib.FDAS_INVALID_ARG
    assert L.fdas_prepare_bank(sp, 85, 256, 1000, bk, None) == _lib.FDAS_UNSUPPORTED
    assert L.fdas_prepare_bank(sp, 85, 256, 2048, _fake(0x2008), None) == _lib.FDAS_INVALID_ARG
    assert L.fdas_make_templates(3.0, 2.0, 64, 512, sp, bk, None) == _lib.FDAS_INVALID_ARG
    assert L.fdas_make_templates(20.0, 2.0, 64, 512, None, bk, None) == _lib.FDAS_INVALID_ARG
    assert L.fdas_make_templates(20.0, 2.0, 63, 512, sp, bk, None) == _lib.FDAS_UNSUPPORTED


def test_bank_elems():
    assert _lib.fdas_bank_elems(85, 2048) == 86 * 2048
    assert _lib.fdas_bank_elems(0, 2048) == 0


def test_autotune_validation_before_any_device_call():
    L = _lib.lib()
    p = _fake(0x10000)
    out = _lib.Tuning()
    wsb = L.fdas_autotune_workspace_bytes(85, 4)
    assert wsb >= 86 * 8192 * 8
    args = lambda ws, wsb_, K=85, M=256, n=4, cap=1 << 20, flags=0: (
        p, K, M, p, p, n, cap, p, ws, wsb_, flags, None, ctypes.byref(out))
    assert L.fdas_autotune_batched(*args(p, wsb - 1)) == _lib.FDAS_WORKSPACE_TOO_SMALL
    assert L.fdas_autotune_batched(*args(_fake(0x10010), wsb)) == _lib.FDAS_INVALID_ARG
    assert L.fdas_autotune_batched(*args(p, wsb, n=0)) == _lib.FDAS_INVALID_ARG
    assert L.fdas_autotune_batched(*args(p, wsb, M=255)) == _lib.FDAS_INVALID_ARG
    assert L.fdas_autotune_batched(*args(p, wsb, cap=0)) == _lib.FDAS_INVALID_ARG
    assert L.fdas_autotune_batched(*args(p, wsb, flags=4)) == _lib.FDAS_INVALID_ARG
    assert L.fdas_autotune_batched(p, 85, 256, p, p, 4, 1 << 20, p, p, wsb, 0, None,
                                   None) == _lib.FDAS_INVALID_ARG


def test_autotune_candidates_cover_lengths_lanes_and_grids():
    # every supported L from 512 with M <= L/2, both lane counts from 1024 on,
    # grid factors 1 and 2
    c = _lib.fdas_autotune_candidates(85, 256)
    got = {(x["L"], x["E"], x["grid_factor"]) for x in c}
    want = {(L, E, g) for L in (512, 1024, 2048, 4096, 8192)
            for E in ((8,) if L == 512 else (16, 8)) for g in (1, 2)}
    assert got == want and len(c) == len(want)
    # wide templates rule out the short segments
    assert {x["L"] for x in _lib.fdas_autotune_candidates(201, 512)} == {1024, 2048, 4096, 8192}
    with pytest.raises(_lib.FdasError):
        _lib.fdas_autotune_candidates(85, 255)


def test_r2c_validation_before_any_device_call():
    L = _lib.lib()
    n = 1 << 20
    wsb = L.fdas_r2c_workspace_bytes(n)
    assert wsb >= (n // 2) * 8
    for bad in (0, 1 << 12, (1 << 20) + 2, 3 << 18, 1 << 28, -4):
        assert L.fdas_r2c_workspace_bytes(bad) == 0
        assert L.fdas_r2c(_fake(0x10000), bad, 1.0, _fake(0x4000000), _fake(0x8000000), wsb,
                          None) == _lib.FDAS_UNSUPPORTED
    x, spec, ws = _fake(0x10000000), _fake(0x20000000), _fake(0x30000000)
    assert L.fdas_r2c(x, n, 1.0, spec, ws, wsb - 1, None) == _lib.FDAS_WORKSPACE_TOO_SMALL
    assert L.fdas_r2c(None, n, 1.0, spec, ws, wsb, None) == _lib.FDAS_INVALID_ARG
    assert L.fdas_r2c(_fake(0x10000004), n, 1.0, spec, ws, wsb, None) == _lib.FDAS_INVALID_ARG
    assert L.fdas_r2c(x, n, 1.0, spec, _fake(0x30000080), wsb, None) == _lib.FDAS_INVALID_ARG
    # overlapping buffers: spec inside x, ws overlapping spec
    assert L.fdas_r2c(x, n, 1.0, _fake(0x10000000 + 8 * 1024), ws, wsb, None) == \
        _lib.FDAS_INVALID_ARG
    assert L.fdas_r2c(x, n, 1.0, spec, _fake(0x20000000 + 4096 * 256), wsb, None) == \
        _lib.FDAS_INVALID_ARG


def test_r2c_batched_validation_before_any_device_call():
    L = _lib.lib()
    n, S = 1 << 20, 3
    wsb = L.fdas_r2c_batched_workspace_bytes(n, S)
    assert wsb == S * (n // 2) * 8
    assert L.fdas_r2c_batched_workspace_bytes(n, 0) == 0
    assert L.fdas_r2c_batched_workspace_bytes(n, 65536) == 0
    assert L.fdas_r2c_batched_workspace_bytes(3 << 18, 1) == 0
    x, spec, ws = _fake(0x10000000), _fake(0x40000000), _fake(0x80000000)
    assert L.fdas_r2c_batched(x, 3 << 18, S, 1.0, spec, ws, wsb, None) == _lib.FDAS_UNSUPPORTED
    for bad in (0, -1, 65536):
        assert L.fdas_r2c_batched(x, n, bad, 1.0, spec, ws, wsb, None) == _lib.FDAS_INVALID_ARG
    assert L.fdas_r2c_batched(x, n, S, 1.0, spec, ws, wsb - 1, None) == \
        _lib.FDAS_WORKSPACE_TOO_SMALL
    assert L.fdas_r2c_batched(None, n, S, 1.0, spec, ws, wsb, None) == _lib.FDAS_INVALID_ARG
    assert L.fdas_r2c_batched(x, n, S, 1.0, spec, _fake(0x80000080), wsb, None) == \
        _lib.FDAS_INVALID_ARG
    # the third series' samples reach into spec, spec's last series into ws
    assert L.fdas_r2c_batched(x, n, S, 1.0, _fake(0x10000000 + 4 * n * 2 + 8), ws, wsb,
                              None) == _lib.FDAS_INVALID_ARG
    assert L.fdas_r2c_batched(x, n, S, 1.0, spec, _fake(0x40000000 + 8 * (n // 2 + 1) * 2 + 256),
                              wsb, None) == _lib.FDAS_INVALID_ARG


def test_symmetric_bank_validation():
    L = _lib.lib()
    assert L.fdas_bank_sym_elems(85, 2048) == 44 * 2048
    assert L.fdas_bank_sym_elems(1, 512) == 2 * 512
    for K in (0, 84, -1):
        assert L.fdas_bank_sym_elems(K, 2048) == 0
    p = _fake(0x10000)
    assert L.fdas_prepare_bank_sym(p, 84, 256, 2048, p, None) == _lib.FDAS_INVALID_ARG
    assert L.fdas_correlate_sym(p, 1000, p, 84, 256, 2048, p, None) == _lib.FDAS_INVALID_ARG
    assert L.fdas_correlate_sym(p, 1000, p, 85, 255, 2048, p, None) == _lib.FDAS_UNSUPPORTED
    assert L.fdas_correlate_sym_ex(p, 1000, p, 85, 256, 2048, p, -1, None) == _lib.FDAS_INVALID_ARG


def test_fourier2_validation_before_any_device_call():
    L = _lib.lib()
    p = _fake(0x10000)
    # M + 2 must fit L/2
    assert L.fdas_make_templates_half(ctypes.c_double(84.0), ctypes.c_double(2.0), 1024, 2048, p,
                                      p, None) == _lib.FDAS_UNSUPPORTED
    assert L.fdas_correlate_fourier2(p, 1000, p, p, 85, 1024, 2048, p, None) == \
        _lib.FDAS_UNSUPPORTED
    assert L.fdas_correlate_fourier2(p, 1000, p, p, 85, 256, 2048, _fake(0x10004), None) == \
        _lib.FDAS_INVALID_ARG
    assert L.fdas_correlate_fourier2(p, 1000, p, None, 85, 256, 2048, p, None) == \
        _lib.FDAS_INVALID_ARG
    assert L.fdas_correlate_fourier2_ex(p, 1000, p, p, 85, 256, 2048, p, -3, None) == \
        _lib.FDAS_INVALID_ARG


def test_harmonic_validation_before_any_device_call():
    L = _lib.lib()
    kh, nh = ctypes.c_int(), ctypes.c_int64()
    assert L.fdas_harmonic_shape(1000, 85, 4, ctypes.byref(kh), ctypes.byref(nh)) == _lib.FDAS_OK
    assert (kh.value, nh.value) == (21, 250)
    for N, K, H in ((1000, 84, 4), (1000, 85, 3), (1000, 85, 128), (-1, 85, 2), (1000, 0, 2),
                    (1000, 4097, 2), ((1 << 32) + 1, 85, 2)):
        assert L.fdas_harmonic_shape(N, K, H, ctypes.byref(kh), ctypes.byref(nh)) == \
            _lib.FDAS_INVALID_ARG
        assert L.fdas_harmonic_sum(_fake(0x1000), N, K, H, None, _fake(0x9000000), None) == \
            _lib.FDAS_INVALID_ARG
    assert L.fdas_harmonic_shape(1000, 85, 4, None, ctypes.byref(nh)) == _lib.FDAS_INVALID_ARG
    plane, sums = _fake(0x10000000), _fake(0x20000000)
    # NULL, misaligned, overlapping buffers, a previous fold for H = 1
    assert L.fdas_harmonic_sum(None, 1000, 85, 4, None, sums, None) == _lib.FDAS_INVALID_ARG
    assert L.fdas_harmonic_sum(plane, 1000, 85, 4, None, _fake(0x20000002), None) == \
        _lib.FDAS_INVALID_ARG
    assert L.fdas_harmonic_sum(plane, 1000, 85, 4, None, _fake(0x10000000 + 4 * 1000),
                               None) == _lib.FDAS_INVALID_ARG
    assert L.fdas_harmonic_sum(plane, 1000, 85, 4, _fake(0x20000000 + 64), sums, None) == \
        _lib.FDAS_INVALID_ARG
    assert L.fdas_harmonic_sum(plane, 1000, 85, 1, sums, _fake(0x30000000), None) == \
        _lib.FDAS_INVALID_ARG
    # candidates: negative capacity, NULL / misaligned count or output
    out, count = _fake(0x40000000), _fake(0x50000000)
    assert L.fdas_find_candidates(sums, 1000, 85, 4, 1.0, out, -1, count, None) == \
        _lib.FDAS_INVALID_ARG
    assert L.fdas_find_candidates(sums, 1000, 85, 4, 1.0, out, 10, None, None) == \
        _lib.FDAS_INVALID_ARG
    assert L.fdas_find_candidates(sums, 1000, 85, 4, 1.0, _fake(0x40000004), 10, count,
                                  None) == _lib.FDAS_INVALID_ARG
    assert L.fdas_find_candidates(sums, 1000, 85, 4, 1.0, out, 10, _fake(0x50000002),
                                  None) == _lib.FDAS_INVALID_ARG
    assert L.fdas_find_candidates(None, 1000, 85, 4, 1.0, out, 10, count, None) == \
        _lib.FDAS_INVALID_ARG


def test_stream_probe_validation_before_any_device_call():
    L = _lib.lib()
    buf, sums = _fake(0x10000000), _fake(0x20000000)
    assert _lib.STREAM_PARTIALS == 2048
    assert L.fdas_stream_write(buf, -1, 1.0, None) == _lib.FDAS_INVALID_ARG
    assert L.fdas_stream_write(None, 0, 1.0, None) == _lib.FDAS_OK          # nothing to do
    assert L.fdas_stream_write(None, 16, 1.0, None) == _lib.FDAS_INVALID_ARG
    assert L.fdas_stream_write(_fake(0x10000008), 16, 1.0, None) == _lib.FDAS_INVALID_ARG
    assert L.fdas_stream_read(buf, -1, sums, None) == _lib.FDAS_INVALID_ARG
    assert L.fdas_stream_read(buf, 16, None, None) == _lib.FDAS_INVALID_ARG
    assert L.fdas_stream_read(None, 16, sums, None) == _lib.FDAS_INVALID_ARG
    assert L.fdas_stream_read(_fake(0x10000004), 16, sums, None) == _lib.FDAS_INVALID_ARG
    assert L.fdas_stream_read(buf, 16, _fake(0x20000002), None) == _lib.FDAS_INVALID_ARG
    # the partial sums inside the buffer being read
    assert L.fdas_stream_read(buf, 1 << 20, _fake(0x10000000 + 4096), None) == \
        _lib.FDAS_INVALID_ARG

