"""ctypes binding of libfdas.so: the C-ABI calls under the same names.

Argument marshalling only -- every step of the correlation runs in the HIP
kernels of the library.  Tensors are torch device tensors (complex64 /
float32); the stream defaults to torch's current stream on the tensor's
device.  If the library is missing the import of this module fails loudly:
there is no fallback path.
"""
from __future__ import annotations

import ctypes
import os

HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(HERE, "libfdas.so")

FDAS_OK = 0
FDAS_INVALID_ARG = 1
FDAS_UNSUPPORTED = 2
FDAS_WORKSPACE_TOO_SMALL = 3
FDAS_HIP_ERROR = 4

# (name, restype, argtypes) of every symbol declared in include/fdas.h
_P = ctypes.c_void_p
_I = ctypes.c_int
_I64 = ctypes.c_int64
_D = ctypes.c_double
_SZ = ctypes.c_size_t
SIGNATURES = [
    ("fdas_version", ctypes.c_char_p, []),
    ("fdas_status_string", ctypes.c_char_p, [_I]),
    ("fdas_last_error", ctypes.c_char_p, []),
    ("fdas_num_templates", _I, [_D, _D, ctypes.POINTER(_I)]),
    ("fdas_template_response", _I, [_D, _D, ctypes.POINTER(_D), ctypes.POINTER(_D)]),
    ("fdas_make_templates_host", _I, [_D, _D, _I, _P]),
    ("fdas_bank_elems", _I64, [_I, _I]),
    ("fdas_prepare_bank", _I, [_P, _I, _I, _I, _P, _P]),
    ("fdas_make_templates", _I, [_D, _D, _I, _I, _P, _P, _P]),
    ("fdas_correlate", _I, [_P, _I64, _P, _I, _I, _I, _P, _P]),
    ("fdas_correlate_ex", _I, [_P, _I64, _P, _I, _I, _I, _P, _I, _P]),
    ("fdas_correlate_interbin", _I, [_P, _I64, _P, _I, _I, _I, _P, _P]),
    ("fdas_correlate_interbin_ex", _I, [_P, _I64, _P, _I, _I, _I, _P, _I, _P]),
    ("fdas_batched_workspace_bytes", _SZ, [_I]),
    ("fdas_correlate_batched", _I, [_P, _P, _I, _I64, _P, _I, _I, _I, _P, _P, _SZ, _P]),
    ("fdas_correlate_batched_ex", _I, [_P, _P, _I, _I64, _P, _I, _I, _I, _P, _I, _I, _P, _SZ,
                                       _P]),
    ("fdas_correlate_batched_noalloc", _I, [_P, _P, _I, _I64, _P, _I, _I, _I, _P, _P]),
    ("fdas_autotune_workspace_bytes", _SZ, [_I, _I]),
    ("fdas_autotune_candidates", _I, [_I, _I, _P, _I, ctypes.POINTER(_I)]),
    ("fdas_batched_resident_grid", _I, [_I, _I, _I, ctypes.POINTER(_I)]),
    ("fdas_autotune_batched", _I, [_P, _I, _I, _P, _P, _I, _I64, _P, _P, _SZ, _I, _P, _P]),
    ("fdas_backward_batched_workspace_bytes", _SZ, [_I64, _I, _I, _I, _I, _I, _I]),
    ("fdas_correlate_backward_batched", _I, [_P, _P, _I, _I64, _P, _I, _I, _I, _P, _P, _P, _I,
                                             _P, _SZ, _P]),
    ("fdas_backward_workspace_bytes", _SZ, [_I64, _I, _I, _I, _I]),
    ("fdas_correlate_backward", _I, [_P, _I64, _P, _I, _I, _I, _P, _P, _P, _P, _SZ, _P]),
    ("fdas_correlate_backward_ex", _I, [_P, _I64, _P, _I, _I, _I, _P, _P, _P, _I, _P, _SZ, _P]),
    ("fdas_bank_sym_elems", _I64, [_I, _I]),
    ("fdas_prepare_bank_sym", _I, [_P, _I, _I, _I, _P, _P]),
    ("fdas_correlate_sym", _I, [_P, _I64, _P, _I, _I, _I, _P, _P]),
    ("fdas_correlate_sym_ex", _I, [_P, _I64, _P, _I, _I, _I, _P, _I, _P]),
    ("fdas_make_templates_half", _I, [_D, _D, _I, _I, _P, _P, _P]),
    ("fdas_correlate_fourier2", _I, [_P, _I64, _P, _P, _I, _I, _I, _P, _P]),
    ("fdas_correlate_fourier2_ex", _I, [_P, _I64, _P, _P, _I, _I, _I, _P, _I, _P]),
    ("fdas_r2c_workspace_bytes", _SZ, [_I64]),
    ("fdas_r2c", _I, [_P, _I64, ctypes.c_float, _P, _P, _SZ, _P]),
    ("fdas_harmonic_shape", _I, [_I64, _I, _I, ctypes.POINTER(_I), ctypes.POINTER(_I64)]),
    ("fdas_harmonic_sum", _I, [_P, _I64, _I, _I, _P, _P, _P]),
    ("fdas_find_candidates", _I, [_P, _I64, _I, _I, ctypes.c_float, _P, _I, _P, _P]),
    ("fdas_harmonic_batched_workspace_bytes", _SZ, [_I]),
    ("fdas_harmonic_sum_batched", _I, [_P, _P, _I, _I, _I, _P, _P, _P, _SZ, _P]),
    ("fdas_find_candidates_batched", _I, [_P, _P, _I, _I, _I, ctypes.c_float, _P, _I, _P, _P,
                                          _SZ, _P]),
    ("fdas_r2c_batched_workspace_bytes", _SZ, [_I64, _I]),
    ("fdas_r2c_batched", _I, [_P, _I64, _I, ctypes.c_float, _P, _P, _SZ, _P]),
    ("fdas_stream_write", _I, [_P, _I64, ctypes.c_float, _P]),
    ("fdas_stream_read", _I, [_P, _I64, _P, _P]),
    ("fdas_lds_probe", _I, [_P, _I, _I, _I, _P, _P, _P]),
]

# partial sums written by fdas_stream_read
STREAM_PARTIALS = 2048

# fdas_candidate: {int64 r; int32 row; float power} (16 bytes)
CANDIDATE_BYTES = 16


class FdasError(RuntimeError):
    def __init__(self, status: int, where: str, detail: str):
        self.status = status
        super().__init__(f"{where}: status {status} ({status_string(status)}): {detail}")


_lib = None


def lib() -> ctypes.CDLL:
    """The loaded library (raises if it has not been built)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise ImportError(f"{LIB_PATH} is missing: build it with "
                              "`python -m paper_1804_05335_amd.build` (no fallback exists)")
        L = ctypes.CDLL(LIB_PATH)
        for name, res, args in SIGNATURES:
            fn = getattr(L, name)
            fn.restype = res
            fn.argtypes = args
        _lib = L
    return _lib


def status_string(status: int) -> str:
    return lib().fdas_status_string(status).decode()


def _check(status: int, where: str) -> None:
    if status != FDAS_OK:
        raise FdasError(status, where, lib().fdas_last_error().decode())


def _ptr(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


def _stream(stream, t):
    if stream is not None:
        return ctypes.c_void_p(int(stream))
    import torch
    return ctypes.c_void_p(torch.cuda.current_stream(t.device).cuda_stream)


def _require(t, dtype, name, numel=None):
    import torch
    if not isinstance(t, torch.Tensor):
        raise TypeError(f"{name} must be a torch tensor")
    if t.dtype != dtype:
        raise TypeError(f"{name} must be {dtype}, got {t.dtype}")
    if not t.is_cuda:
        raise ValueError(f"{name} must be a device tensor")
    if not t.is_contiguous():
        raise ValueError(f"{name} must be contiguous")
    if numel is not None and t.numel() < numel:
        raise ValueError(f"{name} has {t.numel()} elements, needs {numel}")


# ---- host-only calls ---------------------------------------------------------

def fdas_version() -> str:
    return lib().fdas_version().decode()


def fdas_num_templates(zmax: float, dz: float) -> int:
    K = ctypes.c_int(0)
    _check(lib().fdas_num_templates(zmax, dz, ctypes.byref(K)), "fdas_num_templates")
    return K.value


def fdas_template_response(q: float, z: float) -> complex:
    re, im = ctypes.c_double(), ctypes.c_double()
    _check(lib().fdas_template_response(q, z, ctypes.byref(re), ctypes.byref(im)),
           "fdas_template_response")
    return complex(re.value, im.value)


def fdas_make_templates_host(zmax: float, dz: float, M: int):
    """Template bank T[K][M] as a numpy complex64 array (host FP64, rounded once)."""
    import numpy as np
    K = fdas_num_templates(zmax, dz)
    out = np.empty((K, M), dtype=np.complex64)
    _check(lib().fdas_make_templates_host(zmax, dz, M, out.ctypes.data_as(ctypes.c_void_p)),
           "fdas_make_templates_host")
    return out


def fdas_bank_elems(K: int, L: int) -> int:
    return int(lib().fdas_bank_elems(K, L))


# ---- device calls --------------------------------------------------------------

def fdas_prepare_bank(taps, K: int, M: int, L: int, bank, stream=None) -> None:
    import torch
    _require(taps, torch.complex64, "taps", K * M)
    _require(bank, torch.complex64, "bank", fdas_bank_elems(K, L))
    _check(lib().fdas_prepare_bank(_ptr(taps), K, M, L, _ptr(bank), _stream(stream, taps)),
           "fdas_prepare_bank")


def fdas_make_templates(zmax: float, dz: float, M: int, L: int, taps, bank=None,
                        stream=None) -> None:
    import torch
    K = fdas_num_templates(zmax, dz)
    _require(taps, torch.complex64, "taps", K * M)
    if bank is not None:
        _require(bank, torch.complex64, "bank", fdas_bank_elems(K, L))
    _check(lib().fdas_make_templates(zmax, dz, M, L, _ptr(taps), _ptr(bank),
                                     _stream(stream, taps)), "fdas_make_templates")


def fdas_correlate(spec, N: int, bank, K: int, M: int, L: int, plane, stream=None) -> None:
    import torch
    _require(spec, torch.complex64, "spec", N)
    _require(bank, torch.complex64, "bank", fdas_bank_elems(K, L))
    _require(plane, torch.float32, "plane", K * N)
    _check(lib().fdas_correlate(_ptr(spec), N, _ptr(bank), K, M, L, _ptr(plane),
                                _stream(stream, spec)), "fdas_correlate")


def fdas_correlate_ex(spec, N: int, bank, K: int, M: int, L: int, plane, grid: int,
                      stream=None) -> None:
    import torch
    _require(spec, torch.complex64, "spec", N)
    _require(bank, torch.complex64, "bank", fdas_bank_elems(K, L))
    _require(plane, torch.float32, "plane", K * N)
    _check(lib().fdas_correlate_ex(_ptr(spec), N, _ptr(bank), K, M, L, _ptr(plane), grid,
                                   _stream(stream, spec)), "fdas_correlate_ex")


def fdas_correlate_interbin(spec, N: int, bank, K: int, M: int, L: int, plane2,
                            stream=None) -> None:
    fdas_correlate_interbin_ex(spec, N, bank, K, M, L, plane2, 0, stream)


def fdas_correlate_interbin_ex(spec, N: int, bank, K: int, M: int, L: int, plane2, grid: int,
                               stream=None) -> None:
    import torch
    _require(spec, torch.complex64, "spec", N)
    _require(bank, torch.complex64, "bank", fdas_bank_elems(K, L))
    _require(plane2, torch.float32, "plane2", 2 * K * N)
    _check(lib().fdas_correlate_interbin_ex(_ptr(spec), N, _ptr(bank), K, M, L, _ptr(plane2),
                                            grid, _stream(stream, spec)),
           "fdas_correlate_interbin")


def fdas_batched_workspace_bytes(nspec: int) -> int:
    return int(lib().fdas_batched_workspace_bytes(nspec))


def batched_capacity(specs, planes, K: int) -> int:
    """Bins a packed batch's buffers hold: specs elements, and planes floats
    over K (the call clamps the device offsets to this)."""
    return min(specs.numel(), planes.numel() // K)


def fdas_correlate_batched(specs, offsets, nspec: int, bank, K: int, M: int, L: int, planes,
                           ws, stream=None) -> None:
    fdas_correlate_batched_ex(specs, offsets, nspec, bank, K, M, L, planes, 0, 0, ws, stream)


def fdas_correlate_batched_ex(specs, offsets, nspec: int, bank, K: int, M: int, L: int, planes,
                              E: int, grid: int, ws, stream=None) -> None:
    import torch
    _require(specs, torch.complex64, "specs")
    _require(offsets, torch.int64, "offsets", nspec + 1)
    _require(bank, torch.complex64, "bank", fdas_bank_elems(K, L))
    _require(planes, torch.float32, "planes")
    _require(ws, torch.uint8, "ws", fdas_batched_workspace_bytes(nspec))
    _check(lib().fdas_correlate_batched_ex(_ptr(specs), _ptr(offsets), nspec,
                                           batched_capacity(specs, planes, K), _ptr(bank), K, M,
                                           L, _ptr(planes), E, grid, _ptr(ws), ws.numel(),
                                           _stream(stream, specs)),
           "fdas_correlate_batched")


# most spectra fdas_correlate_batched_noalloc takes (its fixed device array)
NOALLOC_MAX_SPECTRA = 65536


def fdas_correlate_batched_noalloc(specs, offsets, nspec: int, bank, K: int, M: int, L: int,
                                   planes, stream=None) -> None:
    """fdas_correlate_batched without a workspace (the library's fixed device
    array holds the segment prefix): for callers that cannot allocate."""
    import torch
    _require(specs, torch.complex64, "specs")
    _require(offsets, torch.int64, "offsets", nspec + 1)
    _require(bank, torch.complex64, "bank", fdas_bank_elems(K, L))
    _require(planes, torch.float32, "planes")
    _check(lib().fdas_correlate_batched_noalloc(_ptr(specs), _ptr(offsets), nspec,
                                                batched_capacity(specs, planes, K), _ptr(bank),
                                                K, M, L, _ptr(planes), _stream(stream, specs)),
           "fdas_correlate_batched_noalloc")


def fdas_backward_workspace_bytes(N: int, K: int, M: int, L: int, zchunk: int = 0) -> int:
    return int(lib().fdas_backward_workspace_bytes(N, K, M, L, zchunk))


def fdas_correlate_backward(spec, N: int, bank, K: int, M: int, L: int, dLdP, grad_spec,
                            grad_taps, ws, stream=None) -> None:
    fdas_correlate_backward_ex(spec, N, bank, K, M, L, dLdP, grad_spec, grad_taps, 0, ws, stream)


def fdas_correlate_backward_ex(spec, N: int, bank, K: int, M: int, L: int, dLdP, grad_spec,
                               grad_taps, zchunk: int, ws, stream=None) -> None:
    import torch
    _require(spec, torch.complex64, "spec", N)
    _require(bank, torch.complex64, "bank", fdas_bank_elems(K, L))
    _require(dLdP, torch.float32, "dLdP", K * N)
    if grad_spec is not None:
        _require(grad_spec, torch.complex64, "grad_spec", N)
    if grad_taps is not None:
        _require(grad_taps, torch.complex64, "grad_taps", K * M)
    _require(ws, torch.uint8, "ws", fdas_backward_workspace_bytes(N, K, M, L, zchunk))
    _check(lib().fdas_correlate_backward_ex(_ptr(spec), N, _ptr(bank), K, M, L, _ptr(dLdP),
                                            _ptr(grad_spec), _ptr(grad_taps), zchunk, _ptr(ws),
                                            ws.numel(), _stream(stream, spec)),
           "fdas_correlate_backward")


def fdas_backward_batched_workspace_bytes(capacity: int, nspec: int, K: int, M: int, L: int,
                                          zchunk: int = 0, want: int = 3) -> int:
    """want: 1 = spectra gradient, 2 = taps gradient, 3 = both."""
    return int(lib().fdas_backward_batched_workspace_bytes(capacity, nspec, K, M, L, zchunk, want))


def fdas_correlate_backward_batched(specs, offsets, nspec: int, bank, K: int, M: int, L: int,
                                    dLdP, grad_specs, grad_taps, ws, zchunk: int = 0,
                                    stream=None) -> None:
    """Adjoint of the batched forward: dLdP packed like the planes, grad_specs
    like the spectra (or None), grad_taps [K][M] summed over the batch (or
    None)."""
    import torch
    _require(specs, torch.complex64, "specs")
    _require(offsets, torch.int64, "offsets", nspec + 1)
    _require(bank, torch.complex64, "bank", fdas_bank_elems(K, L))
    _require(dLdP, torch.float32, "dLdP")
    cap = min(specs.numel(), dLdP.numel() // K)
    if grad_specs is not None:
        _require(grad_specs, torch.complex64, "grad_specs")
        cap = min(cap, grad_specs.numel())
    if grad_taps is not None:
        _require(grad_taps, torch.complex64, "grad_taps", K * M)
    want = (1 if grad_specs is not None else 0) | (2 if grad_taps is not None else 0)
    _require(ws, torch.uint8, "ws",
             fdas_backward_batched_workspace_bytes(cap, nspec, K, M, L, zchunk, want))
    _check(lib().fdas_correlate_backward_batched(_ptr(specs), _ptr(offsets), nspec, cap,
                                                 _ptr(bank), K, M, L, _ptr(dLdP),
                                                 _ptr(grad_specs), _ptr(grad_taps), zchunk,
                                                 _ptr(ws), ws.numel(), _stream(stream, specs)),
           "fdas_correlate_backward_batched")


def fdas_autotune_workspace_bytes(K: int, nspec: int) -> int:
    return int(lib().fdas_autotune_workspace_bytes(K, nspec))


class Tuning(ctypes.Structure):
    """fdas_tuning: a launch shape of the batched forward and its time."""
    _fields_ = [("L", _I), ("E", _I), ("grid_factor", _I), ("grid", _I), ("from_cache", _I),
                ("ms", _D)]

    def as_dict(self) -> dict:
        return {f: getattr(self, f) for f, _ in self._fields_}


TUNE_NO_CACHE = 1
TUNE_REFRESH = 2


def fdas_autotune_candidates(K: int, M: int):
    """The (L, E, grid_factor) shapes the autotuner times, in its order."""
    n = _I(0)
    _check(lib().fdas_autotune_candidates(K, M, None, 0, ctypes.byref(n)),
           "fdas_autotune_candidates")
    arr = (Tuning * n.value)()
    _check(lib().fdas_autotune_candidates(K, M, ctypes.cast(arr, _P), n.value, ctypes.byref(n)),
           "fdas_autotune_candidates")
    return [a.as_dict() for a in arr]


def fdas_batched_resident_grid(L: int, E: int, M: int) -> int:
    g = _I(0)
    _check(lib().fdas_batched_resident_grid(L, E, M, ctypes.byref(g)),
           "fdas_batched_resident_grid")
    return g.value


def fdas_autotune_batched(taps, K: int, M: int, specs, offsets, nspec: int, planes, ws,
                          flags: int = 0, stream=None) -> dict:
    """The fastest launch shape for this batch: a dict with L, E, grid_factor,
    grid (for fdas_correlate_batched_ex), from_cache and ms."""
    import torch
    _require(taps, torch.complex64, "taps", K * M)
    _require(specs, torch.complex64, "specs")
    _require(offsets, torch.int64, "offsets", nspec + 1)
    _require(planes, torch.float32, "planes")
    _require(ws, torch.uint8, "ws", fdas_autotune_workspace_bytes(K, nspec))
    out = Tuning()
    _check(lib().fdas_autotune_batched(_ptr(taps), K, M, _ptr(specs), _ptr(offsets), nspec,
                                       batched_capacity(specs, planes, K), _ptr(planes),
                                       _ptr(ws), ws.numel(), flags, _stream(stream, specs),
                                       ctypes.byref(out)),
           "fdas_autotune_batched")
    return out.as_dict()


def fdas_r2c_workspace_bytes(n: int) -> int:
    return int(lib().fdas_r2c_workspace_bytes(n))


def fdas_r2c(x, n: int, scale: float, spec, ws, stream=None) -> None:
    import torch
    _require(x, torch.float32, "x", n)
    _require(spec, torch.complex64, "spec", n // 2 + 1)
    _require(ws, torch.uint8, "ws", fdas_r2c_workspace_bytes(n))
    _check(lib().fdas_r2c(_ptr(x), n, scale, _ptr(spec), _ptr(ws), ws.numel(),
                          _stream(stream, x)), "fdas_r2c")


def fdas_r2c_batched_workspace_bytes(n: int, nseries: int) -> int:
    return int(lib().fdas_r2c_batched_workspace_bytes(n, nseries))


def fdas_r2c_batched(x, n: int, nseries: int, scale: float, spec, ws, stream=None) -> None:
    import torch
    _require(x, torch.float32, "x", nseries * n)
    _require(spec, torch.complex64, "spec", nseries * (n // 2 + 1))
    _require(ws, torch.uint8, "ws", fdas_r2c_batched_workspace_bytes(n, nseries))
    _check(lib().fdas_r2c_batched(_ptr(x), n, nseries, scale, _ptr(spec), _ptr(ws), ws.numel(),
                                  _stream(stream, x)), "fdas_r2c_batched")


def fdas_bank_sym_elems(K: int, L: int) -> int:
    return int(lib().fdas_bank_sym_elems(K, L))


def fdas_prepare_bank_sym(taps, K: int, M: int, L: int, bank_sym, stream=None) -> None:
    import torch
    _require(taps, torch.complex64, "taps", K * M)
    _require(bank_sym, torch.complex64, "bank_sym", fdas_bank_sym_elems(K, L))
    _check(lib().fdas_prepare_bank_sym(_ptr(taps), K, M, L, _ptr(bank_sym), _stream(stream, taps)),
           "fdas_prepare_bank_sym")


def fdas_correlate_sym(spec, N: int, bank_sym, K: int, M: int, L: int, plane,
                       stream=None) -> None:
    fdas_correlate_sym_ex(spec, N, bank_sym, K, M, L, plane, 0, stream)


def fdas_correlate_sym_ex(spec, N: int, bank_sym, K: int, M: int, L: int, plane, grid: int,
                          stream=None) -> None:
    import torch
    _require(spec, torch.complex64, "spec", N)
    _require(bank_sym, torch.complex64, "bank_sym", fdas_bank_sym_elems(K, L))
    _require(plane, torch.float32, "plane", K * N)
    _check(lib().fdas_correlate_sym_ex(_ptr(spec), N, _ptr(bank_sym), K, M, L, _ptr(plane), grid,
                                       _stream(stream, spec)), "fdas_correlate_sym")


def fdas_make_templates_half(zmax: float, dz: float, M: int, L: int, taps_half, bank_half=None,
                             stream=None) -> None:
    import torch
    K = fdas_num_templates(zmax, dz)
    _require(taps_half, torch.complex64, "taps_half", K * (M + 2))
    if bank_half is not None:
        _require(bank_half, torch.complex64, "bank_half", fdas_bank_elems(K, L))
    _check(lib().fdas_make_templates_half(zmax, dz, M, L, _ptr(taps_half), _ptr(bank_half),
                                          _stream(stream, taps_half)), "fdas_make_templates_half")


def fdas_correlate_fourier2(spec, N: int, bank, bank_half, K: int, M: int, L: int, plane2,
                            stream=None) -> None:
    fdas_correlate_fourier2_ex(spec, N, bank, bank_half, K, M, L, plane2, 0, stream)


def fdas_correlate_fourier2_ex(spec, N: int, bank, bank_half, K: int, M: int, L: int, plane2,
                               grid: int, stream=None) -> None:
    import torch
    _require(spec, torch.complex64, "spec", N)
    _require(bank, torch.complex64, "bank", fdas_bank_elems(K, L))
    _require(bank_half, torch.complex64, "bank_half", fdas_bank_elems(K, L))
    _require(plane2, torch.float32, "plane2", 2 * K * N)
    _check(lib().fdas_correlate_fourier2_ex(_ptr(spec), N, _ptr(bank), _ptr(bank_half), K, M, L,
                                            _ptr(plane2), grid, _stream(stream, spec)),
           "fdas_correlate_fourier2")


def fdas_harmonic_shape(N: int, K: int, H: int):
    """(K_H, N_H) of the H-fold harmonic sum of a [K][N] plane."""
    kh, nh = _I(), _I64()
    _check(lib().fdas_harmonic_shape(N, K, H, ctypes.byref(kh), ctypes.byref(nh)),
           "fdas_harmonic_shape")
    return kh.value, nh.value


def fdas_harmonic_sum(plane, N: int, K: int, H: int, prev, sums, stream=None) -> None:
    import torch
    KH, NH = fdas_harmonic_shape(N, K, H)
    _require(plane, torch.float32, "plane", K * N)
    if prev is not None:
        KHp, NHp = fdas_harmonic_shape(N, K, H // 2)
        _require(prev, torch.float32, "prev", KHp * NHp)
    _require(sums, torch.float32, "sums", KH * NH)
    _check(lib().fdas_harmonic_sum(_ptr(plane), N, K, H, _ptr(prev), _ptr(sums),
                                   _stream(stream, plane)), "fdas_harmonic_sum")


def fdas_find_candidates(sums, N: int, K: int, H: int, threshold: float, out, capacity: int,
                         count, stream=None) -> None:
    """out: uint8 device tensor of capacity * 16 bytes (fdas_candidate
    records); count: int32 device tensor of one element."""
    import torch
    KH, NH = fdas_harmonic_shape(N, K, H)
    _require(sums, torch.float32, "sums", KH * NH)
    _require(out, torch.uint8, "out", capacity * CANDIDATE_BYTES)
    _require(count, torch.int32, "count", 1)
    _check(lib().fdas_find_candidates(_ptr(sums), N, K, H, threshold, _ptr(out), capacity,
                                      _ptr(count), _stream(stream, sums)),
           "fdas_find_candidates")


def fdas_harmonic_batched_workspace_bytes(nspec: int) -> int:
    return int(lib().fdas_harmonic_batched_workspace_bytes(nspec))


def fdas_harmonic_sum_batched(planes, offsets, nspec: int, K: int, H: int, prev, sums, ws,
                              stream=None) -> None:
    """offsets: int64 device tensor of nspec + 1 packed-bin offsets; sizes
    of planes / prev / sums are the caller's (they follow from the host
    copy of the offsets)."""
    import torch
    _require(planes, torch.float32, "planes")
    _require(offsets, torch.int64, "offsets", nspec + 1)
    if prev is not None:
        _require(prev, torch.float32, "prev")
    _require(sums, torch.float32, "sums")
    _require(ws, torch.uint8, "ws", fdas_harmonic_batched_workspace_bytes(nspec))
    _check(lib().fdas_harmonic_sum_batched(_ptr(planes), _ptr(offsets), nspec, K, H, _ptr(prev),
                                           _ptr(sums), _ptr(ws), ws.numel(),
                                           _stream(stream, planes)),
           "fdas_harmonic_sum_batched")


def fdas_find_candidates_batched(sums, offsets, nspec: int, K: int, H: int, threshold: float,
                                 out, capacity: int, count, ws, stream=None) -> None:
    import torch
    _require(sums, torch.float32, "sums")
    _require(offsets, torch.int64, "offsets", nspec + 1)
    _require(out, torch.uint8, "out", capacity * CANDIDATE_BYTES)
    _require(count, torch.int32, "count", 1)
    _require(ws, torch.uint8, "ws", fdas_harmonic_batched_workspace_bytes(nspec))
    _check(lib().fdas_find_candidates_batched(_ptr(sums), _ptr(offsets), nspec, K, H, threshold,
                                              _ptr(out), capacity, _ptr(count), _ptr(ws),
                                              ws.numel(), _stream(stream, sums)),
           "fdas_find_candidates_batched")


def fdas_stream_write(dst, value: float, stream=None) -> None:
    """dst (float32 device tensor, 16-byte aligned) filled with `value` by
    the streaming write probe."""
    import torch
    _require(dst, torch.float32, "dst")
    _check(lib().fdas_stream_write(_ptr(dst), dst.numel(), value, _stream(stream, dst)),
           "fdas_stream_write")


def fdas_stream_read(src, sums, stream=None) -> None:
    """Streaming read probe: STREAM_PARTIALS partial sums of src (float32
    device tensor, 16-byte aligned) into sums."""
    import torch
    _require(src, torch.float32, "src")
    _require(sums, torch.float32, "sums", STREAM_PARTIALS)
    _check(lib().fdas_stream_read(_ptr(src), src.numel(), _ptr(sums), _stream(stream, src)),
           "fdas_stream_read")


def fdas_lds_probe(pattern, mode: int, iters: int, groups: int, cycles, sink,
                   stream=None) -> None:
    """LDS bank probe: pattern int32[64] (device), mode 0/1/2 = 64-bit
    write / 64-bit read / 128-bit write; cycles int64[groups], sink
    float32[64 * groups]."""
    import torch
    _require(pattern, torch.int32, "pattern", 64)
    _require(cycles, torch.int64, "cycles", groups)
    _require(sink, torch.float32, "sink", 64 * groups)
    _check(lib().fdas_lds_probe(_ptr(pattern), mode, iters, groups, _ptr(cycles), _ptr(sink),
                                _stream(stream, pattern)),
           "fdas_lds_probe")
