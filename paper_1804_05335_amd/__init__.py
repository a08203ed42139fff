"""MI355X-native FDAS correlation (Dimoudi et al. 2018) -- Python surface.

The work happens in ``libfdas.so`` (hand-written HIP for gfx950, C ABI in
``include/fdas.h``); this package marshals torch device tensors into it.
There is no CPU fallback: if the library is missing, calls raise.

    import torch, paper_1804_05335_amd as fdas
    taps, bank = fdas.make_bank(zmax=84, dz=2, M=256, L=2048)
    plane = fdas.correlate(spec, bank, K=taps.shape[0], M=256, L=2048)
"""
from __future__ import annotations

from ._lib import (FdasError, fdas_bank_elems, fdas_correlate, fdas_correlate_ex,  # noqa: F401
                   fdas_make_templates, fdas_make_templates_host, fdas_num_templates,
                   fdas_prepare_bank, fdas_template_response, fdas_version, lib)


def make_bank(zmax: float, dz: float, M: int, L: int, device="cuda"):
    """Templates (K x M complex64) and the prepared bank for segment length L."""
    import torch
    K = fdas_num_templates(zmax, dz)
    taps = torch.empty(K * M, dtype=torch.complex64, device=device)
    bank = torch.empty(fdas_bank_elems(K, L), dtype=torch.complex64, device=device)
    fdas_make_templates(zmax, dz, M, L, taps, bank)
    return taps.view(K, M), bank


def prepare_bank(taps, L: int):
    """Prepared bank for arbitrary taps (K x M complex64 device tensor)."""
    import torch
    K, M = taps.shape
    bank = torch.empty(fdas_bank_elems(K, L), dtype=torch.complex64, device=taps.device)
    fdas_prepare_bank(taps.contiguous(), K, M, L, bank)
    return bank


def correlate(spec, bank, K: int, M: int, L: int, plane=None, zchunk: int = 0):
    """f-fdot power plane [K][N] float32 of one complex64 spectrum."""
    import torch
    N = spec.numel()
    if plane is None:
        plane = torch.empty((K, N), dtype=torch.float32, device=spec.device)
    fdas_correlate_ex(spec, N, bank, K, M, L, plane, zchunk)
    return plane
