"""MI355X-native FDAS correlation (Dimoudi et al. 2018) -- Python surface.

The work happens in ``libfdas.so`` (hand-written HIP for gfx950, C ABI in
``include/fdas.h``); this package marshals torch device tensors into it.
There is no CPU fallback: if the library is missing, calls raise.

    import torch, paper_1804_05335_amd as fdas
    taps, bank = fdas.make_bank(zmax=84, dz=2, M=256, L=2048)
    plane = fdas.correlate(spec, bank, K=taps.shape[0], M=256, L=2048)
"""
from __future__ import annotations

from ._lib import (FdasError, fdas_backward_workspace_bytes, fdas_bank_elems,  # noqa: F401
                   fdas_batched_workspace_bytes, fdas_correlate, fdas_correlate_backward,
                   fdas_correlate_backward_ex, fdas_correlate_batched,
                   fdas_correlate_batched_ex, fdas_correlate_ex, fdas_correlate_interbin,
                   fdas_correlate_interbin_ex, fdas_make_templates,
                   fdas_make_templates_host, fdas_num_templates, fdas_prepare_bank,
                   fdas_r2c, fdas_r2c_workspace_bytes, fdas_template_response, fdas_version,
                   fdas_bank_sym_elems, fdas_correlate_sym, fdas_correlate_sym_ex,
                   fdas_prepare_bank_sym, fdas_make_templates_half, fdas_correlate_fourier2,
                   fdas_correlate_fourier2_ex, fdas_harmonic_shape, fdas_harmonic_sum,
                   fdas_find_candidates, fdas_harmonic_batched_workspace_bytes,
                   fdas_harmonic_sum_batched, fdas_find_candidates_batched,
                   fdas_stream_write, fdas_stream_read, fdas_r2c_batched,
                   fdas_r2c_batched_workspace_bytes, fdas_correlate_backward_batched,
                   fdas_backward_batched_workspace_bytes, fdas_autotune_batched,
                   fdas_autotune_candidates, fdas_batched_resident_grid,
                   fdas_correlate_batched_noalloc, fdas_lds_probe, lib)


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


def correlate(spec, bank, K: int, M: int, L: int, plane=None, grid: int = 0):
    """f-fdot power plane [K][N] float32 of one complex64 spectrum
    (grid: persistent workgroups, 0 = fill the device)."""
    import torch
    N = spec.numel()
    if plane is None:
        plane = torch.empty((K, N), dtype=torch.float32, device=spec.device)
    fdas_correlate_ex(spec, N, bank, K, M, L, plane, grid)
    return plane


def correlate_interbin(spec, bank, K: int, M: int, L: int, plane2=None, grid: int = 0):
    """Interbinned plane [K][2N] (Sec. 3, eq. f-interp): even columns the bin
    powers, odd columns the half-bin estimates |(pi/4)(Y_r - Y_r+1)|^2."""
    import torch
    N = spec.numel()
    if plane2 is None:
        plane2 = torch.empty((K, 2 * N), dtype=torch.float32, device=spec.device)
    fdas_correlate_interbin_ex(spec, N, bank, K, M, L, plane2, grid)
    return plane2


def pack(spectra, device="cuda"):
    """Pack a list of 1-D complex64 spectra: (specs, offsets[nspec+1] int64)."""
    import torch
    lens = [int(s.numel()) for s in spectra]
    offs = torch.zeros(len(lens) + 1, dtype=torch.int64)
    if lens:
        offs[1:] = torch.cumsum(torch.tensor(lens, dtype=torch.int64), 0)
    specs = torch.cat([s.reshape(-1).to(device) for s in spectra]) if spectra else \
        torch.zeros(0, dtype=torch.complex64, device=device)
    return specs.contiguous(), offs.to(device)


def correlate_batched(specs, offsets, bank, K: int, M: int, L: int, planes=None, ws=None,
                      grid: int = 0, E: int = 0):
    """Planes of packed spectra in one persistent launch.

    ``offsets`` is the device int64 tensor of nspec + 1 offsets; plane b is
    ``planes[K*offsets[b] : K*offsets[b+1]].view(K, N_b)``.  ``planes`` and
    the workspace ``ws`` are allocated when not given (pass them to keep the
    call allocation-free, e.g. under graph capture).  ``E`` and ``grid`` are
    the launch shape (0 = defaults; see fdas_autotune_batched).
    """
    import torch
    from ._lib import fdas_batched_workspace_bytes, fdas_correlate_batched_ex
    nspec = offsets.numel() - 1
    if planes is None:
        total = int(offsets[-1].item()) if nspec >= 0 else 0
        planes = torch.empty(K * total, dtype=torch.float32, device=specs.device)
    if ws is None:
        ws = torch.empty(max(fdas_batched_workspace_bytes(nspec), 1), dtype=torch.uint8,
                         device=specs.device)
    fdas_correlate_batched_ex(specs, offsets, nspec, bank, K, M, L, planes, E, grid, ws)
    return planes


def correlate_backward_batched(specs, offsets, bank, K: int, M: int, L: int, dLdP,
                               want_spectra: bool = True, want_taps: bool = True, ws=None,
                               zchunk: int = 0):
    """Gradients of Lw = sum_b sum w_b P_b for a packed batch: (grad_specs
    packed like ``specs`` or None, grad_taps [K][M] summed over the batch or
    None).  ``dLdP`` is packed like the planes of correlate_batched."""
    import torch
    nspec = offsets.numel() - 1
    cap = min(specs.numel(), dLdP.numel() // K)
    gs = torch.empty(cap, dtype=torch.complex64, device=specs.device) if want_spectra else None
    gt = torch.empty((K, M), dtype=torch.complex64, device=specs.device) if want_taps else None
    want = (1 if want_spectra else 0) | (2 if want_taps else 0)
    if ws is None:
        ws = torch.empty(max(fdas_backward_batched_workspace_bytes(cap, nspec, K, M, L, zchunk,
                                                                   want), 1),
                         dtype=torch.uint8, device=specs.device)
    fdas_correlate_backward_batched(specs, offsets, nspec, bank, K, M, L, dLdP, gs, gt, ws,
                                    zchunk)
    return gs, gt


def spectrum_from_series(x, scale: float = 1.0, spec=None, ws=None):
    """Real-to-complex transform of a float32 device time series of n
    samples: the n/2 + 1 bins scale * sum_t x[t] exp(-2 pi i k t / n).
    ``spec`` and the workspace ``ws`` are allocated when not given."""
    import torch
    n = x.numel()
    if spec is None:
        spec = torch.empty(n // 2 + 1, dtype=torch.complex64, device=x.device)
    if ws is None:
        ws = torch.empty(max(fdas_r2c_workspace_bytes(n), 1), dtype=torch.uint8, device=x.device)
    fdas_r2c(x, n, scale, spec, ws)
    return spec


def spectra_from_series(x, scale: float = 1.0):
    """Real-to-complex transform of nseries equal-length float32 device time
    series (a [nseries][n] tensor) in one launch per pass: a [nseries][n/2 + 1]
    complex64 tensor, each row bitwise the spectrum_from_series of its
    series.  With offsets b (n/2 + 1), b = 0 .. nseries, its flat view is a
    packed batch for correlate_batched (spectra of n/2 + 1 bins)."""
    import torch
    nseries, n = x.shape
    spec = torch.empty((nseries, n // 2 + 1), dtype=torch.complex64, device=x.device)
    ws = torch.empty(max(fdas_r2c_batched_workspace_bytes(n, nseries), 1), dtype=torch.uint8,
                     device=x.device)
    fdas_r2c_batched(x.contiguous().view(-1), n, nseries, scale, spec.view(-1), ws)
    return spec


def prepare_bank_sym(taps, L: int):
    """Symmetric bank (rows z >= 0 only) from K x M templates, K odd."""
    import torch
    K, M = taps.shape
    bank = torch.empty(fdas_bank_sym_elems(K, L), dtype=torch.complex64, device=taps.device)
    fdas_prepare_bank_sym(taps.contiguous(), K, M, L, bank)
    return bank


def correlate_sym(spec, bank_sym, K: int, M: int, L: int, plane=None, grid: int = 0):
    """fdas_correlate with a symmetric bank: the same K x N plane."""
    import torch
    N = spec.numel()
    if plane is None:
        plane = torch.empty((K, N), dtype=torch.float32, device=spec.device)
    fdas_correlate_sym_ex(spec, N, bank_sym, K, M, L, plane, grid)
    return plane


def make_bank_half(zmax: float, dz: float, M: int, L: int, device="cuda"):
    """Half-bin templates (K x (M+2)) and their bank for the two-bin Fourier
    interpolation."""
    import torch
    K = fdas_num_templates(zmax, dz)
    taps = torch.empty(K * (M + 2), dtype=torch.complex64, device=device)
    bank = torch.empty(fdas_bank_elems(K, L), dtype=torch.complex64, device=device)
    fdas_make_templates_half(zmax, dz, M, L, taps, bank)
    return taps.view(K, M + 2), bank


def correlate_fourier2(spec, bank, bank_half, K: int, M: int, L: int, plane2=None, grid: int = 0):
    """[K][2N] plane: integer bins in the even columns, the half-bin matched
    filter in the odd ones."""
    import torch
    N = spec.numel()
    if plane2 is None:
        plane2 = torch.empty((K, 2 * N), dtype=torch.float32, device=spec.device)
    fdas_correlate_fourier2_ex(spec, N, bank, bank_half, K, M, L, plane2, grid)
    return plane2


def harmonic_sums(plane, max_fold: int):
    """[S_1 = plane, S_2, S_4, ..., S_max_fold] of a [K][N] float32 plane
    (Sec. 3 harmonic summing), each fold built on the previous one."""
    import torch
    K, N = plane.shape
    folds = [plane]
    H = 2
    while H <= max_fold:
        KH, NH = fdas_harmonic_shape(N, K, H)
        out = torch.empty((KH, NH), dtype=torch.float32, device=plane.device)
        fdas_harmonic_sum(plane, N, K, H, folds[-1] if H > 2 else None, out)
        folds.append(out)
        H *= 2
    return folds


def candidates(sums, N: int, K: int, H: int, threshold: float, capacity: int = 1 << 16):
    """Peaks of one fold above `threshold` (Sec. 3): (r int64, row int32,
    power float32) host arrays sorted by (row, r), and the total count
    (which may exceed `capacity`; then only `capacity` are returned)."""
    import numpy as np
    import torch
    out = torch.empty(max(capacity, 1) * 16, dtype=torch.uint8, device=sums.device)
    count = torch.zeros(1, dtype=torch.int32, device=sums.device)
    fdas_find_candidates(sums, N, K, H, threshold, out, capacity, count)
    n = int(count.item())
    rec = np.frombuffer(out.cpu().numpy().tobytes(), dtype=np.dtype(
        [("r", "<i8"), ("row", "<i4"), ("power", "<f4")]))[:min(n, capacity)]
    order = np.lexsort((rec["r"], rec["row"]))
    rec = rec[order]
    return rec["r"].copy(), rec["row"].copy(), rec["power"].copy(), n


def search(x, zmax: float, dz: float, M: int, L: int, max_fold: int, thresholds,
           capacity: int = 1 << 16):
    """The search path of Sec. 3 on one device time series: real-to-complex
    transform (scaled by 1/sqrt(n), so white noise of unit variance gives
    unit mean power), the f-fdot plane, harmonic sums up to ``max_fold``
    and the peaks of each fold above ``thresholds[H]`` (a dict keyed by the
    fold, 1 = the plane itself; folds without a threshold are skipped).
    Returns {H: (r, row, power, count)} with the candidates of each fold as
    host arrays sorted by (row, r); the fundamental's drift is
    z = (row - (K - 1)/2) dz.  Every step runs in the library's kernels."""
    n = x.numel()
    N = n // 2
    spec = spectrum_from_series(x, 1.0 / float(n) ** 0.5)[:N].contiguous()
    taps, bank = make_bank(zmax, dz, M, L, device=x.device)
    K = taps.shape[0]
    plane = correlate(spec, bank, K, M, L)
    folds = harmonic_sums(plane, max_fold)
    out = {}
    H = 1
    for S in folds:
        if H in thresholds:
            out[H] = candidates(S, N, K, H, float(thresholds[H]), capacity)
        H *= 2
    return out


def fold_prefix(offsets_host, H: int):
    """C_H[b] = sum_{b' < b} ceil(N_b'/H) for packed-bin offsets (host int64
    array of nspec + 1): fold H of spectrum b starts at K_H * C_H[b]."""
    import numpy as np
    lens = np.maximum(np.diff(np.asarray(offsets_host, dtype=np.int64)), 0)
    pre = np.zeros(len(lens) + 1, dtype=np.int64)
    np.cumsum((lens + H - 1) // H, out=pre[1:])
    return pre


def harmonic_sums_batched(planes, offsets, K: int, max_fold: int):
    """Folds 2, 4, .., max_fold of the planes of correlate_batched (flat
    float32 device tensor; offsets the int64 device tensor of nspec + 1
    packed-bin offsets), each fold built on the previous one in one launch
    for all spectra.  Returns the list [planes, S_2, S_4, ...] of flat
    tensors; fold H of spectrum b is S_H[K_H C_H[b] : K_H C_H[b+1]] viewed
    as [K_H][ceil(N_b/H)] (see fold_prefix)."""
    import torch
    offs = offsets.cpu().numpy()
    nspec = len(offs) - 1
    ws = torch.empty(max(fdas_harmonic_batched_workspace_bytes(nspec), 1), dtype=torch.uint8,
                     device=planes.device)
    folds = [planes]
    H = 2
    while H <= max_fold:
        KH, _ = fdas_harmonic_shape(0, K, H)
        total = int(fold_prefix(offs, H)[-1])
        out = torch.empty(max(KH * total, 1), dtype=torch.float32, device=planes.device)
        fdas_harmonic_sum_batched(planes, offsets, nspec, K, H, folds[-1] if H > 2 else None,
                                  out, ws)
        folds.append(out)
        H *= 2
    return folds


def candidates_batched(sums, offsets, K: int, H: int, threshold: float, capacity: int = 1 << 16):
    """Peaks above `threshold` of fold H of every spectrum: (spectrum int64,
    r int64, row int32, power float32) host arrays sorted by (spectrum, row,
    r), and the total count."""
    import numpy as np
    import torch
    nspec = offsets.numel() - 1
    ws = torch.empty(max(fdas_harmonic_batched_workspace_bytes(nspec), 1), dtype=torch.uint8,
                     device=sums.device)
    out = torch.empty(max(capacity, 1) * 16, dtype=torch.uint8, device=sums.device)
    count = torch.zeros(1, dtype=torch.int32, device=sums.device)
    fdas_find_candidates_batched(sums, offsets, nspec, K, H, threshold, out, capacity, count, ws)
    n = int(count.item())
    rec = np.frombuffer(out.cpu().numpy().tobytes(), dtype=np.dtype(
        [("r", "<i8"), ("row", "<i4"), ("power", "<f4")]))[:min(n, capacity)]
    offs = offsets.cpu().numpy()
    spec = np.searchsorted(offs, rec["r"], side="right") - 1
    r = rec["r"] - offs[spec]
    order = np.lexsort((r, rec["row"], spec))
    return spec[order], r[order], rec["row"][order].copy(), rec["power"][order].copy(), n


def search_batched(x, zmax: float, dz: float, M: int, L: int, max_fold: int, thresholds,
                   capacity: int = 1 << 16):
    """The search path of Sec. 3 on nseries equal-length device time series
    (a float32 [nseries][n] tensor), each step one launch (per pass or fold)
    for the whole batch: real-to-complex transforms scaled by 1/sqrt(n), the
    planes, harmonic sums up to ``max_fold`` and the peaks of each fold above
    ``thresholds[H]``.  Each spectrum keeps its Nyquist bin (n/2 + 1 bins),
    as the batched transform packs them.  Returns {H: (series, r, row, power,
    count)} with host arrays sorted by (series, row, r)."""
    import torch
    nseries, n = x.shape
    nb = n // 2 + 1
    specs = spectra_from_series(x, 1.0 / float(n) ** 0.5)
    offs = torch.arange(nseries + 1, dtype=torch.int64, device=x.device) * nb
    taps, bank = make_bank(zmax, dz, M, L, device=x.device)
    K = taps.shape[0]
    planes = correlate_batched(specs.view(-1), offs, bank, K, M, L)
    folds = harmonic_sums_batched(planes, offs, K, max_fold)
    out = {}
    H = 1
    for S in folds:
        if H in thresholds:
            out[H] = candidates_batched(S, offs, K, H, float(thresholds[H]), capacity)
        H *= 2
    return out

