"""torch.autograd.Function around the fused forward and the adjoint kernels.

    plane = FdasCorrelate.apply(spec, taps, L)     # spec [N] c64, taps [K][M] c64
    (plane * w).sum().backward()                   # spec.grad, taps.grad

Forward prepares the bank from the taps and runs fdas_correlate; backward
runs fdas_correlate_backward, which recomputes the segment FFTs instead of
storing the complex plane.  Saved for backward: the spectrum, the taps and
the prepared bank ((K + 1) x L complex).  Gradients follow PyTorch's complex
convention (dL/dRe + i dL/dIm).
"""
from __future__ import annotations

import torch

from . import _lib


class FdasCorrelate(torch.autograd.Function):
    @staticmethod
    def forward(ctx, spec, taps, L: int):
        K, M = taps.shape
        spec_c = spec.detach().contiguous()
        taps_c = taps.detach().contiguous()
        bank = torch.empty(_lib.fdas_bank_elems(K, L), dtype=torch.complex64, device=spec.device)
        _lib.fdas_prepare_bank(taps_c, K, M, L, bank)
        N = spec_c.numel()
        plane = torch.empty((K, N), dtype=torch.float32, device=spec.device)
        _lib.fdas_correlate_ex(spec_c, N, bank, K, M, L, plane, 0)
        ctx.save_for_backward(spec_c, bank)
        ctx.L, ctx.K, ctx.M = L, K, M
        return plane

    @staticmethod
    def backward(ctx, grad_plane):
        spec, bank = ctx.saved_tensors
        L, K, M = ctx.L, ctx.K, ctx.M
        N = spec.numel()
        need_spec, need_taps = ctx.needs_input_grad[0], ctx.needs_input_grad[1]
        if not (need_spec or need_taps):
            return None, None, None
        w = grad_plane.to(torch.float32).contiguous()
        gs = torch.empty(N, dtype=torch.complex64, device=spec.device) if need_spec else None
        gt = torch.empty((K, M), dtype=torch.complex64, device=spec.device) if need_taps else None
        ws = torch.empty(_lib.fdas_backward_workspace_bytes(N, K, M, L, 0), dtype=torch.uint8,
                         device=spec.device)
        _lib.fdas_correlate_backward(spec, N, bank, K, M, L, w, gs, gt, ws)
        return gs, gt, None


def correlate(spec, taps, L: int):
    """Differentiable f-fdot plane [K][N] of spectrum ``spec`` with ``taps``."""
    return FdasCorrelate.apply(spec, taps, L)
