"""GPU checks at the large-zmax geometry: 201 templates (z = -200..200 step 2)
x 512 taps, segment 8192, 64 ragged spectra of 2^21..2^22 bins.

- batched forward over all 64 spectra (plane ~156 GB in HBM), sampled
  against the FP64 oracle;
- gradient w.r.t. a full-length input spectrum (the adjoint recomputes the
  segment FFTs, no complex plane is stored), sampled bins against the oracle's
  per-bin gradient;
- full gradients (spectrum and taps) at the same geometry on a shortened
  spectrum against the oracle's full adjoint.
"""
import numpy as np
import pytest

import fdas_synth as syn
from oracle import native
from oracle import templates as ot

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

TOL = 1e-5


@pytest.fixture(scope="module")
def fd():
    import paper_1804_05335_amd as f
    f.lib()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return f


@pytest.fixture(scope="module")
def w5():
    return syn.workload(5)


def _rel(got, ref):
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


def test_workload5_batched_forward_sampled(fd, w5):
    K, M, L = w5.K, w5.M, w5.L
    taps, bank = fd.make_bank(w5.zmax, w5.dz, M, L)
    packed, o = w5.packed()
    specs = torch.from_numpy(packed).cuda()
    offs = torch.from_numpy(o).cuda()
    planes = fd.correlate_batched(specs, offs, bank, K, M, L)
    torch.cuda.synchronize()
    T = ot.templates(w5.zmax, w5.dz, M)
    rng = np.random.default_rng(5)
    B = L - M
    for b in (0, 31, 63):
        n = len(w5.spectra[b])
        view = planes[K * o[b]:K * o[b + 1]].view(K, n)
        bounds = ((np.arange(1, -(-n // B)) * B)[:, None] + np.arange(-2, 3)[None, :]).ravel()
        sig = np.concatenate([int(r) + np.arange(-4, 5) for _, _, r, _ in w5.signals[b]])
        cols = np.unique(np.concatenate([np.arange(0, 32), np.arange(n - 32, n), bounds, sig,
                                         rng.integers(0, n, 400)]))
        cols = cols[(cols >= 0) & (cols < n)]
        zi = np.repeat(np.arange(K), len(cols)).astype(np.int32)
        ri = np.tile(cols, K).astype(np.int64)
        got = view[torch.from_numpy(zi.astype(np.int64)).cuda(),
                   torch.from_numpy(ri).cuda()].cpu().numpy()
        ref = native.power_points(w5.spectra[b], T, zi, ri)
        assert _rel(got, ref) < TOL, b
    # checked in slices: an elementwise mask of the whole ~146 GB plane would
    # not fit next to it
    for part in planes.split(1 << 30):
        assert bool(torch.isfinite(part).all())
    del planes
    torch.cuda.empty_cache()


def _grad_spec(fd, spec, bank, K, M, L, w):
    N = spec.numel()
    gs = torch.empty(N, dtype=torch.complex64, device="cuda")
    ws = torch.empty(fd.fdas_backward_workspace_bytes(N, K, M, L, 0), dtype=torch.uint8,
                     device="cuda")
    fd.fdas_correlate_backward(spec, N, bank, K, M, L, w, gs, None, ws)
    torch.cuda.synchronize()
    return gs


def test_workload5_spectrum_gradient_full_length_sampled(fd, w5):
    K, M, L = w5.K, w5.M, w5.L
    _, bank = fd.make_bank(w5.zmax, w5.dz, M, L)
    b = int(np.argmax(w5.lengths))                       # the longest spectrum
    A = w5.spectra[b]
    N = len(A)
    w = np.random.default_rng(55).random((K, N), dtype=np.float32)
    gs = _grad_spec(fd, torch.from_numpy(A).cuda(), bank, K, M, L, torch.from_numpy(w).cuda())
    B = L - M
    rng = np.random.default_rng(56)
    ks = np.unique(np.concatenate([[0, 1, N - 1, N - 2, B - 1, B, 7 * B + 3],
                                   rng.integers(0, N, 24)]))
    ref = native.grad_spec_points(A, ot.templates(w5.zmax, w5.dz, M), w, ks)
    got = gs[torch.from_numpy(ks).cuda()].cpu().numpy()
    # relative to the largest gradient component over the sample and a
    # bulk estimate of the full gradient's scale
    scale = max(np.max(np.abs(ref)), float(gs.abs().max()))
    assert np.max(np.abs(got - ref)) / scale < TOL


def test_workload5_geometry_full_gradients_short_spectrum(fd):
    K, M, L = 201, 512, 8192
    A = syn.random_spectrum(505, 40000)
    A = A + syn.chirp_spectrum(40000, [(7.0, 0.4, 20000.25, -150.0)]).astype(np.complex64)
    taps_h = fd.fdas_make_templates_host(200.0, 2.0, M)
    tt = torch.from_numpy(taps_h).cuda()
    bank = fd.prepare_bank(tt, L)
    w = np.random.default_rng(57).random((K, len(A)), dtype=np.float32)
    N = len(A)
    gs = torch.empty(N, dtype=torch.complex64, device="cuda")
    gt = torch.empty((K, M), dtype=torch.complex64, device="cuda")
    ws = torch.empty(fd.fdas_backward_workspace_bytes(N, K, M, L, 0), dtype=torch.uint8,
                     device="cuda")
    fd.fdas_correlate_backward(torch.from_numpy(A).cuda(), N, bank, K, M, L,
                               torch.from_numpy(w).cuda(), gs, gt, ws)
    torch.cuda.synchronize()
    # the oracle's own closed-form templates on the reference side
    rA, rT = native.grads(A, ot.templates(200.0, 2.0, M), w)
    assert _rel(gs.cpu().numpy(), rA) < TOL
    assert _rel(gt.cpu().numpy(), rT) < TOL
