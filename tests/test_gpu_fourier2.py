"""GPU parity of the two-bin Fourier interpolation (Sec. 3: the half-bin
matched filter, templates and signal at doubled resolution) against the FP64
oracle: full planes at the 2^16-bin workload for every segment length,
sampled integer and half-bin columns at the 2^21-bin / 85-template workload,
and agreement of the integer columns with the plain plane."""
import numpy as np
import pytest

import fdas_synth as syn
from oracle import direct, native
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


def _rel(got, ref):
    return float(np.max(np.abs(got.astype(np.float64) - ref)) / np.max(ref))


@pytest.mark.parametrize("L", [256, 512, 1024, 2048, 4096, 8192])
def test_fourier2_full_plane_workload1(fd, L):
    w = syn.workload(1)
    taps, bank = fd.make_bank(w.zmax, w.dz, w.M, L)
    _, bank_h = fd.make_bank_half(w.zmax, w.dz, w.M, L)
    K = taps.shape[0]
    spec = torch.from_numpy(w.spectra[0]).cuda()
    P2 = fd.correlate_fourier2(spec, bank, bank_h, K, w.M, L).cpu().numpy()
    ref = direct.fourier_interpolated_power(w.spectra[0], w.zmax, w.dz, w.M)
    assert _rel(P2, ref) < TOL
    # the integer columns come from the (M + 2)-tap segment tiling shared
    # with the half-bin bank: the plain plane up to FP32 rounding
    plain = fd.correlate(spec, bank, K, w.M, L).cpu().numpy()
    assert _rel(P2[:, 0::2], plain.astype(np.float64)) < TOL


def test_fourier2_workload2_sampled(fd):
    w = syn.workload(2)
    K, M, L = w.K, w.M, 2048
    N = len(w.spectra[0])
    _, bank = fd.make_bank(w.zmax, w.dz, M, L)
    _, bank_h = fd.make_bank_half(w.zmax, w.dz, M, L)
    P2 = fd.correlate_fourier2(torch.from_numpy(w.spectra[0]).cuda(), bank, bank_h, K, M, L)
    rng = np.random.default_rng(4)
    Bh = L - (M + 2)
    cols = [(np.arange(1, -(-N // Bh)) * Bh)[:, None] + np.arange(-3, 3)[None, :]]
    for _, _, r, _ in w.signals[0]:
        cols.append(int(r) + np.arange(-6, 7))
    cols.append(np.array([0, 1, 2, N - 3, N - 2, N - 1]))
    cols = np.unique(np.clip(np.concatenate([c.ravel() for c in cols]), 0, N - 1))
    zi = np.concatenate([np.repeat(np.arange(K), len(cols)), rng.integers(0, K, 60000)])
    ri = np.concatenate([np.tile(cols, K), rng.integers(0, N, 60000)]).astype(np.int64)
    half = P2[torch.from_numpy(zi).cuda(), torch.from_numpy(2 * ri + 1).cuda()].cpu().numpy()
    ref_h = direct.fourier_half_points(w.spectra[0], w.zmax, w.dz, M, zi, ri)
    whole = P2[torch.from_numpy(zi).cuda(), torch.from_numpy(2 * ri).cuda()].cpu().numpy()
    ref_w = native.power_points(w.spectra[0], ot.templates(w.zmax, w.dz, M), zi.astype(np.int32), ri)
    scale = max(np.max(ref_h), np.max(ref_w))
    assert np.max(np.abs(half - ref_h)) < TOL * scale
    assert np.max(np.abs(whole - ref_w)) < TOL * scale
