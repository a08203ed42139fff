"""GPU parity of the interbinned plane (Sec. 3, eq. f-interp) against the
FP64 oracle: full planes at the 2^16-bin workload for every segment length,
sampled columns (bin and half-bin) at the 2^21-bin / 85-template workload,
and bitwise agreement of the even columns with the plain plane."""
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


@pytest.fixture(scope="module")
def w1():
    return syn.workload(1)


@pytest.mark.parametrize("L", [256, 512, 1024, 2048, 4096, 8192])
def test_interbin_full_plane_workload1(fd, w1, L):
    _, bank = fd.make_bank(w1.zmax, w1.dz, w1.M, L)
    spec = torch.from_numpy(w1.spectra[0]).cuda()
    P2 = fd.correlate_interbin(spec, bank, w1.K, w1.M, L).cpu().numpy()
    ref = direct.interbinned_power(w1.spectra[0], ot.templates(w1.zmax, w1.dz, w1.M))
    assert _rel(P2, ref) < TOL
    plain = fd.correlate(spec, bank, w1.K, w1.M, L).cpu().numpy()
    assert np.array_equal(P2[:, 0::2], plain)
    # the injected signal sits at r0 = 20000.3, z0 = +8: the peak is at z0
    # and the oracle's value there is its maximum (the half-bin 20000.5 is
    # nearer than bin 20000, so column 40001 wins)
    zz, cc = np.unravel_index(np.argmax(P2), P2.shape)
    assert ot.z_grid(w1.zmax, w1.dz)[zz] == 8.0 and cc in (40000, 40001)
    assert ref[zz, cc] >= ref.max() * (1 - 2 * TOL)


@pytest.mark.parametrize("N", [1, 2, 447, 448, 449, 5000])
def test_interbin_ragged_random_taps(fd, N):
    L, M, K = 512, 64, 4
    taps = syn.random_taps(N + 3, K, M)
    bank = fd.prepare_bank(torch.from_numpy(taps).cuda(), L)
    A = syn.random_spectrum(N + 4, N)
    P2 = fd.correlate_interbin(torch.from_numpy(A).cuda(), bank, K, M, L).cpu().numpy()
    assert _rel(P2, direct.interbinned_power(A, taps)) < TOL


def test_interbin_workload2_sampled(fd):
    w = syn.workload(2)
    K, M, L = w.K, w.M, 2048
    N = len(w.spectra[0])
    _, bank = fd.make_bank(w.zmax, w.dz, M, L)
    P2 = fd.correlate_interbin(torch.from_numpy(w.spectra[0]).cuda(), bank, K, M, L)
    rng = np.random.default_rng(22)
    B = L - M
    cols = [2 * (np.arange(1, -(-N // B)) * B)[:, None] + np.arange(-4, 4)[None, :]]
    for _, _, r, _ in w.signals[0]:
        cols.append(2 * int(r) + np.arange(-20, 21))
    cols.append(np.array([0, 1, 2, 3, 2 * N - 4, 2 * N - 3, 2 * N - 2, 2 * N - 1]))
    cols = np.unique(np.clip(np.concatenate([c.ravel() for c in cols]), 0, 2 * N - 1))
    zi = np.repeat(np.arange(K), len(cols)).astype(np.int32)
    ci = np.tile(cols, K).astype(np.int64)
    zr = rng.integers(0, K, 200000).astype(np.int32)
    cr = rng.integers(0, 2 * N, 200000)
    zi, ci = np.concatenate([zi, zr]), np.concatenate([ci, cr])
    got = P2[torch.from_numpy(zi.astype(np.int64)).cuda(), torch.from_numpy(ci).cuda()].cpu().numpy()
    ref = native.interbin_points(w.spectra[0], ot.templates(w.zmax, w.dz, M), zi, ci)
    assert _rel(got, ref) < TOL


# Lane 63's neighbour at the wave edges: a lane rotation in one-wave
# workgroups (L = 1024), LDS slots behind a barrier with 2, 4 and 8 waves;
# M/2 = 0, 1 and 2 lane slots without valid outputs at each end (the
# kernels drop those slots at compile time).  Three segments and a ragged
# tail; two persistent workgroups (many segments and templates each) and the
# resident grid.
@pytest.mark.parametrize("L,M", [(1024, 128), (1024, 256), (2048, 128), (2048, 512),
                                 (4096, 256), (4096, 512), (4096, 1024), (8192, 512)])
@pytest.mark.parametrize("grid", [2, 0])
def test_interbin_wave_edges_random_taps(fd, L, M, grid):
    K = 3
    N = 3 * (L - M) + 37
    taps = syn.random_taps(L + M, K, M)
    bank = fd.prepare_bank(torch.from_numpy(taps).cuda(), L)
    A = syn.random_spectrum(L + 3 * M, N)
    spec = torch.from_numpy(A).cuda()
    P2 = fd.correlate_interbin(spec, bank, K, M, L, grid=grid).cpu().numpy()
    assert _rel(P2, direct.interbinned_power(A, taps)) < TOL
    plain = fd.correlate(spec, bank, K, M, L).cpu().numpy()
    assert np.array_equal(P2[:, 0::2], plain)
