"""GPU parity of the symmetric bank (rows z >= 0 only; row -z read as the
conjugate mirror of row z, Sec. 4.2 +/-z symmetry): full planes at the
2^16-bin workload for every segment length, sampled points at the 2^21-bin /
85-template workload and at the 201-template, 512-tap, segment-8192 geometry,
and the +/-z identity P_{-z}(A) = P_z(conj A) on the GPU's own planes."""
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


def _rel(got, ref):
    return float(np.max(np.abs(got.astype(np.float64) - ref)) / np.max(ref))


@pytest.mark.parametrize("L", [256, 512, 1024, 2048, 4096, 8192])
def test_symmetric_bank_workload1(fd, L):
    w = syn.workload(1)
    taps, bank = fd.make_bank(w.zmax, w.dz, w.M, L)
    K = taps.shape[0]
    sym = fd.prepare_bank_sym(taps, L)
    spec = torch.from_numpy(w.spectra[0]).cuda()
    P = fd.correlate_sym(spec, sym, K, w.M, L).cpu().numpy()
    ref = native.power(w.spectra[0], ot.templates(w.zmax, w.dz, w.M))
    assert _rel(P, ref) < TOL
    full = fd.correlate(spec, bank, K, w.M, L).cpu().numpy()
    assert _rel(P, full.astype(np.float64)) < TOL
    # +/-z: the plane of conj(A) is the z-reversed plane of A
    Pc = fd.correlate_sym(torch.conj(spec).resolve_conj().contiguous(), sym, K, w.M, L)
    assert _rel(Pc.cpu().numpy()[::-1], P.astype(np.float64)) < TOL


def _sampled(fd, A, zmax, dz, M, L, seed, nrand):
    taps = torch.from_numpy(fd.fdas_make_templates_host(zmax, dz, M)).cuda()
    K = taps.shape[0]
    sym = fd.prepare_bank_sym(taps, L)
    N = len(A)
    P = fd.correlate_sym(torch.from_numpy(A).cuda(), sym, K, M, L)
    B = L - M
    rng = np.random.default_rng(seed)
    cols = np.unique(np.concatenate([np.arange(0, 16), np.arange(N - 16, N),
                                     ((np.arange(1, -(-N // B)) * B)[:, None]
                                      + np.arange(-2, 3)[None, :]).ravel()]))
    cols = cols[(cols >= 0) & (cols < N)]
    zi = np.concatenate([np.repeat(np.arange(K), len(cols)), rng.integers(0, K, nrand)]).astype(np.int32)
    ri = np.concatenate([np.tile(cols, K), rng.integers(0, N, nrand)]).astype(np.int64)
    got = P[torch.from_numpy(zi.astype(np.int64)).cuda(), torch.from_numpy(ri).cuda()].cpu().numpy()
    ref = native.power_points(A, ot.templates(zmax, dz, M), zi, ri)
    assert _rel(got, ref) < TOL


def test_symmetric_bank_workload2_sampled(fd):
    w = syn.workload(2)
    _sampled(fd, w.spectra[0], w.zmax, w.dz, w.M, 2048, 2, 100000)


def test_symmetric_bank_large_zmax_segment_8192(fd):
    w = syn.workload(5, nspec=1)
    _sampled(fd, w.spectra[0], w.zmax, w.dz, w.M, 8192, 5, 40000)


@pytest.mark.parametrize("L", [512, 2048])
def test_symmetric_bank_grid_invariance(fd, L):
    """Persistent grids of other sizes split the (segment, template) items
    elsewhere: workgroup ranges start, end and cross the first stored row
    (z = 0) at other templates, and the plane is the same bit for bit."""
    w = syn.workload(1)
    taps, _ = fd.make_bank(w.zmax, w.dz, w.M, L)
    K = taps.shape[0]
    sym = fd.prepare_bank_sym(taps, L)
    spec = torch.from_numpy(w.spectra[0]).cuda()
    ref = fd.correlate_sym(spec, sym, K, w.M, L).cpu()
    for grid in (1, 3, 7, 64, 1000):
        got = fd.correlate_sym(spec, sym, K, w.M, L, grid=grid).cpu()
        assert torch.equal(got, ref), grid

