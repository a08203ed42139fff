"""GPU parity of the real-to-complex front end (Sec. 4.1) against the FP64
oracle: every pass plan from 2^13 to 2^26 samples, sampled literal-DFT bins
at the paper's largest size (2^24 samples, Sec. 6), a replayed graph
capture, and the end-to-end path time series -> spectrum -> f-fdot plane
checked on sampled points against the oracle's own pipeline."""
import numpy as np
import pytest

import fdas_synth as syn
from oracle import native, r2c
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


def _run(fd, x, scale):
    xd = torch.from_numpy(x).cuda()
    spec = fd.spectrum_from_series(xd, scale)
    torch.cuda.synchronize()
    return spec.cpu().numpy().astype(np.complex128)


@pytest.mark.parametrize("log2n", list(range(13, 27)))
def test_r2c_vs_oracle(fd, log2n):
    n = 1 << log2n
    x = syn.time_series(100 + log2n, n, [(0.2, 1.0, n / 5 + 0.37, -17.0)])
    scale = 1.0 / np.sqrt(n)
    got = _run(fd, x, scale)
    ref = r2c.spectrum(x, scale)
    assert got.shape == ref.shape
    assert np.max(np.abs(got - ref)) < TOL * np.max(np.abs(ref))
    assert np.linalg.norm(got - ref) < 1e-6 * np.linalg.norm(ref)


def test_r2c_largest_paper_size_literal_bins(fd):
    n = 1 << 24
    r0 = 3_000_000.25
    x = syn.time_series(24, n, [(0.05, 0.0, r0, 40.0)])
    got = _run(fd, x, 1.0)
    ks = np.unique(np.concatenate([[0, 1, 2, n // 4, n // 2 - 1, n // 2],
                                   np.arange(int(r0) - 30, int(r0) + 31, 10),
                                   np.random.default_rng(5).integers(0, n // 2 + 1, 10)]))
    ref = r2c.dft_points(x, ks)
    full = r2c.spectrum(x)
    assert np.max(np.abs(got[ks] - ref)) < TOL * np.max(np.abs(full))
    assert np.max(np.abs(got - full)) < TOL * np.max(np.abs(full))


def test_r2c_graph_replay(fd):
    n = 1 << 20
    xs = [syn.time_series(s, n) for s in (1, 2, 3)]
    xd = torch.from_numpy(xs[0]).cuda()
    spec = torch.empty(n // 2 + 1, dtype=torch.complex64, device="cuda")
    ws = torch.empty(fd.fdas_r2c_workspace_bytes(n), dtype=torch.uint8, device="cuda")
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        fd.fdas_r2c(xd, n, 1.0, spec, ws)
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        fd.fdas_r2c(xd, n, 1.0, spec, ws)
    for x in xs[1:] + xs[:1]:
        xd.copy_(torch.from_numpy(x))
        spec.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        got = spec.clone()
        eager = fd.spectrum_from_series(xd, 1.0)
        torch.cuda.synchronize()
        assert torch.equal(got, eager)
        _ = torch.randn(1000, device="cuda").sum()


def test_series_to_plane_end_to_end(fd):
    # a real accelerated sinusoid in unit-variance noise: r2c with scale
    # 1/sqrt(n) gives bins of unit mean noise power, then the correlation
    n = 1 << 22
    r0, z0 = 1_234_567.3, 24.0
    x = syn.time_series(7, n, [(0.02, 0.5, r0, z0)])
    xd = torch.from_numpy(x).cuda()
    spec = fd.spectrum_from_series(xd, 1.0 / np.sqrt(n))
    N = n // 2
    zmax, dz, M, L = 40.0, 2.0, 128, 2048
    taps, bank = fd.make_bank(zmax, dz, M, L)
    K = taps.shape[0]
    plane = fd.correlate(spec[:N], bank, K, M, L)
    torch.cuda.synchronize()
    # the oracle's own pipeline on sampled points around the signal and elsewhere
    A = r2c.spectrum(x, 1.0 / np.sqrt(n))[:N]
    T = ot.templates(zmax, dz, M)
    cols = np.concatenate([np.arange(int(r0) - 40, int(r0) + 41),
                           np.random.default_rng(1).integers(0, N, 500), [0, 1, N - 2, N - 1]])
    zi = np.repeat(np.arange(K), len(cols)).astype(np.int32)
    ri = np.tile(cols, K).astype(np.int64)
    got = plane[torch.from_numpy(zi.astype(np.int64)).cuda(),
                torch.from_numpy(ri).cuda()].cpu().numpy()
    ref = native.power_points(A, T, zi, ri)
    assert np.max(np.abs(got - ref)) < TOL * np.max(ref)
    # the signal is found at its frequency and frequency derivative
    zz, rr = np.unravel_index(int(torch.argmax(plane).item()), plane.shape)
    assert abs(ot.z_grid(zmax, dz)[zz] - z0) <= dz and abs(rr - r0) <= 1.0


@pytest.mark.parametrize("log2n,nseries", [(13, 5), (16, 64), (22, 3), (24, 2)])
def test_r2c_batched_bitwise_equals_single(fd, log2n, nseries):
    """Equal-length series in one launch per pass: every series' bins are
    bitwise those of the single-series call (the separate split at 2^13, the
    fused last pass above it), and nothing is written past the batch."""
    n = 1 << log2n
    xs = np.stack([syn.time_series(1000 * log2n + b, n, [(0.3, 0.7 * b, n / 9 + 0.3 * b, 2.0 * b)])
                   for b in range(nseries)])
    xd = torch.from_numpy(xs).cuda()
    guard = 64
    buf = torch.full((nseries * (n // 2 + 1) + guard,), complex(-3.0, 5.0), dtype=torch.complex64,
                     device="cuda")
    spec = buf[:nseries * (n // 2 + 1)]
    ws = torch.empty(fd.fdas_r2c_batched_workspace_bytes(n, nseries), dtype=torch.uint8,
                     device="cuda")
    scale = 1.0 / np.sqrt(n)
    fd.fdas_r2c_batched(xd.view(-1), n, nseries, scale, spec, ws)
    torch.cuda.synchronize()
    assert torch.all(buf[-guard:] == complex(-3.0, 5.0))
    got = spec.view(nseries, n // 2 + 1)
    for b in range(nseries):
        one = fd.spectrum_from_series(xd[b].contiguous(), scale)
        torch.cuda.synchronize()
        assert torch.equal(got[b], one), b
    # one series against the oracle as well
    ref = r2c.spectrum(xs[-1], scale)
    assert np.max(np.abs(got[-1].cpu().numpy() - ref)) < TOL * np.max(np.abs(ref))


def test_batched_series_to_planes(fd):
    """Many equal-length series -> spectra (one launch per pass) -> planes of
    all of them (one launch), the spectra packed with offsets b (n/2 + 1):
    each plane bitwise the single-series path's."""
    n, nseries = 1 << 16, 6
    xs = np.stack([syn.time_series(50 + b, n, [(0.2, 0.0, 7000.4 + 300 * b, 4.0 * b - 10)])
                   for b in range(nseries)])
    xd = torch.from_numpy(xs).cuda()
    scale = 1.0 / np.sqrt(n)
    specs = fd.spectra_from_series(xd, scale)
    nb = n // 2 + 1
    offs = torch.arange(nseries + 1, dtype=torch.int64, device="cuda") * nb
    zmax, dz, M, L = 20.0, 2.0, 64, 512
    taps, bank = fd.make_bank(zmax, dz, M, L)
    K = taps.shape[0]
    planes = fd.correlate_batched(specs.view(-1), offs, bank, K, M, L)
    torch.cuda.synchronize()
    for b in range(nseries):
        one = fd.correlate(fd.spectrum_from_series(xd[b].contiguous(), scale), bank, K, M, L)
        torch.cuda.synchronize()
        assert torch.equal(planes[K * nb * b:K * nb * (b + 1)].view(K, nb), one), b
