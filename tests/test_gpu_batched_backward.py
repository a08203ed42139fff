"""GPU checks of the batched adjoint (fdas_correlate_backward_batched) and of
the batched forward's second lane geometry.

- every spectrum's gradient bitwise equal to the single-spectrum adjoint with
  the same template chunking, the taps gradient equal to the batch sum of
  the oracle's, on a ragged batch with empty and one-bin members;
- a captured graph replayed on new batches written in place equals the
  eager call;
- the large-zmax workload (64 ragged spectra of 2^21..2^22 bins, 201 x 512
  taps) at full size, spectra gradient in one call, sampled bins against the
  oracle's per-bin gradient with the oracle's own templates;
- the batched forward at 8 and 16 values per lane against the oracle.
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


def _rel(got, ref):
    return float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))


def _batch(lens, seed):
    specs = [syn.random_spectrum(seed + i, n) for i, n in enumerate(lens)]
    o = np.zeros(len(lens) + 1, dtype=np.int64)
    o[1:] = np.cumsum(lens)
    packed = np.concatenate(specs).astype(np.complex64) if lens else np.zeros(0, np.complex64)
    return specs, packed, o


@pytest.mark.parametrize("L,M,zchunk", [(512, 128, 9), (2048, 256, 0), (1024, 64, 85)])
def test_backward_batched_bitwise_per_spectrum(fd, L, M, zchunk):
    zmax, dz = 84.0, 2.0
    K = fd.fdas_num_templates(zmax, dz)
    taps_h = fd.fdas_make_templates_host(zmax, dz, M)
    taps = torch.from_numpy(taps_h).cuda()
    bank = fd.prepare_bank(taps, L)
    lens = [30000, 0, 1, 3 * (L - M) + 11, 777, 12345]
    specs, packed, o = _batch(lens, 300 + L)
    rng = np.random.default_rng(L + M)
    w = [rng.random((K, n), dtype=np.float32) for n in lens]
    wpk = np.concatenate([x.reshape(-1) for x in w])
    sd, od, wd = (torch.from_numpy(packed).cuda(), torch.from_numpy(o).cuda(),
                  torch.from_numpy(wpk).cuda())
    gA, gT = fd.correlate_backward_batched(sd, od, bank, K, M, L, wd, zchunk=zchunk)
    torch.cuda.synchronize()
    T = ot.templates(zmax, dz, M)
    sumT = np.zeros((K, M), dtype=np.complex128)
    zc = zchunk if zchunk else K
    for b, n in enumerate(lens):
        if n == 0:
            continue
        a1 = torch.empty(n, dtype=torch.complex64, device="cuda")
        t1 = torch.empty((K, M), dtype=torch.complex64, device="cuda")
        ws = torch.empty(fd.fdas_backward_workspace_bytes(n, K, M, L, zc), dtype=torch.uint8,
                         device="cuda")
        fd.fdas_correlate_backward_ex(sd[o[b]:o[b + 1]], n, bank, K, M, L,
                                      wd[K * o[b]:K * o[b + 1]], a1, t1, zc, ws)
        torch.cuda.synchronize()
        if zchunk:
            assert torch.equal(gA[o[b]:o[b + 1]], a1), b
        rA, rT = native.grads(specs[b], T, w[b])
        assert _rel(gA[o[b]:o[b + 1]].cpu().numpy(), rA) < TOL, b
        sumT += rT
    assert _rel(gT.cpu().numpy(), sumT) < TOL


def test_backward_batched_graph_replay(fd):
    L, M, zmax = 1024, 128, 20.0
    taps, bank = fd.make_bank(zmax, 2.0, M, L)
    K = taps.shape[0]
    cap = 200000
    specs = torch.zeros(cap, dtype=torch.complex64, device="cuda")
    offs = torch.zeros(7, dtype=torch.int64, device="cuda")
    wts = torch.zeros(K * cap, dtype=torch.float32, device="cuda")
    gA = torch.zeros(cap, dtype=torch.complex64, device="cuda")
    gT = torch.zeros((K, M), dtype=torch.complex64, device="cuda")
    ws = torch.zeros(fd.fdas_backward_batched_workspace_bytes(cap, 6, K, M, L, 0, 3),
                     dtype=torch.uint8, device="cuda")

    def fill(seed):
        rng = np.random.default_rng(seed)
        lens = rng.integers(0, 30000, 6)
        o = np.zeros(7, dtype=np.int64)
        o[1:] = np.cumsum(lens)
        specs[:o[-1]].copy_(torch.from_numpy(syn.random_spectrum(seed, int(o[-1]))))
        wts[:K * o[-1]].copy_(torch.from_numpy(rng.random(K * int(o[-1]), dtype=np.float32)))
        offs.copy_(torch.from_numpy(o))
        return o

    def call():
        fd.fdas_correlate_backward_batched(specs, offs, 6, bank, K, M, L, wts, gA, gT, ws)

    fill(1)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        call()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        call()
    for seed in (2, 3, 4):
        o = fill(seed)
        gA.fill_(float("nan"))
        gT.fill_(float("nan"))
        g.replay()
        torch.cuda.synchronize()
        ga, gt = gA.clone(), gT.clone()
        call()
        torch.cuda.synchronize()
        assert torch.equal(ga, gA) and torch.equal(gt, gT), seed
        # bins past the batch are zero
        assert bool((ga[o[-1]:] == 0).all())
        _ = torch.randn(1000, device="cuda").sum()


@pytest.fixture(scope="module")
def w5():
    return syn.workload(5)


@pytest.mark.parametrize("L", [8192, 2048])
def test_workload5_batched_spectra_gradient_sampled(fd, w5, L):
    # all 64 spectra in one call; w ~ U(0,1) drawn on the device (156 GB),
    # copied back for the spectra that are checked
    K, M = w5.K, w5.M
    _, bank = fd.make_bank(w5.zmax, w5.dz, M, L)
    packed, o = w5.packed()
    total = int(o[-1])
    specs = torch.from_numpy(packed).cuda()
    offs = torch.from_numpy(o).cuda()
    gen = torch.Generator(device="cuda")
    gen.manual_seed(505)
    wts = torch.rand(K * total, generator=gen, dtype=torch.float32, device="cuda")
    gA, gT = fd.correlate_backward_batched(specs, offs, bank, K, M, L, wts, want_taps=False)
    torch.cuda.synchronize()
    assert gT is None and gA.numel() == total
    T = ot.templates(w5.zmax, w5.dz, M)
    B = L - M
    rng = np.random.default_rng(L)
    for b in (0, int(np.argmax(w5.lengths))):
        n = len(w5.spectra[b])
        wb = wts[K * o[b]:K * o[b + 1]].view(K, n).cpu().numpy()
        ks = np.unique(np.concatenate([[0, 1, n - 1, n - 2, B - 1, B, B + 1, 5 * B - 1],
                                       rng.integers(0, n, 12)]))
        ref = native.grad_spec_points(w5.spectra[b], T, wb, ks)
        got = gA[o[b] + torch.from_numpy(ks).cuda()].cpu().numpy()
        scale = max(np.max(np.abs(ref)), float(gA[o[b]:o[b + 1]].abs().max()))
        assert np.max(np.abs(got - ref)) / scale < TOL, b
    assert bool(torch.isfinite(gA).all())
    del wts, gA, specs
    torch.cuda.empty_cache()


@pytest.mark.parametrize("L,M,E", [(8192, 512, 8), (8192, 512, 16), (2048, 256, 8),
                                   (1024, 128, 8), (4096, 256, 8)])
def test_batched_forward_values_per_lane_vs_oracle(fd, L, M, E):
    zmax = 40.0
    taps, bank = fd.make_bank(zmax, 2.0, M, L)
    K = taps.shape[0]
    lens = [3 * (L - M) + 17, 1, 0, L - M, 5000]
    specs, packed, o = _batch(lens, 800 + E)
    sd, od = torch.from_numpy(packed).cuda(), torch.from_numpy(o).cuda()
    planes = fd.correlate_batched(sd, od, bank, K, M, L, E=E)
    planes_default = fd.correlate_batched(sd, od, bank, K, M, L)
    torch.cuda.synchronize()
    T = ot.templates(zmax, 2.0, M)
    for b, n in enumerate(lens):
        if n == 0:
            continue
        got = planes[K * o[b]:K * o[b + 1]].view(K, n).cpu().numpy()
        ref = native.power(specs[b], T)
        assert _rel(got, ref) < TOL, b
        d = planes_default[K * o[b]:K * o[b + 1]].view(K, n).cpu().numpy()
        assert _rel(got, d) < TOL, b
