"""GPU parity of harmonic summing and peak candidates (Sec. 3: harmonic
summing, threshold and peak search) against the oracle.

The sums are FP32 in the order h = 1..H on both sides, so they must agree
bit for bit, chained on the previous fold or built from scratch, and the
candidate sets must be identical -- on random planes up to the headline
plane's size (85 x 2^21).  End to end, a pulsed accelerated signal in a
time series goes through the real-to-complex front end, the correlation and
the harmonic sums on the GPU and through the FP64 oracle's pipeline; the
sums agree to 1e-5 of their peak and both find the signal's fundamental.
"""
import numpy as np
import pytest

import fdas_synth as syn
from oracle import harmonic as oh
from oracle import native, r2c
from oracle import templates as ot

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu

FOLDS = (1, 2, 4, 8, 16, 32)


@pytest.fixture(scope="module")
def fd():
    import paper_1804_05335_amd as f
    f.lib()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return f


def _from_scratch(fd, Pd, H):
    K, N = Pd.shape
    KH, NH = fd.fdas_harmonic_shape(N, K, H)
    out = torch.full((KH, NH), float("nan"), dtype=torch.float32, device="cuda")
    fd.fdas_harmonic_sum(Pd, N, K, H, None, out)
    return out


def _candidate_set(fd, S, N, K, H, thr):
    r, row, power, n = fd.candidates(S, N, K, H, thr, capacity=1 << 20)
    assert n == len(r)
    c = (K - 1) // 2
    row0 = c - (S.shape[0] - 1) // 2
    return sorted(zip((row - row0).tolist(), r.tolist())), power


@pytest.mark.parametrize("K,N", [(85, 65539), (201, 40000), (3, 5), (1, 1000)])
def test_sums_bitwise_chained_and_from_scratch(fd, K, N):
    P = syn.random_plane(11, K, N)
    Pd = torch.from_numpy(P).cuda()
    folds = fd.harmonic_sums(Pd, 32)
    torch.cuda.synchronize()
    for H, S in zip(FOLDS, folds):
        ref = oh.harmonic_sum(P, H)
        assert np.array_equal(S.cpu().numpy(), ref), H
        assert np.array_equal(_from_scratch(fd, Pd, H).cpu().numpy(), ref), H


@pytest.mark.parametrize("H", [1, 2, 4, 8, 16])
def test_candidates_equal_the_oracle_set(fd, H):
    K, N = 85, 65539
    P = syn.random_plane(12, K, N)
    S = oh.harmonic_sum(P, H)
    thr = float(np.quantile(S, 0.995))
    ref = sorted(map(tuple, oh.peaks(S, thr).tolist()))
    got, power = _candidate_set(fd, torch.from_numpy(S).cuda(), N, K, H, thr)
    assert len(ref) > 0 and got == ref
    assert np.all(power > thr)


def test_headline_plane_size(fd):
    # 85 x 2^21, the plane of the headline correlation workload
    K, N = 85, 1 << 21
    P = syn.random_plane(13, K, N)
    Pd = torch.from_numpy(P).cuda()
    folds = fd.harmonic_sums(Pd, 32)
    torch.cuda.synchronize()
    for H, S in zip(FOLDS[1:], folds[1:]):
        ref = oh.harmonic_sum(P, H)
        assert np.array_equal(S.cpu().numpy(), ref), H
        if H == 8:
            thr = float(np.quantile(ref, 0.9999))
            want = sorted(map(tuple, oh.peaks(ref, thr).tolist()))
            got, _ = _candidate_set(fd, S, N, K, H, thr)
            assert len(want) > 0 and got == want


def test_pulsar_through_the_whole_path(fd):
    # n = 2^17 samples, a pulsed signal with 8 equal harmonics at r0 =
    # 2000.02 (harmonic h within 0.16 bin of h * 2000), z0 = 4 (harmonic 8 at
    # z = 32 <= zmax = 40); 41 templates x 64 taps
    n, r0, z0 = 1 << 17, 2000.02, 4.0
    zmax, dz, M, L = 40.0, 2.0, 64, 512
    x = syn.pulsed_series(3, n, r0, z0, 8, 0.02)
    scale = 1.0 / np.sqrt(n)
    N = n // 2
    spec = fd.spectrum_from_series(torch.from_numpy(x).cuda(), scale)[:N].contiguous()
    taps, bank = fd.make_bank(zmax, dz, M, L)
    K = taps.shape[0]
    plane = fd.correlate(spec, bank, K, M, L)
    folds = fd.harmonic_sums(plane, 8)
    torch.cuda.synchronize()
    A = r2c.spectrum(x.astype(np.float64), scale)[:N]
    Pref = native.power(A, ot.templates(zmax, dz, M))
    c = (K - 1) // 2
    for H, S in zip((1, 2, 4, 8), folds):
        ref = oh.harmonic_sum_f64(Pref, H)
        got = S.cpu().numpy()
        assert np.max(np.abs(got - ref)) < 1e-5 * np.max(ref), H
    S8 = folds[3].cpu().numpy()
    kk, rr = np.unravel_index(np.argmax(S8), S8.shape)
    row = c - c // 8 + kk
    assert (row - c) * dz == z0 and rr == int(round(r0))
    ref8 = oh.harmonic_sum_f64(Pref, 8)
    assert np.unravel_index(np.argmax(ref8), ref8.shape) == (kk, rr)
    # the 8-fold sum gathers several times the fundamental's own power
    assert S8[kk, rr] > 4.0 * plane[row, rr].item()
    r, rows, power, cnt = fd.candidates(folds[3], N, K, 8, 0.5 * float(S8[kk, rr]))
    assert cnt >= 1 and np.any((rows == row) & (r == rr))


def test_search_path_finds_the_pulsar(fd):
    # the same pulsed signal through the library's one-call search path
    n, r0, z0 = 1 << 17, 2000.02, 4.0
    x = torch.from_numpy(syn.pulsed_series(3, n, r0, z0, 8, 0.02)).cuda()
    res = fd.search(x, 40.0, 2.0, 64, 512, 8, {1: 15.0, 8: 60.0})
    r, row, power, cnt = res[8]
    K = 41
    c = (K - 1) // 2
    assert cnt >= 1 and np.any((row == c + int(z0 / 2.0)) & (r == int(round(r0))))
    best = np.argmax(power)
    assert (row[best] - c) * 2.0 == z0 and r[best] == int(round(r0))
    assert set(res) == {1, 8}


def test_graph_capture_and_replay(fd):
    # folds 2..8 and the candidates of fold 8 captured once, replayed on new
    # planes written in place; every replay equals the eager calls
    K, N = 41, 50000
    planes = [syn.random_plane(s, K, N) for s in (21, 22, 23)]
    Pd = torch.from_numpy(planes[0]).cuda()
    shapes = [fd.fdas_harmonic_shape(N, K, H) for H in (2, 4, 8)]
    outs = [torch.empty(s, dtype=torch.float32, device="cuda") for s in shapes]
    cap = 4096
    cbuf = torch.empty(cap * 16, dtype=torch.uint8, device="cuda")
    count = torch.zeros(1, dtype=torch.int32, device="cuda")
    thr = 12.0

    def run():
        fd.fdas_harmonic_sum(Pd, N, K, 2, None, outs[0])
        fd.fdas_harmonic_sum(Pd, N, K, 4, outs[0], outs[1])
        fd.fdas_harmonic_sum(Pd, N, K, 8, outs[1], outs[2])
        fd.fdas_find_candidates(outs[2], N, K, 8, thr, cbuf, cap, count)

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        run()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run()
    for P in planes[1:] + planes[:1]:
        Pd.copy_(torch.from_numpy(P))
        for o in outs:
            o.fill_(float("nan"))
        count.fill_(-1)
        g.replay()
        torch.cuda.synchronize()
        got = [o.cpu().numpy() for o in outs]
        n_graph = int(count.item())
        run()                                   # eager, same buffers
        torch.cuda.synchronize()
        for a, o in zip(got, outs):
            assert np.array_equal(a, o.cpu().numpy())
        assert n_graph == int(count.item()) and n_graph > 0
        ref = oh.harmonic_sum(P, 8)
        assert np.array_equal(got[2], ref)
        assert n_graph == len(oh.peaks(ref, thr))


def test_harmonic_sums_of_the_interbinned_plane(fd):
    # columns of the interbinned plane are half bins, so the harmonics of a
    # half-bin fundamental land on the grid: a pulsed signal at r0 = 2000.5
    # is found at half-bin 4001 with ~3x the 8-fold power of the plain plane
    from oracle import direct
    n, r0, z0 = 1 << 17, 2000.5, 4.0
    zmax, dz, M, L = 40.0, 2.0, 64, 512
    x = syn.pulsed_series(4, n, r0, z0, 8, 0.02)
    scale = 1.0 / np.sqrt(n)
    N = n // 2
    spec = fd.spectrum_from_series(torch.from_numpy(x).cuda(), scale)[:N].contiguous()
    taps, bank = fd.make_bank(zmax, dz, M, L)
    K = taps.shape[0]
    c = (K - 1) // 2
    plane2 = fd.correlate_interbin(spec, bank, K, M, L)
    plane = fd.correlate(spec, bank, K, M, L)
    S2 = fd.harmonic_sums(plane2, 8)[3].cpu().numpy()
    S1 = fd.harmonic_sums(plane, 8)[3].cpu().numpy()
    A = r2c.spectrum(x.astype(np.float64), scale)[:N]
    ref = oh.harmonic_sum_f64(direct.interbinned_power(A, ot.templates(zmax, dz, M)), 8)
    assert np.max(np.abs(S2 - ref)) < 1e-5 * np.max(ref)
    kk, cc = np.unravel_index(np.argmax(S2), S2.shape)
    assert ((c - c // 8 + kk) - c) * dz == z0 and cc == int(2 * r0)
    assert S2.max() > 2.0 * S1.max()


def _packed_planes(K, lens, seed):
    planes = [syn.random_plane(seed + b, K, n) for b, n in enumerate(lens)]
    flat = np.concatenate([p.reshape(-1) for p in planes] + [np.zeros(0, np.float32)])
    offs = np.concatenate([[0], np.cumsum(lens)]).astype(np.int64)
    return planes, flat.astype(np.float32), offs


def test_batched_folds_bitwise_per_spectrum(fd):
    # ragged batch with an empty and a one-bin spectrum; all folds in one
    # launch each, bitwise equal to the oracle and to single-spectrum calls
    K = 85
    lens = [70001, 0, 1, 4096, 33333, 65536, 5, 12000]
    planes, flat, offs = _packed_planes(K, lens, 40)
    Pd = torch.from_numpy(flat).cuda()
    od = torch.from_numpy(offs).cuda()
    folds = fd.harmonic_sums_batched(Pd, od, K, 32)
    torch.cuda.synchronize()
    for H, S in zip(FOLDS[1:], folds[1:]):
        KH, _ = fd.fdas_harmonic_shape(0, K, H)
        pre = fd.fold_prefix(offs, H)
        host = S.cpu().numpy()
        for b, n in enumerate(lens):
            got = host[KH * pre[b]:KH * pre[b + 1]].reshape(KH, -1)
            assert np.array_equal(got, oh.harmonic_sum(planes[b], H)), (H, b)
            if n > 0:
                single = _from_scratch(fd, torch.from_numpy(planes[b]).cuda(), H)
                assert np.array_equal(got, single.cpu().numpy()), (H, b)


def test_batched_candidates_equal_the_oracle_sets(fd):
    K = 41
    lens = [20000, 7, 0, 9999, 30001]
    planes, flat, offs = _packed_planes(K, lens, 50)
    Pd = torch.from_numpy(flat).cuda()
    od = torch.from_numpy(offs).cuda()
    folds = fd.harmonic_sums_batched(Pd, od, K, 8)
    c = (K - 1) // 2
    for H, S in zip((2, 4, 8), folds[1:]):
        KH, _ = fd.fdas_harmonic_shape(0, K, H)
        ref_folds = [oh.harmonic_sum(p, H) for p in planes]
        allv = np.concatenate([f.reshape(-1) for f in ref_folds])
        thr = float(np.quantile(allv, 0.999))
        want = []
        for b, f in enumerate(ref_folds):
            for k, r in oh.peaks(f, thr):
                want.append((b, int(r), int(c - (KH - 1) // 2 + k)))
        spec, r, row, power, n = fd.candidates_batched(S, od, K, H, thr, capacity=1 << 18)
        assert n == len(want) > 0
        assert sorted(zip(spec.tolist(), r.tolist(), row.tolist())) == sorted(want)
        assert np.all(power > thr)


def test_batched_graph_replay(fd):
    K = 41
    lens = [30000, 0, 1234, 9000]
    planes, flat, offs = _packed_planes(K, lens, 60)
    Pd = torch.from_numpy(flat).cuda()
    od = torch.from_numpy(offs).cuda()
    nspec = len(lens)
    ws = torch.empty(fd.fdas_harmonic_batched_workspace_bytes(nspec), dtype=torch.uint8,
                     device="cuda")
    outs = []
    for H in (2, 4, 8):
        KH, _ = fd.fdas_harmonic_shape(0, K, H)
        outs.append(torch.empty(KH * int(fd.fold_prefix(offs, H)[-1]), dtype=torch.float32,
                                device="cuda"))
    cap = 1 << 14
    cbuf = torch.empty(cap * 16, dtype=torch.uint8, device="cuda")
    count = torch.zeros(1, dtype=torch.int32, device="cuda")

    def run():
        fd.fdas_harmonic_sum_batched(Pd, od, nspec, K, 2, None, outs[0], ws)
        fd.fdas_harmonic_sum_batched(Pd, od, nspec, K, 4, outs[0], outs[1], ws)
        fd.fdas_harmonic_sum_batched(Pd, od, nspec, K, 8, outs[1], outs[2], ws)
        fd.fdas_find_candidates_batched(outs[2], od, nspec, K, 8, 12.0, cbuf, cap, count, ws)

    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):
        run()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        run()
    for seed in (61, 62, 60):
        new_planes, new_flat, _ = _packed_planes(K, lens, seed)
        Pd.copy_(torch.from_numpy(new_flat))
        for o in outs:
            o.fill_(float("nan"))
        count.fill_(-1)
        g.replay()
        torch.cuda.synchronize()
        got = [o.cpu().numpy() for o in outs]
        n_graph = int(count.item())
        run()
        torch.cuda.synchronize()
        for a, o in zip(got, outs):
            assert np.array_equal(a, o.cpu().numpy())
        assert n_graph == int(count.item())
        KH, _ = fd.fdas_harmonic_shape(0, K, 8)
        pre = fd.fold_prefix(offs, 8)
        n_ref = 0
        for b in range(nspec):
            ref = oh.harmonic_sum(new_planes[b], 8)
            assert np.array_equal(got[2][KH * pre[b]:KH * pre[b + 1]].reshape(KH, -1), ref)
            n_ref += len(oh.peaks(ref, 12.0))
        assert n_graph == n_ref


def test_batched_folds_of_correlated_planes(fd):
    # 32 spectra of the ragged correlation workload, planes from
    # correlate_batched; the batched folds equal the per-spectrum folds of
    # the same planes (the planes themselves are checked against the oracle
    # in the batched correlation tests)
    w = syn.workload(3, nspec=32)
    taps, bank = fd.make_bank(w.zmax, w.dz, w.M, 2048)
    K = taps.shape[0]
    specs, od = fd.pack([torch.from_numpy(s) for s in w.spectra])
    planes = fd.correlate_batched(specs, od, bank, K, w.M, 2048)
    folds = fd.harmonic_sums_batched(planes, od, K, 8)
    torch.cuda.synchronize()
    offs = od.cpu().numpy()
    for H, S in zip((2, 4, 8), folds[1:]):
        KH, _ = fd.fdas_harmonic_shape(0, K, H)
        pre = fd.fold_prefix(offs, H)
        for b in (0, 7, 31):
            n = int(offs[b + 1] - offs[b])
            single = _from_scratch(fd, planes[K * offs[b]:K * offs[b + 1]].view(K, n), H)
            assert torch.equal(S[KH * pre[b]:KH * pre[b + 1]].view(KH, -1), single), (H, b)


def test_search_batched_equals_per_series_path(fd):
    """Four series, each with a pulsar at its own (r0, z0), searched in one
    batched call: the candidate sets of every fold equal those of the
    single-series kernels on the same n/2 + 1-bin spectra, and each series'
    strongest 8-fold peak is its pulsar."""
    n = 1 << 17
    zmax, dz, M, L = 40.0, 2.0, 64, 512
    pulsars = [(2000.02, 4.0), (3100.02, -2.0), (1500.02, 2.0), (2600.02, 0.0)]
    xs = np.stack([syn.pulsed_series(10 + b, n, r0, z0, 8, 0.02)
                   for b, (r0, z0) in enumerate(pulsars)])
    xd = torch.from_numpy(xs).cuda()
    thr = {1: 15.0, 2: 25.0, 8: 60.0}
    res = fd.search_batched(xd, zmax, dz, M, L, 8, thr)
    assert set(res) == set(thr)
    taps, bank = fd.make_bank(zmax, dz, M, L)
    K = taps.shape[0]
    c = (K - 1) // 2
    nb = n // 2 + 1
    for b, (r0, z0) in enumerate(pulsars):
        spec = fd.spectrum_from_series(xd[b].contiguous(), 1.0 / np.sqrt(n))
        plane = fd.correlate(spec, bank, K, M, L)
        folds = fd.harmonic_sums(plane, 8)
        for H, S in zip((1, 2, 4, 8), folds):
            if H not in thr:
                continue
            r1, row1, p1, n1 = fd.candidates(S, nb, K, H, thr[H])
            sb, rb, rowb, pb, _ = res[H]
            sel = sb == b
            assert np.array_equal(rb[sel], r1) and np.array_equal(rowb[sel], row1), (b, H)
            assert np.array_equal(pb[sel], p1), (b, H)
        sel = res[8][0] == b
        best = np.argmax(res[8][3][sel])
        assert (res[8][2][sel][best] - c) * dz == z0 and res[8][1][sel][best] == int(round(r0))
