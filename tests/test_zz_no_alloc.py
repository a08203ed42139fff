"""GPU check of the allocation-free batched correlation (collected last).

fdas_correlate_batched_noalloc keeps the segment prefix in the library's
fixed device array instead of a caller workspace.  Called through the C ABI
twice in a row -- a larger batch, then a smaller one, so the second call
runs over the first call's leftovers in that array -- its planes must equal
(bitwise) those of fdas_correlate_batched with a workspace on the same
inputs, and every output must be written.  Sizes beyond the array's maximum
are rejected before anything is launched.  Captured in a graph, for the
callers it is for, it replays on new batches written in place.
"""
import numpy as np
import pytest

import fdas_synth as syn
from oracle import native
from oracle import templates as ot

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fd():
    import paper_1804_05335_amd as f
    f.lib()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return f


def _batch(seed, nspec, L, M):
    rng = np.random.default_rng(seed)
    lens = [int(x) for x in np.exp(rng.uniform(np.log(2.0 ** 12), np.log(2.0 ** 16), nspec))]
    # degenerate members: empty, one bin, exactly one segment
    lens[1] = 0
    lens[2] = 1
    lens[-1] = L - M
    return [syn.random_spectrum(seed * 1000 + b, n) for b, n in enumerate(lens)]


def _run_both(fd, spectra, bank, K, M, L):
    specs, offs = fd.pack([torch.from_numpy(s) for s in spectra])
    total = int(offs[-1].item())
    nspec = len(spectra)
    ref = torch.full((K * total,), float("nan"), dtype=torch.float32, device="cuda")
    ws = torch.empty(fd.fdas_batched_workspace_bytes(nspec), dtype=torch.uint8, device="cuda")
    fd.fdas_correlate_batched(specs, offs, nspec, bank, K, M, L, ref, ws)
    got = torch.full((K * total,), float("nan"), dtype=torch.float32, device="cuda")
    fd._lib.fdas_correlate_batched_noalloc(specs, offs, nspec, bank, K, M, L, got)
    torch.cuda.synchronize()
    return specs, offs, ref, got


@pytest.mark.parametrize("L,M", [(2048, 256), (512, 64)])
def test_noalloc_equals_workspace_call_twice(fd, L, M):
    zmax, dz = 40.0, 2.0
    taps, bank = fd.make_bank(zmax, dz, M, L)
    K = taps.shape[0]
    for call, (seed, nspec) in enumerate([(11, 40), (12, 9)]):
        spectra = _batch(seed, nspec, L, M)
        print(f"noalloc L={L} M={M} call {call}: nspec={nspec} "
              f"bins={sum(len(s) for s in spectra)}", flush=True)
        specs, offs, ref, got = _run_both(fd, spectra, bank, K, M, L)
        assert not torch.isnan(ref).any()
        assert not torch.isnan(got).any()
        assert torch.equal(got, ref), call
        # and one member against the FP64 oracle
        o = offs.cpu().numpy()
        b = 0
        n = int(o[b + 1] - o[b])
        view = got[K * o[b]:K * o[b + 1]].view(K, n).cpu().numpy()
        want = native.power(spectra[b], ot.templates(zmax, dz, M))
        assert np.max(np.abs(view - want)) / np.max(want) < 1e-5


def test_noalloc_rejects_oversized_batch(fd):
    L, M = 512, 64
    taps, bank = fd.make_bank(20.0, 2.0, M, L)
    K = taps.shape[0]
    n = fd._lib.NOALLOC_MAX_SPECTRA + 1
    specs = torch.zeros(4, dtype=torch.complex64, device="cuda")
    offs = torch.zeros(n + 1, dtype=torch.int64, device="cuda")
    planes = torch.zeros(4 * K, dtype=torch.float32, device="cuda")
    with pytest.raises(fd.FdasError, match="allocation-free"):
        fd._lib.fdas_correlate_batched_noalloc(specs, offs, n, bank, K, M, L, planes)


def test_noalloc_graph_replay_on_new_batches(fd):
    # captured once; offsets and spectra rewritten in place before each
    # replay, every replay equal to an eager call with a workspace, eager
    # work in between
    L, M, zmax = 512, 64, 20.0
    taps, bank = fd.make_bank(zmax, 2.0, M, L)
    K = taps.shape[0]
    nspec, cap = 8, 120000
    specs = torch.zeros(cap, dtype=torch.complex64, device="cuda")
    offs = torch.zeros(nspec + 1, dtype=torch.int64, device="cuda")
    planes = torch.zeros(K * cap, dtype=torch.float32, device="cuda")

    def fill(seed):
        rng = np.random.default_rng(seed)
        lens = rng.integers(0, 15000, nspec)
        o = np.zeros(nspec + 1, dtype=np.int64)
        o[1:] = np.cumsum(lens)
        specs[:o[-1]].copy_(torch.from_numpy(syn.random_spectrum(seed, int(o[-1]))))
        offs.copy_(torch.from_numpy(o))
        return o

    def call():
        fd._lib.fdas_correlate_batched_noalloc(specs, offs, nspec, bank, K, M, L, planes)

    fill(1)
    torch.cuda.synchronize()
    s = torch.cuda.Stream()
    s.wait_stream(torch.cuda.current_stream())
    with torch.cuda.stream(s):   # warm-up outside capture
        call()
    torch.cuda.current_stream().wait_stream(s)
    torch.cuda.synchronize()
    g = torch.cuda.CUDAGraph()
    with torch.cuda.graph(g):
        call()
    ws = torch.empty(fd.fdas_batched_workspace_bytes(nspec), dtype=torch.uint8, device="cuda")
    for seed in (2, 3, 4):
        o = fill(seed)
        planes.fill_(-1.0)
        print(f"noalloc graph replay seed {seed}: bins={int(o[-1])}", flush=True)
        g.replay()
        torch.cuda.synchronize()
        got = planes[:K * o[-1]].clone()
        ref = torch.full((K * int(o[-1]),), float("nan"), dtype=torch.float32, device="cuda")
        fd.fdas_correlate_batched(specs[:o[-1]], offs, nspec, bank, K, M, L, ref, ws)
        torch.cuda.synchronize()
        assert torch.equal(got, ref), seed
        _ = torch.randn(1000, device="cuda").sum()   # unrelated eager work between replays
