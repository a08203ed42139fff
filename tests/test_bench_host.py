"""Host-side logic of bench.py (no GPU): the one-GPU guard, the algorithmic
work model the roofline uses, and the rule that HBM traffic is read from a
counter summary only when it was taken from the current kernel sources."""
import os
import subprocess
import sys

import bench

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused_with_a_message():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"],
                       capture_output=True, text=True, timeout=120)
    assert r.returncode == 2
    assert "one GPU" in r.stderr
    assert r.stdout == ""


def test_forward_work_model_at_the_headline_size():
    # 2^21 bins, 85 templates x 256 taps, L = 2048: B = 1792, S = ceil(N / B)
    N, K, M, L = 1 << 21, 85, 256, 2048
    S = -(-N // (L - M))
    assert S == 1171
    nbytes, flops = bench.forward_work(N, K, M, L)
    # spectrum read once, plane written once, bank read once
    assert nbytes == 8 * N + 4 * K * N + 8 * K * L
    fft = 4.25 * L * 11
    assert flops == S * fft + S * K * (6 * L + fft) + 3 * K * N


def test_lds_and_adjoint_work_models():
    N, K, M, L = 1 << 21, 85, 256, 2048
    # two exchanges of L complex values per transform, K + 1 transforms per
    # segment: about 3.3 GB written (and read again) per launch at the
    # headline size; reads run at twice the write rate
    assert bench.forward_lds_bytes(N, K, M, L) == 1171 * 86 * 2 * L * 8
    assert bench.LDS_READ_PEAK_GBS == 2 * bench.LDS_WRITE_PEAK_GBS
    # adjoint at 2^20 bins, 85 x 128 taps, L = 512: windows of L - M owned bins
    N, K, M, L = 1 << 20, 85, 128, 512
    S = -(-N // (L - M))
    fft = 4.25 * L * 9
    b_spec, f_spec = bench.backward_work(N, K, M, L, False)
    b_full, f_full = bench.backward_work(N, K, M, L, True)
    assert b_spec == 8 * N + 4 * K * N + 8 * K * L + 8 * N
    assert b_full == b_spec + 8 * K * M
    assert f_spec == S * 2 * fft + S * K * (2 * fft + 16 * L)
    # the taps: X conj(G) accumulated per template and window, one inverse
    # transform per template
    assert f_full == f_spec + S * K * 8 * L + K * fft
    r = bench.roof_pair(b_full, f_full, 1.0)
    assert abs(r["hbm_GBps"] - b_full / 1e6) < 0.01 and 0 < r["alu_frac"] < 1


def test_paper_units():
    # points/s x 128 us / K: 7e11 points/s at 85 templates is about 1.05e6 series
    u = bench.paper_units(7e11, 85)
    assert u["real_time_series"] == round(7e11 * 128e-6 / 85)
    # the paper's own counts convert back to its derived 2e10 points/s at K = 64
    assert abs(bench.PAPER_P100_SERIES_2E21[64] * 64 / 128e-6 - 2.08e10) < 0.01e10


def _summary(path, khash, fetch, write):
    with open(path, "w") as f:
        f.write("# summary\n\n| counter | value |\n|---|---|\n| FETCH_SIZE | 1 KiB |\n\n")
        f.write(f"kernel_sources_hash: {khash}\n")
        f.write(f"fetch_bytes_per_launch: {fetch}\nwrite_bytes_per_launch: {write}\n")


def test_traffic_only_from_summaries_of_the_current_sources(tmp_path, monkeypatch):
    cur = bench.kernel_sources_hash()
    os.makedirs(tmp_path / "profiles")
    monkeypatch.setattr(bench, "ROOT", str(tmp_path))
    monkeypatch.setattr(bench, "kernel_sources_hash", lambda files=None: cur)
    _summary(tmp_path / "profiles" / "now.md", cur, 100, 23)
    _summary(tmp_path / "profiles" / "old.md", "0" * 16, 100, 23)
    assert bench.read_traffic("now.md") == 123.0
    assert bench.read_traffic("old.md") is None
    assert bench.read_traffic("missing.md") is None


def test_kernel_sources_hash_is_stable_and_short():
    a, b = bench.kernel_sources_hash(), bench.kernel_sources_hash()
    assert a == b and len(a) == 16 and int(a, 16) >= 0
    # a summary can name the files of its kernel: the hash then covers those only
    f = bench.kernel_sources_hash(["fdas_r2c.hip", "fdas_fft.hpp"])
    assert f == bench.kernel_sources_hash(["fdas_fft.hpp", "fdas_r2c.hip"]) and f != a
