"""GPU check of the streaming probes the benchmark reads the HBM ceiling
from: the write fills exactly the buffer (tails included, nothing past it)
and the read's partial sums add up to the buffer's exact sum."""
import numpy as np
import pytest

torch = pytest.importorskip("torch")
pytestmark = pytest.mark.gpu


@pytest.fixture(scope="module")
def fd():
    import paper_1804_05335_amd as f
    f.lib()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return f


@pytest.mark.parametrize("n", [0, 1, 3, 4, 1027, (1 << 20) + 5, 1 << 28])
def test_write_then_read(fd, n):
    P = fd._lib.STREAM_PARTIALS
    guard = 1 << 12
    buf = torch.full((n + 2 * guard,), -7.0, dtype=torch.float32, device="cuda")
    arr = buf[guard:guard + n]
    if n:
        fd.fdas_stream_write(arr, 1.5)
    torch.cuda.synchronize()
    assert torch.all(buf[:guard] == -7.0) and torch.all(buf[guard + n:] == -7.0)
    assert torch.all(arr == 1.5)
    # small integers: every partial and the total are exact in FP32 / FP64
    vals = (torch.arange(n, device="cuda", dtype=torch.int64) % 7).to(torch.float32)
    sums = torch.full((P,), float("nan"), dtype=torch.float32, device="cuda")
    fd.fdas_stream_read(vals, sums)
    torch.cuda.synchronize()
    got = sums.cpu().numpy().astype(np.float64)
    assert np.all(np.isfinite(got))
    assert got.sum() == float(vals.double().sum().item())
