"""The LDS bank rules the segment transforms' layout is built for, measured
on the device with the library's LDS bank probe (fdas_lds_probe).

One wave repeats one LDS access, lane l at element pattern[l]; the loop's
cycles per access rise when a pass of the access puts two lanes on one bank.
The patterns tell the candidate rules apart:
  * 64-bit writes go in passes of 16 lanes over 32 banks: lanes 0-15 at
    values 0..15 and 16-31 at 32..47 are conflict-free (PA), lanes 0-7 at
    0..7 and 8-15 at 16..23 are not (PB: 16 apart is the same bank);
  * 64-bit reads go in passes of 32 lanes over 64 banks: the other way round
    (PB is conflict-free, PA is not: 32 values apart is the same bank);
  * 128-bit writes go in passes of 8 lanes: a stride of 2 pairs conflicts,
    8-lane runs 32 pairs apart (PC) do not.
Run as a script it prints every pattern's cycles per access (the probe's
summary under profiles/ was made that way).
"""
import pytest

torch = pytest.importorskip("torch")

PATTERNS = {
    "contiguous": lambda l: l,
    "stride2": lambda l: 2 * l,
    "stride16": lambda l: 16 * l,
    "PA": lambda l: (l & 15) + 32 * (l >> 4),
    "PB": lambda l: (l & 7) + 16 * ((l >> 3) & 1) + 8 * ((l >> 4) & 1) + 32 * (l >> 5),
    "PC": lambda l: (l & 7) + 32 * ((l >> 3) & 1) + 8 * (l >> 4),
}
MODES = {0: "64-bit write", 1: "64-bit read", 2: "128-bit write"}
ITERS, GROUPS = 512, 256


def measure(fd, mode, name):
    pat = torch.tensor([PATTERNS[name](l) for l in range(64)], dtype=torch.int32, device="cuda")
    cyc = torch.empty(GROUPS, dtype=torch.int64, device="cuda")
    sink = torch.empty(64 * GROUPS, dtype=torch.float32, device="cuda")
    fd.fdas_lds_probe(pat, mode, ITERS, GROUPS, cyc, sink)
    torch.cuda.synchronize()
    return float(cyc.double().median().item()) / ITERS


@pytest.fixture(scope="module")
def fd():
    import paper_1804_05335_amd as f
    f.lib()
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    return f


# (mode, conflict-free patterns, conflicting patterns)
RULES = [(0, ["contiguous", "PA"], ["PB", "stride2", "stride16"]),
         (1, ["contiguous", "PB"], ["PA", "stride2", "stride16"]),
         (2, ["contiguous", "PA", "PB", "PC"], ["stride2", "stride16"])]


@pytest.mark.gpu
@pytest.mark.parametrize("mode,free,conflicting", RULES)
def test_lds_bank_rules(fd, mode, free, conflicting):
    base = measure(fd, mode, "contiguous")
    for name in free:
        c = measure(fd, mode, name)
        print(f"{MODES[mode]} {name}: {c:.2f} cycles per access (contiguous {base:.2f})")
        assert c < base + 0.75, (mode, name, c, base)
    for name in conflicting:
        c = measure(fd, mode, name)
        print(f"{MODES[mode]} {name}: {c:.2f} cycles per access (contiguous {base:.2f})")
        assert c > base + 1.5, (mode, name, c, base)


if __name__ == "__main__":
    import os
    import sys
    sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))
    import paper_1804_05335_amd as f
    f.lib()
    for mode in MODES:
        for name in PATTERNS:
            print(f"{MODES[mode]:14s} {name:10s} {measure(f, mode, name):7.2f} cycles per access",
                  flush=True)
