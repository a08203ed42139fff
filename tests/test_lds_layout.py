"""The transforms' LDS layout against gfx950's LDS bank rules (CPU model).

Measured on the device with an LDS probe (one wave timing each access pattern
and rocprofv3's SQ_LDS_BANK_CONFLICT): a 64-bit LDS read is served in two
passes of 32 lanes over 64 four-byte banks, a 64-bit write in four passes of
16 lanes over 32 banks, and a 128-bit write in eight passes of 8 lanes over
32 banks.  A pass is conflict-free when its lanes' accesses cover distinct
banks, i.e. (counting in complex values of 8 bytes):
  * 64-bit reads:  the 32 lanes' indices are distinct mod 32;
  * 64-bit writes: the 16 lanes' indices are distinct mod 16;
  * 128-bit writes (two adjacent complex values): the 8 lanes' pair indices
    are distinct mod 8.
Every exchange of every transform plan is enumerated here with the index
formulas of the Stockham passes (butterfly j of pass (NS, R) writes its i-th
output to (j / NS) NS R + j mod NS + i NS; after the exchange lane t reads
t + m T), mapped through the library's lds_pad, and checked against these
rules; at L = 8192 the first pass (NS = 1) writes adjacent output pairs with
one 128-bit store, so those pairs must stay adjacent and 16-byte aligned in
the layout (checked for every plan).
"""
import ctypes

import numpy as np
import pytest

PLANS = {  # (L, E): radices, as the library's Plan<L, E>
    (256, 4): (4, 4, 4, 4),
    (512, 8): (8, 8, 8),
    (1024, 8): (8, 8, 8, 2),
    (1024, 16): (16, 16, 4),
    (2048, 8): (8, 8, 8, 4),
    (2048, 16): (16, 16, 8),
    (4096, 8): (8, 8, 8, 8),
    (4096, 16): (16, 16, 16),
    (8192, 8): (8, 8, 8, 8, 2),
    (8192, 16): (16, 16, 16, 2),
}


@pytest.fixture(scope="module")
def lib():
    from tests.emu import build_emu
    lib = ctypes.CDLL(build_emu.build_lds_layout())
    lib.emu_lds_pad.restype = ctypes.c_int
    lib.emu_lds_pad.argtypes = [ctypes.c_int, ctypes.c_int]
    lib.emu_pair_writes.restype = ctypes.c_int
    lib.emu_pair_writes.argtypes = [ctypes.c_int]
    return lib


def _distinct(vals, mod):
    return len({v % mod for v in vals}) == len(vals)


@pytest.mark.parametrize("pair", [False, True])
@pytest.mark.parametrize("L,E", sorted(PLANS))
def test_layout_is_a_bijection(lib, L, E, pair):
    img = [lib.emu_lds_pad(i, pair) for i in range(L)]
    assert sorted(img) == list(range(L))


def test_pair_writes_only_at_8192(lib):
    assert [lib.emu_pair_writes(L) for L in (256, 512, 1024, 2048, 4096, 8192)] == [0] * 5 + [1]


def _check_plan(pad, L, E, pair):
    radices = PLANS[(L, E)]
    T = L // E
    NS = 1
    for p, R in enumerate(radices[:-1]):       # the last pass writes no LDS
        NB = E // R
        for u in range(NB):
            j = np.arange(T) + u * T
            base = (j // NS) * (NS * R) + (j % NS)
            if NS == 1 and pair:
                # adjacent output pairs (2q, 2q + 1) in one 128-bit store
                for q in range(R // 2):
                    lo = [pad(b + 2 * q) for b in base]
                    hi = [pad(b + 2 * q + 1) for b in base]
                    assert all(h == x + 1 and x % 2 == 0 for x, h in zip(lo, hi)), (L, E, q)
                    for g0 in range(0, T, 8):
                        assert _distinct([x // 2 for x in lo[g0:g0 + 8]], 8), (L, E, p, q, g0)
            else:
                for i in range(R):
                    addr = [pad(b + i * NS) for b in base]
                    for g0 in range(0, T, 16):
                        assert _distinct(addr[g0:g0 + 16], 16), (L, E, p, i, g0)
        for m in range(E):
            addr = [pad(t + m * T) for t in range(T)]
            for g0 in range(0, T, 32):
                assert _distinct(addr[g0:g0 + 32], 32), (L, E, p, m, g0)
        NS *= R


@pytest.mark.parametrize("L,E", sorted(PLANS))
def test_exchanges_are_bank_conflict_free(lib, L, E):
    # the layout and write width each plan uses; both maps are also checked
    # on every plan, so either would serve any length
    pair = bool(lib.emu_pair_writes(L))
    _check_plan(lambda i: lib.emu_lds_pad(int(i), pair), L, E, pair)
    _check_plan(lambda i: lib.emu_lds_pad(int(i), not pair), L, E, not pair)


def _xor5_layout(idx):
    # an earlier layout: the low five bits XORed with a function of idx >> 5
    h = idx >> 5
    g = (h & 7) | ((((h >> 1) ^ (h >> 3)) & 1) << 3) | ((((h >> 2) ^ (h >> 3)) & 1) << 4)
    return idx ^ g


def test_bank_rules_have_teeth():
    # Plain stride-16 first-pass writes put all 16 lanes of a pass on one bank,
    # and the earlier five-bit XOR layout, conflict-free for the reads, still
    # pairs the lanes of those writes two to a bank -- the 2-way conflicts the
    # counters showed on half of that layout's exchange writes.
    idx = [16 * t for t in range(16)]
    assert len({i % 16 for i in idx}) == 1
    assert len({_xor5_layout(i) % 16 for i in idx}) == 8
    assert all(_distinct([_xor5_layout(t + 32 * a) for t in range(32)], 32) for a in range(8))
