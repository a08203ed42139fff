"""Pins for the oracle's templates (Sec. 2, eq. 23 and the text around it).

The closed form is checked against things other than itself: quadrature of
the defining integral, the Kronecker delta at z = 0, evenness in q at integer
offsets, Parseval's energy, and the scalloping loss the paper prints.
"""
import os

import numpy as np
import pytest

from oracle import templates as ot
from tests.quadrature import response_quadrature as _quadrature

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("z", [0.0, 2.0, -2.0, 8.0, -20.0, 84.0, -84.0, 200.0, -200.0, 7.3])
def test_closed_form_matches_quadrature(z):
    q = np.concatenate([np.arange(-260, 261, 13, dtype=np.float64),
                        np.array([-0.5, 0.3, 0.5, 1.7, 99.25, -150.75])])
    ref = _quadrature(q, z)
    got = ot.response(q, z)
    assert np.max(np.abs(got - ref)) < 1e-11


def test_zero_z_template_is_delta():
    T = ot.templates(20.0, 2.0, 64)
    k0 = 10  # z = 0 row for zmax = 20, dz = 2
    assert ot.z_grid(20.0, 2.0)[k0] == 0.0
    row = T[k0]
    assert abs(row[32] - 1.0) < 1e-15
    assert np.max(np.abs(np.delete(row, 32))) < 1e-12


@pytest.mark.parametrize("z", [2.0, 8.0, 84.0, 200.0])
def test_even_in_integer_offset(z):
    # R(-q, z) = exp(-i 2 pi q) R(q, z) (substitute u -> 1 - u); at integer q
    # the factor is 1, so tap sign conventions cannot matter on the bin grid.
    q = np.arange(-300, 301, dtype=np.float64)
    r = ot.response(q, z)
    assert np.max(np.abs(r - r[::-1])) < 1e-12
    # off the grid the reflection carries the phase exp(-i 2 pi q)
    qh = np.linspace(-50.3, 50.3, 77)
    rh = ot.response(qh, z)
    assert np.max(np.abs(ot.response(-qh, z) - np.exp(-2j * np.pi * qh) * rh)) < 1e-12


@pytest.mark.parametrize("z", [2.0, 20.0, 84.0, 200.0])
def test_conjugate_symmetry_of_bank(z):
    # +/-z templates are complex conjugates of each other on the tap grid
    # (the symmetry the paper exploits, Sec. 4.2 first paragraph).
    e = ot.tap_offsets(512)
    assert np.max(np.abs(ot.response(e, -z) - np.conj(ot.response(e, z)))) < 1e-12


@pytest.mark.parametrize("z", [0.0, 8.0, 84.0, 200.0])
def test_parseval_energy_is_one(z):
    # sum over all integer q of |R(q,z)|^2 = int_0^1 |x(u)|^2 du = 1 for the
    # normalised (unit-amplitude) response; the tail beyond |q| > Q is
    # bounded by ~ 2 / (pi^2 (Q - |z|)).
    Q = 20000
    q = np.arange(-Q, Q + 1, dtype=np.float64)
    s = np.sum(np.abs(ot.response(q, z)) ** 2)
    assert abs(s - 1.0) < 3.0 / (np.pi ** 2 * (Q - abs(z)))


def test_paper_scalloping_loss():
    rows = [l.split() for l in open(os.path.join(GOLDEN, "scalloping_loss.txt"))
            if l.strip() and not l.startswith("#")]
    for off, z, pct, digits in rows:
        loss = 100.0 * (1.0 - abs(ot.response(np.array([float(off)]), float(z))[0]))
        assert round(loss, int(digits) - 2) == float(pct)
        assert abs(loss - 100.0 * (1.0 - 2.0 / np.pi)) < 1e-12


def test_z_grid_and_offsets():
    z = ot.z_grid(84.0, 2.0)
    assert len(z) == 85 and z[0] == -84.0 and z[-1] == 84.0 and z[42] == 0.0
    e = ot.tap_offsets(8)
    assert list(e) == [-4, -3, -2, -1, 0, 1, 2, 3]
