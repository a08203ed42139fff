"""Pins for the oracle's loss gradients.

Lw = sum w |Y|^2 is a real quadratic form in (Re A, Im A) and in
(Re T, Im T), so central finite differences are exact up to rounding for
any step: they pin the analytic adjoint formulas independently.
"""
import numpy as np
import pytest

import fdas_synth as syn
from oracle import direct, native


def _setup(seed, N=40, K=3, M=8):
    rng = np.random.default_rng(seed)
    A = (rng.normal(size=N) + 1j * rng.normal(size=N)) / np.sqrt(2)
    T = (rng.normal(size=(K, M)) + 1j * rng.normal(size=(K, M))) / np.sqrt(2 * M)
    w = rng.random((K, N))
    return A, T, w


def _fd_grad(f, x, h):
    g = np.zeros_like(x)
    flat = x.reshape(-1)
    gf = g.reshape(-1)
    for i in range(flat.size):
        for unit, part in ((1.0, "re"), (1j, "im")):
            xp = flat.copy(); xp[i] += unit * h
            xm = flat.copy(); xm[i] -= unit * h
            d = (f(xp.reshape(x.shape)) - f(xm.reshape(x.shape))) / (2 * h)
            gf[i] += d if part == "re" else 1j * d
    return g


@pytest.mark.parametrize("h", [1e-2, 1.0])
def test_grad_A_central_differences(h):
    A, T, w = _setup(0)
    gA, _ = direct.grads(A, T, w)
    fd = _fd_grad(lambda a: direct.loss(a, T, w), A, h)
    assert np.max(np.abs(gA - fd)) < 1e-9 * np.max(np.abs(fd))


@pytest.mark.parametrize("h", [1e-2, 1.0])
def test_grad_T_central_differences(h):
    A, T, w = _setup(1)
    _, gT = direct.grads(A, T, w)
    fd = _fd_grad(lambda t: direct.loss(A, t, w), T, h)
    assert np.max(np.abs(gT - fd)) < 1e-9 * np.max(np.abs(fd))


def test_grads_at_edges_and_odd_sizes():
    A, T, w = _setup(2, N=7, K=2, M=12)   # M > N: every output touches an edge
    gA, gT = direct.grads(A, T, w)
    assert np.max(np.abs(gA - _fd_grad(lambda a: direct.loss(a, T, w), A, 0.5))) < 1e-9
    assert np.max(np.abs(gT - _fd_grad(lambda t: direct.loss(A, t, w), T, 0.5))) < 1e-9


def test_c_grads_match_numpy():
    A, T, w = _setup(3, N=3000, K=5, M=32)
    w = w.astype(np.float32)
    gA, gT = direct.grads(A, T, w)
    cA, cT = native.grads(A, T, w)
    assert np.max(np.abs(gA - cA)) < 1e-11 * np.max(np.abs(gA))
    assert np.max(np.abs(gT - cT)) < 1e-11 * np.max(np.abs(gT))


def test_grad_of_linear_weights_is_adjoint_of_correlation():
    # With w = 1 the gradient w.r.t. A is 2 C^H C A, where C is the
    # correlation operator; check <C x, C y> identities via random probes.
    A, T, _ = _setup(4, N=64, K=2, M=8)
    w = np.ones((2, 64))
    gA, _ = direct.grads(A, T, w)
    rng = np.random.default_rng(5)
    x = rng.normal(size=64) + 1j * rng.normal(size=64)
    # directional derivative of Lw along x equals Re <gA, x>
    eps = 1e-3
    d = (direct.loss(A + eps * x, T, w) - direct.loss(A - eps * x, T, w)) / (2 * eps)
    assert abs(d - np.real(np.vdot(gA, x))) < 1e-9 * abs(d)
    # and the plain spectrum is unaffected by the synth helpers
    assert syn.random_spectrum(1, 4).dtype == np.complex64


def test_c_grad_spec_points_match_full_gradient():
    # the per-point spectrum gradient (used for sampled checks at full size)
    # equals the full adjoint at every bin, including both edges
    A, T, w = _setup(6, N=700, K=4, M=24)
    w = w.astype(np.float32)
    gA, _ = direct.grads(A, T, w)
    ks = np.array([0, 1, 5, 11, 12, 13, 350, 687, 688, 699], dtype=np.int64)
    got = native.grad_spec_points(A, T, w, ks)
    assert np.max(np.abs(got - gA[ks])) < 1e-11 * np.max(np.abs(gA))
