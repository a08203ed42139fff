"""Composite Gauss-Legendre quadrature of the template's defining integral
(test helper, independent of both the oracle's and the library's closed
forms): int_0^1 exp(i 2 pi [q u + z (u^2 - u)/2]) du."""
import numpy as np


def response_quadrature(q, z, panels=1200, order=16):
    x, wts = np.polynomial.legendre.leggauss(order)
    edges = np.linspace(0.0, 1.0, panels + 1)
    a, b = edges[:-1], edges[1:]
    u = (0.5 * (b - a))[:, None] * x[None, :] + (0.5 * (a + b))[:, None]
    w = (0.5 * (b - a))[:, None] * wts[None, :]
    u, w = u.ravel(), w.ravel()
    q = np.asarray(q, dtype=np.float64)
    phase = 2 * np.pi * (q[:, None] * u[None, :] + 0.5 * z * (u * u - u)[None, :])
    return (np.exp(1j * phase) * w[None, :]).sum(axis=1)
