"""Pin of the oracle's radiative outer boundary (Sec. V): an outgoing
spherical wave phi = g(r - t)/r, Pi = g'(r - t)/r is an exact solution of the
wave system for which the radiative condition with v = 1, U_inf = 0 holds
exactly, so the error stays at truncation level while the pulse leaves the
box and converges (2nd order: the boundary stencils are of 2nd order)."""
import numpy as np
import pytest

from oracle import oracle as O


def _exact(X, Y, Z, t, w=0.4, r0=1.0):
    r = np.sqrt(X ** 2 + Y ** 2 + Z ** 2)
    g = lambda s: np.exp(-(s - r0) ** 2 / w ** 2)
    dg = lambda s: -2 * (s - r0) / w ** 2 * g(s)
    return g(r - t) / r, dg(r - t) / r


def _run(N, T, L=2.0):
    h = 2 * L / N
    xlo = -L + 0.5 * h  # no grid point at the origin
    H = O.Hierarchy(O.WAVE, (N, N, N), (xlo, xlo, xlo), h, [(1, [((0, 0, 0), (N - 1, N - 1, N - 1))])])
    H.set_open([1.0, 1.0], [0.0, 0.0])
    x = xlo + (np.arange(N + 6) - 3) * h
    Z, Y, X = np.meshgrid(x, x, x, indexing="ij")
    H.set(0, 0, np.stack(_exact(X, Y, Z, 0.0)))
    nsteps = int(round(T / (0.25 * h)))
    for _ in range(nsteps):
        H.step(0.25 * h, O.params(sigma=0.1))
    u = H.get(0, 0)[:, 3:-3, 3:-3, 3:-3]
    xi = x[3:-3]
    Z, Y, X = np.meshgrid(xi, xi, xi, indexing="ij")
    ephi, _ = _exact(X, Y, Z, T)
    return np.sum(np.abs(u[0] - ephi)) / np.sum(np.abs(ephi))


def test_outgoing_spherical_wave_leaves_through_radiative_boundary():
    e24, e48 = _run(24, 1.5), _run(48, 1.5)
    assert e48 < 0.03, e48
    assert 1.7 < np.log2(e24 / e48) < 3.5, (e24, e48)
