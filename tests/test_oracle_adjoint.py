"""Pins of the oracle's discrete adjoint of the periodic wave RK4 step: the
dot-product identity against the (spectrally pinned) forward oracle, and the
gradient of the sphere objective against central differences."""
import numpy as np

from oracle import oracle as O
from paper_1806_04182_amd import synth


def _J(U, xlo, h, rad):
    return O.sphere_integral(U, 0, xlo, h, rad)


def test_rhs_adjoint_dot_product():
    rng = np.random.default_rng(0)
    n = (9, 7, 6)
    h = (0.2, 0.2, 0.2)
    v = synth.embed(rng.standard_normal((2, n[2], n[1], n[0])))
    O.fill_periodic(v)
    w = synth.embed(rng.standard_normal((2, n[2], n[1], n[0])))
    Lv = O.rhs(O.WAVE, v, h)
    lhs = np.sum(synth.interior(Lv) * synth.interior(w))
    A = O.wave_rhs_adjoint(w, h)
    O.fill_periodic_adjoint(A)
    rhs = np.sum(synth.interior(A) * synth.interior(v))
    assert abs(lhs - rhs) < 1e-12 * max(1.0, abs(lhs))


def test_rk4_adjoint_dot_product_with_forward():
    """<P^n v, lam_T> computed by the forward oracle equals <v, lam_0> from the
    reverse sweep, for a random v (J is linear in the state)."""
    rng = np.random.default_rng(1)
    n = (12, 10, 8)
    dx = 2.0 / 12
    h = (dx, dx, dx)
    xlo = (-1.0, -1.0, -1.0)
    v = synth.embed(rng.standard_normal((2, n[2], n[1], n[0])))
    U = v.copy()
    nsteps = 7
    dt = 0.25 * dx
    O.rk_run(O.WAVE, O.RK4, U, h, dt, nsteps)
    J = _J(U, xlo, h, 0.6)
    lam0 = O.wave_adjoint_run(n, h, xlo, dt, nsteps, 0.6)
    assert abs(J - np.sum(synth.interior(lam0) * synth.interior(v))) < 1e-12 * max(1.0, abs(J))


def test_gradient_matches_central_differences_and_closed_form():
    n = (16, 16, 16)
    dx = 2.0 / 16
    h = (dx, dx, dx)
    xlo = (-1.0, -1.0, -1.0)
    nsteps, dt, rad = 10, 0.25 * dx, 0.6
    p0 = np.array([1.0, 0.3, 0.05, -0.1, 0.07])

    def J(p):
        U = synth.embed(synth.wave_gaussian(n, xlo, dx, amp=p[0], width=p[1], centre=p[2:], period=(2, 2, 2)))
        O.rk_run(O.WAVE, O.RK4, U, h, dt, nsteps)
        return _J(U, xlo, h, rad)

    lam0 = synth.interior(O.wave_adjoint_run(n, h, xlo, dt, nsteps, rad))[0]
    # d phi_0 / d p on the grid (closed form of the Gaussian)
    z, y, x = synth.grid((0, 0, 0), n, dx)
    d = [x - 1 - p0[2], y - 1 - p0[3], z - 1 - p0[4]]
    d = [di - 2 * np.round(di / 2) for di in d]
    r2 = d[0] ** 2 + d[1] ** 2 + d[2] ** 2
    E = np.exp(-r2 / p0[1] ** 2)
    dphi = [E, p0[0] * E * 2 * r2 / p0[1] ** 3] + [p0[0] * E * 2 * di / p0[1] ** 2 for di in d]
    grad = np.array([np.sum(lam0 * np.broadcast_to(g, lam0.shape)) for g in dphi])
    J0 = J(p0)
    assert abs(grad[0] - J0 / p0[0]) < 1e-12 * abs(J0)  # J is linear in A
    for i in range(5):
        e = np.zeros(5)
        e[i] = 1e-6
        fd = (J(p0 + e) - J(p0 - e)) / 2e-6
        assert abs(fd - grad[i]) < 1e-6 * max(abs(grad[i]), 1e-3 * abs(J0)), (i, fd, grad[i])
