"""Pins of the oracle's puncture initial data (Sec. V: the Brill-Lindquist
conformal factor of eq. conformal_factor, the Bowen-York extrinsic curvature,
the lapse psi^-2) against what the mathematics fixes: psi - 1 is harmonic
away from the punctures and 2 r (psi - 1) = m far from a single hole (its
mass); the Bowen-York tensor psi^6 At_ij is trace free and divergence free
(the momentum constraint of conformally flat, maximal data) and carries the
hole's momentum and spin as the surface integrals P_i = (1/8 pi) oint A_ij n^j
dS and J_i = (1/8 pi) oint eps_ijk x^j A^kl n_l dS."""
import numpy as np

from oracle import oracle as O

HOLES = [(0.8, (-0.4, 0.3, 0.1), (0.05, -0.2, 0.1), (0.1, 0.3, -0.25)),
         (0.5, (0.7, -0.2, -0.3), (-0.1, 0.15, 0.0), (0.0, -0.1, 0.2))]
SYM = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]


def _box(N, lo=1.5, hi=2.5):
    """An N^3 grid on [lo, hi]^3 with two extra points on every side (for a
    4th-order stencil), away from both punctures."""
    h = (hi - lo) / (N - 1)
    ax = lo + h * np.arange(-2, N + 2)
    Z, Y, X = np.meshgrid(ax, ax, ax, indexing="ij")
    return X, Y, Z, h


def _d1(f, axis, h):
    """4th-order centred first derivative on the inner points of a (z, y, x) array."""
    s = [slice(2, -2)] * 3
    def sh(k):
        t = list(s)
        t[axis] = slice(2 + k, f.shape[axis] - 2 + k if f.shape[axis] - 2 + k != 0 else None)
        return f[tuple(t)]
    return (8.0 * (sh(1) - sh(-1)) - (sh(2) - sh(-2))) / (12.0 * h)


def _d2(f, axis, h):
    s = [slice(2, -2)] * 3
    def sh(k):
        t = list(s)
        t[axis] = slice(2 + k, f.shape[axis] - 2 + k if f.shape[axis] - 2 + k != 0 else None)
        return f[tuple(t)]
    return (-sh(2) + 16.0 * sh(1) - 30.0 * sh(0) + 16.0 * sh(-1) - sh(-2)) / (12.0 * h * h)


def test_conformal_factor_is_harmonic_away_from_the_punctures():
    errs = []
    for N in (12, 24, 48):
        X, Y, Z, h = _box(N)
        psi = O.ccz4_puncture_at(X, Y, Z, HOLES)[0] ** -0.25
        lap = sum(_d2(psi, a, h) for a in range(3))
        errs.append(np.max(np.abs(lap)))
    o = np.log2(errs[1] / errs[2])
    assert 3.7 < o < 4.3, (errs, o)


def test_far_field_gives_the_bare_mass_and_the_lapse_is_psi_minus_two():
    m, c = 1.3, (0.2, -0.1, 0.4)
    hole = [(m, c, (0.0, 0.0, 0.0), (0.0, 0.0, 0.0))]
    r = np.array([5.0, 50.0, 500.0])
    x = c[0] + r * 0.6
    y = c[1] - r * 0.8
    z = np.full_like(r, c[2])
    U = O.ccz4_puncture_at(x, y, z, hole)
    psi = U[0] ** -0.25
    assert np.allclose(2.0 * r * (psi - 1.0), m, rtol=1e-12, atol=0)
    assert np.allclose(U[18] ** 2, U[0], rtol=1e-14, atol=0)
    # the rest of the state: gt = delta, everything else zero (At too: no P, S)
    for q, (i, j) in enumerate(SYM):
        assert np.all(U[1 + q] == (1.0 if i == j else 0.0))
        assert np.all(U[8 + q] == 0.0)
    for f in [7] + list(range(14, 18)) + list(range(19, 25)):
        assert np.all(U[f] == 0.0)


def _Ahat(X, Y, Z, holes):
    U = O.ccz4_puncture_at(X, Y, Z, holes)
    A = np.empty((3, 3) + X.shape)
    psi6 = U[0] ** -1.5
    for q, (i, j) in enumerate(SYM):
        A[i, j] = A[j, i] = U[8 + q] * psi6
    return A


def test_bowen_york_tensor_is_trace_free_and_divergence_free():
    errs = []
    for N in (12, 24, 48):
        X, Y, Z, h = _box(N)
        A = _Ahat(X, Y, Z, HOLES)
        scale = np.max(np.abs(A))
        assert np.max(np.abs(A[0, 0] + A[1, 1] + A[2, 2])) < 1e-15 * scale
        # arrays are (z, y, x): axis 2 - j differentiates along x_j
        div = [sum(_d1(A[i, j], 2 - j, h) for j in range(3)) for i in range(3)]
        errs.append(max(np.max(np.abs(d)) for d in div))
    o = np.log2(errs[1] / errs[2])
    assert 3.7 < o < 4.3, (errs, o)


def _sphere(R, c, nt=24, nph=48):
    """Gauss-Legendre in cos(theta) x uniform in phi: exact for the
    polynomial integrands in n below."""
    mu, wmu = np.polynomial.legendre.leggauss(nt)
    ph = 2 * np.pi * np.arange(nph) / nph
    MU, PH = np.meshgrid(mu, ph, indexing="ij")
    st = np.sqrt(1 - MU ** 2)
    n = np.array([st * np.cos(PH), st * np.sin(PH), MU])
    w = (wmu[:, None] * np.ones_like(PH)) * (2 * np.pi / nph) * R * R
    x = [c[d] + R * n[d] for d in range(3)]
    return x, n, w


def test_bowen_york_surface_integrals_give_momentum_and_spin():
    m, c, P, S = 0.9, (0.3, -0.2, 0.5), np.array([0.07, -0.11, 0.05]), np.array([-0.2, 0.15, 0.33])
    hole = [(m, c, tuple(P), tuple(S))]
    eps = np.zeros((3, 3, 3))
    eps[0, 1, 2] = eps[1, 2, 0] = eps[2, 0, 1] = 1.0
    eps[0, 2, 1] = eps[2, 1, 0] = eps[1, 0, 2] = -1.0
    for R in (0.5, 3.0):
        x, n, w = _sphere(R, c)
        A = _Ahat(x[0], x[1], x[2], hole)
        An = np.einsum("ij...,j...->i...", A, n)
        Pg = np.array([np.sum(An[i] * w) for i in range(3)]) / (8 * np.pi)
        r = np.array([x[d] - c[d] for d in range(3)])
        Jg = np.array([np.sum(np.einsum("jk,j...,k...->...", eps[i], r, An) * w) for i in range(3)]) / (8 * np.pi)
        assert np.allclose(Pg, P, rtol=0, atol=1e-13), (R, Pg, P)
        assert np.allclose(Jg, S, rtol=0, atol=1e-13), (R, Jg, S)
