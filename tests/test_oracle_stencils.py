"""Pins of the oracle's finite-difference stencils (Sec. II.B.1) against
calculus: exactness on monomials, first error term, KO symbol."""
import math

import numpy as np
import pytest

from oracle import oracle as O


def _line(p, h, n=13, c=6, x0=0.37):
    x = x0 + (np.arange(n) - c) * h
    return x ** p, x0


@pytest.mark.parametrize("h", [0.1, 0.05])
def test_d1_exact_to_degree4_and_error_at_5(h):
    for p in range(0, 5):
        u, x0 = _line(p, h)
        exact = p * x0 ** (p - 1) if p > 0 else 0.0
        assert abs(O.stencil("d1", u, 6, 1, h) - exact) < 1e-10 * max(1, abs(exact))
    # first error term: D1 x^5 - 5 x^4 = -(h^4/30) * 5! / 4! ... = -4 h^4 (for x^5)
    u, x0 = _line(5, h)
    err = O.stencil("d1", u, 6, 1, h) - 5 * x0 ** 4
    assert abs(err - (-4.0 * h ** 4)) < 1e-9


@pytest.mark.parametrize("h", [0.1, 0.03])
def test_d2_exact_to_degree5(h):
    for p in range(0, 6):
        u, x0 = _line(p, h)
        exact = p * (p - 1) * x0 ** (p - 2) if p > 1 else 0.0
        assert abs(O.stencil("d2", u, 6, 1, h) - exact) < 1e-8 * max(1, abs(exact))
    u, x0 = _line(6, h)
    err = O.stencil("d2", u, 6, 1, h) - 30 * x0 ** 4
    # truncation: -(h^4/90) u^(6) = -(h^4/90) * 720 = -8 h^4
    assert abs(err + 8.0 * h ** 4) < 1e-8


@pytest.mark.parametrize("beta", [-0.7, 0.4, 0.0])
def test_lopsided_advection_exact_to_degree4(beta):
    h = 0.05
    for p in range(0, 5):
        u, x0 = _line(p, h)
        exact = p * x0 ** (p - 1) if p > 0 else 0.0
        assert abs(O.stencil("adv", u, 6, 1, h, beta) - exact) < 1e-9 * max(1, abs(exact))
    # one-sidedness: beta > 0 must not read i-2, beta < 0 must not read i+2
    u = np.zeros(13)
    u[6 - 2] = 1.0
    v = O.stencil("adv", u, 6, 1, h, 0.5)
    assert v == 0.0
    u = np.zeros(13)
    u[6 + 2] = 1.0
    assert O.stencil("adv", u, 6, 1, h, -0.5) == 0.0


def test_ko_annihilates_degree5_and_symbol():
    h, sigma = 0.1, 0.3
    for p in range(0, 6):
        u, _ = _line(p, h)
        assert abs(O.stencil("ko", u, 6, 1, h, sigma)) < 1e-9
    u, _ = _line(6, h)
    # sixth central difference of x^6 is 6! h^6
    assert abs(O.stencil("ko", u, 6, 1, h, sigma) - sigma / (64 * h) * 720 * h ** 6) < 1e-12
    # Nyquist mode (-1)^i: Q = -sigma/h * u (dissipative)
    u = (-1.0) ** np.arange(13)
    assert abs(O.stencil("ko", u, 6, 1, h, sigma) - (-sigma / h) * u[6]) < 1e-12


def test_mixed_derivative_exact_to_degree4_each_axis():
    h1, h2 = 0.1, 0.07
    n = 9
    x = 0.2 + (np.arange(n) - 4) * h1
    y = -0.3 + (np.arange(n) - 4) * h2
    for a in range(5):
        for b in range(5):
            u = np.ascontiguousarray((y[:, None] ** b) * (x[None, :] ** a))
            c = 4 * n + 4
            exact = (a * x[4] ** (a - 1) if a else 0.0) * (b * y[4] ** (b - 1) if b else 0.0)
            got = O.dmix(u.ravel(), c, 1, h1, n, h2)
            assert abs(got - exact) < 1e-9 * max(1, abs(exact)), (a, b)


def test_difference_form_on_offset_background():
    """A 1e-10 perturbation on an O(1) background: the stencils are evaluated as
    weighted differences, so the result equals the one on the bare
    perturbation to close to its own precision."""
    rng = np.random.default_rng(1)
    eps = 1e-10 * rng.uniform(-1, 1, 13)
    h = 1 / 32
    for name, extra in (("d1", ()), ("d2", ()), ("ko", (0.1,)), ("adv", (0.3,))):
        a = O.stencil(name, 1.0 + eps, 6, 1, h, *extra)
        b = O.stencil(name, eps, 6, 1, h, *extra)
        # rounding of 1+eps costs ~1e-16 absolute per point
        scale = {"d1": 1 / h, "d2": 1 / h ** 2, "ko": 1 / h, "adv": 1 / h}[name]
        assert abs(a - b) < 64 * 2.3e-16 * scale
