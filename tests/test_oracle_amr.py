"""Pins of the oracle's prolongation, dense output, BOR and sub-cycled AMR
step (Sec. III, App. C, App. D)."""
import os
from fractions import Fraction

import numpy as np
import pytest

from oracle import oracle as O
from paper_1806_04182_amd import synth

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_lagrange_midpoint_matches_paper():
    vals = [l for l in open(os.path.join(GOLD, "lagrange_midpoint.txt")) if not l.startswith("#")]
    nums = [int(v) for v in vals[0].split()]
    w = O.lagrange6(0.5)
    assert np.allclose(w, np.array(nums[:6]) / nums[6], rtol=0, atol=1e-15)


@pytest.mark.parametrize("xi", [0.0, 1 / 3, 0.5, 2 / 3, 0.25])
def test_lagrange_exact_to_degree5(xi):
    w = O.lagrange6(xi)
    nodes = np.arange(-2, 4)
    for p in range(6):
        assert abs(np.dot(w, nodes.astype(float) ** p) - xi ** p) < 1e-13


def test_dense_output_endpoints():
    cw = [l for l in open(os.path.join(GOLD, "rk44_tableau.txt")) if l.startswith("c ")][0].split()[1:]
    c = [int(cw[2 * i]) / int(cw[2 * i + 1]) for i in range(4)]
    for j in range(4):
        assert O.dense_rk4(j, 0, 0.0) == 0.0
        assert abs(O.dense_rk4(j, 0, 1.0) - c[j]) < 1e-15
    # b'(0) = (1, 0, 0, 0): the interpolant starts with slope k1
    assert [O.dense_rk4(j, 1, 0.0) for j in range(4)] == [1.0, 0.0, 0.0, 0.0]


def _rk4_stages(lam, u0, dt):
    k1 = dt * lam * u0
    k2 = dt * lam * (u0 + k1 / 2)
    k3 = dt * lam * (u0 + k2 / 2)
    k4 = dt * lam * (u0 + k3)
    return [k1, k2, k3, k4], [u0, u0 + k1 / 2, u0 + k2 / 2, u0 + k3]


@pytest.mark.parametrize("lam", [-1.3, 0.7])
def test_bor_ratio1_reproduces_coarse_stages(lam):
    """With R = 1 the fine grid steps with the coarse step, so its BOR stage
    states must be the coarse RK4 stage states themselves."""
    u0 = np.array([0.8, -0.3, 1.7])
    dt = 0.2
    k, stages = _rk4_stages(lam, u0, dt)
    for s in range(1, 5):
        got = O.bor_rk4(1, 0, s, dt, u0, k)
        assert np.allclose(got, stages[s - 1], rtol=0, atol=1e-15)


@pytest.mark.parametrize("R", [2, 3])
def test_bor_fine_stages_are_consistent(R):
    """For u' = lam u, the fine stage states of step r approximate the exact
    RK4 stages started from the exact solution at t^{n+r/R}, with error
    O(dt^4) (ratio between two dt's about 16)."""
    lam, u0 = -1.1, np.array([1.0])
    errs = []
    for dt in (0.2, 0.1):
        k, _ = _rk4_stages(lam, u0, dt)
        e = 0.0
        for r in range(R):
            ur = u0 * np.exp(lam * dt * r / R)
            _, ref = _rk4_stages(lam, ur, dt / R)
            for s in range(1, 5):
                e = max(e, abs(O.bor_rk4(R, r, s, dt, u0, k)[0] - ref[s - 1][0]))
        errs.append(e)
    assert 3.5 < np.log2(errs[0] / errs[1]) < 5.0


def _fmr_wave_run(N_unit, R, T=2.5, L=6.0, width=0.25, mode=O.TIME_BOR, window=None, scheme=O.RK4):
    """1D wave (Sec. IV.A set-up, shortened): periodic x in [-2, -2 + L), pulse
    at x = 0, one refined level over [1, 2] with ratio R, RK4 with the given
    time refinement (BOR by default).  Returns the L1 error at T, or with
    window = (t0, t1) the largest reflection integral Q = int_{-2}^{-1} |phi|
    dx over steps in that time window."""
    N0 = int(L * N_unit)
    dx0 = 1.0 / N_unit
    lo_c, hi_c = int(3 * N_unit), int(4 * N_unit)
    levels = [(1, [((0, 0, 0), (N0 - 1, 0, 0))]),
              (R, [((R * lo_c, 0, 0), (R * hi_c, R - 1, R - 1))])]
    H = O.Hierarchy(O.WAVE, (N0, 1, 1), (-2.0, 0.0, 0.0), dx0, levels)
    H.set_time_mode(mode)
    H.set_scheme(scheme)

    def exact(x, t):
        g = lambda s: np.exp(-(s ** 2) / width ** 2)
        return sum(0.5 * (g(x - t + m * L) + g(x + t + m * L)) for m in (-1, 0, 1))

    x0 = -2.0 + np.arange(N0) * dx0
    H.set(0, 0, synth.embed(np.stack([exact(x0, 0.0), 0 * x0])[:, None, None, :]))
    xf = -2.0 + (R * lo_c + np.arange(R * (hi_c - lo_c) + 1)) * dx0 / R
    f0 = np.broadcast_to(exact(xf, 0.0), (R, R, xf.size))
    H.set(1, 0, synth.embed(np.stack([f0, 0 * f0])))
    dt0 = 0.25 * dx0
    prm = O.params(sigma=0.1)
    if window is not None:
        inside, q, t = (x0 >= -2.0) & (x0 <= -1.0), 0.0, 0.0
        while t < window[1] - 1e-12:
            H.step(dt0, prm)
            t += dt0
            if t >= window[0]:
                q = max(q, np.sum(np.abs(synth.interior(H.get(0, 0))[0, 0, 0][inside])) * dx0)
        return q
    nsteps = int(round(T / dt0))
    for _ in range(nsteps):
        H.step(dt0, prm)
    got = synth.interior(H.get(0, 0))[0, 0, 0]
    return np.sum(np.abs(got - exact(x0, T))) * dx0


@pytest.mark.parametrize("R", [2, 3])
def test_fmr_wave_bor_converges_order4(R):
    errs = [_fmr_wave_run(n, R, width=0.3) for n in (12, 24, 48)]
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert 3.5 < orders[-1] < 4.8, (errs, orders)


@pytest.mark.parametrize("mode,lo,hi", [(O.TIME_BO, 3.5, 4.8), (O.TIME_NOSUB, 3.5, 4.8), (O.TIME_BO1, 0.7, 1.6)])
def test_fmr_wave_time_refinement_orders(mode, lo, hi):
    """Sec. III.B / IV.A: without sub-cycling and with Berger-Oliger using the
    dense output the global error converges at 4th order; the linear
    Berger-Oliger (BO1) only at 1st order."""
    errs = [_fmr_wave_run(n, 2, width=0.3, mode=mode) for n in (12, 24, 48)]
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert lo < orders[-1] < hi, (errs, orders)


@pytest.mark.parametrize("mode,lo,hi", [(O.TIME_BOR, 3.5, 5.5), (O.TIME_BO1, 0.7, 1.6)])
def test_fmr_wave_reflections(mode, lo, hi):
    """The reflection integral Q over [-2, -1] while only the reflection of
    the pulse entering the refined region crosses it (domain length 10, the
    exact Q is below 1e-11 there): BOR reflections vanish at 4th order, BO1
    ones at 1st order (Sec. IV.A)."""
    qs = [_fmr_wave_run(n, 2, L=10.0, width=0.25, mode=mode, window=(3.2, 4.2)) for n in (12, 24, 48)]
    orders = np.log2(np.array(qs[:-1]) / np.array(qs[1:]))
    assert lo < orders[-1] < hi, (qs, orders)


def test_fmr_wave_bo_reflections_first_order():
    """Berger-Oliger with the dense output: at the paper's resolutions
    (coarse dx = 1/80 and 1/160; pulse width 0.25 here, which makes BOR's
    advantage show already at 1/80) the reflection integral Q falls only at
    1st order, although the global error converges at 4th order, and BOR
    reflections are several times smaller (Sec. IV.A, reflection figure)."""
    qs = [_fmr_wave_run(n, 2, L=10.0, width=0.25, mode=O.TIME_BO, window=(3.2, 4.2)) for n in (80, 160)]
    order = np.log2(qs[0] / qs[1])
    assert 0.6 < order < 1.5, (qs, order)
    q_bor = _fmr_wave_run(80, 2, L=10.0, width=0.25, mode=O.TIME_BOR, window=(3.2, 4.2))
    assert q_bor < qs[0] / 3, (q_bor, qs[0])


def test_time_refinement_states_reduce_to_known_values():
    """At the start of a parent step every strategy gives U^n for stage 1 of
    fine step 0; without sub-cycling the states are the parent's RK4 stages;
    BO1 at theta = 1 and BO at theta = 1 are U^{n+1}."""
    rng = np.random.default_rng(0)
    Un = rng.standard_normal(7)
    k = [rng.standard_normal(7) for _ in range(4)]
    un1 = Un + (k[0] + 2 * k[1] + 2 * k[2] + k[3]) / 6
    for mode in (O.TIME_BOR, O.TIME_BO, O.TIME_BO1, O.TIME_NOSUB):
        assert np.array_equal(O.time_state(mode, 2, 0, 1, 0.1, Un, k), Un)
    for s, ref in ((2, Un + 0.5 * k[0]), (3, Un + 0.5 * k[1]), (4, Un + k[2])):
        assert np.allclose(O.time_state(O.TIME_NOSUB, 1, 0, s, 0.1, Un, k), ref, rtol=0, atol=1e-15)
    # fine step r = R - 1, stage 4 sits at theta = 1
    for mode in (O.TIME_BO, O.TIME_BO1):
        assert np.allclose(O.time_state(mode, 3, 2, 4, 0.1, Un, k), un1, rtol=0, atol=1e-14)


def test_restriction_is_injection_and_fill_same_is_copy():
    rng = np.random.default_rng(2)
    N0 = (8, 8, 8)
    levels = [(1, [((0, 0, 0), (3, 7, 7)), ((4, 0, 0), (7, 7, 7))]),
              (3, [((6, 6, 6), (11, 14, 8)), ((12, 6, 6), (17, 14, 8))])]
    H = O.Hierarchy(O.WAVE, N0, (0, 0, 0), 0.125, levels)
    arrays = {}
    for l, (_, boxes) in enumerate(levels):
        for p in range(len(boxes)):
            a = rng.standard_normal(H.shape(l, p))
            arrays[(l, p)] = a
            H.set(l, p, a)
    H.restrict(1)
    H.fill_same(0)
    c0 = H.get(0, 0)
    f0 = arrays[(1, 0)]
    # coarse (2,2,2) = fine (6,6,6) -> local (3,3,3) in fine patch 0
    assert np.array_equal(c0[:, 3 + 2, 3 + 2, 3 + 2], f0[:, 3, 3, 3])
    # untouched coarse point keeps its value
    assert np.array_equal(c0[:, 3 + 0, 3 + 0, 3 + 0], arrays[(0, 0)][:, 3, 3, 3])
    # ghost of coarse patch 0 at x = 4 is patch 1's interior x = 4 (restricted value
    # only where fine covers it)
    c1 = H.get(0, 1)
    assert np.array_equal(c0[:, 3 + 5, 3 + 5, 3 + 4], c1[:, 3 + 5, 3 + 5, 3 + 0])
    # periodic ghost: x = -1 of patch 0 is x = 7 of patch 1
    assert np.array_equal(c0[:, 3 + 1, 3 + 1, 2], c1[:, 3 + 1, 3 + 1, 3 + 3])



def _ssp3_stages(lam, u0, dt):
    k1 = dt * lam * u0
    k2 = dt * lam * (u0 + k1)
    k3 = dt * lam * (u0 + 0.25 * k1 + 0.25 * k2)
    return [k1, k2, k3], [u0, u0 + k1, u0 + 0.25 * k1 + 0.25 * k2]


def test_ssp3_dense_output_end_values():
    """App. C: b(0) = 0 and b(1) = the SSP-RK3 weights (1, 1, 4)/6."""
    for j, w in enumerate((1 / 6, 1 / 6, 4 / 6)):
        assert O.dense_ssp3(j, 0, 0.0) == 0.0
        assert abs(O.dense_ssp3(j, 0, 1.0) - w) < 1e-16


@pytest.mark.parametrize("R", [2, 3])
def test_bor_ssp3_fine_stages_are_consistent(R):
    """App. D for SSP-RK3: for u' = lam u the fine stage states of step r
    approximate the SSP-RK3 stages started from the exact solution at
    t^{n+r/R} with error O(dt^3) (the dense output is of 2nd order)."""
    lam, u0 = -1.1, np.array([1.0])
    errs = []
    for dt in (0.1, 0.05):
        k, _ = _ssp3_stages(lam, u0, dt)
        e = 0.0
        for r in range(R):
            ur = u0 * np.exp(lam * dt * r / R)
            _, ref = _ssp3_stages(lam, ur, dt / R)
            for st in range(1, 4):
                got = O.time_state(O.TIME_BOR, R, r, st, dt, u0, k, scheme=O.SSPRK3)
                e = max(e, abs(got[0] - ref[st - 1][0]))
        errs.append(e)
    assert 2.6 < np.log2(errs[0] / errs[1]) < 3.6, errs


def test_ssp3_time_states_reduce_to_known_values():
    """SSP-RK3: every strategy gives U^n at fine step 0, stage 1; without
    sub-cycling the states are the parent's stage states; BO and BO1 at
    theta = 1 (last fine step, stage 2 at c = 1) give U^{n+1}."""
    rng = np.random.default_rng(3)
    Un = rng.standard_normal(7)
    k = [rng.standard_normal(7) for _ in range(3)]
    un1 = Un + (k[0] + k[1] + 4 * k[2]) / 6
    for mode in (O.TIME_BOR, O.TIME_BO, O.TIME_BO1, O.TIME_NOSUB):
        assert np.array_equal(O.time_state(mode, 2, 0, 1, 0.1, Un, k, scheme=O.SSPRK3), Un)
    for st, ref in ((2, Un + k[0]), (3, Un + 0.25 * k[0] + 0.25 * k[1])):
        got = O.time_state(O.TIME_NOSUB, 1, 0, st, 0.1, Un, k, scheme=O.SSPRK3)
        assert np.allclose(got, ref, rtol=0, atol=1e-15)
    for mode in (O.TIME_BO, O.TIME_BO1):
        got = O.time_state(mode, 3, 2, 2, 0.1, Un, k, scheme=O.SSPRK3)
        assert np.allclose(got, un1, rtol=0, atol=1e-14)


def test_fmr_wave_ssp3_bor_converges_order3():
    """The FMR wave with SSP-RK3 and BOR (App. D): the global error falls at
    3rd order (the integrator's), with BO1 at 1st."""
    errs = [_fmr_wave_run(n, 2, width=0.3, scheme=O.SSPRK3) for n in (12, 24, 48)]
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert 2.6 < orders[-1] < 4.2, (errs, orders)
    errs = [_fmr_wave_run(n, 2, width=0.3, scheme=O.SSPRK3, mode=O.TIME_BO1) for n in (12, 24, 48)]
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert 0.7 < orders[-1] < 1.6, (errs, orders)
