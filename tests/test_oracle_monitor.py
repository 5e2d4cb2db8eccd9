"""Pins of the oracle's constraint and dissipation monitors (Sec. V: Theta,
Z^i = chi (Ghat^i - Gt^i)/2, the Theta-equation bracket H_Z, the conformal
constraints ln det gt and tr At; Sec. II.B.1: the KO term) against exact
solutions, the covariant Z4 equation and the KO Fourier symbol."""
import numpy as np

from oracle import oracle as O
from paper_1806_04182_amd import synth
from tests.test_oracle_ccz4 import _gauge_wave, _lapse_pulse_2d
from tests.test_oracle_ccz4_terms import (AT, CHI, GH, GT, KH, SYM, TH, Smooth, dspec, grad_spec, grid, inv3,
                                          to_state, unit_det_metric)


def _mon(st, h, prm=None):
    U = synth.embed(np.ascontiguousarray(st))
    O.fill_periodic(U)
    return O.monitor(O.CCZ4, U, h, prm)


def test_monitors_vanish_at_order4_on_the_gauge_wave():
    """The gauge wave is an exact vacuum solution with Theta = Z = 0: H_Z (the
    Hamiltonian constraint there) and |Z| are truncation errors that fall at
    4th order; ln det gt and tr At are zero to rounding (the data are
    conformally unimodular and traceless)."""
    errs = []
    for N in (24, 48, 96):
        m = _mon(_gauge_wave(N, 0.0), 2.0 / N)
        errs.append([np.max(np.abs(m["hz"])), np.max(m["z"])])
        assert np.max(np.abs(m["lndet"])) < 1e-14 and np.max(np.abs(m["tra"])) < 1e-14
        assert np.all(m["theta"] == 0.0)
    o = np.log2(np.array(errs[1]) / np.array(errs[2]))
    assert np.all((o > 3.6) & (o < 4.6)), (errs, o)


def test_hz_is_the_ricci_scalar_plus_twice_div_z():
    """On a time-symmetric slice (At = 0, trKhat = -2 Theta, so trK = 0) of an
    arbitrary conformal metric with Z^i != 0, H_Z = R + 2 D_i Z^i exactly in
    the continuum (the quadratic K terms cancel): the oracle's value converges
    at 4th order to the spectral Ricci scalar of gamma = gt / chi plus twice
    the covariant divergence of Z; |Z| converges to sqrt(gamma_ij Z^i Z^j) of
    the Z^i put into Ghat."""
    errs = []
    for N in (24, 48):
        rng = np.random.default_rng(8)
        gtf = unit_det_metric(rng, 0.08)
        chis, ths = Smooth(rng, 0.15), Smooth(rng, 0.1)
        Zs = [Smooth(rng, 0.05) for _ in range(3)]
        X = grid(N)
        gt = gtf(X)
        gti = inv3(gt)
        chi = np.exp(chis(X))
        Th = ths(X)
        Zu = np.array([z(X) for z in Zs])
        Gt = -np.array([sum(dspec(gti[i, j], j) for j in range(3)) for i in range(3)])
        g, gi = gt / chi, gti * chi
        dg = np.moveaxis(np.array([grad_spec(g[i, j]) for i in range(3) for j in range(3)]).reshape(
            3, 3, 3, *chi.shape), 2, 0)
        Gam = 0.5 * np.einsum("kl...,ilj...->kij...", gi, dg + np.einsum("jli...->ilj...", dg)
                              - np.einsum("lij...->ilj...", dg))
        dGam = np.array([[[grad_spec(Gam[k, i, j]) for j in range(3)] for i in range(3)] for k in range(3)])
        Ric = (np.einsum("kijk...->ij...", dGam) - np.einsum("kikj...->ij...", dGam)
               + np.einsum("kkm...,mij...->ij...", Gam, Gam) - np.einsum("kjm...,mik...->ij...", Gam, Gam))
        # D_i Z^i = d_i Z^i + Gamma^i_ik Z^k
        divZ = sum(dspec(Zu[i], i) for i in range(3)) + np.einsum("iik...,k...->...", Gam, Zu)
        hz = np.einsum("ij...,ij...->...", gi, Ric) + 2 * divZ
        zn = np.sqrt(np.einsum("ij...,i...,j...->...", g, Zu, Zu))
        fields = {CHI: chi, KH: -2 * Th, TH: Th}
        for q, (i, j) in enumerate(SYM):
            fields[GT + q] = gt[i, j]
        for i in range(3):
            fields[GH + i] = Gt[i] + 2 * Zu[i] / chi
        m = _mon(to_state(fields), 2.0 / N)
        T = lambda a: a.transpose(2, 1, 0)
        errs.append([np.max(np.abs(m["hz"] - T(hz))) / np.max(np.abs(hz)),
                     np.max(np.abs(m["z"] - T(zn))) / np.max(zn)])
        assert np.max(np.abs(m["theta"] - T(Th))) == 0.0
        assert np.max(np.abs(m["lndet"])) < 1e-14 and np.max(np.abs(m["tra"])) == 0.0
    o = np.log2(np.array(errs[0]) / np.array(errs[1]))
    assert np.all((o > 3.5) & (o < 5.5)), (errs, o)


def test_conformal_constraint_monitors_are_the_definitions():
    """ln det gt and tr At on arbitrary data (not on the constraint surface):
    numpy's determinant and the trace with numpy's inverse."""
    N = 8
    rng = np.random.default_rng(2)
    X = grid(N)
    gt = unit_det_metric(rng, 0.1)(X) * np.exp(0.05 * Smooth(rng, 1.0)(X))
    At = np.array([[Smooth(rng, 0.1)(X) for _ in range(3)] for _ in range(3)])
    At = 0.5 * (At + np.einsum("ij...->ji...", At))
    fields = {}
    for q, (i, j) in enumerate(SYM):
        fields[GT + q] = gt[i, j]
        fields[AT + q] = At[i, j]
    m = _mon(to_state(fields), 2.0 / N)
    det = np.linalg.det(np.moveaxis(gt, (0, 1), (-2, -1)))
    tra = np.einsum("ij...,ij...->...", inv3(gt), At)
    T = lambda a: a.transpose(2, 1, 0)
    assert np.max(np.abs(m["lndet"] - T(np.log(det)))) < 1e-14
    assert np.max(np.abs(m["tra"] - T(tra))) < 1e-14


def test_ko_monitor_is_the_fourier_symbol():
    """Single Fourier modes per field: the KO term of field f is exactly
    -(sigma/h) sum_d sin^6(theta_d/2) times the mode; the monitor is the
    root of the sum of their squares over the fields (CCZ4 and the wave)."""
    N, sig = 12, 0.2
    h = 2.0 / N
    X = grid(N)
    rng = np.random.default_rng(1)
    for system, nf, base in ((O.CCZ4, 25, synth.CCZ4_FLAT), (O.WAVE, 2, np.zeros(2))):
        st = np.zeros((nf, N, N, N))
        ref = np.zeros((N, N, N))
        for f in range(nf):
            k = rng.integers(-3, 4, 3)
            mode = 1e-3 * np.cos(np.pi * (k[0] * X[0] + k[1] * X[1] + k[2] * X[2]) + rng.uniform(0, 6))
            st[f] = (base[f] + mode).transpose(2, 1, 0)
            sym = -(sig / h) * sum(np.sin(np.pi * k[d] * h / 2) ** 6 for d in range(3))
            ref += (sym * mode.transpose(2, 1, 0)) ** 2
        U = synth.embed(st)
        O.fill_periodic(U)
        ko = O.monitor(system, U, h, O.params(sigma=sig))["ko"]
        # the modes ride on O(1) backgrounds: rounding of the stored values is 1e-16 absolute
        assert np.max(np.abs(ko - np.sqrt(ref))) < 1e-12 * np.max(np.sqrt(ref))


def test_lapse_pulse_monitors_converge_order4():
    """A pure-gauge evolution (lapse pulse on flat space): Theta, |Z|, H_Z,
    ln det gt and tr At are zero in the continuum and self-converge to zero at
    4th order (RK4 and the Sec. II.B.1 stencils; dissipation is 5th order)."""
    T = 0.5
    norms = []
    for N in (32, 64):
        dx = 2.0 / N
        U = synth.embed(_lapse_pulse_2d(N))
        nsteps = int(round(T / (0.25 * dx)))
        O.rk_run(O.CCZ4, O.RK4, U, (dx, dx, dx), T / nsteps, nsteps, O.params())
        n = O.monitor_norms(O.CCZ4, U, dx)
        assert n["nonfinite"] == 0
        # L2 norms over the 2D slice (one point thick in z)
        norms.append(np.array([np.sqrt(n[k][1] / dx) for k in ("theta", "z", "hz", "lndet", "tra")]))
    order = np.log2(norms[0] / norms[1])
    assert np.all(norms[1] > 0)
    assert np.all((order > 3.5) & (order < 5.2)), order


def test_monitor_norms_count_non_finite_values():
    n = (5, 4, 3)
    st = synth.ccz4_minkowski_noise(n, amp=1e-3, seed=1)
    st[3, 1, 2, 3] = np.nan
    st[20, 0, 0, 0] = np.inf
    U = synth.embed(st)
    O.fill_periodic(U)
    assert O.monitor_norms(O.CCZ4, U, 0.2)["nonfinite"] == 2
