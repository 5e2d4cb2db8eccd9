"""Pins of the oracle's CCZ4 right-hand side (Sec. V) against exact solutions
of the Einstein equations that the discrete system must approach at 4th order."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1806_04182_amd import synth

CHI, GT, KH, AT, GH, TH, ALP, BETA, BB = 0, 1, 7, 8, 14, 17, 18, 19, 22
SYM = [(0, 0), (0, 1), (0, 2), (1, 1), (1, 2), (2, 2)]


def test_minkowski_rhs_is_exactly_zero():
    U = synth.embed(np.broadcast_to(synth.CCZ4_FLAT[:, None, None, None], (25, 5, 6, 7)).copy())
    O.fill_periodic(U)
    for up in (0.0, 1.0):
        R = O.rhs(O.CCZ4, U, (0.1, 0.2, 0.15), O.params(upwind=up))
        assert np.all(synth.interior(R) == 0.0)


def _gauge_wave(N, t, A=0.05):
    """Flat metric -H dt^2 + H dx^2 + dy^2 + dz^2, H = 1 + A sin(pi (x - t)):
    alpha = sqrt(H), beta = 0, gamma_xx = H, K_xx = H'/(2 sqrt H); harmonic
    slicing d_t alpha = -alpha^2 K holds.  Conformal variables:
    chi = H^(-1/3), gt = diag(H^(2/3), H^(-1/3), H^(-1/3)), At = chi (K_ij - gamma_ij K/3),
    Ghat^x = Gt^x = -d_x gt^{xx} = (2/3) H^(-5/3) H'."""
    x = -1.0 + 2.0 * np.arange(N) / N
    u = x - t
    H = 1 + A * np.sin(np.pi * u)
    Hp = A * np.pi * np.cos(np.pi * u)
    chi = H ** (-1 / 3)
    Kxx = Hp / (2 * np.sqrt(H))
    K = Kxx / H
    out = np.zeros((25, 1, 1, N))
    out[CHI] = chi
    out[GT + 0] = H ** (2 / 3)
    out[GT + 3] = H ** (-1 / 3)
    out[GT + 5] = H ** (-1 / 3)
    out[KH] = K
    out[AT + 0] = chi * (Kxx - H * K / 3)
    out[AT + 3] = chi * (-K / 3)
    out[AT + 5] = chi * (-K / 3)
    out[GH] = 2 / 3 * H ** (-5 / 3) * Hp
    out[ALP] = np.sqrt(H)
    return out


def test_gauge_wave_order4():
    prm = O.params(bm_f0=1.0, bm_f1=0.0, gd_g=0.0, gd_eta=2.0, sigma=0.1)
    errs = []
    T = 0.5
    for N in (24, 48, 96):
        dx = 2.0 / N
        U = synth.embed(_gauge_wave(N, 0.0))
        nsteps = int(round(T / (0.25 * dx)))
        O.rk_run(O.CCZ4, O.RK4, U, (dx, dx, dx), T / nsteps, nsteps, prm)
        ex = _gauge_wave(N, T)
        got = synth.interior(U)
        e = 0.0
        for f in (CHI, GT, GT + 3, KH, AT, AT + 3, GH, ALP, TH):
            e += np.sum(np.abs(got[f] - ex[f])) / N
        errs.append(e)
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert 3.6 < orders[-1] < 4.6, (errs, orders)


# ---- flat space in curvilinear coordinates with a static lapse ----------

_A = np.array([[0.3, 0.5, -0.4], [0.2, -0.3, 0.6], [-0.5, 0.4, 0.25]])
_PH = np.array([[0.1, 0.7, -0.3], [0.4, -0.2, 0.9], [0.6, 0.3, -0.8]])
_EPS = 0.06


def _curvilinear(N):
    """X^a = x^a + eps S^a(x), S^a = sum_m A_am sin(pi x_m + ph_am); gamma_ij =
    sum_a J^a_i J^a_j; alpha = 1 + 0.1 sin(pi x + .3) sin(pi y - .2) cos(pi z).
    Returns the CCZ4 state (K = At = Theta = beta = B = 0) and the exact
    right-hand side, nonzero only for trKhat = -gamma^ij D_i D_j alpha and
    At_ij = -chi [D_i D_j alpha]^TF."""
    x1 = -1.0 + 2.0 * np.arange(N) / N
    X = np.meshgrid(x1, x1, x1, indexing="ij")  # X[m][i, j, k] = coordinate m at (x_i, y_j, z_k)
    sh = X[0].shape
    J = np.zeros((3, 3) + sh)
    dJ = np.zeros((3, 3, 3) + sh)  # dJ[k, a, i] = d_k J^a_i (nonzero only for k == i)
    for a in range(3):
        for i in range(3):
            J[a, i] = (a == i) + _EPS * _A[a, i] * np.pi * np.cos(np.pi * X[i] + _PH[a, i])
            dJ[i, a, i] = -_EPS * _A[a, i] * np.pi ** 2 * np.sin(np.pi * X[i] + _PH[a, i])
    g = np.einsum("ai...,aj...->ij...", J, J)
    dg = np.einsum("kai...,aj...->kij...", dJ, J) + np.einsum("ai...,kaj...->kij...", J, dJ)
    gm = np.moveaxis(g, (0, 1), (-2, -1))
    gi = np.moveaxis(np.linalg.inv(gm), (-2, -1), (0, 1))
    det = np.linalg.det(gm)
    chi = det ** (-1 / 3)
    dchi = -chi / 3 * np.einsum("ij...,kij...->k...", gi, dg)
    gt = chi * g
    dgt = dchi[:, None, None] * g[None] + chi * dg
    gti = gi / chi
    Gl = 0.5 * (np.einsum("jik...->ijk...", dgt) + np.einsum("kij...->ijk...", dgt) - dgt)
    Gu = np.einsum("il...,ljk...->ijk...", gti, Gl)
    Gcon = np.einsum("jk...,ijk...->i...", gti, Gu)
    # lapse and its physical second covariant derivative
    s = [np.sin(np.pi * X[0] + 0.3), np.sin(np.pi * X[1] - 0.2), np.cos(np.pi * X[2])]
    ds = [np.pi * np.cos(np.pi * X[0] + 0.3), np.pi * np.cos(np.pi * X[1] - 0.2), -np.pi * np.sin(np.pi * X[2])]
    dds = [-np.pi ** 2 * s[0], -np.pi ** 2 * s[1], -np.pi ** 2 * s[2]]
    alp = 1 + 0.1 * s[0] * s[1] * s[2]
    dalp = np.zeros((3,) + sh)
    ddalp = np.zeros((3, 3) + sh)
    for k in range(3):
        f = [s[0], s[1], s[2]]
        f[k] = ds[k]
        dalp[k] = 0.1 * f[0] * f[1] * f[2]
        for l in range(3):
            f = [s[0], s[1], s[2]]
            if k == l:
                f[k] = dds[k]
            else:
                f[k] = ds[k]
                f[l] = ds[l]
            ddalp[k, l] = 0.1 * f[0] * f[1] * f[2]
    Gphys = 0.5 * np.einsum("kl...,ilj...->kij...", gi,
                            np.einsum("ilj...->ilj...", dg) + np.einsum("jli...->ilj...", dg)
                            - np.einsum("lij...->ilj...", dg))
    DDa = ddalp - np.einsum("kij...,k...->ij...", Gphys, dalp)
    lap = np.einsum("ij...,ij...->...", gi, DDa)
    st = np.zeros((25,) + sh)
    ex = np.zeros((25,) + sh)
    st[CHI] = chi
    for q, (i, j) in enumerate(SYM):
        st[GT + q] = gt[i, j]
        ex[AT + q] = -chi * (DDa[i, j] - g[i, j] * lap / 3)
    for i in range(3):
        st[GH + i] = Gcon[i]
    st[ALP] = alp
    ex[KH] = -lap
    # (i, j, k) meshgrid index -> (z, y, x) storage order
    return np.ascontiguousarray(st.transpose(0, 3, 2, 1)), np.ascontiguousarray(ex.transpose(0, 3, 2, 1))


def test_static_curvilinear_flat_space_order4():
    """Ricci of a flat metric in curvilinear coordinates vanishes; with K = 0
    and a static lapse, only trKhat and At evolve, by the lapse's covariant
    Hessian.  Pins Christoffels, Ricci, the conformal split, Z, D_i D_j alpha."""
    errs = []
    prm = O.params(sigma=0.1)
    for N in (12, 24, 48):
        st, ex = _curvilinear(N)
        U = synth.embed(st)
        O.fill_periodic(U)
        R = synth.interior(O.rhs(O.CCZ4, U, 2.0 / N, prm))
        errs.append(np.max(np.abs(R - ex)))
    orders = np.log2(np.array(errs[:-1]) / np.array(errs[1:]))
    assert orders[-1] > 3.5, (errs, orders)


def test_ccz4_axis_permutation():
    N = 10
    base = synth.ccz4_minkowski_noise((N, 1, 1), amp=1e-3, seed=2)
    # the same data laid along y
    U1 = synth.embed(base)
    U2 = synth.embed(np.ascontiguousarray(base.transpose(0, 1, 3, 2)))
    # rotate tensor components x->y, y->z, z->x for the y-run
    def rot_fields(a):
        out = a.copy()
        perm3 = {0: 1, 1: 2, 2: 0}
        for q, (i, j) in enumerate(SYM):
            ii, jj = sorted((perm3[i], perm3[j]))
            q2 = SYM.index((ii, jj))
            out[GT + q2] = a[GT + q]
            out[AT + q2] = a[AT + q]
        for base_ in (GH, BETA, BB):
            for i in range(3):
                out[base_ + perm3[i]] = a[base_ + i]
        return out
    U2 = rot_fields(U2)
    O.fill_periodic(U1)
    O.fill_periodic(U2)
    h = 2.0 / N
    R1 = O.rhs(O.CCZ4, U1, h)
    R1i = synth.interior(R1)[:, 0, 0, :]
    R2i = synth.interior(O.rhs(O.CCZ4, U2, h))[:, 0, :, 0]
    R1rot = rot_fields(R1i[:, None, None, :])[:, 0, 0, :]
    scale = np.max(np.abs(R1i))
    assert np.max(np.abs(R1rot - R2i)) < 1e-12 * scale


def _lapse_pulse_2d(N, A=0.1, w=0.5):
    """Flat space (gt = I, chi = 1, K = 0, Ghat = 0) with a smooth periodic
    lapse alpha = 1 + A exp(-(sin^2(pi x / 2) + sin^2(pi y / 2)) / w^2) on an
    N x N x 1 grid of [-1, 1)^2: pure gauge, so the constraints are zero in
    the continuum and the discrete violations are truncation errors."""
    x = -1.0 + 2.0 * np.arange(N) / N
    X, Y = np.meshgrid(x, x, indexing="xy")
    s = (np.sin(np.pi * X / 2) ** 2 + np.sin(np.pi * Y / 2) ** 2) / w ** 2
    out = np.empty((25, 1, N, N))
    out[:] = synth.CCZ4_FLAT[:, None, None, None]
    out[ALP, 0] = 1 + A * np.exp(-s)
    return out


def test_noisy_minkowski_stays_bounded():
    """Robust stability: Minkowski plus 1e-10 noise on every field.  The first
    steps amplify the grid-scale noise by a bounded factor (second differences
    of white noise, about 40x at 16^3, growing with the resolution); after
    that the deviation from flat space must not grow (no exponential mode),
    over 50 RK4 steps."""
    n = (16, 16, 16)
    dx = 2.0 / 16
    U = synth.embed(synth.ccz4_minkowski_noise(n, amp=1e-10, seed=3))
    flat = synth.CCZ4_FLAT[:, None, None, None]
    dev0 = np.max(np.abs(synth.interior(U) - flat))
    O.fill_periodic(U)
    hz0 = np.sqrt(O.monitor_norms(O.CCZ4, U, dx)["hz"][1])
    devs, hzs = [], []
    for _ in range(10):
        O.rk_run(O.CCZ4, O.RK4, U, (dx, dx, dx), 0.25 * dx, 5, O.params())
        devs.append(np.max(np.abs(synth.interior(U) - flat)))
        hzs.append(np.sqrt(O.monitor_norms(O.CCZ4, U, dx)["hz"][1]))
    assert max(devs) <= 1e4 * dev0, (dev0, devs)
    assert max(devs[5:]) <= max(devs[:5]), devs
    # the Hamiltonian-type constraint (L2 of H_Z) is damped, not amplified
    assert max(hzs) <= 10 * hz0 and max(hzs[5:]) <= max(hzs[:5]), (hz0, hzs)


def _nonflat_state(n, dx, seed):
    st = synth.ccz4_lapse_pulse(n, (-1, -1, -1), dx, amp=0.2, width=0.4)
    st = st + synth.ccz4_minkowski_noise(n, amp=1e-2, seed=seed) - synth.CCZ4_FLAT[:, None, None, None]
    U = synth.embed(st)
    O.fill_periodic(U)
    return U


def test_jvp_build_repeats_the_rhs_and_matches_central_differences():
    """The dual-number build of the oracle: its value part is the right-hand
    side bit for bit, and its derivative part is the limit of central
    difference quotients (error falling as eps^2)."""
    n, dx = (5, 4, 4), 0.15
    U = _nonflat_state(n, dx, 2)
    rng = np.random.default_rng(0)
    V = synth.embed(rng.standard_normal((25,) + tuple(reversed(n))))
    O.fill_periodic(V)
    R, RV = O.ccz4_rhs_jvp(U, V, dx)
    I = (slice(None), slice(3, -3), slice(3, -3), slice(3, -3))
    assert np.array_equal(R[I], O.rhs(O.CCZ4, U, dx)[I])
    errs = []
    for eps in (1e-5, 1e-6):
        fd = (O.rhs(O.CCZ4, U + eps * V, dx) - O.rhs(O.CCZ4, U - eps * V, dx)) / (2 * eps)
        errs.append(np.max(np.abs(fd[I] - RV[I])) / np.max(np.abs(RV[I])))
    assert errs[1] < 1e-9 and errs[1] < errs[0], errs
