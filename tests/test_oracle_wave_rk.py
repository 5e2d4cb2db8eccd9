"""Pins of the oracle's Runge-Kutta schemes (eq. eRK, Table RK44, App. D) and
of the periodic wave system (Sec. IV.A) against closed forms and a spectral
solution that shares no stencil code with the oracle."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1806_04182_amd import synth


@pytest.mark.parametrize("z", [-0.5, 0.3j, -1.0 + 0.5j, 0.2 - 2.0j])
def test_rk_amplification_polynomials(z):
    p4 = 1 + z + z ** 2 / 2 + z ** 3 / 6 + z ** 4 / 24
    p3 = 1 + z + z ** 2 / 2 + z ** 3 / 6
    assert abs(O.rk_scalar(O.RK4, z) - p4) < 1e-15 * max(1, abs(p4))
    assert abs(O.rk_scalar(O.SSPRK3, z) - p3) < 1e-15 * max(1, abs(p3))


def _spectral_wave(U0, h, dt, nsteps, sigma):
    """Exact solution of the discrete periodic system: every Fourier mode
    evolves by P4(dt M_k), M_k = [[q, -1], [-lam, q]], with lam the symbol of
    D_xx + D_yy + D_zz and q the symbol of the summed KO operator."""
    phi = np.fft.fftn(U0[0])
    pi = np.fft.fftn(U0[1])
    nz, ny, nx = U0[0].shape
    lam = 0
    q = 0
    for ax, (n, hd) in enumerate(zip((nz, ny, nx), (h[2], h[1], h[0]))):
        th = 2 * np.pi * np.fft.fftfreq(n)
        shape = [1, 1, 1]
        shape[ax] = n
        th = th.reshape(shape)
        lam = lam + (-2 * np.cos(2 * th) + 32 * np.cos(th) - 30) / (12 * hd * hd)
        q = q - (sigma / hd) * np.sin(th / 2) ** 6 * 64 / 64
    # P4(dt M) applied as a 2x2 matrix polynomial, elementwise per mode
    a11 = dt * q + 0 * lam
    a12 = -dt * np.ones_like(a11)
    a21 = -dt * lam + 0 * a11
    a22 = dt * q + 0 * lam

    def matmul(A, B):
        return (A[0] * B[0] + A[1] * B[2], A[0] * B[1] + A[1] * B[3],
                A[2] * B[0] + A[3] * B[2], A[2] * B[1] + A[3] * B[3])

    Z = (a11, a12, a21, a22)
    I = (np.ones_like(a11), np.zeros_like(a11), np.zeros_like(a11), np.ones_like(a11))
    P = I
    term = I
    for k in range(1, 5):
        term = matmul(term, Z)
        P = tuple(p + t / np.prod(range(1, k + 1)) for p, t in zip(P, term))
    for _ in range(nsteps):
        phi, pi = P[0] * phi + P[1] * pi, P[2] * phi + P[3] * pi
    return np.real(np.fft.ifftn(phi)), np.real(np.fft.ifftn(pi))


def test_wave_matches_spectral_solution():
    n = (16, 12, 10)
    dx = 2.0 / 16
    h = (dx, dx, dx)
    U0 = synth.wave_gaussian(n, (-1, -1, -1), dx, width=0.3, centre=(0.1, -0.05, 0.2),
                             period=(2.0, 12 * dx, 10 * dx))
    U0[1] = 0.3 * synth.uniform(5, 0, 1, *np.meshgrid(np.arange(16), np.arange(12),
                                                       np.arange(10), indexing="ij")).transpose(2, 1, 0)
    dt = 0.25 * dx
    U = synth.embed(U0)
    O.rk_run(O.WAVE, O.RK4, U, h, dt, 20, O.params(sigma=0.1))
    phi, pi = _spectral_wave(U0, h, dt, 20, 0.1)
    got = synth.interior(U)
    assert np.max(np.abs(got[0] - phi)) < 1e-13
    assert np.max(np.abs(got[1] - pi)) < 1e-13


def test_wave_plane_wave_order4():
    """phi = sin(pi (x + y + z) - w t), Pi = -d_t phi, w = pi sqrt(3)."""
    errs = []
    for N in (8, 16, 32):
        dx = 2.0 / N
        n = (N, N, N)
        z, y, x = synth.grid((0, 0, 0), n, dx)
        x = x - 1
        y = y - 1
        z = z - 1
        w = np.pi * np.sqrt(3)
        ph = lambda t: np.broadcast_to(np.sin(np.pi * (x + y + z) - w * t), (N, N, N))
        pi = lambda t: np.broadcast_to(w * np.cos(np.pi * (x + y + z) - w * t), (N, N, N))
        U = synth.embed(np.stack([ph(0.0), pi(0.0)]))
        T = 0.5
        nsteps = int(round(T / (0.25 * dx)))
        O.rk_run(O.WAVE, O.RK4, U, (dx,) * 3, T / nsteps, nsteps, O.params(sigma=0.1))
        e = np.sum(np.abs(synth.interior(U)[0] - ph(T))) * dx ** 3
        errs.append(e)
    orders = [np.log2(errs[i] / errs[i + 1]) for i in range(2)]
    assert 3.7 < orders[-1] < 4.6, orders


def test_periodic_fill_is_modular_copy():
    rng = np.random.default_rng(0)
    U = synth.embed(rng.standard_normal((2, 2, 5, 4)))
    O.fill_periodic(U)
    nf, NZ, NY, NX = U.shape
    for k in range(NZ):
        for j in range(NY):
            for i in range(NX):
                s = U[:, 3 + (k - 3) % 2, 3 + (j - 3) % 5, 3 + (i - 3) % 4]
                assert np.array_equal(U[:, k, j, i], s)
