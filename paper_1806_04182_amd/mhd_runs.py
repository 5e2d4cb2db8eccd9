"""The MHD tests of Sec. IV.B on the library's driver (RK4, BOR sub-cycling):

- the circularly polarised Alfven wave in 2D (periodic [0, 2]^2, alpha = pi/4,
  dt = dx/(4 sqrt 2), three crossing times), unigrid or with FMR (ratio 2/2:
  levels over [0.5, 1.5]^2 and [0.75, 1.25]^2; ratio 4: one level over
  [0.5, 1.5]^2); the relative L1 error of B_x on the coarse level against the
  initial data, to which the wave returns after three crossing times;
- the Brio-Wu shock tube (Gamma = 2, t = 0.2) on the periodic line [0, 4)
  with the mirror jump at x = 2.5 (its waves stay in x > 1), B_y on [0, 1] of
  the coarse level, unigrid (dt = 0.2 dx, the paper's step) or with FMR
  (ratio 2/2 over [0.34, 0.66] and [0.4, 0.6]; ratio 4 over [0.4, 0.6]) with
  dt = 0.15 dx on the coarse level (and the same Courant factor on every
  level): at 0.2 the sub-cycled coarse-fine interfaces are past their
  stability limit for this tube, and WENO3 with RK4, or WENO5-Z with SSP-RK3
  and BOR, develop a negative pressure one fine cell inside the finest
  level's boundary when the compound wave reaches it (t ~ 0.05).
"""
from __future__ import annotations

import numpy as np

from . import molamr as M
from . import synth

ALFVEN_L = 2.0
BW_L = 4.0
BW_CFL = 0.2       # unigrid Brio-Wu: dt = 0.2 dx (Sec. IV.B.3)
BW_CFL_FMR = 0.15  # with FMR: the interfaces' stability limit is below 0.2 (module notes)


def _run(levels, N0, dx0, system, init, dt0, nsteps, ssp3=False):
    """Build the patchset, set every patch from init(n, h, lo), run nsteps
    coarse steps (RK4 from a captured graph, or SSP-RK3 with BOR for SSP-RK3);
    return the patchset and states."""
    import torch
    ps = M.Patchset(M.Hierarchy(N0, (0.0, 0.0, 0.0), dx0, levels), system)
    st = ps.alloc_states()
    h = dx0
    for l, (R, boxes) in enumerate(levels):
        if l:
            h /= R
        arrs = []
        for lo, hi in boxes:
            n = tuple(hi[d] - lo[d] + 1 for d in range(3))
            arrs.append(synth.embed(init(n, h, lo)))
        st[l]["U"].copy_(torch.from_numpy(ps.pack(l, arrs)))
    if ssp3:
        for _ in range(nsteps):
            ps.advance(st, dt0, M.MOL_BATCHED | M.MOL_ADV_SSPRK3)
    else:
        g = ps.graph_create(st, dt0)
        for _ in range(nsteps):
            g.launch()
        del g
    torch.cuda.synchronize()
    return ps, st


def alfven_levels(N, fmr=None):
    """Level list of the Alfven box with N coarse points per axis (N % 8 == 0)."""
    levels = [(1, [((0, 0, 0), (N - 1, N - 1, 0))])]
    if fmr == "2/2":
        a, b = N // 4, 3 * N // 4
        levels.append((2, [((2 * a, 2 * a, 0), (2 * b, 2 * b, 1))]))
        a, b = 3 * N // 8, 5 * N // 8
        levels.append((2, [((4 * a, 4 * a, 0), (4 * b, 4 * b, 3))]))
    elif fmr == "4":
        a, b = N // 4, 3 * N // 4
        levels.append((4, [((4 * a, 4 * a, 0), (4 * b, 4 * b, 3))]))
    return levels


def alfven_error(N, recon=M.MOL_RECON_WENO5Z, flux=M.MOL_FLUX_LLF, fmr=None, crossings=3, state=False):
    """Relative L1 error of B_x on the coarse level after `crossings`
    crossing times (t_CT = L / cos alpha)."""
    dx0 = ALFVEN_L / N
    dt0 = dx0 / (4.0 * np.sqrt(2.0))
    T = crossings * ALFVEN_L * np.sqrt(2.0)
    nsteps = int(round(T / dt0))
    sysd = M.System(M.MOL_MHD, sigma=0.0, gamma_ad=5.0 / 3.0, mhd_recon=recon, mhd_flux=flux)
    init = lambda n, h, lo: synth.mhd_cp_alfven(n, h, lo, ALFVEN_L)
    ps, st = _run(alfven_levels(N, fmr), (N, N, 1), dx0, sysd, init, dt0, nsteps)
    got = synth.interior(ps.unpack(0, st[0]["U"])[0])
    ex = synth.mhd_cp_alfven((N, N, 1), dx0, (0, 0, 0), ALFVEN_L)
    err = float(np.sum(np.abs(got[5] - ex[5])) / np.sum(np.abs(ex[5])))
    return (err, got) if state else err


def brio_wu_levels(N, fmr=None):
    """Level list of the Brio-Wu line with N coarse points per unit length
    (N % 50 == 0)."""
    levels = [(1, [((0, 0, 0), (int(BW_L * N) - 1, 0, 0))])]
    ix = lambda x, f: int(round(x * N * f))
    if fmr == "2/2":
        levels.append((2, [((ix(0.34, 2), 0, 0), (ix(0.66, 2), 1, 1))]))
        levels.append((2, [((ix(0.4, 4), 0, 0), (ix(0.6, 4), 3, 3))]))
    elif fmr == "4":
        levels.append((4, [((ix(0.4, 4), 0, 0), (ix(0.6, 4), 3, 3))]))
    return levels


def brio_wu(N, recon=M.MOL_RECON_WENO5Z, flux=M.MOL_FLUX_LLF, fmr=None, t_end=0.2, ssp3=False, cfl=None):
    """Coarse-level state on [0, 1] (8 conserved fields x N + 1 points) at
    t_end; dt = cfl dx (default BW_CFL unigrid, BW_CFL_FMR with FMR)."""
    dx0 = 1.0 / N
    dt0 = (cfl if cfl is not None else (BW_CFL_FMR if fmr else BW_CFL)) * dx0
    nsteps = int(round(t_end / dt0))
    sysd = M.System(M.MOL_MHD, sigma=0.0, gamma_ad=2.0, mhd_recon=recon, mhd_flux=flux)
    init = lambda n, h, lo: synth.mhd_brio_wu(n, h, lo)
    ps, st = _run(brio_wu_levels(N, fmr), (int(BW_L * N), 1, 1), dx0, sysd, init, dt0, nsteps, ssp3)
    got = synth.interior(ps.unpack(0, st[0]["U"])[0])[:, 0, 0, :]
    return got[:, : N + 1]


def brio_wu_error(U, ref, Nref):
    """Relative L1 error of B_y of a coarse run against a finer reference
    sampled at the coincident points."""
    N = U.shape[1] - 1
    r = ref[6, :: Nref // N][: N + 1]
    return float(np.sum(np.abs(U[6] - r)) / np.sum(np.abs(r)))
