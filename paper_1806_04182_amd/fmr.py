"""The FMR wave experiment of Sec. IV.A on the library's sub-cycled driver.

A 1D pulse (Gaussian of width 0.173 at rest at x = 0) on a periodic channel
x in [-2, 8) (one point thick in y and z) crosses a refined region over
x in [1, 2].  The reflection integral
Q(t) = integral over [-2, -1] of |phi| dx is reduced on the device after every
coarse step (`mol_box_norms`), so the run measures the reflections that the
time-refinement strategy (MOL_TIME_*) leaves at the coarse-fine interfaces.

Hierarchies: one refined level with ratio R over [1, 2], or (ratios (2, 2))
a second level of ratio 2 nested over [1.25, 1.75].
"""
from __future__ import annotations

import numpy as np

from . import molamr as M
from . import synth


def channel_levels(n_unit: int, ratios=(2,), L: float = 10.0):
    """Levels of the channel: coarse dx = 1/n_unit over [-2, -2 + L); the
    first refined level covers [1, 2]; a further level covers [1.25, 1.75]."""
    N0 = int(round(L * n_unit))
    levels = [(1, [((0, 0, 0), (N0 - 1, 0, 0))])]
    # refined intervals, as coarse-level coordinates measured from x = -2
    spans = [(3.0, 4.0), (3.25, 3.75)]
    f = 1
    for d, R in enumerate(ratios):
        f *= R
        a, b = (int(round(s * n_unit * f)) for s in spans[d])
        levels.append((R, [((a, 0, 0), (b, f - 1, f - 1))]))
    return levels, (N0, 1, 1)


class ChannelRun:
    """Device state of one FMR channel run."""

    def __init__(self, n_unit: int, ratios=(2,), L: float = 10.0, width: float = 0.173, sigma: float = 0.1):
        import torch
        self.levels, self.N0 = channel_levels(n_unit, ratios, L)
        self.dx0 = 1.0 / n_unit
        self.L, self.width = L, width
        self.ps = M.Patchset(M.Hierarchy(self.N0, (-2.0, 0.0, 0.0), self.dx0, self.levels),
                             M.System(M.MOL_WAVE, sigma=sigma))
        self.states = self.ps.alloc_states()
        h = self.dx0
        for l, (R, boxes) in enumerate(self.levels):
            if l:
                h /= R
            arrs = []
            for lo, hi in boxes:
                n = tuple(hi[d] - lo[d] + 1 for d in range(3))
                x = -2.0 + (lo[0] + np.arange(n[0])) * h
                phi = np.broadcast_to(synth.wave_channel_pulse(x, 0.0, L, width), (n[2], n[1], n[0]))
                arrs.append(synth.embed(np.stack([phi, np.zeros_like(phi)])))
            self.states[l]["U"].copy_(torch.from_numpy(self.ps.pack(l, arrs)))
        self.t = 0.0

    def run(self, t_end: float, tmode: int = M.MOL_TIME_BOR, window=None, courant: float = 0.25):
        """Advance to t_end with dt0 = courant dx0 (courant dx_finest without
        sub-cycling).  With window = (t0, t1): returns the array of Q after
        every coarse step whose time lies in [t0, t1]."""
        import torch
        fine = self.dx0
        for R, _ in self.levels[1:]:
            fine /= R
        dt0 = courant * (fine if tmode == M.MOL_TIME_NOSUB else self.dx0)
        nsteps = int(round((t_end - self.t) / dt0))
        times = self.t + dt0 * np.arange(1, nsteps + 1)
        take = np.zeros(nsteps, bool) if window is None else (times >= window[0] - 1e-12) & (times <= window[1] + 1e-12)
        out = torch.zeros((max(int(take.sum()), 1), 5), dtype=torch.float64, device="cuda")
        q = 0
        for s in range(nsteps):
            self.ps.advance(self.states, dt0, M.MOL_BATCHED | tmode)
            if take[s]:
                self.ps.box_norms(0, self.states[0]["U"], 0, 0.0, (-2.0, -np.inf, -np.inf), (-1.0, np.inf, np.inf),
                                  out[q])
                q += 1
        self.t += nsteps * dt0
        torch.cuda.synchronize()
        # the channel is one point thick: the box sum is Q dx0^2
        return out[:q, 0].cpu().numpy() / self.dx0 ** 2

    def level_state(self, l: int):
        return self.ps.unpack(l, self.states[l]["U"])


def reflection_q(n_unit: int, tmode: int, ratios=(2,), window=(3.2, 4.2)) -> float:
    """Largest Q over the window in which only the reflection of the pulse
    entering the refined region crosses [-2, -1] (L = 10)."""
    run = ChannelRun(n_unit, ratios)
    return float(np.max(run.run(window[1], tmode, window)))
