"""Adaptive mesh refinement on the library: the AMR wave experiment of Sec. IV.A.

A 1D pulse (Gaussian of width 0.173 at rest at x = 0) on a periodic channel
x in [-2, 8) (one point thick in y and z on level 0) splits into two halves
that travel in opposite directions.  One refined level of ratio R follows
them: every `regrid_dt` time units the level-0 state is tagged where
|phi| >= threshold (`mol_tag`), the tags are grown by `buffer` (a length) and
clustered into boxes (`mol_cluster`), a patchset with the new fine boxes is
built, and the state moves over (`mol_regrid_*`: copies where the old fine
level held a point, quintic Lagrange interpolation from level 0 elsewhere).
Between regrids the hierarchy advances with the sub-cycled driver under the
chosen time refinement (MOL_TIME_*).

Defaults: tags grown by 0.1 and a regrid every 0.0125 time units (two
coarse steps at dx0 = 1/40), both fixed in physical units so that the refined
region follows the pulse in the same way at every resolution.

Fine boxes: a level-0 box [a, b] becomes the fine box [R a, R b] per axis, or
[R a, R N - 1] when b is the last level-0 point N - 1, so that a region that
reaches the periodic edge is refined up to the edge.
"""
from __future__ import annotations

import numpy as np

from . import molamr as M
from . import synth


def fine_boxes(coarse_boxes, R: int, dims) -> list:
    out = []
    for lo, hi in coarse_boxes:
        flo = tuple(R * lo[d] for d in range(3))
        fhi = tuple(R * hi[d] + (R - 1 if hi[d] == dims[d] - 1 else 0) for d in range(3))
        out.append((flo, fhi))
    return out


class AmrChannelRun:
    """Device state and driver of one AMR channel run."""

    def __init__(self, n_unit: int, R: int = 2, L: float = 10.0, width: float = 0.173, threshold: float = 1e-3,
                 buffer: float = 0.1, regrid_dt: float = 0.0125, sigma: float = 0.1):
        import torch
        self.n_unit, self.R, self.L, self.width = n_unit, R, L, width
        self.dx0 = 1.0 / n_unit
        self.N0 = (int(round(L * n_unit)), 1, 1)
        self.xlo = (-2.0, 0.0, 0.0)
        self.threshold = threshold
        self.buffer_pts = int(round(buffer * n_unit))
        self.regrid_dt = regrid_dt
        self.system = M.System(M.MOL_WAVE, sigma=sigma)
        self.level0 = [((0, 0, 0), (self.N0[0] - 1, 0, 0))]
        self.flags = torch.zeros(self.N0[::-1], dtype=torch.uint8, device="cuda")
        # initial hierarchy: tag the exact data on level 0 alone
        ps0 = M.Patchset(self._hier([]), self.system)
        U0 = ps0.alloc(0)
        U0.copy_(torch.from_numpy(ps0.pack(0, [self._exact(0, b) for b in self.level0])))
        boxes = self._boxes(ps0, U0)
        self.ps = M.Patchset(self._hier(boxes), self.system)
        self.states = self.ps.alloc_states()
        for l in range(2):
            self.states[l]["U"].copy_(torch.from_numpy(
                self.ps.pack(l, [self._exact(l, b) for b in self.ps.hier.levels[l][1]])))
        self.t = 0.0
        self.history = [(0.0, boxes)]
        self.regrids = 0

    def _hier(self, boxes):
        levels = [(1, self.level0)]
        if boxes:
            levels.append((self.R, boxes))
        return M.Hierarchy(self.N0, self.xlo, self.dx0, levels)

    def _exact(self, l: int, box):
        lo, hi = box
        h = self.dx0 / (self.R if l else 1)
        n = tuple(hi[d] - lo[d] + 1 for d in range(3))
        x = self.xlo[0] + (lo[0] + np.arange(n[0])) * h
        phi = np.broadcast_to(synth.wave_channel_pulse(x, 0.0, self.L, self.width), (n[2], n[1], n[0]))
        return synth.embed(np.stack([phi, np.zeros_like(phi)]))

    def _boxes(self, ps, U0):
        self.flags.zero_()
        ps.tag(0, U0, 0, self.threshold, self.flags)
        coarse = M.cluster(self.flags.cpu().numpy(), self.buffer_pts)
        if not coarse:
            raise RuntimeError("nothing is tagged: the refined level would be empty")
        return fine_boxes(coarse, self.R, self.N0)

    def regrid(self) -> bool:
        """Re-tag level 0 and move to the new fine boxes; False when they
        are unchanged."""
        boxes = self._boxes(self.ps, self.states[0]["U"])
        if boxes == self.ps.hier.levels[1][1]:
            return False
        ps = M.Patchset(self._hier(boxes), self.system, prev=self.ps)  # level 0 taken over
        states = ps.alloc_states()
        M.Regrid(ps, self.ps).apply([s["U"] for s in self.states], [s["U"] for s in states])
        self.ps, self.states = ps, states
        self.history.append((self.t, boxes))
        self.regrids += 1
        return True

    def dt0(self, tmode: int, courant: float = 0.25) -> float:
        return courant * self.dx0 / (self.R if tmode == M.MOL_TIME_NOSUB else 1)

    def run(self, t_end: float, tmode: int = M.MOL_TIME_BOR, courant: float = 0.25, checkpoints=()):
        """Advance to t_end, regridding every regrid_dt; returns the level-0
        phi (interior, x only) at each checkpoint time."""
        import torch
        dt0 = self.dt0(tmode, courant)
        every = max(int(round(self.regrid_dt / dt0)), 1)
        nsteps = int(round((t_end - self.t) / dt0))
        marks = {int(round((t - self.t) / dt0)): t for t in checkpoints}
        out = {}
        for s in range(1, nsteps + 1):
            self.ps.advance(self.states, dt0, M.MOL_BATCHED | tmode)
            self.t += dt0
            if s in marks:
                out[marks[s]] = self.phi0()
            if s % every == 0 and s < nsteps:
                self.regrid()
        torch.cuda.synchronize()
        return out

    def phi0(self) -> np.ndarray:
        return self.ps.unpack(0, self.states[0]["U"])[0][0, 3, 3, 3:-3].copy()

    def level_state(self, l: int):
        return self.ps.unpack(l, self.states[l]["U"])


def convergence_order(phis, r: int = 2) -> float:
    """n_c = log_r(||U_0 - U_1||_1 / ||U_1 - U_2||_1) over the points of the
    coarsest grid (Sec. IV); phis: level-0 values of three runs at
    resolutions dx, dx/r, dx/r^2 (vertex centred, so point i of the coarsest
    grid is point r i and r^2 i of the others)."""
    a, b, c = phis
    b, c = b[::r], c[::r * r]
    return float(np.log(np.abs(a - b).sum() / np.abs(b - c).sum()) / np.log(r))
