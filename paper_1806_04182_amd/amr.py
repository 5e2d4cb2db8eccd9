"""Adaptive mesh refinement on the library: the AMR wave experiment of Sec. IV.A.

A 1D pulse (Gaussian of width 0.173 at rest at x = 0) on a periodic channel
x in [-2, 8) (one point thick in y and z on level 0) splits into two halves
that travel in opposite directions.  Refined levels of ratio R follow them:
every `regrid_dt` time units each level l but the finest is tagged where
|phi| >= thresholds[l] (`mol_tag`), the tags are grown by `buffer` (a length)
and clustered into boxes (`mol_cluster`) for level l+1, which is kept inside
level l with room for the prolongation stencils; a patchset with the new
boxes is built (taking over the unchanged levels), and the state moves over
(`mol_regrid_*`: copies where the old level held a point, quintic Lagrange
interpolation from the new parent elsewhere).  The paper's experiment has one
refined level; more levels repeat the tagging on the new levels (Sec. III.A).
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


def nest(boxes, parent_boxes, R: int, dims, margin: int = 6) -> list:
    """The parts of `boxes` (level l+1 index space) that lie inside the parent
    level's boxes shrunk by `margin` parent points on every axis the parent box
    does not span whole (dims: the parent level's extent), so that the
    prolongation stencils of the new level's ghost points stay on the parent
    level."""
    out = []
    for plo, phi in parent_boxes:
        lo, hi = [], []
        for d in range(3):
            if plo[d] == 0 and phi[d] == dims[d] - 1:
                lo.append(0)
                hi.append(R * dims[d] - 1)
            else:
                lo.append(R * (plo[d] + margin))
                hi.append(R * (phi[d] - margin))
        for blo, bhi in boxes:
            c_lo = tuple(max(blo[d], lo[d]) for d in range(3))
            c_hi = tuple(min(bhi[d], hi[d]) for d in range(3))
            if all(c_lo[d] <= c_hi[d] for d in range(3)):
                out.append((c_lo, c_hi))
    return sorted(out, key=lambda b: (b[0][2], b[0][1], b[0][0]))


class AmrChannelRun:
    """Device state and driver of one AMR channel run with `len(thresholds)`
    adaptive levels: level l+1 refines where |phi| >= thresholds[l] on level
    l, nested inside level l."""

    def __init__(self, n_unit: int, R: int = 2, L: float = 10.0, width: float = 0.173, threshold: float = 1e-3,
                 buffer: float = 0.1, regrid_dt: float = 0.0125, sigma: float = 0.1, thresholds=None):
        import torch
        self.n_unit, self.R, self.L, self.width = n_unit, R, L, width
        self.dx0 = 1.0 / n_unit
        self.N0 = (int(round(L * n_unit)), 1, 1)
        self.xlo = (-2.0, 0.0, 0.0)
        self.thresholds = tuple(thresholds) if thresholds is not None else (threshold,)
        self.threshold = self.thresholds[0]
        self.buffer = buffer
        self.buffer_pts = int(round(buffer * n_unit))
        self.regrid_dt = regrid_dt
        self.system = M.System(M.MOL_WAVE, sigma=sigma)
        self.level0 = [((0, 0, 0), (self.N0[0] - 1, 0, 0))]
        self.nlev = len(self.thresholds) + 1
        # initial hierarchy, level by level: tag the exact data of the finest
        # level built so far
        boxes = []
        for l in range(self.nlev - 1):
            ps = M.Patchset(self._hier(boxes), self.system)
            U = ps.alloc(l)
            U.copy_(torch.from_numpy(ps.pack(l, [self._exact(l, b) for b in ps.hier.levels[l][1]])))
            boxes = boxes + [self._boxes(ps, l, U)]
        self.ps = M.Patchset(self._hier(boxes), self.system)
        self.states = self.ps.alloc_states()
        for l in range(self.nlev):
            self.states[l]["U"].copy_(torch.from_numpy(
                self.ps.pack(l, [self._exact(l, b) for b in self.ps.hier.levels[l][1]])))
        self.t = 0.0
        self.history = [(0.0, boxes)]
        self.regrids = 0

    def _hier(self, boxes):
        levels = [(1, self.level0)] + [(self.R, b) for b in boxes]
        return M.Hierarchy(self.N0, self.xlo, self.dx0, levels)

    def _h(self, l: int) -> float:
        return self.dx0 / self.R ** l

    def _period(self, l: int):
        return tuple(n * self.R ** l for n in self.N0)

    def _exact(self, l: int, box):
        lo, hi = box
        h = self._h(l)
        n = tuple(hi[d] - lo[d] + 1 for d in range(3))
        x = self.xlo[0] + (lo[0] + np.arange(n[0])) * h
        phi = np.broadcast_to(synth.wave_channel_pulse(x, 0.0, self.L, self.width), (n[2], n[1], n[0]))
        return synth.embed(np.stack([phi, np.zeros_like(phi)]))

    def _boxes(self, ps, l: int, U, parent_boxes=None):
        """Boxes of level l+1 from the tags of level l of `ps`."""
        import torch
        per = self._period(l)
        flags = torch.zeros(per[::-1], dtype=torch.uint8, device="cuda")
        ps.tag(l, U, 0, self.thresholds[l], flags)
        coarse = M.cluster(flags.cpu().numpy(), int(round(self.buffer / self._h(l))))
        boxes = fine_boxes(coarse, self.R, per)
        if l > 0:
            parent = parent_boxes if parent_boxes is not None else ps.hier.levels[l][1]
            boxes = nest(boxes, parent, self.R, per)
        if not boxes:
            raise RuntimeError(f"nothing is tagged on level {l}: level {l + 1} would be empty")
        return boxes

    def regrid(self) -> bool:
        """Re-tag every level but the finest (level l's tags on its current
        data give level l+1, nested in the new level l) and move to the new
        boxes; False when nothing changes."""
        new = []
        for l in range(self.nlev - 1):
            new.append(self._boxes(self.ps, l, self.states[l]["U"], new[-1] if l else None))
        if new == [self.ps.hier.levels[l][1] for l in range(1, self.nlev)]:
            return False
        ps = M.Patchset(self._hier(new), self.system, prev=self.ps)  # unchanged levels taken over
        states = ps.alloc_states()
        M.Regrid(ps, self.ps).apply([s["U"] for s in self.states], [s["U"] for s in states])
        self.ps, self.states = ps, states
        self.history.append((self.t, new))
        self.regrids += 1
        return True

    def dt0(self, tmode: int, courant: float = 0.25) -> float:
        return courant * (self._h(self.nlev - 1) if tmode == M.MOL_TIME_NOSUB else self.dx0)

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
