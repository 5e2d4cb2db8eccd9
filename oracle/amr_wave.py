"""Oracle driver of the AMR wave experiment (Sec. IV.A, Sec. III.A).

TEST INFRASTRUCTURE ONLY.  A periodic channel of N0 level-0 points (one point
thick in y and z) with refined levels of ratio R that follow the solution:
every `every` coarse steps each level l but the finest is tagged where
|phi| >= thresholds[l] on its interior, the tags are grown and clustered
(oracle.tag, oracle.cluster) in level-l index space, each box [a, b] is
refined as [R a, R b] per axis ([R a, R N - 1] when b = N - 1, so a region that
reaches the periodic edge is refined up to it) and, above level 1, clipped to
the new parent boxes shrunk by six parent points; the state moves to the new
hierarchy with orc_hier_regrid.  Between regrids the oracle's sub-cycled step
advances it.  With one threshold this is the paper's single refined level.

Initial data come from the caller: init(level, (lo, hi), h) -> ghosted array.
"""
from __future__ import annotations

import numpy as np

from . import oracle as O


def refine(coarse_boxes, R: int, dims) -> list:
    boxes = []
    for lo, hi in coarse_boxes:
        f_lo = tuple(R * a for a in lo)
        f_hi = tuple(R * b + (R - 1 if b == n - 1 else 0) for b, n in zip(hi, dims))
        boxes.append((f_lo, f_hi))
    return boxes


def inside_parent(boxes, parent_boxes, R: int, dims, margin: int = 6) -> list:
    """Clip new level-(l+1) boxes to the parent level's boxes, each shrunk by
    `margin` parent points on the axes it does not span whole (so that the
    6-point prolongation stencils of the new level's ghosts stay on the parent
    level); dims is the parent level's extent."""
    out = []
    for plo, phi in parent_boxes:
        lim = []
        for d in range(3):
            whole = plo[d] == 0 and phi[d] == dims[d] - 1
            lim.append((0, R * dims[d] - 1) if whole else (R * (plo[d] + margin), R * (phi[d] - margin)))
        for blo, bhi in boxes:
            lo = tuple(max(blo[d], lim[d][0]) for d in range(3))
            hi = tuple(min(bhi[d], lim[d][1]) for d in range(3))
            if all(lo[d] <= hi[d] for d in range(3)):
                out.append((lo, hi))
    out.sort(key=lambda b: (b[0][2], b[0][1], b[0][0]))
    return out


class AmrChannel:
    """thresholds[l]: criterion on level l for level l+1 (default: the one
    `threshold`); buffer_pts: growth of the tags in level-0 points (times
    R^l on level l)."""

    def __init__(self, N0, xlo, dx0: float, R: int, threshold: float, buffer_pts: int, init, tmode: int = 0,
                 prm: O.Params | None = None, thresholds=None):
        self.N0, self.xlo, self.dx0, self.R = tuple(N0), tuple(xlo), dx0, R
        self.thresholds = tuple(thresholds) if thresholds is not None else (threshold,)
        self.buffer_pts, self.tmode = buffer_pts, tmode
        self.prm = prm or O.params()
        self.nlev = len(self.thresholds) + 1
        self.level0 = [((0, 0, 0), (self.N0[0] - 1, self.N0[1] - 1, self.N0[2] - 1))]
        self.init = init
        boxes = []
        for l in range(self.nlev - 1):
            H = self._hier(boxes)
            self._set_exact(H)
            boxes = boxes + [self._boxes(H, l, boxes[-1] if boxes else None)]
        self.H = self._hier(boxes)
        self._set_exact(self.H)
        self.boxes = boxes
        self.history = [(0.0, boxes)]
        self.t = 0.0

    def _set_exact(self, H):
        for l, (_, bl) in enumerate(H.levels):
            for p, b in enumerate(bl):
                H.set(l, p, self.init(l, b, self.dx0 / self.R ** l))

    def _hier(self, boxes):
        H = O.Hierarchy(O.WAVE, self.N0, self.xlo, self.dx0, [(1, self.level0)] + [(self.R, b) for b in boxes])
        H.set_time_mode(self.tmode)
        return H

    def _boxes(self, H, l: int, parent):
        """level-(l+1) boxes from the tags of H's level l"""
        dims = tuple(n * self.R ** l for n in self.N0)
        flags = np.zeros(dims[::-1], np.uint8)
        for p, (lo, hi) in enumerate(H.levels[l][1]):
            phi = H.get(l, p)[0, 3:-3, 3:-3, 3:-3]
            flags[lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1] = O.tag(phi, self.thresholds[l])
        coarse = O.cluster(flags, self.buffer_pts * self.R ** l)
        boxes = refine(coarse, self.R, dims)
        if l > 0:
            boxes = inside_parent(boxes, parent, self.R, dims)
        assert boxes, "nothing tagged"
        return boxes

    def regrid(self) -> None:
        new = []
        for l in range(self.nlev - 1):
            new.append(self._boxes(self.H, l, new[-1] if new else None))
        if new == self.boxes:
            return
        Hn = self._hier(new)
        Hn.regrid_from(self.H)
        self.H, self.boxes = Hn, new
        self.history.append((self.t, new))

    def run(self, dt0: float, nsteps: int, every: int) -> None:
        for s in range(1, nsteps + 1):
            self.H.step(dt0, self.prm)
            self.t += dt0
            if s % every == 0 and s < nsteps:
                self.regrid()

    def level(self, l: int):
        return [self.H.get(l, p) for p in range(len(self.H.levels[l][1]))]
