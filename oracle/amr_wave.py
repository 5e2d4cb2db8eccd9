"""Oracle driver of the AMR wave experiment (Sec. IV.A, Sec. III.A).

TEST INFRASTRUCTURE ONLY.  A periodic channel of N0 level-0 points (one point
thick in y and z) with one refined level of ratio R that follows the solution:
every `every` coarse steps the level-0 interior phi is tagged where
|phi| >= threshold, the tags are grown and clustered (oracle.tag,
oracle.cluster), each level-0 box [a, b] is refined as [R a, R b] per axis
([R a, R N - 1] when b = N - 1, so a region that reaches the periodic edge is
refined up to it), and the state moves to the new hierarchy with
orc_hier_regrid.  Between regrids the oracle's sub-cycled step advances it.

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


class AmrChannel:
    def __init__(self, N0, xlo, dx0: float, R: int, threshold: float, buffer_pts: int, init, tmode: int = 0,
                 prm: O.Params | None = None):
        self.N0, self.xlo, self.dx0, self.R = tuple(N0), tuple(xlo), dx0, R
        self.threshold, self.buffer_pts, self.tmode = threshold, buffer_pts, tmode
        self.prm = prm or O.params()
        self.level0 = [((0, 0, 0), (self.N0[0] - 1, self.N0[1] - 1, self.N0[2] - 1))]
        u0 = init(0, self.level0[0], dx0)
        boxes = self._boxes(u0)
        self.H = self._hier(boxes)
        self.H.set(0, 0, u0)
        for p, b in enumerate(boxes):
            self.H.set(1, p, init(1, b, dx0 / R))
        self.boxes = boxes
        self.history = [(0.0, boxes)]
        self.t = 0.0

    def _hier(self, boxes):
        H = O.Hierarchy(O.WAVE, self.N0, self.xlo, self.dx0, [(1, self.level0), (self.R, boxes)])
        H.set_time_mode(self.tmode)
        return H

    def _boxes(self, u0):
        phi = u0[0, 3:-3, 3:-3, 3:-3]
        coarse = O.cluster(O.tag(phi, self.threshold), self.buffer_pts)
        assert coarse, "nothing tagged"
        return refine(coarse, self.R, self.N0)

    def regrid(self) -> None:
        boxes = self._boxes(self.H.get(0, 0))
        if boxes == self.boxes:
            return
        Hn = self._hier(boxes)
        Hn.regrid_from(self.H)
        self.H, self.boxes = Hn, boxes
        self.history.append((self.t, boxes))

    def run(self, dt0: float, nsteps: int, every: int) -> None:
        for s in range(1, nsteps + 1):
            self.H.step(dt0, self.prm)
            self.t += dt0
            if s % every == 0 and s < nsteps:
                self.regrid()

    def level(self, l: int):
        return [self.H.get(l, p) for p in range(len(self.H.levels[l][1]))]
