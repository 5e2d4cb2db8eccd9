"""A single spinning black hole on the library's driver (Sec. V, single BH):
puncture data (Brill-Lindquist conformal factor, Bowen-York spin, lapse
psi^-2), CCZ4 with 1+log slicing (f = 2/alpha), Gamma-driver (g = 3/4,
eta = 2/M), KO dissipation, RK4 with BOR sub-cycling, nested levels of ratio 2
and radiative outer boundaries (v = 1, U_inf the flat values)."""
from __future__ import annotations

import numpy as np

from . import molamr as M
from . import synth  # noqa: F401  (flat values of the radiative boundary)


def nested_levels(nlev: int, N: int):
    """nlev levels of N points per axis, each covering half the width of its
    parent (ratio 2, centred); returns the level list."""
    levels = [(1, [((0, 0, 0), (N - 1,) * 3)])]
    for l in range(1, nlev):
        lo = (N // 2) * (2 ** l - 1)
        levels.append((2, [((lo,) * 3, (lo + N - 1,) * 3)]))
    return levels


class SingleBH:
    def __init__(self, nlev=5, N=32, L=16.0, mass=1.0, spin=0.2, sigma=0.1):
        import torch
        self.levels = nested_levels(nlev, N)
        self.dx0 = 2.0 * L / N
        hf = self.dx0 / 2 ** (nlev - 1)
        # index 0 at -L + hf/2 on every level: no grid point at the puncture
        self.xlo = (-L + 0.5 * hf,) * 3
        self.ps = M.Patchset(M.Hierarchy((N, N, N), self.xlo, self.dx0, self.levels, open=True),
                             M.System(M.MOL_CCZ4, sigma=sigma, gd_eta=2.0 / mass))
        self.ps.set_radiative([1.0] * 25, list(synth.CCZ4_FLAT))
        self.holes = [(mass, (0.0, 0.0, 0.0), (0.0, 0.0, 0.0), (0.0, 0.0, spin * mass * mass))]
        self.st = self.ps.alloc_states()
        for l in range(len(self.levels)):
            # data on the whole ghosted box: on level 0 the ghost shell is
            # evolved state (radiative boundary), not filled
            self.ps.ccz4_puncture(l, self.holes, self.st[l]["U"], whole=True)
        torch.cuda.synchronize()
        self.t = 0.0
        self.graph = self.ps.graph_create(self.st, 0.25 * self.dx0)

    def run(self, t_end):
        import torch
        dt0 = 0.25 * self.dx0
        n = int(round((t_end - self.t) / dt0))
        for _ in range(n):
            self.graph.launch()
        torch.cuda.synchronize()
        self.t += n * dt0

    def level(self, l):
        return synth.interior(self.ps.unpack(l, self.st[l]["U"])[0])

    def field_at(self, f, x):
        """Field f at the grid point nearest (x, 0, 0) on the finest level
        that holds it."""
        for l in range(len(self.levels) - 1, -1, -1):
            h = self.dx0 / 2 ** l
            lo = self.levels[l][1][0][0]
            i = int(round((x - self.xlo[0]) / h)) - lo[0]
            j = int(round((0.0 - self.xlo[1]) / h)) - lo[1]
            k = int(round((0.0 - self.xlo[2]) / h)) - lo[2]
            u = self.level(l)
            if 0 <= i < u.shape[3] and 0 <= j < u.shape[2] and 0 <= k < u.shape[1]:
                return float(u[f][k, j, i])
        raise ValueError("(x, 0, 0) outside every level")

    def summary(self):
        """Lapse and conformal factor at the finest level, and finiteness."""
        u = self.level(len(self.levels) - 1)
        c = [s // 2 for s in u.shape[1:]]
        return {"t": self.t, "finite": bool(all(np.isfinite(self.level(l)).all() for l in range(len(self.levels)))),
                "alpha_min": float(u[18].min()), "chi_min": float(u[0].min()),
                "alpha_centre": float(u[18][c[0], c[1], c[2]])}
