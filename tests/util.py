"""Helpers shared by the tests (no method arithmetic here)."""
import numpy as np


def parity_err(got, ref):
    """Per-field e_f = max|G - O| / max(max|O|, 1) over the given arrays."""
    got = np.asarray(got)
    ref = np.asarray(ref)
    nf = ref.shape[0]
    return np.array([np.max(np.abs(got[f] - ref[f])) / max(np.max(np.abs(ref[f])), 1.0) for f in range(nf)])


def interior(a):
    return a[:, 3:-3, 3:-3, 3:-3]


def stencil_ghost_mask(n):
    """Ghost points that stencils read: faces to depth 3, edges to depth 2."""
    nx, ny, nz = n
    m = np.zeros((nz + 6, ny + 6, nx + 6), dtype=bool)
    for k in range(nz + 6):
        for j in range(ny + 6):
            for i in range(nx + 6):
                dep = []
                for a, nn in ((i - 3, nx), (j - 3, ny), (k - 3, nz)):
                    dep.append(-a if a < 0 else (a - nn + 1 if a >= nn else 0))
                nout = sum(d > 0 for d in dep)
                if nout == 1 or (nout == 2 and max(dep) <= 2):
                    m[k, j, i] = True
    return m
