"""Levels whose buffers exceed 2^31 doubles (64-bit offsets in every kernel
that indexes them): a CCZ4 level of two 448 x 448 x 224 patches (puncture
data from the device kernel, periodic ghost fill across the two patches) and
a wave patch of 1024^3.  The right-hand side at sampled points, among them
the last point of the buffer, is compared with the oracle evaluated on each
point's 7^3 neighbourhood read back from the device, and the ghost values
in those neighbourhoods with the interior values they are images of."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1806_04182_amd import molamr as M

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    return torch


def _flat(ps, p, nf, ix, iy, iz):
    """Flat level-buffer indices of fields 0..nf-1 at ghosted coordinates
    (ix, iy, iz) (arrays of equal shape) of patch p."""
    L = ps.layouts[0]
    nx, ny, nz = L["dims"][p]
    px, fs, off = L["pitches"][p], L["fstrides"][p], L["offsets"][p]
    pt = (iz.astype(np.int64) * (ny + 6) + iy) * px + ix
    return off + np.arange(nf, dtype=np.int64).reshape((nf,) + (1,) * pt.ndim) * fs + pt[None]


def _gather(buf, idx):
    torch = _torch()
    t = torch.from_numpy(idx.reshape(-1)).cuda()
    return buf.index_select(0, t).cpu().numpy().reshape(idx.shape)


def _owner(ps, g):
    """Patch and local interior coordinates of global interior point g."""
    for p, (lo, hi) in enumerate(ps.hier.levels[0][1]):
        if all(lo[d] <= g[d] <= hi[d] for d in range(3)):
            return p, tuple(g[d] - lo[d] for d in range(3))
    raise AssertionError(g)


def _check_points(ps, U, R, nf, dx, prm, system, pts):
    period = ps.period(0)
    for p, (i, j, k) in pts:
        print("max-size point", system, p, (i, j, k), flush=True)
        ax = np.arange(-3, 4)
        iz, iy, ix = np.meshgrid(k + 3 + ax, j + 3 + ax, i + 3 + ax, indexing="ij")
        sub = _gather(U, _flat(ps, p, nf, ix, iy, iz))
        # ghost entries of the neighbourhood equal the interior values they image
        lo = ps.hier.levels[0][1][p][0]
        n = ps.layouts[0]["dims"][p]
        for c in np.ndindex(7, 7, 7):
            loc = (i + c[2] - 3, j + c[1] - 3, k + c[0] - 3)
            if all(0 <= loc[d] < n[d] for d in range(3)):
                continue
            g = tuple((lo[d] + loc[d]) % period[d] for d in range(3))
            q, ql = _owner(ps, g)
            src = _gather(U, _flat(ps, q, nf, *[np.array([ql[d] + 3]) for d in range(3)]))[:, 0]
            assert np.array_equal(sub[:, c[0], c[1], c[2]], src), (p, (i, j, k), c)
        ref = O.rhs(system, np.ascontiguousarray(sub), dx, prm)[:, 3, 3, 3]
        got = _gather(R, _flat(ps, p, nf, *[np.array([v + 3]) for v in (i, j, k)]))[:, 0]
        err = np.abs(got - ref) / np.maximum(np.abs(ref), 1.0)
        assert np.all(err < TOL), ((p, i, j, k), err)


def test_ccz4_level_beyond_2_31_doubles():
    torch = _torch()
    N = 448
    dx = 2.0 / N
    boxes = [((0, 0, 0), (N - 1, N - 1, N // 2 - 1)), ((0, 0, N // 2), (N - 1, N - 1, N - 1))]
    ps = M.Patchset(M.Hierarchy((N, N, N), (-1.0, -1.0, -1.0), dx, [(1, boxes)]), M.System(M.MOL_CCZ4))
    assert ps.layouts[0]["nelems"] > 2 ** 31
    # two spinning, moving holes outside the box: smooth, non-trivial data
    holes = [(0.7, (2.6, 0.3, -0.2), (0.1, -0.05, 0.02), (0.05, 0.1, -0.2)),
             (0.4, (-0.4, -2.8, 0.5), (0.0, 0.1, 0.0), (0.0, 0.0, 0.1))]
    U = ps.alloc(0)
    ps.ccz4_puncture(0, holes, U)
    ps.fill_ghosts(0, U)
    R = ps.alloc(0)
    ps.rhs(0, U, R)
    torch.cuda.synchronize()
    rng = np.random.default_rng(5)
    h = N // 2
    pts = [(1, (N - 1, N - 1, h - 1)), (0, (0, 0, 0)), (1, (0, 0, 0)), (0, (N - 1, N - 1, h - 1)),
           (1, (N - 2, 1, h - 3))] + [(int(rng.integers(0, 2)), tuple(int(v) for v in rng.integers(0, [N, N, h])))
                                      for _ in range(5)]
    _check_points(ps, U, R, 25, dx, O.params(), O.CCZ4, pts)
    del U, R
    torch.cuda.empty_cache()


def test_wave_patch_beyond_2_31_doubles():
    torch = _torch()
    N = 1024
    dx = 2.0 / N
    ps = M.Patchset(M.single_patch((N, N, N), (-1.0, -1.0, -1.0), dx), M.System(M.MOL_WAVE, sigma=0.1))
    assert ps.layouts[0]["nelems"] > 2 ** 31
    U = ps.alloc(0)
    ps.wave_gaussian(0, [1.0, 0.3, 0.1, -0.2, 0.05], U)
    ps.fill_ghosts(0, U)
    R = ps.alloc(0)
    ps.rhs(0, U, R)
    torch.cuda.synchronize()
    rng = np.random.default_rng(6)
    pts = [(0, (N - 1, N - 1, N - 1)), (0, (0, 0, 0)), (0, (N - 1, 0, N - 2))] + \
          [(0, tuple(int(v) for v in rng.integers(0, N, 3))) for _ in range(5)]
    _check_points(ps, U, R, 2, dx, O.params(sigma=0.1), O.WAVE, pts)
    del U, R
    torch.cuda.empty_cache()
