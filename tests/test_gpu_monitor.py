"""GPU parity of the constraint and dissipation monitors (mol_monitor)
against the oracle's: element by element at every interior point (the
pointwise output) and the deterministic reductions, on ragged multi-tile
patches, the 96^3 benchmark patch, a multi-patch level and the wave."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1806_04182_amd import molamr as M
from paper_1806_04182_amd import synth
from tests.test_gpu_amr import _setup

pytestmark = pytest.mark.gpu

TOL = 1e-12


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    return torch


def _run(ps, level, U, which):
    torch = _torch()
    out = torch.zeros(M.MOL_MON_OUT, dtype=torch.float64, device="cuda")
    point = ps.alloc(level)
    point.fill_(np.nan)
    ps.monitor(level, U, which, out, pointwise=point)
    torch.cuda.synchronize()
    return out.cpu().numpy(), ps.unpack(level, point)


def _compare(got_pts, got_red, ref_pts, which, dV, ref_nonfinite=0):
    """got_pts: (nf, ...) ghosted array of one patch; ref_pts: dict of the
    oracle's interior arrays.  Element-wise per monitor, then reductions."""
    rank = 0
    for q, name in enumerate(M.MONITORS):
        if not (which >> q) & 1:
            assert np.all(got_red[3 * q:3 * q + 3] == 0.0)
            continue
        g = got_pts[rank][3:-3, 3:-3, 3:-3]
        o = ref_pts[name]
        e = np.max(np.abs(g - o)) / max(np.max(np.abs(o)), 1.0)
        assert e <= TOL, (name, e)
        rank += 1
    assert got_red[-1] == ref_nonfinite


def _reductions_match(got_red, ref_pts, which, dV):
    for q, name in enumerate(M.MONITORS):
        if not (which >> q) & 1:
            continue
        v = np.concatenate([a.ravel() for a in ref_pts[name]])
        ref = (np.sum(np.abs(v)) * dV, np.sum(v * v) * dV, np.max(np.abs(v)))
        for s in range(3):
            assert abs(got_red[3 * q + s] - ref[s]) <= 1e-11 * max(abs(ref[s]), 1e-300) + 1e-300, (name, s)


@pytest.mark.parametrize("kind,n", [("strong", (19, 13, 9)), ("noise", (96, 96, 96)), ("strong", (33, 5, 17))])
def test_ccz4_monitors_match_oracle(kind, n):
    torch = _torch()
    print("monitor ccz4", kind, n, flush=True)
    dx = 2.0 / max(n)
    if kind == "noise":
        st = synth.ccz4_minkowski_noise(n, amp=1e-10, seed=0)
    else:
        st = synth.ccz4_lapse_pulse(n, (-1, -1, -1), dx, amp=0.2, width=0.4)
        st = st + synth.ccz4_minkowski_noise(n, amp=1e-2, seed=2) - synth.CCZ4_FLAT[:, None, None, None]
    U0 = synth.embed(st)
    O.fill_periodic(U0)
    ps = M.Patchset(M.single_patch(n, (-1, -1, -1), dx), M.System(M.MOL_CCZ4, sigma=0.1))
    U = torch.from_numpy(ps.pack(0, [U0])).cuda()
    ref = O.monitor(O.CCZ4, U0, dx, O.params(sigma=0.1))
    for which in (M.MOL_MON_ALL, M.MOL_MON_HZ | M.MOL_MON_TRA):
        red, pts = _run(ps, 0, U, which)
        _compare(pts[0], red, ref, which, dx ** 3)
        _reductions_match(red, {k: [v] for k, v in ref.items()}, which, dx ** 3)


def test_monitors_on_a_multipatch_level():
    """Level 1 of the three-level test hierarchy (ragged patches whose ghosts
    come from neighbours and from prolongation): every patch element-wise,
    and the level reduction against the oracle's values over all patches."""
    torch = _torch()
    ps, H, data, levels, dx0 = _setup(O.CCZ4)
    l = 1
    h = dx0 / levels[1][0]
    for ll, arrs in enumerate(data):
        for p, a in enumerate(arrs):
            H.set(ll, p, a)
    H.fill_same(l)
    arrs = [H.get(l, p) for p in range(len(levels[l][1]))]
    U = torch.from_numpy(ps.pack(l, arrs)).cuda()
    # ghosts of the level exactly as the oracle holds them (same-level copies;
    # the coarse-fine ghosts are whatever the data put there, on both sides)
    red, pts = _run(ps, l, U, M.MOL_MON_ALL)
    refs = [O.monitor(O.CCZ4, a, h, O.params(sigma=0.1)) for a in arrs]
    for p, ref in enumerate(refs):
        _compare(pts[p], red, ref, M.MOL_MON_ALL, h ** 3)
    _reductions_match(red, {k: [r[k] for r in refs] for k in M.MONITORS}, M.MOL_MON_ALL, h ** 3)


def test_wave_ko_monitor_and_errors():
    torch = _torch()
    n = (21, 10, 7)
    dx = 0.1
    rng = np.random.default_rng(3)
    U0 = synth.embed(rng.standard_normal((2,) + tuple(reversed(n))))
    O.fill_periodic(U0)
    ps = M.Patchset(M.single_patch(n, (0, 0, 0), dx), M.System(M.MOL_WAVE, sigma=0.3))
    U = torch.from_numpy(ps.pack(0, [U0])).cuda()
    red, pts = _run(ps, 0, U, M.MOL_MON_KO)
    ref = O.monitor(O.WAVE, U0, dx, O.params(sigma=0.3))
    _compare(pts[0], red, ref, M.MOL_MON_KO, dx ** 3)
    _reductions_match(red, {k: [v] for k, v in ref.items()}, M.MOL_MON_KO, dx ** 3)
    out = torch.zeros(M.MOL_MON_OUT, dtype=torch.float64, device="cuda")
    with pytest.raises(M.MolError, match="only MOL_MON_KO"):
        ps.monitor(0, U, M.MOL_MON_HZ, out)
    with pytest.raises(M.MolError, match="empty or unknown"):
        ps.monitor(0, U, 0, out)
    with pytest.raises(M.MolError, match="empty or unknown"):
        ps.monitor(0, U, 1 << 6, out)


def test_monitor_counts_non_finite_values():
    torch = _torch()
    n = (12, 9, 8)
    dx = 0.2
    st = synth.ccz4_minkowski_noise(n, amp=1e-3, seed=4)
    st[3, 2, 4, 5] = np.nan
    st[20, 7, 8, 11] = np.inf
    U0 = synth.embed(st)
    O.fill_periodic(U0)
    ps = M.Patchset(M.single_patch(n, (0, 0, 0), dx), M.System(M.MOL_CCZ4))
    U = torch.from_numpy(ps.pack(0, [U0])).cuda()
    red, _ = _run(ps, 0, U, M.MOL_MON_ALL)
    ref = O.monitor_norms(O.CCZ4, U0, dx)
    assert red[-1] == ref["nonfinite"] == 2
    # the sums leave out the non-finite monitor values, on both sides
    for q, name in enumerate(M.MONITORS):
        for s in range(3):
            assert abs(red[3 * q + s] - ref[name][s]) <= 1e-11 * max(abs(ref[name][s]), 1e-300) + 1e-300, (name, s)
