"""Element-wise parity at the benchmark sizes, in the launch configurations
that bench.py times: the 96^3 CCZ4 patch (graph-replayed RK4 step), the
128^3 MHD patch (SSP-RK3, default and autotuned z-chunk), one coarse step of
the 200-patch three-level hierarchy (wave system, graph replay), the wave
adjoint at 64^3 over 200 steps, and the CCZ4 reverse RK4 step at 48^3.

The oracle runs single-threaded here: each case costs 5-40 s of host time."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1806_04182_amd import molamr as M
from paper_1806_04182_amd import synth
from tests.util import parity_err

pytestmark = pytest.mark.gpu

TOL = 1e-12
I = (slice(None), slice(3, -3), slice(3, -3), slice(3, -3))


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    return torch


@pytest.mark.parametrize("kind", ["noise", "strong"])
def test_ccz4_96_rk4_step_all_points(kind):
    """The headline workload: one RK4 step of the 96^3 periodic patch replayed
    from the captured graph (4 x (fill + stage)), all 25 fields at all
    points.  'noise' is the benchmark data (Minkowski + 1e-10 noise, seed 0);
    'strong' is a lapse pulse + 1e-2 noise, so every term is O(1)."""
    torch = _torch()
    n = (96, 96, 96)
    dx = 2.0 / 96
    dt = 0.25 * dx
    print("ccz4 96^3 graph step", kind, flush=True)
    if kind == "noise":
        st0 = synth.ccz4_minkowski_noise(n, amp=1e-10, seed=0)
    else:
        st0 = synth.ccz4_lapse_pulse(n, (-1, -1, -1), dx, amp=0.2, width=0.4)
        st0 = st0 + synth.ccz4_minkowski_noise(n, amp=1e-2, seed=1) - synth.CCZ4_FLAT[:, None, None, None]
    U0 = synth.embed(st0)
    ps = M.Patchset(M.single_patch(n, (-1, -1, -1), dx), M.System(M.MOL_CCZ4))
    st = ps.alloc_states()
    st[0]["U"].copy_(torch.from_numpy(ps.pack(0, [U0])))
    g = ps.graph_create(st, dt)
    g.launch()
    torch.cuda.synchronize()
    got = ps.unpack(0, st[0]["U"])[0]
    del g, st, ps
    ref = U0.copy()
    O.fill_periodic(ref)
    O.rk_run(O.CCZ4, O.RK4, ref, dx, dt, 1, O.params())
    e = parity_err(got[I], ref[I])
    print("ccz4 96^3 e_f max", e.max(), flush=True)
    assert np.all(e <= TOL), e


@pytest.mark.parametrize("zchunk", [None, 4])
def test_mhd_128_ssprk3_step_all_points(zchunk):
    """MHD 128^3 (the OT-like state, seed 1): one SSP-RK3 step, fill + fused
    stage per stage, with the default launch shape and with the z-chunk the
    autotuner picks at this size."""
    torch = _torch()
    n = (128, 128, 128)
    dx = 1.0 / 128
    dt = 0.2 * dx
    print("mhd 128^3 step zchunk", zchunk, flush=True)
    U0 = synth.embed(synth.mhd_ot_like(n, seed=1, N=n))
    ps = M.Patchset(M.single_patch(n, (0, 0, 0), dx), M.System(M.MOL_MHD, sigma=0.0))
    if zchunk is not None:
        ps.set_tiling(0, (15, 15, zchunk))
    U = torch.from_numpy(ps.pack(0, [U0])).cuda()
    S0, S1 = ps.alloc(0), ps.alloc(0)
    for s, (Us, Uo) in enumerate([(U, S0), (S0, S1), (S1, U)], start=1):
        ps.fill_ghosts(0, Us)
        ps.rk_stage(0, M.MOL_SSPRK3, s, dt, U, Us, None, Uo)
    torch.cuda.synchronize()
    got = ps.unpack(0, U)[0]
    del U, S0, S1, ps
    ref = U0.copy()
    O.fill_periodic(ref)
    O.rk_run(O.MHD, O.SSPRK3, ref, dx, dt, 1, O.params(sigma=0.0))
    e = parity_err(got[I], ref[I])
    print("mhd 128^3 e_f max", e.max(), flush=True)
    assert np.all(e <= TOL), e


def test_amr_200_patch_hierarchy_coarse_step():
    """The three-level, 200-patch hierarchy of the batched-AMR workload
    (ratios 2 and 3, interiors 16-48 points per axis, seeded compositions):
    one BOR sub-cycled coarse step of the wave system replayed from the
    captured graph, every patch of every level against the oracle."""
    torch = _torch()
    levels, N0, dx0 = synth.amr_three_levels(0)
    assert sum(len(b) for _, b in levels) == 200
    print("amr 200 patches: building", flush=True)
    data = []
    h = dx0
    for l, (R, boxes) in enumerate(levels):
        if l:
            h /= R
        arrs = []
        for lo, hi in boxes:
            nn = tuple(hi[d] - lo[d] + 1 for d in range(3))
            st = synth.wave_gaussian(nn, (-1, -1, -1), h, width=0.35, centre=(0.05, -0.02, 0.1), lo=lo)
            st[1] = 0.1 * synth.wave_gaussian(nn, (-1, -1, -1), h, width=0.5, lo=lo)[0]
            arrs.append(synth.embed(st))
        data.append(arrs)
    dt0 = 0.25 * dx0
    ps = M.Patchset(M.Hierarchy(N0, (-1, -1, -1), dx0, levels), M.System(M.MOL_WAVE, sigma=0.1))
    states = ps.alloc_states()
    for l, arrs in enumerate(data):
        states[l]["U"].copy_(torch.from_numpy(ps.pack(l, arrs)))
    for l in range(len(levels)):
        ps.fill_ghosts(l, states[l]["U"])
    g = ps.graph_create(states, dt0)
    g.launch()
    torch.cuda.synchronize()
    got = [ps.unpack(l, states[l]["U"]) for l in range(len(levels))]
    del g, states, ps
    print("amr 200 patches: oracle step", flush=True)
    H = O.Hierarchy(O.WAVE, N0, (-1, -1, -1), dx0, levels)
    for l, arrs in enumerate(data):
        for p, a in enumerate(arrs):
            H.set(l, p, a)
    for l in range(len(levels)):
        H.fill_same(l)
    H.step(dt0, O.params(sigma=0.1))
    worst = 0.0
    for l in range(len(levels)):
        for p in range(len(levels[l][1])):
            e = parity_err(got[l][p][I], H.get(l, p)[I])
            worst = max(worst, e.max())
            assert np.all(e <= TOL), (l, p, e)
    print("amr 200 patches e_f max", worst, flush=True)


def test_wave_adjoint_64_200_steps_matches_oracle():
    """The wave adjoint workload: dJ/dU_0 of J = sum_{|x|<0.6} phi dV after
    200 RK4 steps at 64^3 (the reverse sweep the autograd function runs),
    element by element against the oracle's reverse sweep."""
    torch = _torch()
    n = (64, 64, 64)
    dx = 2.0 / 64
    dt = 0.25 * dx
    xlo = (-1.0, -1.0, -1.0)
    ps = M.Patchset(M.single_patch(n, xlo, dx), M.System(M.MOL_WAVE, sigma=0.1))
    lam = ps.alloc(0)
    w = [ps.alloc(0) for _ in range(3)]
    ps.sphere_adjoint(0, 0, 0.6, 1.0, lam)
    for _ in range(200):
        ps.rk4_adjoint_step(0, dt, lam, w)
    torch.cuda.synchronize()
    got = ps.unpack(0, lam)[0]
    print("wave adjoint 64^3: oracle sweep", flush=True)
    ref = O.wave_adjoint_run(n, (dx, dx, dx), xlo, dt, 200, 0.6, O.params(sigma=0.1))
    sc = max(np.max(np.abs(ref)), 1e-300)
    err = np.max(np.abs(got[I] - ref[I])) / sc
    print("wave adjoint 64^3 rel err", err, flush=True)
    assert err <= TOL, err


def test_ccz4_48_reverse_step_dot_product_with_oracle_jvp():
    """The CCZ4 adjoint workload's reverse RK4 step at 48^3 (the kept-stage
    form the autograd function uses) on the lapse-pulse state with 1e-2
    noise: <lam', v> equals <lam, dU'/dU v>, the tangent built from the
    oracle's right-hand side and its exact JVP."""
    torch = _torch()
    n = (48, 48, 48)
    dx = 2.0 / 48
    dt = 0.25 * dx
    st0 = synth.ccz4_lapse_pulse(n, (-1, -1, -1), dx, amp=0.1, width=0.4)
    st0 = st0 + synth.ccz4_minkowski_noise(n, amp=1e-2, seed=9) - synth.CCZ4_FLAT[:, None, None, None]
    U = synth.embed(st0)
    O.fill_periodic(U)
    rng = np.random.default_rng(11)
    shape = (25,) + tuple(reversed(n))
    lam, v = rng.standard_normal(shape), rng.standard_normal(shape)
    print("ccz4 48^3 reverse step: oracle tangent", flush=True)
    V = synth.embed(v)
    O.fill_periodic(V)
    Us, Vs, tan = U.copy(), V.copy(), v.copy()
    for b, c in ((0.5, 1 / 6), (0.5, 1 / 3), (1.0, 1 / 3), (None, 1 / 6)):
        R, RV = O.ccz4_rhs_jvp(Us, Vs, dx)
        tan = tan + c * dt * RV[I]
        if b is None:
            break
        Us = U.copy()
        Us[I] = U[I] + b * dt * R[I]
        O.fill_periodic(Us)
        Vs = V.copy()
        Vs[I] = V[I] + b * dt * RV[I]
        O.fill_periodic(Vs)
    ref = np.sum(lam * tan)
    ps = M.Patchset(M.single_patch(n, (-1, -1, -1), dx), M.System(M.MOL_CCZ4))
    Un = torch.from_numpy(ps.pack(0, [U])).cuda()
    stages = [Un] + [ps.alloc(0) for _ in range(3)]
    acc, Unext = ps.alloc(0), ps.alloc(0)
    for s in range(1, 5):
        out = stages[s] if s < 4 else Unext
        ps.rk_stage(0, M.MOL_RK4, s, dt, Un, stages[s - 1], acc, out)
        ps.fill_ghosts(0, out)
    L = torch.from_numpy(ps.pack(0, [synth.embed(lam)])).cuda()
    ps.rk4_adjoint_step_stages(0, dt, L, [ps.alloc(0) for _ in range(3)], stages=stages, work=ps.alloc_work(0))
    torch.cuda.synchronize()
    got = np.sum(synth.interior(ps.unpack(0, L)[0]) * v)
    print("ccz4 48^3 reverse step", got, ref, flush=True)
    assert abs(got - ref) <= 1e-12 * abs(ref), (got, ref)
