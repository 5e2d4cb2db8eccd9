"""GPU adjoint of the CCZ4 right-hand side and of the RK4 step, against the
oracle's exact derivative (its right-hand side compiled with dual numbers):
element by element on a small periodic patch, and through dot-product
identities on ragged multi-tile patches; plus the gradient of the lapse-pulse
objective against central differences."""
import numpy as np
import pytest

from oracle import oracle as O
from paper_1806_04182_amd import molamr as M
from paper_1806_04182_amd import synth

pytestmark = pytest.mark.gpu


def _torch():
    import torch
    assert torch.cuda.is_available(), "GPU test needs a GPU"
    return torch


def _state(n, dx, seed):
    """Strongly non-flat CCZ4 state (lapse pulse + 1e-2 noise on every field),
    ghosts filled periodically."""
    st = synth.ccz4_lapse_pulse(n, (-1, -1, -1), dx, amp=0.2, width=0.4)
    st = st + synth.ccz4_minkowski_noise(n, amp=1e-2, seed=seed) - synth.CCZ4_FLAT[:, None, None, None]
    U = synth.embed(st)
    O.fill_periodic(U)
    return U


def _gpu_vjp(ps, U, lam_int):
    """(dR/dU)^T lam with the ghost contributions folded into their owners."""
    torch = _torch()
    Ud = torch.from_numpy(ps.pack(0, [U])).cuda()
    Ld = torch.from_numpy(ps.pack(0, [synth.embed(lam_int)])).cuda()
    out = ps.alloc(0)
    work = ps.alloc_work(0)
    ps.rhs_adjoint(0, Ud, Ld, out, work)
    ps.fill_ghosts_adjoint(0, out)
    torch.cuda.synchronize()
    return synth.interior(ps.unpack(0, out)[0])


@pytest.mark.parametrize("upwind", [1, 0])
def test_rhs_adjoint_matches_oracle_elementwise(upwind):
    n, dx = (5, 4, 4), 0.15
    U = _state(n, dx, 7)
    lam = np.random.default_rng(1).standard_normal((25,) + tuple(reversed(n)))
    ps = M.Patchset(M.single_patch(n, (-1, -1, -1), dx), M.System(M.MOL_CCZ4, upwind=upwind))
    got = _gpu_vjp(ps, U, lam)
    ref = O.ccz4_rhs_vjp_periodic(U, lam, dx, O.params(upwind=float(upwind)))
    sc = np.maximum(np.max(np.abs(ref), axis=(1, 2, 3)), 1.0)
    err = np.max(np.abs(got - ref), axis=(1, 2, 3)) / sc
    assert np.all(err < 1e-12), err


@pytest.mark.parametrize("n", [(19, 13, 9), (8, 8, 8)])
def test_rhs_adjoint_dot_product_with_oracle_jvp(n):
    """<(dR/dU)^T lam, v> = <lam, (dR/dU) P v> for random v; P the periodic fill."""
    dx = 2.0 / max(n)
    U = _state(n, dx, 3)
    rng = np.random.default_rng(2)
    shape = (25,) + tuple(reversed(n))
    lam, v = rng.standard_normal(shape), rng.standard_normal(shape)
    ps = M.Patchset(M.single_patch(n, (-1, -1, -1), dx), M.System(M.MOL_CCZ4))
    got = _gpu_vjp(ps, U, lam)
    V = synth.embed(v)
    O.fill_periodic(V)
    _, JV = O.ccz4_rhs_jvp(U, V, dx)
    a, b = np.sum(got * v), np.sum(lam * synth.interior(JV))
    assert abs(a - b) <= 1e-12 * np.sum(np.abs(got * v)), (a, b)


@pytest.mark.parametrize("n", [(10, 8, 6), (10, 8, 7)])
def test_rk4_adjoint_step_dot_product_with_oracle_jvp(n):
    """One reverse RK4 step against the tangent of one forward step built from
    the oracle's right-hand side and its exact JVP, stage by stage.  With
    fewer than 7 points on an axis the step gathers over the ghosted box and
    folds the ghost entries back (fill transpose); from 7 on, over the
    interior with periodic stencil images and a fused stage epilogue."""
    torch = _torch()
    dx = 2.0 / 10
    dt = 0.25 * dx
    U = _state(n, dx, 5)
    rng = np.random.default_rng(4)
    shape = (25,) + tuple(reversed(n))
    lam, v = rng.standard_normal(shape), rng.standard_normal(shape)
    # oracle: stage states and the tangent of U' = U + (k1 + 2 k2 + 2 k3 + k4)/6
    I = (slice(None), slice(3, -3), slice(3, -3), slice(3, -3))
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
    # GPU reverse step
    ps = M.Patchset(M.single_patch(n, (-1, -1, -1), dx), M.System(M.MOL_CCZ4))
    Un = torch.from_numpy(ps.pack(0, [U])).cuda()
    L = torch.from_numpy(ps.pack(0, [synth.embed(lam)])).cuda()
    w = [ps.alloc(0) for _ in range(6)]
    ps.rk4_adjoint_step(0, dt, L, w, Un=Un, work=ps.alloc_work(0))
    torch.cuda.synchronize()
    got = np.sum(synth.interior(ps.unpack(0, L)[0]) * v)
    assert abs(got - ref) <= 1e-12 * abs(ref), (got, ref)


def test_rk4_adjoint_step_from_kept_stages_equals_recomputing_step():
    """mol_rk4_adjoint_step_stages with the stage states produced by the
    forward stage launches gives the same lam, bit for bit, as
    mol_rk4_adjoint_step, which recomputes them (the same kernels in the same
    order); the wave form with no stage states too."""
    torch = _torch()
    n = (12, 9, 7)
    dx = 2.0 / 12
    dt = 0.25 * dx
    print("kept-stage reverse step", n, flush=True)
    ps = M.Patchset(M.single_patch(n, (-1, -1, -1), dx), M.System(M.MOL_CCZ4))
    Un = torch.from_numpy(ps.pack(0, [_state(n, dx, 6)])).cuda()
    rng = np.random.default_rng(7)
    lam0 = torch.from_numpy(ps.pack(0, [synth.embed(rng.standard_normal((25,) + tuple(reversed(n))))])).cuda()
    work = ps.alloc_work(0)
    L1 = lam0.clone()
    ps.rk4_adjoint_step(0, dt, L1, [ps.alloc(0) for _ in range(6)], Un=Un, work=work)
    stages = [Un] + [ps.alloc(0) for _ in range(3)]
    acc, Unext = ps.alloc(0), ps.alloc(0)
    for s in range(1, 5):
        out = stages[s] if s < 4 else Unext
        ps.rk_stage(0, M.MOL_RK4, s, dt, Un, stages[s - 1], acc, out)
        ps.fill_ghosts(0, out)
    L2 = lam0.clone()
    ps.rk4_adjoint_step_stages(0, dt, L2, [ps.alloc(0) for _ in range(3)], stages=stages, work=work)
    torch.cuda.synchronize()
    assert torch.equal(L1, L2)
    with pytest.raises(M.MolError):
        ps.rk4_adjoint_step_stages(0, dt, L2, [ps.alloc(0) for _ in range(3)], stages=stages[:3] + [L2], work=work)
    # wave: linear, no stage states
    pw = M.Patchset(M.single_patch(n, (-1, -1, -1), dx), M.System(M.MOL_WAVE, sigma=0.1))
    lw = torch.from_numpy(pw.pack(0, [synth.embed(rng.standard_normal((2,) + tuple(reversed(n))))])).cuda()
    a, b = lw.clone(), lw.clone()
    pw.rk4_adjoint_step(0, dt, a, [pw.alloc(0) for _ in range(3)])
    pw.rk4_adjoint_step_stages(0, dt, b, [pw.alloc(0) for _ in range(3)])
    torch.cuda.synchronize()
    assert torch.equal(a, b)


def test_lapse_objective_gradient_matches_central_differences():
    torch = _torch()
    from paper_1806_04182_amd.adjoint import ccz4_lapse_objective
    n = (16, 16, 16)
    dx = 2.0 / 16
    ps = M.Patchset(M.single_patch(n, (-1, -1, -1), dx), M.System(M.MOL_CCZ4))
    p0 = np.array([0.1, 0.4, 0.05, -0.1, 0.02])
    nsteps, dt, R = 8, 0.25 * dx, 0.6
    prm = torch.tensor(p0, dtype=torch.float64, requires_grad=True)
    J = ccz4_lapse_objective(prm, ps, nsteps, dt, R, 3)
    J.backward()
    g = prm.grad.numpy()
    h = 1e-6
    fd = np.zeros(5)
    for i in range(5):
        pp, pm = p0.copy(), p0.copy()
        pp[i] += h
        pm[i] -= h
        Jp = float(ccz4_lapse_objective(torch.tensor(pp), ps, nsteps, dt, R, 3))
        Jm = float(ccz4_lapse_objective(torch.tensor(pm), ps, nsteps, dt, R, 3))
        fd[i] = (Jp - Jm) / (2 * h)
    err = np.abs(g - fd) / np.maximum(np.abs(fd), 1e-3 * np.max(np.abs(fd)))
    assert np.all(err < 1e-6), (g, fd, err)


def test_rhs_adjoint_on_a_level_of_ragged_patches_matches_oracle():
    """A periodic level tiled by four patches of different sizes (each its own
    offset and interior-only slot layout in the workspace; ghost entries
    folded across patch faces by the fill transpose): element by element
    against the oracle's exact derivative on the whole periodic box."""
    torch = _torch()
    n, dx = (7, 6, 3), 0.15
    U = _state(n, dx, 11)
    lam = np.random.default_rng(5).standard_normal((25,) + tuple(reversed(n)))
    ref = O.ccz4_rhs_vjp_periodic(U, lam, dx, O.params(upwind=1.0))
    # x split 3 + 4, y split 3 + 3 (inclusive boxes in level index space)
    boxes = [((0, 0, 0), (2, 2, 2)), ((3, 0, 0), (6, 2, 2)), ((0, 3, 0), (2, 5, 2)), ((3, 3, 0), (6, 5, 2))]
    ps = M.Patchset(M.Hierarchy(n, (-1, -1, -1), dx, [(1, boxes)]), M.System(M.MOL_CCZ4, upwind=1))
    G = 3
    Up, Lp = [], []
    for lo, hi in boxes:
        sl = (slice(None), slice(lo[2], hi[2] + 1 + 2 * G), slice(lo[1], hi[1] + 1 + 2 * G),
              slice(lo[0], hi[0] + 1 + 2 * G))
        Up.append(U[sl].copy())  # U is ghosted and periodic: the patch with its ghosts
        Lp.append(synth.embed(lam[:, lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1]))
    Ud = torch.from_numpy(ps.pack(0, Up)).cuda()
    Ld = torch.from_numpy(ps.pack(0, Lp)).cuda()
    out = ps.alloc(0)
    ps.rhs_adjoint(0, Ud, Ld, out, ps.alloc_work(0))
    ps.fill_ghosts_adjoint(0, out)
    torch.cuda.synchronize()
    got = np.zeros_like(ref)
    for (lo, hi), a in zip(boxes, ps.unpack(0, out)):
        got[:, lo[2]:hi[2] + 1, lo[1]:hi[1] + 1, lo[0]:hi[0] + 1] = synth.interior(a)
    sc = np.maximum(np.max(np.abs(ref), axis=(1, 2, 3)), 1.0)
    err = np.max(np.abs(got - ref), axis=(1, 2, 3)) / sc
    assert np.all(err < 1e-12), err
