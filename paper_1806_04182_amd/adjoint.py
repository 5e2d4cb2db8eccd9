"""Gradients of sphere-integral objectives with respect to Gaussian
initial-data parameters, as torch.autograd.Functions: the periodic scalar
wave, and CCZ4 with a lapse pulse.

Wave.

Forward: phi_0 = A exp(-|x - c|^2 / w^2), Pi_0 = 0 (mol_wave_gaussian); nsteps
RK4 steps (mol_advance, one periodic level); J = sum_{|x| < R} phi dV
(mol_norms).  Checkpoints of the state are kept every `every` steps.
Backward: lam_T = dJ/dU_T (mol_sphere_adjoint), then the reverse RK4 sweep
(mol_rk4_adjoint_step) segment by segment from the last checkpoint to the
first, and dJ/dp = <lam_0, dU_0/dp> (mol_wave_gaussian_vjp).  The wave operator
is linear, so its transpose does not depend on the forward states: the
segments are not recomputed.

CCZ4.  Forward: flat data with alpha = 1 + A exp(-|x - c|^2 / w^2)
(mol_ccz4_lapse_pulse); nsteps RK4 steps; J = sum_{|x| < R} (alpha - 1) dV.
Backward: the operator is nonlinear, so each segment is recomputed forward
from its checkpoint with the stage kernels, keeping the four stage states of
every step, then the reverse RK4 steps (mol_rk4_adjoint_step_stages, which
needs no further recomputation) run from the last step of the segment back
to its checkpoint; dJ/dp through
mol_ccz4_lapse_pulse_vjp.  All arithmetic runs in libmolamr.
"""
from __future__ import annotations

import torch

from . import molamr as M


class WaveSphereObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, prm: torch.Tensor, ps: M.Patchset, nsteps: int, dt: float, radius: float, every: int = 20):
        p = [float(v) for v in prm.detach().cpu()]
        st = ps.alloc_states()
        ps.wave_gaussian(0, p, st[0]["U"])
        ps.fill_ghosts(0, st[0]["U"])
        ckpts = [st[0]["U"].clone()]
        for s in range(nsteps):
            ps.advance(st, dt)
            if (s + 1) % every == 0 and s + 1 < nsteps:
                ckpts.append(st[0]["U"].clone())
        out = torch.zeros(5, dtype=torch.float64, device=st[0]["U"].device)
        ps.norms(0, st[0]["U"], 0, 0.0, radius, out)
        ctx.ps, ctx.p, ctx.nsteps, ctx.dt, ctx.radius, ctx.every = ps, p, nsteps, dt, radius, every
        ctx.ckpts = ckpts
        return out[3].detach().cpu().reshape(())

    @staticmethod
    def backward(ctx, gJ):
        ps = ctx.ps
        lam = ps.alloc(0)
        w = [ps.alloc(0) for _ in range(3)]
        ps.sphere_adjoint(0, 0, ctx.radius, float(gJ), lam)
        # segments [k*every, (k+1)*every) in reverse order
        nseg = (ctx.nsteps + ctx.every - 1) // ctx.every
        for k in reversed(range(nseg)):
            steps = min(ctx.every, ctx.nsteps - k * ctx.every)
            for _ in range(steps):
                ps.rk4_adjoint_step(0, ctx.dt, lam, w)
        g = torch.zeros(5, dtype=torch.float64, device=lam.device)
        ps.wave_gaussian_vjp(0, ctx.p, lam, g)
        return g.cpu(), None, None, None, None, None


def sphere_objective(prm, ps, nsteps, dt, radius, every=20):
    return WaveSphereObjective.apply(prm, ps, nsteps, dt, radius, every)


ALPHA = 18  # lapse: field index of the CCZ4 state


class Ccz4LapseObjective(torch.autograd.Function):
    @staticmethod
    def forward(ctx, prm: torch.Tensor, ps: M.Patchset, nsteps: int, dt: float, radius: float, every: int = 20):
        p = [float(v) for v in prm.detach().cpu()]
        st = ps.alloc_states()
        ps.ccz4_lapse_pulse(0, p, st[0]["U"])
        ps.fill_ghosts(0, st[0]["U"])
        ckpts = [st[0]["U"].clone()]
        for s_ in range(nsteps):
            ps.advance(st, dt)
            if (s_ + 1) % every == 0 and s_ + 1 < nsteps:
                ckpts.append(st[0]["U"].clone())
        out = torch.zeros(5, dtype=torch.float64, device=st[0]["U"].device)
        ps.norms(0, st[0]["U"], ALPHA, 1.0, radius, out)
        ctx.ps, ctx.p, ctx.nsteps, ctx.dt, ctx.radius, ctx.every = ps, p, nsteps, dt, radius, every
        ctx.ckpts = ckpts
        return out[3].detach().cpu().reshape(())

    @staticmethod
    def backward(ctx, gJ):
        ps = ctx.ps
        lam = ps.alloc(0)
        w = [ps.alloc(0) for _ in range(3)]
        work = ps.alloc_work(0)
        ps.sphere_adjoint(0, ALPHA, ctx.radius, float(gJ), lam)
        acc = ps.alloc(0)
        nseg = (ctx.nsteps + ctx.every - 1) // ctx.every
        # the four stage states of every step of one segment, allocated once
        # and reused by every segment
        kept = [[ps.alloc(0) for _ in range(4)] for _ in range(min(ctx.every, ctx.nsteps))]
        # on a level that is one periodic patch of at least 6 points per axis
        # the stage kernel writes the periodic ghost images of its output
        # (the values the ghost fill would copy), so no fill is needed there
        dims = ps.layouts[0]["dims"]
        images = ps.nlev == 1 and len(dims) == 1 and min(dims[0]) >= 6 and not ps.hier.open
        for k in reversed(range(nseg)):
            steps = min(ctx.every, ctx.nsteps - k * ctx.every)
            # the segment recomputed from its checkpoint with the forward
            # stages (the kernels and order of mol_advance), keeping the four
            # stage states of every step (ghosts filled) for the reverse
            # steps; each step's last stage writes the next step's U^n, and
            # the segment's last step stops after its fourth stage state
            kept[0][0].copy_(ctx.ckpts[k])
            for j, stages in enumerate(kept[:steps]):
                for s in range(1, 5):
                    if s == 4 and j + 1 == steps:
                        break
                    out = stages[s] if s < 4 else kept[j + 1][0]
                    ps.rk_stage(0, M.MOL_RK4, s, ctx.dt, stages[0], stages[s - 1], acc, out)
                    if not images:
                        ps.fill_ghosts(0, out)
            for stages in reversed(kept[:steps]):
                ps.rk4_adjoint_step_stages(0, ctx.dt, lam, w, stages=stages, work=work)
        del kept
        g = torch.zeros(5, dtype=torch.float64, device=lam.device)
        ps.ccz4_lapse_pulse_vjp(0, ctx.p, lam, g)
        return g.cpu(), None, None, None, None, None


def ccz4_lapse_objective(prm, ps, nsteps, dt, radius, every=20):
    return Ccz4LapseObjective.apply(prm, ps, nsteps, dt, radius, every)

