#!/usr/bin/env python3
"""Throughput of the CCZ4 method-of-lines hot path on one MI355X.

Workload (default): CCZ4 on one periodic 96^3 patch with 3 ghost points,
RK4 with dt = dx/4, 4th-order FD + lop-sided advection + KO (sigma = 0.1),
1+log slicing, Gamma-driver shift, kappa_z = kappa_c = 0.1, FP64, Minkowski
plus uniform seeded noise of amplitude 1e-10 on all 25 fields.  One step is
one RK4 step: 4 x (ghost fill + fused RHS/stage kernel), replayed from a
captured HIP graph.  value = interior points x RK stages / second.

Prints one JSON line on stdout; progress goes to stderr.
"""
from __future__ import annotations

import argparse
import json
import math
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "CCZ4 FP64 point-updates/s per RK stage: plain vs batched patches; adjoint/fwd"
HBM_PEAK_GBS = 8000.0
FP64_PEAK_TFLOPS = 78.6
CCZ4_BYTES_PER_PT_STAGE = 25 * 4.25 * 8  # U^n, U^(s), Acc, Uout traffic averaged over the 4 RK4 stages


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def cpu_baseline(n=96, steps=2):
    """The oracle (single-threaded C) on a bounded sample of the same workload:
    `steps` RK4 steps of the n^3 periodic patch with the same data recipe."""
    from oracle import oracle as O
    from paper_1806_04182_amd import synth
    dx = 2.0 / 96
    U = synth.embed(synth.ccz4_minkowski_noise((n, n, n), amp=1e-10, seed=0))
    t0 = time.perf_counter()
    O.rk_run(O.CCZ4, O.RK4, U, dx, 0.25 * dx, steps, O.params())
    dt = time.perf_counter() - t0
    return {"value": n ** 3 * 4 * steps / dt, "unit": "pt-stage/s", "cores": 1, "kind": "oracle",
            "sample": f"{steps} RK4 steps ({4 * steps} stages) of the {n}^3 periodic CCZ4 patch, same data "
                      f"recipe, {dt:.1f} s wall on one host core"}


def fill_minkowski_noise(ps, level, U, seed):
    """Minkowski plus 1e-10 uniform noise on every field of a level buffer
    (device-side seeded generator; ghosts are filled by the first stage)."""
    import torch
    g = torch.Generator(device="cuda")
    g.manual_seed(seed)
    from paper_1806_04182_amd import synth
    L = ps.layouts[level]
    U.zero_()
    for p, off in enumerate(L["offsets"]):
        fs = L["fstrides"][p]
        for f in range(25):
            blk = U[off + f * fs: off + (f + 1) * fs]
            blk.uniform_(-1e-10, 1e-10, generator=g)
            blk.add_(float(synth.CCZ4_FLAT[f]))


def amr_bench(M, steps=2):
    """Three levels (R = 2, 3), 200 patches, BOR sub-cycling: one coarse step
    as a captured HIP graph (batched: one launch per level and operation) vs
    the same step with one launch per patch and operation, no graph."""
    import torch
    from paper_1806_04182_amd import synth
    levels, N0, dx0 = synth.amr_three_levels(0)
    t0 = time.perf_counter()
    ps = M.Patchset(M.Hierarchy(N0, (-1, -1, -1), dx0, levels), M.System(M.MOL_CCZ4))
    tbuild = time.perf_counter() - t0
    log(f"bench: AMR patchset built in {tbuild:.1f} s")
    st = ps.alloc_states()
    for l in range(len(levels)):
        fill_minkowski_noise(ps, l, st[l]["U"], 100 + l)
    pts = [sum((hi[0] - lo[0] + 1) * (hi[1] - lo[1] + 1) * (hi[2] - lo[2] + 1) for lo, hi in b) for _, b in levels]
    stages = 4 * pts[0] + 8 * pts[1] + 24 * pts[2]
    dt0 = 0.25 * dx0
    res = {}
    g = ps.graph_create(st, dt0)
    stream = torch.cuda.current_stream()
    for mode in ("batched", "plain"):
        run = (lambda: g.launch(stream)) if mode == "batched" else (lambda: ps.advance(st, dt0, M.MOL_PLAIN, stream))
        run()
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        t0 = time.perf_counter()
        e0.record(stream)
        for _ in range(steps):
            run()
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / steps
        res[mode] = {"ms_per_coarse_step": ms, "pt_stage_per_s": stages / (ms * 1e-3),
                     "wall_ms_per_coarse_step": (time.perf_counter() - t0) * 1e3 / steps}
        log(f"bench: AMR {mode}: {ms:.1f} ms per coarse step")
    # the same graph after autotuning every level's stage launch (patch order;
    # the CCZ4 tile is fixed)
    tilings, dtl = [], dt0
    for l in range(len(levels)):
        dtl = dtl / levels[l][0] if l else dtl
        tilings.append(ps.autotune(l, st[l], dtl, reps=3))
    for l in range(len(levels)):
        fill_minkowski_noise(ps, l, st[l]["U"], 100 + l)
    gt = ps.graph_create(st, dt0)
    gt.launch(stream)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(steps):
        gt.launch(stream)
    e1.record(stream)
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1) / steps
    res["batched_autotuned"] = {"ms_per_coarse_step": ms, "pt_stage_per_s": stages / (ms * 1e-3),
                                "tilings": tilings}
    log(f"bench: AMR batched, autotuned: {ms:.1f} ms per coarse step")
    del gt
    # time-refinement strategies (batched launches, no graph): the cost of
    # advancing the hierarchy by dt0; without sub-cycling every level takes
    # the finest level's step, dt0 / 6
    strat = {}
    for name, tm, calls in (("BOR", M.MOL_TIME_BOR, 1), ("BO", M.MOL_TIME_BO, 1), ("BO1", M.MOL_TIME_BO1, 1),
                            ("NOSUB", M.MOL_TIME_NOSUB, 6)):
        ps.advance(st, dt0 / calls, M.MOL_BATCHED | tm, stream)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        for _ in range(calls):
            ps.advance(st, dt0 / calls, M.MOL_BATCHED | tm, stream)
        e1.record(stream)
        torch.cuda.synchronize()
        strat[name] = {"ms_per_dt0": e0.elapsed_time(e1), "calls_per_dt0": calls}
        log(f"bench: AMR {name}: {strat[name]['ms_per_dt0']:.1f} ms per dt0")
    res["time_strategies"] = strat
    out = torch.zeros(5, dtype=torch.float64, device="cuda")
    ps.norms(0, st[0]["U"], 18, 1.0, 0.6, out)
    torch.cuda.synchronize()
    res["batched_over_plain"] = res["plain"]["ms_per_coarse_step"] / res["batched"]["ms_per_coarse_step"]
    res["config"] = {"levels": 3, "ratios": [2, 3], "patches": sum(len(b) for _, b in levels),
                     "points_per_level": pts, "pt_stages_per_coarse_step": stages,
                     "patch_interior_range": [16, 48], "host_schedule_build_s": tbuild,
                     "nonfinite_after_run": int(out[4].item())}
    del g
    return res


def fmr_bench(M):
    """The FMR wave experiment (Sec. IV.A) on the GPU driver: the largest
    reflection integral Q while the reflection of the pulse entering the
    refined region crosses [-2, -1], at coarse dx = 1/40, 1/80, 1/160, per
    time-refinement strategy, and ratio 4 against ratio 2/2 (BOR)."""
    import numpy as np
    from paper_1806_04182_amd import fmr
    res = {"resolutions": [40, 80, 160], "window": [3.2, 4.2]}
    t0 = time.perf_counter()
    for name, tm in (("BOR", M.MOL_TIME_BOR), ("BO", M.MOL_TIME_BO), ("BO1", M.MOL_TIME_BO1),
                     ("NOSUB", M.MOL_TIME_NOSUB)):
        q = [fmr.reflection_q(n, tm) for n in (40, 80, 160)]
        res[name] = {"Q": q, "orders": [float(np.log2(q[i] / q[i + 1])) for i in range(2)]}
        log(f"bench: FMR {name}: Q {q}, orders {res[name]['orders']}")
    res["ratio4_vs_2x2_BOR_dx1_80"] = {"ratio4": fmr.reflection_q(80, M.MOL_TIME_BOR, ratios=(4,)),
                                      "ratio2x2": fmr.reflection_q(80, M.MOL_TIME_BOR, ratios=(2, 2))}
    res["wall_s"] = time.perf_counter() - t0
    return res


def amr_wave_bench(M):
    """The AMR wave experiment (Sec. IV.A) on the library: one refined level
    (ratio 2) following the two halves of the pulse, regridded every 0.0125
    from tags |phi| >= 1e-3 (mol_tag, mol_cluster, mol_regrid_*).  Convergence
    factor n_c at t = 1.25, 2.5, 3.75, 5 for dx0 = 1/40, 1/80, 1/160 per
    time-refinement strategy, and the cost of a regrid in the 1/160 BOR run."""
    import numpy as np
    from paper_1806_04182_amd import amr
    times = (1.25, 2.5, 3.75, 5.0)
    res = {"resolutions": [40, 80, 160], "times": list(times), "threshold": 1e-3, "buffer": 0.1,
           "regrid_dt": 0.0125}
    t0 = time.perf_counter()
    for name, tm in (("BOR", M.MOL_TIME_BOR), ("BO", M.MOL_TIME_BO), ("NOSUB", M.MOL_TIME_NOSUB)):
        phis = []
        for n in (40, 80, 160):
            run = amr.AmrChannelRun(n)
            t1 = time.perf_counter()
            phis.append(run.run(5.0, tm, checkpoints=times))
            if n == 160 and name == "BOR":
                wall = time.perf_counter() - t1
                # the same run without regrids (first boxes kept) isolates their cost
                still = amr.AmrChannelRun(n, regrid_dt=1e9)
                t2 = time.perf_counter()
                still.run(5.0, tm)
                wall_still = time.perf_counter() - t2
                res["run_1_160_BOR"] = {"wall_s": wall, "coarse_steps": int(round(5.0 / run.dt0(tm))),
                                        "regrids": run.regrids, "wall_without_regrids_s": wall_still,
                                        "ms_per_regrid": 1e3 * (wall - wall_still) / max(run.regrids, 1)}
        nc = [amr.convergence_order([p[t] for p in phis]) for t in times]
        res[name] = {"n_c": nc}
        log(f"bench: AMR wave {name}: n_c {np.round(nc, 2).tolist()}")
    res["wall_s"] = time.perf_counter() - t0
    return res


def single_bh_bench(M, nlev=8, N=64, L=128.0, t_end=20.0):
    """A single spinning black hole (M = 1, a = 0.2; Sec. V) on nested
    ratio-2 levels shaped like the paper's ratio-2 mesh (eight levels of N^3
    points, outer radiative boundary at L, finest spacing 2L/N/2^7), RK4 with
    BOR sub-cycling from a captured graph."""
    import torch
    from paper_1806_04182_amd.bh_runs import SingleBH
    t0 = time.perf_counter()
    bh = SingleBH(nlev=nlev, N=N, L=L)
    setup = time.perf_counter() - t0
    bh.run(1.0)  # warm-up
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    steps0 = bh.t
    e0.record()
    bh.run(t_end)
    e1.record()
    torch.cuda.synchronize()
    ms = e0.elapsed_time(e1)
    nsteps = int(round((bh.t - steps0) / (0.25 * bh.dx0)))
    pts = nlev * N ** 3
    pt_stages = 4 * N ** 3 * sum(2 ** l for l in range(nlev)) * nsteps
    s = bh.summary()
    res = {"config": {"levels": nlev, "points_per_level": N ** 3, "outer_boundary": L,
                      "finest_spacing": 2 * L / N / 2 ** (nlev - 1), "spin": 0.2},
           "t_end": bh.t, "coarse_steps": nsteps, "ms_per_coarse_step": ms / nsteps,
           "pt_stage_per_s": pt_stages / (ms * 1e-3), "total_points": pts, "setup_s": setup,
           "finite": s["finite"], "alpha_r1": bh.field_at(18, 1.0), "alpha_r8": bh.field_at(18, 8.0)}
    log(f"bench: single BH: {ms / nsteps:.1f} ms per coarse step, alpha(r=1) {res['alpha_r1']:.3f}")
    return res


def _time_objective(fn, p, *args):
    import torch
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    J = fn(p, *args)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    J.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    return J, t1 - t0, t2 - t1


def adjoint_bench(M, n=64, nsteps=200, every=20, n_ccz4=48):
    """Wave 64^3 and CCZ4 48^3 (lapse pulse), 200 RK4 steps, checkpoints every
    20: forward (with the objective) and backward (reverse sweep, recomputed
    segments for CCZ4, initial-data VJP) wall times."""
    import torch
    from paper_1806_04182_amd.adjoint import ccz4_lapse_objective, sphere_objective
    dx = 2.0 / n
    ps = M.Patchset(M.single_patch((n, n, n), (-1, -1, -1), dx), M.System(M.MOL_WAVE, sigma=0.1))
    p = torch.tensor([1.0, 0.2, 0.1, -0.05, 0.02], dtype=torch.float64, requires_grad=True)
    sphere_objective(p, ps, 4, 0.25 * dx, 0.6, every)  # warm-up
    J, fwd, bwd = _time_objective(sphere_objective, p, ps, nsteps, 0.25 * dx, 0.6, every)
    res = {"workload": f"wave_{n}^3_rk4_{nsteps}_steps_checkpoint_{every}", "fwd_s": fwd, "bwd_s": bwd,
           "bwd_over_fwd": bwd / fwd, "fwd_plus_bwd_over_fwd": (fwd + bwd) / fwd,
           "dJ_dA_minus_J": float(p.grad[0]) - float(J.detach())}
    log(f"bench: CCZ4 adjoint {n_ccz4}^3")
    dx = 2.0 / n_ccz4
    ps = M.Patchset(M.single_patch((n_ccz4,) * 3, (-1, -1, -1), dx), M.System(M.MOL_CCZ4))
    p = torch.tensor([0.1, 0.4, 0.05, -0.1, 0.02], dtype=torch.float64, requires_grad=True)
    p0 = torch.tensor([0.1, 0.4, 0.05, -0.1, 0.02], dtype=torch.float64, requires_grad=True)
    ccz4_lapse_objective(p0, ps, 4, 0.25 * dx, 0.6, every).backward()  # warm-up
    J, fwd, bwd = _time_objective(ccz4_lapse_objective, p, ps, nsteps, 0.25 * dx, 0.6, every)
    res["ccz4"] = {"workload": f"ccz4_{n_ccz4}^3_lapse_pulse_rk4_{nsteps}_steps_checkpoint_{every}", "fwd_s": fwd,
                   "bwd_s": bwd, "bwd_over_fwd": bwd / fwd, "fwd_plus_bwd_over_fwd": (fwd + bwd) / fwd,
                   "J": float(J.detach()), "dJ_dA": float(p.grad[0])}
    return res


def stage_kernel_time(ps, M, st, scheme, dt, reps=10):
    """Average duration of the fused stage kernel alone (HIP events on the
    launch stream), cycling through the scheme's stages."""
    import torch
    stream = torch.cuda.current_stream()
    U, a, b, acc = st[0]["U"], st[0]["S0"], st[0]["S1"], st[0]["acc"]
    ps.fill_ghosts(0, U, stream=stream)
    seq = ([(1, U, a), (2, a, b), (3, b, a), (4, a, b)] if scheme == M.MOL_RK4
           else [(1, U, a), (2, a, b), (3, b, a)])
    def run(n):
        for _ in range(n):
            for s, Us, Uo in seq:
                ps.rk_stage(0, scheme, s, dt, U, Us, acc, Uo, stream=stream)
    run(1)
    torch.cuda.synchronize()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    run(reps)
    e1.record(stream)
    torch.cuda.synchronize()
    return e0.elapsed_time(e1) / (reps * len(seq))


# Workloads whose stage kernel is profiled alone (rocprofv3 counters): system,
# points per axis, scheme, the data the benchmark gives them
PROFILE_CASES = {"ccz4_96": ("ccz4", 96), "wave_256": ("wave", 256), "wave_512": ("wave", 512),
                 "mhd_128": ("mhd", 128)}


def _single_patch_case(M, system, n):
    """Patchset, states, scheme and dt of the benchmark's single-patch
    workloads, with their data in place."""
    import torch
    from paper_1806_04182_amd import synth
    if system == "ccz4":
        dx = 2.0 / n
        ps = M.Patchset(M.single_patch((n, n, n), (-1, -1, -1), dx), M.System(M.MOL_CCZ4))
        st = ps.alloc_states()
        st[0]["U"].copy_(torch.from_numpy(ps.pack(0, [synth.embed(
            synth.ccz4_minkowski_noise((n, n, n), amp=1e-10, seed=0))])))
        return ps, st, M.MOL_RK4, 0.25 * dx
    if system == "wave":
        dx = 2.0 / n
        ps = M.Patchset(M.single_patch((n, n, n), (-1, -1, -1), dx), M.System(M.MOL_WAVE, sigma=0.1))
        st = ps.alloc_states()
        ps.wave_gaussian(0, [1.0, 0.2, *synth.wave_centre(0)], st[0]["U"])
        return ps, st, M.MOL_RK4, 0.25 * dx
    dx = 1.0 / n
    ps = M.Patchset(M.single_patch((n, n, n), (0, 0, 0), dx), M.System(M.MOL_MHD, sigma=0.0))
    st = ps.alloc_states()
    st[0]["U"].copy_(torch.from_numpy(ps.pack(0, [synth.embed(synth.mhd_ot_like((n, n, n), seed=0))])))
    return ps, st, M.MOL_SSPRK3, 0.2 * dx


def profile_case(M, name):
    system, n = PROFILE_CASES[name]
    ps, st, scheme, dt = _single_patch_case(M, system, n)
    kms = stage_kernel_time(ps, M, st, scheme, dt, reps=5)
    return {"case": name, "points": n ** 3, "stage_kernel_ms": kms}


def profile_record(case, pts):
    """The committed rocprofv3 counter record of one workload's stage kernel
    (HBM bytes per launch, FP64 FLOP per point-stage), or None when the
    kernel sources changed since it was taken or the workload differs."""
    from paper_1806_04182_amd import profsum
    path = os.path.join(ROOT, "profiles", profsum.CASES[case]["file"])
    try:
        rec = json.load(open(path))
    except (OSError, ValueError):
        return None
    if rec.get("source_sha256") != profsum.source_hash(profsum.CASES[case]["sources"]) or rec.get("points") != pts:
        return None
    return rec


def _counter_fields(case, pts, kms, alg_bytes_per_pt):
    """Counter-based HBM traffic and FP64 rate of a stage kernel beside its
    algorithmic bytes, from the committed record (None entries when stale)."""
    from paper_1806_04182_amd import profsum
    rec = profile_record(case, pts)
    if rec is None:
        return {"counter_record": None}
    tf = rec["fp64_flop_per_pt_stage"] * pts / (kms * 1e-3) / 1e12
    return {"counter_record": "profiles/" + profsum.CASES[case]["file"],
            "counter_bytes_per_pt_stage": rec["hbm_bytes_per_launch"] / pts,
            "traffic_over_algorithmic": rec["hbm_bytes_per_launch"] / (alg_bytes_per_pt * pts),
            "roofline_fp64": {"bound": "alu", "achieved": tf, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                              "frac": tf / FP64_PEAK_TFLOPS, "flop_per_pt_stage": rec["fp64_flop_per_pt_stage"],
                              "flop_count": "executed (SQ_INSTS_VALU_FLOPS_FP64 x 64 lanes)"}}


def wave_mhd_bench(M):
    """Secondary paths: the scalar wave (32^3, 20 steps; and 256^3, where the
    state is far larger than the caches) and MHD (128^3, SSP-RK3)."""
    import torch
    from paper_1806_04182_amd import synth
    out = {}
    for n in (32, 128, 256, 512):
        log(f"bench: wave {n}^3")
        dx = 2.0 / n
        ps = M.Patchset(M.single_patch((n, n, n), (-1, -1, -1), dx), M.System(M.MOL_WAVE, sigma=0.1))
        st = ps.alloc_states()
        ps.wave_gaussian(0, [1.0, 0.2, *synth.wave_centre(0)], st[0]["U"])
        # the 20-step run as one graph of 20 steps (as for the headline); a
        # one-step graph and one launch of the 20-step graph warm up first
        steps = 20
        g = ps.graph_create(st, 0.25 * dx)
        gk = ps.graph_create(st, 0.25 * dx, nsteps=steps)
        stream = torch.cuda.current_stream()
        g.launch(stream)
        gk.launch(stream)
        torch.cuda.synchronize()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        gk.launch(stream)
        gk.launch(stream)
        e1.record(stream)
        torch.cuda.synchronize()
        ms = e0.elapsed_time(e1) / (2 * steps)
        kms = stage_kernel_time(ps, M, st, M.MOL_RK4, 0.25 * dx)
        gbs = 68.0 * n ** 3 / (kms * 1e-3) / 1e9
        out[f"wave_{n}^3"] = {"pt_stage_per_s": n ** 3 * 4 / (ms * 1e-3), "ms_per_step": ms,
                               "steps_per_graph_launch": steps,
                               "stage_kernel_ms": kms, "stage_kernel_GBs_algorithmic": gbs,
                               "hbm_frac": gbs / HBM_PEAK_GBS, "bytes_per_pt_stage": 68.0}
        if f"wave_{n}" in PROFILE_CASES:
            out[f"wave_{n}^3"].update(_counter_fields(f"wave_{n}", n ** 3, kms, 68.0))
        tuned = ps.autotune(0, st[0], 0.25 * dx, reps=3)
        tkms = stage_kernel_time(ps, M, st, M.MOL_RK4, 0.25 * dx)
        out[f"wave_{n}^3"]["autotuned"] = {"tiling": tuned, "stage_kernel_ms": tkms,
                                           "hbm_frac": 68.0 * n ** 3 / (tkms * 1e-3) / 1e9 / HBM_PEAK_GBS}
        del g, gk, ps, st
        torch.cuda.empty_cache()
    for n in (192,):
        log(f"bench: MHD {n}^3")
        dx = 1.0 / n
        ps = M.Patchset(M.single_patch((n, n, n), (0, 0, 0), dx), M.System(M.MOL_MHD, sigma=0.0))
        st = ps.alloc_states()
        st[0]["U"].copy_(torch.from_numpy(ps.pack(0, [synth.embed(synth.mhd_ot_like((n, n, n), seed=0))])))
        kms = stage_kernel_time(ps, M, st, M.MOL_SSPRK3, 0.2 * dx)
        out[f"mhd_{n}^3"] = {"pt_stage_per_s": n ** 3 / (kms * 1e-3), "stage_kernel_ms": kms,
                             "stage_kernel_GBs_algorithmic": 171.0 * n ** 3 / (kms * 1e-3) / 1e9}
        del ps, st
    n = 128
    log(f"bench: MHD {n}^3")
    dx = 1.0 / n
    ps = M.Patchset(M.single_patch((n, n, n), (0, 0, 0), dx), M.System(M.MOL_MHD, sigma=0.0))
    st = ps.alloc_states()
    st[0]["U"].copy_(torch.from_numpy(ps.pack(0, [synth.embed(synth.mhd_ot_like((n, n, n), seed=0))])))
    kms = stage_kernel_time(ps, M, st, M.MOL_SSPRK3, 0.2 * dx)
    gbs = 171.0 * n ** 3 / (kms * 1e-3) / 1e9
    out["mhd_128^3"] = {"pt_stage_per_s": n ** 3 / (kms * 1e-3), "stage_kernel_ms": kms,
                        "stage_kernel_GBs_algorithmic": gbs, "hbm_frac": gbs / HBM_PEAK_GBS,
                        "bytes_per_pt_stage": 171.0}
    out["mhd_128^3"].update(_counter_fields("mhd_128", n ** 3, kms, 171.0))
    tuned = ps.autotune(0, st[0], 0.2 * dx, reps=3)
    st[0]["U"].copy_(torch.from_numpy(ps.pack(0, [synth.embed(synth.mhd_ot_like((n, n, n), seed=0))])))
    out["mhd_128^3"]["autotuned"] = {"tiling": tuned,
                                     "stage_kernel_ms": stage_kernel_time(ps, M, st, M.MOL_SSPRK3, 0.2 * dx)}
    # reconstruction and flux variants on the same data (App. A, B; Sec. II.B.2)
    var = {}
    for rname, rec in (("weno5z", M.MOL_RECON_WENO5Z), ("weno5js", M.MOL_RECON_WENO5JS), ("weno3", M.MOL_RECON_WENO3)):
        for fname, fl in (("llf", M.MOL_FLUX_LLF), ("hll", M.MOL_FLUX_HLL), ("split", M.MOL_FLUX_SPLIT)):
            psv = M.Patchset(M.single_patch((n, n, n), (0, 0, 0), dx),
                             M.System(M.MOL_MHD, sigma=0.0, mhd_recon=rec, mhd_flux=fl))
            stv = psv.alloc_states()
            stv[0]["U"].copy_(st[0]["U"])
            var[f"{rname}_{fname}"] = {"stage_kernel_ms": stage_kernel_time(psv, M, stv, M.MOL_SSPRK3, 0.2 * dx)}
            del psv, stv
    out["mhd_variants_128^3"] = var
    return out


def mhd_runs_bench(M):
    """The MHD tests of Sec. IV.B on the GPU driver: relative L1 error of B_x
    of the CP Alfven wave after three crossing times (N = 32, 64, 128) per
    reconstruction, and of B_y of the Brio-Wu tube at t = 0.2 (N = 50 .. 400,
    against WENO5-Z at N = 3200) unigrid and with FMR."""
    import numpy as np
    from paper_1806_04182_amd import mhd_runs as R
    t0 = time.perf_counter()
    res = {"alfven": {}, "brio_wu": {}}
    for name, rec in (("weno5z", M.MOL_RECON_WENO5Z), ("weno5js", M.MOL_RECON_WENO5JS), ("weno3", M.MOL_RECON_WENO3)):
        e = [R.alfven_error(N, rec) for N in (32, 64, 128)]
        res["alfven"][name] = {"N": [32, 64, 128], "err_Bx": e, "orders": list(np.log2(np.array(e[:-1]) / np.array(e[1:])))}
        log(f"bench: Alfven {name}: {e}")
    ref = R.brio_wu(3200)
    res["brio_wu"]["dt_over_dx"] = {"unigrid": R.BW_CFL, "fmr": R.BW_CFL_FMR}
    runs = [("unigrid", {}), ("2/2", {"fmr": "2/2"}), ("4", {"fmr": "4"}),
            ("2/2_weno3", {"fmr": "2/2", "recon": M.MOL_RECON_WENO3}), ("unigrid_weno3", {"recon": M.MOL_RECON_WENO3}),
            ("2/2_ssprk3_bor", {"fmr": "2/2", "ssp3": True})]
    for name, kw in runs:
        e = [R.brio_wu_error(R.brio_wu(N, **kw), ref, 3200) for N in (50, 100, 200, 400)]
        bad = [N for N, x in zip((50, 100, 200, 400), e) if not math.isfinite(x)]
        res["brio_wu"][name] = {"N": [50, 100, 200, 400], "err_By": [x if math.isfinite(x) else None for x in e],
                                "nonfinite_N": bad}
        log(f"bench: Brio-Wu {name}: {e}")
    res["wall_s"] = time.perf_counter() - t0
    return res


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=96)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=96)
    ap.add_argument("--no-extras", action="store_true", help="skip the AMR and adjoint measurements")
    ap.add_argument("--no-fmr", action="store_true",
                    help="skip the FMR reflection, MHD and AMR wave test runs (many small launches; kept out of kernel traces)")
    ap.add_argument("--paths-only", action="store_true",
                    help="measure only the wave and MHD paths and print their JSON")
    ap.add_argument("--profile-case", choices=sorted(PROFILE_CASES),
                    help="run only the stage-kernel timing of one workload (for counter collection)")
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: the library has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    log("bench: importing torch")
    import numpy as np
    import torch
    from paper_1806_04182_amd import molamr as M
    from paper_1806_04182_amd import synth

    assert torch.cuda.is_available(), "no GPU"
    if args.paths_only:
        print(json.dumps(wave_mhd_bench(M)), flush=True)
        return
    if args.profile_case:
        print(json.dumps(profile_case(M, args.profile_case)), flush=True)
        return
    n = args.n
    dx = 2.0 / n
    dt = 0.25 * dx
    ps = M.Patchset(M.single_patch((n, n, n), (-1, -1, -1), dx), M.System(M.MOL_CCZ4))
    log(f"bench: patchset {n}^3 built")
    st = ps.alloc_states()
    # warm-up: a graph of one step; timed: one graph of K steps (every step
    # leaves U with filled ghosts, so the steps after the first skip the fill
    # of U before their first stage)
    g = ps.graph_create(st, dt)
    gk = ps.graph_create(st, dt, nsteps=args.steps)
    stream = torch.cuda.current_stream()
    # K timed steps after W warm-up steps for each data seed 0..4; the median
    # run is reported
    runs = []
    for seed in range(5):
        st[0]["U"].copy_(torch.from_numpy(ps.pack(0, [synth.embed(
            synth.ccz4_minkowski_noise((n, n, n), amp=1e-10, seed=seed))])))
        for _ in range(args.warmup):
            g.launch(stream)
        torch.cuda.synchronize()
        t0 = time.perf_counter()
        e0 = torch.cuda.Event(enable_timing=True)
        e1 = torch.cuda.Event(enable_timing=True)
        e0.record(stream)
        gk.launch(stream)
        e1.record(stream)
        torch.cuda.synchronize()
        wall = time.perf_counter() - t0
        runs.append((e0.elapsed_time(e1), wall, seed))
        log(f"bench: seed {seed}: {args.steps} steps in {runs[-1][0]:.2f} ms (events), {wall * 1e3:.2f} ms (wall)")
    ms, wall, seed_med = sorted(runs)[len(runs) // 2]
    pts = n ** 3
    value = pts * 4 * args.steps / (ms * 1e-3)

    # dominant kernel: the fused CCZ4 stage kernel, timed alone on the same stream
    reps = 10
    a, b = st[0]["S0"], st[0]["S1"]
    ps.fill_ghosts(0, st[0]["U"], stream=stream)
    torch.cuda.synchronize()
    k0 = torch.cuda.Event(enable_timing=True)
    k1 = torch.cuda.Event(enable_timing=True)
    k0.record(stream)
    for _ in range(reps):
        ps.rk_stage(0, M.MOL_RK4, 1, dt, st[0]["U"], st[0]["U"], st[0]["acc"], a, stream=stream)
        ps.rk_stage(0, M.MOL_RK4, 2, dt, st[0]["U"], a, st[0]["acc"], b, stream=stream)
        ps.rk_stage(0, M.MOL_RK4, 3, dt, st[0]["U"], b, st[0]["acc"], a, stream=stream)
        ps.rk_stage(0, M.MOL_RK4, 4, dt, st[0]["U"], a, st[0]["acc"], b, stream=stream)
    k1.record(stream)
    torch.cuda.synchronize()
    kms_alone = k0.elapsed_time(k1) / (4 * reps)
    # the same kernel inside the timed region: the K-step graph is 4 K stage
    # launches and one ghost fill, back to back; its event time minus the
    # fill's (timed alone) over the 4 K launches
    f0 = torch.cuda.Event(enable_timing=True)
    f1 = torch.cuda.Event(enable_timing=True)
    f0.record(stream)
    for _ in range(reps):
        ps.fill_ghosts(0, st[0]["U"], stream=stream)
    f1.record(stream)
    torch.cuda.synchronize()
    fill_ms = f0.elapsed_time(f1) / reps
    kms = (ms - fill_ms) / (4 * args.steps)
    gbs = CCZ4_BYTES_PER_PT_STAGE * pts / (kms * 1e-3) / 1e9
    log(f"bench: stage kernel {kms:.3f} ms avg in the timed region ({kms_alone:.3f} ms timed alone), "
        f"{gbs:.1f} GB/s algorithmic")

    # check the state stayed finite (robust-stability data)
    out = torch.zeros(5, dtype=torch.float64, device="cuda")
    ps.norms(0, st[0]["U"], 18, 1.0, 0.6, out, stream=stream)
    torch.cuda.synchronize()
    nonfinite = int(out[4].item())

    res = {
        "metric": METRIC,
        "value": value,
        "unit": "pt-stage/s",
        "n_gpus": 1,
        "steps": args.steps,
        "warmup": args.warmup,
        "ms_per_step": ms / args.steps,
        "seeds": {"median_seed": seed_med, "pt_stage_per_s": [pts * 4 * args.steps / (r[0] * 1e-3) for r in runs]},
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"ccz4_{n}^3_periodic_rk4_minkowski_noise1e-10", "points": pts,
                   "stages_per_step": 4, "graph": True, "steps_per_graph_launch": args.steps,
                   "nonfinite_after_run": nonfinite},
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "ccz4_stage_kernel", "kernel_ms": kms, "kernel_ms_alone": kms_alone,
                     "kernel_ms_from": "timed region: (K-step graph time - one ghost fill) / (4 K launches)",
                     "bytes_per_pt_stage": CCZ4_BYTES_PER_PT_STAGE},
    }
    rec = profile_record("ccz4_96", pts)
    if rec is not None:
        res["roofline"]["traffic"] = rec["hbm_bytes_per_launch"]
        # the same kernel against the FP64 vector peak, with the executed FP64
        # FLOP per point-stage from the counter record
        tf = rec["fp64_flop_per_pt_stage"] * pts / (kms * 1e-3) / 1e12
        res["roofline_fp64"] = {"bound": "alu", "achieved": tf, "peak": FP64_PEAK_TFLOPS, "unit": "TFLOP/s",
                                "frac": tf / FP64_PEAK_TFLOPS, "flop_per_pt_stage": rec["fp64_flop_per_pt_stage"],
                                "flop_count": "executed (SQ_INSTS_VALU_FLOPS_FP64 x 64 lanes)"}
    if not args.no_extras:
        log("bench: batched AMR hierarchy")
        res["amr_plain_vs_batched"] = amr_bench(M)
        if not args.no_fmr:
            log("bench: FMR reflections")
            res["fmr_reflections"] = fmr_bench(M)
            log("bench: MHD tests")
            res["mhd_runs"] = mhd_runs_bench(M)
            log("bench: AMR wave")
            res["amr_wave"] = amr_wave_bench(M)
        log("bench: single black hole")
        res["single_bh"] = single_bh_bench(M)
        log("bench: adjoint")
        res["adjoint"] = adjoint_bench(M)
        log("bench: wave and MHD paths")
        res["other_paths"] = wave_mhd_bench(M)
    if not args.no_cpu_baseline:
        log("bench: timing the CPU oracle sample")
        res["cpu_baseline"] = cpu_baseline(args.cpu_n)
        res["cpu_baseline"]["host_cpu"] = _cpu_name()
        res["cpu_baseline"]["nproc"] = os.cpu_count()
    print(json.dumps(res), flush=True)


def _cpu_name():
    try:
        for line in open("/proc/cpuinfo"):
            if line.startswith("model name"):
                return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


if __name__ == "__main__":
    main()
