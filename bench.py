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


def cpu_baseline(n=24, seconds_hint=20.0):
    """The oracle (single-threaded C) on a bounded sample of the same workload:
    one RK4 step of an n^3 periodic patch with the same data recipe."""
    import numpy as np
    from oracle import oracle as O
    from paper_1806_04182_amd import synth
    dx = 2.0 / 96
    U = synth.embed(synth.ccz4_minkowski_noise((n, n, n), amp=1e-10, seed=0))
    t0 = time.perf_counter()
    O.rk_run(O.CCZ4, O.RK4, U, dx, 0.25 * dx, 1, O.params())
    dt = time.perf_counter() - t0
    return {"value": n ** 3 * 4 / dt, "unit": "pt-stage/s", "cores": 1, "kind": "oracle",
            "sample": f"one RK4 step (4 stages) of a {n}^3 periodic CCZ4 patch, same data recipe, "
                      f"{dt:.1f} s wall on one host core"}


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=20)
    ap.add_argument("--warmup", type=int, default=3)
    ap.add_argument("--n", type=int, default=96)
    ap.add_argument("--no-cpu-baseline", action="store_true")
    ap.add_argument("--cpu-n", type=int, default=24)
    args = ap.parse_args()
    if args.gpus != 1:
        print("bench.py measures one GPU: this build has no multi-GPU path "
              "(run with --gpus 1)", file=sys.stderr)
        sys.exit(2)

    log("bench: importing torch")
    import numpy as np
    import torch
    from paper_1806_04182_amd import molamr as M
    from paper_1806_04182_amd import synth

    assert torch.cuda.is_available(), "no GPU"
    n = args.n
    dx = 2.0 / n
    dt = 0.25 * dx
    ps = M.Patchset(M.single_patch((n, n, n), (-1, -1, -1), dx), M.System(M.MOL_CCZ4))
    log(f"bench: patchset {n}^3 built")
    st = ps.alloc_states()
    st[0]["U"].copy_(torch.from_numpy(ps.pack(0, [synth.embed(synth.ccz4_minkowski_noise((n, n, n), amp=1e-10, seed=0))])))
    U0 = st[0]["U"].clone()
    g = ps.graph_create(st, dt)
    stream = torch.cuda.current_stream()
    for _ in range(args.warmup):
        g.launch(stream)
    torch.cuda.synchronize()
    log("bench: warmup done")
    t0 = time.perf_counter()
    e0 = torch.cuda.Event(enable_timing=True)
    e1 = torch.cuda.Event(enable_timing=True)
    e0.record(stream)
    for _ in range(args.steps):
        g.launch(stream)
    e1.record(stream)
    torch.cuda.synchronize()
    wall = time.perf_counter() - t0
    ms = e0.elapsed_time(e1)
    log(f"bench: {args.steps} steps in {ms:.2f} ms (events), {wall * 1e3:.2f} ms (wall)")
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
    kms = k0.elapsed_time(k1) / (4 * reps)
    gbs = CCZ4_BYTES_PER_PT_STAGE * pts / (kms * 1e-3) / 1e9
    log(f"bench: stage kernel {kms:.3f} ms avg, {gbs:.1f} GB/s algorithmic")

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
        "higher_is_better": True,
        "scaling": "weak",
        "vs_baseline": None,
        "dtype": "f64",
        "data": "synthetic",
        "config": {"workload": f"ccz4_{n}^3_periodic_rk4_minkowski_noise1e-10", "points": pts,
                   "stages_per_step": 4, "graph": True, "nonfinite_after_run": nonfinite},
        "roofline": {"bound": "hbm", "achieved": gbs, "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": gbs / HBM_PEAK_GBS, "traffic": None,
                     "kernel": "ccz4_stage_kernel", "kernel_ms": kms,
                     "bytes_per_pt_stage": CCZ4_BYTES_PER_PT_STAGE},
    }
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
