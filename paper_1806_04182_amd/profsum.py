"""Summaries of rocprofv3 output for the measurement record.

`python -m paper_1806_04182_amd.profsum <outdir> [<dest>]` reads the rocprofv3 CSV
folders written by the profiling commands listed in <outdir>/commands.json
(ktrace: the kernel trace of the benchmark; pmc_<COUNTER>_<case>: one counter
over `bench.py --profile-case <case>`, which runs only one workload's stage
kernel; copy_FETCH_SIZE, copy_WRITE_SIZE: a plain 1 GiB device copy) and
writes, under <dest> (default profiles/):

  stage_kernels_kernel_trace.md   per-kernel duration statistics
  stage_kernels_counters.md       HBM bytes and FP64 FLOP per dispatch of
                                  every workload's stage kernel
  <case record>.json              the record bench.py reads per workload
                                  (tied to the kernel sources by a hash)

HBM bytes: FETCH_SIZE and WRITE_SIZE (KiB per dispatch) scaled by the ratio
of the known size of the 1 GiB copy to what the same counter reads for it.
FP64 FLOP: SQ_INSTS_VALU_FLOPS_FP64 counts per wave instruction, so it is
multiplied by the 64 lanes of a wave.
"""
from __future__ import annotations

import collections
import csv
import hashlib
import json
import os
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
# host.cpp fixes the level layout (row pitches, alignment) and the default
# launch shapes, which change the bytes a stage kernel moves
COMMON = ("k_common.h", "molamr_int.h", "host.cpp")
CCZ4_SOURCES = ("k_ccz4.hip",) + COMMON
COPY_BYTES = 1 << 30
COUNTERS = ("FETCH_SIZE", "WRITE_SIZE", "SQ_INSTS_VALU_FLOPS_FP64")

# per workload: the stage kernel's name prefix, its points, the sources that
# determine it, the record file and a description
CASES = {
    "ccz4_96": {"prefix": "mol::ccz4_stage_kernel", "points": 96 ** 3, "sources": CCZ4_SOURCES,
                "file": "ccz4_stage_96cube_traffic.json", "workload": "ccz4 96^3 periodic patch, RK4 stages 1-4"},
    "wave_256": {"prefix": "mol::wave_", "points": 256 ** 3, "sources": ("k_wave.hip",) + COMMON,
                 "file": "wave_stage_256cube_traffic.json", "workload": "wave 256^3 periodic patch, RK4 stages 1-4"},
    "wave_512": {"prefix": "mol::wave_", "points": 512 ** 3, "sources": ("k_wave.hip",) + COMMON,
                 "file": "wave_stage_512cube_traffic.json", "workload": "wave 512^3 periodic patch, RK4 stages 1-4"},
    "mhd_128": {"prefix": "mol::mhd_stage_kernel", "points": 128 ** 3, "sources": ("k_mhd.hip",) + COMMON,
                "file": "mhd_stage_128cube_traffic.json",
                "workload": "mhd 128^3 periodic patch (WENO5-Z, LLF), SSP-RK3 stages 1-3"},
}


def source_hash(files) -> str:
    """Hash of the sources that determine a stage kernel."""
    h = hashlib.sha256()
    for f in files:
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


def ccz4_source_hash() -> str:
    return source_hash(CCZ4_SOURCES)


def _rows(folder):
    with open(os.path.join(folder, "run_counter_collection.csv")) as fh:
        return list(csv.DictReader(fh))


def _short(name: str) -> str:
    name = name.replace("(anonymous namespace)::", "")
    return name.split("(")[0] if not name.startswith("void") else name.split("(")[0][5:]


def counter_means(folder, counter):
    """{(kernel, grid size): (dispatches, mean counter value)}."""
    acc = collections.defaultdict(list)
    for r in _rows(folder):
        if r["Counter_Name"] == counter:
            acc[(_short(r["Kernel_Name"]), int(r["Grid_Size"]))].append(float(r["Counter_Value"]))
    return {k: (len(v), sum(v) / len(v)) for k, v in acc.items()}


def copy_scale(folder, counter, expect_kib):
    """Known KiB of the 1 GiB copy divided by the counter's reading for it."""
    best = None
    for (name, grid), (n, v) in counter_means(folder, counter).items():
        if "copy" in name.lower() or "elementwise" in name.lower():
            # the copy kernel is the one whose reading is largest
            if best is None or v > best:
                best = v
    return expect_kib / best


def kernel_trace_md(folder, cmd):
    """Per-kernel statistics, split by grid size (the same kernel runs on
    levels and patches of different sizes)."""
    with open(os.path.join(folder, "run_kernel_trace.csv")) as fh:
        rows = list(csv.DictReader(fh))
    acc = collections.defaultdict(list)
    for r in rows:
        grid = int(r["Grid_Size_X"]) * int(r["Grid_Size_Y"]) * int(r["Grid_Size_Z"])
        acc[(_short(r["Kernel_Name"]), grid)].append((int(r["End_Timestamp"]) - int(r["Start_Timestamp"])) / 1e3)
    total = sum(sum(v) for v in acc.values())
    out = ["# rocprofv3 kernel-trace summary of the benchmark", "", "Command (run from the repository root):",
           "", "    " + cmd, "",
           "Kernels of this library with at least 0.1% of the GPU time, by grid size (work-items).", "",
           "| kernel | grid | calls | avg (us) | min (us) | max (us) | share |", "|---|---|---|---|---|---|---|"]
    for (name, grid), v in sorted(acc.items(), key=lambda kv: -sum(kv[1])):
        if not name.startswith("mol::") or sum(v) < 1e-3 * total:
            continue
        out.append(f"| {name} | {grid} | {len(v)} | {sum(v) / len(v):.1f} | {min(v):.1f} | {max(v):.1f} | "
                   f"{100 * sum(v) / total:.2f}% |")
    return "\n".join(out) + "\n"


def main(outdir, prof=os.path.join(ROOT, "profiles")):
    os.makedirs(prof, exist_ok=True)
    cmds = json.load(open(os.path.join(outdir, "commands.json")))
    with open(os.path.join(prof, "stage_kernels_kernel_trace.md"), "w") as fh:
        fh.write(kernel_trace_md(os.path.join(outdir, "ktrace"), cmds["ktrace"]))
    fscale = copy_scale(os.path.join(outdir, "copy_FETCH_SIZE"), "FETCH_SIZE", COPY_BYTES / 1024)
    wscale = copy_scale(os.path.join(outdir, "copy_WRITE_SIZE"), "WRITE_SIZE", COPY_BYTES / 1024)
    lines = ["# HBM bytes and FP64 FLOP per dispatch of the stage kernels (rocprofv3 counters)", "",
             "Commands (one counter per run, each over `bench.py --profile-case <case>`, which times only that",
             "workload's stage kernel, 5 cycles of the scheme's stages after one warm-up cycle):", ""]
    lines += ["    " + cmds[k] for k in sorted(cmds) if k != "ktrace"]
    lines += ["", f"Copy calibration (1 GiB device copy): FETCH_SIZE scale {fscale:.3f}, "
                  f"WRITE_SIZE scale {wscale:.3f}.", "",
              "| case | kernel | grid | dispatches | HBM read (MB) | HBM write (MB) | B per point | FP64 FLOP per point |",
              "|---|---|---|---|---|---|---|---|"]
    records = {}
    for case, c in CASES.items():
        got = {}
        for ctr in COUNTERS:
            folder = os.path.join(outdir, f"pmc_{ctr}_{case}")
            if not os.path.isdir(folder):
                break
            got[ctr] = {k: v for k, v in counter_means(folder, ctr).items() if k[0].startswith(c["prefix"])}
        if len(got) != len(COUNTERS):
            continue
        # the stage kernel is the one dispatched most often in the case's run
        key = max(got["FETCH_SIZE"], key=lambda k: got["FETCH_SIZE"][k][0])
        n, fr = got["FETCH_SIZE"][key]
        wr = got["WRITE_SIZE"][key][1]
        fl = got["SQ_INSTS_VALU_FLOPS_FP64"][key][1] * 64
        rd_b, wr_b = fr * 1024 * fscale, wr * 1024 * wscale
        pts = c["points"]
        lines.append(f"| {case} | {key[0]} | {key[1]} | {n} | {rd_b / 1e6:.1f} | {wr_b / 1e6:.1f} | "
                     f"{(rd_b + wr_b) / pts:.1f} | {fl / pts:.1f} |")
        rec = {"kernel": key[0], "grid": key[1], "workload": c["workload"], "points": pts,
               "source_sha256": source_hash(c["sources"]), "dispatches": n,
               "fetch_kib_per_dispatch_raw": fr, "write_kib_per_dispatch_raw": wr,
               "fetch_scale": fscale, "write_scale": wscale,
               "hbm_bytes_per_launch": rd_b + wr_b,
               "fp64_flop_per_launch": fl, "fp64_flop_per_pt_stage": fl / pts,
               "command": cmds.get(f"FETCH_SIZE_{case}", "")}
        with open(os.path.join(prof, c["file"]), "w") as fh:
            json.dump(rec, fh, indent=1)
        records[case] = rec
    with open(os.path.join(prof, "stage_kernels_counters.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    print(json.dumps(records, indent=1))


if __name__ == "__main__":
    main(*sys.argv[1:3])
