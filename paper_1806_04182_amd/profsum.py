"""Summaries of rocprofv3 output for the measurement record.

`python -m paper_1806_04182_amd.profsum <outdir>` reads the rocprofv3 CSV
folders written by the profiling commands listed in the generated files
(under <outdir>: ktrace; pmc_FETCH_SIZE, pmc_WRITE_SIZE, pmc_FLOPS for the
CCZ4 benchmark and the same with suffix _paths for the wave and MHD paths;
copy_FETCH_SIZE, copy_WRITE_SIZE) and writes, under profiles/:

  stage_kernels_kernel_trace.md   per-kernel duration statistics
  stage_kernels_counters.md       HBM bytes and FP64 FLOP per dispatch,
                                  grouped by kernel and grid size
  ccz4_stage_96cube_traffic.json  the record bench.py reads for the CCZ4
                                  stage kernel (tied to the kernel sources
                                  by a hash)

HBM bytes: FETCH_SIZE and WRITE_SIZE (KiB per dispatch) scaled by the ratio
of the known size of a plain 1 GiB device copy to what the same counter
reads for it.  FP64 FLOP: SQ_INSTS_VALU_FLOPS_FP64 counts per wave
instruction, so it is multiplied by the 64 lanes of a wave.
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
CCZ4_SOURCES = ("k_ccz4.hip", "k_common.h", "molamr_int.h")
COPY_BYTES = 1 << 30
CCZ4_POINTS = 96 ** 3


def ccz4_source_hash() -> str:
    """Hash of the sources that determine the CCZ4 stage kernel."""
    h = hashlib.sha256()
    for f in CCZ4_SOURCES:
        with open(os.path.join(HERE, "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()


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


def main(outdir):
    prof = os.path.join(ROOT, "profiles")
    cmds = json.load(open(os.path.join(outdir, "commands.json")))
    with open(os.path.join(prof, "stage_kernels_kernel_trace.md"), "w") as fh:
        fh.write(kernel_trace_md(os.path.join(outdir, "ktrace"), cmds["ktrace"]))
    fscale = copy_scale(os.path.join(outdir, "copy_FETCH_SIZE"), "FETCH_SIZE", COPY_BYTES / 1024)
    wscale = copy_scale(os.path.join(outdir, "copy_WRITE_SIZE"), "WRITE_SIZE", COPY_BYTES / 1024)
    fetch, write, flops = {}, {}, {}
    for tag in ("", "_paths"):
        fetch.update(counter_means(os.path.join(outdir, "pmc_FETCH_SIZE" + tag), "FETCH_SIZE"))
        write.update(counter_means(os.path.join(outdir, "pmc_WRITE_SIZE" + tag), "WRITE_SIZE"))
        flops.update(counter_means(os.path.join(outdir, "pmc_FLOPS" + tag), "SQ_INSTS_VALU_FLOPS_FP64"))
    lines = ["# HBM bytes and FP64 FLOP per dispatch (rocprofv3 counters)", "", "Commands (one counter per run):", ""]
    lines += ["    " + cmds[k] for k in ("fetch", "write", "flops", "fetch_paths", "write_paths", "flops_paths",
                                          "copy_fetch", "copy_write")]
    lines += ["", f"Copy calibration (1 GiB device copy): FETCH_SIZE scale {fscale:.3f}, WRITE_SIZE scale {wscale:.3f}.",
              "", "| kernel | grid | dispatches | HBM read (MB) | HBM write (MB) | FP64 GFLOP |", "|---|---|---|---|---|---|"]
    for key in sorted(set(fetch) | set(write) | set(flops)):
        if key[0].startswith("at::") or "rocclr" in key[0]:
            continue
        n = fetch.get(key, (0, 0))[0]
        rd = fetch.get(key, (0, float("nan")))[1] * 1024 * fscale / 1e6
        wr = write.get(key, (0, float("nan")))[1] * 1024 * wscale / 1e6
        fl = flops.get(key, (0, float("nan")))[1] * 64 / 1e9
        lines.append(f"| {key[0]} | {key[1]} | {n} | {rd:.1f} | {wr:.1f} | {fl:.3f} |")
    with open(os.path.join(prof, "stage_kernels_counters.md"), "w") as fh:
        fh.write("\n".join(lines) + "\n")
    # the CCZ4 96^3 stage kernel: its grid is the tile count of one 96^3 patch
    ck = [k for k in fetch if k[0].startswith("mol::ccz4_stage_kernel") and k[1] == CCZ4_POINTS]
    assert len(ck) == 1, ck
    k = ck[0]
    rec = {
        "kernel": k[0], "workload": "ccz4 96^3 periodic patch, RK4 stages 1-4", "points": CCZ4_POINTS,
        "source_sha256": ccz4_source_hash(), "dispatches": fetch[k][0],
        "fetch_kib_per_dispatch_raw": fetch[k][1], "write_kib_per_dispatch_raw": write[k][1],
        "fetch_scale": fscale, "write_scale": wscale,
        "hbm_bytes_per_launch": fetch[k][1] * 1024 * fscale + write[k][1] * 1024 * wscale,
        "fp64_flop_per_launch": flops[k][1] * 64,
        "fp64_flop_per_pt_stage": flops[k][1] * 64 / CCZ4_POINTS,
    }
    with open(os.path.join(prof, "ccz4_stage_96cube_traffic.json"), "w") as fh:
        json.dump(rec, fh, indent=1)
    print(json.dumps(rec, indent=1))


if __name__ == "__main__":
    main(sys.argv[1])
