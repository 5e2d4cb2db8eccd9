"""The rocprofv3 summariser on synthetic CSV output: counter means per kernel
and grid, the copy calibration, the per-workload records (bytes scaled by
the calibration, FLOP times 64 lanes, the source hash), the kernel-trace
table, and the benchmark's check that a record is tied to the current
sources."""
import csv
import json
import os

from paper_1806_04182_amd import profsum as P

COLS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id", "Grid_Size",
        "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size", "Scratch_Size", "VGPR_Count",
        "Accum_VGPR_Count", "SGPR_Count", "Counter_Name", "Counter_Value", "Start_Timestamp", "End_Timestamp"]


def _pmc(folder, counter, rows):
    os.makedirs(folder)
    with open(os.path.join(folder, "run_counter_collection.csv"), "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(COLS)
        for k, (name, grid, value) in enumerate(rows):
            w.writerow([k, k, "Agent 1", 1, 1, 1, grid, 1, name, 256, 0, 0, 128, 0, 32, counter, value, 0, 1])


def _trace(folder, rows):
    os.makedirs(folder)
    with open(os.path.join(folder, "run_kernel_trace.csv"), "w", newline="") as fh:
        w = csv.writer(fh)
        w.writerow(["Kernel_Name", "Grid_Size_X", "Grid_Size_Y", "Grid_Size_Z", "Start_Timestamp", "End_Timestamp"])
        for name, grid, t0, t1 in rows:
            w.writerow([name, grid, 1, 1, t0, t1])


def test_records_and_tables(tmp_path):
    out = tmp_path / "prof"
    ccz4 = "void mol::(anonymous namespace)::ccz4_stage_kernel<8, 8, 4, true>(mol::StageArgs)"
    fill = "mol::(anonymous namespace)::fill_kernel(mol::GhostCopy const*, long, int, double*)"
    copy = "void at::native::elementwise_copy_kernel(int)"
    pts = P.CASES["ccz4_96"]["points"]
    # the stage kernel four times (the most frequent), the fill once
    _pmc(str(out / "pmc_FETCH_SIZE_ccz4_96"), "FETCH_SIZE", [(ccz4, pts, 100.0)] * 3 + [(ccz4, pts, 140.0)] +
         [(fill, 999, 5.0)])
    _pmc(str(out / "pmc_WRITE_SIZE_ccz4_96"), "WRITE_SIZE", [(ccz4, pts, 50.0)] * 4 + [(fill, 999, 1.0)])
    _pmc(str(out / "pmc_SQ_INSTS_VALU_FLOPS_FP64_ccz4_96"), "SQ_INSTS_VALU_FLOPS_FP64", [(ccz4, pts, 1000.0)] * 4)
    # a 1 GiB copy that the counters read as half (fetch) and exactly (write)
    _pmc(str(out / "copy_FETCH_SIZE"), "FETCH_SIZE", [(copy, 1, (1 << 30) / 1024 / 2)])
    _pmc(str(out / "copy_WRITE_SIZE"), "WRITE_SIZE", [(copy, 1, (1 << 30) / 1024)])
    _trace(str(out / "ktrace"), [(ccz4, pts, 0, 500_000), (ccz4, pts, 600_000, 1_000_000), (fill, 999, 0, 10_000)])
    cmds = {"ktrace": "rocprofv3 --kernel-trace ...", "FETCH_SIZE_ccz4_96": "rocprofv3 --pmc FETCH_SIZE ..."}
    (out / "commands.json").write_text(json.dumps(cmds))
    dest = tmp_path / "summary"
    P.main(str(out), str(dest))
    rec = json.loads((dest / P.CASES["ccz4_96"]["file"]).read_text())
    assert rec["dispatches"] == 4 and rec["grid"] == pts
    assert rec["fetch_scale"] == 2.0 and rec["write_scale"] == 1.0
    assert rec["hbm_bytes_per_launch"] == (110.0 * 1024 * 2.0 + 50.0 * 1024)
    assert rec["fp64_flop_per_launch"] == 64000.0
    assert rec["fp64_flop_per_pt_stage"] == 64000.0 / pts
    assert rec["source_sha256"] == P.source_hash(P.CASES["ccz4_96"]["sources"]) == P.ccz4_source_hash()
    # cases without counter folders get no record
    assert not (dest / P.CASES["mhd_128"]["file"]).exists()
    trace = (dest / "stage_kernels_kernel_trace.md").read_text()
    line = [l for l in trace.splitlines() if l.startswith("| mol::ccz4_stage_kernel")][0]
    assert "| 2 | 450.0 | 400.0 | 500.0 |" in line
    assert "rocprofv3 --kernel-trace" in trace
    table = (dest / "stage_kernels_counters.md").read_text()
    assert "| ccz4_96 | mol::ccz4_stage_kernel<8, 8, 4, true> |" in table
