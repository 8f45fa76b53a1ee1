"""The profile summary's per-linearisation totals: every pass of a GN
linearisation (certified search, queued search, term pass of either kind)
is counted, the gradient's term pass and other kernels are not, and the
totals are divided by the number of term passes."""
import csv
import io
import subprocess
import sys

COLS = ["Correlation_Id", "Dispatch_Id", "Agent_Id", "Queue_Id", "Process_Id", "Thread_Id",
        "Grid_Size", "Kernel_Id", "Kernel_Name", "Workgroup_Size", "LDS_Block_Size",
        "Scratch_Size", "VGPR_Count", "Accum_VGPR_Count", "SGPR_Count", "Counter_Name",
        "Counter_Value", "Start_Timestamp", "End_Timestamp"]
NS = "far::(anonymous namespace)::"
KERNELS = [  # (name, SQ_INSTS_VALU): only the first five belong to linearisations
    (f"void {NS}k_linearize<float, false, 256, false, false, true, false>(far::MapView)", 1000.0),
    (f"void {NS}k_cert<256, false>(far::MapView)", 100.0),
    (f"void {NS}k_search(far::MapView)", 10.0),
    (f"void {NS}k_linearize<float, false, 256, false, false, false, false>(far::MapView)", 1.0),
    (f"void {NS}k_reduce_solve(int)", 0.0),
    (f"void {NS}k_linearize<float, true, 256, false, false, true, false>(far::MapView)", 5e5),
    (f"void {NS}k_grid_cov<5>(far::GridView)", 7e5),
    ("__amd_rocclr_fillBufferAligned", 9e5),
]


def test_counters_take_every_linearisation_pass(tmp_path):
    buf = io.StringIO()
    w = csv.writer(buf, quoting=csv.QUOTE_NONNUMERIC)
    w.writerow(COLS)
    for d, (name, valu) in enumerate(KERNELS, 1):
        w.writerow([d, d, "Agent 1", 1, 1, 1, 256, d, name, 256, 0, 0, 8, 0, 16,
                    "SQ_INSTS_VALU", valu, 0, 1])
    p = tmp_path / "pmc_sq_256_counter_collection.csv"
    p.write_text(buf.getvalue())
    out = subprocess.run([sys.executable, "-m", "paper_2606_26010_amd.profsum", "counters", "256",
                          str(p)], capture_output=True, text=True, check=True).stdout
    vals = dict(line.split(" = ") for line in out.strip().splitlines())
    assert vals["linearisations"] == "2"                  # two term passes, not the gradient's
    assert float(vals["valu_insts"]) == (1000.0 + 100.0 + 10.0 + 1.0) / 2
