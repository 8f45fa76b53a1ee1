"""Summaries of rocprofv3 runs of the benchmark (kernel trace and counters).

    python -m paper_2606_26010_amd.profsum trace <kernel_stats.csv>
    python -m paper_2606_26010_amd.profsum counters <tile> <counter_collection.csv>...
    python -m paper_2606_26010_amd.profsum kernel <name prefix> <counter_collection.csv>...

`trace` prints calls, total and average duration per kernel.  `counters`
prints, per GN-iteration linearisation of the batched align (its passes
k_cert, k_search and the term pass k_linearize), the totals of
every counter the given runs collected, divided by the number of
linearisations (term-pass dispatches), with the bytes moved between the L2
and the fabric (Infinity Cache and HBM) from the request-size counters:
read = 32 RDREQ_32B + 64 RDREQ_64B + 128 RDREQ_128B, write = 64 WRREQ_64B +
32 (WRREQ - WRREQ_64B).  The output is the key = value form bench.py reads.
"""
import collections
import csv
import hashlib
import os
import re
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
ROOT = os.path.dirname(HERE)
KERNEL_SOURCES = ["paper_2606_26010_amd/csrc/far_gicp.hip", "paper_2606_26010_amd/csrc/far_knn.h",
                  "paper_2606_26010_amd/csrc/far_internal.h"]
LIN_PASSES = ("k_cert<", "k_search", "k_linearize<")


def short(name):
    n = name.replace("void ", "").replace("far::(anonymous namespace)::", "")
    return re.sub(r"\(.*", "", n)


def fingerprint():
    h = hashlib.sha256()
    for f in KERNEL_SOURCES:
        with open(os.path.join(ROOT, f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def trace(path):
    rows = list(csv.DictReader(open(path)))
    print(f"{'kernel':70s} {'calls':>6s} {'total_ms':>10s} {'avg_us':>10s} {'pct':>6s}")
    for r in rows:
        print(f"{short(r['Name'])[:70]:70s} {int(r['Calls']):6d} "
              f"{float(r['TotalDurationNs']) / 1e6:10.3f} {float(r['AverageNs']) / 1e3:10.2f} "
              f"{float(r['Percentage']):6.2f}")


def counters(tile, paths):
    tot = collections.defaultdict(float)
    n_lin = {}
    for p in paths:
        lin = set()
        for r in csv.DictReader(open(p)):
            k = short(r["Kernel_Name"])
            if not k.startswith(LIN_PASSES):
                continue
            if k.startswith("k_linearize<"):
                targs = [a.strip() for a in k[k.index("<") + 1:k.rindex(">")].split(",")]
                if targs[1] != "false":     # the gradient's term pass is no linearisation
                    continue
                lin.add(r["Dispatch_Id"])
            tot[r["Counter_Name"]] += float(r["Counter_Value"])
        n_lin[p] = len(lin)
    n = max(n_lin.values()) if n_lin else 0
    if n == 0 or len(set(n_lin.values())) != 1:
        sys.exit(f"linearisation counts differ between runs or are zero: {n_lin}")
    per = {k: v / n for k, v in tot.items()}
    out = {"kernel_sources_sha256_16": fingerprint(), "tile": str(tile),
           "kernels": "k_cert+k_search+k_linearize", "linearisations": n}
    g = per.get
    if "TCC_EA0_RDREQ_128B_sum" in per:
        out["fabric_read_bytes"] = (32 * g("TCC_EA0_RDREQ_32B_sum", 0) +
                                    64 * g("TCC_EA0_RDREQ_64B_sum", 0) +
                                    128 * g("TCC_EA0_RDREQ_128B_sum", 0))
    if "TCC_EA0_WRREQ_sum" in per:
        w64 = g("TCC_EA0_WRREQ_64B_sum", 0)
        out["fabric_write_bytes"] = 64 * w64 + 32 * (g("TCC_EA0_WRREQ_sum") - w64)
    names = {"TCC_HIT_sum": "tcc_hit", "TCC_MISS_sum": "tcc_miss", "SQ_INSTS_VALU": "valu_insts",
             "SQ_INSTS_SALU": "salu_insts", "SQ_INSTS_LDS": "lds_insts",
             "SQ_INSTS_VMEM_RD": "vmem_rd_insts", "SQ_INSTS_VMEM_WR": "vmem_wr_insts",
             "SQ_WAVES": "waves", "SQ_WAVE_CYCLES": "wave_cycles",
             "SQ_BUSY_CU_CYCLES": "busy_cu_cycles", "FETCH_SIZE": "fetch_size_kib",
             "WRITE_SIZE": "write_size_kib"}
    for c, v in sorted(per.items()):
        out[names.get(c, c.lower())] = v
    for k, v in out.items():
        print(f"{k} = {v:.1f}" if isinstance(v, float) else f"{k} = {v}")


def kernel(prefix, paths):
    """Per-dispatch averages of every counter of the kernels whose name
    starts with prefix, with the L2-to-fabric bytes as in counters()."""
    tot = collections.defaultdict(float)
    n_disp = {}
    for p in paths:
        disp = set()
        for r in csv.DictReader(open(p)):
            if short(r["Kernel_Name"]).startswith(prefix):
                disp.add(r["Dispatch_Id"])
                tot[r["Counter_Name"]] += float(r["Counter_Value"])
        n_disp[p] = len(disp)
    n = max(n_disp.values()) if n_disp else 0
    if n == 0 or len(set(n_disp.values())) != 1:
        sys.exit(f"dispatch counts differ between runs or are zero: {n_disp}")
    per = {k: v / n for k, v in tot.items()}
    print(f"kernel = {prefix}")
    print(f"dispatches = {n}")
    g = per.get
    if "TCC_EA0_RDREQ_128B_sum" in per:
        print(f"fabric_read_bytes = {32 * g('TCC_EA0_RDREQ_32B_sum', 0) + 64 * g('TCC_EA0_RDREQ_64B_sum', 0) + 128 * g('TCC_EA0_RDREQ_128B_sum', 0):.1f}")
    if "TCC_EA0_WRREQ_sum" in per:
        w64 = g("TCC_EA0_WRREQ_64B_sum", 0)
        print(f"fabric_write_bytes = {64 * w64 + 32 * (g('TCC_EA0_WRREQ_sum') - w64):.1f}")
    for c, v in sorted(per.items()):
        print(f"{c.lower()} = {v:.1f}")


def main(argv):
    if len(argv) >= 2 and argv[0] == "trace":
        trace(argv[1])
    elif len(argv) >= 3 and argv[0] == "counters":
        counters(int(argv[1]), argv[2:])
    elif len(argv) >= 3 and argv[0] == "kernel":
        kernel(argv[1], argv[2:])
    else:
        sys.exit(__doc__)


if __name__ == "__main__":
    main(sys.argv[1:])
