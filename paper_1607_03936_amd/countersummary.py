"""Per-kernel averages of rocprofv3 counter runs (--pmc, one counter set per run) and the derived
utilization figures.

python -m paper_1607_03936_amd.countersummary <kernel regex> <counter_collection.csv> [...]

For every kernel whose name matches the regex: dispatches, mean duration and the mean value of
each counter per dispatch over all given runs, then
  MFMA busy %     100 SQ_VALU_MFMA_BUSY_CYCLES / (GRBM_GUI_ACTIVE / 8 XCDs x 256 CUs x 4 SIMDs)
                  (GRBM_GUI_ACTIVE is reported summed over the eight XCDs)
  FP64 MFMA rate  512 SQ_INSTS_VALU_MFMA_MOPS_F64 flops / duration, against 78.6 TFLOP/s
  BF16 MFMA rate  512 SQ_INSTS_VALU_MFMA_MOPS_BF16 flops / duration, against 2500 TFLOP/s (dense)
  LDS conflict %  100 SQ_LDS_BANK_CONFLICT / SQ_LDS_IDX_ACTIVE
  L2 hit %        100 TCC_HIT_sum / (TCC_HIT_sum + TCC_MISS_sum)
"""
from __future__ import annotations

import csv
import re
import sys
from collections import defaultdict

XCDS, CUS, SIMDS = 8, 256, 4
F64_PEAK_TFLOPS = 78.6
BF16_PEAK_TFLOPS = 2500.0


def short(name: str) -> str:
    name = re.sub(r"wb::\(anonymous namespace\)::", "", name)
    return re.sub(r"\(.*\)$", "", name).replace("void ", "")


def collect(pattern: str, paths):
    rx = re.compile(pattern)
    vals = defaultdict(lambda: defaultdict(list))   # kernel -> counter -> values
    durs = defaultdict(dict)                        # kernel -> (file, dispatch) -> ns
    for path in paths:
        with open(path, newline="") as fh:
            for row in csv.DictReader(fh):
                name = row["Kernel_Name"]
                if not rx.search(name):
                    continue
                k = short(name)
                vals[k][row["Counter_Name"]].append(float(row["Counter_Value"]))
                durs[k][(path, row["Dispatch_Id"])] = (int(row["End_Timestamp"]) -
                                                       int(row["Start_Timestamp"]))
    return vals, durs


def mean(v):
    return sum(v) / len(v) if v else float("nan")


def summarize(pattern: str, paths) -> str:
    vals, durs = collect(pattern, paths)
    out = []
    for k in sorted(vals):
        c = {n: mean(v) for n, v in vals[k].items()}
        dur_ns = mean(list(durs[k].values()))
        out.append(f"{k}: {len(durs[k])} dispatches over the runs, mean duration {dur_ns / 1e3:.1f} us")
        for n in sorted(c):
            out.append(f"  {n:<32} {c[n]:>16.1f}  per dispatch")
        if c.get("SQ_VALU_MFMA_BUSY_CYCLES") and "GRBM_GUI_ACTIVE" in c:
            cyc = c["GRBM_GUI_ACTIVE"] / XCDS
            out.append(f"  MFMA busy                        {100 * c['SQ_VALU_MFMA_BUSY_CYCLES'] / (cyc * CUS * SIMDS):>15.1f} %")
        if c.get("SQ_INSTS_VALU_MFMA_MOPS_F64"):
            tf = 512 * c["SQ_INSTS_VALU_MFMA_MOPS_F64"] / dur_ns / 1e3
            out.append(f"  FP64 MFMA rate                   {tf:>15.2f} TFLOP/s "
                       f"({100 * tf / F64_PEAK_TFLOPS:.1f} % of {F64_PEAK_TFLOPS})")
        if c.get("SQ_INSTS_VALU_MFMA_MOPS_BF16"):
            tb = 512 * c["SQ_INSTS_VALU_MFMA_MOPS_BF16"] / dur_ns / 1e3
            out.append(f"  BF16 MFMA rate                   {tb:>15.2f} TFLOP/s "
                       f"({100 * tb / BF16_PEAK_TFLOPS:.2f} % of {BF16_PEAK_TFLOPS:g})")
        if "SQ_LDS_BANK_CONFLICT" in c and c.get("SQ_LDS_IDX_ACTIVE"):
            out.append(f"  LDS bank conflict                {100 * c['SQ_LDS_BANK_CONFLICT'] / c['SQ_LDS_IDX_ACTIVE']:>15.1f} % of LDS cycles")
        if "TCC_HIT_sum" in c and "TCC_MISS_sum" in c:
            h, m = c["TCC_HIT_sum"], c["TCC_MISS_sum"]
            out.append(f"  L2 hit                           {100 * h / (h + m):>15.1f} %")
    return "\n".join(out)


if __name__ == "__main__":
    print(summarize(sys.argv[1], sys.argv[2:]))
