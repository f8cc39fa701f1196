"""HBM traffic per launch from rocprofv3 counter runs of opbench.py (FETCH_SIZE and WRITE_SIZE in
separate runs), calibrated against the plain device copy of the same run.

python -m paper_1607_03936_amd.trafficsummary <out.json> <workload> <fetch.csv> <write.csv> [...]

Each workload names the counter_collection.csv of its FETCH_SIZE run and of its WRITE_SIZE run
(opbench.py <workload> <reps> copy).  The copy leg moves a known number of bytes (the velocity
vector, read once and written once), so bytes / counter gives each counter's unit; the factors of
all workloads are averaged.  An A apply is two kernels (the brick scatter, on the matrix cores or
with LDS lines, and its face sums, or the element pass and its node sums); prints a text summary
of both and writes the per-apply bytes of the pair to <out.json>, keyed like bench.py's kernel
keys, with the source hash of the kernels the counters were taken on.
"""
from __future__ import annotations

import csv
import hashlib
import json
import os
import re
import sys
from collections import defaultdict

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
sys.path.insert(0, ROOT)

A_KERNEL = re.compile(r"k_op_(brick|elem)<\d, 3, double, 9, 0, 0>|k_op_(mfma)<3, double, 9, 0>")
FACE_KERNEL = re.compile(r"k_(face|node)_sum<(\d), 3, double, true, 0>")


def source_hash() -> str:
    h = hashlib.sha256()
    for f in ("kernels.hip", "rules.h", "kernels.h"):
        with open(os.path.join(ROOT, "paper_1607_03936_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def read(path):
    """{kernel class: [counter value per dispatch]}, plus the copy dispatches as (grid, value)."""
    per = defaultdict(list)
    names = {}
    copies = []
    with open(path, newline="") as fh:
        for row in csv.DictReader(fh):
            name, val = row["Kernel_Name"], float(row["Counter_Value"])
            if "copyBuffer" in name:
                copies.append((int(row["Grid_Size"]), val))
            elif A_KERNEL.search(name):
                per["A"].append(val)
                mt = A_KERNEL.search(name)
                names["A"] = mt.group(1) or mt.group(2)
            elif FACE_KERNEL.search(name):
                per["face"].append(val)
                names["face"] = FACE_KERNEL.search(name).group(1)
    per["names"] = names
    return per, copies


def copy_kib(copies):
    """Counter value per full-vector copy: the dispatches with the largest grid."""
    g = max(c[0] for c in copies)
    vals = [v for gs, v in copies if gs == g]
    return sum(vals) / len(vals)


def main(argv):
    out = argv[0]
    rest = argv[1:]
    assert len(rest) % 3 == 0, "expected <workload> <fetch.csv> <write.csv> triples"
    from synthetic import WORKLOADS
    rows, ff, fw = [], [], []
    for i in range(0, len(rest), 3):
        name, fcsv, wcsv = rest[i:i + 3]
        w = WORKLOADS[name]
        M = w.k * w.N + 1
        u_dof = 3 * M ** 3
        nq = w.N ** 3 * (w.k + 1) ** 3
        fper, fcop = read(fcsv)
        wper, wcop = read(wcsv)
        vec_kib = 8 * u_dof / 1024
        ff.append(vec_kib / copy_kib(fcop))
        fw.append(vec_kib / copy_kib(wcop))
        rows.append((name, w, u_dof, nq, fper, wper))
    kf, kw = sum(ff) / len(ff), sum(fw) / len(fw)
    print(f"# calibration: FETCH_SIZE x {kf:.3f}, WRITE_SIZE x {kw:.3f} (KiB per dispatch; "
          f"per workload {', '.join(f'{a:.3f}/{b:.3f}' for a, b in zip(ff, fw))})")
    print(f"# kernel sources: hash {source_hash()}")
    print(f"{'workload':<10} {'kernel':<30} {'disp':>5} {'FETCH KiB':>10} {'WRITE KiB':>10} "
          f"{'read MB':>9} {'write MB':>9} {'traffic MB':>10} {'algo MB':>9} {'ratio':>6}")
    kernels = {}
    for name, w, u_dof, nq, fper, wper in rows:
        algo = 8.0 * (2 * u_dof + nq)
        tot = {"fetch_kib": 0.0, "write_kib": 0.0, "bytes": 0.0}
        form = fper["names"].get("A", "brick")
        for cls in ("A", "face"):
            if not fper.get(cls) or not wper.get(cls):
                continue
            fk = sum(fper[cls]) / len(fper[cls])
            wk = sum(wper[cls]) / len(wper[cls])
            rd, wr = fk * kf * 1024, wk * kw * 1024
            tot["fetch_kib"] += fk
            tot["write_kib"] += wk
            tot["bytes"] += rd + wr
            if cls == "A":
                label = (f"k_op_mfma<3,double,9,0>" if form == "mfma"
                         else f"k_op_{form}<{w.k + 1},3,double,9,0,0>")
            else:
                label = f"k_{fper['names'].get('face', 'face')}_sum (same applies)"
            print(f"{name:<10} {label:<30} {len(fper[cls]):>5} {fk:>10.0f} {wk:>10.0f} {rd / 1e6:>9.2f} "
                  f"{wr / 1e6:>9.2f} {(rd + wr) / 1e6:>10.2f} {'':>9} {'':>6}")
        print(f"{name:<10} {'whole apply (both kernels)':<30} {'':>5} {tot['fetch_kib']:>10.0f} "
              f"{tot['write_kib']:>10.0f} {'':>9} {'':>9} {tot['bytes'] / 1e6:>10.2f} {algo / 1e6:>9.2f} "
              f"{tot['bytes'] / algo:>6.2f}")
        key = f"op nc=3 k={w.k} N={w.N} flags=A+dir f64"
        kernels[key] = {"fetch_kib": round(tot["fetch_kib"]), "write_kib": round(tot["write_kib"]),
                        "bytes_per_launch": round(tot["bytes"])}
    rec = {"source_hash": source_hash(),
           "calibration": {"FETCH_SIZE": round(kf, 3), "WRITE_SIZE": round(kw, 3),
                           "reference": "device copy of the velocity vector (opbench.py copy leg)"},
           "kernels": kernels}
    with open(out, "w") as fh:
        json.dump(rec, fh, indent=1)
        fh.write("\n")


if __name__ == "__main__":
    main(sys.argv[1:])
