"""Summarize a rocprofv3 --kernel-trace --stats database into a short text table (times in us).

python -m paper_1607_03936_amd.profsummary <results.db> [top]
"""
from __future__ import annotations

import re
import sqlite3
import sys


def short(name: str) -> str:
    name = re.sub(r"wb::\(anonymous namespace\)::", "", name)
    name = re.sub(r"\(.*\)$", "", name)
    return name


def summarize(db: str, top: int = 30) -> str:
    con = sqlite3.connect(db)
    rows = con.execute("select name, total_calls, total_duration, average, percentage "
                       "from top_kernels").fetchall()
    total = sum(r[2] for r in rows)
    out = [f"{'kernel':<60} {'calls':>7} {'total_us':>11} {'avg_us':>9} {'%':>6}"]
    for n, c, t, a, p in rows[:top]:
        out.append(f"{short(n)[:60]:<60} {c:>7} {t:>11.1f} {a:>9.3f} {p:>6.2f}")
    out.append(f"{'TOTAL':<60} {sum(r[1] for r in rows):>7} {total:>11.1f}")
    return "\n".join(out)


if __name__ == "__main__":
    print(summarize(sys.argv[1], int(sys.argv[2]) if len(sys.argv) > 2 else 30))
