"""Stand-alone operator timing for profiling runs: repeated A(mu) applies on a workload.

python -m paper_1607_03936_amd.opbench <workload> <reps> [copy]
The optional `copy` leg runs a plain device copy of the velocity vector (calibration of
hardware byte counters against a kernel of known traffic)."""
from __future__ import annotations

import os
import sys
import time

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))


def main():
    import torch

    from paper_1607_03936_amd import wbfbt as wb
    from synthetic import WORKLOADS
    w = WORKLOADS[sys.argv[1]]
    reps = int(sys.argv[2])
    m = wb.Mesh(w.N, w.k)
    v = wb.Viscosity.sinker(m, w.centers(), w.delta, w.omega, w.mu_min, w.mu_max)
    x = torch.rand(m.u_len, dtype=torch.float64, device="cuda")
    y = torch.empty_like(x)
    for _ in range(3):
        wb.wb_apply_A(m, v, x, y)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        wb.wb_apply_A(m, v, x, y)
    torch.cuda.synchronize()
    dt = (time.perf_counter() - t0) / reps
    print(f"{sys.argv[1]}: {reps} A applies, {dt * 1e6:.1f} us each (wall, incl. face pass)", flush=True)
    if len(sys.argv) > 3 and sys.argv[3] == "copy":
        z = torch.empty_like(x)
        for _ in range(reps):
            z.copy_(x)
        torch.cuda.synchronize()
        print(f"copy of {x.numel() * 8} bytes x {reps}", flush=True)


if __name__ == "__main__":
    main()
