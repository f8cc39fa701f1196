"""Stand-alone operator timing for profiling runs: repeated A(mu) applies on a workload.

python -m paper_1607_03936_amd.opbench <workload> <reps> [copy] [fp32|bf16x3|bf16x1]
The optional `copy` leg runs a plain device copy of the velocity vector (calibration of
hardware byte counters against a kernel of known traffic); a precision name applies the
reduced-precision A (FP32 buffers; the BF16 forms contract on the matrix cores) instead of the
FP64 one."""
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
    extra = sys.argv[3:]
    prec = {"fp32": wb.WB_FP32, "bf16x3": wb.WB_BF16, "bf16x1": wb.WB_BF16X1}
    form = next((a for a in extra if a in prec), None)
    m = wb.Mesh(w.N, w.k)
    v = wb.Viscosity.sinker(m, w.centers(), w.delta, w.omega, w.mu_min, w.mu_max)
    dt = torch.float64 if form is None else torch.float32
    x = torch.rand(m.u_len, dtype=dt, device="cuda")
    y = torch.empty_like(x)

    def apply():
        if form is None:
            wb.wb_apply_A(m, v, x, y)
        else:
            wb.wb_apply_A_lowp(m, v, prec[form], x, y)
    for _ in range(3):
        apply()
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    for _ in range(reps):
        apply()
    torch.cuda.synchronize()
    dt_s = (time.perf_counter() - t0) / reps
    print(f"{sys.argv[1]} {form or 'fp64'}: {reps} A applies, {dt_s * 1e6:.1f} us each (wall, incl. face pass)",
          flush=True)
    if "copy" in extra:
        z = torch.empty_like(x)
        for _ in range(reps):
            z.copy_(x)
        torch.cuda.synchronize()
        print(f"copy of {x.numel() * x.element_size()} bytes x {reps}", flush=True)


if __name__ == "__main__":
    main()
