"""Robustness sweep of the two Schur approximations, the experiment of Sec. 8 (Table 1) on seeded
sinker fields: FGMRES iterations to a 1e-6 residual reduction for n sinkers x dynamic ratio DR,
with the diagonalized inverse viscosity-weighted pressure mass M_p(1/mu) (eq. 4) and with w-BFBT
(eq. 8), the same velocity multigrid for both.

python -m paper_1607_03936_amd.sweep [--N 32] [--k 2] [--max-iter 1000] [--json out.json]
                                    [--sinkers 1,4,...] [--ratios 1e4,...] [--amp]

--amp instead runs the boundary amplification study of Sec. 5 (Table 2): w-BFBT with
a_l x a_r in {1, 2, 4, 8, 16, 32}^2 on S16 at DR 1e6 (or the given sinkers and ratio).
--weights instead compares the w-BFBT weights sqrt(mu) and (mu^2 + |grad mu|^2)^(1/4) (the
remark of Sec. 4) and diag(A)-BFBT (Sec. 4) over the given sinkers and ratios.

Sinker sets: n in {1, 4, 8, 12, 16, 20, 24, 28}, centres from the seeded generator (seed 100 + n),
delta 200, omega 0.1, beta 10, mu in [DR^-1/2, DR^1/2]; a_l = 1, a_r = max(1, (N/16) 2^(k-2)).
A solve that reaches the iteration cap is reported as '>cap'.
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

sys.path.insert(0, os.path.dirname(os.path.dirname(os.path.abspath(__file__))))

SINKERS = (1, 4, 8, 12, 16, 20, 24, 28)
RATIOS = (1e4, 1e6, 1e8, 1e10)


def main(argv=None):
    ap = argparse.ArgumentParser(description=__doc__.splitlines()[0])
    ap.add_argument("--N", type=int, default=32)
    ap.add_argument("--k", type=int, default=2)
    ap.add_argument("--max-iter", type=int, default=1000)
    ap.add_argument("--json", default=None)
    ap.add_argument("--sinkers", default=",".join(str(n) for n in SINKERS))
    ap.add_argument("--ratios", default=",".join(f"{r:g}" for r in RATIOS))
    ap.add_argument("--amp", action="store_true")
    ap.add_argument("--weights", action="store_true")
    a = ap.parse_args(argv)
    sinkers = [int(x) for x in a.sinkers.split(",")]
    ratios = [float(x) for x in a.ratios.split(",")]
    if a.amp:
        return amplification(a)
    if a.weights:
        return weight_forms(a, sinkers, ratios)

    import torch

    from paper_1607_03936_amd import wbfbt as wb
    from synthetic import sinker_centers
    wb.lib()
    m = wb.Mesh(a.N, a.k)
    a_r = max(1.0, (a.N / 16) * 2.0 ** (a.k - 2))
    f = torch.empty(m.u_len, dtype=torch.float64, device="cuda")
    u = torch.empty(m.u_len, dtype=torch.float64, device="cuda")
    p = torch.empty(m.p_len, dtype=torch.float64, device="cuda")
    rows = []
    for n in sinkers:
        c = sinker_centers(100 + n, n)
        for dr in ratios:
            lo, hi = dr ** -0.5, dr ** 0.5
            v = wb.Viscosity.sinker(m, c, 200.0, 0.1, lo, hi)
            wb.wb_rhs_sinker(m, c, 200.0, 0.1, 10.0, f)
            rec = {"sinkers": n, "dr": dr}
            for label, approx in (("mass", 1), ("wbfbt", 0)):
                s = wb.Solver(m, v, a_l=1.0, a_r=a_r, schur_approx=approx, max_iter=a.max_iter)
                torch.cuda.synchronize()
                t0 = time.perf_counter()
                rep = s.solve(f, u, p, allow_noconv=True)
                torch.cuda.synchronize()
                rec[label] = {"iters": rep.iters, "rel_res": rep.rel_res,
                              "converged": rep.rel_res <= 1e-6, "solve_s": time.perf_counter() - t0}
                del s
            rows.append(rec)
            print(f"S{n}-rand DR {dr:.0e}: M_p(1/mu) {rec['mass']['iters']:>5} "
                  f"({'ok' if rec['mass']['converged'] else 'cap'})   w-BFBT {rec['wbfbt']['iters']:>4}",
                  flush=True)
            del v

    def cell(r):
        return f"{r['iters']}" if r["converged"] else f">{r['iters']}"
    for label, title in (("mass", "M_p(1/mu), diagonalized"), ("wbfbt", "w-BFBT")):
        print(f"\n{title}: FGMRES iterations, {a.N}^3 Q{a.k}, rows #sinkers, columns DR")
        print(f"{'':>10}" + "".join(f"{dr:>10.0e}" for dr in ratios))
        for n in sinkers:
            line = f"{'S%d-rand' % n:>10}"
            for dr in ratios:
                r = next(x for x in rows if x["sinkers"] == n and x["dr"] == dr)
                line += f"{cell(r[label]):>10}"
            print(line)
    if a.json:
        with open(a.json, "w") as fh:
            json.dump({"N": a.N, "k": a.k, "max_iter": a.max_iter, "rows": rows}, fh, indent=1)


AMPS = (1, 2, 4, 8, 16, 32)


def weight_forms(a, sinkers, ratios):
    import torch

    from paper_1607_03936_amd import wbfbt as wb
    from synthetic import sinker_centers
    wb.lib()
    m = wb.Mesh(a.N, a.k)
    a_r = max(1.0, (a.N / 16) * 2.0 ** (a.k - 2))
    f = torch.empty(m.u_len, dtype=torch.float64, device="cuda")
    u = torch.empty(m.u_len, dtype=torch.float64, device="cuda")
    p = torch.empty(m.p_len, dtype=torch.float64, device="cuda")
    rows = []
    for n in sinkers:
        c = sinker_centers(100 + n, n)
        for dr in ratios:
            v = wb.Viscosity.sinker(m, c, 200.0, 0.1, dr ** -0.5, dr ** 0.5)
            wb.wb_rhs_sinker(m, c, 200.0, 0.1, 10.0, f)
            rec = {"sinkers": n, "dr": dr}
            for label, wf in (("sqrt", 0), ("grad", 1), ("diagA", 2)):
                amp_r = 1.0 if wf == 2 else a_r
                s = wb.Solver(m, v, a_l=1.0, a_r=amp_r, weights=wf, max_iter=a.max_iter)
                rep = s.solve(f, u, p, allow_noconv=True)
                rec[label] = rep.iters if rep.rel_res <= 1e-6 else -rep.iters
                del s
            rows.append(rec)
            print(f"S{n}-rand DR {dr:.0e}: w-BFBT sqrt(mu) {abs(rec['sqrt'])}  gradient {abs(rec['grad'])}"
                  f"  diag(A)-BFBT {abs(rec['diagA'])}{'' if rec['diagA'] > 0 else ' (cap)'}", flush=True)
    if a.json:
        with open(a.json, "w") as fh:
            json.dump({"N": a.N, "k": a.k, "rows": rows}, fh, indent=1)


def amplification(a):
    import torch

    from paper_1607_03936_amd import wbfbt as wb
    from synthetic import sinker_centers
    wb.lib()
    n = 16 if a.sinkers == ",".join(str(x) for x in SINKERS) else int(a.sinkers.split(",")[0])
    dr = 1e6 if a.ratios == ",".join(f"{r:g}" for r in RATIOS) else float(a.ratios.split(",")[0])
    m = wb.Mesh(a.N, a.k)
    c = sinker_centers(100 + n, n)
    v = wb.Viscosity.sinker(m, c, 200.0, 0.1, dr ** -0.5, dr ** 0.5)
    f = torch.empty(m.u_len, dtype=torch.float64, device="cuda")
    u = torch.empty(m.u_len, dtype=torch.float64, device="cuda")
    p = torch.empty(m.p_len, dtype=torch.float64, device="cuda")
    wb.wb_rhs_sinker(m, c, 200.0, 0.1, 10.0, f)
    its = {}
    for al in AMPS:
        for ar in AMPS:
            s = wb.Solver(m, v, a_l=float(al), a_r=float(ar), max_iter=a.max_iter)
            rep = s.solve(f, u, p, allow_noconv=True)
            its[(al, ar)] = rep.iters if rep.rel_res <= 1e-6 else -rep.iters
            del s
        print(f"a_l {al}: " + " ".join(f"{abs(its[(al, ar)])}" for ar in AMPS), flush=True)
    print(f"\nw-BFBT FGMRES iterations, {a.N}^3 Q{a.k}, S{n}-rand, DR {dr:.0e}; rows a_l, columns a_r")
    print(f"{'':>6}" + "".join(f"{ar:>6}" for ar in AMPS))
    for al in AMPS:
        print(f"{al:>6}" + "".join(f"{(str(its[(al, ar)]) if its[(al, ar)] > 0 else '>' + str(-its[(al, ar)])):>6}"
                                   for ar in AMPS))
    if a.json:
        with open(a.json, "w") as fh:
            json.dump({"N": a.N, "k": a.k, "sinkers": n, "dr": dr,
                       "iters": {f"{al},{ar}": v_ for (al, ar), v_ in its.items()}}, fh, indent=1)


if __name__ == "__main__":
    main()
