#!/usr/bin/env python3
"""Benchmark of the w-BFBT Stokes hot path on one MI355X.

One step = the whole hot path on the largest seeded multi-sinker workload (64^3 Q3 x P2-disc,
48 sinkers, DR 1e10): viscosity at the quadrature points and nodes, body force, solver setup
(multigrid hierarchies, w-BFBT weights and diagonals, Chebyshev bounds, coarsest
factorizations) and the FP64 FGMRES solve to relative residual 1e-6.  `value` = (u-DOF + p-DOF)
per second of step time (GDoF/s, whole job; every input resident in HBM).  A step that does not
converge stops the benchmark.

Also reported:
- the A(mu) apply of the workload (median of five runs of 100 applies bracketed by HIP events on
  their stream), its kernels and its roofline (algorithmic bytes, HBM traffic from the committed
  counter summary), and the rate of a device copy of the velocity vector on the same box;
- the kernel classes of one eagerly launched step;
- the precision forms (FP32, BF16x3 on the matrix cores) and the learned coarse correction at the
  workload, each with its error against the FP64 solution and its device memory;
- the other workloads: 16^3 Q4 (precision forms), 48^3 Q2 (learned correction), 32^3 Q2;
- the CPU oracle on the machine's host: the assembled A apply on the full 32^3 Q2 input (one thread)
  and the oracle solve on a bounded sample with the workload's parameters.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--config c5]
"""
from __future__ import annotations

import argparse
import json
import os
import sys
import time

ROOT = os.path.dirname(os.path.abspath(__file__))
sys.path.insert(0, ROOT)

METRIC = "A(μ)-apply GDoF/s + %HBM peak; Stokes solve s to 1e-6, FP64 vs mixed/learned"
HBM_PEAK_GBS = 8000.0
# bounded CPU-oracle sample: the 32^3 Q2 workload's parameters (16 sinkers, DR 1e6) on a 16^3
# mesh.  The largest workload's parameters (48 sinkers of diameter 0.04, DR 1e10) are not resolved
# by meshes the oracle solves in seconds: on 6^3 Q3 its FGMRES has not converged after 300
# iterations.
CPU_SAMPLE = ("c2", 16)


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def op_bytes(key: str) -> float:
    """Algorithmic HBM bytes of one operator launch of the given kernel class."""
    parts = dict(p.split("=") for p in key.split() if "=" in p)
    nc, k, N = int(parts["nc"]), int(parts["k"]), int(parts["N"])
    flags = parts["flags"]
    es = 8 if key.endswith("f64") else 4
    nn = (k * N + 1) ** 3
    E = N ** 3
    nq = E * (k + 1) ** 3
    npm = E * k * (k + 1) * (k + 2) // 6
    b = 0.0
    if flags.startswith("A"):
        b += es * (2 * nc * nn + nq)                 # read u, write y, read coefficient
    if "+BT" in flags:
        b += es * npm + (0 if flags.startswith("A") else es * nc * nn)
    if "+B" in flags.replace("+BT", ""):
        b += es * npm + (0 if flags.startswith("A") else es * nc * nn)
    if "+scale" in flags:
        b += es * nn
    return b


class NotConverged(RuntimeError):
    pass


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c5")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-forms", action="store_true", help="skip the precision forms")
    ap.add_argument("--no-learned", action="store_true", help="skip the learned correction")
    ap.add_argument("--no-others", action="store_true", help="skip the other workloads")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(domain decomposition over RCCL is a design note, not code).", file=sys.stderr)
        sys.exit(2)

    import torch

    from paper_1607_03936_amd import wbfbt as wb
    from synthetic import WORKLOADS

    torch.cuda.set_device(0)
    wb.lib()
    w = WORKLOADS[args.config]
    run = Run(wb, torch, w)
    log(f"[bench] workload {w.name}: N={w.N} k={w.k} u-DOF={run.mesh.u_len} p-DOF={run.mesh.p_len}")
    for i in range(args.warmup):
        r = run.step()
        log(f"[bench] warmup {i}: setup {r['setup_s']:.3f}s solve {r['solve_s']:.3f}s "
            f"iters {r['iters']} res {r['rel_res']:.2e}")
    torch.cuda.synchronize()
    steps = []
    t0 = time.perf_counter()
    for i in range(args.steps):
        r = run.step()
        steps.append(r)
        log(f"[bench] step {i}: setup {r['setup_s']:.3f}s solve {r['solve_s']:.3f}s "
            f"iters {r['iters']} res {r['rel_res']:.2e}")
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t0
    ms_per_step = 1e3 * t_total / args.steps
    u64, p64 = run.u.clone(), run.p.clone()

    def med(key):
        v = sorted(s[key] for s in steps)
        return v[len(v) // 2]

    solve = {w.name: {"fp64": {"setup_s": round(med("setup_s"), 4), "solve_s": round(med("solve_s"), 4),
                               "iters": int(med("iters")), "rel_res": max(s["rel_res"] for s in steps),
                               "device_bytes": steps[-1]["device_bytes"]}}}

    # kernel classes of one step with every launch issued eagerly (graph replays carry no
    # per-launch events)
    wb.wb_profile_enable(True)
    wb.wb_profile_summary(reset=True)
    r = run.step(use_graph=0)
    torch.cuda.synchronize()
    wb.wb_profile_enable(False)
    prof = wb.wb_profile_summary(reset=True)
    log(f"[bench] eager profiled step: setup {r['setup_s']:.3f}s solve {r['solve_s']:.3f}s iters {r['iters']}")
    step_total = sum(v[1] for v in prof.values())
    step_kernels = [{"kernel": k, "launches": n, "ms": round(ms, 3), "share": round(ms / step_total, 4)}
                    for k, (n, ms) in sorted(prof.items(), key=lambda kv: -kv[1][1])[:8]]

    # the A(mu) apply of the workload
    a_apply = measure_a_apply(wb, torch, run.mesh, run.visc())
    log(f"[bench] A apply {w.name}: {a_apply['avg_ms'] * 1e3:.1f} us, {a_apply['gdofs']} GDoF/s, "
        f"{a_apply['hbm_frac']:.3f} of HBM peak, {a_apply['frac_of_copy']:.3f} of the device copy "
        f"({a_apply['copy_GBs']:.0f} GB/s)")

    if not args.no_forms:
        for name, prec in (("fp32", wb.WB_FP32), ("bf16x3_mfma", wb.WB_BF16)):
            r = run.step(prec)
            solve[w.name][name] = form_row(r, run, u64, p64)
            log(f"[bench] {w.name} {name}: {r['iters']} its, solve {r['solve_s']:.3f}s, "
                f"du {solve[w.name][name]['rel_err_u_vs_fp64']:.1e}")
    if not args.no_learned:
        solve[w.name]["learned"] = learned_form(run, u64, p64, solve[w.name]["fp64"])
    run.free()
    del run
    torch.cuda.empty_cache()

    others = {}
    if not args.no_others:
        plan = {"c3": ("fp32", "bf16x3_mfma"), "c4": ("learned",), "c2": ()}
        for cname, forms in plan.items():
            if cname == w.name:
                continue
            wc = WORKLOADS[cname]
            rc = Run(wb, torch, wc)
            rc.step()
            r = rc.step()
            row = {"fp64": {"setup_s": round(r["setup_s"], 4), "solve_s": round(r["solve_s"], 4),
                            "iters": r["iters"], "rel_res": r["rel_res"],
                            "device_bytes": r["device_bytes"]}}
            uc, pc = rc.u.clone(), rc.p.clone()
            for name in forms:
                if name == "learned":
                    if not args.no_learned:
                        row[name] = learned_form(rc, uc, pc, row["fp64"])
                    continue
                prec = {"fp32": wb.WB_FP32, "bf16x3_mfma": wb.WB_BF16}[name]
                rc.step(prec)
                r = rc.step(prec)
                row[name] = form_row(r, rc, uc, pc)
            aa = measure_a_apply(wb, torch, rc.mesh, rc.visc())
            others[cname] = {"workload": wc.describe(), "solve": row,
                             "a_apply": {k: aa[k] for k in ("kernel", "avg_ms", "gdofs", "hbm_frac",
                                                          "cache_note")}}
            log(f"[bench] {cname}: " + ", ".join(f"{k} {v['iters']} its {v['solve_s']:.3f}s"
                                                for k, v in row.items() if "iters" in v))
            rc.free()
            del rc
            torch.cuda.empty_cache()

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(WORKLOADS[CPU_SAMPLE[0]], CPU_SAMPLE[1])

    dof = run_dofs(w)
    out = {
        "metric": METRIC,
        "value": round(dof / (ms_per_step * 1e-3) / 1e9, 5),
        "unit": "GDoF/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": w.describe(),
                   "u_dof": w.u_dof, "p_dof": w.p_dof,
                   "step": "viscosity + body force + solver setup + FP64 FGMRES solve to 1e-6"},
        "converged": True,
        "solve": solve,
        "a_apply": a_apply,
        "step_kernels_eager": step_kernels,
        "roofline": {"kernel": a_apply["kernel"], "bound": "hbm", "achieved": a_apply["algorithmic_GBs"],
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(a_apply["algorithmic_GBs"] / HBM_PEAK_GBS, 4),
                     "traffic": a_apply["traffic_bytes_per_launch"], "launches": a_apply["launches"],
                     "avg_ms": a_apply["avg_ms"], "bytes_per_launch": a_apply["bytes_per_launch"]},
        "other_workloads": others,
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def run_dofs(w):
    return w.u_dof + w.p_dof


class Run:
    """The hot path on one workload: fresh viscosity, body force, solver, solve."""

    def __init__(self, wb, torch, w):
        self.wb, self.torch, self.w = wb, torch, w
        self.centers = w.centers()
        self.mesh = wb.Mesh(w.N, w.k)
        self.f = torch.empty(self.mesh.u_len, dtype=torch.float64, device="cuda")
        self.u = torch.empty(self.mesh.u_len, dtype=torch.float64, device="cuda")
        self.p = torch.empty(self.mesh.p_len, dtype=torch.float64, device="cuda")
        self._visc = None

    def visc(self):
        w, wb = self.w, self.wb
        if self._visc is None:
            self._visc = wb.Viscosity.sinker(self.mesh, self.centers, w.delta, w.omega, w.mu_min, w.mu_max)
        return self._visc

    def step(self, prec=None, use_graph=1, solver_kw=None):
        wb, torch, w = self.wb, self.torch, self.w
        prec = wb.WB_FP64 if prec is None else prec
        t0 = time.perf_counter()
        v = wb.Viscosity.sinker(self.mesh, self.centers, w.delta, w.omega, w.mu_min, w.mu_max)
        wb.wb_rhs_sinker(self.mesh, self.centers, w.delta, w.omega, w.beta, self.f)
        s = wb.Solver(self.mesh, v, a_l=w.a_l, a_r=w.a_r, precond_prec=prec, use_graph=use_graph,
                      **(solver_kw or {}))
        t1 = time.perf_counter()
        rep = s.solve(self.f, self.u, self.p, allow_noconv=True)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        if rep.rel_res > 1e-6:
            raise NotConverged(f"{w.name}: FGMRES stopped at relative residual {rep.rel_res:.2e} "
                               f"after {rep.iters} iterations")
        out = {"setup_s": t1 - t0, "solve_s": t2 - t1, "iters": rep.iters, "rel_res": rep.rel_res,
               "device_bytes": int(rep.device_bytes)}
        del s, v
        return out

    def free(self):
        self._visc = None


def form_row(r, run, u64, p64):
    torch = run.torch
    du = (torch.linalg.norm(run.u - u64) / torch.linalg.norm(u64)).item()
    dp = (torch.linalg.norm(run.p - p64) / torch.linalg.norm(p64)).item()
    return {"setup_s": round(r["setup_s"], 4), "solve_s": round(r["solve_s"], 4), "iters": r["iters"],
            "rel_res": r["rel_res"], "rel_err_u_vs_fp64": du, "rel_err_p_vs_fp64": dp,
            "device_bytes": r["device_bytes"]}


def measure_a_apply(wb, torch, mesh, v, reps=100):
    x = torch.rand(mesh.u_len, dtype=torch.float64, device="cuda")
    y = torch.zeros(mesh.u_len, dtype=torch.float64, device="cuda")
    for _ in range(10):
        wb.wb_apply_A(mesh, v, x, y)
    torch.cuda.synchronize()
    # the whole apply (both of its kernels), timed over `reps` back-to-back applies with HIP events
    # on the stream they are launched on; the median of five such runs
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    runs = []
    for _ in range(5):
        e0.record(st)
        for _ in range(reps):
            wb.wb_apply_A(mesh, v, x, y)
        e1.record(st)
        torch.cuda.synchronize()
        runs.append(e0.elapsed_time(e1) / reps)
    t_avg = sorted(runs)[len(runs) // 2]
    # STREAM-copy reference on the same box: a device copy of the velocity vector (read + write)
    z = torch.empty_like(x)
    for _ in range(3):
        z.copy_(x)
    e0.record(st)
    for _ in range(reps):
        z.copy_(x)
    e1.record(st)
    torch.cuda.synchronize()
    copy_gbs = 2 * x.numel() * x.element_size() / (e0.elapsed_time(e1) / reps * 1e-3) / 1e9
    del z
    # per-kernel split (each kernel bracketed by its own events, which adds a little per kernel)
    wb.wb_profile_enable(True)
    wb.wb_profile_summary(reset=True)
    for _ in range(reps):
        wb.wb_apply_A(mesh, v, x, y)
    torch.cuda.synchronize()
    wb.wb_profile_enable(False)
    aprof = wb.wb_profile_summary(reset=True)
    # an apply is two kernels: the element pass (brick march, or all elements into the element
    # buffer) and the second pass (brick-face sums, or node sums); rates count both
    a_key, (a_n, a_ms) = next((k, x) for k, x in aprof.items() if k.startswith("op "))
    a_bytes = op_bytes(a_key)
    faces = [x for k, x in aprof.items() if k.startswith("op-faces")]
    f_avg = faces[0][1] / faces[0][0] if faces else 0.0
    del x, y
    return {"kernel": a_key, "launches": reps, "avg_ms": round(t_avg, 5),
            "first_kernel_avg_ms": round(a_ms / a_n, 5), "second_kernel_avg_ms": round(f_avg, 5),
            "gdofs": round(mesh.u_len / (t_avg * 1e-3) / 1e9, 3),
            "algorithmic_GBs": round(a_bytes / (t_avg * 1e-3) / 1e9, 1),
            "hbm_frac": round(a_bytes / (t_avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "copy_GBs": round(copy_gbs, 1),
            "frac_of_copy": round(a_bytes / (t_avg * 1e-3) / 1e9 / copy_gbs, 4),
            "timing": "median of 5 runs of %d back-to-back applies after 10 warm-ups" % reps,
            "bytes_per_launch": a_bytes,
            "traffic_bytes_per_launch": traffic_for(a_key),
            "cache_note": ("working set %.0f MB %s the 256 MB Infinity Cache"
                           % (a_bytes / 1e6, "fits in" if a_bytes < 256e6 else "exceeds"))}


def learned_form(run, u64, p64, plain):
    """Train the learned coarse correction on solver-generated pairs from seeded fields that
    exclude the evaluation field, then solve with it; reported next to the plain FP64 solve."""
    from synthetic import learned_fields
    wb, torch, w = run.wb, run.torch, run.w
    s = wb.Solver(run.mesh, run.visc(), a_l=w.a_l, a_r=w.a_r, use_learned=1)
    train, valid = learned_fields(w)
    t0 = time.perf_counter()
    tr = s.learned_train(train + valid, n_valid=len(valid), pairs_per_field=1, epochs=20, batch=16,
                         lr=1e-4, delta=w.delta, omega=w.omega, mu_min=w.mu_min, mu_max=w.mu_max)
    t_train = time.perf_counter() - t0
    u = torch.empty_like(u64)
    p = torch.empty_like(p64)
    s.solve(run.f, u, p, allow_noconv=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rep = s.solve(run.f, u, p, allow_noconv=True)
    torch.cuda.synchronize()
    tv = time.perf_counter() - t0
    du = (torch.linalg.norm(u - u64) / torch.linalg.norm(u64)).item()
    out = {"solve_s": round(tv, 4), "iters": rep.iters, "rel_res": rep.rel_res,
           "converged": rep.rel_res <= 1e-6, "learned_reduction_at_lc": rep.learned_reduction,
           "accepted_steps": rep.learned_used,
           "rejected_or_switched": rep.fell_back, "rel_err_u_vs_fp64": du,
           "device_bytes": int(rep.device_bytes),
           "vs_plain": {"iters": plain["iters"], "solve_s": plain["solve_s"]},
           "training": {"fields": len(train), "valid_fields": len(valid), "pairs": tr.n_pairs,
                        "loss_first_epoch": round(tr.loss_first, 4),
                        "loss_last_epoch": round(tr.loss_last, 4),
                        "valid_loss": round(tr.valid_loss, 4), "pairs_s": round(tr.t_pairs_s, 2),
                        "adam_s": round(tr.t_train_s, 2), "total_s": round(t_train, 2)}}
    log(f"[bench] {w.name} learned: {rep.iters} its {tv:.3f}s (plain {plain['iters']} its "
        f"{plain['solve_s']:.3f}s), loss {tr.loss_first:.3f} -> {tr.loss_last:.3f}, valid {tr.valid_loss:.3f}")
    del s
    return out


def kernel_source_hash():
    import hashlib
    h = hashlib.sha256()
    for f in ("kernels.hip", "rules.h", "kernels.h"):
        with open(os.path.join(ROOT, "paper_1607_03936_amd", "csrc", f), "rb") as fh:
            h.update(fh.read())
    return h.hexdigest()[:16]


def traffic_for(kernel_key):
    """HBM bytes per launch of the kernel class from the committed rocprofv3 counter summary
    (FETCH_SIZE and WRITE_SIZE, scaled by the copy-kernel calibration), or None when no summary
    covers this kernel or the kernel sources changed since the counters were taken."""
    path = os.path.join(ROOT, "profiles", "hbm_traffic.json")
    if not os.path.exists(path):
        return None
    with open(path) as fh:
        rec = json.load(fh)
    if rec.get("source_hash") != kernel_source_hash():
        return None
    ent = rec.get("kernels", {}).get(kernel_key)
    return None if ent is None else ent["bytes_per_launch"]


def cpu_model():
    try:
        with open("/proc/cpuinfo") as fh:
            for line in fh:
                if line.startswith("model name"):
                    return line.split(":", 1)[1].strip()
    except OSError:
        pass
    return "unknown"


def cpu_baseline(w, Ns):
    """The oracle (assembled scipy CSR, multigrid, FGMRES) on the host.
    - value: time to solution (assembly, preconditioner setup, FGMRES to 1e-6) of the oracle on
      an Ns^3 sample with workload w's parameters, in GDoF/s, dense BLAS on all host cores
      (sparse products in scipy run on one thread);
    - a_apply_csr_32cubed_q2: the assembled A apply y = A u on the full 32^3 Q2 input, one
      thread (nnz, seconds per apply, GDoF/s)."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import fem, sinker
    from oracle import solver as osolver
    from synthetic import WORKLOADS, random_vector
    ncpu = os.cpu_count() or 1
    with threadpool_limits(ncpu):
        t0 = time.perf_counter()
        st = osolver.Stokes(Ns, w.k, w.centers(), w.delta, w.omega, w.mu_min, w.mu_max,
                            a_l=w.a_l, a_r=w.a_r)
        P = osolver.Preconditioner(st)
        t1 = time.perf_counter()
        b = np.concatenate([st.F, np.zeros(st.np_)])
        x, it, hist = osolver.fgmres(st.stokes_matvec, b, P.apply, rtol=1e-6, max_iter=300)
        t2 = time.perf_counter()
    t_setup, t_solve = t1 - t0, t2 - t1
    dof = st.mesh.u_dof + st.mesh.p_dof
    converged = hist[-1] <= 1e-6
    sample = (f"oracle solve of the {w.name} parameters (Q{w.k}, {w.n_sinkers} sinkers, delta "
              f"{w.delta:g}, omega {w.omega:g}, DR {w.dr:g}) on {Ns}^3 elements ({dof} DOF): assembly "
              f"+ multigrid setup {t_setup:.2f}s, {it} FGMRES iterations {t_solve:.2f}s, "
              + ("converged to 1e-6" if converged else f"not converged (residual {hist[-1]:.1e})"))
    log(f"[bench] cpu: {sample}")
    # assembled A apply on the full 32^3 Q2 input (the same input as the GPU's 32^3 Q2 apply)
    w2 = WORKLOADS["c2"]
    with threadpool_limits(1):
        t0 = time.perf_counter()
        m = fem.Mesh(w2.N, w2.k)
        mu = sinker.viscosity(m.quad_points(), w2.centers(), w2.delta, w2.omega, w2.mu_min, w2.mu_max)
        A = fem.assemble_A(m, mu)
        t_asm = time.perf_counter() - t0
        u = random_vector(17, m.u_dof)
        reps = 5
        t0 = time.perf_counter()
        for _ in range(reps):
            A @ u
        t_app = (time.perf_counter() - t0) / reps
    csr = {"nnz": int(A.nnz), "u_dof": m.u_dof, "s_per_apply": round(t_app, 4),
           "gdofs": round(m.u_dof / t_app / 1e9, 6), "threads": 1, "assembly_s": round(t_asm, 2)}
    log(f"[bench] cpu: CSR A@u on 32^3 Q2: nnz {A.nnz}, {t_app:.3f}s per apply")
    del A
    return {"value": round(dof / (t_setup + t_solve) / 1e9, 8),
            "unit": "GDoF/s", "cores": ncpu, "kind": "oracle", "sample": sample,
            "converged": bool(converged), "cpu_model": cpu_model(), "os_cpu_count": ncpu,
            "a_apply_csr_32cubed_q2": csr}


if __name__ == "__main__":
    main()
