#!/usr/bin/env python3
"""Benchmark of the w-BFBT Stokes hot path on one MI355X.

One step = the whole hot path on the seeded multi-sinker workload: viscosity at
the quadrature points and nodes, body force, solver setup (multigrid hierarchy,
w-BFBT weights and diagonals, Chebyshev bounds, coarsest factorizations) and the
FP64 FGMRES solve to relative residual 1e-6.  `value` = (u-DOF + p-DOF) per
second of step time (GDoF/s, whole job); the FGMRES preconditioner applies are
replayed from a HIP graph.  Also reported: the kernel classes of one eagerly
launched step, the A(mu)-apply rate and roofline (100 applies bracketed by HIP
events on their stream, at the workload and at 64^3 Q3, where the working set
exceeds the Infinity Cache), the mixed-precision form, and the CPU oracle on a
bounded sample.

python bench.py [--gpus 1] [--steps K] [--warmup W] [--config c2]
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

# bounded CPU-oracle samples: same parameters, smaller mesh, full solve when it converges
CPU_SAMPLE = {"c1": 4, "c2": 24, "c3": 4, "c4": 8, "c5": 4}


def log(*a):
    print(*a, file=sys.stderr, flush=True)


def op_bytes(key: str, mesh_N: int, k_fine: int) -> float:
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


def main():
    ap = argparse.ArgumentParser()
    ap.add_argument("--gpus", type=int, default=1)
    ap.add_argument("--steps", type=int, default=3)
    ap.add_argument("--warmup", type=int, default=1)
    ap.add_argument("--config", default="c2")
    ap.add_argument("--no-cpu", action="store_true")
    ap.add_argument("--no-mixed", action="store_true")
    ap.add_argument("--no-big", action="store_true", help="skip the 64^3 Q3 A-apply measurement")
    ap.add_argument("--no-learned", action="store_true", help="skip training the learned correction")
    args = ap.parse_args()
    if args.gpus != 1 or int(os.environ.get("WORLD_SIZE", "1")) != 1:
        print("bench.py runs on one GPU only: this build has no multi-GPU path "
              "(domain decomposition over RCCL is a design note, not code).", file=sys.stderr)
        sys.exit(2)

    import numpy as np
    import torch

    from paper_1607_03936_amd import wbfbt as wb
    from synthetic import WORKLOADS

    w = WORKLOADS[args.config]
    centers = w.centers()
    torch.cuda.set_device(0)
    wb.lib()
    mesh = wb.Mesh(w.N, w.k)
    dof = mesh.u_len + mesh.p_len
    f = torch.empty(mesh.u_len, dtype=torch.float64, device="cuda")
    u = torch.empty(mesh.u_len, dtype=torch.float64, device="cuda")
    p = torch.empty(mesh.p_len, dtype=torch.float64, device="cuda")

    def step(prec=wb.WB_FP64, use_graph=1):
        t0 = time.perf_counter()
        v = wb.Viscosity.sinker(mesh, centers, w.delta, w.omega, w.mu_min, w.mu_max)
        wb.wb_rhs_sinker(mesh, centers, w.delta, w.omega, w.beta, f)
        s = wb.Solver(mesh, v, a_l=w.a_l, a_r=w.a_r, precond_prec=prec, use_graph=use_graph)
        t1 = time.perf_counter()
        rep = s.solve(f, u, p, allow_noconv=True)
        torch.cuda.synchronize()
        t2 = time.perf_counter()
        del s, v
        return rep, t1 - t0, t2 - t1

    log(f"[bench] workload {args.config}: N={w.N} k={w.k} u-DOF={mesh.u_len} p-DOF={mesh.p_len}")
    for i in range(args.warmup):
        rep, ts, tv = step()
        log(f"[bench] warmup {i}: setup {ts:.3f}s solve {tv:.3f}s iters {rep.iters} res {rep.rel_res:.2e}")
    torch.cuda.synchronize()
    setups, solves, iters, res = [], [], [], []
    t0 = time.perf_counter()
    for i in range(args.steps):
        rep, ts, tv = step()
        setups.append(ts)
        solves.append(tv)
        iters.append(rep.iters)
        res.append(rep.rel_res)
        log(f"[bench] step {i}: setup {ts:.3f}s solve {tv:.3f}s iters {rep.iters} res {rep.rel_res:.2e}")
    torch.cuda.synchronize()
    t_total = time.perf_counter() - t0
    ms_per_step = 1e3 * t_total / args.steps
    u64, p64 = u.clone(), p.clone()

    # kernel classes of one step, from an untimed step with every launch issued eagerly
    # (launches replayed from the graph carry no per-launch events)
    wb.wb_profile_enable(True)
    wb.wb_profile_summary(reset=True)
    rep, ts, tv = step(use_graph=0)
    torch.cuda.synchronize()
    wb.wb_profile_enable(False)
    prof = wb.wb_profile_summary(reset=True)
    log(f"[bench] eager profiled step: setup {ts:.3f}s solve {tv:.3f}s iters {rep.iters}")
    step_total = sum(v[1] for v in prof.values())
    step_kernels = [{"kernel": k, "launches": n, "ms": round(ms, 3),
                     "share": round(ms / step_total, 4)}
                    for k, (n, ms) in sorted(prof.items(), key=lambda kv: -kv[1][1])[:6]]

    # the A(mu) apply y = A u at the finest level: 100 back-to-back applies, each bracketed by
    # HIP events on the stream it is launched on
    a_apply = measure_a_apply(wb, torch, mesh, w, centers)
    log(f"[bench] A apply {w.name}: {a_apply['avg_ms'] * 1e3:.1f} us, {a_apply['gdofs']} GDoF/s")
    a_big = None
    if not args.no_big and w.name != "c5":
        wbig = WORKLOADS["c5"]
        mbig = wb.Mesh(wbig.N, wbig.k)
        a_big = measure_a_apply(wb, torch, mbig, wbig, wbig.centers())
        log(f"[bench] A apply c5: {a_big['avg_ms'] * 1e3:.1f} us, {a_big['gdofs']} GDoF/s")
        del mbig
        torch.cuda.empty_cache()

    forms = {"fp64": {"setup_s": round(float(np.median(setups)), 4),
                      "solve_s": round(float(np.median(solves)), 4),
                      "iters": int(np.median(iters)), "rel_res": float(max(res))}}
    if not args.no_mixed:
        rep, ts, tv = step(wb.WB_FP32)
        du = (torch.linalg.norm(u - u64) / torch.linalg.norm(u64)).item()
        dp = (torch.linalg.norm(p - p64) / torch.linalg.norm(p64)).item()
        forms["mixed_fp32"] = {"setup_s": round(ts, 4), "solve_s": round(tv, 4), "iters": rep.iters,
                               "rel_res": rep.rel_res, "rel_err_u_vs_fp64": du,
                               "rel_err_p_vs_fp64": dp}
        log(f"[bench] mixed: setup {ts:.3f}s solve {tv:.3f}s iters {rep.iters} du {du:.1e} dp {dp:.1e}")
        rep, ts, tv = step(wb.WB_BF16)
        du = (torch.linalg.norm(u - u64) / torch.linalg.norm(u64)).item()
        dp = (torch.linalg.norm(p - p64) / torch.linalg.norm(p64)).item()
        forms["mixed_bf16x3_mfma"] = {"setup_s": round(ts, 4), "solve_s": round(tv, 4),
                                      "iters": rep.iters, "rel_res": rep.rel_res,
                                      "rel_err_u_vs_fp64": du, "rel_err_p_vs_fp64": dp}
        log(f"[bench] bf16x3: setup {ts:.3f}s solve {tv:.3f}s iters {rep.iters} du {du:.1e} dp {dp:.1e}")
    if not args.no_learned:
        forms["learned"] = learned_form(wb, torch, mesh, w, centers, f, u64, p64)

    cpu = None
    if not args.no_cpu:
        cpu = cpu_baseline(w, CPU_SAMPLE[args.config])

    out = {
        "metric": METRIC,
        "value": round(dof / (ms_per_step * 1e-3) / 1e9, 5),
        "unit": "GDoF/s",
        "n_gpus": 1, "steps": args.steps, "warmup": args.warmup,
        "ms_per_step": round(ms_per_step, 3),
        "higher_is_better": True, "scaling": "weak", "vs_baseline": None,
        "dtype": "f64", "data": "synthetic",
        "config": {"workload": f"{args.config}: {w.N}^3 elements, Q{w.k} x P{w.k - 1}-disc, "
                               f"{w.n_sinkers} seeded sinkers, delta {w.delta:g}, omega {w.omega:g}, "
                               f"DR {w.dr:g}, a_r {w.a_r:g}, FGMRES(100) to 1e-6",
                   "u_dof": mesh.u_len, "p_dof": mesh.p_len,
                   "step": "viscosity + body force + solver setup + FP64 FGMRES solve"},
        "solve": forms,
        "a_apply": a_apply,
        "a_apply_64cubed_q3": a_big,
        "step_kernels_eager": step_kernels,
        "roofline": {"kernel": a_apply["kernel"], "bound": "hbm", "achieved": a_apply["algorithmic_GBs"],
                     "peak": HBM_PEAK_GBS, "unit": "GB/s",
                     "frac": round(a_apply["algorithmic_GBs"] / HBM_PEAK_GBS, 4),
                     "traffic": traffic_for(a_apply["kernel"]), "launches": a_apply["launches"],
                     "avg_ms": a_apply["avg_ms"], "bytes_per_launch": a_apply["bytes_per_launch"]},
        "cpu_baseline": cpu,
    }
    print(json.dumps(out), flush=True)


def measure_a_apply(wb, torch, mesh, w, centers, reps=100):
    v = wb.Viscosity.sinker(mesh, centers, w.delta, w.omega, w.mu_min, w.mu_max)
    x = torch.rand(mesh.u_len, dtype=torch.float64, device="cuda")
    y = torch.zeros(mesh.u_len, dtype=torch.float64, device="cuda")
    for _ in range(10):
        wb.wb_apply_A(mesh, v, x, y)
    torch.cuda.synchronize()
    # the whole apply (both of its kernels), timed over `reps` back-to-back applies with HIP events
    # on the stream they are launched on
    st = torch.cuda.current_stream()
    e0, e1 = torch.cuda.Event(enable_timing=True), torch.cuda.Event(enable_timing=True)
    e0.record(st)
    for _ in range(reps):
        wb.wb_apply_A(mesh, v, x, y)
    e1.record(st)
    torch.cuda.synchronize()
    t_avg = e0.elapsed_time(e1) / reps
    # per-kernel split (each kernel bracketed by its own events, which adds a little per kernel)
    wb.wb_profile_enable(True)
    wb.wb_profile_summary(reset=True)
    for _ in range(reps):
        wb.wb_apply_A(mesh, v, x, y)
    torch.cuda.synchronize()
    wb.wb_profile_enable(False)
    aprof = wb.wb_profile_summary(reset=True)
    # an apply is two kernels: the element pass (the brick scatter, or all elements into the
    # element buffer) and the second pass (brick-face sums, or node sums); rates count both
    a_key, (a_n, a_ms) = next((k, x) for k, x in aprof.items() if k.startswith("op "))
    a_avg = a_ms / a_n
    a_bytes = op_bytes(a_key, mesh.N, mesh.k)
    faces = [x for k, x in aprof.items() if k.startswith("op-faces")]
    f_avg = faces[0][1] / faces[0][0] if faces else 0.0
    del v, x, y
    return {"kernel": a_key, "launches": reps, "avg_ms": round(t_avg, 5),
            "first_kernel_avg_ms": round(a_avg, 5), "second_kernel_avg_ms": round(f_avg, 5),
            "gdofs": round(mesh.u_len / (t_avg * 1e-3) / 1e9, 3),
            "algorithmic_GBs": round(a_bytes / (t_avg * 1e-3) / 1e9, 1),
            "hbm_frac": round(a_bytes / (t_avg * 1e-3) / 1e9 / HBM_PEAK_GBS, 4),
            "bytes_per_launch": a_bytes,
            "traffic_bytes_per_launch": traffic_for(a_key),
            "cache_note": ("working set %.0f MB %s the 256 MB Infinity Cache"
                           % (a_bytes / 1e6, "fits in" if a_bytes < 256e6 else "exceeds"))}


def learned_form(wb, torch, mesh, w, centers, f, u64, p64, n_fields=250, pairs=8, epochs=20):
    """Train the learned coarse correction on seeded fields 1000.. (not the evaluation field),
    then solve with it; reported next to the plain FP64 solve (same preconditioner otherwise)."""
    from synthetic import sinker_centers
    v = wb.Viscosity.sinker(mesh, centers, w.delta, w.omega, w.mu_min, w.mu_max)
    s = wb.Solver(mesh, v, a_l=w.a_l, a_r=w.a_r, use_learned=1)
    fields = [sinker_centers(1000 + i, w.n_sinkers) for i in range(n_fields)]
    tr = s.learned_train(fields, pairs_per_field=pairs, epochs=epochs, batch=8, lr=1e-3,
                         n_valid=n_fields // 10, delta=w.delta, omega=w.omega, mu_min=w.mu_min,
                         mu_max=w.mu_max)
    u = torch.empty_like(u64)
    p = torch.empty_like(p64)
    s.solve(f, u, p, allow_noconv=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    rep = s.solve(f, u, p, allow_noconv=True)
    torch.cuda.synchronize()
    tv = time.perf_counter() - t0
    du = (torch.linalg.norm(u - u64) / torch.linalg.norm(u64)).item()
    out = {"solve_s": round(tv, 4), "iters": rep.iters, "rel_res": rep.rel_res,
           "accepted_steps": rep.learned_used, "rejected_or_switched": rep.fell_back,
           "rel_err_u_vs_fp64": du,
           "training": {"fields": n_fields, "pairs": tr.n_pairs, "epochs": epochs,
                        "loss_first_epoch": round(tr.loss_first, 4),
                        "loss_last_epoch": round(tr.loss_last, 4),
                        "valid_loss": round(tr.valid_loss, 4),
                        "pairs_s": round(tr.t_pairs_s, 2), "adam_s": round(tr.t_train_s, 2)}}
    log(f"[bench] learned: {rep.iters} its {tv:.3f}s, loss {tr.loss_first:.3f} -> {tr.loss_last:.3f}")
    del s, v
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


def cpu_baseline(w, Ns):
    """The oracle (assembled scipy CSR, multigrid, FGMRES), one thread, same workload parameters
    on an Ns^3 mesh; value in GDoF/s of time to solution."""
    import numpy as np
    from threadpoolctl import threadpool_limits

    from oracle import solver as osolver
    with threadpool_limits(1):
        t0 = time.perf_counter()
        st = osolver.Stokes(Ns, w.k, w.centers(), w.delta, w.omega, w.mu_min, w.mu_max,
                            a_l=w.a_l, a_r=w.a_r)
        P = osolver.Preconditioner(st)
        t1 = time.perf_counter()
        b = np.concatenate([st.F, np.zeros(st.np_)])
        cap = 200
        x, it, hist = osolver.fgmres(st.stokes_matvec, b, P.apply, rtol=1e-6, max_iter=cap)
        t2 = time.perf_counter()
    dof = st.mesh.u_dof + st.mesh.p_dof
    converged = hist[-1] <= 1e-6
    sample = (f"oracle on the same sinker field and order at {Ns}^3 elements ({dof} DOF): "
              f"assembly + multigrid setup {t1 - t0:.2f}s, {it} FGMRES iterations {t2 - t1:.2f}s, "
              + ("converged to 1e-6" if converged else f"not converged at the {cap}-iteration cap "
                 f"(residual {hist[-1]:.1e}); value uses the time of the capped run"))
    log(f"[bench] cpu: {sample}")
    return {"value": round(dof / (t2 - t0) / 1e9, 8), "unit": "GDoF/s", "cores": 1, "kind": "oracle",
            "sample": sample}


if __name__ == "__main__":
    main()
