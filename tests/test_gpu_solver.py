"""GPU parity of the solver layer (setup products, V-cycles, w-BFBT, block preconditioner, FGMRES)
against the FP64 oracle, through the C-ABI."""
import numpy as np
import pytest

from oracle import fem, solver
from synthetic import WORKLOADS, custom, random_vector

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")


def _wb():
    from paper_1607_03936_amd import wbfbt
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    wbfbt.lib()
    return wbfbt


def dev(a):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=torch.float64, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy()


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


# c1 (two levels), an h-coarsened Q2 case, and Q3, Q4 and Q5 cases; then small meshes with the
# larger workloads' contrasts and sinker sets: DR 1e10 at Q2 (8 sinkers), the 64^3 Q3 parameters
# (48 sinkers, delta 300, omega 0.04, DR 1e10) on 4^3, the 48^3 Q2 parameters (32 sinkers, DR 1e10)
# on 12^3, whose h-hierarchy ends at 6^3 like 48^3, and the 16^3 Q4 parameters (24 sinkers, omega
# 0.05, DR 1e8) on 4^3.  At these contrasts the coefficient coarsening clamps.
SETUPS = {
    "c1": WORKLOADS["c1"],
    "n8k2": custom("n8k2", 8, 2, n_sinkers=8, dr=1e6, a_r=2.0, seed=5),
    "n4k3": custom("n4k3", 4, 3, n_sinkers=4, dr=1e4, a_r=2.0, seed=6),
    "n4k4": custom("n4k4", 4, 4, n_sinkers=3, dr=1e4, a_l=2.0, a_r=1.0, seed=7),
    "n4k5": custom("n4k5", 4, 5, n_sinkers=3, dr=1e4, a_r=2.0, seed=8),
    "n8k2dr10": custom("n8k2dr10", 8, 2, n_sinkers=8, dr=1e10, a_r=2.0, seed=9),
    "n4k3c5": custom("n4k3c5", 4, 3, n_sinkers=48, delta=300.0, omega=0.04, dr=1e10, a_r=2.0, seed=10),
    "n12k2c4": custom("n12k2c4", 12, 2, n_sinkers=32, dr=1e10, seed=11),
    "n4k4c3": custom("n4k4c3", 4, 4, n_sinkers=24, omega=0.05, dr=1e8, seed=12),
}

_cache = {}


def _pair(name):
    if name in _cache:
        return _cache[name]
    wb = _wb()
    w = SETUPS[name]
    c = w.centers()
    st = solver.Stokes(w.N, w.k, c, w.delta, w.omega, w.mu_min, w.mu_max, a_l=w.a_l, a_r=w.a_r)
    P = solver.Preconditioner(st)
    m = wb.Mesh(w.N, w.k)
    v = wb.Viscosity.sinker(m, c, w.delta, w.omega, w.mu_min, w.mu_max)
    s = wb.Solver(m, v, a_l=w.a_l, a_r=w.a_r)
    _cache[name] = (w, st, P, m, v, s)
    return _cache[name]


@pytest.mark.parametrize("name", list(SETUPS))
def test_setup_products(name):
    w, st, P, m, v, s = _pair(name)
    om = st.mesh
    # weights (eq. 8, Sec. 5)
    assert _rel(host(s.query(0, 0, om.n_nodes)), 1.0 / st.C_nodes) < 1e-13
    assert _rel(host(s.query(1, 0, om.n_nodes)), 1.0 / st.D_nodes) < 1e-13
    # discontinuous K diagonals
    assert _rel(host(s.query(4, 0, om.p_dof)), P.disc["l"][1]) < 1e-12
    assert _rel(host(s.query(5, 0, om.p_dof)), P.disc["r"][1]) < 1e-12
    # velocity hierarchy: schedule, coarsened viscosity, Jacobi diagonals, Chebyshev bounds
    lv = s.levels(0)
    assert [(N, k) for N, k, _ in lv] == solver.level_schedule(w.N, w.k)
    for li, L in enumerate(P.A_mg.levels):
        E, n3 = L.mesh.E, L.mesh.n ** 3
        assert _rel(host(s.query(3, li, E * n3)), L.coef.reshape(-1)) < 1e-13
        dinv = host(s.query(2, li, L.mesh.u_dof))
        assert _rel(dinv[L.idx], L.dinv) < 1e-12
        if li + 1 < len(P.A_mg.levels):
            assert abs(lv[li][2] - L.lmax) <= 1e-9 * L.lmax
    for side, mg in ((0, P.Pl_mg), (1, P.Pr_mg)):
        lp = s.levels(1 + side)
        for li, L in enumerate(mg.levels):
            E, n3 = L.mesh.E, L.mesh.n ** 3
            assert _rel(host(s.query(6 + side, li, E * n3)), L.coef.reshape(-1)) < 1e-13
            if li + 1 < len(mg.levels):
                assert abs(lp[li][2] - L.lmax) <= 1e-9 * L.lmax
        if side == 0:
            assert _rel(host(s.query(8, 0, om.n_nodes)), mg.levels[0].dinv) < 1e-12
    kl = s.levels(3)
    assert abs(kl[0][2] - P.disc["l"][3]) <= 1e-9 * P.disc["l"][3]
    assert abs(kl[1][2] - P.disc["r"][3]) <= 1e-9 * P.disc["r"][3]


@pytest.mark.parametrize("name", list(SETUPS))
def test_apply_K_and_vcycles(name):
    w, st, P, m, v, s = _pair(name)
    om = st.mesh
    r = st.remove_mean(random_vector(21, om.p_dof))
    out = torch.empty(om.p_dof, dtype=torch.float64, device="cuda")
    for side, K in ((0, st.Kl), (1, st.Kr)):
        s.apply_K(side, dev(r), out)
        assert _rel(host(out), K @ r) < 1e-12
        s.vcycle_K(side, dev(r), out)
        assert _rel(host(out), P.k_vcycle("l" if side == 0 else "r", r)) < 1e-9
    s.wbfbt(dev(r), out)
    assert _rel(host(out), P.wbfbt(r)) < 1e-9
    ru = random_vector(22, om.u_dof)
    ru[om.vel_boundary] = 0.0
    zu = torch.empty(om.u_dof, dtype=torch.float64, device="cuda")
    s.vcycle_A(dev(ru), zu)
    want = st.embed_u(P.a_vcycle(ru[st.idx]))
    assert _rel(host(zu), want) < 1e-9
    zp = torch.empty(om.p_dof, dtype=torch.float64, device="cuda")
    s.precond(dev(ru), dev(r), zu, zp)
    ref = P.apply(np.concatenate([ru[st.idx], r]))
    assert _rel(host(zu), st.embed_u(ref[:st.nu])) < 1e-9
    assert _rel(host(zp), ref[st.nu:]) < 1e-9


@pytest.mark.parametrize("name", ["c1", "n4k3", "n4k4"])
def test_fgmres_solution_matches_direct_solve(name):
    wb = _wb()
    w, st, P, m, v, s = _pair(name)
    om = st.mesh
    f = torch.empty(om.u_dof, dtype=torch.float64, device="cuda")
    wb.wb_rhs_sinker(m, w.centers(), w.delta, w.omega, w.beta, f)
    assert _rel(host(f)[st.idx], st.F) < 1e-13
    u = torch.empty(om.u_dof, dtype=torch.float64, device="cuda")
    p = torch.empty(om.p_dof, dtype=torch.float64, device="cuda")
    tight = wb.Solver(m, v, a_l=w.a_l, a_r=w.a_r, rtol=1e-11, max_iter=2000)
    rep = tight.solve(f, u, p)
    assert rep.rel_res <= 1e-11
    u_ref, p_ref = st.direct_solve()
    uh, ph = host(u), host(p)
    assert np.linalg.norm(uh[st.idx] - u_ref) <= 1e-8 * np.linalg.norm(u_ref)
    assert np.linalg.norm(ph - p_ref) <= 1e-8 * np.linalg.norm(p_ref)
    assert np.all(uh[om.vel_boundary] == 0.0)
    # at the paper's tolerance the iteration count matches the oracle's FGMRES
    rep6 = s.solve(f, u, p)
    b = np.concatenate([st.F, np.zeros(st.np_)])
    _, it_oracle, _ = solver.fgmres(st.stokes_matvec, b, P.apply, rtol=1e-6)
    assert rep6.rel_res <= 1e-6
    assert abs(rep6.iters - it_oracle) <= 2, (rep6.iters, it_oracle)


@pytest.mark.parametrize("name", ["n8k2dr10", "n4k3c5", "n12k2c4", "n4k4c3"])
def test_fgmres_high_contrast_matches_oracle(name):
    # contrasts 1e8 - 1e10: a direct solve is no reference there (condition numbers near 1/eps)
    # and relative residuals near 1e-11 are out of reach in FP64, so the solve at the paper's
    # tolerance is checked by its iteration count against the oracle's FGMRES and by its residual
    # under the oracle's own operator
    wb = _wb()
    w, st, P, m, v, _ = _pair(name)
    om = st.mesh
    f = torch.empty(om.u_dof, dtype=torch.float64, device="cuda")
    wb.wb_rhs_sinker(m, w.centers(), w.delta, w.omega, w.beta, f)
    assert _rel(host(f)[st.idx], st.F) < 1e-13
    u = torch.empty(om.u_dof, dtype=torch.float64, device="cuda")
    p = torch.empty(om.p_dof, dtype=torch.float64, device="cuda")
    # coarse meshes do not resolve these sinker sets and need hundreds of iterations
    s = wb.Solver(m, v, a_l=w.a_l, a_r=w.a_r, max_iter=5000)
    rep = s.solve(f, u, p)
    b = np.concatenate([st.F, np.zeros(st.np_)])
    _, it_oracle, _ = solver.fgmres(st.stokes_matvec, b, P.apply, rtol=1e-6, max_iter=5000)
    assert rep.rel_res <= 1e-6
    print(f"{name}: {rep.iters} FGMRES iterations (oracle {it_oracle})")
    assert abs(rep.iters - it_oracle) <= max(2, it_oracle // 20), (rep.iters, it_oracle)
    uh, ph = host(u), host(p)
    assert np.all(uh[om.vel_boundary] == 0.0)
    res = b - st.stokes_matvec(np.concatenate([uh[st.idx], ph]))
    assert np.linalg.norm(res) <= 1.01e-6 * np.linalg.norm(b)


def test_fgmres_order_5_matches_oracle():
    # Q5 x P4-disc (the order sweep's top order): the FGMRES iteration count and solution at the
    # paper's tolerance against the oracle's FGMRES with the oracle's preconditioner
    wb = _wb()
    w, st, P, m, v, s = _pair("n4k5")
    om = st.mesh
    f = torch.empty(om.u_dof, dtype=torch.float64, device="cuda")
    wb.wb_rhs_sinker(m, w.centers(), w.delta, w.omega, w.beta, f)
    assert _rel(host(f)[st.idx], st.F) < 1e-13
    u = torch.empty(om.u_dof, dtype=torch.float64, device="cuda")
    p = torch.empty(om.p_dof, dtype=torch.float64, device="cuda")
    rep = s.solve(f, u, p)
    b = np.concatenate([st.F, np.zeros(st.np_)])
    _, it_oracle, _ = solver.fgmres(st.stokes_matvec, b, P.apply, rtol=1e-6)
    assert rep.rel_res <= 1e-6
    assert abs(rep.iters - it_oracle) <= 2, (rep.iters, it_oracle)
    uh, ph = host(u), host(p)
    assert np.all(uh[om.vel_boundary] == 0.0)
    # the solution's residual under the oracle's own operator
    res = b - st.stokes_matvec(np.concatenate([uh[st.idx], ph]))
    assert np.linalg.norm(res) <= 1.01e-6 * np.linalg.norm(b)


@pytest.mark.parametrize("name,mc", [("n8k2", True), ("n4k3", True), ("n4k3", False)])
def test_brick_form_preconditioner_matches_oracle(name, mc):
    # every A and Poisson apply in the brick form (the form large problems use): K_w, the
    # V-cycles and the preconditioner against the oracle, and the FGMRES iteration count; at
    # order 3 both the matrix-core kernel and the LDS line kernel (their Chebyshev and residual
    # epilogues included)
    wb = _wb()
    w, st, P, m, v, _ = _pair(name)
    om = st.mesh
    prev = wb.wb_set_two_pass_limit(0.0)
    prev_mc = wb.wb_set_matrix_core_ops(mc)
    try:
        s = wb.Solver(m, v, a_l=w.a_l, a_r=w.a_r)
        r = st.remove_mean(random_vector(31, om.p_dof))
        out = torch.empty(om.p_dof, dtype=torch.float64, device="cuda")
        s.vcycle_K(0, dev(r), out)
        assert _rel(host(out), P.k_vcycle("l", r)) < 1e-9
        ru = random_vector(32, om.u_dof)
        ru[om.vel_boundary] = 0.0
        zu = torch.empty(om.u_dof, dtype=torch.float64, device="cuda")
        zp = torch.empty(om.p_dof, dtype=torch.float64, device="cuda")
        s.precond(dev(ru), dev(r), zu, zp)
        ref = P.apply(np.concatenate([ru[st.idx], r]))
        assert _rel(host(zu), st.embed_u(ref[:st.nu])) < 1e-9
        assert _rel(host(zp), ref[st.nu:]) < 1e-9
        f = torch.empty(om.u_dof, dtype=torch.float64, device="cuda")
        wb.wb_rhs_sinker(m, w.centers(), w.delta, w.omega, w.beta, f)
        u = torch.empty(om.u_dof, dtype=torch.float64, device="cuda")
        rep = s.solve(f, u, zp)
        b = np.concatenate([st.F, np.zeros(st.np_)])
        _, it_oracle, _ = solver.fgmres(st.stokes_matvec, b, P.apply, rtol=1e-6)
        assert rep.rel_res <= 1e-6
        assert abs(rep.iters - it_oracle) <= 2, (rep.iters, it_oracle)
    finally:
        wb.wb_set_two_pass_limit(prev)
        wb.wb_set_matrix_core_ops(prev_mc)


@pytest.mark.parametrize("name,brick", [("n8k2", False), ("n4k5", False), ("n4k3", True)])
def test_mixed_precision_preconditioner_reaches_tolerance(name, brick):
    # brick: order-3 applies in the brick form (FP32 storage, FP64 matrix-core arithmetic)
    wb = _wb()
    w, st, P, m, v, s = _pair(name)
    om = st.mesh
    if not brick:
        _mixed_precision_solve(wb, w, om, m, v, s)
        return
    prev = wb.wb_set_two_pass_limit(0.0)
    try:
        _mixed_precision_solve(wb, w, om, m, v, wb.Solver(m, v, a_l=w.a_l, a_r=w.a_r))
    finally:
        wb.wb_set_two_pass_limit(prev)


def _mixed_precision_solve(wb, w, om, m, v, s):
    f = torch.empty(om.u_dof, dtype=torch.float64, device="cuda")
    wb.wb_rhs_sinker(m, w.centers(), w.delta, w.omega, w.beta, f)
    u64 = torch.empty(om.u_dof, dtype=torch.float64, device="cuda")
    p64 = torch.empty(om.p_dof, dtype=torch.float64, device="cuda")
    r64 = s.solve(f, u64, p64)
    s32 = wb.Solver(m, v, a_l=w.a_l, a_r=w.a_r, precond_prec=wb.WB_FP32)
    u32 = torch.empty_like(u64)
    p32 = torch.empty_like(p64)
    r32 = s32.solve(f, u32, p32)
    assert r32.rel_res <= 1e-6 and r64.rel_res <= 1e-6
    assert r32.iters <= r64.iters + 3
    du = np.linalg.norm(host(u32) - host(u64)) / np.linalg.norm(host(u64))
    assert du < 1e-4


@pytest.mark.parametrize("prec", ["fp64", "fp32"])
def test_graph_replayed_preconditioner_matches_eager(prec):
    """FGMRES replays the captured preconditioner graph once per iteration, with eager kernels
    and host synchronizations between replays; three solves in a row on one solver must match
    the eager solve (the LDS-window sums may round in a different order, hence a tolerance)."""
    wb = _wb()
    w, st, P, m, v, s = _pair("n8k2")
    om = st.mesh
    pp = wb.WB_FP64 if prec == "fp64" else wb.WB_FP32
    f = torch.empty(om.u_dof, dtype=torch.float64, device="cuda")
    wb.wb_rhs_sinker(m, w.centers(), w.delta, w.omega, w.beta, f)
    eager = wb.Solver(m, v, a_l=w.a_l, a_r=w.a_r, precond_prec=pp, use_graph=0)
    ue = torch.empty(om.u_dof, dtype=torch.float64, device="cuda")
    pe = torch.empty(om.p_dof, dtype=torch.float64, device="cuda")
    re = eager.solve(f, ue, pe)
    graph = wb.Solver(m, v, a_l=w.a_l, a_r=w.a_r, precond_prec=pp, use_graph=1)
    tol = 1e-9 if prec == "fp64" else 1e-5
    for _ in range(3):
        ug = torch.full_like(ue, float("nan"))
        pg = torch.full_like(pe, float("nan"))
        rg = graph.solve(f, ug, pg)
        assert abs(rg.iters - re.iters) <= 1, (rg.iters, re.iters)
        assert rg.rel_res <= 1e-6
        assert _rel(host(ug), host(ue)) < tol
        assert _rel(host(pg), host(pe)) < tol


@pytest.mark.parametrize("name", ["n8k2", "n4k4"])
@pytest.mark.parametrize("form", ["bf16x3", "bf16x1"])
def test_bf16_mfma_preconditioner_reaches_tolerance(name, form):
    """Preconditioner applies in FP32 with BF16 matrix-core contractions; FP64 FGMRES, weights,
    diagonals and coarsest solve.  The outer solve still reaches 1e-6 and its solution agrees
    with the FP64-preconditioned one to the accuracy the tolerance allows.  With split operands
    the iteration count stays at the FP64 count; single BF16 products cost iterations."""
    wb = _wb()
    w, st, P, m, v, s = _pair(name)
    om = st.mesh
    f = torch.empty(om.u_dof, dtype=torch.float64, device="cuda")
    wb.wb_rhs_sinker(m, w.centers(), w.delta, w.omega, w.beta, f)
    u64 = torch.empty(om.u_dof, dtype=torch.float64, device="cuda")
    p64 = torch.empty(om.p_dof, dtype=torch.float64, device="cuda")
    r64 = s.solve(f, u64, p64)
    prec = wb.WB_BF16 if form == "bf16x3" else wb.WB_BF16X1
    sb = wb.Solver(m, v, a_l=w.a_l, a_r=w.a_r, precond_prec=prec)
    ub = torch.empty_like(u64)
    pb = torch.empty_like(p64)
    rb = sb.solve(f, ub, pb)
    du = np.linalg.norm(host(ub) - host(u64)) / np.linalg.norm(host(u64))
    dp = np.linalg.norm(host(pb) - host(p64)) / np.linalg.norm(host(p64))
    print(f"{name} {form}: FP64 {r64.iters} its, BF16 {rb.iters} its, du {du:.2e} dp {dp:.2e}")
    assert rb.rel_res <= 1e-6
    assert du < 1e-4 and dp < 1e-3
    if form == "bf16x3":
        assert rb.iters <= r64.iters + 3
    else:
        assert rb.iters <= 2 * r64.iters + 5


def test_schur_sign_both_readings_match_oracle():
    """Both readings of the Schur block of eq. (3): -S~ (default) and +S~ as printed; the GPU
    preconditioner and FGMRES iteration counts follow the oracle for each, and -S~ needs fewer
    iterations."""
    wb = _wb()
    w, st, P, m, v, s = _pair("n8k2")
    om = st.mesh
    f = torch.empty(om.u_dof, dtype=torch.float64, device="cuda")
    wb.wb_rhs_sinker(m, w.centers(), w.delta, w.omega, w.beta, f)
    b = np.concatenate([st.F, np.zeros(st.np_)])
    its = {}
    for sign in (-1, 1):
        Po = P if sign == -1 else solver.Preconditioner(st, schur_sign=1)
        sg = wb.Solver(m, v, a_l=w.a_l, a_r=w.a_r, schur_sign=sign)
        ru = random_vector(41, om.u_dof)
        ru[om.vel_boundary] = 0.0
        rp = st.remove_mean(random_vector(42, om.p_dof))
        zu = torch.empty(om.u_dof, dtype=torch.float64, device="cuda")
        zp = torch.empty(om.p_dof, dtype=torch.float64, device="cuda")
        sg.precond(dev(ru), dev(rp), zu, zp)
        ref = Po.apply(np.concatenate([ru[st.idx], rp]))
        assert _rel(host(zu), st.embed_u(ref[:st.nu])) < 1e-9
        assert _rel(host(zp), ref[st.nu:]) < 1e-9
        u = torch.empty(om.u_dof, dtype=torch.float64, device="cuda")
        p = torch.empty(om.p_dof, dtype=torch.float64, device="cuda")
        rep = sg.solve(f, u, p)
        _, it_o, _ = solver.fgmres(st.stokes_matvec, b, Po.apply, rtol=1e-6)
        assert abs(rep.iters - it_o) <= 2, (sign, rep.iters, it_o)
        its[sign] = rep.iters
    assert its[-1] < its[1], its


@pytest.mark.parametrize("name", ["n8k2", "n4k3"])
def test_assembled_q1_levels_match_element_kernels(name):
    """Q1 multigrid levels applied as assembled 27-point stencils (built from the element
    kernel's own element matrices) give the element-kernel V-cycles up to rounding order, and
    both match the oracle; assemble_mb = 0 keeps the element kernels on every smoothed level
    (the coarsest dense solve is built from its stencil either way)."""
    wb = _wb()
    w, st, P, m, v, s = _pair(name)
    om = st.mesh
    sols = {mb: wb.Solver(m, v, a_l=w.a_l, a_r=w.a_r, assemble_mb=mb) for mb in (0.0, 1e6)}
    ru = random_vector(51, om.u_dof)
    ru[om.vel_boundary] = 0.0
    r = st.remove_mean(random_vector(52, om.p_dof))
    out = {}
    for mb, sv in sols.items():
        assert [L[:2] for L in sv.levels(0)] == [L[:2] for L in s.levels(0)]
        for li, (L, Lo) in enumerate(zip(sv.levels(0), P.A_mg.levels)):
            if li + 1 < len(P.A_mg.levels):
                assert abs(L[2] - Lo.lmax) <= 1e-9 * Lo.lmax
        zu = torch.empty(om.u_dof, dtype=torch.float64, device="cuda")
        sv.vcycle_A(dev(ru), zu)
        zl = torch.empty(om.p_dof, dtype=torch.float64, device="cuda")
        sv.vcycle_K(0, dev(r), zl)
        zr = torch.empty(om.p_dof, dtype=torch.float64, device="cuda")
        sv.vcycle_K(1, dev(r), zr)
        out[mb] = (host(zu), host(zl), host(zr))
        assert _rel(out[mb][0], st.embed_u(P.a_vcycle(ru[st.idx]))) < 1e-9
        assert _rel(out[mb][1], P.k_vcycle("l", r)) < 1e-9
        assert _rel(out[mb][2], P.k_vcycle("r", r)) < 1e-9
    for a, b in zip(out[0.0], out[1e6]):
        assert _rel(a, b) < 1e-11
    f = torch.empty(om.u_dof, dtype=torch.float64, device="cuda")
    wb.wb_rhs_sinker(m, w.centers(), w.delta, w.omega, w.beta, f)
    its = []
    for sv in sols.values():
        u = torch.empty(om.u_dof, dtype=torch.float64, device="cuda")
        p = torch.empty(om.p_dof, dtype=torch.float64, device="cuda")
        rep = sv.solve(f, u, p)
        assert rep.rel_res <= 1e-6
        its.append(rep.iters)
    assert abs(its[0] - its[1]) <= 1, its


@pytest.mark.parametrize("name", ["n8k2", "n4k3"])
def test_mass_schur_baseline_matches_oracle(name):
    """The diagonalized M_p(1/mu) Schur approximation (eq. 4, the baseline of Sec. 8): its
    inverse diagonal, the block preconditioner with it, and the FGMRES iteration count follow
    the oracle."""
    wb = _wb()
    w, st, P, m, v, s = _pair(name)
    om = st.mesh
    sm = wb.Solver(m, v, a_l=w.a_l, a_r=w.a_r, schur_approx=1)
    Pm = solver.Preconditioner(st, schur="mass")
    assert _rel(host(sm.query(9, 0, om.p_dof)), 1.0 / Pm.mass_diag) < 1e-13
    ru = random_vector(61, om.u_dof)
    ru[om.vel_boundary] = 0.0
    rp = st.remove_mean(random_vector(62, om.p_dof))
    zu = torch.empty(om.u_dof, dtype=torch.float64, device="cuda")
    zp = torch.empty(om.p_dof, dtype=torch.float64, device="cuda")
    sm.precond(dev(ru), dev(rp), zu, zp)
    ref = Pm.apply(np.concatenate([ru[st.idx], rp]))
    assert _rel(host(zp), ref[st.nu:]) < 1e-12
    assert _rel(host(zu), st.embed_u(ref[:st.nu])) < 1e-9
    f = torch.empty(om.u_dof, dtype=torch.float64, device="cuda")
    wb.wb_rhs_sinker(m, w.centers(), w.delta, w.omega, w.beta, f)
    u = torch.empty(om.u_dof, dtype=torch.float64, device="cuda")
    p = torch.empty(om.p_dof, dtype=torch.float64, device="cuda")
    rep = sm.solve(f, u, p)
    assert rep.rel_res <= 1e-6
    b = np.concatenate([st.F, np.zeros(st.np_)])
    _, it_o, _ = solver.fgmres(st.stokes_matvec, b, Pm.apply, rtol=1e-6)
    assert abs(rep.iters - it_o) <= 2, (rep.iters, it_o)


@pytest.mark.parametrize("name", ["n8k2", "n4k3"])
def test_gradient_weights_match_oracle(name):
    """The viscosity-gradient w-BFBT weights (remark of Sec. 4): lumped weight masses, Poisson
    coefficient, K_w V-cycle and FGMRES count follow the oracle."""
    wb = _wb()
    w = SETUPS[name]
    c = w.centers()
    st = solver.Stokes(w.N, w.k, c, w.delta, w.omega, w.mu_min, w.mu_max, a_l=w.a_l, a_r=w.a_r,
                       weights="grad")
    P = solver.Preconditioner(st)
    om = st.mesh
    m = wb.Mesh(w.N, w.k)
    v = wb.Viscosity.sinker(m, c, w.delta, w.omega, w.mu_min, w.mu_max)
    s = wb.Solver(m, v, a_l=w.a_l, a_r=w.a_r, weights=1)
    assert _rel(host(s.query(0, 0, om.n_nodes)), 1.0 / st.C_nodes) < 1e-13
    assert _rel(host(s.query(1, 0, om.n_nodes)), 1.0 / st.D_nodes) < 1e-13
    E, n3 = om.E, om.n ** 3
    assert _rel(host(s.query(6, 0, E * n3)), P.Pl_mg.levels[0].coef.reshape(-1)) < 1e-13
    r = st.remove_mean(random_vector(71, om.p_dof))
    out = torch.empty(om.p_dof, dtype=torch.float64, device="cuda")
    s.vcycle_K(0, dev(r), out)
    assert _rel(host(out), P.k_vcycle("l", r)) < 1e-9
    f = torch.empty(om.u_dof, dtype=torch.float64, device="cuda")
    wb.wb_rhs_sinker(m, c, w.delta, w.omega, w.beta, f)
    u = torch.empty(om.u_dof, dtype=torch.float64, device="cuda")
    p = torch.empty(om.p_dof, dtype=torch.float64, device="cuda")
    rep = s.solve(f, u, p)
    assert rep.rel_res <= 1e-6
    b = np.concatenate([st.F, np.zeros(st.np_)])
    _, it_o, _ = solver.fgmres(st.stokes_matvec, b, P.apply, rtol=1e-6)
    assert abs(rep.iters - it_o) <= 2, (rep.iters, it_o)


@pytest.mark.parametrize("name", ["n8k2", "n4k3"])
def test_diag_a_bfbt_matches_oracle(name):
    """diag(A)-BFBT (C = D = diag(A), Sec. 4): the per-DOF weights, the K_w diagonal, the Poisson
    coefficient, the K_w V-cycle and the FGMRES count follow the oracle."""
    wb = _wb()
    w = SETUPS[name]
    c = w.centers()
    st = solver.Stokes(w.N, w.k, c, w.delta, w.omega, w.mu_min, w.mu_max, a_l=1.0, a_r=1.0,
                       weights="diagA")
    P = solver.Preconditioner(st)
    om = st.mesh
    m = wb.Mesh(w.N, w.k)
    v = wb.Viscosity.sinker(m, c, w.delta, w.omega, w.mu_min, w.mu_max)
    s = wb.Solver(m, v, a_l=1.0, a_r=1.0, weights=2)
    assert _rel(host(s.query(0, 0, om.u_dof))[st.idx], st.Cinv) < 1e-13
    assert _rel(host(s.query(4, 0, om.p_dof)), P.disc["l"][1]) < 1e-12
    E, n3 = om.E, om.n ** 3
    assert _rel(host(s.query(6, 0, E * n3)), P.Pl_mg.levels[0].coef.reshape(-1)) < 1e-13
    r = st.remove_mean(random_vector(81, om.p_dof))
    out = torch.empty(om.p_dof, dtype=torch.float64, device="cuda")
    s.apply_K(0, dev(r), out)
    assert _rel(host(out), st.Kl @ r) < 1e-12
    s.vcycle_K(0, dev(r), out)
    assert _rel(host(out), P.k_vcycle("l", r)) < 1e-9
    f = torch.empty(om.u_dof, dtype=torch.float64, device="cuda")
    wb.wb_rhs_sinker(m, c, w.delta, w.omega, w.beta, f)
    u = torch.empty(om.u_dof, dtype=torch.float64, device="cuda")
    p = torch.empty(om.p_dof, dtype=torch.float64, device="cuda")
    rep = s.solve(f, u, p)
    assert rep.rel_res <= 1e-6
    b = np.concatenate([st.F, np.zeros(st.np_)])
    _, it_o, _ = solver.fgmres(st.stokes_matvec, b, P.apply, rtol=1e-6)
    assert abs(rep.iters - it_o) <= 2, (rep.iters, it_o)


def test_solver_rejects_invalid_options():
    """Out-of-range options fail with WB_EINVAL and a message, and leave no solver behind."""
    wb = _wb()
    w, st, P, m, v, s = _pair("n8k2")
    for kw, msg in ((dict(schur_approx=2), "schur_approx"), (dict(weights=3), "weights"),
                    (dict(assemble_mb=-1.0), "assemble_mb"), (dict(schur_sign=0), "schur_sign"),
                    (dict(lanczos_steps=5000), "lanczos_steps")):
        with pytest.raises(wb.WbError) as ei:
            wb.Solver(m, v, **kw)
        assert ei.value.code == wb.WB_EINVAL and msg in str(ei.value), (kw, str(ei.value))


def _oracle_subsolve(st, P, which, b):
    """The oracle's GMRES on A (which = 0) or K_l / K_r (1 / 2) with one V-cycle as preconditioner."""
    if which == 0:
        return solver.fgmres(lambda x: st.A @ x, b, P.a_vcycle, rtol=1e-6, max_iter=500)
    K, side = (st.Kl, "l") if which == 1 else (st.Kr, "r")
    return solver.fgmres(lambda x: K @ x, st.remove_mean(b), lambda v: P.k_vcycle(side, v), rtol=1e-6,
                         max_iter=500)


@pytest.mark.parametrize("name", ["n8k2", "n4k3", "n8k2dr10"])
def test_subsolve_matches_oracle(name):
    # the component sub-solves of the paper's Table 3: GMRES on A u = f and on K_l, K_r p = g, each
    # with one V-cycle as preconditioner, against the oracle's GMRES with its V-cycles
    w, st, P, m, v, s = _pair(name)
    om = st.mesh
    ru = random_vector(41, om.u_dof)
    ru[om.vel_boundary] = 0.0
    x = torch.empty(om.u_dof, dtype=torch.float64, device="cuda")
    rep = s.subsolve(0, dev(ru), x)
    xo, it_o, _ = _oracle_subsolve(st, P, 0, ru[st.idx])
    assert rep.rel_res <= 1e-6
    assert abs(rep.iters - it_o) <= 2, (rep.iters, it_o)
    assert _rel(host(x)[st.idx], xo) < 1e-5
    rp = random_vector(42, om.p_dof)
    xp = torch.empty(om.p_dof, dtype=torch.float64, device="cuda")
    for which in (1, 2):
        rep = s.subsolve(which, dev(rp), xp)
        xo, it_o, _ = _oracle_subsolve(st, P, which, rp)
        assert rep.rel_res <= 1e-6
        assert abs(rep.iters - it_o) <= 2, (which, rep.iters, it_o)
        assert _rel(host(xp), st.remove_mean(xo)) < 1e-5


def test_subsolve_iterations_at_32cubed_q2():
    # the Table 3 setting (k = 2, 32^3, 16 sinkers, DR 1e6, a_r = 2) with seeded centres: the
    # paper reports 18 GMRES iterations for A and 7 for K_r; different centres, so only
    # convergence and a band around those counts are checked (parity unpinned)
    wb = _wb()
    w = WORKLOADS["c2"]
    m = wb.Mesh(w.N, w.k)
    v = wb.Viscosity.sinker(m, w.centers(), w.delta, w.omega, w.mu_min, w.mu_max)
    s = wb.Solver(m, v, a_l=w.a_l, a_r=w.a_r)
    om = fem.Mesh(w.N, w.k)
    ru = random_vector(43, m.u_len)
    ru[om.vel_boundary] = 0.0
    ru = dev(ru)
    x = torch.empty(m.u_len, dtype=torch.float64, device="cuda")
    rep_a = s.subsolve(0, ru, x)
    rp = dev(random_vector(44, m.p_len))
    xp = torch.empty(m.p_len, dtype=torch.float64, device="cuda")
    rep_k = s.subsolve(2, rp, xp)
    print(f"32^3 Q2 sub-solves: A {rep_a.iters} iterations, K_r {rep_k.iters} iterations")
    assert rep_a.rel_res <= 1e-6 and rep_k.rel_res <= 1e-6
    assert 2 <= rep_a.iters <= 36 and 2 <= rep_k.iters <= 14


def test_solution_matches_oracle_fgmres_at_32cubed_q2():
    # the 32^3 Q2 workload (16 sinkers, DR 1e6) in full: the GPU FP64 solve against the oracle's
    # FGMRES driven to relative residual 1e-11 (paper eq. 2, the discrete solution)
    wb = _wb()
    w = WORKLOADS["c2"]
    c = w.centers()
    st = solver.Stokes(w.N, w.k, c, w.delta, w.omega, w.mu_min, w.mu_max, a_l=w.a_l, a_r=w.a_r)
    P = solver.Preconditioner(st)
    b = np.concatenate([st.F, np.zeros(st.np_)])
    xr, it_r, hist = solver.fgmres(st.stokes_matvec, b, P.apply, rtol=1e-11, max_iter=400)
    assert hist[-1] <= 1e-11
    u_ref, p_ref = xr[:st.nu], st.remove_mean(xr[st.nu:])
    m = wb.Mesh(w.N, w.k)
    v = wb.Viscosity.sinker(m, c, w.delta, w.omega, w.mu_min, w.mu_max)
    f = torch.empty(m.u_len, dtype=torch.float64, device="cuda")
    wb.wb_rhs_sinker(m, c, w.delta, w.omega, w.beta, f)
    u = torch.empty(m.u_len, dtype=torch.float64, device="cuda")
    p = torch.empty(m.p_len, dtype=torch.float64, device="cuda")
    errs = {}
    for rtol in (1e-6, 1e-7, 1e-8):
        s = wb.Solver(m, v, a_l=w.a_l, a_r=w.a_r, rtol=rtol)
        rep = s.solve(f, u, p)
        assert rep.rel_res <= rtol
        uh, ph = host(u)[st.idx], st.remove_mean(host(p))
        errs[rtol] = (np.linalg.norm(uh - u_ref) / np.linalg.norm(u_ref),
                      np.linalg.norm(ph - p_ref) / np.linalg.norm(p_ref), rep.iters)
        del s
    print("32^3 Q2 solution error against the oracle (rtol: du, dp, iterations):", errs)
    # at the paper's tolerance the solution is within 1e-4; driven to 1e-8 it is within 1e-6
    assert max(errs[1e-6][:2]) <= 1e-4
    assert max(errs[1e-8][:2]) <= 1e-6


@pytest.mark.parametrize("N", [11, 20])
def test_matrix_core_levels_match_line_kernels_across_bricks(N):
    """Order 3 in the brick form on meshes with several bricks in x, y and z (ragged tiles): the
    V-cycles of A and of both K_w, and the block preconditioner, with the matrix-core level
    operators (operator, brick-face sums, then the epilogue as its own pass) against the LDS-line
    kernels with the epilogue fused.  Both are the same operators up to rounding order.  (N = 20
    coarsens to 5^3; an odd N above 11 would leave a large coarsest level for the host's dense
    factorization.)"""
    wb = _wb()
    w = custom(f"n{N}k3", N, 3, n_sinkers=6, dr=1e6, seed=40 + N)
    m = wb.Mesh(N, 3)
    v = wb.Viscosity.sinker(m, w.centers(), w.delta, w.omega, w.mu_min, w.mu_max)
    ru = random_vector(71, m.u_len)
    rp = random_vector(72, m.p_len)
    prev_limit = wb.wb_set_two_pass_limit(0.0)
    prev_mc = wb.wb_set_matrix_core_ops(True)
    try:
        s = wb.Solver(m, v, a_l=w.a_l, a_r=w.a_r, use_graph=0)
        out = {}
        for on in (True, False):
            wb.wb_set_matrix_core_ops(on)
            za = torch.empty(m.u_len, dtype=torch.float64, device="cuda")
            s.vcycle_A(dev(ru), za)
            zk = []
            for side in (0, 1):
                z = torch.empty(m.p_len, dtype=torch.float64, device="cuda")
                s.vcycle_K(side, dev(rp), z)
                zk.append(host(z))
            zu = torch.empty(m.u_len, dtype=torch.float64, device="cuda")
            zp = torch.empty(m.p_len, dtype=torch.float64, device="cuda")
            s.precond(dev(ru), dev(rp), zu, zp)
            out[on] = (host(za), zk[0], zk[1], host(zu), host(zp))
    finally:
        wb.wb_set_two_pass_limit(prev_limit)
        wb.wb_set_matrix_core_ops(prev_mc)
    for a, b in zip(out[True], out[False]):
        assert np.all(np.isfinite(a))
        assert _rel(a, b) < 1e-10
