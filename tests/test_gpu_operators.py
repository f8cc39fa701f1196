"""GPU parity of the operator layer against the FP64 oracle (through the C-ABI).

Sizes span several thread blocks with a ragged tail: the operator kernel packs
256 / (k+1)^2 elements per block (64, 28, 16, 10 for k = 1..4).
"""
import numpy as np
import pytest

from oracle import fem, sinker, solver
from synthetic import WORKLOADS, sinker_centers, random_vector

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


CASES = [(9, 1), (8, 2), (7, 3), (5, 4), (3, 5)]
# the BF16 matrix-core forms are built for k <= 4
BF16_CASES = [c for c in CASES if c[1] <= 4]


@pytest.mark.parametrize("N,k", CASES)
def test_sinker_viscosity_and_load(N, k):
    wb = _wb()
    c = sinker_centers(11, 6)
    m = wb.Mesh(N, k)
    v = wb.Viscosity.sinker(m, c, 200.0, 0.1, 1e-3, 1e3)
    mq, mn = v.get()
    om = fem.Mesh(N, k)
    want_q = sinker.viscosity(om.quad_points(), c, 200.0, 0.1, 1e-3, 1e3).reshape(-1)
    want_n = sinker.viscosity(om.node_xyz, c, 200.0, 0.1, 1e-3, 1e3)
    assert _rel(host(mq), want_q) < 1e-13
    assert _rel(host(mn), want_n) < 1e-13
    f = torch.empty(m.u_len, dtype=torch.float64, device="cuda")
    wb.wb_rhs_sinker(m, c, 200.0, 0.1, 10.0, f)
    F = fem.assemble_load(om, sinker.body_force(om.quad_points(), c, 200.0, 0.1, 10.0))
    F[om.vel_boundary] = 0.0
    assert _rel(host(f), F) < 1e-13


@pytest.mark.parametrize("N,k", CASES)
def test_apply_A_matches_assembled(N, k):
    wb = _wb()
    om = fem.Mesh(N, k)
    rng = np.random.default_rng(N * 10 + k)
    mu_q = np.exp(rng.uniform(-6, 6, (om.E, om.n ** 3)))        # contrast ~1e5
    mu_n = np.exp(rng.uniform(-6, 6, om.n_nodes))
    m = wb.Mesh(N, k)
    v = wb.Viscosity.values(m, dev(mu_q.ravel()), dev(mu_n))
    u = random_vector(3, om.u_dof)
    y = torch.empty(m.u_len, dtype=torch.float64, device="cuda")
    wb.wb_apply_A(m, v, dev(u), y)
    A = fem.assemble_A(om, mu_q)
    ui = u.copy()
    ui[om.vel_boundary] = 0.0                                   # boundary input is ignored
    want = A @ ui
    want[om.vel_boundary] = 0.0                                 # boundary output is zero
    got = host(y)
    assert _rel(got, want) < 1e-12
    assert np.all(got[om.vel_boundary] == 0.0)


@pytest.mark.parametrize("N,k", CASES[1:])
def test_apply_B_BT_stokes_match_assembled(N, k):
    wb = _wb()
    om = fem.Mesh(N, k)
    rng = np.random.default_rng(k)
    mu_q = np.exp(rng.uniform(-3, 3, (om.E, om.n ** 3)))
    m = wb.Mesh(N, k)
    v = wb.Viscosity.values(m, dev(mu_q.ravel()), dev(np.ones(om.n_nodes)))
    u = random_vector(5, om.u_dof)
    p = random_vector(6, om.p_dof)
    ui = u.copy()
    ui[om.vel_boundary] = 0.0
    B = fem.assemble_B(om)
    pg = torch.empty(m.p_len, dtype=torch.float64, device="cuda")
    wb.wb_apply_B(m, dev(u), pg)
    assert _rel(host(pg), B @ ui) < 1e-12
    ug = torch.empty(m.u_len, dtype=torch.float64, device="cuda")
    wb.wb_apply_BT(m, dev(p), ug)
    want = B.T @ p
    want[om.vel_boundary] = 0.0
    assert _rel(host(ug), want) < 1e-12
    yu = torch.empty(m.u_len, dtype=torch.float64, device="cuda")
    yp = torch.empty(m.p_len, dtype=torch.float64, device="cuda")
    wb.wb_apply_stokes(m, v, dev(u), dev(p), yu, yp)
    A = fem.assemble_A(om, mu_q)
    wu = A @ ui + B.T @ p
    wu[om.vel_boundary] = 0.0
    assert _rel(host(yu), wu) < 1e-12
    assert _rel(host(yp), B @ ui) < 1e-12


def test_bf16_forms_rejected_at_order_5():
    wb = _wb()
    m = wb.Mesh(3, 5)
    nq = m.q_len
    v = wb.Viscosity.values(m, dev(np.ones(nq)), dev(np.ones(m.n_nodes)))
    u = torch.zeros(m.u_len, dtype=torch.float32, device="cuda")
    y = torch.empty_like(u)
    with pytest.raises(Exception, match="k <= 4"):
        wb.wb_apply_A_lowp(m, v, wb.WB_BF16, u, y)


def test_apply_A_fp32_error_is_single_precision():
    wb = _wb()
    N, k = 8, 2
    om = fem.Mesh(N, k)
    rng = np.random.default_rng(0)
    mu_q = np.exp(rng.uniform(-3, 3, (om.E, om.n ** 3)))
    m = wb.Mesh(N, k)
    v = wb.Viscosity.values(m, dev(mu_q.ravel()), dev(np.ones(om.n_nodes)))
    u = random_vector(1, om.u_dof)
    y32 = torch.empty(m.u_len, dtype=torch.float32, device="cuda")
    wb.wb_apply_A_lowp(m, v, wb.WB_FP32, dev(u).float(), y32)
    ui = u.copy()
    ui[om.vel_boundary] = 0
    want = fem.assemble_A(om, mu_q) @ ui
    want[om.vel_boundary] = 0
    err = np.linalg.norm(host(y32).astype(np.float64) - want) / np.linalg.norm(want)
    assert 1e-9 < err < 1e-5


@pytest.mark.parametrize("N,k", BF16_CASES)
@pytest.mark.parametrize("form", ["bf16x1", "bf16x3"])
def test_apply_A_bf16_mfma_error(N, k, form):
    """BF16 forms: every 1D contraction runs on the BF16 matrix cores with FP32 accumulation.
    A value passes through six contractions (three forward, three transposed).  bf16x1 rounds the
    table and the line to BF16 (unit roundoff 2^-9 each), so the relative error is a few times
    6 * 2 * 2^-9 ~ 2.3e-2 at most; bf16x3 keeps high and low BF16 parts of both and drops only the
    low x low product and the rounding of the low parts (~2^-16 per contraction, ~2e-4 for six).
    Both must stay above the FP32 level (~1e-7), which shows the matrix-core path ran."""
    wb = _wb()
    om = fem.Mesh(N, k)
    rng = np.random.default_rng(3)
    mu_q = np.exp(rng.uniform(-3, 3, (om.E, om.n ** 3)))
    m = wb.Mesh(N, k)
    v = wb.Viscosity.values(m, dev(mu_q.ravel()), dev(np.ones(om.n_nodes)))
    u = random_vector(4, om.u_dof)
    ui = u.copy()
    ui[om.vel_boundary] = 0
    want = fem.assemble_A(om, mu_q) @ ui
    want[om.vel_boundary] = 0
    y = torch.empty(m.u_len, dtype=torch.float32, device="cuda")
    prec = wb.WB_BF16X1 if form == "bf16x1" else wb.WB_BF16
    wb.wb_apply_A_lowp(m, v, prec, dev(u).float(), y)
    yh = host(y).astype(np.float64)
    err = np.linalg.norm(yh - want) / np.linalg.norm(want)
    print(f"{form} A apply N={N} k={k}: relative error {err:.3e}")
    assert np.all(yh[om.vel_boundary] == 0.0)
    if form == "bf16x1":
        assert 1e-4 < err < 2.5e-2
    else:
        assert 3e-7 < err < 2e-4


@pytest.mark.parametrize("name", ["c2", "c5"])
def test_apply_A_full_size_sampled_rows(name):
    # the workload sizes, checked on sampled rows computed element by element by the oracle
    wb = _wb()
    w = WORKLOADS[name]
    c = w.centers()
    m = wb.Mesh(w.N, w.k)
    v = wb.Viscosity.sinker(m, c, w.delta, w.omega, w.mu_min, w.mu_max)
    om = fem.Mesh(w.N, w.k)
    u = random_vector(17, om.u_dof)
    u[om.vel_boundary] = 0.0
    y = torch.empty(m.u_len, dtype=torch.float64, device="cuda")
    wb.wb_apply_A(m, v, dev(u), y)
    got = host(y)

    def mu_of(els):
        return sinker.viscosity(om.quad_points(els), c, w.delta, w.omega, w.mu_min, w.mu_max)

    rng = np.random.default_rng(99)
    interior = om.vel_interior
    dofs = rng.choice(interior, 200, replace=False)
    # include the first and last interior DOFs (block tails) and DOFs next to the boundary
    dofs = np.concatenate([dofs, interior[:3], interior[-3:]])
    want = fem.apply_A_rows(om, mu_of, u, dofs)
    scale = np.abs(want).max()
    assert np.abs(got[dofs] - want).max() <= 1e-12 * scale
    assert np.all(got[om.vel_boundary] == 0.0)


@pytest.mark.parametrize("name", ["c2", "c5"])
def test_apply_B_BT_full_size_sampled_rows(name):
    # the divergence and gradient at the workload sizes (their launch shapes at full size),
    # checked on sampled elements and velocity DOFs computed element by element by the oracle
    wb = _wb()
    w = WORKLOADS[name]
    m = wb.Mesh(w.N, w.k)
    om = fem.Mesh(w.N, w.k)
    n3, npm = om.n ** 3, om.n_p
    Be = fem.element_div(w.k, om.h)
    u = random_vector(21, om.u_dof)
    u[om.vel_boundary] = 0.0
    p = random_vector(22, om.p_dof)
    pg = torch.empty(m.p_len, dtype=torch.float64, device="cuda")
    wb.wb_apply_B(m, dev(u), pg)
    ug = torch.empty(m.u_len, dtype=torch.float64, device="cuda")
    wb.wb_apply_BT(m, dev(p), ug)
    got_p, got_u = host(pg), host(ug)

    rng = np.random.default_rng(23)
    els = np.concatenate([rng.choice(om.E, 200, replace=False), [0, 1, om.E - 2, om.E - 1]])
    for e in els:
        gd = np.concatenate([c * om.n_nodes + om.elem_nodes[e] for c in range(3)])
        want = Be @ u[gd]
        assert np.abs(got_p[e * npm:(e + 1) * npm] - want).max() <= 1e-12 * np.abs(want).max()

    interior = om.vel_interior
    dofs = np.concatenate([rng.choice(interior, 200, replace=False), interior[:3], interior[-3:]])
    want = np.zeros(len(dofs))
    for t, d in enumerate(dofs):
        c, g = divmod(int(d), om.n_nodes)
        for e in fem.elements_of_node(om, g):
            li = int(np.flatnonzero(om.elem_nodes[e] == g)[0])
            want[t] += Be[:, c * n3 + li] @ p[e * npm:(e + 1) * npm]
    assert np.abs(got_u[dofs] - want).max() <= 1e-12 * np.abs(want).max()
    assert np.all(got_u[om.vel_boundary] == 0.0)


@pytest.mark.parametrize("N,k", [(8, 2), (5, 4)])
def test_apply_A_brick_and_two_pass_forms_match_assembled(N, k):
    # the two forms of the A apply (brick scatter with face sums; element pass with node sums),
    # each against the assembled oracle
    wb = _wb()
    om = fem.Mesh(N, k)
    rng = np.random.default_rng(11)
    mu_q = np.exp(rng.uniform(-3, 3, (om.E, om.n ** 3)))
    m = wb.Mesh(N, k)
    v = wb.Viscosity.values(m, dev(mu_q.ravel()), dev(np.ones(om.n_nodes)))
    u = random_vector(12, om.u_dof)
    ui = u.copy()
    ui[om.vel_boundary] = 0.0
    want = fem.assemble_A(om, mu_q) @ ui
    want[om.vel_boundary] = 0.0
    prev = wb.wb_set_two_pass_limit(128.0)
    try:
        for limit in (0.0, 128.0):
            wb.wb_set_two_pass_limit(limit)
            y = torch.empty(m.u_len, dtype=torch.float64, device="cuda")
            wb.wb_apply_A(m, v, dev(u), y)
            assert _rel(host(y), want) < 1e-12, limit
    finally:
        wb.wb_set_two_pass_limit(prev)


@pytest.mark.parametrize("N", [4, 11])
def test_apply_A_q3_matrix_core_form_matches_assembled(N):
    # order 3 above the two-pass size: the matrix-core brick kernel (x and y contractions on the
    # FP64 matrix cores) and the LDS line kernel, each against the assembled oracle; N = 11 gives
    # ragged tiles in x and y and one-layer brick chunks in z.  The matrix-core form sums each
    # node's contributions in a fixed order, so repeated applies agree bit for bit.
    wb = _wb()
    om = fem.Mesh(N, 3)
    rng = np.random.default_rng(N)
    mu_q = 10.0 ** rng.uniform(-4, 4, (om.E, om.n ** 3))
    m = wb.Mesh(N, 3)
    v = wb.Viscosity.values(m, dev(mu_q.ravel()), dev(np.ones(om.n_nodes)))
    u = random_vector(13, om.u_dof)
    ui = u.copy()
    ui[om.vel_boundary] = 0.0
    want = fem.assemble_A(om, mu_q) @ ui
    want[om.vel_boundary] = 0.0
    prev_limit = wb.wb_set_two_pass_limit(0.0)
    prev_mc = wb.wb_set_matrix_core_ops(True)
    try:
        for on in (True, False):
            wb.wb_set_matrix_core_ops(on)
            y = torch.empty(m.u_len, dtype=torch.float64, device="cuda")
            wb.wb_apply_A(m, v, dev(u), y)
            got = host(y)
            assert _rel(got, want) < 1e-12, on
            assert np.all(got[om.vel_boundary] == 0.0)
            if on:
                y2 = torch.empty(m.u_len, dtype=torch.float64, device="cuda")
                wb.wb_apply_A(m, v, dev(u), y2)
                assert np.array_equal(host(y2), got)
    finally:
        wb.wb_set_two_pass_limit(prev_limit)
        wb.wb_set_matrix_core_ops(prev_mc)


@pytest.mark.parametrize("N", [4, 11])
def test_stokes_operator_q3_brick_forms_match_assembled(N):
    # order 3 above the two-pass size: with the matrix cores the Stokes operator runs as the
    # matrix-core A, then B^T added, then B; without them as the fused LDS-line kernel
    wb = _wb()
    om = fem.Mesh(N, 3)
    rng = np.random.default_rng(60 + N)
    mu_q = 10.0 ** rng.uniform(-4, 4, (om.E, om.n ** 3))
    m = wb.Mesh(N, 3)
    v = wb.Viscosity.values(m, dev(mu_q.ravel()), dev(np.ones(om.n_nodes)))
    u = random_vector(15, om.u_dof)
    p = random_vector(16, om.p_dof)
    ui = u.copy()
    ui[om.vel_boundary] = 0.0
    B = fem.assemble_B(om)
    wu = fem.assemble_A(om, mu_q) @ ui + B.T @ p
    wu[om.vel_boundary] = 0.0
    wp = B @ ui
    prev_limit = wb.wb_set_two_pass_limit(0.0)
    prev_mc = wb.wb_set_matrix_core_ops(True)
    try:
        for on in (True, False):
            wb.wb_set_matrix_core_ops(on)
            yu = torch.full((m.u_len,), float("nan"), dtype=torch.float64, device="cuda")
            yp = torch.full((m.p_len,), float("nan"), dtype=torch.float64, device="cuda")
            wb.wb_apply_stokes(m, v, dev(u), dev(p), yu, yp)
            assert _rel(host(yu), wu) < 1e-12, on
            assert _rel(host(yp), wp) < 1e-12, on
    finally:
        wb.wb_set_two_pass_limit(prev_limit)
        wb.wb_set_matrix_core_ops(prev_mc)


@pytest.mark.parametrize("N", [4, 11])
def test_apply_A_q3_fp32_storage_forms(N):
    # the FP32 precision form at order 3 above the two-pass size: FP32 vectors and coefficient in
    # memory, FP64 arithmetic on the matrix cores (or FP32 line contractions in LDS with the
    # matrix cores switched off).  Both round to FP32 (relative error 1e-9 .. 1e-5 against the
    # assembled FP64 oracle); the matrix-core form only rounds its inputs and outputs, so it
    # lands closer than the FP32-arithmetic line form.
    wb = _wb()
    om = fem.Mesh(N, 3)
    rng = np.random.default_rng(40 + N)
    mu_q = 10.0 ** rng.uniform(-4, 4, (om.E, om.n ** 3))
    m = wb.Mesh(N, 3)
    v = wb.Viscosity.values(m, dev(mu_q.ravel()), dev(np.ones(om.n_nodes)))
    u = random_vector(14, om.u_dof)
    ui = u.copy()
    ui[om.vel_boundary] = 0.0
    want = fem.assemble_A(om, mu_q) @ ui
    want[om.vel_boundary] = 0.0
    prev_limit = wb.wb_set_two_pass_limit(0.0)
    prev_mc = wb.wb_set_matrix_core_ops(True)
    errs = {}
    try:
        for on in (True, False):
            wb.wb_set_matrix_core_ops(on)
            y = torch.empty(m.u_len, dtype=torch.float32, device="cuda")
            wb.wb_apply_A_lowp(m, v, wb.WB_FP32, dev(u).float(), y)
            got = host(y).astype(np.float64)
            errs[on] = _rel(got, want)
            assert np.all(got[om.vel_boundary] == 0.0)
            if on:
                y2 = torch.empty_like(y)
                wb.wb_apply_A_lowp(m, v, wb.WB_FP32, dev(u).float(), y2)
                assert torch.equal(y, y2)
    finally:
        wb.wb_set_two_pass_limit(prev_limit)
        wb.wb_set_matrix_core_ops(prev_mc)
    print(f"FP32 A N={N} k=3: matrix cores {errs[True]:.2e}, LDS lines {errs[False]:.2e}")
    assert 1e-9 < errs[True] < 1e-5 and 1e-9 < errs[False] < 1e-5
    assert errs[True] <= errs[False]


@pytest.mark.parametrize("N,k", [c for c in BF16_CASES if c[1] >= 2])
@pytest.mark.parametrize("form", ["fp32", "bf16x3", "bf16x1"])
def test_apply_B_BT_low_precision(N, k, form):
    """Reduced-precision divergence and gradient against the assembled oracle.  FP32: FP32 rounding
    (relative error 1e-9 .. 1e-5).  BF16 on the matrix cores: three contractions per value,
    bf16x3 about 2^-16 each, bf16x1 about 2^-8 each, both above the FP32 level."""
    wb = _wb()
    om = fem.Mesh(N, k)
    m = wb.Mesh(N, k)
    B = fem.assemble_B(om)
    u = random_vector(51, om.u_dof)
    ui = u.copy()
    ui[om.vel_boundary] = 0.0
    p = random_vector(52, om.p_dof)
    prec = {"fp32": wb.WB_FP32, "bf16x3": wb.WB_BF16, "bf16x1": wb.WB_BF16X1}[form]
    pg = torch.empty(m.p_len, dtype=torch.float32, device="cuda")
    wb.wb_apply_B_lowp(m, prec, dev(u).float(), pg)
    ug = torch.empty(m.u_len, dtype=torch.float32, device="cuda")
    wb.wb_apply_BT_lowp(m, prec, dev(p).float(), ug)
    want_p = B @ ui
    want_u = B.T @ p
    want_u[om.vel_boundary] = 0.0
    ep = np.linalg.norm(host(pg).astype(np.float64) - want_p) / np.linalg.norm(want_p)
    eu = np.linalg.norm(host(ug).astype(np.float64) - want_u) / np.linalg.norm(want_u)
    print(f"{form} N={N} k={k}: B {ep:.2e}, B^T {eu:.2e}")
    assert np.all(host(ug)[om.vel_boundary] == 0.0)
    lo, hi = {"fp32": (1e-10, 1e-5), "bf16x3": (3e-8, 2e-4), "bf16x1": (1e-4, 2.5e-2)}[form]
    assert lo < ep < hi and lo < eu < hi
