"""GPU parity of the learned coarse correction against the oracle (network forward, loss,
gradients, Adam, node feature, guarded correction step) and what training buys the solve."""
import numpy as np
import pytest
import scipy.sparse as sp

from oracle import learned as OL
from oracle import fem, sinker, solver
from synthetic import WORKLOADS, custom, random_vector, sinker_centers

pytestmark = pytest.mark.gpu

torch = pytest.importorskip("torch")

H = 16


def _wb():
    from paper_1607_03936_amd import wbfbt
    assert torch.cuda.is_available(), "GPU tests need a GPU"
    wbfbt.lib()
    return wbfbt


def dev(a, dtype=torch.float32):
    return torch.as_tensor(np.ascontiguousarray(a), dtype=dtype, device="cuda")


def host(t):
    torch.cuda.synchronize()
    return t.detach().cpu().numpy().astype(np.float64)


def _rel(a, b):
    return np.abs(a - b).max() / max(np.abs(b).max(), 1e-300)


def test_parameter_count_matches_oracle():
    wb = _wb()
    assert wb.lib().wb_net_param_count() == OL.n_params(H)


@pytest.mark.parametrize("M,B", [(9, 2), (5, 1), (17, 1)])
def test_forward_loss_and_gradient_match_oracle(M, B):
    """FP32 kernels vs the FP64 oracle.  Each output sums at most 16 * 27 = 432 products per
    layer over four layers, so its relative error is bounded by about 4 * 432 * 2^-24 ~ 1e-4;
    the weight gradients sum 256 products per block in FP32 before an FP64 sum over blocks,
    hence a few 1e-5 of their largest entry.  M = 9 and 17 span several 8 x 8 x 4 node tiles
    with ragged tails; M = 5 is a single partial tile."""
    wb = _wb()
    rng = np.random.default_rng(M * 10 + B)
    p = OL.init_params(H, 3) + 0.05 * rng.standard_normal(OL.n_params(H))
    x = rng.standard_normal((B, 4, M, M, M))
    t = rng.standard_normal((B, 3, M, M, M))
    w = rng.uniform(0.0, 2.0, (B, 3, M, M, M))
    p32, x32, t32, w32 = (a.astype(np.float32).astype(np.float64) for a in (p, x, t, w))
    loss_o, g_o = OL.loss_and_grad(p32, x32, t32, w32, H)
    out_o = OL.forward(p32, x32, H)
    out = torch.empty(B * 3 * M ** 3, dtype=torch.float32, device="cuda")
    grad = torch.empty(OL.n_params(H), dtype=torch.float32, device="cuda")
    loss = wb.wb_net_eval(M, B, dev(p), dev(x), out, dev(t), dev(w), grad)
    assert _rel(host(out), out_o.reshape(-1)) < 1e-4
    assert abs(loss - loss_o) <= 1e-4 * abs(loss_o)
    assert _rel(host(grad), g_o) < 2e-4
    # forward only
    out2 = torch.empty_like(out)
    wb.wb_net_eval(M, B, dev(p), dev(x), out2)
    assert torch.equal(out, out2)


def test_adam_step_matches_oracle():
    wb = _wb()
    rng = np.random.default_rng(5)
    n = OL.n_params(H)
    p, g = rng.standard_normal(n), rng.standard_normal(n)
    m, v = rng.standard_normal(n) * 0.1, rng.uniform(0, 0.1, n)
    want, wm, wv = OL.adam_step(p, g, m, v, 3, 1e-3)
    P, G, Mm, V = dev(p), dev(g), dev(m), dev(v)
    wb.wb_net_adam(P, G, Mm, V, 3, 1e-3)
    assert _rel(host(Mm), wm) < 1e-6 and _rel(host(V), wv) < 1e-6
    assert np.abs(host(P) - want).max() < 1e-6


def test_node_feature_matches_oracle():
    wb = _wb()
    N = 9
    rng = np.random.default_rng(6)
    coef = 10.0 ** rng.uniform(-4, 4, (N ** 3, 8))
    feat = torch.empty((N + 1) ** 3, dtype=torch.float32, device="cuda")
    wb.wb_net_feature(N, dev(coef, torch.float64), feat)
    assert np.abs(host(feat) - OL.node_log_mu(coef, N)).max() < 1e-6


_cache = {}


def _problem():
    """16^3 Q2 sinker problem: velocity levels Q2 16 -> Q1 16 -> Q1 8 (learned) -> Q1 4."""
    if "p" in _cache:
        return _cache["p"]
    wb = _wb()
    w = custom("l16", 16, 2, n_sinkers=6, dr=1e6, a_r=1.0, seed=11)
    m = wb.Mesh(w.N, w.k)
    v = wb.Viscosity.sinker(m, w.centers(), w.delta, w.omega, w.mu_min, w.mu_max)
    _cache["p"] = (w, m, v)
    return _cache["p"]


def test_guarded_probe_matches_oracle():
    wb = _wb()
    w, m, v = _problem()
    s = wb.Solver(m, v, a_l=w.a_l, a_r=w.a_r)
    lc, M, n = s.learned_info()
    assert (lc, M, n) == (2, 9, OL.n_params(H))
    p = OL.init_params(H, 9)
    s.learned_set(p)
    assert np.array_equal(s.learned_get(), p.astype(np.float32))
    # oracle level lc of the velocity hierarchy on the same viscosity
    mesh = fem.Mesh(w.N, w.k)
    mu_q = sinker.viscosity(mesh.quad_points(), w.centers(), w.delta, w.omega, w.mu_min, w.mu_max)
    Hh = solver.Hierarchy(w.N, w.k, mu_q, "velocity", 1000)
    L = Hh.levels[lc]
    full = 3 * M ** 3
    E = sp.csr_matrix((np.ones(L.idx.size), (L.idx, np.arange(L.idx.size))), shape=(full, L.idx.size))
    A = (E @ L.A @ E.T).tocsr()
    d = A.diagonal()
    feat = OL.node_log_mu(L.coef, L.N)
    r = random_vector(31, full)
    r[d == 0] = 0.0
    delta = torch.empty(full, dtype=torch.float64, device="cuda")
    alpha = s.learned_probe(dev(r, torch.float64), delta)
    p32 = p.astype(np.float32).astype(np.float64)
    d_o, a_o = OL.guarded_correction(A, d, feat.astype(np.float32), r, p32, H, M)
    assert _rel(host(delta), d_o) < 1e-4
    assert abs(alpha - a_o) <= 1e-4 * max(abs(a_o), 1e-3)
    assert np.all(host(delta)[d == 0] == 0.0)


def _oracle_learned_step(w, lc, M, params):
    """The oracle's learned coarse correction at level lc of the velocity hierarchy on the
    problem's viscosity: (hierarchy, step) with step(r) = alpha delta on interior vectors."""
    mesh = fem.Mesh(w.N, w.k)
    mu_q = sinker.viscosity(mesh.quad_points(), w.centers(), w.delta, w.omega, w.mu_min, w.mu_max)
    Hh = solver.Hierarchy(w.N, w.k, mu_q, "velocity", 1000)
    L = Hh.levels[lc]
    full = 3 * M ** 3
    E = sp.csr_matrix((np.ones(L.idx.size), (L.idx, np.arange(L.idx.size))), shape=(full, L.idx.size))
    A = (E @ L.A @ E.T).tocsr()
    d = A.diagonal()
    feat = OL.node_log_mu(L.coef, L.N).astype(np.float32)
    p32 = np.asarray(params, np.float32).astype(np.float64)

    def step(r):
        rf = np.zeros(full)
        rf[L.idx] = r
        delta, alpha = OL.guarded_correction(A, d, feat, rf, p32, H, M)
        return alpha * delta[L.idx]
    return Hh, step


def test_learned_vcycle_matches_oracle():
    # the V-cycle with the network in place of the coarse-grid correction below level lc
    wb = _wb()
    w, m, v = _problem()
    s = wb.Solver(m, v, a_l=w.a_l, a_r=w.a_r, use_learned=1)
    lc, M, n = s.learned_info()
    p = np.random.default_rng(5).normal(0.0, 0.05, n)
    s.learned_set(p)
    Hh, step = _oracle_learned_step(w, lc, M, p)
    om = fem.Mesh(w.N, w.k)
    # a smooth right-hand side (the sinker body force), for which the coarse-grid correction
    # matters, plus a random part
    f = torch.empty(om.u_dof, dtype=torch.float64, device="cuda")
    wb.wb_rhs_sinker(m, w.centers(), w.delta, w.omega, w.beta, f)
    ru = host(f) + 1e-3 * np.abs(host(f)).max() * random_vector(33, om.u_dof)
    ru[om.vel_boundary] = 0.0
    zu = torch.empty(om.u_dof, dtype=torch.float64, device="cuda")
    s.vcycle_A(dev(ru, torch.float64), zu)
    L0 = Hh.levels[0]
    want = np.zeros(om.u_dof)
    want[L0.idx] = Hh.vcycle(ru[L0.idx], 0, (lc, step))
    assert _rel(host(zu), want) < 1e-4
    # the plain cycle differs: the correction really stands in for the recursion
    plain = np.zeros(om.u_dof)
    plain[L0.idx] = Hh.vcycle(ru[L0.idx], 0)
    assert _rel(want, plain) > 1e-3


def test_corrupted_network_falls_back_to_the_plain_vcycle():
    # a network whose output is garbage: the first preconditioner apply rejects it, and the solve
    # runs with the plain V-cycle (same iterations and solution as the plain solver)
    wb = _wb()
    w, m, v = _problem()
    f = torch.empty(m.u_len, dtype=torch.float64, device="cuda")
    wb.wb_rhs_sinker(m, w.centers(), w.delta, w.omega, w.beta, f)
    u0 = torch.empty(m.u_len, dtype=torch.float64, device="cuda")
    p0 = torch.empty(m.p_len, dtype=torch.float64, device="cuda")
    r0 = wb.Solver(m, v, a_l=w.a_l, a_r=w.a_r).solve(f, u0, p0)
    s = wb.Solver(m, v, a_l=w.a_l, a_r=w.a_r, use_learned=1)
    lc, M, n = s.learned_info()
    s.learned_set(np.random.default_rng(6).normal(0.0, 3.0, n))
    u1 = torch.empty_like(u0)
    p1 = torch.empty_like(p0)
    r1 = s.solve(f, u1, p1)
    assert r1.fell_back >= 1 and r1.learned_reduction > 0.9
    assert r1.iters == r0.iters and r1.rel_res <= 1e-6
    assert (torch.linalg.norm(u1 - u0) / torch.linalg.norm(u0)).item() < 1e-10
    assert len(r1.history) == r1.iters and r1.history[-1] <= 1e-6


def test_training_and_solve_with_the_learned_correction():
    """Train on solver-generated pairs from seeded fields distinct from the evaluation field (seeds
    1000.., validation 3000..), then solve with the network standing in for the coarse-grid
    correction at level lc.  Training must reduce the loss; the solve must reach the tolerance with
    the plain solution's accuracy, whether the check keeps the network or falls back."""
    wb = _wb()
    w, m, v = _problem()
    f = torch.empty(m.u_len, dtype=torch.float64, device="cuda")
    wb.wb_rhs_sinker(m, w.centers(), w.delta, w.omega, w.beta, f)
    u0 = torch.empty(m.u_len, dtype=torch.float64, device="cuda")
    p0 = torch.empty(m.p_len, dtype=torch.float64, device="cuda")
    plain = wb.Solver(m, v, a_l=w.a_l, a_r=w.a_r)
    r0 = plain.solve(f, u0, p0)
    s = wb.Solver(m, v, a_l=w.a_l, a_r=w.a_r, use_learned=1)
    train = [sinker_centers(1000 + i, 6) for i in range(96)]
    valid = [sinker_centers(3000 + i, 6) for i in range(8)]
    rep = s.learned_train(train + valid, pairs_per_field=1, epochs=15, batch=4, lr=2e-3,
                          n_valid=len(valid), delta=w.delta, omega=w.omega, mu_min=w.mu_min,
                          mu_max=w.mu_max)
    print(f"train: pairs {rep.n_pairs} loss {rep.loss_first:.3e} -> {rep.loss_last:.3e} "
          f"valid {rep.valid_loss:.3e} ({rep.t_pairs_s:.2f}s pairs, {rep.t_train_s:.2f}s Adam)")
    assert rep.n_pairs == 104 and rep.loss_last < 0.9 * rep.loss_first
    assert 0.0 < rep.valid_loss < 2.0 * rep.loss_last + 1.0
    u1 = torch.empty_like(u0)
    p1 = torch.empty_like(p0)
    r1 = s.solve(f, u1, p1)
    print(f"solve: plain {r0.iters} its, learned {r1.iters} its (reduction at lc "
          f"{r1.learned_reduction:.3f}, accepted {r1.learned_used}, rejected/switched {r1.fell_back})")
    assert r1.rel_res <= 1e-6
    du = (torch.linalg.norm(u1 - u0) / torch.linalg.norm(u0)).item()
    assert du < 1e-4
    if r1.fell_back == 0:
        assert r1.learned_used > 0
    # the graph-replayed learned preconditioner matches the eagerly launched one
    eager = wb.Solver(m, v, a_l=w.a_l, a_r=w.a_r, use_learned=1, use_graph=0)
    eager.learned_set(s.learned_get())
    u2 = torch.empty_like(u0)
    p2 = torch.empty_like(p0)
    r2 = eager.solve(f, u2, p2)
    assert abs(r2.iters - r1.iters) <= 1
    assert (torch.linalg.norm(u2 - u1) / torch.linalg.norm(u1)).item() < 1e-8
