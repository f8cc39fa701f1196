"""Pins of the learned-correction oracle: convolution definition, adjoint, gradients, Adam,
node feature and the guarded correction step."""
import numpy as np
import pytest

from oracle import learned as L


def test_conv3d_matches_nested_loops():
    rng = np.random.default_rng(0)
    B, C, O, M = 2, 2, 3, 3
    x = rng.standard_normal((B, C, M, M, M))
    W = rng.standard_normal((O, C, 27))
    b = rng.standard_normal(O)
    y = L.conv3d(x, W, b)
    for bb in range(B):
        for o in range(O):
            for z in range(M):
                for yy in range(M):
                    for xx in range(M):
                        s = b[o]
                        for c in range(C):
                            for dz in range(3):
                                for dy in range(3):
                                    for dx in range(3):
                                        zi, yi, xi = z + dz - 1, yy + dy - 1, xx + dx - 1
                                        if 0 <= zi < M and 0 <= yi < M and 0 <= xi < M:
                                            s += W[o, c, dx + 3 * dy + 9 * dz] * x[bb, c, zi, yi, xi]
                        assert abs(y[bb, o, z, yy, xx] - s) < 1e-12


def test_conv3d_adjoint_identity():
    rng = np.random.default_rng(1)
    x = rng.standard_normal((2, 3, 5, 5, 5))
    gy = rng.standard_normal((2, 4, 5, 5, 5))
    W = rng.standard_normal((4, 3, 27))
    lhs = (L.conv3d(x, W, np.zeros(4)) * gy).sum()
    rhs = (x * L.conv3d_adjoint(gy, W)).sum()
    assert abs(lhs - rhs) <= 1e-11 * abs(lhs)


def test_conv3d_weight_gradient_is_exact_derivative():
    rng = np.random.default_rng(2)
    x = rng.standard_normal((2, 3, 4, 4, 4))
    gy = rng.standard_normal((2, 2, 4, 4, 4))
    W = rng.standard_normal((2, 3, 27))
    b = rng.standard_normal(2)
    dW, db = L.conv3d_wgrad(x, gy)
    f0 = (L.conv3d(x, W, b) * gy).sum()
    for (o, c, t) in [(0, 0, 0), (1, 2, 13), (0, 1, 26), (1, 0, 5)]:
        W1 = W.copy()
        W1[o, c, t] += 1.0          # the output is linear in W: the difference is exact
        assert abs((L.conv3d(x, W1, b) * gy).sum() - f0 - dW[o, c, t]) < 1e-9
    b1 = b.copy()
    b1[1] += 1.0
    assert abs((L.conv3d(x, W, b1) * gy).sum() - f0 - db[1]) < 1e-9


def test_network_gradient_matches_central_differences():
    H, M, B = 4, 4, 2
    rng = np.random.default_rng(3)
    p = L.init_params(H, 7) + 0.01 * rng.standard_normal(L.n_params(H))
    x = rng.standard_normal((B, 4, M, M, M))
    t = rng.standard_normal((B, 3, M, M, M))
    w = rng.uniform(0.5, 1.5, (B, 3, M, M, M))
    loss, g = L.loss_and_grad(p, x, t, w, H)
    eps = 1e-6
    idx = rng.choice(p.size, 25, replace=False)
    for i in idx:
        pp, pm = p.copy(), p.copy()
        pp[i] += eps
        pm[i] -= eps
        fd = (L.loss_and_grad(pp, x, t, w, H)[0] - L.loss_and_grad(pm, x, t, w, H)[0]) / (2 * eps)
        assert abs(fd - g[i]) <= 1e-5 * max(1.0, abs(g[i])), (i, fd, g[i])
    # a mistake in the activation slope would show here: the loss must match a direct evaluation
    o = L.forward(p, x, H)
    assert abs(loss - (w * (o - t) ** 2).sum() / B) < 1e-12


def test_adam_first_step_is_signed_learning_rate():
    g = np.array([3.0, -0.5, 1e-3, 0.0])
    p = np.ones(4)
    p1, m, v = L.adam_step(p, g, np.zeros(4), np.zeros(4), 1, 0.01)
    want = 1 - 0.01 * np.array([1.0, -1.0, 1.0, 0.0])
    assert np.allclose(p1, want, atol=1e-6)
    assert np.allclose(m, 0.1 * g) and np.allclose(v, 0.001 * g * g)


def test_node_feature_constant_and_two_valued_fields():
    N = 4
    coef = np.full((N ** 3, 8), 1e3)
    f = L.node_log_mu(coef, N)
    assert np.allclose(f, 3.0 / 5.0)
    # mu = 1 for ex < 2, 100 for ex >= 2: nodes x < 2 see only 0, x > 2 only 2/5, x = 2 the mean
    ex = np.arange(N ** 3) % N
    coef = np.where(ex[:, None] < 2, 1.0, 100.0) * np.ones((1, 8))
    f = L.node_log_mu(coef, N).reshape(N + 1, N + 1, N + 1)
    assert np.allclose(f[:, :, :2], 0.0) and np.allclose(f[:, :, 3:], 0.4)
    assert np.allclose(f[:, :, 2], 0.2)


def test_guarded_correction_never_increases_the_residual():
    import scipy.sparse as sp
    rng = np.random.default_rng(4)
    M, H = 4, 4
    n = 3 * M ** 3
    R = sp.random(n, n, density=0.05, random_state=5)
    A = (R @ R.T + sp.eye(n)).tocsr()
    d = A.diagonal()
    feat = rng.uniform(-1, 1, M ** 3)
    r = rng.standard_normal(n)
    p = L.init_params(H, 1)
    delta, alpha = L.guarded_correction(A, d, feat, r, p, H, M)
    assert 0.0 <= alpha <= 2.0
    assert np.linalg.norm(r - alpha * (A @ delta)) <= np.linalg.norm(r) * (1 + 1e-12)
    # exact inverse output: alpha = 1 and the residual vanishes
    e = np.linalg.solve(A.toarray(), r)
    Ad = A @ e
    assert abs(float(r @ Ad) / float(Ad @ Ad) - 1.0) < 1e-10


def test_vcycle_learned_hook_replaces_the_coarse_correction():
    # with the hook set to the plain coarse-grid correction of level lc (restriction, the cycle
    # below, prolongation), the hooked V-cycle is the plain V-cycle; with a zero correction it is
    # pre- and post-smoothing alone
    import numpy as np

    from oracle import fem, solver
    m = fem.Mesh(8, 2)
    mu = np.exp(np.random.default_rng(3).uniform(-2, 2, (m.E, m.n ** 3)))
    Hh = solver.Hierarchy(8, 2, mu, "velocity", 1000)
    lc = 1
    L = Hh.levels[lc]
    b = np.random.default_rng(4).uniform(-1, 1, Hh.levels[0].A.shape[0])
    plain = Hh.vcycle(b)
    same = Hh.vcycle(b, 0, (lc, lambda r: L.P @ Hh.vcycle(L.P.T @ r, lc + 1)))
    assert np.array_equal(plain, same)
    zero = Hh.vcycle(b, 0, (lc, lambda r: np.zeros_like(r)))
    assert np.abs(zero - plain).max() > 1e-6 * np.abs(plain).max()
