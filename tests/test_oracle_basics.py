"""Pins of the oracle's building blocks: rules, bases, DOF counts, sinker field, generator."""
import os

import numpy as np
import pytest

from oracle import fem, sinker, solver

GOLDEN = os.path.join(os.path.dirname(__file__), "golden")


@pytest.mark.parametrize("n", [2, 3, 4, 5, 6])
def test_gauss_and_gll_exactness(n):
    xg, wg = fem.gauss_rule(n)
    xl, wl = fem.gll_points(n), fem.gll_weights(n)
    for p in range(2 * n):           # Gauss: exact to degree 2n-1
        exact = (1.0 - (-1.0) ** (p + 1)) / (p + 1)
        assert abs(np.sum(wg * xg ** p) - exact) < 1e-13
    for p in range(2 * n - 2):       # GLL: exact to degree 2n-3
        exact = (1.0 - (-1.0) ** (p + 1)) / (p + 1)
        assert abs(np.sum(wl * xl ** p) - exact) < 1e-13
    assert xl[0] == -1.0 and xl[-1] == 1.0 and np.all(wl > 0)


@pytest.mark.parametrize("n", [2, 3, 4, 5])
def test_lagrange_cardinal_and_derivative(n):
    nodes = fem.gll_points(n)
    V, _ = fem.lagrange(nodes, nodes)
    assert np.allclose(V, np.eye(n), atol=1e-14)
    # interpolating x^p (p < n) is exact, and so is its derivative
    x = np.linspace(-1, 1, 7)
    V, D = fem.lagrange(nodes, x)
    for p in range(n):
        assert np.allclose(V @ nodes ** p, x ** p, atol=1e-13)
        assert np.allclose(D @ nodes ** p, p * x ** max(p - 1, 0) if p else 0 * x, atol=1e-12)


def test_dof_counts_match_table3():
    rows = np.loadtxt(os.path.join(GOLDEN, "table3_dofs.txt"))
    for k, lev, a_r, u, p, tot in rows:
        k, N = int(k), 2 ** int(lev)
        M = k * N + 1
        u_dof = 3 * M ** 3                       # includes boundary nodes
        p_dof = N ** 3 * len(fem.modes(k))
        # printed to two decimals, truncated or rounded
        assert abs(u_dof / 1e6 - u) <= 0.01, (k, lev)
        assert abs(p_dof / 1e6 - p) <= 0.01, (k, lev)
        assert abs((u_dof + p_dof) / 1e6 - tot) <= 0.01, (k, lev)
        if N <= 8:
            m = fem.Mesh(N, k)
            assert m.u_dof == u_dof and m.p_dof == p_dof


def test_a_r_schedule_matches_table3():
    from synthetic import default_a_r
    rows = np.loadtxt(os.path.join(GOLDEN, "table3_dofs.txt"))
    for k, lev, a_r, *_ in rows:
        assert default_a_r(2 ** int(lev), int(k)) == a_r


def test_mode_count_and_order():
    for k in range(1, 6):
        ms = fem.modes(k)
        assert len(ms) == k * (k + 1) * (k + 2) // 6
        assert ms[0] == (0, 0, 0)
        assert all(a + b + c <= k - 1 for a, b, c in ms)
    assert fem.modes(2) == [(0, 0, 0), (1, 0, 0), (0, 1, 0), (0, 0, 1)]


def test_sinker_field_properties():
    rng = np.random.default_rng(3)
    centers = rng.random((5, 3))
    mu_min, mu_max = 1e-3, 1e3
    # viscosity equals mu_max at each centre and inside the plateau of diameter omega
    mu_c = sinker.viscosity(centers, centers, 200.0, 0.1, mu_min, mu_max)
    assert np.allclose(mu_c, mu_max, rtol=0, atol=1e-12)
    near = centers + np.array([0.04, 0.0, 0.0])
    assert np.allclose(sinker.viscosity(near, centers, 200.0, 0.1, mu_min, mu_max), mu_max)
    x = rng.random((1000, 3))
    mu = sinker.viscosity(x, centers, 200.0, 0.1, mu_min, mu_max)
    assert np.all(mu >= mu_min) and np.all(mu <= mu_max)
    # no sinkers: chi is the empty product 1, so mu = mu_min and f = 0
    assert np.allclose(sinker.viscosity(x, np.zeros((0, 3)), 200.0, 0.1, mu_min, mu_max), mu_min)
    assert np.allclose(sinker.body_force(x, np.zeros((0, 3)), 200.0, 0.1), 0.0)
    # single sinker, one point at distance d: closed form
    c = np.array([[0.5, 0.5, 0.5]])
    d = 0.2
    chi = 1.0 - np.exp(-200.0 * (d - 0.05) ** 2)
    assert abs(sinker.chi(np.array([0.5 + d, 0.5, 0.5]), c, 200.0, 0.1) - chi) < 1e-15
    f = sinker.body_force(np.array([0.5 + d, 0.5, 0.5]), c, 200.0, 0.1, 10.0)
    assert np.allclose(f, [0, 0, 10.0 * (chi - 1.0)])


def test_splitmix64_published_values():
    # first two outputs of SplitMix64 from state 0 are 0xe220a8397b1dcdaf, 0x6e789e6aa1b965f4
    u = solver.splitmix64_uniform(0, 1)
    top53 = 0xe220a8397b1dcdaf >> 11
    assert u[0] == 2.0 * (top53 / 2.0 ** 53) - 1.0
    assert np.all(np.abs(solver.splitmix64_uniform(7, 10000)) <= 1.0)
