"""Pins of the oracle functions that the operator pins do not reach.

* the scalar Poisson stiffness (the continuous Q_k re-discretization of K_w, Sec. 6): the energy
  of a polynomial equals its exact integral (sympy), constants span the kernel, and a Q_k
  manufactured Dirichlet solution is reproduced exactly;
* the coefficient coarsening (the L2 adjoint of element-wise interpolation, Sec. 6) on a field
  of contrast 1e10, where the adjoint undershoots: unclamped entries equal an independently
  evaluated adjoint, clamped ones the element minimum;
* the row-wise A evaluation used for the sampled full-size GPU checks: equal to the assembled
  rows at corner, edge, face and interior nodes, and the element lists equal a brute-force scan.
"""
import itertools

import numpy as np
import pytest
import scipy.sparse.linalg as spla
import sympy as sy

from oracle import fem
from synthetic import random_vector

X, Y, Z = sy.symbols("x y z")


def _random_qk_poly(k, seed):
    """A polynomial of degree <= k in each variable (so in Q_k) with seeded coefficients."""
    rng = np.random.default_rng(seed)
    terms = []
    for i, j, l in itertools.product(range(k + 1), repeat=3):
        if rng.random() < 0.5 or (i, j, l) == (k, k, k):
            terms.append(sy.Rational(int(rng.integers(-9, 10)), int(rng.integers(1, 5)))
                         * X ** i * Y ** j * Z ** l)
    return sum(terms)


def _at_nodes(expr, m):
    f = sy.lambdify((X, Y, Z), expr, "numpy")
    p = m.node_xyz
    return np.broadcast_to(f(p[:, 0], p[:, 1], p[:, 2]), (m.n_nodes,)).astype(float)


@pytest.mark.parametrize("k", [2, 3, 4])
def test_poisson_energy_equals_exact_integral(k):
    # u^T L u = sum_e c_e int_e |grad u|^2 for u in Q_k, integrated exactly by sympy per element.
    N = 2
    m = fem.Mesh(N, k)
    u = _random_qk_poly(k, 10 + k)
    uh = _at_nodes(u, m)
    g2 = sum(sy.diff(u, v) ** 2 for v in (X, Y, Z))
    h = sy.Rational(1, N)
    elem_int = []
    for e in range(m.E):
        ex, ey, ez = m.eidx[e]
        elem_int.append(float(sy.integrate(g2, (X, ex * h, (ex + 1) * h), (Y, ey * h, (ey + 1) * h),
                                           (Z, ez * h, (ez + 1) * h))))
    elem_int = np.array(elem_int)
    # constant coefficient
    L1 = fem.assemble_poisson(m, np.full((m.E, m.n ** 3), 2.5))
    assert abs(uh @ (L1 @ uh) - 2.5 * elem_int.sum()) <= 1e-11 * 2.5 * elem_int.sum()
    # element-wise constant coefficient: each element's energy carries its own coefficient
    ce = np.random.default_rng(k).uniform(1e-3, 1e3, m.E)
    Lc = fem.assemble_poisson(m, np.repeat(ce[:, None], m.n ** 3, axis=1))
    want = (ce * elem_int).sum()
    assert abs(uh @ (Lc @ uh) - want) <= 1e-11 * want
    # symmetric, constants in the kernel (Neumann), positive semi-definite energy
    assert abs(Lc - Lc.T).max() <= 1e-13 * abs(Lc).max()
    assert np.abs(Lc @ np.ones(m.n_nodes)).max() <= 1e-12 * abs(Lc).max()


@pytest.mark.parametrize("N,k", [(2, 2), (3, 2), (2, 3), (1, 4)])
def test_poisson_manufactured_dirichlet_solution_exact(N, k):
    # -div(c grad u*) = f with c = 1.5 and u* = x(1-x)y(1-y)z(1-z) in Q_2 (subset of Q_k):
    # the Galerkin solution with exactly integrated load is u* itself.
    c = 1.5
    us = X * (1 - X) * Y * (1 - Y) * Z * (1 - Z)
    f = -c * sum(sy.diff(us, v, 2) for v in (X, Y, Z))
    m = fem.Mesh(N, k)
    L = fem.assemble_poisson(m, np.full((m.E, m.n ** 3), c))
    fq = sy.lambdify((X, Y, Z), f, "numpy")
    xq = m.quad_points()
    vals = np.broadcast_to(fq(xq[..., 0], xq[..., 1], xq[..., 2]), xq.shape[:-1])
    R = fem.reference(k)
    Fe = np.einsum("q,eq,qi->ei", R["W"] * m.h ** 3 / 8.0, vals, R["Phi"])
    F = np.zeros(m.n_nodes)
    np.add.at(F, m.elem_nodes, Fe)
    I = np.flatnonzero(~m.boundary)
    sol = spla.spsolve(L[I][:, I].tocsc(), F[I])
    exact = _at_nodes(us, m)
    assert np.abs(sol - exact[I]).max() <= 1e-11 * np.abs(exact).max()


def _adjoint_p_direct(fine, nf, nc):
    """c_j = <P e_j, f>_fine / W_c(j), e_j the j-th coarse Gauss-Lagrange polynomial, evaluated
    point by point (no matrix of the oracle's)."""
    xf, wf = fem.gauss_rule(nf)
    xc, wc = fem.gauss_rule(nc)
    Lc, _ = fem.lagrange(xc, xf)                      # [qf, qc]: coarse cardinal at fine points
    out = np.zeros((fine.shape[0], nc ** 3))
    for jz, jy, jx in itertools.product(range(nc), repeat=3):
        j = jx + nc * (jy + nc * jz)
        acc = np.zeros(fine.shape[0])
        for qz, qy, qx in itertools.product(range(nf), repeat=3):
            q = qx + nf * (qy + nf * qz)
            acc += Lc[qx, jx] * Lc[qy, jy] * Lc[qz, jz] * wf[qx] * wf[qy] * wf[qz] * fine[:, q]
        out[:, j] = acc / (wc[jx] * wc[jy] * wc[jz])
    return out


def _contrast_field(E, n, seed):
    """Per element, Gauss values of contrast 1e10: one large value, the rest tiny."""
    rng = np.random.default_rng(seed)
    f = 10.0 ** rng.uniform(-5, -4, (E, n ** 3))
    hot = rng.integers(0, n ** 3, E)
    f[np.arange(E), hot] = 10.0 ** rng.uniform(4.5, 5, E)
    return f


@pytest.mark.parametrize("nf,nc", [(3, 2), (5, 3), (4, 2)])
def test_coefficient_p_clamp_on_high_contrast(nf, nc):
    # Reading: the adjoint is kept wherever it stays above the element's smallest fine value and
    # replaced by that value elsewhere, so coarse operators keep a positive coefficient.  On a
    # field of contrast 1e10 the adjoint undershoots (it turns negative next to a spike).
    fine = _contrast_field(40, nf, nf + 7 * nc)
    adj = _adjoint_p_direct(fine, nf, nc)
    lo = fine.min(axis=1, keepdims=True)
    out = fem.coarsen_coefficient_p(fine, nf, nc)
    on = adj < lo
    assert on.any() and (~on).any()
    assert (adj < 0).any()                             # without the clamp: indefinite operators
    assert np.allclose(out[~on], adj[~on], rtol=1e-12, atol=0)
    assert np.array_equal(out[on], np.broadcast_to(lo, out.shape)[on])
    assert np.all(out > 0)


def test_coefficient_h_clamp_on_high_contrast():
    Nf, n = 4, 3
    Nc = Nf // 2
    fine = _contrast_field(Nf ** 3, n, 3)
    out = fem.coarsen_coefficient_h(fine, Nf, n)
    # direct adjoint: coarse cardinal polynomials at the children's Gauss points (child s of a
    # coarse element covers [s-1, s] in coarse reference coordinates), weights w_f / 2 per dim
    xf, wf = fem.gauss_rule(n)
    xc, wc = fem.gauss_rule(n)
    mf = fem.Mesh(Nf, 1)
    adj = np.zeros((Nc ** 3, n ** 3))
    lo = np.full(Nc ** 3, np.inf)
    for ce in range(Nc ** 3):
        cx, cy, cz = ce % Nc, (ce // Nc) % Nc, ce // (Nc * Nc)
        for sz, sy_, sx in itertools.product(range(2), repeat=3):
            fe = (2 * cx + sx) + Nf * ((2 * cy + sy_) + Nf * (2 * cz + sz))
            lo[ce] = min(lo[ce], fine[fe].min())
            Lx, _ = fem.lagrange(xc, 0.5 * (xf + 2 * sx - 1))
            Ly, _ = fem.lagrange(xc, 0.5 * (xf + 2 * sy_ - 1))
            Lz, _ = fem.lagrange(xc, 0.5 * (xf + 2 * sz - 1))
            for jz, jy, jx in itertools.product(range(n), repeat=3):
                j = jx + n * (jy + n * jz)
                for qz, qy, qx in itertools.product(range(n), repeat=3):
                    q = qx + n * (qy + n * qz)
                    adj[ce, j] += (Lx[qx, jx] * Ly[qy, jy] * Lz[qz, jz] * wf[qx] * wf[qy] * wf[qz]
                                   / 8.0 * fine[fe, q])
        adj[ce] /= fem.kron3(wc, wc, wc)
    assert mf.E == Nf ** 3
    on = adj < lo[:, None]
    assert on.any() and (~on).any()
    assert np.allclose(out[~on], adj[~on], rtol=1e-12, atol=0)
    assert np.array_equal(out[on], np.broadcast_to(lo[:, None], out.shape)[on])


@pytest.mark.parametrize("k", [2, 3, 4])
def test_elements_of_node_brute_force(k):
    m = fem.Mesh(3, k)
    for g in range(m.n_nodes):
        want = sorted(np.flatnonzero((m.elem_nodes == g).any(axis=1)).tolist())
        assert sorted(fem.elements_of_node(m, g)) == want


@pytest.mark.parametrize("k", [2, 3, 4])
def test_apply_A_rows_equal_assembled_rows(k):
    m = fem.Mesh(3, k)
    rng = np.random.default_rng(k)
    mu = 10.0 ** rng.uniform(-3, 3, (m.E, m.n ** 3))
    A = fem.assemble_A(m, mu)
    u = rng.uniform(-1, 1, m.u_dof)
    M = m.M
    picks = {
        "corner": 0,
        "edge": 1,                                        # on the x edge y = z = 0
        "face": 1 + M * 1,                                # on the face z = 0
        "vertex between 8 elements": k + M * (k + M * k),
        "edge between 4 elements": 1 + M * (k + M * k),
        "face between 2 elements": 1 + M * (1 + M * k),
        "element interior": 1 + M * (1 + M * 1),
        "far corner": m.n_nodes - 1,
    }
    dofs = [c * m.n_nodes + g for g in picks.values() for c in range(3)]
    got = fem.apply_A_rows(m, lambda els: mu[els], u, dofs)
    want = A[dofs] @ u
    assert np.allclose(got, want, rtol=1e-12, atol=1e-12 * np.abs(want).max())


@pytest.mark.parametrize("N,k", [(2, 2), (2, 3), (1, 4)])
def test_modal_restriction_equals_lumped_mass_projection_of_residuals(N, k):
    """The modal <-> nodal transfer of the K_w multigrid (Sec. 6) is an L2 projection with a
    lumped nodal mass.  For a residual (a dual vector r over the pressure modes) the projection
    onto the continuous nodal space and back to a dual vector is
        M~_Q (M~_Q^-1 G^T M_psi^-1 r) = G^T M_psi^-1 r,
    G[m, i] = int psi_m phi_i, M_psi = diag(int psi_m^2) (orthogonal modes): the lumping cancels
    and the result is I^T r, I the element-wise L2 projection the oracle uses.  G, M_psi and the
    lumped M~_Q are built here from a tensor Gauss rule of 2k+4 points, numpy's Legendre series
    and the Lagrange product formula on GLL nodes found as roots of (1 - x^2) P_k'."""
    from numpy.polynomial import legendre as L
    m = fem.Mesh(N, k)
    n, M, h = k + 1, m.M, 1.0 / N
    dk = L.legder(np.eye(k + 1)[k])
    gll = np.sort(np.concatenate([[-1.0, 1.0], L.legroots(dk)]))
    xq, wq = L.leggauss(2 * k + 4)

    def lag(i, x):
        v = np.ones_like(x)
        for j in range(n):
            if j != i:
                v = v * (x - gll[j]) / (gll[i] - gll[j])
        return v

    def leg(a, x):
        return L.legval(x, np.eye(a + 1)[a])

    B = np.array([lag(i, xq) for i in range(n)])            # [node, q]
    P = np.array([leg(a, xq) for a in range(k)])            # [mode, q]
    jac = (h / 2) ** 3
    G1 = (B[None, :, :] * P[:, None, :] * wq).sum(-1)       # 1D int P_a l_i
    Mp1 = (P * P * wq).sum(-1)                              # 1D int P_a^2
    int1 = (B * wq).sum(-1)                                 # 1D int l_i
    r = random_vector(77, m.p_dof)
    lumped = np.zeros(m.n_nodes)
    Gt_r = np.zeros(m.n_nodes)
    for e in range(m.E):
        ex, ey, ez = e % N, (e // N) % N, e // (N * N)
        for c in range(n):
            for b in range(n):
                for a in range(n):
                    g = (ex * k + a) + M * ((ey * k + b) + M * (ez * k + c))
                    lumped[g] += jac * int1[a] * int1[b] * int1[c]
                    for mi, (pa, pb, pc) in enumerate(m.modes):
                        Gmi = jac * G1[pa, a] * G1[pb, b] * G1[pc, c]
                        Mpsi = jac * Mp1[pa] * Mp1[pb] * Mp1[pc]
                        Gt_r[g] += Gmi * r[e * m.n_p + mi] / Mpsi
    projected = Gt_r / lumped                               # nodal function, lumped projection
    dual = lumped * projected
    want = fem.modal_projection(m).T @ r
    assert np.allclose(dual, want, rtol=0, atol=1e-13 * np.abs(want).max())
