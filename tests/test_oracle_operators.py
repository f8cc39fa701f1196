"""Pins of the assembled operators against closed forms, invariants and exact solutions."""
import numpy as np
import pytest
import scipy.sparse as sp
import scipy.sparse.linalg as spla
import sympy as sy

from oracle import fem, solver

X, Y, Z = sy.symbols("x y z")


def _rigid_modes(m):
    nn = m.n_nodes
    P = m.node_xyz
    out = []
    for c in range(3):
        v = np.zeros(3 * nn)
        v[c * nn:(c + 1) * nn] = 1.0
        out.append(v)
    for a, b in ((0, 1), (1, 2), (0, 2)):
        v = np.zeros(3 * nn)
        v[a * nn:(a + 1) * nn] = P[:, b]
        v[b * nn:(b + 1) * nn] = -P[:, a]
        out.append(v)
    return out


@pytest.mark.parametrize("N,k", [(2, 2), (2, 3), (1, 4), (3, 1), (1, 5)])
def test_A_rigid_body_kernel_and_symmetry(N, k):
    m = fem.Mesh(N, k)
    mu = np.random.default_rng(N + k).uniform(1e-2, 1e2, (m.E, m.n ** 3))
    A = fem.assemble_A(m, mu)
    assert abs(A - A.T).max() <= 1e-12 * abs(A).max()
    for v in _rigid_modes(m):
        assert np.abs(A @ v).max() <= 1e-12 * abs(A).max()
    # a non-rigid field is not in the kernel
    v = np.tile(m.node_xyz[:, 0] ** 2, 3)
    assert np.abs(A @ v).max() > 1e-6 * abs(A).max()


@pytest.mark.parametrize("N,k", [(2, 2), (3, 2), (2, 3)])
def test_A_spd_under_dirichlet(N, k):
    m = fem.Mesh(N, k)
    mu = np.random.default_rng(1).uniform(1e-3, 1e3, (m.E, m.n ** 3))
    A = fem.assemble_A(m, mu)[m.vel_interior][:, m.vel_interior].toarray()
    np.linalg.cholesky(A)     # raises if not SPD


def _laplace_plus_graddiv(m):
    """Vector-Laplacian stiffness plus the div-div matrix, assembled from their own integrands."""
    R = fem.reference(m.k)
    s = 2.0 / m.h
    detJ = m.h ** 3 / 8.0
    G = [g * s for g in R["G"]]
    n3 = m.n ** 3
    Ke = np.zeros((3 * n3, 3 * n3))
    lap = sum(np.einsum("q,qi,qj->ij", R["W"] * detJ, g, g) for g in G)
    for c in range(3):
        Ke[c * n3:(c + 1) * n3, c * n3:(c + 1) * n3] += lap
        for d in range(3):
            Ke[c * n3:(c + 1) * n3, d * n3:(d + 1) * n3] += np.einsum(
                "q,qi,qj->ij", R["W"] * detJ, G[c], G[d])
    gd = np.concatenate([c * m.n_nodes + m.elem_nodes for c in range(3)], axis=1)
    rows = np.repeat(gd, 3 * n3, axis=1).ravel()
    cols = np.tile(gd, (1, 3 * n3)).ravel()
    vals = np.broadcast_to(Ke, (m.E, 3 * n3, 3 * n3)).ravel()
    return sp.coo_matrix((vals, (rows, cols)), shape=(m.u_dof, m.u_dof)).tocsr()


@pytest.mark.parametrize("N,k", [(2, 2), (2, 3)])
def test_A_constant_viscosity_is_laplace_plus_graddiv(N, k):
    # 2||eps(v)||^2 = ||grad v||^2 + ||div v||^2 for v in H^1_0 (integration by parts)
    m = fem.Mesh(N, k)
    A = fem.assemble_A(m, np.ones((m.E, m.n ** 3)))
    L = _laplace_plus_graddiv(m)
    I = m.vel_interior
    diff = (A[I][:, I] - L[I][:, I])
    assert abs(diff).max() <= 1e-12 * abs(A).max()
    # on the full space (boundary DOFs kept) they must differ
    assert abs(A - L).max() > 1e-3 * abs(A).max()


def _poly_fn(expr):
    f = sy.lambdify((X, Y, Z), expr, "numpy")
    return lambda p: np.broadcast_to(f(p[..., 0], p[..., 1], p[..., 2]), p.shape[:-1]).astype(float)


@pytest.mark.parametrize("N,k,c", [(2, 2, 0), (3, 2, 2), (2, 3, 1)])
def test_A_manufactured_solution_exact(N, k, c):
    # u* = x(1-x) y(1-y) z(1-z) e_c is in Q_k cap H^1_0; with mu = 1 the Galerkin solution is u*.
    g = X * (1 - X) * Y * (1 - Y) * Z * (1 - Z)
    u = [0, 0, 0]
    u[c] = g
    grad = [[sy.diff(u[i], v) for v in (X, Y, Z)] for i in range(3)]
    sig = [[grad[i][j] + grad[j][i] for j in range(3)] for i in range(3)]      # 2 eps(u)
    f = [-sum(sy.diff(sig[i][j], v) for j, v in enumerate((X, Y, Z))) for i in range(3)]
    m = fem.Mesh(N, k)
    xq = m.quad_points()
    fq = np.stack([_poly_fn(fi)(xq) for fi in f], axis=-1)
    F = fem.assemble_load(m, fq)
    A = fem.assemble_A(m, np.ones((m.E, m.n ** 3)))
    I = m.vel_interior
    sol = spla.spsolve(A[I][:, I].tocsc(), F[I])
    exact = np.concatenate([_poly_fn(ui if ui != 0 else sy.Integer(0))(m.node_xyz) for ui in u])
    assert np.abs(sol - exact[I]).max() <= 1e-10 * np.abs(exact).max()


@pytest.mark.parametrize("N,k", [(2, 2), (2, 3), (1, 4), (1, 5)])
def test_B_annihilates_constants_and_BT_kills_constant_pressure(N, k):
    m = fem.Mesh(N, k)
    B = fem.assemble_B(m)
    nn = m.n_nodes
    for c in range(3):
        v = np.zeros(3 * nn)
        v[c * nn:(c + 1) * nn] = 1.0
        assert np.abs(B @ v).max() < 1e-14
    ones = np.zeros(m.p_dof)
    ones[::m.n_p] = 1.0
    bt = (B.T @ ones)[m.vel_interior]
    assert np.abs(bt).max() < 1e-14
    # but not on the boundary DOFs: no-slip is what makes constants a null space
    assert np.abs((B.T @ ones)[m.vel_boundary]).max() > 1e-3 * m.h ** 2


@pytest.mark.parametrize("k", [2, 3, 4, 5])
def test_B_is_minus_divergence_integral(k):
    # (B u)_{e,m} = -int_e psi_m div u; independent 8-point Gauss integration of a polynomial field
    m = fem.Mesh(2, k)
    u_expr = [X ** 2 * Y + Z, Y * Z ** 2 - X, X * Y * Z]
    if k >= 3:
        u_expr[0] += X ** 3
    fns = [_poly_fn(e) for e in u_expr]
    u = np.concatenate([fn(m.node_xyz) for fn in fns])
    Bu = fem.assemble_B(m) @ u
    div = sy.lambdify((X, Y, Z), sum(sy.diff(e, v) for e, v in zip(u_expr, (X, Y, Z))), "numpy")
    xg, wg = np.polynomial.legendre.leggauss(8)
    h = m.h
    for e in [0, 3, 7]:
        ex, ey, ez = m.eidx[e]
        for mi, (a, b, c) in enumerate(m.modes):
            tot = 0.0
            for i, xi in enumerate(xg):
                for j, eta in enumerate(xg):
                    for l, zeta in enumerate(xg):
                        x = (ex + 0.5 * (xi + 1)) * h
                        y = (ey + 0.5 * (eta + 1)) * h
                        z = (ez + 0.5 * (zeta + 1)) * h
                        psi = (np.polynomial.legendre.Legendre.basis(a)(xi)
                               * np.polynomial.legendre.Legendre.basis(b)(eta)
                               * np.polynomial.legendre.Legendre.basis(c)(zeta))
                        tot += wg[i] * wg[j] * wg[l] * psi * div(x, y, z)
            assert abs(Bu[e * m.n_p + mi] - (-tot * h ** 3 / 8)) < 1e-13


def test_load_vector_exact_for_polynomial_force():
    # F_i = int f . phi_i; summing F over all nodes of component c gives int f_c (partition of unity)
    m = fem.Mesh(3, 2)
    fz = X * Y ** 2 + Z
    fq = np.zeros(m.quad_points().shape)
    fq[..., 2] = _poly_fn(fz)(m.quad_points())
    F = fem.assemble_load(m, fq)
    exact = float(sy.integrate(fz, (X, 0, 1), (Y, 0, 1), (Z, 0, 1)))
    nn = m.n_nodes
    assert abs(F[2 * nn:].sum() - exact) < 1e-14
    assert np.abs(F[:2 * nn]).max() == 0.0
    # and F . u_h = int f . u for u in Q_k
    uz = _poly_fn(X ** 2 * Z)(m.node_xyz)
    exact2 = float(sy.integrate(fz * X ** 2 * Z, (X, 0, 1), (Y, 0, 1), (Z, 0, 1)))
    assert abs(F[2 * nn:] @ uz - exact2) < 1e-14


@pytest.mark.parametrize("k", [2, 3])
def test_lumped_weighted_mass(k):
    m = fem.Mesh(3, k)
    # unit weight: the lumped mass sums to the volume and is positive
    d = fem.lumped_weighted_mass(m, np.ones(m.n_nodes), np.ones(m.E))
    assert np.all(d > 0) and abs(d.sum() - 1.0) < 1e-13
    # weight w(x) = 1 + x y: GLL quadrature of a degree-(1,1,0) field is exact
    w = 1.0 + m.node_xyz[:, 0] * m.node_xyz[:, 1]
    d = fem.lumped_weighted_mass(m, w, np.ones(m.E))
    assert abs(d.sum() - 1.25) < 1e-13
    # amplification a on boundary elements scales only their contributions
    d1 = fem.lumped_weighted_mass(m, np.ones(m.n_nodes), np.ones(m.E))
    d2 = fem.lumped_weighted_mass(m, np.ones(m.n_nodes), fem.element_amplification(m, 4.0))
    assert abs(d2.sum() - (26 * 4.0 + 1.0) / 27) < 1e-13          # 26 of 27 elements touch the boundary
    assert np.all(d2 >= d1 - 1e-15)
    interior_elem = set(m.elem_nodes[13])
    only_boundary_elems = [g for g in range(m.n_nodes)
                           if g not in interior_elem and g in set(m.elem_nodes[0])]
    assert np.allclose(d2[only_boundary_elems], 4.0 * d1[only_boundary_elems], rtol=1e-14)
    # the interior element's own interior nodes are untouched by the amplification
    c = m.elem_nodes[13].reshape(m.n, m.n, m.n)[1:-1, 1:-1, 1:-1].ravel()
    assert np.allclose(d2[c], d1[c], rtol=1e-14)


@pytest.mark.parametrize("Nc,kc,Nf,kf", [(2, 1, 2, 2), (2, 2, 2, 4), (2, 1, 2, 3), (2, 1, 4, 1), (3, 1, 6, 1)])
def test_prolongation_reproduces_coarse_space(Nc, kc, Nf, kf):
    P = fem.prolongation(Nc, kc, Nf, kf)
    mc, mf = fem.Mesh(Nc, kc), fem.Mesh(Nf, kf)
    # a global polynomial of degree kc per direction lies in both spaces
    fn = lambda p: (p[:, 0] ** kc) * (1 + p[:, 1]) * (2 - p[:, 2] ** kc)
    assert np.allclose(P @ fn(mc.node_xyz), fn(mf.node_xyz), atol=1e-13)
    # piecewise coarse functions: a coarse hat function restricted to the fine nodes
    e = np.zeros(mc.n_nodes)
    e[mc.n_nodes // 2] = 1.0
    v = P @ e
    assert abs(v.max() - 1.0) < 1e-14 and v.min() > -0.2


@pytest.mark.parametrize("k", [2, 3, 4, 5])
def test_modal_projection_reproduces_pressure_polynomials(k):
    m = fem.Mesh(2, k)
    I = fem.modal_projection(m)
    q = m.node_xyz[:, 0] + 2 * m.node_xyz[:, 1] - m.node_xyz[:, 2]
    p = I @ q
    h = m.h
    for e in range(m.E):
        xc = (m.eidx[e] + 0.5) * h
        want = {(0, 0, 0): xc[0] + 2 * xc[1] - xc[2], (1, 0, 0): h / 2, (0, 1, 0): h, (0, 0, 1): -h / 2}
        for mi, md in enumerate(m.modes):
            assert abs(p[e * m.n_p + mi] - want.get(md, 0.0)) < 1e-13


@pytest.mark.parametrize("nf,nc", [(3, 2), (5, 3), (4, 2)])
def test_coefficient_p_coarsening_is_l2_adjoint(nf, nc):
    rng = np.random.default_rng(nf)
    E = 3
    fine = rng.uniform(1, 2, (E, nf ** 3))
    coarse = fem.coarsen_coefficient_p(fine, nf, nc)
    # independent check: <P c, f>_fine = <c, P* f>_coarse with P = interpolation of the
    # coarse Gauss-Lagrange polynomial at the fine Gauss points
    xf, wf = fem.gauss_rule(nf)
    xc, wc = fem.gauss_rule(nc)
    P1, _ = fem.lagrange(xc, xf)
    P3 = fem.kron3(P1, P1, P1)
    Wf, Wc = fem.kron3(wf, wf, wf), fem.kron3(wc, wc, wc)
    cvec = rng.uniform(-1, 1, (E, nc ** 3))
    lhs = np.einsum("ef,f,ef->e", cvec @ P3.T, Wf, fine)
    # clamping only acts where the projection undershoots; these smooth-ish fields do not
    assert np.all(coarse > fine.min(axis=1, keepdims=True) - 1e-15)
    rhs = np.einsum("ec,c,ec->e", cvec, Wc, coarse)
    assert np.allclose(lhs, rhs, rtol=1e-12)
    # constants are reproduced
    assert np.allclose(fem.coarsen_coefficient_p(np.full((E, nf ** 3), 3.0), nf, nc), 3.0)


def test_coefficient_h_coarsening_reproduces_linear_fields():
    # a globally linear field sampled at the fine Gauss points is reproduced at the coarse ones
    Nf, n = 4, 2
    mf, mc = fem.Mesh(Nf, n - 1), fem.Mesh(Nf // 2, n - 1)
    fn = lambda p: 2.0 + p[..., 0] + 0.5 * p[..., 1] - 0.25 * p[..., 2]
    out = fem.coarsen_coefficient_h(fn(mf.quad_points()), Nf, n)
    assert np.allclose(out, fn(mc.quad_points()), atol=1e-13)
    # the total integral is preserved for arbitrary positive data (adjoint of interpolation of 1)
    rng = np.random.default_rng(0)
    fine = rng.uniform(1, 2, (Nf ** 3, n ** 3))
    wf = fem.kron3(*[fem.gauss_rule(n)[1]] * 3)
    coarse = fem.coarsen_coefficient_h(fine, Nf, n)
    assert abs((fine @ wf).sum() / 8 - (coarse @ wf).sum()) < 1e-12


def test_interpolant_gradient_and_gradient_weights():
    """The gradient of the element-wise Q_k interpolant is exact for polynomials of degree k
    (at the nodes and at the Gauss points); for a constant viscosity the gradient weights are
    sqrt(mu), so the lumped masses and the Poisson coefficient equal the sqrt(mu) ones."""
    for N, k in ((3, 2), (2, 3)):
        m = fem.Mesh(N, k)
        x = m.node_xyz
        f = lambda X: 1.0 + 2 * X[..., 0] ** k - 3 * X[..., 1] * X[..., 2] ** (k - 1) + X[..., 2]
        df = lambda X: np.stack([2 * k * X[..., 0] ** (k - 1), -3 * X[..., 2] ** (k - 1),
                                 -3 * (k - 1) * X[..., 1] * X[..., 2] ** (k - 2) + 1.0], axis=-1)
        gn = fem.interpolant_gradient(m, f(x), "nodes")
        assert np.allclose(gn, df(x[m.elem_nodes]), rtol=0, atol=1e-11)
        xq = m.quad_points()
        gq = fem.interpolant_gradient(m, f(x), "gauss")
        assert np.allclose(gq, df(xq), rtol=0, atol=1e-11)
        mu = 7.0
        w_en, w_q = fem.gradient_weights(m, np.full(m.n_nodes, mu), np.full((m.E, m.n ** 3), mu))
        assert np.allclose(w_q, np.sqrt(mu), rtol=1e-15)
        a_e = fem.element_amplification(m, 3.0)
        assert np.allclose(fem.lumped_weighted_mass_elem(m, w_en, a_e),
                           fem.lumped_weighted_mass(m, np.full(m.n_nodes, np.sqrt(mu)), a_e), rtol=1e-13)
