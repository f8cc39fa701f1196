"""Assembled FP64 finite elements for the Q_k x P_{k-1}^disc Stokes discretization.

TEST INFRASTRUCTURE ONLY (see the package header).

Follows the paper's discretization (Sec. 1.2, eq. 2): continuous nodal Q_k
velocity on a uniform hexahedral mesh of the unit cube, discontinuous modal
P_{k-1} pressure, no-slip Dirichlet velocity.  Readings where the paper is
silent: velocity nodes at the Gauss-Lobatto-Legendre (GLL) points; Gauss-Legendre
quadrature with k+1 points per direction; pressure modes are tensor Legendre
polynomials L_a L_b L_c with a+b+c <= k-1 in the order listed by ``modes``.

Conventions
-----------
* reference element [-1,1]^3, affine map x = x_e + (h/2)(xi + 1), |J| = (h/2)^3;
* element e = ex + N (ey + N ez); local node i = a + n (b + n c), n = k+1;
* global node g = gi + M (gj + M gl), M = kN + 1, gi = ex k + a;
* velocity vector laid out [3][n_nodes]; pressure laid out [E][n_p];
* quadrature index q = qx + n (qy + n qz).

Parity status: every assembled operator here is pinned by closed-form or
brute-force checks in tests/test_oracle_*.py.
"""
from __future__ import annotations

import functools

import numpy as np
import scipy.sparse as sp
from numpy.polynomial import legendre as npleg


# ----------------------------------------------------------------------------
# 1D rules and bases
# ----------------------------------------------------------------------------

def gauss_rule(n: int):
    """Gauss-Legendre points and weights on [-1, 1] (exact to degree 2n-1)."""
    x, w = npleg.leggauss(n)
    return np.asarray(x, dtype=np.float64), np.asarray(w, dtype=np.float64)


def gll_points(n: int) -> np.ndarray:
    """Gauss-Lobatto-Legendre points: +-1 and the roots of P'_{n-1}."""
    if n == 2:
        return np.array([-1.0, 1.0])
    c = np.zeros(n)
    c[-1] = 1.0
    inner = np.sort(np.real(npleg.legroots(npleg.legder(c))))
    return np.concatenate(([-1.0], inner, [1.0]))


def gll_weights(n: int) -> np.ndarray:
    """GLL weights 2 / (n (n-1) P_{n-1}(x_i)^2)."""
    x = gll_points(n)
    c = np.zeros(n)
    c[-1] = 1.0
    return 2.0 / (n * (n - 1) * npleg.legval(x, c) ** 2)


def lagrange(nodes, x):
    """Lagrange basis through ``nodes``: values V[i, a] = l_a(x_i), derivatives D[i, a]."""
    nodes = np.asarray(nodes, dtype=np.float64)
    x = np.atleast_1d(np.asarray(x, dtype=np.float64))
    n = len(nodes)
    V = np.ones((len(x), n))
    D = np.zeros((len(x), n))
    for a in range(n):
        for m in range(n):
            if m != a:
                V[:, a] *= (x - nodes[m]) / (nodes[a] - nodes[m])
        for m in range(n):
            if m == a:
                continue
            t = np.full(len(x), 1.0 / (nodes[a] - nodes[m]))
            for j in range(n):
                if j != a and j != m:
                    t *= (x - nodes[j]) / (nodes[a] - nodes[j])
            D[:, a] += t
    return V, D


def legendre(a: int, x) -> np.ndarray:
    """Unnormalized Legendre polynomial P_a(x) (P_a(1) = 1)."""
    c = np.zeros(a + 1)
    c[a] = 1.0
    return npleg.legval(np.asarray(x, dtype=np.float64), c)


def modes(k: int):
    """Pressure modes (a, b, c), a+b+c <= k-1; c slowest, a fastest."""
    out = []
    for c in range(k):
        for b in range(k - c):
            for a in range(k - b - c):
                out.append((a, b, c))
    return out


def kron3(Z, Y, X):
    """Tensor product with the z factor slowest and the x factor fastest."""
    return np.kron(Z, np.kron(Y, X))


# ----------------------------------------------------------------------------
# Mesh
# ----------------------------------------------------------------------------

class Mesh:
    """Uniform N^3 hexahedral mesh of (0,1)^3 carrying Q_k nodes (GLL)."""

    def __init__(self, N: int, k: int):
        assert N >= 1 and k >= 1
        self.N, self.k, self.n = N, k, k + 1
        self.h = 1.0 / N
        self.M = k * N + 1
        self.n_nodes = self.M ** 3
        self.E = N ** 3
        self.modes = modes(k) if k >= 1 else []
        self.n_p = len(self.modes)
        n, M = self.n, self.M
        ex, ey, ez = np.meshgrid(np.arange(N), np.arange(N), np.arange(N), indexing="ij")
        ex, ey, ez = (v.transpose(2, 1, 0).ravel() for v in (ex, ey, ez))  # e = ex + N(ey + N ez)
        self.eidx = np.stack([ex, ey, ez], axis=1)
        a, b, c = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
        a, b, c = (v.transpose(2, 1, 0).ravel() for v in (a, b, c))          # i = a + n(b + n c)
        gi = ex[:, None] * k + a[None, :]
        gj = ey[:, None] * k + b[None, :]
        gl = ez[:, None] * k + c[None, :]
        self.elem_nodes = gi + M * (gj + M * gl)                              # [E, n^3]
        # 1D node coordinates
        xi = gll_points(n)
        x1 = np.zeros(M)
        for e1 in range(N):
            x1[e1 * k:e1 * k + n] = (e1 + 0.5 * (xi + 1.0)) * self.h
        self.x1 = x1
        g = np.arange(self.n_nodes)
        i1, j1, l1 = g % M, (g // M) % M, g // (M * M)
        self.node_xyz = np.stack([x1[i1], x1[j1], x1[l1]], axis=1)
        self.boundary = ((i1 == 0) | (i1 == M - 1) | (j1 == 0) | (j1 == M - 1)
                         | (l1 == 0) | (l1 == M - 1))
        # velocity DOF masks ([3][n_nodes] layout)
        self.vel_boundary = np.tile(self.boundary, 3)
        self.vel_interior = np.flatnonzero(~self.vel_boundary)
        # elements whose closure touches the boundary (the set Omega_D of Sec. 5)
        self.touches_boundary = np.any((self.eidx == 0) | (self.eidx == N - 1), axis=1)

    @property
    def u_dof(self):
        return 3 * self.n_nodes

    @property
    def p_dof(self):
        return self.E * self.n_p

    def quad_points(self, elements=None):
        """Physical Gauss points, [E, n^3, 3] (or of the given elements only)."""
        xg, _ = gauss_rule(self.n)
        n = self.n
        qa, qb, qc = np.meshgrid(np.arange(n), np.arange(n), np.arange(n), indexing="ij")
        qa, qb, qc = (v.transpose(2, 1, 0).ravel() for v in (qa, qb, qc))
        loc = np.stack([xg[qa], xg[qb], xg[qc]], axis=1)                     # [n^3, 3]
        eidx = self.eidx if elements is None else self.eidx[np.asarray(elements)]
        return (eidx[:, None, :] + 0.5 * (loc[None, :, :] + 1.0)) * self.h


# ----------------------------------------------------------------------------
# Reference element
# ----------------------------------------------------------------------------

@functools.lru_cache(maxsize=None)
def reference(k: int):
    """Tensors of the reference element for order k.

    Returns dict with Phi[q, i], G[d][q, i] (reference gradients), W[q],
    Psi[q, m] (pressure modes at the Gauss points) and the 1D tables."""
    n = k + 1
    xq, wq = gauss_rule(n)
    xn = gll_points(n)
    B1, D1 = lagrange(xn, xq)
    Phi = kron3(B1, B1, B1)
    G = [kron3(B1, B1, D1), kron3(B1, D1, B1), kron3(D1, B1, B1)]
    W = kron3(wq, wq, wq)
    ms = modes(k)
    Psi = np.zeros((n ** 3, len(ms)))
    for m, (a, b, c) in enumerate(ms):
        Psi[:, m] = kron3(legendre(c, xq), legendre(b, xq), legendre(a, xq))
    return dict(n=n, xq=xq, wq=wq, xn=xn, B1=B1, D1=D1, Phi=Phi, G=G, W=W, Psi=Psi)


@functools.lru_cache(maxsize=None)
def _visc_quad_kernel(k: int, h: float):
    """K[q, (c,i), (d,j)] = 2 W_q |J| eps(phi_i e_c) : eps(phi_j e_d) for unit viscosity."""
    R = reference(k)
    n3 = R["n"] ** 3
    detJ = (0.5 * h) ** 3
    g = np.stack([Gd * (2.0 / h) for Gd in R["G"]], axis=-1)                 # [q, i, 3]
    eps = np.zeros((3, n3, n3, 3, 3))                                          # [c, i, q, a, b]
    for c in range(3):
        eps[c, :, :, c, :] += 0.5 * g.transpose(1, 0, 2)
        eps[c, :, :, :, c] += 0.5 * g.transpose(1, 0, 2)
    K = 2.0 * np.einsum("q,ciqab,djqab->qcidj", R["W"] * detJ, eps, eps)
    return K.reshape(n3, 3 * n3, 3 * n3)


def element_viscous(k: int, h: float, mu_q: np.ndarray) -> np.ndarray:
    """A_e[(c,i),(d,j)] = sum_q 2 mu_q W_q |J| eps(phi_i e_c):eps(phi_j e_d); mu_q [E, n^3]."""
    return np.einsum("eq,qij->eij", mu_q, _visc_quad_kernel(k, h))


def element_div(k: int, h: float) -> np.ndarray:
    """B_e[m, (d,j)] = - sum_q W_q |J| psi_m(x_q) d_d phi_j(x_q)  (B = -div, Sec. 3.1)."""
    R = reference(k)
    detJ = (0.5 * h) ** 3
    n3 = R["n"] ** 3
    Be = np.zeros((len(modes(k)), 3 * n3))
    for d in range(3):
        Be[:, d * n3:(d + 1) * n3] = -np.einsum("q,qm,qj->mj", R["W"] * detJ, R["Psi"],
                                                R["G"][d] * (2.0 / h))
    return Be


def pressure_mass_diag(mesh: Mesh, mu_q: np.ndarray) -> np.ndarray:
    """Diagonal of the inverse viscosity-weighted pressure mass M_p(1/mu) (Sec. 3.1, eq. 4):
    [M_p(1/mu)]_{(e,m),(e,m)} = sum_q W_q |J| psi_m(x_q)^2 / mu_q, laid out [E][n_p].

    Reading: the paper diagonalizes M_p(1/mu) by lumping against the coefficient vector of the
    constant function.  In an L2-orthogonal (Legendre) modal basis that vector is the first
    mode alone, and its lumped entries int psi_m / mu vanish for m > 0 wherever mu is constant,
    so the diagonal of M_p(1/mu) is taken instead; for the constant mode the two coincide."""
    R = reference(mesh.k)
    detJ = (0.5 * mesh.h) ** 3
    return np.einsum("q,qm,eq->em", R["W"] * detJ, R["Psi"] ** 2, 1.0 / mu_q).reshape(-1)


def _vel_gdofs(mesh: Mesh) -> np.ndarray:
    return np.concatenate([c * mesh.n_nodes + mesh.elem_nodes for c in range(3)], axis=1)


def assemble_A(mesh: Mesh, mu_q: np.ndarray, chunk: int = 512) -> sp.csr_matrix:
    """Global viscous-stress matrix on the full [3][n_nodes] space (no Dirichlet)."""
    gd = _vel_gdofs(mesh)
    nl = gd.shape[1]
    rows, cols, vals = [], [], []
    for s in range(0, mesh.E, chunk):
        Ae = element_viscous(mesh.k, mesh.h, mu_q[s:s + chunk])
        g = gd[s:s + chunk]
        rows.append(np.repeat(g, nl, axis=1).ravel())
        cols.append(np.tile(g, (1, nl)).ravel())
        vals.append(Ae.ravel())
    A = sp.coo_matrix((np.concatenate(vals), (np.concatenate(rows), np.concatenate(cols))),
                      shape=(mesh.u_dof, mesh.u_dof))
    return A.tocsr()


def assemble_B(mesh: Mesh) -> sp.csr_matrix:
    """Global divergence matrix, [p_dof, u_dof] (no Dirichlet)."""
    Be = element_div(mesh.k, mesh.h)
    gd = _vel_gdofs(mesh)
    n_p = mesh.n_p
    rows = (np.arange(mesh.E)[:, None] * n_p + np.arange(n_p)[None, :])
    R = np.repeat(rows[:, :, None], gd.shape[1], axis=2)
    C = np.repeat(gd[:, None, :], n_p, axis=1)
    V = np.broadcast_to(Be, R.shape)
    return sp.coo_matrix((V.ravel(), (R.ravel(), C.ravel())),
                         shape=(mesh.p_dof, mesh.u_dof)).tocsr()


def assemble_load(mesh: Mesh, f_q: np.ndarray) -> np.ndarray:
    """F[(c, g)] = sum_e sum_q W_q |J| f_c(x_q) phi_i(x_q); f_q [E, n^3, 3]."""
    R = reference(mesh.k)
    detJ = mesh.h ** 3 / 8.0
    F = np.zeros(mesh.u_dof)
    for c in range(3):
        Fe = np.einsum("q,eq,qi->ei", R["W"] * detJ, f_q[:, :, c], R["Phi"])
        np.add.at(F, c * mesh.n_nodes + mesh.elem_nodes, Fe)
    return F


def element_amplification(mesh: Mesh, a: float) -> np.ndarray:
    """a_e = a on elements touching the Dirichlet boundary, 1 elsewhere (Sec. 5)."""
    return np.where(mesh.touches_boundary, a, 1.0)


def lumped_weighted_mass(mesh: Mesh, w_nodes: np.ndarray, a_e: np.ndarray) -> np.ndarray:
    """Row sums of the weighted velocity mass matrix built with GLL quadrature.

    M_e[i, j] = sum_{q in GLL} a_e w(x_q) phi_i(x_q) phi_j(x_q) omega_q |J|;
    the lumped diagonal is M 1 (eq. 4 applied to the velocity space, eq. 8).
    w_nodes: weight function at the global velocity nodes, [n_nodes].
    Returns the diagonal per node (identical for the 3 components)."""
    n = mesh.n
    xn = gll_points(n)
    wn = gll_weights(n)
    V1, _ = lagrange(xn, xn)                      # basis at GLL quadrature points
    Vq = kron3(V1, V1, V1)                        # [q, i]
    Wq = kron3(wn, wn, wn) * mesh.h ** 3 / 8.0
    wq = w_nodes[mesh.elem_nodes] * a_e[:, None]  # quadrature points coincide with nodes
    Me = np.einsum("eq,q,qi,qj->eij", wq, Wq, Vq, Vq)
    rowsum = Me.sum(axis=2)
    d = np.zeros(mesh.n_nodes)
    np.add.at(d, mesh.elem_nodes, rowsum)
    return d


def interpolant_gradient(mesh: Mesh, f_nodes: np.ndarray, at: str = "nodes") -> np.ndarray:
    """Gradient of the element-wise Q_k nodal interpolant of a nodal field, per element at its
    GLL nodes (at="nodes") or at its Gauss points (at="gauss"): [E, n^3, 3]."""
    n = mesh.n
    xn = gll_points(n)
    V, D = lagrange(xn, xn if at == "nodes" else gauss_rule(n)[0])
    Gs = (kron3(V, V, D), kron3(V, D, V), kron3(D, V, V))      # d/dx, d/dy, d/dz
    fe = f_nodes[mesh.elem_nodes]                               # [E, n^3]
    return np.stack([fe @ G.T for G in Gs], axis=-1) * (2.0 / mesh.h)


def gradient_weights(mesh: Mesh, mu_nodes: np.ndarray, mu_q: np.ndarray):
    """Viscosity-gradient w-BFBT weights w = (mu^2 + |grad mu|^2)^(1/4) (remark in Sec. 4), with
    grad mu the gradient of the element-wise Q_k interpolant of mu: per element at its nodes
    [E, n^3] (for the lumped masses) and at the Gauss points [E, n^3] (for the Poisson
    coefficient 1/w)."""
    gn = interpolant_gradient(mesh, mu_nodes, "nodes")
    gq = interpolant_gradient(mesh, mu_nodes, "gauss")
    w_en = (mu_nodes[mesh.elem_nodes] ** 2 + (gn ** 2).sum(axis=-1)) ** 0.25
    w_q = (mu_q ** 2 + (gq ** 2).sum(axis=-1)) ** 0.25
    return w_en, w_q


def lumped_weighted_mass_elem(mesh: Mesh, w_en: np.ndarray, a_e: np.ndarray) -> np.ndarray:
    """lumped_weighted_mass with the weight given per element at its nodes [E, n^3] (a weight
    that differs between the elements sharing a node)."""
    wn = gll_weights(mesh.n)
    Wq = kron3(wn, wn, wn) * mesh.h ** 3 / 8.0
    d = np.zeros(mesh.n_nodes)
    np.add.at(d, mesh.elem_nodes, a_e[:, None] * w_en * Wq[None, :])
    return d


def lumped_weighted_mass_gauss(mesh: Mesh, w_q: np.ndarray) -> np.ndarray:
    """Row sums of the weighted mass matrix with Gauss quadrature (comparison reading)."""
    R = reference(mesh.k)
    Me_rows = np.einsum("eq,q,qi->ei", w_q, R["W"] * mesh.h ** 3 / 8.0, R["Phi"])
    d = np.zeros(mesh.n_nodes)
    np.add.at(d, mesh.elem_nodes, Me_rows)
    return d


def assemble_poisson(mesh: Mesh, c_q: np.ndarray) -> sp.csr_matrix:
    """Scalar stiffness L[g, g'] = sum_e sum_q c_q W_q |J| grad phi_i . grad phi_j (Neumann)."""
    R = reference(mesh.k)
    detJ = mesh.h ** 3 / 8.0
    s = (2.0 / mesh.h) ** 2
    Kq = sum(np.einsum("qi,qj->qij", Gd, Gd) for Gd in R["G"]) * (R["W"] * detJ * s)[:, None, None]
    Le = np.einsum("eq,qij->eij", c_q, Kq)
    g = mesh.elem_nodes
    nl = g.shape[1]
    rows = np.repeat(g, nl, axis=1).ravel()
    cols = np.tile(g, (1, nl)).ravel()
    return sp.coo_matrix((Le.ravel(), (rows, cols)), shape=(mesh.n_nodes, mesh.n_nodes)).tocsr()


# ----------------------------------------------------------------------------
# Transfers
# ----------------------------------------------------------------------------

def global_basis_1d(Nc: int, kc: int, x: np.ndarray) -> np.ndarray:
    """Values of the continuous 1D Q_kc basis on Nc elements at points x: [len(x), kc Nc + 1]."""
    hc = 1.0 / Nc
    xn = gll_points(kc + 1)
    out = np.zeros((len(x), kc * Nc + 1))
    for r, xv in enumerate(x):
        e = min(int(np.floor(xv / hc + 1e-12)), Nc - 1)
        xi = 2.0 * (xv / hc - e) - 1.0
        V, _ = lagrange(xn, [xi])
        out[r, e * kc:e * kc + kc + 1] = V[0]
    return out


def prolongation_1d(Nc: int, kc: int, Nf: int, kf: int) -> np.ndarray:
    """P1[i_f, I_c] = coarse global basis function I_c evaluated at fine node i_f."""
    P = global_basis_1d(Nc, kc, _x1(Nf, kf))
    P[np.abs(P) < 1e-14] = 0.0
    return P


def _x1(N, k):
    xi = gll_points(k + 1)
    x1 = np.zeros(k * N + 1)
    for e1 in range(N):
        x1[e1 * k:e1 * k + k + 1] = (e1 + 0.5 * (xi + 1.0)) / N
    return x1


def prolongation(Nc: int, kc: int, Nf: int, kf: int) -> sp.csr_matrix:
    """Scalar 3D prolongation, the tensor product of the 1D one (z slowest)."""
    P1 = sp.csr_matrix(prolongation_1d(Nc, kc, Nf, kf))
    return sp.kron(P1, sp.kron(P1, P1)).tocsr()


def modal_projection(mesh: Mesh) -> sp.csr_matrix:
    """I: Q_k nodal -> P_{k-1} modal, the element-wise L2 projection.

    I_e[m, i] = (int_e psi_m phi_i) / (int_e psi_m^2), Gauss quadrature (exact)."""
    R = reference(mesh.k)
    num = np.einsum("q,qm,qi->mi", R["W"], R["Psi"], R["Phi"])
    den = np.einsum("q,qm->m", R["W"], R["Psi"] ** 2)
    Ie = num / den[:, None]
    n_p = mesh.n_p
    rows = np.repeat((np.arange(mesh.E)[:, None] * n_p + np.arange(n_p)[None, :])[:, :, None],
                     mesh.elem_nodes.shape[1], axis=2)
    cols = np.repeat(mesh.elem_nodes[:, None, :], n_p, axis=1)
    vals = np.broadcast_to(Ie, rows.shape)
    return sp.coo_matrix((vals.ravel(), (rows.ravel(), cols.ravel())),
                         shape=(mesh.p_dof, mesh.n_nodes)).tocsr()


# ----------------------------------------------------------------------------
# Coefficient coarsening: the L2 adjoint of element-wise interpolation
# ----------------------------------------------------------------------------

def _coarsen_matrix(nf: int, nc: int, children: int) -> np.ndarray:
    """Q[qc, (s, qf)] with mu_c = W_c^-1 P^T W_f mu_f in 1D (weights include Jacobians).

    children = 1: same element (p-coarsening); children = 2: two halves (h-coarsening)."""
    xf, wf = gauss_rule(nf)
    xc, wc = gauss_rule(nc)
    cols = []
    for s in range(children):
        xi = xf if children == 1 else 0.5 * (xf + 2 * s - 1)   # fine point in coarse coords
        P, _ = lagrange(xc, xi)                                   # [qf, qc]
        wfs = wf / children
        cols.append((P * wfs[:, None]).T / wc[:, None])          # [qc, qf]
    return np.concatenate(cols, axis=1)


def coarsen_coefficient_p(coef_q: np.ndarray, nf: int, nc: int) -> np.ndarray:
    """Same mesh, n_f^3 -> n_c^3 Gauss points per element; clamped below by the element minimum."""
    Q = _coarsen_matrix(nf, nc, 1)
    Q3 = kron3(Q, Q, Q)
    out = coef_q @ Q3.T
    return np.maximum(out, coef_q.min(axis=1, keepdims=True))


def coarsen_coefficient_h(coef_q: np.ndarray, Nf: int, n: int) -> np.ndarray:
    """Nf^3 -> (Nf/2)^3 elements, n^3 Gauss points each; clamped below by the children minimum."""
    Nc = Nf // 2
    Q = _coarsen_matrix(n, n, 2)                                # [qc, (s, qf)]
    # gather the children of each coarse element into a [Ec, (2n)^3] array ordered (s,qf) per dim
    f = coef_q.reshape(Nf, Nf, Nf, n, n, n)                     # [ez, ey, ex, qz, qy, qx]
    f = f.reshape(Nc, 2, Nc, 2, Nc, 2, n, n, n)                 # [cz, sz, cy, sy, cx, sx, qz, qy, qx]
    f = f.transpose(0, 2, 4, 1, 6, 3, 7, 5, 8)                  # [cz, cy, cx, sz, qz, sy, qy, sx, qx]
    f = f.reshape(Nc ** 3, (2 * n) ** 3)
    out = f @ kron3(Q, Q, Q).T
    return np.maximum(out, f.min(axis=1, keepdims=True))


# ----------------------------------------------------------------------------
# Row-wise evaluation for large meshes (sampled parity checks)
# ----------------------------------------------------------------------------

def elements_of_node(mesh: Mesh, g: int):
    """Elements whose closure contains global node g."""
    M, k, N = mesh.M, mesh.k, mesh.N
    idx = (g % M, (g // M) % M, g // (M * M))
    cand = []
    for gi in idx:
        c = {gi // k} if gi % k else {gi // k - 1, gi // k}
        cand.append(sorted(e for e in c if 0 <= e < N))
    return [ex + N * (ey + N * ez) for ez in cand[2] for ey in cand[1] for ex in cand[0]]


def apply_A_rows(mesh: Mesh, mu_q_of, u: np.ndarray, dofs) -> np.ndarray:
    """(A u)_i for the velocity DOFs i = c * n_nodes + g, by element sums (no assembly).

    mu_q_of(elements) -> [len(elements), n^3] viscosity at those elements' Gauss points."""
    out = np.zeros(len(dofs))
    nn = mesh.n_nodes
    for r, dof in enumerate(dofs):
        c, g = divmod(int(dof), nn)
        els = elements_of_node(mesh, g)
        Ae = element_viscous(mesh.k, mesh.h, mu_q_of(np.array(els)))
        for t, e in enumerate(els):
            loc = int(np.flatnonzero(mesh.elem_nodes[e] == g)[0])
            gd = np.concatenate([cc * nn + mesh.elem_nodes[e] for cc in range(3)])
            out[r] += Ae[t, c * mesh.n ** 3 + loc] @ u[gd]
    return out
