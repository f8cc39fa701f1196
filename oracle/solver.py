"""Solver-side oracle: w-BFBT, multigrid, block preconditioner, flexible GMRES.

TEST INFRASTRUCTURE ONLY (see the package header).

Written from the paper's definitions:

* upper block-triangular right preconditioner and GMRES (eq. 3);
* the inverse viscosity-weighted pressure mass Schur approximation, diagonalized (Sec. 3.1,
  eq. 4; the comparison baseline of Sec. 8);
* BFBT / w-BFBT inverse Schur approximation (eq. 7, 8) with lumped
  sqrt(mu)-weighted velocity masses and Dirichlet amplification (Sec. 5);
* pressure Poisson K_w = B D_w^-1 B^T and its V-cycle through a continuous Q_k
  Poisson re-discretization with coefficient 1/w (eq. 11, 12, Sec. 6);
* p- then h-multigrid V-cycles with Chebyshev-accelerated point-Jacobi
  smoothing, 3 pre and 3 post, re-discretized coarse operators with the
  viscosity coarsened by the L2 adjoint of element-wise interpolation (Sec. 6).

Readings where the paper is silent (also listed in the design notes):
Chebyshev interval [0.1, 1.1] * lambda_max(D^-1 A) from 10 Jacobi-CG (Lanczos)
steps started from a counter-based splitmix64 vector; p-coarsening halves the
order (4->2->1, 3->1, 2->1); h-coarsening halves N while N/2 >= 4; the
coarsest level is solved directly (pseudo-inverse for the Neumann Poisson).

Parity status:
* exact w-BFBT, Schur complement, saddle direct solve, FGMRES: pinned
  (spectral lower bound, scaling invariances, two-iteration property,
  brute-force least-squares GMRES history, manufactured exact solutions);
* Chebyshev smoother, Lanczos estimate: pinned (closed-form polynomial on
  diagonal matrices, exact eigenvalue on small spectra);
* V-cycles (A and K_w) and the approximate w-BFBT: parity unpinned beyond
  their building blocks -- they are iterations; only convergence ranges are
  checked against the paper's Table 3.
"""
from __future__ import annotations

import numpy as np
import scipy.linalg as sla
import scipy.sparse as sp
import scipy.sparse.linalg as spla

from . import fem, sinker

MASK64 = (1 << 64) - 1


# ----------------------------------------------------------------------------
# counter-based generator (splitmix64, Steele/Lea/Flood 2014)
# ----------------------------------------------------------------------------

def splitmix64_uniform(seed: int, count: int) -> np.ndarray:
    """u_i = 2 * U(splitmix64(seed * 2^32 + i)) - 1, U = top 53 bits / 2^53."""
    with np.errstate(over="ignore"):
        x = np.uint64((seed << 32) & MASK64) + np.arange(count, dtype=np.uint64)
        z = x + np.uint64(0x9E3779B97F4A7C15)
        z = (z ^ (z >> np.uint64(30))) * np.uint64(0xBF58476D1CE4E5B9)
        z = (z ^ (z >> np.uint64(27))) * np.uint64(0x94D049BB133111EB)
        z = z ^ (z >> np.uint64(31))
    u = (z >> np.uint64(11)).astype(np.float64) * (1.0 / 9007199254740992.0)
    return 2.0 * u - 1.0


# ----------------------------------------------------------------------------
# Chebyshev-Jacobi smoothing and the Lanczos (CG) eigenvalue estimate
# ----------------------------------------------------------------------------

def chebyshev(A, dinv, b, x, lmin, lmax, degree=3, x_zero=False):
    """Chebyshev acceleration of point Jacobi for A x = b on [lmin, lmax] (degree steps)."""
    theta = 0.5 * (lmax + lmin)
    delta = 0.5 * (lmax - lmin)
    sigma = theta / delta
    rho = 1.0 / sigma
    x = np.zeros_like(b) if x_zero else x.copy()
    r = b.copy() if x_zero else b - A @ x
    d = dinv * r / theta
    x = x + d
    for _ in range(degree - 1):
        r = r - A @ d
        rho_new = 1.0 / (2.0 * sigma - rho)
        d = rho_new * rho * d + (2.0 * rho_new / delta) * (dinv * r)
        x = x + d
        rho = rho_new
    return x


def lanczos_max(A, dinv, b0, steps=10):
    """Largest eigenvalue of D^-1 A from `steps` Jacobi-preconditioned CG iterations.

    The CG coefficients give the Lanczos tridiagonal T; returns max eig(T)."""
    r = b0.copy()
    z = dinv * r
    p = z.copy()
    rz = float(r @ z)
    alphas, betas = [], []
    for _ in range(steps):
        q = A @ p
        pq = float(p @ q)
        if rz <= 0.0 or pq <= 0.0:
            break
        alpha = rz / pq
        r = r - alpha * q
        z = dinv * r
        rz_new = float(r @ z)
        beta = rz_new / rz
        alphas.append(alpha)
        betas.append(beta)
        rz = rz_new
        p = z + beta * p
        if rz <= 0.0:
            break
    m = len(alphas)
    T = np.zeros((m, m))
    for j in range(m):
        T[j, j] = 1.0 / alphas[j] + (betas[j - 1] / alphas[j - 1] if j > 0 else 0.0)
        if j + 1 < m:
            T[j, j + 1] = T[j + 1, j] = np.sqrt(betas[j]) / alphas[j]
    return float(np.linalg.eigvalsh(T)[-1])


# ----------------------------------------------------------------------------
# Multigrid hierarchy description (shared reading of the paper's HMG, Sec. 6)
# ----------------------------------------------------------------------------

def level_schedule(N: int, k: int):
    """[(N, k), ...] from fine to coarsest: halve k to 1, then halve N while N/2 >= 4."""
    levels = [(N, k)]
    while k > 1:
        k = max(1, k // 2)
        levels.append((N, k))
    while N % 2 == 0 and N // 2 >= 4:
        N //= 2
        levels.append((N, k))
    return levels


def coarsen_schedule(coef_q, levels):
    """Coefficient at each level's Gauss points by the L2 adjoint of interpolation."""
    out = [coef_q]
    for (Nf, kf), (Nc, kc) in zip(levels[:-1], levels[1:]):
        c = out[-1]
        if Nc == Nf:
            out.append(fem.coarsen_coefficient_p(c, kf + 1, kc + 1))
        else:
            out.append(fem.coarsen_coefficient_h(c, Nf, kf + 1))
    return out


class _Level:
    pass


class Hierarchy:
    """V-cycle over re-discretized levels; `kind` is 'velocity' (Dirichlet) or 'poisson' (Neumann)."""

    def __init__(self, N, k, coef_q, kind, seed_base, degree=3, lanczos_steps=10):
        self.kind = kind
        self.degree = degree
        sched = level_schedule(N, k)
        coefs = coarsen_schedule(coef_q, sched)
        self.levels = []
        for li, ((Nl, kl), cl) in enumerate(zip(sched, coefs)):
            L = _Level()
            L.N, L.k, L.coef = Nl, kl, cl
            L.mesh = fem.Mesh(Nl, kl)
            if kind == "velocity":
                Afull = fem.assemble_A(L.mesh, cl)
                L.idx = L.mesh.vel_interior
                L.full = L.mesh.u_dof
            else:
                Afull = fem.assemble_poisson(L.mesh, cl)
                L.idx = np.arange(L.mesh.n_nodes)
                L.full = L.mesh.n_nodes
            L.A = Afull[L.idx][:, L.idx].tocsr()
            L.dinv = 1.0 / L.A.diagonal()
            if li < len(sched) - 1:
                start = splitmix64_uniform(seed_base + li, L.full)[L.idx]
                if kind == "poisson":
                    start = start - start.mean()
                lam = lanczos_max(L.A, L.dinv, start, lanczos_steps)
                L.lmin, L.lmax = 0.1 * lam, 1.1 * lam
            self.levels.append(L)
        # transfers: P_l maps level l+1 (coarse) to level l (fine), reduced spaces
        for li in range(len(self.levels) - 1):
            F, C = self.levels[li], self.levels[li + 1]
            P = fem.prolongation(C.N, C.k, F.N, F.k)
            if kind == "velocity":
                P = sp.block_diag([P, P, P]).tocsr()
            F.P = P[F.idx][:, C.idx].tocsr()
        last = self.levels[-1]
        Ad = last.A.toarray()
        if kind == "velocity":
            self.coarse = lambda b: sla.cho_solve(sla.cho_factor(Ad), b)
        else:
            pinv = np.linalg.pinv(Ad)
            self.coarse = lambda b: pinv @ b

    def vcycle(self, b, li=0, learned=None):
        """One V-cycle from level li.  learned = (lc, step): at level lc the coarse-grid
        correction (restriction, the cycle below, prolongation) is replaced by x += step(r), r the
        residual after pre-smoothing (the learned coarse correction; no paper content)."""
        L = self.levels[li]
        if li == len(self.levels) - 1:
            return self.coarse(b)
        x = chebyshev(L.A, L.dinv, b, None, L.lmin, L.lmax, self.degree, x_zero=True)
        r = b - L.A @ x
        if learned is not None and li == learned[0]:
            x = x + learned[1](r)
        else:
            ec = self.vcycle(L.P.T @ r, li + 1, learned)
            x = x + L.P @ ec
        return chebyshev(L.A, L.dinv, b, x, L.lmin, L.lmax, self.degree)


# ----------------------------------------------------------------------------
# The Stokes problem: blocks, weights, w-BFBT
# ----------------------------------------------------------------------------

class Stokes:
    """Assembled multi-sinker Stokes problem on the interior velocity DOFs."""

    def __init__(self, N, k, centers, delta, omega, mu_min, mu_max, beta=10.0,
                 a_l=1.0, a_r=1.0, mu_fn=None, f_fn=None, weights="sqrt"):
        self.mesh = m = fem.Mesh(N, k)
        xq = m.quad_points()
        if mu_fn is None:
            mu_fn = lambda x: sinker.viscosity(x, centers, delta, omega, mu_min, mu_max)
        if f_fn is None:
            f_fn = lambda x: sinker.body_force(x, centers, delta, omega, beta)
        self.mu_q = mu_fn(xq)                                   # [E, n^3]
        self.mu_nodes = mu_fn(m.node_xyz)                       # [n_nodes]
        self.Afull = fem.assemble_A(m, self.mu_q)
        self.Bfull = fem.assemble_B(m)
        self.Ffull = fem.assemble_load(m, f_fn(xq))
        self.Ffull[m.vel_boundary] = 0.0
        self.idx = m.vel_interior
        self.A = self.Afull[self.idx][:, self.idx].tocsr()
        self.B = self.Bfull[:, self.idx].tocsr()
        self.F = self.Ffull[self.idx]
        self.a_l, self.a_r = a_l, a_r
        # BFBT weighting matrices: w-BFBT with sqrt(mu) (Sec. 4) or the viscosity-gradient weights
        # of the remark there, or diag(A)-BFBT (C = D = diag(A), Sec. 4)
        self.weights = weights
        if weights == "sqrt":
            sq = np.sqrt(self.mu_nodes)
            self.C_nodes = fem.lumped_weighted_mass(m, sq, fem.element_amplification(m, a_l))
            self.D_nodes = fem.lumped_weighted_mass(m, sq, fem.element_amplification(m, a_r))
            self.w_q = np.sqrt(self.mu_q)
        elif weights == "grad":
            w_en, self.w_q = fem.gradient_weights(m, self.mu_nodes, self.mu_q)
            self.C_nodes = fem.lumped_weighted_mass_elem(m, w_en, fem.element_amplification(m, a_l))
            self.D_nodes = fem.lumped_weighted_mass_elem(m, w_en, fem.element_amplification(m, a_r))
        else:
            assert weights == "diagA"
            # Reading: the K_w multigrid needs a Poisson coefficient 1/w; diag(A) is taken as the
            # lumped mass of an effective weight, w_eff(x_i) = mean_c diag(A)_(i,c) / m_i (m the
            # unweighted lumped mass), and the coefficient is the element mean of the nodal 1/w_eff
            # (a Q_k interpolant of the nodal values can turn negative between nodes of strongly
            # different weight)
            dA = self.Afull.diagonal().reshape(3, m.n_nodes)
            mass = fem.lumped_weighted_mass(m, np.ones(m.n_nodes), np.ones(m.E))
            self.w_eff = dA.mean(axis=0) / mass
            c_e = (1.0 / self.w_eff[m.elem_nodes]).mean(axis=1)
            self.w_q = np.repeat((1.0 / c_e)[:, None], m.n ** 3, axis=1)
            self.C_nodes = self.D_nodes = None
        if weights == "diagA":
            self.Cinv = self.Dinv = 1.0 / self.A.diagonal()
        else:
            self.Cinv = 1.0 / np.tile(self.C_nodes, 3)[self.idx]
            self.Dinv = 1.0 / np.tile(self.D_nodes, 3)[self.idx]
        self.Kl = (self.B @ sp.diags(self.Cinv) @ self.B.T).tocsr()
        self.Kr = (self.B @ sp.diags(self.Dinv) @ self.B.T).tocsr()
        self.nu, self.np_ = len(self.idx), m.p_dof
        self.ones_p = np.zeros(m.p_dof)
        self.ones_p[::m.n_p] = 1.0                              # constant pressure function

    # -- vector helpers ------------------------------------------------------
    def embed_u(self, ui):
        u = np.zeros(self.mesh.u_dof)
        u[self.idx] = ui
        return u

    def remove_mean(self, p):
        """Subtract the mean of the constant mode (uniform mesh: the L2 mean)."""
        p = p.copy()
        p[::self.mesh.n_p] -= p[::self.mesh.n_p].mean()
        return p

    def stokes_matvec(self, x):
        u, p = x[:self.nu], x[self.nu:]
        return np.concatenate([self.A @ u + self.B.T @ p, self.B @ u])

    def stokes_matrix(self):
        return sp.bmat([[self.A, self.B.T], [self.B, None]]).tocsr()

    # -- exact pieces ----------------------------------------------------------
    def k_pinv_solve(self, K, r):
        """Mean-constrained solve: K x = r - proj, 1_psi^T x = 0."""
        r = self.remove_mean(r)
        one = self.ones_p[:, None]
        S = sp.bmat([[K, sp.csr_matrix(one)], [sp.csr_matrix(one.T), None]]).tocsc()
        sol = spla.spsolve(S, np.concatenate([r, [0.0]]))
        return sol[:-1]

    def middle(self, q):
        """B C^-1 A D^-1 B^T q."""
        return self.B @ (self.Cinv * (self.A @ (self.Dinv * (self.B.T @ q))))

    def wbfbt_exact(self, r):
        """S_w^-1 r = K_l^+ (B C^-1 A D^-1 B^T) K_r^+ r (eq. 8) with exact inverses."""
        y = self.k_pinv_solve(self.Kr, r)
        return self.remove_mean(self.k_pinv_solve(self.Kl, self.middle(y)))

    def schur_dense(self):
        Ad = self.A.toarray()
        Bd = self.B.toarray()
        return Bd @ np.linalg.solve(Ad, Bd.T)

    def direct_solve(self):
        """Saddle-point solve with the pressure mean fixed to zero (Lagrange multiplier)."""
        one = sp.csr_matrix(self.ones_p[None, :])
        Z = sp.csr_matrix((1, self.nu))
        S = sp.bmat([[self.A, self.B.T, None],
                     [self.B, None, one.T],
                     [None, one, None]]).tocsc()
        rhs = np.concatenate([self.F, np.zeros(self.np_), [0.0]])
        sol = spla.spsolve(S, rhs)
        return sol[:self.nu], sol[self.nu:self.nu + self.np_]


class Preconditioner:
    """Upper block-triangular preconditioner (eq. 3) with multigrid blocks and w-BFBT."""

    def __init__(self, st: Stokes, degree=3, schur_sign=-1, schur="wbfbt"):
        self.st = st
        # Schur approximation: w-BFBT (eq. 8) or the diagonal of M_p(1/mu) (eq. 4)
        assert schur in ("wbfbt", "mass")
        self.schur = schur
        self.mass_diag = fem.pressure_mass_diag(st.mesh, st.mu_q)
        # Sign of the Schur block of the preconditioner.  The paper's S = B A^-1 B^T is the
        # negated Schur complement of the saddle matrix (footnote of Sec. 1.1), so the block
        # that approximates the saddle matrix's own Schur complement is -S~ (schur_sign = -1,
        # one eigenvalue cluster at 1; its FGMRES counts match Table 3); +1 is eq. (3) taken
        # literally (clusters at +1 and -1).
        self.schur_sign = schur_sign
        m = st.mesh
        # velocity hierarchy on mu (Sec. 6), Poisson hierarchies on 1/w (eq. 11, 12, Sec. 5)
        self.A_mg = Hierarchy(m.N, m.k, st.mu_q, "velocity", 1000, degree)
        c_l = 1.0 / (fem.element_amplification(m, st.a_l)[:, None] * st.w_q)
        c_r = 1.0 / (fem.element_amplification(m, st.a_r)[:, None] * st.w_q)
        self.Pl_mg = Hierarchy(m.N, m.k, c_l, "poisson", 2000, degree)
        self.Pr_mg = Hierarchy(m.N, m.k, c_r, "poisson", 3000, degree)
        self.I = fem.modal_projection(m)
        self.degree = degree
        self.disc = {}
        for side, K, seed in (("l", st.Kl, 4000), ("r", st.Kr, 5000)):
            dinv = 1.0 / K.diagonal()
            start = st.remove_mean(splitmix64_uniform(seed, st.np_))
            lam = lanczos_max(K, dinv, start)
            self.disc[side] = (K, dinv, 0.1 * lam, 1.1 * lam)

    def k_vcycle(self, side, b):
        """One K_w V-cycle: discontinuous smoothing, Q_k Poisson V-cycle, smoothing, mean removal."""
        K, dinv, lmin, lmax = self.disc[side]
        mg = self.Pl_mg if side == "l" else self.Pr_mg
        x = chebyshev(K, dinv, b, None, lmin, lmax, self.degree, x_zero=True)
        r = b - K @ x
        ec = mg.vcycle(self.I.T @ r)
        x = x + self.I @ ec
        x = chebyshev(K, dinv, b, x, lmin, lmax, self.degree)
        return self.st.remove_mean(x)

    def wbfbt(self, r):
        """Approximate S_w^-1 r: K_l V-cycle of the middle product of the K_r V-cycle."""
        st = self.st
        y = self.k_vcycle("r", st.remove_mean(r))
        return self.k_vcycle("l", st.remove_mean(st.middle(y)))

    def mass_schur(self, r):
        """Approximate S^-1 r by the inverse of the diagonalized M_p(1/mu), mean removed."""
        return self.st.remove_mean(r / self.mass_diag)

    def a_vcycle(self, b):
        return self.A_mg.vcycle(b)

    def apply(self, x):
        """[u~; p~] = P^-1 [r_u; r_p], P = [[A~, B^T], [0, schur_sign S~]] (eq. 3)."""
        st = self.st
        ru, rp = x[:st.nu], x[st.nu:]
        zs = self.wbfbt(rp) if self.schur == "wbfbt" else self.mass_schur(rp)
        zp = self.schur_sign * zs
        zu = self.a_vcycle(ru - st.B.T @ zp)
        return np.concatenate([zu, zp])


def fgmres(matvec, b, precond, rtol=1e-6, restart=100, max_iter=1000):
    """Right-preconditioned flexible GMRES(restart), x0 = 0, modified Gram-Schmidt.

    Stops when ||b - K x_j|| <= rtol ||b|| (Euclidean).  Returns (x, iters, history)."""
    n = len(b)
    x = np.zeros(n)
    bnorm = np.linalg.norm(b)
    hist = [1.0]
    it = 0
    if bnorm == 0.0:
        return x, 0, hist
    r = b.copy()
    while it < max_iter:
        beta = np.linalg.norm(r)
        V = np.zeros((restart + 1, n))
        Z = np.zeros((restart, n))
        H = np.zeros((restart + 1, restart))
        cs = np.zeros(restart)
        sn = np.zeros(restart)
        g = np.zeros(restart + 1)
        g[0] = beta
        V[0] = r / beta
        j_done = 0
        for j in range(restart):
            Z[j] = precond(V[j])
            w = matvec(Z[j])
            for i in range(j + 1):
                H[i, j] = w @ V[i]
                w = w - H[i, j] * V[i]
            H[j + 1, j] = np.linalg.norm(w)
            if H[j + 1, j] > 0:
                V[j + 1] = w / H[j + 1, j]
            for i in range(j):
                t = cs[i] * H[i, j] + sn[i] * H[i + 1, j]
                H[i + 1, j] = -sn[i] * H[i, j] + cs[i] * H[i + 1, j]
                H[i, j] = t
            den = np.hypot(H[j, j], H[j + 1, j])
            cs[j], sn[j] = H[j, j] / den, H[j + 1, j] / den
            H[j, j] = den
            H[j + 1, j] = 0.0
            g[j + 1] = -sn[j] * g[j]
            g[j] = cs[j] * g[j]
            it += 1
            j_done = j + 1
            hist.append(abs(g[j + 1]) / bnorm)
            if abs(g[j + 1]) <= rtol * bnorm or it >= max_iter:
                break
        y = sla.solve_triangular(H[:j_done, :j_done], g[:j_done])
        x = x + Z[:j_done].T @ y
        r = b - matvec(x)
        if np.linalg.norm(r) <= rtol * bnorm:
            break
    return x, it, hist
