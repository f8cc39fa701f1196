// Launchers of the HIP kernels (host side).  All launches go to `st`.
#pragma once

#include <string>

#include "wb_internal.h"

namespace wb {

// HIP-event timing of operator launches (off by default); summary lines are
// "<kernel class>\t<launches>\t<total ms>".
void profile_enable(bool on);
std::string profile_summary(bool reset);

// Operator flags: viscous/Poisson stiffness, gradient B^T p, divergence B u, Dirichlet mask,
// and (FP32 data only) 1D contractions in BF16 on the matrix cores with FP32 accumulation:
// F_MF one product of BF16-rounded operands, F_MF3 operands split into BF16 high and low parts
// (three products).
enum : int { F_A = 1, F_BT = 2, F_B = 4, F_DIR = 8, F_MF = 16, F_MF3 = 32 };

// Sum-factorized element operator on a level with N elements/dir and order k.
// NC = 3 (viscous stress, coef = mu) or 1 (scalar Poisson, coef = c).
//   y    = op(u)  (or y += op(u) when add)  [NC][nn]; every node is written, no zeroing needed
//   pout = B u   (written)                   [E][np]
//   sin: optional per-node input scaling.
// Operators that scatter to nodes (A, the fused Stokes operator) run in two kernels, with `work`
// at least op_workspace_bytes(NC, N, k, sizeof(double)) bytes (valid for FP32 data as well):
//  - A alone while its element contributions fit in the two-pass limit (96 MiB of FP64 by
//    default, at most 128 MiB): all elements in parallel into
//    an element buffer in `work`, then per-node sums of the at most eight contributions;
//  - otherwise, and for the fused Stokes operator: blocks own bricks of elements and accumulate
//    in LDS; values on internal brick faces pass through `work` and are summed by a second kernel.
// B alone and B^T alone (outside the BF16 forms) use the uniform mesh's tensor-product element
// matrix instead: B one element x-line per lane, B^T one node line segment per thread, one
// kernel each and no workspace.
size_t op_workspace_bytes(int NC, int N, int k, size_t elem_size);
// Workspace the operator needs in the form it takes when the two-pass element buffer may use at
// most `cap` bytes (the brick form otherwise).
size_t op_workspace_bytes_capped(int NC, int N, int k, size_t elem_size, size_t cap);
// While alive, operator launches of this thread use the two-pass form only if its element buffer
// takes at most `bytes` (for callers that bring a fixed workspace).
struct WorkspaceCap {
  explicit WorkspaceCap(size_t bytes);
  ~WorkspaceCap();
  WorkspaceCap(const WorkspaceCap&) = delete;
  WorkspaceCap& operator=(const WorkspaceCap&) = delete;
  size_t prev;
};
// Process-wide size limit (MB = 10^6 bytes of FP64 element contributions, clamped to 128 MiB; 96
// MiB by default) below which A applies use the two-pass form; returns the previous limit.
double set_two_pass_limit(double mb);
// FP64 order-3 applies of A and the Poisson operator above the two-pass size: on the FP64 matrix
// cores (on != 0, the default) or with line contractions staged in LDS; returns the previous setting.
int set_matrix_core_ops(int on);

// What an operator kernel does with each finished output value v at index j:
//   EPI_STORE       y_j = v (or y_j += v when add)
//   EPI_RESID       r_j = b_j - v
//   EPI_CHEB_FIRST  r_j = b_j - v, dnew_j = alpha dinv_j r_j       (first Chebyshev step, x0 != 0;
//                                                                 x += dnew is left to the next)
//   EPI_CHEB_STEP   r_j -= v, dnew_j = alpha dold_j + beta dinv_j r_j, x_j += dnew_j
//                   (+ dold_j when add_old: the deferred first correction)
//   EPI_CHEB_ZERO   the first two Chebyshev steps from x0 = 0 in one apply: the operator's
//                   input is d0 = gamma dinv b, formed as it is read (u is not used), then
//                   r_j = b_j - v, dnew_j = alpha d0_j + beta dinv_j r_j, x_j = d0_j + dnew_j
// Buffers written by an epilogue must not be read by the same operator (its input is dold or
// x for EPI_CHEB_STEP / EPI_RESID, so dnew != dold).
enum : int { EPI_STORE = 0, EPI_RESID = 1, EPI_CHEB_FIRST = 2, EPI_CHEB_STEP = 3, EPI_CHEB_ZERO = 4 };
template <typename T>
struct Epi {
  int mode = EPI_STORE;
  int add_old = 0;
  T alpha = T(0), beta = T(0), gamma = T(0);
  T* r = nullptr;
  const T* dold = nullptr;
  T* dnew = nullptr;
  T* x = nullptr;
  const T* dinv = nullptr;
  const T* b = nullptr;
};
template <typename T>
void launch_op(hipStream_t st, int flags, int NC, int N, int k, const T* u, T* y, const T* coef,
               const T* pin, T* pout, const T* sin, bool add, void* work);
// The same with an output epilogue: built for the level operators (F_A, F_A | F_DIR; node
// outputs) and for the divergence F_B | F_DIR (pressure outputs pout, indexed e n_p + m).
template <typename T>
void launch_op_epi(hipStream_t st, int flags, int NC, int N, int k, const T* u, T* y, const T* coef,
                   const T* pin, T* pout, const T* sin, bool add, void* work, const Epi<T>& ep);

// Assembled Q1 levels.  The level operator (A, with the Dirichlet mask when NC = 3; Neumann when
// NC = 1) on N^3 Q1 elements is stored as a 27-point stencil per node:
//   S[((o NC + c) NC + d) nn + i] = entry (node i, component c; node i + o, component d),
//   o = (ox+1) + 3 (oy+1) + 9 (oz+1), ox, oy, oz in {-1, 0, 1}; nn = (N+1)^3.
// assemble_q1 builds S (q1_stencil_len doubles) from the element kernel's own element matrices
// in ae (q1_elem_matrix_len doubles, scratch).  launch_stencil_epi applies it with the epilogues
// of launch_op_epi: the same operator up to rounding order.
size_t q1_elem_matrix_len(int NC, int N);
size_t q1_stencil_len(int NC, int N);
void assemble_q1(hipStream_t st, int NC, int N, bool dir, const double* coef, double* ae, double* S);
template <typename T>
void launch_stencil_epi(hipStream_t st, int NC, int N, const T* S, const T* u, T* y, bool add,
                        const Epi<T>& ep);

// Coarse tail of a scalar (Neumann) V-cycle in one workgroup: on an assembled Q1 level with
// M^3 <= TAIL_MAX nodes (stencil S, inverse diagonal dinv), Chebyshev-Jacobi pre-smoothing from
// x = 0 (deg steps; inv_theta and the step coefficients alpha[it], beta[it], it = 1..deg-1, of
// the level's interval), residual, restriction to the next level (Mc = (M+1)/2 nodes per
// direction, linear 2:1 weights), the dense coarsest solve xc[gidx[r]] = sum_c G[r,c] bc[gidx[c]]
// (nd = Mc^3 rows), prolongation and post-smoothing.  x = V-cycle(b), b and x of length M^3.
constexpr int TAIL_THREADS = 1024, TAIL_MAX = 1024, TAIL_MAXDEG = 8;
template <typename T>
struct TailArgs {
  int M = 0, Mc = 0, nd = 0, deg = 0;
  const T* S = nullptr;
  const T* dinv = nullptr;
  const double* G = nullptr;
  const int* gidx = nullptr;
  T inv_theta = T(0);
  T alpha[TAIL_MAXDEG] = {}, beta[TAIL_MAXDEG] = {};
};
template <typename T>
void launch_vcycle_tail(hipStream_t st, const TailArgs<T>& a, const T* b, T* x);

// Inverse of the diagonal of the inverse viscosity-weighted pressure mass M_p(1/mu) (eq. 4):
// out[e n_p + m] = 1 / sum_q W_q |J| psi_m(x_q)^2 / mu_q (mu at the Gauss points).
void launch_pmass_inv(hipStream_t st, int N, int k, const double* mu_q, double* out);

// Jacobi diagonal (not inverted) of the NC-component operator, accumulated into diag (zeroed).
void launch_diag(hipStream_t st, int NC, int N, int k, bool dir, const double* coef, double* diag);
// dinv = 1/diag, 1 on Dirichlet nodes (if dir).
void launch_invert_diag(hipStream_t st, int NC, int N, int k, bool dir, double* d);

// Lumped sqrt(mu)-weighted GLL mass with amplification `amp` on boundary elements (eq. 8, Sec. 5):
// accumulated into cnodes (zeroed), [nn].
void launch_lumped_mass(hipStream_t st, int N, int k, double amp, const double* mu_nodes,
                        double* cnodes);
// dinvK[e*np+m] = 1 / sum_{c,i interior} (B_e[m,(c,i)])^2 dinv_nodes[g(e,i)]
// (per_component: dinv_nodes is [3][n_nodes], one weight per velocity DOF, as for diag(A)-BFBT)
void launch_diag_K(hipStream_t st, int N, int k, const double* bhat, const double* dinv_nodes,
                   double* dinvK, bool per_component = false);
// diag(A)-BFBT Poisson coefficient at the Gauss points, constant per element: the element mean
// of m_i / mean_c diag3[c][i] over its nodes (diag3 the unmasked diag(A), mass the unweighted
// lumped velocity mass), divided by the boundary amplification a_e.
void launch_diag_a_coef(hipStream_t st, int N, int k, double amp, const double* diag3,
                        const double* mass, double* c_q);

// Multi-sinker viscosity at Gauss points (mu_q) and/or body-force z-component (f_q),
// and at the velocity nodes.
void launch_sinker_q(hipStream_t st, int N, int k, const double* centers, int ns, double delta,
                     double omega, double mu_min, double mu_max, double beta, double* mu_q,
                     double* f_q);
void launch_sinker_nodes(hipStream_t st, int N, int k, const double* x1, const double* centers,
                         int ns, double delta, double omega, double mu_min, double mu_max,
                         double* mu_nodes);
// F_z += int f_z phi_i  (F zeroed by the caller), boundary entries untouched (0).
void launch_load(hipStream_t st, int N, int k, const double* f_q, double* F);
// Coefficient transforms at the Gauss points: c = scale / (amp_e sqrt(mu)) with amp_e on
// boundary elements (Poisson coefficient 1/w of eq. 11-12 and Sec. 5) or a plain FP64->FP32 cast.
void launch_poisson_coef(hipStream_t st, int N, int k, double amp, const double* mu_q, double* c_q);
// The same two products with the viscosity-gradient weights w = (mu^2 + |grad mu|^2)^(1/4) of the
// remark in Sec. 4, grad mu from each element's Q_k interpolant of mu_nodes: the lumped mass per
// element node (accumulated into cnodes, zeroed) and 1/(a_e w) at the Gauss points.
void launch_lumped_mass_grad(hipStream_t st, int N, int k, double amp, const double* mu_nodes,
                             double* cnodes);
void launch_poisson_coef_grad(hipStream_t st, int N, int k, double amp, const double* mu_q,
                              const double* mu_nodes, double* c_q);

// Transfers: tensor product of a 1D sparse matrix (rows: cnt / col / val, width W).
// lin21 marks the rows of linear interpolation between nested node lines with
// M_fine = 2 M_coarse - 1 (weight 1 at shared nodes, 1/2 at midpoints: Q1 h-coarsening and the
// Q2 -> Q1 p-step) or of its transpose; those transfers run in a kernel with the weights built in.
struct Rows1D {
  int rows, cols, W;
  const int* cnt;
  const int* col;
  const double* val;
  int lin21;
};
template <typename T>
void launch_kron(hipStream_t st, const Rows1D& R, int NC, bool dir, bool add, const T* in, T* out);

// Element-wise L2 projection Q_k -> P_{k-1} (p = I u, or p += I u with add) and its transpose
// u = I^T p (u overwritten on every node).
template <typename T>
void launch_modal_I(hipStream_t st, int N, int k, const T* u, T* p, bool add);
template <typename T>
void launch_modal_IT(hipStream_t st, int N, int k, const T* p, T* u);

// L2 adjoint of element-wise interpolation of a coefficient at Gauss points (clamped below by
// the local fine minimum): p-coarsening (same mesh) and h-coarsening (2:1).
void launch_coarsen_p(hipStream_t st, int E, int nf, int nc, const double* Q, const double* in,
                      double* out);
void launch_coarsen_h(hipStream_t st, int Nf, int n, const double* Q, const double* in, double* out);

// y[idx[r]] = sum_c G[r, c] x[idx[c]] (FP64 accumulation), r < nd.
template <typename T>
void launch_dense(hipStream_t st, int nd, const double* G, const int* idx, const T* x, T* y);

// Vector kernels.
template <typename T> void launch_fill(hipStream_t st, T* x, T v, size_t n);
template <typename T> void launch_axpby(hipStream_t st, size_t n, T a, const T* x, T b, T* y);
template <typename Ta, typename Tb> void launch_cast(hipStream_t st, size_t n, const Ta* a, Tb* b);
template <typename T>
void launch_scale_nodes(hipStream_t st, int nn, int NC, const T* s, const T* x, T* y);
// Chebyshev: r = b - t (t may be null), d = dinv r / theta, x = x0 + d (x0 = 0 if xzero)
template <typename T>
void launch_cheb_first(hipStream_t st, size_t n, const T* b, const T* t, const T* dinv, T inv_theta,
                       T* d, T* x, T* r, bool xzero);
// y = a x
template <typename T> void launch_scal(hipStream_t st, size_t n, T a, const T* x, T* y);
// zero the boundary nodes of an NC-component nodal vector with M nodes per direction
template <typename T> void launch_mask_boundary(hipStream_t st, int M, int NC, T* x);
// c = a * b (elementwise)
template <typename T> void launch_mul(hipStream_t st, size_t n, const T* a, const T* b, T* c);
// r = b - t
template <typename T> void launch_sub(hipStream_t st, size_t n, const T* b, const T* t, T* r);

// Jacobi-CG step halves with the scalars in device memory: r -= (rz/pq) q, z = dinv r, and
// rz_new = r . z (partial: reduction scratch as for launch_dot); p = z + (rz_new/rz_old) p
// (non-positive denominators give a zero coefficient).
void launch_cg_r(hipStream_t st, size_t n, const double* q, const double* dinv, double* r, double* z,
                 const double* rz, const double* pq, double* partial, double* rz_new);
void launch_cg_p(hipStream_t st, size_t n, const double* z, double* p, const double* rz_new,
                 const double* rz_old);
// y = x / sqrt(*d), d a device scalar (a squared norm); y = 0 when *d <= 0.
void launch_scal_rnorm(hipStream_t st, size_t n, const double* d, const double* x, double* y);
// x_i = 2 U(splitmix64(seed * 2^32 + i)) - 1, zero on boundary nodes of an [NC][M^3] vector
// when M > 0 (the counter-based generator of the eigenvalue-estimate start vectors).
void launch_splitmix_vec(hipStream_t st, size_t n, unsigned long long seed, int M, double* x);
// x -= mean(x) (two-stage sum, deterministic)
void launch_remove_global_mean(hipStream_t st, size_t n, double* x, double* partial, double* scratch);

// Reductions into a device FP64 scalar (block partials summed in block order, deterministic).
// partial: at least RED_BLOCKS + 1 doubles.  Reductions over at most RED_LAST_BLOCKS blocks
// (launch_remove_mean always, launch_dot and launch_cg_r for n <= 256 RED_LAST_BLOCKS) finish in
// the last block to complete, in one launch, and use partial[RED_BLOCKS] as a completion counter,
// which must be zero before the first call (it is left zero); larger ones take a second launch.
template <typename T>
void launch_dot(hipStream_t st, size_t n, const T* x, const T* y, double* partial, double* out);
constexpr int RED_BLOCKS = 1024;
constexpr int MDOT_BLOCKS = 1024;
constexpr int RED_LAST_BLOCKS = 64;  // blocks of the single-launch reductions
// Pressure mean of the constant mode: p[e*np] -= mean_e p[e*np].
template <typename T>
void launch_remove_mean(hipStream_t st, int E, int np, T* p, double* partial, double* scratch);

// FGMRES helpers (FP64): h[v] = V[v] . w for v < nv (V rows of stride ld; partial holds
// MDOT_BLOCKS doubles per vector), w -= sum_v h[v] V[v], x += sum_v y[v] Z[v].
void launch_mdot(hipStream_t st, size_t n, int nv, const double* V, size_t ld, const double* w,
                 double* partial, double* h);
void launch_gemv_sub(hipStream_t st, size_t n, int nv, const double* V, size_t ld, const double* h,
                     double* w);
// w -= sum_v h[v] V[v], then h2[v] = V[v] . w for the updated w, from one read of V (the update of
// one classical Gram-Schmidt sweep and the projections of the next); false (nothing launched) when
// nv exceeds the kernel's LDS staging.
bool launch_gs_sub_dot(hipStream_t st, size_t n, int nv, const double* V, size_t ld,
                       const double* h, double* w, double* partial, double* h2);
void launch_gemv_add(hipStream_t st, size_t n, int nv, const double* Z, size_t ld, const double* y,
                     double* x);

}  // namespace wb
