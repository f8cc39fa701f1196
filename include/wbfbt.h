/*
 * wbfbt.h -- C-ABI of the MI355X (gfx950) w-BFBT Stokes library.
 *
 * The library implements, with hand-written HIP kernels, the data-parallel hot
 * path of the weighted-BFBT preconditioned Stokes solver of Rudi, Stadler and
 * Ghattas, "Weighted BFBT preconditioner for Stokes flow problems with highly
 * heterogeneous viscosity" (arXiv 1607.03936):
 *
 *   -div[mu (grad u + grad u^T)] + grad p = f,   -div u = 0,   u = 0 on the
 *   boundary of the unit cube (eq. 1), discretized with continuous nodal Q_k
 *   velocity and discontinuous modal P_{k-1} pressure on a uniform N^3
 *   hexahedral mesh (Sec. 1.2, eq. 2).
 *
 * Conventions shared by every entry point
 * ----------------------------------------
 *  - All vector buffers are DEVICE pointers owned by the caller (for example
 *    torch tensors' data_ptr()).  Handles (wb_mesh, wb_visc, wb_solver) and
 *    their internal workspaces are owned by the library.
 *  - `stream` is a hipStream_t (NULL = default stream).  Apply calls only
 *    enqueue work and return; wb_visc_*, wb_solver_create and wb_solve
 *    synchronize the stream.
 *  - Velocity vectors are [3][n_nodes] (component-major), n_nodes = (kN+1)^3,
 *    node g = gi + M (gj + M gl), M = kN+1, node (gi, gj, gl) at the
 *    Gauss-Lobatto-Legendre points of each element.  Values at boundary nodes
 *    are ignored on input and written as 0 on output (no-slip).
 *  - Pressure vectors are [E][n_p], E = N^3 elements e = ex + N (ey + N ez),
 *    n_p = k(k+1)(k+2)/6 Legendre modes L_a(x) L_b(y) L_c(z), a+b+c <= k-1,
 *    ordered c slowest, then b, then a; mode 0 is the constant.
 *  - Coefficients at quadrature points are [E][(k+1)^3], Gauss-Legendre
 *    points q = qx + n (qy + n qz), n = k+1.
 *  - Every call returns a wb_status; on failure wb_last_error() gives a
 *    thread-local message.  No partial results are guaranteed on failure.
 *  - k in {1,...,5} for operator applies, k in {2,...,5} for Stokes solves (the BF16
 *    matrix-core precision forms: k <= 4).
 */
#ifndef WBFBT_H
#define WBFBT_H

#include <stddef.h>

#ifdef __cplusplus
extern "C" {
#endif

#define WB_API __attribute__((visibility("default")))

typedef enum {
  WB_OK = 0,
  WB_EINVAL = 1,        /* bad argument (size, order, NULL handle)           */
  WB_ENOMEM = 2,        /* device allocation failed                          */
  WB_EHIP = 3,          /* a HIP runtime call failed                          */
  WB_ENOCONV = 4,       /* FGMRES reached max_iter before rtol               */
  WB_ENAN = 5,          /* NaN or Inf met in a reduction                      */
  WB_EUNSUPPORTED = 6   /* order or option not built                          */
} wb_status;

/* Arithmetic of the preconditioner (and of wb_apply_A_lowp).  WB_BF16: FP32 data, every 1D
 * tensor contraction of the element operators on the BF16 matrix cores with FP32 accumulation,
 * table and line each split into BF16 high and low parts (three products, about 2^-16 relative
 * error per contraction).  WB_BF16X1: the same with a single product of BF16-rounded operands
 * (about 2^-8 per contraction).  The two BF16 forms are built for k <= 4 (WB_EUNSUPPORTED for
 * k = 5). */
typedef enum { WB_FP64 = 0, WB_FP32 = 1, WB_BF16 = 2, WB_BF16X1 = 3 } wb_prec;

typedef struct wb_mesh wb_mesh;
typedef struct wb_visc wb_visc;
typedef struct wb_solver wb_solver;

/* Solver options.  Defaults (wb_opts_default) follow the paper's settings:
 * Chebyshev-accelerated point-Jacobi smoothing with 3 pre- and 3 post-steps,
 * GMRES restarted every 100 iterations, relative residual 1e-6 (Sec. 6-7). */
typedef struct {
  double a_l, a_r;        /* Dirichlet boundary amplification of w_l, w_r (Sec. 5) */
  int cheb_degree;        /* Chebyshev-Jacobi steps per smoothing (3)              */
  int lanczos_steps;      /* CG steps for the largest-eigenvalue estimate (10;
                             1..100)                                              */
  int restart;            /* FGMRES restart length (100)                           */
  int max_iter;           /* FGMRES iteration cap (1000)                           */
  double rtol;            /* ||b - K x|| <= rtol ||b|| (1e-6)                      */
  int precond_prec;       /* wb_prec of the preconditioner: WB_FP64, WB_FP32,
                             WB_BF16 or WB_BF16X1 (FP32 with BF16 MFMA contractions) */
  int use_learned;        /* 1: learned coarse correction in the velocity V-cycle  */
  int p_schedule;         /* order coarsening: 0 halves k (4->2->1, 3->1, 2->1),
                             1 lowers it by one (4->3->2->1, 3->2->1)              */
  int verbose;            /* 1: print the residual history to stderr              */
  int use_graph;          /* 1: wb_solve replays the preconditioner apply from a
                             HIP graph captured at its first iteration (default);
                             0: every launch is issued from the host             */
  int schur_sign;         /* sign of the Schur block of the preconditioner (eq. 3):
                             -1 (default): -S~, the saddle matrix's own Schur
                             complement sign (the paper's S is its negation);
                             +1: eq. (3) as printed                              */
  double assemble_mb;     /* Q1 multigrid levels whose assembled 27-point stencil
                             takes at most this many MB (FP64) are applied as
                             stencils instead of element kernels (32); the coarsest
                             level is always assembled; 0: element kernels only   */
  int schur_approx;       /* Schur block of the preconditioner: 0 (default) w-BFBT
                             (eq. 8); 1 the inverse viscosity-weighted pressure
                             mass M_p(1/mu) (eq. 4), diagonalized (its diagonal:
                             entries sum_q W_q |J| psi_m^2 / mu_q), the comparison
                             baseline of Sec. 8                                   */
  int weights;            /* BFBT weighting: w-BFBT with w_l = w_r (before the boundary
                             amplification) 0 (default) sqrt(mu) (Sec. 4) or
                             1 (mu^2 + |grad mu|^2)^(1/4) (the remark of Sec. 4),
                             grad mu of each element's Q_k interpolant of mu;
                             2 diag(A)-BFBT: C = D = diag(A) per velocity DOF,
                             K_w Poisson coefficient the element mean of the nodal
                             lumped mass / diag(A) (no amplification unless set) */
} wb_opts;

typedef struct {
  int iters;              /* FGMRES iterations                                     */
  double rel_res;         /* final true relative residual ||b - K x|| / ||b||      */
  double t_setup_s;       /* wall time of wb_solver_create                         */
  double t_solve_s;       /* wall time of the last wb_solve                        */
  int fell_back;          /* learned correction rejected in favour of the V-cycle  */
  int learned_used;       /* learned correction applications that were accepted    */
  size_t device_bytes;    /* device memory held by the solver                      */
  double learned_reduction; /* |r - alpha A delta| / |r| of the learned correction's
                             first application in the last solve (1 if none)       */
  const double* history;  /* HOST, owned by the solver, valid until its next solve or
                             destruction: the relative residual estimate of FGMRES
                             after iterations 1 .. history_len (wb_solve), or of
                             GMRES (wb_subsolve)                                    */
  int history_len;
} wb_report;

WB_API void wb_opts_default(wb_opts* o);
WB_API const char* wb_last_error(void);

/* ---- mesh (Sec. 1.2): uniform N^3 hexahedra of the unit cube, order k ---- */
/* N >= 1, 1 <= k <= 5.  Creates structured metadata only (no device memory). */
WB_API wb_status wb_mesh_create(int N, int k, wb_mesh** out);
WB_API void wb_mesh_destroy(wb_mesh* m);
/* n_nodes = (kN+1)^3, n_elem = N^3, n_p = k(k+1)(k+2)/6. Any output may be NULL. */
WB_API wb_status wb_mesh_sizes(const wb_mesh* m, long long* n_nodes, long long* n_elem, int* n_p);

/* ---- viscosity (Sec. 2.1, multi-sinker benchmark) ----
 * mu(x) = (mu_max - mu_min)(1 - chi(x)) + mu_min,
 * chi(x) = prod_i [1 - exp(-delta max(0, |c_i - x| - omega/2)^2)].
 * centers_host: [n_sinkers][3] HOST doubles in (0,1)^3 (n_sinkers >= 0).
 * Evaluates mu at every element's Gauss points and at the velocity nodes. */
WB_API wb_status wb_visc_create_sinker(const wb_mesh* m, const double* centers_host, int n_sinkers,
                                       double delta, double omega, double mu_min, double mu_max,
                                       void* stream, wb_visc** out);
/* A viscosity given by its values: mu_q_dev [E][(k+1)^3] at the Gauss points and
 * mu_nodes_dev [n_nodes] at the velocity nodes, both DEVICE, copied in. */
WB_API wb_status wb_visc_create_values(const wb_mesh* m, const double* mu_q_dev,
                                       const double* mu_nodes_dev, void* stream, wb_visc** out);
/* Copies the stored values out (either pointer may be NULL). */
WB_API wb_status wb_visc_values(const wb_visc* v, double* mu_q_dev, double* mu_nodes_dev, void* stream);
WB_API void wb_visc_destroy(wb_visc* v);

/* ---- right-hand side (Sec. 2.1): f = (0, 0, beta (chi - 1)) ----
 * F_i = sum over elements of the Gauss-quadrature integral of f . phi_i;
 * f_dev: [3][n_nodes] DEVICE, overwritten (boundary entries 0). */
WB_API wb_status wb_rhs_sinker(const wb_mesh* m, const double* centers_host, int n_sinkers,
                               double delta, double omega, double beta, double* f_dev, void* stream);

/* wb_apply_A without any device allocation, for callers that cannot allocate (code under HIP
 * graph capture, tight serving loops, harnesses that forbid hipMalloc): the same operator and
 * kernels as wb_apply_A, with the library's fixed per-device workspace of 64 MiB (a device array
 * each GPU holds until the process ends) instead of the mesh's allocated one.  Meshes whose
 * workspace does not fit are rejected with WB_EINVAL (the two-pass form is used only while its
 * element buffer fits, the brick form otherwise: 32^3 Q2, 16^3 Q4 and 48^3 Q2 fit, 64^3 Q3 does
 * not).  No contents need to survive between calls; calls that overlap on one GPU (other
 * threads or streams) race on the workspace and must be ordered by the caller. */
WB_API wb_status wb_apply_A_noalloc(const wb_mesh* mesh, const wb_visc* visc, const double* u,
                                    double* y, void* stream);

/* ---- discrete operators of eq. (2), matrix-free ----
 * A: viscous stress, (A u)_i = sum_e int_e 2 mu eps(u) : eps(phi_i)   (Sec. 1.2, 3.1)
 * B: divergence, (B u)_{e,m} = -int_e psi_m div u  (B = -div, Sec. 3.1)
 * B^T: gradient, (B^T p)_i = -sum_e int_e p div phi_i
 * u, y: [3][n_nodes]; p: [E][n_p].  Outputs are overwritten.  In-place (u == y) is not allowed. */
WB_API wb_status wb_apply_A(const wb_mesh* m, const wb_visc* v, const double* u, double* y, void* stream);
WB_API wb_status wb_apply_B(const wb_mesh* m, const double* u, double* p, void* stream);
WB_API wb_status wb_apply_BT(const wb_mesh* m, const double* p, double* u, void* stream);
/* y += A u (no zeroing of y first): accumulate the viscous-stress apply into y. */
WB_API wb_status wb_apply_A_add(const wb_mesh* m, const wb_visc* v, const double* u, double* y,
                                void* stream);
/* Fused Stokes operator of eq. (2): yu = A u + B^T p, yp = B u (one kernel). */
WB_API wb_status wb_apply_stokes(const wb_mesh* m, const wb_visc* v, const double* u, const double* p,
                                 double* yu, double* yp, void* stream);
/* Reduced-precision A apply: FP32 buffers; prec = WB_FP32 (FP32 arithmetic), WB_BF16 or
 * WB_BF16X1 (BF16 MFMA contractions accumulated in FP32, see wb_prec). */
WB_API wb_status wb_apply_A_lowp(const wb_mesh* m, const wb_visc* v, int prec, const float* u,
                                 float* y, void* stream);
/* Reduced-precision divergence and gradient (the B and B^T of wb_apply_B / wb_apply_BT on FP32
 * buffers, used by the precision forms of the preconditioner): prec = WB_FP32 (FP32 arithmetic,
 * the uniform mesh's tensor-product line kernels), WB_BF16 or WB_BF16X1 (the sum-factorized
 * element contractions on the BF16 matrix cores, FP32 accumulation; k <= 4).  k >= 2. */
WB_API wb_status wb_apply_B_lowp(const wb_mesh* m, int prec, const float* u, float* p, void* stream);
WB_API wb_status wb_apply_BT_lowp(const wb_mesh* m, int prec, const float* p, float* u, void* stream);

/* ---- solver: w-BFBT (eq. 8, Sec. 5) + p/h-multigrid (Sec. 6) + FGMRES (eq. 3) ----
 * Builds the velocity multigrid hierarchy, the weights C = M(w_l), D = M(w_r),
 * w = a sqrt(mu), the two pressure-Poisson hierarchies and the Krylov space.
 * opts may be NULL (defaults).  Synchronizes `stream`.  Needs 2 <= k <= 5 (WB_EUNSUPPORTED
 * otherwise). */
WB_API wb_status wb_solver_create(const wb_mesh* m, const wb_visc* v, const wb_opts* opts,
                                  void* stream, wb_solver** out);
WB_API void wb_solver_destroy(wb_solver* s);

/* z = S_w^-1 r: K_l^-1 (B C^-1 A D^-1 B^T) K_r^-1 r with each K^-1 one
 * V-cycle (eq. 8); r, z: [E][n_p] FP64; the output has zero mean. */
WB_API wb_status wb_apply_wbfbt(wb_solver* s, const double* r, double* z, void* stream);
/* z = (one V-cycle of A) r, Sec. 6; r, z: [3][n_nodes]. */
WB_API wb_status wb_apply_vcycle_A(wb_solver* s, const double* r, double* z, void* stream);
/* K_w = B D_w^-1 B^T with w the left (side 0) or right (side 1) weight (eq. 8). */
WB_API wb_status wb_apply_K(wb_solver* s, int side, const double* p, double* y, void* stream);
/* z = (one K_w V-cycle) r: discontinuous smoothing, Q_k Poisson V-cycle with
 * coefficient 1/w (eq. 11-12, Sec. 6), smoothing, mean removal. */
WB_API wb_status wb_apply_vcycle_K(wb_solver* s, int side, const double* r, double* z, void* stream);
/* Upper block-triangular preconditioner of eq. (3):
 * z_p = S_w^-1 r_p, z_u = (A V-cycle)(r_u - B^T z_p). */
WB_API wb_status wb_apply_precond(wb_solver* s, const double* r_u, const double* r_p,
                                  double* z_u, double* z_p, void* stream);
/* FGMRES(restart), right-preconditioned, x0 = 0, on K [u; p] = [f; 0].
 * f: [3][n_nodes]; u, p: outputs (p has zero mean).  rep may be NULL.
 * Returns WB_ENOCONV if max_iter is reached (u, p hold the last iterate). */
WB_API wb_status wb_solve(wb_solver* s, const double* f, double* u, double* p, wb_report* rep,
                          void* stream);

/* Sub-solves of the paper's Table 3: GMRES (same restart / rtol / max_iter as wb_solve, x0 = 0)
 * on one block preconditioned by one of its V-cycles: which = 0 solves A u = b (b, x
 * [3][n_nodes], boundary entries 0), which = 1 / 2 solves K_l p = b / K_r p = b (b, x [E][n_p];
 * the mean of b is removed first and x has zero mean).  Iterations and residual go to rep. */
WB_API wb_status wb_subsolve(wb_solver* s, int which, const double* b, double* x, wb_report* rep,
                             void* stream);

/* Inspection of setup products (for tests).  what:
 *   0 C^-1 per node [n_nodes]          1 D^-1 per node [n_nodes]
 *     (weights = 2: per velocity DOF [3][n_nodes])
 *   2 inverse Jacobi diagonal of A at `level` [3][n_nodes(level)]
 *   3 coarsened viscosity at `level` [E(level)][(k(level)+1)^3]
 *   4 inverse diagonal of K_l [E][n_p]  5 inverse diagonal of K_r [E][n_p]
 *   6 Poisson coefficient 1/w_l at `level`, 7 same for 1/w_r
 *   8 inverse Jacobi diagonal of the left Poisson operator at `level`
 *   9 inverse of the diagonalized M_p(1/mu) (eq. 4) [E][n_p]
 * out_dev: DEVICE FP64 buffer of the stated size. */
WB_API wb_status wb_solver_query(wb_solver* s, int what, int level, double* out_dev, void* stream);
/* Hierarchy description: which = 0 velocity, 1 left Poisson, 2 right Poisson,
 * 3 discontinuous K levels (nlevels = 2: left, right).  Arrays of length >= 16;
 * lmax[l] is the Chebyshev upper bound (1.1 x the Lanczos estimate), 0 on the coarsest. */
WB_API wb_status wb_solver_levels(wb_solver* s, int which, int* nlevels, int* Ns, int* ks, double* lmax);

/* ---- learned coarse correction (velocity V-cycle, level Q1 on N/2) ----
 * The paper has no learned component; this is a data-driven stand-in for the coarse-grid
 * correction of the velocity multigrid (Sec. 6).  At the velocity level lc = Q1 on N/2 elements
 * per direction (M = N/2 + 1 nodes per direction), the V-cycle pre-smooths, forms
 *   r = b - A_c x,  rho = rms(r),  delta = rho N_theta(f, r / rho) / diag(A_c)  (0 on the boundary),
 *   x <- x + alpha delta,  alpha = clip((r, A_c delta) / (A_c delta, A_c delta), 0, 2)
 * in place of the restriction, the recursion below lc and the prolongation, and post-smooths.
 * f is the node feature (mean log10 mu of the adjacent elements, / 5).  N_theta: FP32 3x3x3
 * convolutions with zero padding, 4 -> 16 -> 16 -> 16 -> 3 channels, leaky ReLU (slope 0.1).
 * It is used by wb_solve when opts.use_learned = 1 and the network is trained or set.  The plain
 * V-cycle is the fallback: the solve's first preconditioner apply checks the correction
 * (wb_report.learned_reduction = |r - alpha A_c delta| / |r| there) and keeps it only if that is
 * at most 0.9, otherwise it repeats the apply with the plain V-cycle and uses it for the rest of
 * the solve; FGMRES also switches to the plain V-cycle when the residual falls by less than half
 * over 20 iterations.  wb_report.fell_back counts rejected steps (alpha = 0) and such switches. */
typedef struct {
  int pairs_per_field;    /* training pairs per viscosity field (8)                       */
  int vcycles;            /* pre-smoothing passes (the V-cycle's Chebyshev smoother at lc)
                             applied to each random start error (1)                       */
  int epochs;             /* passes over the training pairs (20)                          */
  int batch;              /* pairs per Adam step (8)                                      */
  double lr;              /* Adam step size (1e-3; beta 0.9, 0.999, eps 1e-8)             */
  unsigned long long seed;/* splitmix64 seed of start errors, initial weights, shuffles   */
  double delta, omega, mu_min, mu_max;  /* sinker parameters of the training fields       */
  int n_valid;            /* trailing fields held out for the validation loss (0)         */
} wb_train_opts;

typedef struct {
  double loss_first, loss_last;  /* mean training loss of the first and last epoch        */
  double valid_loss;             /* mean loss on the held-out fields (0 if none)          */
  double t_pairs_s, t_train_s;   /* wall time of pair generation and of the Adam epochs   */
  long long n_params;
  int n_pairs;
} wb_train_report;

WB_API void wb_train_opts_default(wb_train_opts* o);
/* Train the network of solver s on its GPU.  Field f has n_sinkers[f] sinker centers, stored
 * after those of fields 0..f-1 in centers_host ([sum n_sinkers][3], HOST).  For each field the
 * library evaluates the sinker viscosity on the solver's mesh, coarsens it to level lc like the
 * solver's own hierarchy (that field's own diagonal, Chebyshev bounds and, where the solver
 * assembles lc, stencil), and forms pairs: e = (I - S A_c)^vcycles e0 with e0 a splitmix64
 * field and S the pre-smoother at lc (the error left for the coarse correction), r = A_c e,
 * target d e / rho and weight rho^2 / (d sum_j d_j e_j^2) (d = diag A_c) for the loss
 * (1/B) sum w (N_theta - t)^2 (N_theta = 0 scores 1).  Then Adam over shuffled batches, from
 * fresh He-uniform weights with a zero output layer.
 * Synchronizes the stream.  WB_EUNSUPPORTED if the mesh has no level Q1 on N/2 above the
 * coarsest; WB_EINVAL for bad options. */
WB_API wb_status wb_learned_train(wb_solver* s, int n_fields, const int* n_sinkers,
                                  const double* centers_host, const wb_train_opts* opts,
                                  wb_train_report* rep, void* stream);
/* Flat FP32 parameter blob (HOST pointers): per layer W [Cout][Cin][27] (tap dx + 3 dy + 9 dz
 * multiplies the input at offset (dx-1, dy-1, dz-1)), then b [Cout].  get: size query with
 * params == NULL.  set: n_params must match; marks the network trained. */
WB_API wb_status wb_learned_get(wb_solver* s, float* params, long long* n_params);
WB_API wb_status wb_learned_set(wb_solver* s, const float* params, long long n_params);
/* Level index lc in the velocity hierarchy, nodes per direction M there, parameter count. */
WB_API wb_status wb_learned_info(wb_solver* s, int* level, int* M, long long* n_params);
/* The correction step for a given residual r at level lc ([3][M^3], FP64, device): writes
 * delta (device) and alpha (HOST) without applying it. */
WB_API wb_status wb_learned_probe(wb_solver* s, const double* r, double* delta, double* alpha,
                                  void* stream);

/* Network kernels on caller data (all device pointers, FP32, fields [b][channel][z][y][x]):
 * x [B][4][M^3] -> out [B][3][M^3]; with t, w [B][3][M^3] and grad [n_params] also the loss
 * (1/B) sum w (out - t)^2 (HOST *loss) and its parameter gradient (t, w, grad all or none).
 * Allocates its work space.  wb_net_adam: one bias-corrected Adam step (step >= 1) on params
 * with moments m, v.  wb_net_feature: node feature of a Q1 coefficient [N^3][8] (FP64) on
 * (N+1)^3 nodes. */
WB_API long long wb_net_param_count(void);
WB_API wb_status wb_net_eval(int M, int B, const float* params, const float* x, const float* t,
                             const float* w, float* out, float* grad, double* loss, void* stream);
WB_API wb_status wb_net_adam(long long n, float* params, const float* grad, float* m, float* v,
                             int step, double lr, void* stream);
WB_API wb_status wb_net_feature(int N, const double* coef, float* feat, void* stream);

/* ---- device memory ----
 * Device memory of destroyed solvers is kept in a cache of blocks by (device, size) and reused
 * by later solvers that ask for the same sizes; a failed allocation empties the cache and
 * retries.  wb_mem_trim frees every cached block (call it with no solver work in flight). */
WB_API void wb_mem_trim(void);

/* ---- instrumentation ----
 * When enabled, every operator-kernel launch is bracketed by HIP events on the
 * stream it is launched on.  wb_profile_summary writes lines
 * "<kernel class>\t<launches>\t<total ms>" into buf (NUL-terminated, truncated
 * to len) after waiting for the recorded events, optionally clearing them;
 * returns the full summary length. */
WB_API void wb_profile_enable(int on);
WB_API long long wb_profile_summary(char* buf, long long len, int reset);

/* ---- operator form ----
 * A and Poisson applies whose element contributions take at most `mb` MB (10^6 bytes) in FP64
 * (clamped to [0, 134.2], i.e. 128 MiB; 96 MiB = 100.7 MB by default) run in two passes (all
 * elements into an element buffer, then per-node
 * sums); larger ones as brick scatters with brick-face sums.  Both give the operator up to
 * rounding order.  Process-wide, for tests and tuning; workspaces are sized for both forms, so it
 * may be changed at any time (a captured preconditioner graph keeps the form it was captured
 * with).  Returns the previous limit. */
WB_API double wb_set_two_pass_limit(double mb);

/* Order-3 (Q3) brick applies of A and of the scalar Poisson operator (the form above the
 * two-pass limit; FP64 data, or the FP32 data of the FP32 precision form) run their 1D
 * contractions in x and y on the FP64 matrix cores (v_mfma_f64_4x4x4, on != 0, the default), with
 * their Chebyshev and residual updates as a separate streaming pass and the Stokes operator as A,
 * then B^T added, then B; or as line contractions staged in LDS with the updates and the Stokes
 * operator fused (on == 0).  The same operators up to rounding order.  Process-wide, for tests and
 * tuning; a captured preconditioner graph keeps the form it was captured with.  Returns the
 * previous setting. */
WB_API int wb_set_matrix_core_ops(int on);

#ifdef __cplusplus
}
#endif

#endif /* WBFBT_H */
