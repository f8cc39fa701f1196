// Multigrid hierarchies, w-BFBT apply, block preconditioner and FGMRES (host orchestration).
#pragma once

#include <functional>
#include <memory>
#include <vector>

#include "kernels.h"
#include "learned.h"

namespace wb {

// Device allocations owned by one object, released together (into the block cache, see
// mem_trim).  Sizes are rounded up to 256 bytes.
class Arena {
 public:
  Arena() = default;
  Arena(const Arena&) = delete;
  Arena& operator=(const Arena&) = delete;
  ~Arena();
  template <typename T>
  T* alloc(size_t n) {
    return static_cast<T*>(raw(n * sizeof(T)));
  }
  void* raw(size_t bytes);
  size_t bytes() const { return bytes_; }

 private:
  std::vector<void*> ptrs_;
  std::vector<size_t> sizes_;
  size_t bytes_ = 0;
  int dev_ = 0;
};
// Free every cached device block.
void mem_trim();

// One re-discretized level of a hierarchy (velocity: NC = 3, Dirichlet; Poisson: NC = 1, Neumann).
template <typename T>
struct Level {
  int N = 0, k = 0, NC = 3;
  bool dir = true;
  int nn = 0, E = 0;
  size_t len = 0;          // NC * nn
  T* coef = nullptr;       // coefficient at Gauss points [E][(k+1)^3]
  T* dinv = nullptr;       // inverse Jacobi diagonal [len]
  double lmin = 0, lmax = 0;
  T *x = nullptr, *b = nullptr, *r = nullptr, *d = nullptr, *t = nullptr;
  Rows1D P{}, R{};         // prolongation from / restriction to the next coarser level
  const double* Q = nullptr;  // coefficient coarsening matrix from the next finer level
  T* S = nullptr;          // assembled 27-point stencil (Q1 levels within the size limit), else null
};

template <typename T>
struct Hierarchy {
  std::vector<Level<T>> L;
  int nd = 0;              // coarsest dense (pseudo-)inverse size
  double* G = nullptr;     // [nd][nd] FP64
  int* gidx = nullptr;     // dense index -> vector index
};

// The (N, k) level schedule: lower k to 1 (halving, or by one when p_schedule == 1), then
// halve N while N/2 >= 4.
std::vector<std::pair<int, int>> level_schedule(int N, int k, int p_schedule);

struct Solver;
constexpr int LZ_SLOTS = 4096;     // device scalars of the eigenvalue estimates of one setup
constexpr int AUX_STREAMS = 4;     // streams of the concurrent setup estimates

// Preconditioner state in precision T (FP64 or FP32).
template <typename T>
struct Precond {
  Hierarchy<T> A;           // velocity hierarchy (coefficient mu)
  Hierarchy<T> Pois[2];     // left / right Poisson hierarchies (coefficient 1/w)
  T* winv[2] = {nullptr, nullptr};  // C^-1, D^-1 per node [nn]
  T* dk[2] = {nullptr, nullptr};    // inverse diagonal of K_l, K_r [E*np]
  T* mpinv = nullptr;               // inverse diagonal of M_p(1/mu) [E*np] (eq. 4)
  double klmin[2] = {0, 0}, klmax[2] = {0, 0};
  // work
  T *v1 = nullptr, *v2 = nullptr, *vt = nullptr;                       // velocity [3 nn]
  T *pb = nullptr, *px = nullptr, *pr = nullptr, *pd = nullptr, *pt = nullptr, *pm = nullptr,
    *py = nullptr;                                                     // pressure [E np]
  T *cin_u = nullptr, *cin_p = nullptr, *cout_u = nullptr, *cout_p = nullptr;  // casts (FP32)
};

// Learned coarse correction state: network parameters, the node feature of the solver's
// viscosity at the velocity level lc (Q1 on N/2), inference buffers and device counters.
// A learned coarse correction stays in use for a solve when its first application leaves at
// most this fraction of the residual at its level (a reading: the paper has no learned part).
constexpr double LEARNED_ACCEPT = 0.9;

struct Learned {
  int lc = -1, M = 0;
  bool trained = false;
  bool active = true;          // false while training pairs are generated / after stagnation
  float* params = nullptr;     // [net_param_count()]
  float* feat = nullptr;       // [M^3]
  float* xin = nullptr;        // [4][M^3]
  float* elem_tmp = nullptr;   // [(M-1)^3]
  NetWork w1;                  // batch-1 inference buffers
  int* counters = nullptr;     // [2]: accepted, rejected correction steps
};

struct Solver {
  Mesh m;
  wb_opts o;
  hipStream_t st = nullptr;
  Arena arena;
  double* mu_q = nullptr;   // fine viscosity (FP64)
  std::unique_ptr<Precond<double>> pd;
  std::unique_ptr<Precond<float>> pf;
  void* opwork = nullptr;         // face-array workspace shared by all operator applies
  double* red_partial = nullptr;  // reduction scratch
  double* red_out = nullptr;      // [16] device scalars
  double* lz = nullptr;           // [LZ_SLOTS] Lanczos scalars
  double* ae = nullptr;           // element-matrix scratch of the Q1 assembly
  size_t ae_len = 0;
  // setup: eigenvalue estimates of independent levels run concurrently on auxiliary streams,
  // each with its own reduction scratch and face-array workspace
  hipStream_t aux[AUX_STREAMS] = {};
  hipEvent_t aux_ev[AUX_STREAMS] = {};
  hipEvent_t main_ev = nullptr;
  double* aux_partial[AUX_STREAMS] = {};
  void* aux_work[AUX_STREAMS] = {};
  // Krylov space
  size_t n_tot = 0;
  double *V = nullptr, *Z = nullptr, *w = nullptr, *hbuf = nullptr, *mpartial = nullptr;
  // per-iteration Arnoldi results copied to pinned host memory, two slots (one iteration may be
  // enqueued ahead of the host's reading of the previous one), each with its completion event
  double* hpin = nullptr;
  hipEvent_t hev[2] = {};
  double *bvec = nullptr, *xvec = nullptr;
  double t_setup = 0.0;
  // preconditioner apply captured as a HIP graph (on cap_st, into the staging vectors gin/gout)
  hipStream_t cap_st = nullptr;
  hipGraphExec_t pgraph = nullptr;
  double *gin = nullptr, *gout = nullptr;
  // learned correction (optional)
  std::unique_ptr<Learned> learned;
  int learned_used = 0, fell_back = 0;
  double learned_red = 1.0;  // residual reduction of the learned correction's first application
  std::vector<double> history;  // relative residual estimate after each FGMRES iteration
  ~Solver();
};

Solver* solver_create(const Mesh& m, const double* mu_q, const double* mu_nodes, const wb_opts& o,
                      hipStream_t st);

template <typename T>
void apply_wbfbt(Solver& s, Precond<T>& P, const T* r, T* z);
template <typename T>
void apply_vcycle_A(Solver& s, Precond<T>& P, const T* r, T* z);
template <typename T>
void apply_K(Solver& s, Precond<T>& P, int side, const T* p, T* y);
template <typename T>
void apply_vcycle_K(Solver& s, Precond<T>& P, int side, const T* r, T* z);
template <typename T>
void apply_precond(Solver& s, Precond<T>& P, const T* ru, const T* rp, T* zu, T* zp);

// Preconditioner in the solver's configured precision, FP64 in and out.
void apply_precond_any(Solver& s, const double* ru, const double* rp, double* zu, double* zp);

wb_status fgmres(Solver& s, const double* f, double* u, double* p, wb_report* rep);
// GMRES on one block with its V-cycle: which = 0 (A u = f), 1 (K_l p = g), 2 (K_r p = g).
wb_status subsolve(Solver& s, int which, const double* b, double* x, wb_report* rep);

// Training of the learned coarse correction on seeded sinker fields (centers of field f at
// centers + 3 * sum_{g<f} n_sinkers[g]); see wb_learned_train.
struct TrainOpts {
  int pairs_per_field = 8, vcycles = 1, epochs = 20, batch = 8;
  double lr = 1e-3;
  unsigned long long seed = 1000;
  double delta = 200, omega = 0.1, mu_min = 1e-3, mu_max = 1e3;
  int n_valid = 0;  // trailing fields held out for the validation loss
};
struct TrainReport {
  double loss_first = 0, loss_last = 0, valid_loss = 0;
  double t_pairs_s = 0, t_train_s = 0;
  long long n_params = 0;
  int n_pairs = 0;
};
void learned_train(Solver& s, int n_fields, const int* n_sinkers, const double* centers,
                   const TrainOpts& o, TrainReport* rep);
// Guarded correction at level lc for a given residual r (FP64): delta and alpha, no update.
void learned_probe(Solver& s, const double* r, double* delta, double* alpha_host);
// Replace the parameters (device copy from host) and mark the network trained.
void learned_set(Solver& s, const float* params_host);

// host helpers
double dot_host(Solver& s, size_t n, const double* x, const double* y);

}  // namespace wb
