// Hierarchy setup, V-cycles, w-BFBT apply (eq. 8, Sec. 5), block preconditioner (eq. 3) and
// flexible GMRES.  Host code orchestrating the kernels of kernels.hip on one stream.
#include <algorithm>
#include <chrono>
#include <cmath>
#include <cstdio>
#include <cstring>
#include <map>
#include <mutex>
#include <thread>
#include <exception>

#include "solver.h"

namespace wb {

// ------------------------------------------------------------------ arena
// Device blocks released by destroyed arenas are kept per (device, size) and handed to the next
// request of the same size, so that creating solvers of one mesh again and again (a time step
// loop, a benchmark) does not pay hipMalloc / hipFree each time.  An allocation failure empties
// the cache and retries; mem_trim() empties it on request.
namespace {
std::mutex g_pool_mu;
std::multimap<std::pair<int, size_t>, void*> g_pool;

void pool_trim_locked() {
  for (auto& kv : g_pool) {
    int cur = 0;
    (void)hipGetDevice(&cur);
    (void)hipSetDevice(kv.first.first);
    (void)hipFree(kv.second);
    (void)hipSetDevice(cur);
  }
  g_pool.clear();
}
}  // namespace

void mem_trim() {
  std::lock_guard<std::mutex> g(g_pool_mu);
  pool_trim_locked();
}

// Device copies of host-built constant tables (coefficient coarsening matrices, transfer rows,
// the reference divergence).  They depend only on the mesh sizes and orders, so each content is
// uploaded once per device and kept for the process (a few KB each): solver setup then issues no
// blocking host-to-device copies for them.
namespace {
std::mutex g_tab_mu;
std::map<std::string, void*> g_tab;
}  // namespace

const void* const_table(const void* host, size_t bytes) {
  int dev = 0;
  WB_HIP(hipGetDevice(&dev));
  std::string key(reinterpret_cast<const char*>(&dev), sizeof(dev));
  key.append(reinterpret_cast<const char*>(host), bytes);
  std::lock_guard<std::mutex> g(g_tab_mu);
  auto it = g_tab.find(key);
  if (it != g_tab.end()) return it->second;
  void* d = nullptr;
  WB_HIP(hipMalloc(&d, std::max<size_t>(bytes, 8)));
  WB_HIP(hipMemcpy(d, host, bytes, hipMemcpyHostToDevice));
  g_tab.emplace(std::move(key), d);
  return d;
}
template <typename T>
const T* const_table(const std::vector<T>& v) {
  return static_cast<const T*>(const_table(v.data(), sizeof(T) * v.size()));
}

Arena::~Arena() {
  if (ptrs_.empty()) return;
  // queued work on these blocks ends before they can be handed out again (hipFree waited too)
  (void)hipDeviceSynchronize();
  std::lock_guard<std::mutex> g(g_pool_mu);
  for (size_t i = 0; i < ptrs_.size(); ++i) g_pool.emplace(std::make_pair(dev_, sizes_[i]), ptrs_[i]);
}

void* Arena::raw(size_t bytes) {
  bytes = (std::max<size_t>(bytes, 8) + 255) & ~(size_t)255;
  int dev = 0;
  WB_HIP(hipGetDevice(&dev));
  if (ptrs_.empty()) dev_ = dev;
  WB_REQUIRE(dev == dev_, WB_EINVAL, "one arena serves one device");
  void* p = nullptr;
  {
    std::lock_guard<std::mutex> g(g_pool_mu);
    auto it = g_pool.find(std::make_pair(dev, bytes));
    if (it != g_pool.end()) {
      p = it->second;
      g_pool.erase(it);
    }
  }
  if (!p) {
    hipError_t e = hipMalloc(&p, bytes);
    if (e != hipSuccess) {
      (void)hipGetLastError();
      mem_trim();
      e = hipMalloc(&p, bytes);
    }
    if (e != hipSuccess)
      throw Error{WB_ENOMEM, "hipMalloc of " + std::to_string(bytes) + " bytes failed"};
  }
  ptrs_.push_back(p);
  sizes_.push_back(bytes);
  bytes_ += bytes;
  return p;
}

std::vector<std::pair<int, int>> level_schedule(int N, int k, int p_schedule) {
  std::vector<std::pair<int, int>> out{{N, k}};
  while (k > 1) {
    k = p_schedule == 1 ? k - 1 : std::max(1, k / 2);
    out.push_back({N, k});
  }
  while (N % 2 == 0 && N / 2 >= 4) {
    N /= 2;
    out.push_back({N, k});
  }
  return out;
}

namespace {

double now_s() {
  return std::chrono::duration<double>(std::chrono::steady_clock::now().time_since_epoch()).count();
}

// ---------------------------------------------------------------- host linear algebra
// In-place inverse of an SPD matrix (n small): Cholesky A = L L^T, W = L^-1 by forward
// substitution, A^-1 = W^T W accumulated row by row of W (all inner loops contiguous).
void spd_inverse(std::vector<double>& A, int n) {
  std::vector<double> Lm(A);
  for (int j = 0; j < n; ++j) {
    double s = Lm[(size_t)j * n + j];
    for (int p = 0; p < j; ++p) s -= Lm[(size_t)j * n + p] * Lm[(size_t)j * n + p];
    if (!(s > 0.0)) throw Error{WB_ENAN, "coarse operator is not positive definite"};
    const double d = std::sqrt(s);
    Lm[(size_t)j * n + j] = d;
    for (int i = j + 1; i < n; ++i) {
      double t = Lm[(size_t)i * n + j];
      for (int p = 0; p < j; ++p) t -= Lm[(size_t)i * n + p] * Lm[(size_t)j * n + p];
      Lm[(size_t)i * n + j] = t / d;
    }
  }
  // W = L^-1 (lower triangular): row i from the rows above it
  std::vector<double> W((size_t)n * n, 0.0);
  for (int i = 0; i < n; ++i) {
    double* wi = &W[(size_t)i * n];
    wi[i] = 1.0;
    for (int p = 0; p < i; ++p) {
      const double l = Lm[(size_t)i * n + p];
      const double* wp = &W[(size_t)p * n];
      for (int c = 0; c <= p; ++c) wi[c] -= l * wp[c];
    }
    const double inv = 1.0 / Lm[(size_t)i * n + i];
    for (int c = 0; c <= i; ++c) wi[c] *= inv;
  }
  // A^-1 = W^T W: lower triangle by rank-one updates with the rows of W, then mirrored
  std::fill(A.begin(), A.end(), 0.0);
  for (int p = 0; p < n; ++p) {
    const double* wp = &W[(size_t)p * n];
    for (int i = 0; i <= p; ++i) {
      const double wi = wp[i];
      double* ai = &A[(size_t)i * n];
      for (int j = 0; j <= i; ++j) ai[j] += wi * wp[j];
    }
  }
  for (int i = 0; i < n; ++i)
    for (int j = 0; j < i; ++j) A[(size_t)j * n + i] = A[(size_t)i * n + j];
}

// Largest eigenvalue of a symmetric tridiagonal matrix (cyclic Jacobi on the dense form).
double tridiag_max_eig(const std::vector<double>& dg, const std::vector<double>& off) {
  const int m = (int)dg.size();
  std::vector<double> A(m * m, 0.0);
  for (int i = 0; i < m; ++i) {
    A[i * m + i] = dg[i];
    if (i + 1 < m) A[i * m + i + 1] = A[(i + 1) * m + i] = off[i];
  }
  for (int sweep = 0; sweep < 100; ++sweep) {
    double offn = 0.0;
    for (int p = 0; p < m; ++p)
      for (int q = p + 1; q < m; ++q) offn += A[p * m + q] * A[p * m + q];
    if (offn < 1e-30) break;
    for (int p = 0; p < m; ++p)
      for (int q = p + 1; q < m; ++q) {
        const double apq = A[p * m + q];
        if (std::fabs(apq) < 1e-300) continue;
        const double theta = (A[q * m + q] - A[p * m + p]) / (2.0 * apq);
        const double t = (theta >= 0 ? 1.0 : -1.0) / (std::fabs(theta) + std::sqrt(theta * theta + 1.0));
        const double c = 1.0 / std::sqrt(t * t + 1.0), s = t * c;
        for (int r = 0; r < m; ++r) {
          const double arp = A[r * m + p], arq = A[r * m + q];
          A[r * m + p] = c * arp - s * arq;
          A[r * m + q] = s * arp + c * arq;
        }
        for (int r = 0; r < m; ++r) {
          const double apr = A[p * m + r], aqr = A[q * m + r];
          A[p * m + r] = c * apr - s * aqr;
          A[q * m + r] = s * apr + c * aqr;
        }
      }
  }
  double mx = -1e300;
  for (int i = 0; i < m; ++i) mx = std::max(mx, A[i * m + i]);
  return mx;
}

// Counter-based splitmix64 uniform in [-1, 1): u_i = 2 U(mix(seed * 2^32 + i)) - 1.
void splitmix_vector(unsigned long long seed, size_t n, std::vector<double>& out) {
  out.resize(n);
  for (size_t i = 0; i < n; ++i) {
    unsigned long long z = (seed << 32) + (unsigned long long)i + 0x9E3779B97F4A7C15ULL;
    z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
    z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
    z = z ^ (z >> 31);
    out[i] = 2.0 * ((double)(z >> 11) * (1.0 / 9007199254740992.0)) - 1.0;
  }
}

// ---------------------------------------------------------------- 1D transfer tables
Rows1D upload_rows(const std::vector<std::vector<std::pair<int, double>>>& rows, int ncols) {
  int W = 1;
  for (auto& r : rows) W = std::max<int>(W, (int)r.size());
  const int R = (int)rows.size();
  std::vector<int> cnt(R), col((size_t)R * W, 0);
  std::vector<double> val((size_t)R * W, 0.0);
  for (int i = 0; i < R; ++i) {
    cnt[i] = (int)rows[i].size();
    for (int t = 0; t < cnt[i]; ++t) {
      col[(size_t)i * W + t] = rows[i][t].first;
      val[(size_t)i * W + t] = rows[i][t].second;
    }
  }
  Rows1D o;
  o.rows = R;
  o.cols = ncols;
  o.W = W;
  o.lin21 = 0;
  o.cnt = const_table(cnt);
  o.col = const_table(col);
  o.val = const_table(val);
  return o;
}

// P1[i_f][I_c]: coarse continuous 1D basis (Nc elements, order kc) at the fine nodes (Nf, kf).
void make_transfer(int Nc, int kc, int Nf, int kf, Rows1D& P, Rows1D& R) {
  const Tables& tf = tables(kf);
  const Tables& tc = tables(kc);
  const int Mf = kf * Nf + 1, Mc = kc * Nc + 1;
  std::vector<std::vector<std::pair<int, double>>> prow(Mf), rrow(Mc);
  for (int i = 0; i < Mf; ++i) {
    const int ef = std::min(i / kf, Nf - 1), a = i - ef * kf;
    const double x = (ef + 0.5 * (tf.xl[a] + 1.0)) / Nf;
    const int ec = std::min((int)std::floor(x * Nc + 1e-12), Nc - 1);
    const double xi = 2.0 * (x * Nc - ec) - 1.0;
    double V[NMAX];
    lagrange(kc + 1, tc.xl, 1, &xi, V, nullptr);
    for (int b = 0; b <= kc; ++b)
      if (std::fabs(V[b]) > 1e-14) prow[i].push_back({ec * kc + b, V[b]});
  }
  for (int i = 0; i < Mf; ++i)
    for (auto& cv : prow[i]) rrow[cv.first].push_back({i, cv.second});
  P = upload_rows(prow, Mc);
  R = upload_rows(rrow, Mf);
  bool lin = Mf == 2 * Mc - 1;
  for (int i = 0; lin && i < Mf; ++i) {
    const auto& r = prow[i];
    if (i % 2 == 0)
      lin = r.size() == 1 && r[0].first == i / 2 && std::fabs(r[0].second - 1.0) < 1e-13;
    else
      lin = r.size() == 2 && r[0].first == i / 2 && r[1].first == i / 2 + 1 &&
            std::fabs(r[0].second - 0.5) < 1e-13 && std::fabs(r[1].second - 0.5) < 1e-13;
  }
  P.lin21 = R.lin21 = lin ? 1 : 0;
}

// Coarsening matrix Q[qc][(s, qf)] of the L2 adjoint of element-wise interpolation.
std::vector<double> coarsen_matrix(int nf, int nc, int children) {
  const Tables& tf = tables(nf - 1);
  const Tables& tc = tables(nc - 1);
  const int W = children * nf;
  std::vector<double> Q((size_t)nc * W);
  for (int s = 0; s < children; ++s)
    for (int qf = 0; qf < nf; ++qf) {
      const double xi = children == 1 ? tf.xg[qf] : 0.5 * (tf.xg[qf] + 2 * s - 1);
      double V[NMAX];
      lagrange(nc, tc.xg, 1, &xi, V, nullptr);
      for (int qc = 0; qc < nc; ++qc)
        Q[(size_t)qc * W + s * nf + qf] = V[qc] * (tf.wg[qf] / children) / tc.wg[qc];
    }
  return Q;
}

// Reference divergence matrix without the (h/2)^2 factor: bhat[m][c][i] = -sum_q psi_m d_c phi_i w.
std::vector<double> make_bhat(int k) {
  const Tables& t = tables(k);
  const int n = k + 1, n3 = n * n * n;
  std::vector<double> bh((size_t)t.np * 3 * n3, 0.0);
  for (int m = 0; m < t.np; ++m)
    for (int li = 0; li < n3; ++li) {
      const int a = li % n, b = (li / n) % n, c = li / (n * n);
      double s[3] = {0, 0, 0};
      for (int qz = 0; qz < n; ++qz)
        for (int qy = 0; qy < n; ++qy)
          for (int qx = 0; qx < n; ++qx) {
            const double w = t.wg[qx] * t.wg[qy] * t.wg[qz];
            const double psi = t.L[t.ma[m] * n + qx] * t.L[t.mb[m] * n + qy] * t.L[t.mc[m] * n + qz];
            s[0] += w * psi * t.D1[qx * n + a] * t.B[qy * n + b] * t.B[qz * n + c];
            s[1] += w * psi * t.B[qx * n + a] * t.D1[qy * n + b] * t.B[qz * n + c];
            s[2] += w * psi * t.B[qx * n + a] * t.B[qy * n + b] * t.D1[qz * n + c];
          }
      for (int c3 = 0; c3 < 3; ++c3) bh[((size_t)m * 3 + c3) * n3 + li] = -s[c3];
    }
  return bh;
}

// Level operator: the assembled stencil where the level has one, else the element kernels
// (`extra` selects their BF16 contractions).
template <typename T>
void level_op(hipStream_t st, const Level<T>& L, const T* in, T* out, void* work, int extra = 0) {
  if (L.S) return launch_stencil_epi<T>(st, L.NC, L.N, L.S, in, out, false, Epi<T>{});
  launch_op<T>(st, (L.dir ? (F_A | F_DIR) : F_A) | extra, L.NC, L.N, L.k, in, out, L.coef, nullptr,
               nullptr, nullptr, false, work);
}

// The extra operator flags of the level operators of a preconditioner in type T: the BF16
// matrix-core contractions of the BF16 forms.
template <typename T>
inline int mf_flag(const Solver& s) {
  if (sizeof(T) != 4) return 0;
  if (s.o.precond_prec == WB_BF16) return F_MF3;
  if (s.o.precond_prec == WB_BF16X1) return F_MF;
  return 0;
}

// Level operator with an output epilogue (see Epi): the Chebyshev updates and residuals of the
// V-cycle are applied to each node value as the operator finishes it.
template <typename T>
void level_op_epi(Solver& s, const Level<T>& L, const T* in, const Epi<T>& e) {
  if (L.S) return launch_stencil_epi<T>(s.st, L.NC, L.N, L.S, in, nullptr, false, e);
  launch_op_epi<T>(s.st, (L.dir ? (F_A | F_DIR) : F_A) | mf_flag<T>(s), L.NC, L.N, L.k, in, nullptr,
                   L.coef, nullptr, nullptr, nullptr, false, s.opwork, e);
}

// Q1 levels are assembled into 27-point stencils when the stencil fits the size limit
// (assemble_mb); the coarsest level always is (its dense inverse is built from the stencil).
bool assembles(const Solver& s, int NC, int N, int k, bool coarsest) {
  if (k != 1) return false;
  return coarsest || 8.0 * (double)q1_stencil_len(NC, N) <= s.o.assemble_mb * 1e6;
}

// (Re)build the stencil of an assembled level from its current coefficient.
void assemble_level(Solver& s, Level<double>& L) {
  const size_t need = q1_elem_matrix_len(L.NC, L.N);
  if (s.ae_len < need) {
    s.ae = s.arena.alloc<double>(need);
    s.ae_len = need;
  }
  assemble_q1(s.st, L.NC, L.N, L.dir, L.coef, s.ae, L.S);
}

// Chebyshev-accelerated Jacobi (degree steps) on a level, operator and update fused: the
// search directions alternate between L.d and L.t (the operator reads one while its epilogue
// writes the other); with x0 != 0 the first correction is added to x by the next step.
template <typename T>
void cheb_level(Solver& s, Level<T>& L, const T* b, T* x, bool xzero) {
  hipStream_t st = s.st;
  const double theta = 0.5 * (L.lmax + L.lmin), delta = 0.5 * (L.lmax - L.lmin);
  const double sigma = theta / delta;
  double rho = 1.0 / sigma;
  T* d0 = L.d;
  T* d1 = L.t;
  bool pending = false;
  int it = 1;
  if (xzero && s.o.cheb_degree >= 2) {
    // the first two steps in one operator apply (EPI_CHEB_ZERO): d0 is formed as it is read
    const double rho_new = 1.0 / (2.0 * sigma - rho);
    Epi<T> e;
    e.mode = EPI_CHEB_ZERO;
    e.b = b;
    e.r = L.r;
    e.dnew = d1;
    e.x = x;
    e.dinv = L.dinv;
    e.gamma = (T)(1.0 / theta);
    e.alpha = (T)(rho_new * rho);
    e.beta = (T)(2.0 * rho_new / delta);
    level_op_epi<T>(s, L, nullptr, e);
    std::swap(d0, d1);
    rho = rho_new;
    it = 2;
  } else if (xzero) {
    launch_cheb_first<T>(st, L.len, b, nullptr, L.dinv, (T)(1.0 / theta), d0, x, L.r, true);
  } else {
    Epi<T> e;
    e.mode = EPI_CHEB_FIRST;
    e.b = b;
    e.r = L.r;
    e.dnew = d0;
    e.dinv = L.dinv;
    e.alpha = (T)(1.0 / theta);
    level_op_epi<T>(s, L, x, e);
    pending = true;
  }
  for (; it < s.o.cheb_degree; ++it) {
    const double rho_new = 1.0 / (2.0 * sigma - rho);
    Epi<T> e;
    e.mode = EPI_CHEB_STEP;
    e.add_old = pending ? 1 : 0;
    e.r = L.r;
    e.dold = d0;
    e.dnew = d1;
    e.x = x;
    e.dinv = L.dinv;
    e.alpha = (T)(rho_new * rho);
    e.beta = (T)(2.0 * rho_new / delta);
    level_op_epi<T>(s, L, d0, e);
    std::swap(d0, d1);
    pending = false;
    rho = rho_new;
  }
  if (pending) launch_axpby<T>(st, L.len, T(1), d0, T(1), x);
}

// Largest eigenvalue of D^-1 A from `steps` Jacobi-CG steps started from r (device, overwritten).
// The CG scalars stay in device memory, rz[0..steps] then pq[0..steps-1] at lz (2 steps + 1
// doubles); lanczos_finish turns them into the estimate once they are on the host.
template <typename Op>
void lanczos_enqueue(hipStream_t st, const Op& op, size_t len, const double* dinv, int steps,
                     double* r, double* z, double* p, double* q, double* lz, double* partial) {
  double* rz = lz;
  double* pq = lz + steps + 1;
  launch_mul<double>(st, len, dinv, r, z);
  WB_HIP(hipMemcpyAsync(p, z, sizeof(double) * len, hipMemcpyDeviceToDevice, st));
  launch_dot<double>(st, len, r, z, partial, rz);
  for (int it = 0; it < steps; ++it) {
    op(p, q);
    launch_dot<double>(st, len, p, q, partial, pq + it);
    launch_cg_r(st, len, q, dinv, r, z, rz + it, pq + it, partial, rz + it + 1);
    launch_cg_p(st, len, z, p, rz + it + 1, rz + it);
  }
}

double lanczos_finish(const double* h, int steps) {
  std::vector<double> alphas, betas;
  for (int it = 0; it < steps; ++it) {
    const double rzj = h[it], pqj = h[steps + 1 + it], rzn = h[it + 1];
    if (!(rzj > 0.0) || !(pqj > 0.0)) break;
    alphas.push_back(rzj / pqj);
    betas.push_back(rzn / rzj);
    if (!(rzn > 0.0)) break;
  }
  const int m = (int)alphas.size();
  WB_REQUIRE(m > 0, WB_ENAN, "eigenvalue estimate failed (zero operator?)");
  std::vector<double> dg(m), off(std::max(0, m - 1));
  for (int j = 0; j < m; ++j) {
    dg[j] = 1.0 / alphas[j] + (j > 0 ? betas[j - 1] / alphas[j - 1] : 0.0);
    if (j + 1 < m) off[j] = std::sqrt(betas[j]) / alphas[j];
  }
  return tridiag_max_eig(dg, off);
}

// Chebyshev interval [0.1, 1.1] * lambda_max(D^-1 A) of a level, lambda_max from Jacobi-CG
// (Lanczos) steps started from the splitmix64 vector of `seed` (Dirichlet entries zeroed, or
// the mean removed for the Neumann Poisson levels).  Enqueued on `st` with its own reduction
// scratch `partial` (RED_BLOCKS + 64 doubles) and face workspace `work`; the level's work vectors
// are zero again afterwards.
void cheb_bounds_enqueue(Solver& s, Level<double>& L, unsigned long long seed, hipStream_t st,
                         double* partial, void* work, double* lz) {
  const int M = L.k * L.N + 1;
  launch_splitmix_vec(st, L.len, seed, L.dir ? M : 0, L.x);
  if (!L.dir) launch_remove_global_mean(st, L.len, L.x, partial, partial + RED_BLOCKS + 32);
  auto op = [&](const double* in, double* out) { level_op<double>(st, L, in, out, work); };
  lanczos_enqueue(st, op, L.len, L.dinv, s.o.lanczos_steps, L.x, L.b, L.r, L.d, lz, partial);
  for (double* v : {L.x, L.b, L.r, L.d, L.t}) launch_fill<double>(st, v, 0.0, L.len);
}

void set_bounds(Level<double>& L, double lam) {
  L.lmin = 0.1 * lam;
  L.lmax = 1.1 * lam;
}

// The same, finished at once (one host read).
void set_cheb_bounds(Solver& s, Level<double>& L, unsigned long long seed) {
  const int steps = s.o.lanczos_steps;
  cheb_bounds_enqueue(s, L, seed, s.st, s.red_partial, s.opwork, s.lz);
  std::vector<double> h(2 * steps + 1);
  WB_HIP(hipMemcpyAsync(h.data(), s.lz, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s.st));
  WB_HIP(hipStreamSynchronize(s.st));
  set_bounds(L, lanczos_finish(h.data(), steps));
}

// Deferred eigenvalue estimates of a solver setup: each smoothed level's recurrence runs on one
// of the auxiliary streams (round robin; the levels are independent and their launches small),
// its scalars in its own slice of s.lz; finish_setup_estimates reads them all at once.
struct SetupEstimates {
  struct Job {
    double* lmin;
    double* lmax;
    size_t slice;
  };
  std::vector<Job> jobs;
  int next = 0;
};

size_t lz_slice(const Solver& s) { return (size_t)2 * s.o.lanczos_steps + 1; }

double* next_lz(Solver& s, SetupEstimates& E, double* lmin, double* lmax) {
  const size_t slice = E.jobs.size() * lz_slice(s);
  WB_REQUIRE(slice + lz_slice(s) <= (size_t)LZ_SLOTS, WB_EINVAL, "lanczos_steps out of range");
  E.jobs.push_back({lmin, lmax, slice});
  return s.lz + slice;
}

void enqueue_level_bounds(Solver& s, SetupEstimates& E, Level<double>& L, unsigned long long seed) {
  const int k = E.next++ % AUX_STREAMS;
  WB_HIP(hipStreamWaitEvent(s.aux[k], s.main_ev, 0));
  double* lz = next_lz(s, E, &L.lmin, &L.lmax);
  cheb_bounds_enqueue(s, L, seed, s.aux[k], s.aux_partial[k], s.aux_work[k], lz);
}

// Joins the auxiliary streams into s.st and enqueues the read of every pending estimate into h.
void join_setup_estimates(Solver& s, const SetupEstimates& E, std::vector<double>& h) {
  for (int k = 0; k < AUX_STREAMS; ++k) {
    WB_HIP(hipEventRecord(s.aux_ev[k], s.aux[k]));
    WB_HIP(hipStreamWaitEvent(s.st, s.aux_ev[k], 0));
  }
  h.assign(E.jobs.size() * lz_slice(s), 0.0);
  if (!h.empty())
    WB_HIP(hipMemcpyAsync(h.data(), s.lz, sizeof(double) * h.size(), hipMemcpyDeviceToHost, s.st));
}

// After the stream has been synchronized: the Chebyshev intervals from the estimates in h.
void finish_setup_estimates(const Solver& s, const SetupEstimates& E, const std::vector<double>& h) {
  for (const auto& j : E.jobs) {
    const double lam = lanczos_finish(h.data() + j.slice, s.o.lanczos_steps);
    *j.lmin = 0.1 * lam;
    *j.lmax = 1.1 * lam;
  }
}

// Build an FP64 hierarchy on `coef0` (velocity if NC == 3, Poisson if NC == 1).  The
// eigenvalue estimates of its smoothed levels are enqueued into E; the coarsest inverse is
// formed by coarsest_inverse once its stencil is on the host.
void build_hierarchy(Solver& s, Hierarchy<double>& H, int NC, const double* coef0, int seed_base,
                     SetupEstimates& E) {
  hipStream_t st = s.st;
  Arena& ar = s.arena;
  auto sched = level_schedule(s.m.N, s.m.k, s.o.p_schedule);
  const int nl = (int)sched.size();
  H.L.resize(nl);
  for (int li = 0; li < nl; ++li) {
    Level<double>& L = H.L[li];
    L.N = sched[li].first;
    L.k = sched[li].second;
    L.NC = NC;
    L.dir = NC == 3;
    const int M = L.k * L.N + 1, n = L.k + 1;
    L.nn = M * M * M;
    L.E = L.N * L.N * L.N;
    L.len = (size_t)NC * L.nn;
    const size_t ncoef = (size_t)L.E * n * n * n;
    L.coef = ar.alloc<double>(ncoef);
    if (li == 0) {
      WB_HIP(hipMemcpyAsync(L.coef, coef0, sizeof(double) * ncoef, hipMemcpyDeviceToDevice, st));
    } else {
      const Level<double>& F = H.L[li - 1];
      if (F.N == L.N) {
        L.Q = const_table(coarsen_matrix(F.k + 1, n, 1));
        launch_coarsen_p(st, L.E, F.k + 1, n, L.Q, F.coef, L.coef);
      } else {
        L.Q = const_table(coarsen_matrix(n, n, 2));
        launch_coarsen_h(st, F.N, n, L.Q, F.coef, L.coef);
      }
    }
    L.dinv = ar.alloc<double>(L.len);
    launch_fill<double>(st, L.dinv, 0.0, L.len);
    launch_diag(st, NC, L.N, L.k, L.dir, L.coef, L.dinv);
    launch_invert_diag(st, NC, L.N, L.k, L.dir, L.dinv);
    if (assembles(s, NC, L.N, L.k, li + 1 == nl)) {
      L.S = ar.alloc<double>(q1_stencil_len(NC, L.N));
      assemble_level(s, L);
    }
    L.x = ar.alloc<double>(L.len);
    L.b = ar.alloc<double>(L.len);
    L.r = ar.alloc<double>(L.len);
    L.d = ar.alloc<double>(L.len);
    L.t = ar.alloc<double>(L.len);
    for (double* v : {L.x, L.b, L.r, L.d, L.t}) launch_fill<double>(st, v, 0.0, L.len);
    if (li > 0) make_transfer(L.N, L.k, H.L[li - 1].N, H.L[li - 1].k, H.L[li - 1].P, H.L[li - 1].R);
  }
  // Chebyshev bounds from the Lanczos estimate on every smoothed level
  WB_HIP(hipEventRecord(s.main_ev, st));
  for (int li = 0; li + 1 < nl; ++li)
    enqueue_level_bounds(s, E, H.L[li], (unsigned long long)(seed_base + li));
  Level<double>& C = H.L[nl - 1];
  WB_REQUIRE(C.S != nullptr, WB_EUNSUPPORTED, "coarsest level is not Q1");
}

// Coarsest level: dense inverse (velocity: interior DOFs, SPD) or pseudo-inverse (Poisson,
// Neumann), from its stencil Sh (host copy); coarsest_upload puts it on the device.
struct CoarseDense {
  std::vector<double> G;  // [nd][nd]
  std::vector<int> idx;   // level DOF of row r
};

// Host part, touching no device state (the three hierarchies' inverses run on host threads).
CoarseDense coarsest_dense(const Level<double>& C, const std::vector<double>& Sh) {
  const int NC = C.NC;
  const int M = C.k * C.N + 1;
  std::vector<int> idx;
  for (size_t i = 0; i < C.len; ++i) {
    const size_t g = i % C.nn;
    const int gi = (int)(g % M), gj = (int)((g / M) % M), gl = (int)(g / ((size_t)M * M));
    const bool bnd = gi == 0 || gi == M - 1 || gj == 0 || gj == M - 1 || gl == 0 || gl == M - 1;
    if (!C.dir || !bnd) idx.push_back((int)i);
  }
  const int nd = (int)idx.size();
  std::vector<double> Ad((size_t)nd * nd, 0.0);
  std::vector<int> pos(C.len, -1);
  for (int i = 0; i < nd; ++i) pos[idx[i]] = i;
  for (int i = 0; i < nd; ++i) {
    const int c = (int)(idx[i] / C.nn), g = (int)(idx[i] % C.nn);
    const int gx = g % M, gy = (g / M) % M, gz = g / (M * M);
    for (int o = 0; o < 27; ++o) {
      const int jx = gx + o % 3 - 1, jy = gy + (o / 3) % 3 - 1, jz = gz + o / 9 - 1;
      if (jx < 0 || jx >= M || jy < 0 || jy >= M || jz < 0 || jz >= M) continue;
      const int j = jx + M * (jy + M * jz);
      for (int d = 0; d < NC; ++d) {
        const int pj = pos[(size_t)d * C.nn + j];
        if (pj >= 0) Ad[(size_t)i * nd + pj] += Sh[((size_t)(o * NC + c) * NC + d) * C.nn + g];
      }
    }
  }
  for (int i = 0; i < nd; ++i)
    for (int j = i + 1; j < nd; ++j) {
      const double a = 0.5 * (Ad[(size_t)i * nd + j] + Ad[(size_t)j * nd + i]);
      Ad[(size_t)i * nd + j] = Ad[(size_t)j * nd + i] = a;
    }
  if (C.dir) {
    spd_inverse(Ad, nd);
  } else {
    double c = 0.0;
    for (int i = 0; i < nd; ++i) c += Ad[(size_t)i * nd + i];
    c /= nd;
    for (auto& v : Ad) v += c;
    spd_inverse(Ad, nd);
    // G = Pi (L + c 1 1^T)^-1 Pi, Pi = I - 1 1^T / nd
    std::vector<double> rm(nd, 0.0), cm(nd, 0.0);
    double tm = 0.0;
    for (int i = 0; i < nd; ++i)
      for (int j = 0; j < nd; ++j) {
        rm[i] += Ad[(size_t)i * nd + j] / nd;
        cm[j] += Ad[(size_t)i * nd + j] / nd;
        tm += Ad[(size_t)i * nd + j] / ((double)nd * nd);
      }
    for (int i = 0; i < nd; ++i)
      for (int j = 0; j < nd; ++j) Ad[(size_t)i * nd + j] += -rm[i] - cm[j] + tm;
  }
  return CoarseDense{std::move(Ad), std::move(idx)};
}

void coarsest_upload(Solver& s, Hierarchy<double>& H, CoarseDense&& cd,
                     std::vector<std::vector<double>>& keep_d, std::vector<std::vector<int>>& keep_i) {
  hipStream_t st = s.st;
  Arena& ar = s.arena;
  Level<double>& C = H.L.back();
  const int nd = (int)cd.idx.size();
  H.nd = nd;
  H.G = ar.alloc<double>((size_t)nd * nd);
  H.gidx = ar.alloc<int>(nd);
  // the host buffers stay alive (keep_*) until the caller has synchronized the stream
  keep_d.push_back(std::move(cd.G));
  keep_i.push_back(std::move(cd.idx));
  WB_HIP(hipMemcpyAsync(H.G, keep_d.back().data(), sizeof(double) * keep_d.back().size(),
                        hipMemcpyHostToDevice, st));
  WB_HIP(hipMemcpyAsync(H.gidx, keep_i.back().data(), sizeof(int) * nd, hipMemcpyHostToDevice, st));
  launch_fill<double>(st, C.x, 0.0, C.len);
  launch_fill<double>(st, C.t, 0.0, C.len);
}

// FP32 copy of an FP64 hierarchy (coefficients and diagonals cast; transfers and the FP64
// coarsest inverse shared).
void cast_hierarchy(Solver& s, const Hierarchy<double>& Hd, Hierarchy<float>& Hf) {
  hipStream_t st = s.st;
  Arena& ar = s.arena;
  Hf.L.resize(Hd.L.size());
  for (size_t li = 0; li < Hd.L.size(); ++li) {
    const Level<double>& D = Hd.L[li];
    Level<float>& L = Hf.L[li];
    L.N = D.N;
    L.k = D.k;
    L.NC = D.NC;
    L.dir = D.dir;
    L.nn = D.nn;
    L.E = D.E;
    L.len = D.len;
    L.lmin = D.lmin;
    L.lmax = D.lmax;
    L.P = D.P;
    L.R = D.R;
    const size_t ncoef = (size_t)D.E * (D.k + 1) * (D.k + 1) * (D.k + 1);
    L.coef = ar.alloc<float>(ncoef);
    launch_cast<double, float>(st, ncoef, D.coef, L.coef);
    L.dinv = ar.alloc<float>(L.len);
    launch_cast<double, float>(st, L.len, D.dinv, L.dinv);
    if (D.S) {
      const size_t ns = q1_stencil_len(D.NC, D.N);
      L.S = ar.alloc<float>(ns);
      launch_cast<double, float>(st, ns, D.S, L.S);
    }
    L.x = ar.alloc<float>(L.len);
    L.b = ar.alloc<float>(L.len);
    L.r = ar.alloc<float>(L.len);
    L.d = ar.alloc<float>(L.len);
    L.t = ar.alloc<float>(L.len);
    for (float* v : {L.x, L.b, L.r, L.d, L.t}) launch_fill<float>(st, v, 0.0f, L.len);
  }
  Hf.nd = Hd.nd;
  Hf.G = Hd.G;
  Hf.gidx = Hd.gidx;
}

template <typename T>
void alloc_work(Solver& s, Precond<T>& P) {
  Arena& ar = s.arena;
  const size_t vl = (size_t)3 * s.m.nn, pl = (size_t)s.m.E * s.m.np;
  for (T** v : {&P.v1, &P.v2, &P.vt}) *v = ar.alloc<T>(vl);
  for (T** v : {&P.pb, &P.px, &P.pr, &P.pd, &P.pt, &P.pm, &P.py}) *v = ar.alloc<T>(pl);
  P.cin_u = ar.alloc<T>(vl);
  P.cout_u = ar.alloc<T>(vl);
  P.cin_p = ar.alloc<T>(pl);
  P.cout_p = ar.alloc<T>(pl);
}

}  // namespace

double dot_host(Solver& s, size_t n, const double* x, const double* y) {
  launch_dot<double>(s.st, n, x, y, s.red_partial, s.red_out);
  double v = 0.0;
  WB_HIP(hipMemcpyAsync(&v, s.red_out, sizeof(double), hipMemcpyDeviceToHost, s.st));
  WB_HIP(hipStreamSynchronize(s.st));
  return v;
}

// ------------------------------------------------------------------ applies
// Learned coarse correction at the velocity level lc, in place of the recursion below it: from
// the residual r = b - A x after pre-smoothing, delta = rho N(feat, r / rho) / diag(A) and
// x += alpha delta with the residual-minimizing alpha clipped to [0, 2].  Device-side only; the
// dots (r, r), (r, A delta), (A delta, A delta) stay in red_out[8..10] for the acceptance check.
template <typename T>
void learned_delta(Solver& s, Level<T>& L, const T* r, T* delta, T* Ad) {
  Learned& G = *s.learned;
  hipStream_t st = s.st;
  double* sumsq = s.red_out + 8;
  launch_dot<T>(st, L.len, r, r, s.red_partial, sumsq);
  launch_net_input<T>(st, G.M, 1, G.feat, r, sumsq, G.xin);
  net_forward(st, G.params, G.xin, G.w1);
  launch_net_delta<T>(st, G.M, G.w1.z[3], L.dinv, sumsq, delta);
  level_op<T>(st, L, delta, Ad, s.opwork, mf_flag<T>(s));
  launch_dot<T>(st, L.len, r, Ad, s.red_partial, s.red_out + 9);
  launch_dot<T>(st, L.len, Ad, Ad, s.red_partial, s.red_out + 10);
}


// The last smoothed level of a scalar hierarchy and the coarsest solve run as one workgroup when
// the level is an assembled Q1 level small enough for it (see launch_vcycle_tail).
template <typename T>
bool vcycle_tail(Solver& s, Hierarchy<T>& H, int li, const T* b, T* x) {
  const Level<T>& L = H.L[li];
  if (li + 2 != (int)H.L.size() || !L.S || L.NC != 1 || L.dir || !L.R.lin21) return false;
  const Level<T>& C = H.L[li + 1];
  const int M = L.N + 1, Mc = C.N + 1;
  if (M * M * M > TAIL_MAX || H.nd != Mc * Mc * Mc || s.o.cheb_degree > TAIL_MAXDEG) return false;
  TailArgs<T> a;
  a.M = M;
  a.Mc = Mc;
  a.nd = H.nd;
  a.deg = s.o.cheb_degree;
  a.S = L.S;
  a.dinv = L.dinv;
  a.G = H.G;
  a.gidx = H.gidx;
  const double theta = 0.5 * (L.lmax + L.lmin), delta = 0.5 * (L.lmax - L.lmin);
  const double sigma = theta / delta;
  double rho = 1.0 / sigma;
  a.inv_theta = (T)(1.0 / theta);
  for (int it = 1; it < a.deg; ++it) {
    const double rho_new = 1.0 / (2.0 * sigma - rho);
    a.alpha[it] = (T)(rho_new * rho);
    a.beta[it] = (T)(2.0 * rho_new / delta);
    rho = rho_new;
  }
  launch_vcycle_tail<T>(s.st, a, b, x);
  return true;
}

template <typename T>
void vcycle(Solver& s, Hierarchy<T>& H, int li, const T* b, T* x) {
  hipStream_t st = s.st;
  Level<T>& L = H.L[li];
  if (li + 1 == (int)H.L.size()) {
    if (L.dir) launch_fill<T>(st, x, T(0), L.len);
    launch_dense<T>(st, H.nd, H.G, H.gidx, b, x);
    return;
  }
  if (vcycle_tail<T>(s, H, li, b, x)) return;
  cheb_level<T>(s, L, b, x, true);
  Epi<T> res;  // r = b - A x
  res.mode = EPI_RESID;
  res.b = b;
  res.r = L.r;
  level_op_epi<T>(s, L, x, res);
  if (L.NC == 3 && s.learned && li == s.learned->lc && s.learned->trained && s.learned->active &&
      s.o.use_learned) {
    learned_delta<T>(s, L, L.r, L.d, L.t);
    launch_net_guarded_update<T>(st, L.len, s.red_out + 9, x, L.d, s.learned->counters);
  } else {
    Level<T>& C = H.L[li + 1];
    launch_kron<T>(st, L.R, L.NC, C.dir, false, L.r, C.b);
    vcycle<T>(s, H, li + 1, C.b, C.x);
    launch_kron<T>(st, L.P, L.NC, L.dir, true, C.x, x);
  }
  cheb_level<T>(s, L, b, x, false);
}

template <typename T>
const T* fine_mu(Solver& s, Precond<T>& P) {
  return P.A.L[0].coef;
}

// The weight inverse of `side` as the operators' per-node input scaling; with one weight per
// velocity DOF (diag(A)-BFBT) the vector v is scaled here instead and no node scaling is used.
template <typename T>
const T* weight_scaling(Solver& s, Precond<T>& P, int side, T* v) {
  if (s.o.weights != 2) return P.winv[side];
  launch_mul<T>(s.st, (size_t)3 * s.m.nn, P.winv[side], v, v);
  return nullptr;
}

template <typename T>
void apply_K(Solver& s, Precond<T>& P, int side, const T* p, T* y) {
  hipStream_t st = s.st;
  const Mesh& m = s.m;
  launch_op<T>(st, F_BT | F_DIR | mf_flag<T>(s), 3, m.N, m.k, nullptr, P.vt, nullptr, p, nullptr,
               nullptr, false, s.opwork);
  const T* sc = weight_scaling<T>(s, P, side, P.vt);
  launch_op<T>(st, F_B | F_DIR | mf_flag<T>(s), 3, m.N, m.k, P.vt, nullptr, nullptr, nullptr, y, sc,
               false, nullptr);
}

// K_w p with an epilogue on the divergence kernel's output (see Epi).
template <typename T>
void apply_K_epi(Solver& s, Precond<T>& P, int side, const T* p, const Epi<T>& e) {
  hipStream_t st = s.st;
  const Mesh& m = s.m;
  launch_op<T>(st, F_BT | F_DIR | mf_flag<T>(s), 3, m.N, m.k, nullptr, P.vt, nullptr, p, nullptr,
               nullptr, false, s.opwork);
  const T* sc = weight_scaling<T>(s, P, side, P.vt);
  launch_op_epi<T>(st, F_B | F_DIR | mf_flag<T>(s), 3, m.N, m.k, P.vt, nullptr, nullptr, nullptr,
                   nullptr, sc, false, nullptr, e);
}

// Chebyshev-Jacobi on K_w (degree steps, diagonal dk), the updates fused into the divergence
// kernel as in cheb_level; directions alternate between P.pd and P.pt, residual in P.pr.
template <typename T>
void cheb_K(Solver& s, Precond<T>& P, int side, const T* b, T* x, bool xzero) {
  hipStream_t st = s.st;
  const size_t pl = (size_t)s.m.E * s.m.np;
  const double lmin = P.klmin[side], lmax = P.klmax[side];
  const double theta = 0.5 * (lmax + lmin), delta = 0.5 * (lmax - lmin), sigma = theta / delta;
  double rho = 1.0 / sigma;
  T* d0 = P.pd;
  T* d1 = P.pt;
  bool pending = false;
  if (xzero) {
    launch_cheb_first<T>(st, pl, b, nullptr, P.dk[side], (T)(1.0 / theta), d0, x, P.pr, true);
  } else {
    Epi<T> e;
    e.mode = EPI_CHEB_FIRST;
    e.b = b;
    e.r = P.pr;
    e.dnew = d0;
    e.dinv = P.dk[side];
    e.alpha = (T)(1.0 / theta);
    apply_K_epi<T>(s, P, side, x, e);
    pending = true;
  }
  for (int it = 1; it < s.o.cheb_degree; ++it) {
    const double rho_new = 1.0 / (2.0 * sigma - rho);
    Epi<T> e;
    e.mode = EPI_CHEB_STEP;
    e.add_old = pending ? 1 : 0;
    e.r = P.pr;
    e.dold = d0;
    e.dnew = d1;
    e.x = x;
    e.dinv = P.dk[side];
    e.alpha = (T)(rho_new * rho);
    e.beta = (T)(2.0 * rho_new / delta);
    apply_K_epi<T>(s, P, side, d0, e);
    std::swap(d0, d1);
    pending = false;
    rho = rho_new;
  }
  if (pending) launch_axpby<T>(st, pl, T(1), d0, T(1), x);
}

// mean_out = false skips the final mean removal, for an output that only B^T reads (B^T with the
// Dirichlet mask maps a constant pressure to zero).
template <typename T>
void apply_vcycle_K(Solver& s, Precond<T>& P, int side, const T* b, T* x, bool mean_out) {
  hipStream_t st = s.st;
  const Mesh& m = s.m;
  cheb_K<T>(s, P, side, b, x, true);
  Epi<T> res;  // r = b - K_w x
  res.mode = EPI_RESID;
  res.b = b;
  res.r = P.pr;
  apply_K_epi<T>(s, P, side, x, res);
  Hierarchy<T>& H = P.Pois[side];
  Level<T>& L0 = H.L[0];
  launch_modal_IT<T>(st, m.N, m.k, P.pr, L0.b);
  vcycle<T>(s, H, 0, L0.b, L0.x);
  launch_modal_I<T>(st, m.N, m.k, L0.x, x, true);
  cheb_K<T>(s, P, side, b, x, false);
  if (mean_out) launch_remove_mean<T>(st, m.E, m.np, x, s.red_partial, s.red_out + 1);
}

template <typename T>
void apply_vcycle_K(Solver& s, Precond<T>& P, int side, const T* b, T* x) {
  apply_vcycle_K<T>(s, P, side, b, x, true);
}

template <typename T>
void apply_wbfbt(Solver& s, Precond<T>& P, const T* r, T* z) {
  hipStream_t st = s.st;
  const Mesh& m = s.m;
  const size_t pl = (size_t)m.E * m.np, vl = (size_t)3 * m.nn;
  WB_HIP(hipMemcpyAsync(P.pb, r, sizeof(T) * pl, hipMemcpyDeviceToDevice, st));
  launch_remove_mean<T>(st, m.E, m.np, P.pb, s.red_partial, s.red_out + 2);
  apply_vcycle_K<T>(s, P, 1, P.pb, P.py, false);
  // middle product B C^-1 A D^-1 B^T
  launch_op<T>(st, F_BT | F_DIR | mf_flag<T>(s), 3, m.N, m.k, nullptr, P.v1, nullptr, P.py, nullptr, nullptr, false,
               s.opwork);
  const T* sr = weight_scaling<T>(s, P, 1, P.v1);
  launch_op<T>(st, F_A | F_DIR | mf_flag<T>(s), 3, m.N, m.k, P.v1, P.v2, fine_mu(s, P), nullptr, nullptr, sr,
               false, s.opwork);
  const T* sl = weight_scaling<T>(s, P, 0, P.v2);
  // B of a velocity that vanishes on the boundary has zero mean (the integral of its divergence
  // is the boundary flux), so P.pm needs no mean removal
  launch_op<T>(st, F_B | F_DIR | mf_flag<T>(s), 3, m.N, m.k, P.v2, nullptr, nullptr, nullptr, P.pm, sl, false,
               nullptr);
  apply_vcycle_K<T>(s, P, 0, P.pm, z);
}

template <typename T>
void apply_vcycle_A(Solver& s, Precond<T>& P, const T* r, T* z) {
  vcycle<T>(s, P.A, 0, r, z);
}

template <typename T>
void apply_precond(Solver& s, Precond<T>& P, const T* ru, const T* rp, T* zu, T* zp) {
  hipStream_t st = s.st;
  const Mesh& m = s.m;
  const size_t vl = (size_t)3 * m.nn;
  // P = [[A~, B^T], [0, sign S~]] (eq. 3): zp = sign S~^-1 rp, zu = A~^-1 (ru - B^T zp), with
  // S~ the w-BFBT approximation (eq. 8) or the diagonalized M_p(1/mu) (eq. 4)
  if (s.o.schur_approx == 1) {
    launch_mul<T>(st, (size_t)m.E * m.np, P.mpinv, rp, zp);
    launch_remove_mean<T>(st, m.E, m.np, zp, s.red_partial, s.red_out + 2);
  } else {
    apply_wbfbt<T>(s, P, rp, zp);
  }
  if (s.o.schur_sign < 0) launch_scal<T>(st, (size_t)m.E * m.np, T(-1), zp, zp);
  launch_op<T>(st, F_BT | F_DIR | mf_flag<T>(s), 3, m.N, m.k, nullptr, P.v1, nullptr, zp, nullptr, nullptr, false,
               s.opwork);
  launch_sub<T>(st, vl, ru, P.v1, P.v2);
  apply_vcycle_A<T>(s, P, P.v2, zu);
}

template void apply_wbfbt<double>(Solver&, Precond<double>&, const double*, double*);
template void apply_wbfbt<float>(Solver&, Precond<float>&, const float*, float*);
template void apply_vcycle_A<double>(Solver&, Precond<double>&, const double*, double*);
template void apply_vcycle_A<float>(Solver&, Precond<float>&, const float*, float*);
template void apply_K<double>(Solver&, Precond<double>&, int, const double*, double*);
template void apply_K<float>(Solver&, Precond<float>&, int, const float*, float*);
template void apply_vcycle_K<double>(Solver&, Precond<double>&, int, const double*, double*);
template void apply_vcycle_K<float>(Solver&, Precond<float>&, int, const float*, float*);
template void apply_precond<double>(Solver&, Precond<double>&, const double*, const double*, double*,
                                    double*);
template void apply_precond<float>(Solver&, Precond<float>&, const float*, const float*, float*,
                                   float*);

void apply_precond_any(Solver& s, const double* ru, const double* rp, double* zu, double* zp) {
  if (s.o.precond_prec == WB_FP64) {
    apply_precond<double>(s, *s.pd, ru, rp, zu, zp);
    return;
  }
  Precond<float>& P = *s.pf;
  const size_t vl = (size_t)3 * s.m.nn, pl = (size_t)s.m.E * s.m.np;
  launch_cast<double, float>(s.st, vl, ru, P.cin_u);
  launch_cast<double, float>(s.st, pl, rp, P.cin_p);
  apply_precond<float>(s, P, P.cin_u, P.cin_p, P.cout_u, P.cout_p);
  launch_cast<float, double>(s.st, vl, P.cout_u, zu);
  launch_cast<float, double>(s.st, pl, P.cout_p, zp);
}

// ------------------------------------------------------------------ setup
Solver::~Solver() {
  if (pgraph) (void)hipGraphExecDestroy(pgraph);
  for (int b = 0; b < 2; ++b)
    if (hev[b]) (void)hipEventDestroy(hev[b]);
  if (hpin) (void)hipHostFree(hpin);
  if (cap_st) (void)hipStreamDestroy(cap_st);
  for (int k = 0; k < AUX_STREAMS; ++k) {
    if (aux_ev[k]) (void)hipEventDestroy(aux_ev[k]);
    if (aux[k]) (void)hipStreamDestroy(aux[k]);
  }
  if (main_ev) (void)hipEventDestroy(main_ev);
}

namespace {
// Setup phase timing (stderr, with opts.verbose): waits for the stream at each mark.
struct PhaseClock {
  bool on;
  hipStream_t st;
  double t;
  PhaseClock(bool v, hipStream_t s) : on(v), st(s), t(now_s()) {}
  void mark(const char* what) {
    if (!on) return;
    (void)hipStreamSynchronize(st);
    const double n = now_s();
    fprintf(stderr, "setup %-28s %8.3f ms\n", what, 1e3 * (n - t));
    t = n;
  }
};
}  // namespace

Solver* solver_create(const Mesh& m, const double* mu_q, const double* mu_nodes, const wb_opts& o,
                      hipStream_t st) {
  WB_REQUIRE(m.k >= 2 && m.k <= 5, WB_EUNSUPPORTED, "Stokes solves need 2 <= k <= 5");
  WB_REQUIRE(m.k <= 4 || o.precond_prec == WB_FP64 || o.precond_prec == WB_FP32, WB_EUNSUPPORTED,
             "the BF16 precision forms are built for k <= 4");
  WB_REQUIRE(o.cheb_degree >= 1 && o.restart >= 1 && o.max_iter >= 1 && o.rtol > 0, WB_EINVAL,
             "bad solver options");
  WB_REQUIRE(o.a_l >= 1.0 && o.a_r >= 1.0, WB_EINVAL, "boundary amplification must be >= 1");
  WB_REQUIRE(o.p_schedule == 0 || o.p_schedule == 1, WB_EINVAL, "p_schedule must be 0 or 1");
  WB_REQUIRE(o.schur_sign == 1 || o.schur_sign == -1, WB_EINVAL, "schur_sign must be 1 or -1");
  WB_REQUIRE(o.assemble_mb >= 0.0, WB_EINVAL, "assemble_mb must be >= 0");
  WB_REQUIRE(o.schur_approx == 0 || o.schur_approx == 1, WB_EINVAL, "schur_approx must be 0 or 1");
  WB_REQUIRE(o.weights >= 0 && o.weights <= 2, WB_EINVAL, "weights must be 0, 1 or 2");
  WB_REQUIRE(o.lanczos_steps >= 1 && o.lanczos_steps <= 100, WB_EINVAL,
             "lanczos_steps out of range (1..100)");
  WB_REQUIRE(o.precond_prec >= WB_FP64 && o.precond_prec <= WB_BF16X1, WB_EUNSUPPORTED,
             "preconditioner precision not built");
  const double t0 = now_s();
  std::unique_ptr<Solver> sp(new Solver());
  Solver& s = *sp;
  s.m = m;
  s.o = o;
  s.st = st;
  Arena& ar = s.arena;
  s.red_partial = ar.alloc<double>(RED_BLOCKS * 128);
  launch_fill<double>(st, s.red_partial, 0.0, (size_t)RED_BLOCKS * 128);  // the reduction counter
  s.red_out = ar.alloc<double>(16);
  s.lz = ar.alloc<double>(LZ_SLOTS);
  const int n3 = (m.k + 1) * (m.k + 1) * (m.k + 1);
  {
    size_t wbytes = op_workspace_bytes(3, m.N, m.k, sizeof(double));
    for (auto& lv : level_schedule(m.N, m.k, o.p_schedule)) {
      wbytes = std::max(wbytes, op_workspace_bytes(3, lv.first, lv.second, sizeof(double)));
      wbytes = std::max(wbytes, op_workspace_bytes(1, lv.first, lv.second, sizeof(double)));
    }
    s.opwork = ar.raw(wbytes);
    WB_HIP(hipEventCreateWithFlags(&s.main_ev, hipEventDisableTiming));
    for (int k = 0; k < AUX_STREAMS; ++k) {
      WB_HIP(hipStreamCreateWithFlags(&s.aux[k], hipStreamNonBlocking));
      WB_HIP(hipEventCreateWithFlags(&s.aux_ev[k], hipEventDisableTiming));
      s.aux_partial[k] = ar.alloc<double>(RED_BLOCKS + 64);
      launch_fill<double>(st, s.aux_partial[k], 0.0, RED_BLOCKS + 64);  // the reduction counter
      s.aux_work[k] = ar.raw(wbytes);
    }
  }
  SetupEstimates est;
  s.mu_q = ar.alloc<double>((size_t)m.E * n3);
  WB_HIP(hipMemcpyAsync(s.mu_q, mu_q, sizeof(double) * m.E * n3, hipMemcpyDeviceToDevice, st));

  PhaseClock clk(o.verbose != 0, st);
  clk.mark("scratch + mu copy");
  s.pd.reset(new Precond<double>());
  Precond<double>& P = *s.pd;
  build_hierarchy(s, P.A, 3, s.mu_q, 1000, est);
  clk.mark("velocity hierarchy");
  // learned coarse correction: velocity level Q1 on N/2 (if it is a smoothed level)
  for (int li = 0; li + 1 < (int)P.A.L.size(); ++li)
    if (P.A.L[li].k == 1 && 2 * P.A.L[li].N == m.N) {
      std::unique_ptr<Learned> G(new Learned());
      G->lc = li;
      G->M = P.A.L[li].N + 1;
      const size_t M3 = (size_t)G->M * G->M * G->M;
      G->params = ar.alloc<float>(net_param_count());
      launch_fill<float>(st, G->params, 0.f, net_param_count());
      G->feat = ar.alloc<float>(M3);
      G->xin = ar.alloc<float>(4 * M3);
      G->elem_tmp = ar.alloc<float>((size_t)P.A.L[li].E);
      net_work_carve(G->w1, G->M, 1, ar.raw(net_work_bytes(G->M, 1)));
      G->counters = ar.alloc<int>(2);
      launch_node_feature(st, P.A.L[li].N, P.A.L[li].coef, G->feat, G->elem_tmp);
      s.learned = std::move(G);
      break;
    }
  WB_REQUIRE(!o.use_learned || s.learned, WB_EUNSUPPORTED,
             "learned correction needs a velocity level Q1 on N/2 above the coarsest");
  // weights C = M(a_l sqrt(mu)), D = M(a_r sqrt(mu)) (eq. 8, Sec. 5); stored inverted
  const double amps[2] = {o.a_l, o.a_r};
  const double* dbh = const_table(make_bhat(m.k));
  alloc_work(s, P);
  P.mpinv = ar.alloc<double>((size_t)m.E * m.np);
  launch_pmass_inv(st, m.N, m.k, s.mu_q, P.mpinv);
  // diag(A)-BFBT: the unmasked diag(A) and the unweighted lumped mass for its Poisson coefficient
  const bool diag_a = o.weights == 2;
  double *diag3 = nullptr, *mass1 = nullptr;
  if (diag_a) {
    diag3 = ar.alloc<double>((size_t)3 * m.nn);
    launch_fill<double>(st, diag3, 0.0, (size_t)3 * m.nn);
    launch_diag(st, 3, m.N, m.k, false, s.mu_q, diag3);
    double* ones = ar.alloc<double>(m.nn);
    launch_fill<double>(st, ones, 1.0, m.nn);
    mass1 = ar.alloc<double>(m.nn);
    launch_fill<double>(st, mass1, 0.0, m.nn);
    launch_lumped_mass(st, m.N, m.k, 1.0, ones, mass1);
  }
  for (int side = 0; side < 2; ++side) {
    if (diag_a) {
      // C^-1 = D^-1 = diag(A)^-1 per velocity DOF (the masked level-0 Jacobi inverse)
      P.winv[side] = ar.alloc<double>((size_t)3 * m.nn);
      WB_HIP(hipMemcpyAsync(P.winv[side], P.A.L[0].dinv, sizeof(double) * 3 * m.nn,
                            hipMemcpyDeviceToDevice, st));
    } else {
      P.winv[side] = ar.alloc<double>(m.nn);
      launch_fill<double>(st, P.winv[side], 0.0, m.nn);
      if (o.weights == 1) launch_lumped_mass_grad(st, m.N, m.k, amps[side], mu_nodes, P.winv[side]);
      else launch_lumped_mass(st, m.N, m.k, amps[side], mu_nodes, P.winv[side]);
      launch_invert_diag(st, 1, m.N, m.k, false, P.winv[side]);
    }
    P.dk[side] = ar.alloc<double>((size_t)m.E * m.np);
    launch_diag_K(st, m.N, m.k, dbh, P.winv[side], P.dk[side], diag_a);
    // Poisson hierarchy on the coefficient 1/w at the Gauss points (eq. 11, 12)
    double* cq = ar.alloc<double>((size_t)m.E * n3);
    if (diag_a) launch_diag_a_coef(st, m.N, m.k, amps[side], diag3, mass1, cq);
    else if (o.weights == 1) launch_poisson_coef_grad(st, m.N, m.k, amps[side], s.mu_q, mu_nodes, cq);
    else launch_poisson_coef(st, m.N, m.k, amps[side], s.mu_q, cq);
    build_hierarchy(s, P.Pois[side], 1, cq, side == 0 ? 2000 : 3000, est);
  }
  clk.mark("weights + Poisson hierarchies");
  // Chebyshev bounds on the discontinuous K_w levels
  for (int side = 0; side < 2; ++side) {
    const size_t pl = (size_t)m.E * m.np;
    launch_splitmix_vec(st, pl, side == 0 ? 4000ULL : 5000ULL, 0, P.pr);
    launch_remove_mean<double>(st, m.E, m.np, P.pr, s.red_partial, s.red_out + 12);
    auto op = [&](const double* in, double* out) { apply_K<double>(s, P, side, in, out); };
    double* lz = next_lz(s, est, &P.klmin[side], &P.klmax[side]);
    lanczos_enqueue(st, op, pl, P.dk[side], o.lanczos_steps, P.pr, P.pd, P.pt, P.pm, lz, s.red_partial);
  }
  clk.mark("K_w bounds");
  // all eigenvalue estimates and the coarsest stencils: one host read
  {
    std::vector<double> h;
    join_setup_estimates(s, est, h);
    Hierarchy<double>* hs[3] = {&P.A, &P.Pois[0], &P.Pois[1]};
    std::vector<std::vector<double>> Sh(3);
    for (int i = 0; i < 3; ++i) {
      const Level<double>& C = hs[i]->L.back();
      Sh[i].resize(q1_stencil_len(C.NC, C.N));
      WB_HIP(hipMemcpyAsync(Sh[i].data(), C.S, sizeof(double) * Sh[i].size(), hipMemcpyDeviceToHost, st));
    }
    WB_HIP(hipStreamSynchronize(st));
    finish_setup_estimates(s, est, h);
    std::vector<std::vector<double>> keep_d;
    std::vector<std::vector<int>> keep_i;
    // the three dense inverses on host threads, then their uploads in order
    CoarseDense cd[3];
    std::exception_ptr err[3];
    {
      std::vector<std::thread> th;
      for (int i = 0; i < 3; ++i)
        th.emplace_back([&, i] {
          try {
            cd[i] = coarsest_dense(hs[i]->L.back(), Sh[i]);
          } catch (...) {
            err[i] = std::current_exception();
          }
        });
      for (auto& t : th) t.join();
    }
    for (int i = 0; i < 3; ++i)
      if (err[i]) std::rethrow_exception(err[i]);
    for (int i = 0; i < 3; ++i) coarsest_upload(s, *hs[i], std::move(cd[i]), keep_d, keep_i);
    WB_HIP(hipStreamSynchronize(st));
  }
  clk.mark("estimates + coarsest inverses");
  if (o.precond_prec != WB_FP64) {
    s.pf.reset(new Precond<float>());
    Precond<float>& F = *s.pf;
    cast_hierarchy(s, P.A, F.A);
    for (int side = 0; side < 2; ++side) {
      cast_hierarchy(s, P.Pois[side], F.Pois[side]);
      const size_t wl = (o.weights == 2 ? 3 : 1) * (size_t)m.nn;
      F.winv[side] = ar.alloc<float>(wl);
      launch_cast<double, float>(st, wl, P.winv[side], F.winv[side]);
      F.dk[side] = ar.alloc<float>((size_t)m.E * m.np);
      launch_cast<double, float>(st, (size_t)m.E * m.np, P.dk[side], F.dk[side]);
      F.klmin[side] = P.klmin[side];
      F.klmax[side] = P.klmax[side];
    }
    F.mpinv = ar.alloc<float>((size_t)m.E * m.np);
    launch_cast<double, float>(st, (size_t)m.E * m.np, P.mpinv, F.mpinv);
    alloc_work(s, F);
  }
  clk.mark("FP32 copies");
  // Krylov space
  s.n_tot = (size_t)3 * m.nn + (size_t)m.E * m.np;
  const int R = o.restart;
  s.V = ar.alloc<double>((size_t)(R + 1) * s.n_tot);
  s.Z = ar.alloc<double>((size_t)R * s.n_tot);
  s.w = ar.alloc<double>(s.n_tot);
  s.bvec = ar.alloc<double>(s.n_tot);
  s.xvec = ar.alloc<double>(s.n_tot);
  // two slots of (h1, h2, |w|^2) = 2 (R + 2) + 1 values, then the R coefficients of the update
  s.hbuf = ar.alloc<double>((size_t)5 * (R + 2));
  WB_HIP(hipHostMalloc((void**)&s.hpin, sizeof(double) * 2 * (2 * (R + 2) + 1), hipHostMallocDefault));
  for (int b = 0; b < 2; ++b) WB_HIP(hipEventCreateWithFlags(&s.hev[b], hipEventDisableTiming));
  s.mpartial = ar.alloc<double>((size_t)MDOT_BLOCKS * (R + 2));
  clk.mark("Krylov space");
  WB_HIP(hipStreamSynchronize(st));
  s.t_setup = now_s() - t0;
  return sp.release();
}

// ------------------------------------------------------------------ FGMRES
namespace {
void stokes_matvec(Solver& s, const double* x, double* y) {
  const Mesh& m = s.m;
  const size_t vl = (size_t)3 * m.nn;
  launch_op<double>(s.st, F_A | F_BT | F_B | F_DIR, 3, m.N, m.k, x, y, s.mu_q, x + vl, y + vl, nullptr,
                    false, s.opwork);
}
}  // namespace

// Right-preconditioned flexible GMRES(restart) on a vector of length n with x0 = 0, using the
// solver's Krylov storage.  Classical Gram-Schmidt with two passes.  On return s.xvec holds x;
// *iters and *relres the iteration count and the true relative residual.
template <typename MatVec, typename Prec>
wb_status fgmres_core(Solver& s, size_t n, const double* b, MatVec&& matvec, Prec&& precond,
                      double rtol, int max_iter, int* iters, double* relres_out) {
  hipStream_t st = s.st;
  const int R = s.o.restart;
  launch_fill<double>(st, s.xvec, 0.0, n);
  s.history.clear();
  const double bnorm = std::sqrt(dot_host(s, n, b, b));
  int it = 0;
  double relres = 0.0;
  wb_status status = WB_OK;
  if (bnorm > 0.0) {
    WB_HIP(hipMemcpyAsync(s.w, b, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    double beta = bnorm;
    std::vector<double> H((size_t)(R + 1) * R), cs(R), sn(R), g(R + 1);
    std::vector<double> hist;
    const size_t hs = (size_t)2 * (R + 2) + 1;  // one iteration's results: h1, h2, |w|^2
    // Arnoldi step j: v_j (from the previous step's w and its norm, still on the device, unless
    // j = 0), z_j = P v_j, w = K z_j, two classical Gram-Schmidt passes and |w|^2, then the
    // results go to the pinned slot j % 2 and its event is recorded.
    auto enqueue = [&](int j) {
      double* hb = s.hbuf + (size_t)(j & 1) * hs;
      double* vj = s.V + (size_t)j * n;
      double* zj = s.Z + (size_t)j * n;
      if (j > 0) launch_scal_rnorm(st, n, s.hbuf + (size_t)((j - 1) & 1) * hs + 2 * (R + 2), s.w, vj);
      precond(vj, zj);
      matvec(zj, s.w);
      launch_mdot(st, n, j + 1, s.V, n, s.w, s.mpartial, hb);
      if (!launch_gs_sub_dot(st, n, j + 1, s.V, n, hb, s.w, s.mpartial, hb + (R + 2))) {
        launch_gemv_sub(st, n, j + 1, s.V, n, hb, s.w);
        launch_mdot(st, n, j + 1, s.V, n, s.w, s.mpartial, hb + (R + 2));
      }
      launch_gemv_sub(st, n, j + 1, s.V, n, hb + (R + 2), s.w);
      launch_dot<double>(st, n, s.w, s.w, s.red_partial, hb + 2 * (R + 2));
      WB_HIP(hipMemcpyAsync(s.hpin + (size_t)(j & 1) * hs, hb, sizeof(double) * hs,
                            hipMemcpyDeviceToHost, st));
      WB_HIP(hipEventRecord(s.hev[j & 1], st));
    };
    // Step j + 1 is enqueued before step j's results are read (hiding the host round trip) only
    // while the residual estimate is far above the target, so that step j cannot plausibly
    // converge; a step enqueued in vain would delay the solution update by one iteration.
    constexpr double kAhead = 50.0;
    bool done = false;
    while (!done) {
      std::fill(H.begin(), H.end(), 0.0);
      std::fill(g.begin(), g.end(), 0.0);
      g[0] = beta;
      launch_scal<double>(st, n, 1.0 / beta, s.w, s.V);
      int jdone = 0;
      enqueue(0);
      for (int j = 0; j < R; ++j) {
        bool ahead = false;
        if (j + 1 < R && it + 1 < max_iter && std::fabs(g[j]) > kAhead * rtol * bnorm) {
          enqueue(j + 1);
          ahead = true;
        }
        WB_HIP(hipEventSynchronize(s.hev[j & 1]));
        const double* hh = s.hpin + (size_t)(j & 1) * hs;
        const double nrm = std::sqrt(hh[2 * (R + 2)]);
        if (!std::isfinite(nrm)) throw Error{WB_ENAN, "NaN/Inf in the Krylov vector"};
        for (int i = 0; i <= j; ++i) H[(size_t)i * R + j] = hh[i] + hh[(R + 2) + i];
        H[(size_t)(j + 1) * R + j] = nrm;
        for (int i = 0; i < j; ++i) {
          const double a = H[(size_t)i * R + j], bb = H[(size_t)(i + 1) * R + j];
          H[(size_t)i * R + j] = cs[i] * a + sn[i] * bb;
          H[(size_t)(i + 1) * R + j] = -sn[i] * a + cs[i] * bb;
        }
        const double a = H[(size_t)j * R + j], bb = H[(size_t)(j + 1) * R + j];
        const double den = std::hypot(a, bb);
        cs[j] = a / den;
        sn[j] = bb / den;
        H[(size_t)j * R + j] = den;
        H[(size_t)(j + 1) * R + j] = 0.0;
        g[j + 1] = -sn[j] * g[j];
        g[j] = cs[j] * g[j];
        ++it;
        jdone = j + 1;
        if (s.o.verbose) fprintf(stderr, "fgmres %4d  %.3e\n", it, std::fabs(g[j + 1]) / bnorm);
        // stagnation with the learned correction: less than a halving of the residual over the
        // last 20 iterations switches it off for the rest of the solve (flexible GMRES allows
        // the preconditioner to change between iterations)
        hist.push_back(std::fabs(g[j + 1]));
        s.history.push_back(std::fabs(g[j + 1]) / bnorm);
        if (s.learned && s.learned->active && s.learned->trained && s.o.use_learned &&
            hist.size() > 20 && hist.back() > 0.5 * hist[hist.size() - 21]) {
          s.learned->active = false;
          s.fell_back += 1;
          if (s.pgraph) {
            WB_HIP(hipStreamSynchronize(st));
            (void)hipGraphExecDestroy(s.pgraph);
            s.pgraph = nullptr;
          }
        }
        // a step enqueued ahead of a stop runs to completion unused; the update below reads
        // only Z_0 .. Z_j and its own coefficient slot
        if (std::fabs(g[j + 1]) <= rtol * bnorm || it >= max_iter || nrm == 0.0) break;
        if (!ahead && j + 1 < R) enqueue(j + 1);
      }
      std::vector<double> y(jdone);
      for (int i = jdone - 1; i >= 0; --i) {
        double t = g[i];
        for (int c = i + 1; c < jdone; ++c) t -= H[(size_t)i * R + c] * y[c];
        y[i] = t / H[(size_t)i * R + i];
      }
      double* yd = s.hbuf + 2 * hs;
      WB_HIP(hipMemcpyAsync(yd, y.data(), sizeof(double) * jdone, hipMemcpyHostToDevice, st));
      launch_gemv_add(st, n, jdone, s.Z, n, yd, s.xvec);
      // true residual
      matvec(s.xvec, s.w);
      launch_axpby<double>(st, n, 1.0, b, -1.0, s.w);
      beta = std::sqrt(dot_host(s, n, s.w, s.w));
      relres = beta / bnorm;
      if (relres <= rtol) done = true;
      else if (it >= max_iter) {
        status = WB_ENOCONV;
        done = true;
      }
    }
  }
  *iters = it;
  *relres_out = relres;
  return status;
}

// The preconditioner apply of FGMRES replayed from a HIP graph.  Its launch sequence (several
// hundred small kernels for the V-cycles) depends only on the solver, so it is captured once,
// on a solver-owned stream and between fixed staging vectors, and replayed per iteration on the
// solver's stream: the input is copied into gin, the graph runs, the result is copied out of gout.
void precond_graph(Solver& s, const double* v, double* z) {
  const size_t n = s.n_tot, vl = (size_t)3 * s.m.nn;
  hipStream_t st = s.st;
  if (!s.pgraph) {
    if (!s.gin) {
      s.gin = s.arena.alloc<double>(n);
      s.gout = s.arena.alloc<double>(n);
    }
    if (!s.cap_st) WB_HIP(hipStreamCreateWithFlags(&s.cap_st, hipStreamNonBlocking));
    WB_HIP(hipStreamSynchronize(st));
    hipGraph_t g = nullptr;
    WB_HIP(hipStreamBeginCapture(s.cap_st, hipStreamCaptureModeRelaxed));
    s.st = s.cap_st;
    try {
      apply_precond_any(s, s.gin, s.gin + vl, s.gout, s.gout + vl);
    } catch (...) {
      s.st = st;
      (void)hipStreamEndCapture(s.cap_st, &g);
      if (g) (void)hipGraphDestroy(g);
      throw;
    }
    s.st = st;
    WB_HIP(hipStreamEndCapture(s.cap_st, &g));
    const hipError_t e = hipGraphInstantiate(&s.pgraph, g, nullptr, nullptr, 0);
    (void)hipGraphDestroy(g);
    if (e != hipSuccess) {
      s.pgraph = nullptr;
      throw Error{WB_EHIP, std::string("hipGraphInstantiate: ") + hipGetErrorString(e)};
    }
  }
  WB_HIP(hipMemcpyAsync(s.gin, v, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
  WB_HIP(hipGraphLaunch(s.pgraph, st));
  WB_HIP(hipMemcpyAsync(z, s.gout, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
}

// Residual reduction |r - alpha A delta| / |r| of a learned correction from (r, r), (r, A delta),
// (A delta, A delta), alpha clipped to [0, 2] as in the update.
double learned_reduction(double rr, double rad, double aa) {
  if (!(rr > 0.0) || !(aa > 0.0) || !std::isfinite(rr * rad * aa)) return 1.0;
  const double a = std::min(std::max(rad / aa, 0.0), 2.0);
  return std::sqrt(std::max(0.0, rr - 2.0 * a * rad + a * a * aa) / rr);
}

wb_status fgmres(Solver& s, const double* f, double* u, double* p, wb_report* rep) {
  const double t0 = now_s();
  hipStream_t st = s.st;
  const Mesh& m = s.m;
  const size_t n = s.n_tot, vl = (size_t)3 * m.nn, pl = (size_t)m.E * m.np;
  s.learned_used = s.fell_back = 0;
  s.learned_red = 1.0;
  if (s.learned) {
    launch_fill<int>(st, s.learned->counters, 0, 2);
    if (!s.learned->active) {
      s.learned->active = true;
      if (s.pgraph) {
        WB_HIP(hipStreamSynchronize(st));
        (void)hipGraphExecDestroy(s.pgraph);
        s.pgraph = nullptr;
      }
    }
  }
  // b = [f with zero boundary entries; 0]
  WB_HIP(hipMemcpyAsync(s.bvec, f, sizeof(double) * vl, hipMemcpyDeviceToDevice, st));
  launch_mask_boundary<double>(st, m.M, 3, s.bvec);
  launch_fill<double>(st, s.bvec + vl, 0.0, pl);
  int it = 0;
  double relres = 0.0;
  // The learned coarse correction is checked on the solve's first preconditioner apply: kept if
  // it removes enough of the residual at level lc (|r - alpha A delta| <= LEARNED_ACCEPT |r|),
  // else the solve falls back to the plain V-cycle and that apply is repeated.
  bool check_learned = s.learned && s.learned->trained && s.o.use_learned;
  const wb_status status = fgmres_core(
      s, n, s.bvec, [&](const double* x, double* y) { stokes_matvec(s, x, y); },
      [&](const double* v, double* z) {
        if (check_learned) {
          check_learned = false;
          apply_precond_any(s, v, v + vl, z, z + vl);
          double d[3];
          WB_HIP(hipMemcpyAsync(d, s.red_out + 8, sizeof(d), hipMemcpyDeviceToHost, st));
          WB_HIP(hipStreamSynchronize(st));
          s.learned_red = learned_reduction(d[0], d[1], d[2]);
          if (!(s.learned_red <= LEARNED_ACCEPT)) {
            s.learned->active = false;
            s.fell_back += 1;
            if (s.pgraph) {
              (void)hipGraphExecDestroy(s.pgraph);
              s.pgraph = nullptr;
            }
            apply_precond_any(s, v, v + vl, z, z + vl);
          }
          return;
        }
        if (s.o.use_graph) precond_graph(s, v, z);
        else apply_precond_any(s, v, v + vl, z, z + vl);
      },
      s.o.rtol,
      s.o.max_iter, &it, &relres);
  launch_remove_mean<double>(st, m.E, m.np, s.xvec + vl, s.red_partial, s.red_out + 3);
  WB_HIP(hipMemcpyAsync(u, s.xvec, sizeof(double) * vl, hipMemcpyDeviceToDevice, st));
  WB_HIP(hipMemcpyAsync(p, s.xvec + vl, sizeof(double) * pl, hipMemcpyDeviceToDevice, st));
  int cnt[2] = {0, 0};
  if (s.learned) WB_HIP(hipMemcpyAsync(cnt, s.learned->counters, sizeof(cnt), hipMemcpyDeviceToHost, st));
  WB_HIP(hipStreamSynchronize(st));
  // accepted correction steps; rejected ones (alpha = 0) plus a stagnation switch-off
  s.learned_used = cnt[0];
  s.fell_back += cnt[1];
  if (rep) {
    rep->iters = it;
    rep->rel_res = relres;
    rep->t_setup_s = s.t_setup;
    rep->t_solve_s = now_s() - t0;
    rep->fell_back = s.fell_back;
    rep->learned_used = s.learned_used;
    rep->device_bytes = s.arena.bytes();
    rep->learned_reduction = s.learned_red;
    rep->history = s.history.data();
    rep->history_len = (int)s.history.size();
  }
  return status;
}

wb_status subsolve(Solver& s, int which, const double* b_in, double* x, wb_report* rep) {
  const double t0 = now_s();
  hipStream_t st = s.st;
  const Mesh& m = s.m;
  Precond<double>& P = *s.pd;
  const size_t vl = (size_t)3 * m.nn, pl = (size_t)m.E * m.np;
  int it = 0;
  double relres = 0.0;
  wb_status status;
  if (which == 0) {
    // A u = f with one velocity V-cycle as preconditioner
    WB_HIP(hipMemcpyAsync(s.bvec, b_in, sizeof(double) * vl, hipMemcpyDeviceToDevice, st));
    launch_mask_boundary<double>(st, m.M, 3, s.bvec);
    status = fgmres_core(
        s, vl, s.bvec,
        [&](const double* xx, double* yy) {
          launch_op<double>(st, F_A | F_DIR, 3, m.N, m.k, xx, yy, s.mu_q, nullptr, nullptr, nullptr,
                            false, s.opwork);
        },
        [&](const double* v, double* z) { apply_vcycle_A<double>(s, P, v, z); }, s.o.rtol,
        s.o.max_iter, &it, &relres);
    WB_HIP(hipMemcpyAsync(x, s.xvec, sizeof(double) * vl, hipMemcpyDeviceToDevice, st));
  } else {
    // K_w p = g (w left for which == 1, right for which == 2) with one K_w V-cycle; g and p mean-free
    const int side = which - 1;
    WB_HIP(hipMemcpyAsync(s.bvec, b_in, sizeof(double) * pl, hipMemcpyDeviceToDevice, st));
    launch_remove_mean<double>(st, m.E, m.np, s.bvec, s.red_partial, s.red_out + 4);
    status = fgmres_core(
        s, pl, s.bvec, [&](const double* xx, double* yy) { apply_K<double>(s, P, side, xx, yy); },
        [&](const double* v, double* z) { apply_vcycle_K<double>(s, P, side, v, z); }, s.o.rtol,
        s.o.max_iter, &it, &relres);
    launch_remove_mean<double>(st, m.E, m.np, s.xvec, s.red_partial, s.red_out + 4);
    WB_HIP(hipMemcpyAsync(x, s.xvec, sizeof(double) * pl, hipMemcpyDeviceToDevice, st));
  }
  WB_HIP(hipStreamSynchronize(st));
  if (rep) {
    rep->iters = it;
    rep->rel_res = relres;
    rep->t_setup_s = s.t_setup;
    rep->t_solve_s = now_s() - t0;
    rep->fell_back = 0;
    rep->learned_used = 0;
    rep->device_bytes = s.arena.bytes();
    rep->learned_reduction = 1.0;
    rep->history = s.history.data();
    rep->history_len = (int)s.history.size();
  }
  return status;
}

// ------------------------------------------------------------------ learned correction
namespace {
void drop_graph(Solver& s) {
  if (s.pgraph) {
    WB_HIP(hipStreamSynchronize(s.st));
    (void)hipGraphExecDestroy(s.pgraph);
    s.pgraph = nullptr;
  }
}

// coefficient of level `to` from level `to - 1` with the hierarchy's coarsening matrices
void coarsen_level(hipStream_t st, const Level<double>& F, const Level<double>& L, const double* fc,
                   double* lc) {
  if (F.N == L.N) launch_coarsen_p(st, L.E, F.k + 1, L.k + 1, L.Q, fc, lc);
  else launch_coarsen_h(st, F.N, L.k + 1, L.Q, fc, lc);
}
}  // namespace

void learned_set(Solver& s, const float* params_host) {
  WB_REQUIRE(s.learned, WB_EUNSUPPORTED, "no learned level (Q1 on N/2) on this mesh");
  WB_HIP(hipMemcpyAsync(s.learned->params, params_host, sizeof(float) * net_param_count(),
                        hipMemcpyHostToDevice, s.st));
  WB_HIP(hipStreamSynchronize(s.st));
  s.learned->trained = true;
  drop_graph(s);
}

void learned_probe(Solver& s, const double* r, double* delta, double* alpha_host) {
  WB_REQUIRE(s.learned, WB_EUNSUPPORTED, "no learned level (Q1 on N/2) on this mesh");
  Learned& G = *s.learned;
  Level<double>& L = s.pd->A.L[G.lc];
  learned_delta<double>(s, L, r, delta, L.t);
  launch_fill<double>(s.st, L.x, 0.0, L.len);
  launch_net_guarded_update<double>(s.st, L.len, s.red_out + 9, L.x, delta, G.counters);
  WB_HIP(hipMemcpyAsync(alpha_host, s.red_out + 11, sizeof(double), hipMemcpyDeviceToHost, s.st));
  WB_HIP(hipStreamSynchronize(s.st));
}

void learned_train(Solver& s, int n_fields, const int* n_sinkers, const double* centers,
                   const TrainOpts& o, TrainReport* rep) {
  WB_REQUIRE(s.learned, WB_EUNSUPPORTED, "no learned level (Q1 on N/2) on this mesh");
  WB_REQUIRE(n_fields >= 1 && n_sinkers && o.pairs_per_field >= 1 && o.vcycles >= 1 &&
                 o.epochs >= 0 && o.batch >= 1 && o.lr > 0 && o.n_valid >= 0 &&
                 o.n_valid < n_fields && o.mu_min > 0 && o.mu_max >= o.mu_min,
             WB_EINVAL, "bad training options");
  Learned& G = *s.learned;
  hipStream_t st = s.st;
  const Mesh& m = s.m;
  Hierarchy<double>& A = s.pd->A;
  const int lc = G.lc, M = G.M;
  const size_t M3 = (size_t)M * M * M, len = 3 * M3;
  const int ppf = o.pairs_per_field;
  const int nt = n_fields * ppf, nv = o.n_valid * ppf, ntr = nt - nv;
  const int B = std::min(o.batch, ntr);
  int max_ns = 0;
  for (int f = 0; f < n_fields; ++f) {
    WB_REQUIRE(n_sinkers[f] >= 0, WB_EINVAL, "negative sinker count");
    max_ns = std::max(max_ns, n_sinkers[f]);
  }
  WB_REQUIRE(max_ns == 0 || centers, WB_EINVAL, "NULL centers");
  Arena ar;  // training buffers, freed on return
  struct StreamDrain {  // destroyed before `ar`: queued work ends before the buffers are freed
    hipStream_t st;
    ~StreamDrain() { (void)hipStreamSynchronize(st); }
  } drain{st};
  // Training level: the solver's level lc (shape, transfers, coarsening matrices) with each
  // field's own coefficient, diagonal and Chebyshev bounds (and stencil, when the solver
  // assembles that level).  The network stands in for everything below lc, so a pair needs only
  // the field's own operator and smoother at lc.
  Level<double> L0 = A.L[lc];
  {
    const int n = L0.k + 1;
    L0.coef = ar.alloc<double>((size_t)L0.E * n * n * n);
    L0.dinv = ar.alloc<double>(L0.len);
    L0.S = A.L[lc].S ? ar.alloc<double>(q1_stencil_len(3, L0.N)) : nullptr;
    for (double** v : {&L0.x, &L0.b, &L0.r, &L0.d, &L0.t}) *v = ar.alloc<double>(L0.len);
  }
  std::vector<double*> chain(lc + 1, nullptr);
  for (int li = 0; li < lc; ++li) {
    const int n = A.L[li].k + 1;
    chain[li] = ar.alloc<double>((size_t)A.L[li].E * n * n * n);
  }
  chain[lc] = L0.coef;
  double* dcent = ar.alloc<double>(3 * (size_t)std::max(1, max_ns));
  float* X = ar.alloc<float>((size_t)nt * 4 * M3);
  float* Tt = ar.alloc<float>((size_t)nt * 3 * M3);
  float* Wt = ar.alloc<float>((size_t)nt * 3 * M3);
  float* feat = ar.alloc<float>(M3);
  float* etmp = ar.alloc<float>((size_t)L0.E);
  double* e = ar.alloc<double>(len);
  double* bb = ar.alloc<double>(len);
  double* rr = ar.alloc<double>(len);
  double* sums = ar.alloc<double>(4);
  const bool was_active = G.active;
  G.active = false;
  drop_graph(s);
  const double t0 = now_s();
  size_t coff = 0;
  for (int f = 0; f < n_fields; ++f) {
    const int ns = n_sinkers[f];
    if (ns > 0)
      WB_HIP(hipMemcpyAsync(dcent, centers + coff, sizeof(double) * 3 * ns, hipMemcpyHostToDevice, st));
    coff += 3 * (size_t)ns;
    launch_sinker_q(st, m.N, m.k, dcent, ns, o.delta, o.omega, o.mu_min, o.mu_max, 0.0, chain[0],
                    nullptr);
    for (int li = 1; li <= lc; ++li) coarsen_level(st, A.L[li - 1], A.L[li], chain[li - 1], chain[li]);
    launch_fill<double>(st, L0.dinv, 0.0, L0.len);
    launch_diag(st, 3, L0.N, L0.k, true, L0.coef, L0.dinv);
    launch_invert_diag(st, 3, L0.N, L0.k, true, L0.dinv);
    if (L0.S) assemble_level(s, L0);
    for (double* v : {L0.x, L0.b, L0.r, L0.d, L0.t}) launch_fill<double>(st, v, 0.0, L0.len);
    set_cheb_bounds(s, L0, (unsigned long long)(1000 + lc));
    launch_node_feature(st, L0.N, L0.coef, feat, etmp);
    for (int j = 0; j < ppf; ++j) {
      const int pid = f * ppf + j;
      // the error the pre-smoothing at lc leaves of a splitmix64 start: e <- (I - S A) e
      launch_splitmix_field(st, M, o.seed + (unsigned long long)pid, e);
      for (int v = 0; v < o.vcycles; ++v) {
        level_op<double>(st, L0, e, bb, s.opwork);
        cheb_level<double>(s, L0, bb, rr, true);
        launch_axpby<double>(st, len, -1.0, rr, 1.0, e);
      }
      level_op<double>(st, L0, e, rr, s.opwork);  // r = A e
      launch_dot<double>(st, len, rr, rr, s.red_partial, sums);
      launch_energy_diag(st, M, e, L0.dinv, s.red_partial, sums + 1);
      launch_net_pair(st, M, feat, e, rr, L0.dinv, sums, X + (size_t)pid * 4 * M3,
                      Tt + (size_t)pid * 3 * M3, Wt + (size_t)pid * 3 * M3);
    }
  }
  WB_HIP(hipStreamSynchronize(st));
  const double t1 = now_s();
  // Adam on the training pairs (the trailing n_valid fields are held out)
  const size_t np = net_param_count();
  NetWork W;
  net_work_carve(W, M, B, ar.raw(net_work_bytes(M, B)));
  float* grad = ar.alloc<float>(np);
  float* am = ar.alloc<float>(np);
  float* av = ar.alloc<float>(np);
  launch_fill<float>(st, am, 0.f, np);
  launch_fill<float>(st, av, 0.f, np);
  float* bx = ar.alloc<float>((size_t)B * 4 * M3);
  float* bt = ar.alloc<float>((size_t)B * 3 * M3);
  float* bw = ar.alloc<float>((size_t)B * 3 * M3);
  const int nb = ntr / B;
  double* losses = ar.alloc<double>((size_t)std::max(nb, 1));
  net_init(st, G.params, o.seed ^ 0x5EEDULL);
  std::vector<int> perm(ntr);
  for (int i = 0; i < ntr; ++i) perm[i] = i;
  std::vector<double> lh(std::max(nb, 1));
  int step = 0;
  double first = 0.0, last = 0.0;
  for (int ep = 0; ep < o.epochs; ++ep) {
    std::vector<double> u;
    splitmix_vector(o.seed + 7919ULL * (ep + 1), (size_t)ntr, u);
    for (int i = ntr - 1; i > 0; --i) {  // Fisher-Yates with u in [-1, 1)
      const int jj = std::min(i, (int)((0.5 * (u[i] + 1.0)) * (i + 1)));
      std::swap(perm[i], perm[jj]);
    }
    for (int bi = 0; bi < nb; ++bi) {
      for (int j = 0; j < B; ++j) {
        const size_t q = (size_t)perm[bi * B + j];
        WB_HIP(hipMemcpyAsync(bx + (size_t)j * 4 * M3, X + q * 4 * M3, sizeof(float) * 4 * M3,
                              hipMemcpyDeviceToDevice, st));
        WB_HIP(hipMemcpyAsync(bt + (size_t)j * 3 * M3, Tt + q * 3 * M3, sizeof(float) * 3 * M3,
                              hipMemcpyDeviceToDevice, st));
        WB_HIP(hipMemcpyAsync(bw + (size_t)j * 3 * M3, Wt + q * 3 * M3, sizeof(float) * 3 * M3,
                              hipMemcpyDeviceToDevice, st));
      }
      net_forward(st, G.params, bx, W);
      net_backward(st, G.params, bx, bt, bw, W, grad, losses + bi);
      net_adam(st, np, G.params, grad, am, av, ++step, (float)o.lr);
    }
    WB_HIP(hipMemcpyAsync(lh.data(), losses, sizeof(double) * nb, hipMemcpyDeviceToHost, st));
    WB_HIP(hipStreamSynchronize(st));
    double mean = 0.0;
    for (int bi = 0; bi < nb; ++bi) mean += lh[bi];
    mean /= std::max(nb, 1);
    if (ep == 0) first = mean;
    last = mean;
    if (s.o.verbose) fprintf(stderr, "learned epoch %3d  loss %.4e\n", ep, mean);
  }
  // validation loss on the held-out fields (batch 1)
  double vloss = 0.0;
  if (nv > 0) {
    NetWork V1;
    net_work_carve(V1, M, 1, ar.raw(net_work_bytes(M, 1)));
    std::vector<double> vl(nv);
    double* vd = ar.alloc<double>(nv);
    for (int i = 0; i < nv; ++i) {
      const size_t q = (size_t)(ntr + i);
      net_forward(st, G.params, X + q * 4 * M3, V1);
      net_backward(st, G.params, X + q * 4 * M3, Tt + q * 3 * M3, Wt + q * 3 * M3, V1, grad, vd + i);
    }
    WB_HIP(hipMemcpyAsync(vl.data(), vd, sizeof(double) * nv, hipMemcpyDeviceToHost, st));
    WB_HIP(hipStreamSynchronize(st));
    for (double v : vl) vloss += v / nv;
  }
  WB_HIP(hipStreamSynchronize(st));
  G.trained = true;
  G.active = was_active;
  if (rep) {
    rep->loss_first = first;
    rep->loss_last = last;
    rep->valid_loss = vloss;
    rep->t_pairs_s = t1 - t0;
    rep->t_train_s = now_s() - t1;
    rep->n_params = (long long)np;
    rep->n_pairs = nt;
  }
}

}  // namespace wb
