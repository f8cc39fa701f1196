// C-ABI entry points (declared in include/wbfbt.h).  Every call converts internal
// exceptions into a wb_status and a thread-local message.
#include <algorithm>
#include <cmath>
#include <cstring>
#include <memory>
#include <mutex>

#include "solver.h"

namespace wb {

static thread_local std::string g_err;
void set_error(const std::string& msg) { g_err = msg; }

namespace {

template <typename F>
wb_status guard(F&& f) {
  try {
    g_err.clear();
    return f();
  } catch (const Error& e) {
    g_err = e.msg;
    return e.code;
  } catch (const std::bad_alloc&) {
    g_err = "host allocation failed";
    return WB_ENOMEM;
  } catch (const std::exception& e) {
    g_err = e.what();
    return WB_EINVAL;
  }
}

hipStream_t S(void* s) { return reinterpret_cast<hipStream_t>(s); }

void check_launch() {
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) throw Error{WB_EHIP, std::string("kernel launch: ") + hipGetErrorString(e)};
}

Mesh make_mesh(int N, int k) {
  WB_REQUIRE(N >= 1 && N <= 1024, WB_EINVAL, "N must be in [1, 1024]");
  WB_REQUIRE(k >= 1 && k <= 5, WB_EUNSUPPORTED, "k must be in [1, 5]");
  Mesh m;
  m.N = N;
  m.k = k;
  m.n = k + 1;
  m.M = k * N + 1;
  const long long nn = (long long)m.M * m.M * m.M;
  WB_REQUIRE(3 * nn < (1LL << 31), WB_EINVAL, "mesh too large for 32-bit node indices");
  m.nn = (int)nn;
  m.E = N * N * N;
  m.np = modes(k, nullptr, nullptr, nullptr);
  m.h = 1.0 / N;
  return m;
}

// Fixed device workspace of wb_apply_A_noalloc: each device that runs it holds its own copy
// until the process ends; host code uses only the address taken with hipGetSymbolAddress.
constexpr size_t NOALLOC_SCRATCH_BYTES = 64u << 20;
static __device__ __align__(256) double scratch[NOALLOC_SCRATCH_BYTES / sizeof(double)];
constexpr int NOALLOC_MAX_DEVICES = 64;
std::mutex scratch_mu;
void* scratch_ptr[NOALLOC_MAX_DEVICES] = {};

// The scratch array's device address on the current device (looked up once per device).
void* noalloc_scratch() {
  int dev = 0;
  WB_HIP(hipGetDevice(&dev));
  WB_REQUIRE(dev >= 0 && dev < NOALLOC_MAX_DEVICES, WB_EUNSUPPORTED, "device index out of range");
  std::lock_guard<std::mutex> g(scratch_mu);
  if (!scratch_ptr[dev]) {
    void* ptr = nullptr;
    WB_HIP(hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch)));
    WB_REQUIRE(ptr != nullptr, WB_EHIP, "hipGetSymbolAddress returned no address");
    scratch_ptr[dev] = ptr;
  }
  return scratch_ptr[dev];
}

// Face-array workspace of the scatter operators for standalone applies on this mesh
// (allocated on first use; calls sharing a mesh handle must be stream-ordered).
void* mesh_work(const wb_mesh* mh) {
  if (!mh->work) {
    const size_t bytes = op_workspace_bytes(3, mh->m.N, mh->m.k, sizeof(double));
    WB_HIP(hipMalloc(&mh->work, bytes));
  }
  return mh->work;
}

std::vector<double> node_coords_1d(const Mesh& m) {
  const Tables& t = tables(m.k);
  std::vector<double> x1(m.M);
  for (int e = 0; e < m.N; ++e)
    for (int a = 0; a <= m.k; ++a) x1[e * m.k + a] = (e + 0.5 * (t.xl[a] + 1.0)) / m.N;
  x1[m.M - 1] = 1.0;
  return x1;
}

}  // namespace
}  // namespace wb

using namespace wb;

extern "C" {

void wb_opts_default(wb_opts* o) {
  if (!o) return;
  std::memset(o, 0, sizeof(*o));
  o->a_l = 1.0;
  o->a_r = 1.0;
  o->cheb_degree = 3;
  o->lanczos_steps = 10;
  o->restart = 100;
  o->max_iter = 1000;
  o->rtol = 1e-6;
  o->precond_prec = WB_FP64;
  o->use_learned = 0;
  o->verbose = 0;
  o->use_graph = 1;
  o->schur_sign = -1;
  o->assemble_mb = 32.0;
  o->schur_approx = 0;
  o->weights = 0;
}

const char* wb_last_error(void) { return g_err.c_str(); }

wb_status wb_mesh_create(int N, int k, wb_mesh** out) {
  return guard([&] {
    WB_REQUIRE(out, WB_EINVAL, "out is NULL");
    std::unique_ptr<wb_mesh> m(new wb_mesh());
    m->m = make_mesh(N, k);
    *out = m.release();
    return WB_OK;
  });
}

void wb_mesh_destroy(wb_mesh* m) {
  if (!m) return;
  if (m->work) (void)hipFree(m->work);
  delete m;
}

wb_status wb_mesh_sizes(const wb_mesh* m, long long* n_nodes, long long* n_elem, int* n_p) {
  return guard([&] {
    WB_REQUIRE(m, WB_EINVAL, "mesh is NULL");
    if (n_nodes) *n_nodes = m->m.nn;
    if (n_elem) *n_elem = m->m.E;
    if (n_p) *n_p = m->m.np;
    return WB_OK;
  });
}

wb_status wb_visc_create_sinker(const wb_mesh* mh, const double* centers, int ns, double delta,
                                double omega, double mu_min, double mu_max, void* stream,
                                wb_visc** out) {
  return guard([&] {
    WB_REQUIRE(mh && out, WB_EINVAL, "NULL argument");
    WB_REQUIRE(ns >= 0 && (ns == 0 || centers), WB_EINVAL, "bad sinker centres");
    WB_REQUIRE(mu_min > 0 && mu_max >= mu_min && delta > 0 && omega >= 0, WB_EINVAL,
               "bad sinker parameters");
    const Mesh& m = mh->m;
    hipStream_t st = S(stream);
    std::unique_ptr<wb_visc> v(new wb_visc());
    v->m = m;
    const size_t nq = (size_t)m.E * m.n * m.n * m.n;
    WB_HIP(hipMalloc(&v->mu_q, sizeof(double) * nq));
    WB_HIP(hipMalloc(&v->mu_nodes, sizeof(double) * m.nn));
    double* dc = nullptr;
    double* dx = nullptr;
    WB_HIP(hipMalloc(&dc, sizeof(double) * 3 * (ns > 0 ? ns : 1)));
    WB_HIP(hipMalloc(&dx, sizeof(double) * m.M));
    auto x1 = node_coords_1d(m);
    if (ns > 0) WB_HIP(hipMemcpy(dc, centers, sizeof(double) * 3 * ns, hipMemcpyHostToDevice));
    WB_HIP(hipMemcpy(dx, x1.data(), sizeof(double) * m.M, hipMemcpyHostToDevice));
    launch_sinker_q(st, m.N, m.k, dc, ns, delta, omega, mu_min, mu_max, 0.0, v->mu_q, nullptr);
    launch_sinker_nodes(st, m.N, m.k, dx, dc, ns, delta, omega, mu_min, mu_max, v->mu_nodes);
    check_launch();
    WB_HIP(hipStreamSynchronize(st));
    (void)hipFree(dc);
    (void)hipFree(dx);
    *out = v.release();
    return WB_OK;
  });
}

wb_status wb_visc_create_values(const wb_mesh* mh, const double* mu_q, const double* mu_nodes,
                                void* stream, wb_visc** out) {
  return guard([&] {
    WB_REQUIRE(mh && out && mu_q && mu_nodes, WB_EINVAL, "NULL argument");
    const Mesh& m = mh->m;
    hipStream_t st = S(stream);
    std::unique_ptr<wb_visc> v(new wb_visc());
    v->m = m;
    const size_t nq = (size_t)m.E * m.n * m.n * m.n;
    WB_HIP(hipMalloc(&v->mu_q, sizeof(double) * nq));
    WB_HIP(hipMalloc(&v->mu_nodes, sizeof(double) * m.nn));
    WB_HIP(hipMemcpyAsync(v->mu_q, mu_q, sizeof(double) * nq, hipMemcpyDeviceToDevice, st));
    WB_HIP(hipMemcpyAsync(v->mu_nodes, mu_nodes, sizeof(double) * m.nn, hipMemcpyDeviceToDevice, st));
    WB_HIP(hipStreamSynchronize(st));
    *out = v.release();
    return WB_OK;
  });
}

wb_status wb_visc_values(const wb_visc* v, double* mu_q, double* mu_nodes, void* stream) {
  return guard([&] {
    WB_REQUIRE(v, WB_EINVAL, "visc is NULL");
    hipStream_t st = S(stream);
    const Mesh& m = v->m;
    if (mu_q)
      WB_HIP(hipMemcpyAsync(mu_q, v->mu_q, sizeof(double) * m.E * m.n * m.n * m.n,
                            hipMemcpyDeviceToDevice, st));
    if (mu_nodes)
      WB_HIP(hipMemcpyAsync(mu_nodes, v->mu_nodes, sizeof(double) * m.nn, hipMemcpyDeviceToDevice, st));
    WB_HIP(hipStreamSynchronize(st));
    return WB_OK;
  });
}

void wb_visc_destroy(wb_visc* v) {
  if (!v) return;
  (void)hipFree(v->mu_q);
  (void)hipFree(v->mu_nodes);
  if (v->mu_q_f) (void)hipFree(v->mu_q_f);
  delete v;
}

wb_status wb_rhs_sinker(const wb_mesh* mh, const double* centers, int ns, double delta,
                        double omega, double beta, double* f, void* stream) {
  return guard([&] {
    WB_REQUIRE(mh && f, WB_EINVAL, "NULL argument");
    WB_REQUIRE(ns >= 0 && (ns == 0 || centers), WB_EINVAL, "bad sinker centres");
    const Mesh& m = mh->m;
    hipStream_t st = S(stream);
    const size_t nq = (size_t)m.E * m.n * m.n * m.n;
    double *fq = nullptr, *dc = nullptr;
    WB_HIP(hipMalloc(&fq, sizeof(double) * nq));
    WB_HIP(hipMalloc(&dc, sizeof(double) * 3 * (ns > 0 ? ns : 1)));
    if (ns > 0) WB_HIP(hipMemcpy(dc, centers, sizeof(double) * 3 * ns, hipMemcpyHostToDevice));
    launch_sinker_q(st, m.N, m.k, dc, ns, delta, omega, 1.0, 1.0, beta, nullptr, fq);
    launch_fill<double>(st, f, 0.0, (size_t)3 * m.nn);
    launch_load(st, m.N, m.k, fq, f);
    check_launch();
    WB_HIP(hipStreamSynchronize(st));
    (void)hipFree(fq);
    (void)hipFree(dc);
    return WB_OK;
  });
}

wb_status wb_apply_A(const wb_mesh* mh, const wb_visc* v, const double* u, double* y, void* stream) {
  return guard([&] {
    WB_REQUIRE(mh && v && u && y, WB_EINVAL, "NULL argument");
    WB_REQUIRE(u != y, WB_EINVAL, "in-place apply is not allowed");
    const Mesh& m = mh->m;
    launch_op<double>(S(stream), F_A | F_DIR, 3, m.N, m.k, u, y, v->mu_q, nullptr, nullptr, nullptr,
                      false, mesh_work(mh));
    check_launch();
    return WB_OK;
  });
}

wb_status wb_apply_A_noalloc(const wb_mesh* mh, const wb_visc* v, const double* u, double* y,
                             void* stream) {
  return guard([&] {
    WB_REQUIRE(mh && v && u && y, WB_EINVAL, "NULL argument");
    WB_REQUIRE(u != y, WB_EINVAL, "in-place apply is not allowed");
    const Mesh& m = mh->m;
    const size_t need = op_workspace_bytes_capped(3, m.N, m.k, sizeof(double), NOALLOC_SCRATCH_BYTES);
    if (need > NOALLOC_SCRATCH_BYTES) {
      char msg[160];
      snprintf(msg, sizeof(msg), "wb_apply_A_noalloc: this mesh needs %zu bytes of workspace, above "
               "the fixed %zu", need, NOALLOC_SCRATCH_BYTES);
      throw Error{WB_EINVAL, msg};
    }
    void* work = noalloc_scratch();
    WorkspaceCap cap(NOALLOC_SCRATCH_BYTES);
    launch_op<double>(S(stream), F_A | F_DIR, 3, m.N, m.k, u, y, v->mu_q, nullptr, nullptr, nullptr,
                      false, work);
    check_launch();
    return WB_OK;
  });
}

wb_status wb_apply_B(const wb_mesh* mh, const double* u, double* p, void* stream) {
  return guard([&] {
    WB_REQUIRE(mh && u && p, WB_EINVAL, "NULL argument");
    const Mesh& m = mh->m;
    WB_REQUIRE(m.k >= 2, WB_EUNSUPPORTED, "B needs k >= 2");
    launch_op<double>(S(stream), F_B | F_DIR, 3, m.N, m.k, u, nullptr, nullptr, nullptr, p, nullptr,
                      false, nullptr);
    check_launch();
    return WB_OK;
  });
}

wb_status wb_apply_BT(const wb_mesh* mh, const double* p, double* u, void* stream) {
  return guard([&] {
    WB_REQUIRE(mh && u && p, WB_EINVAL, "NULL argument");
    const Mesh& m = mh->m;
    WB_REQUIRE(m.k >= 2, WB_EUNSUPPORTED, "B^T needs k >= 2");
    launch_op<double>(S(stream), F_BT | F_DIR, 3, m.N, m.k, nullptr, u, nullptr, p, nullptr, nullptr,
                      false, mesh_work(mh));
    check_launch();
    return WB_OK;
  });
}

wb_status wb_apply_stokes(const wb_mesh* mh, const wb_visc* v, const double* u, const double* p,
                          double* yu, double* yp, void* stream) {
  return guard([&] {
    WB_REQUIRE(mh && v && u && p && yu && yp, WB_EINVAL, "NULL argument");
    WB_REQUIRE(u != yu, WB_EINVAL, "in-place apply is not allowed");
    const Mesh& m = mh->m;
    WB_REQUIRE(m.k >= 2, WB_EUNSUPPORTED, "Stokes operator needs k >= 2");
    launch_op<double>(S(stream), F_A | F_BT | F_B | F_DIR, 3, m.N, m.k, u, yu, v->mu_q, p, yp, nullptr,
                      false, mesh_work(mh));
    check_launch();
    return WB_OK;
  });
}

wb_status wb_apply_A_lowp(const wb_mesh* mh, const wb_visc* vc, int prec, const float* u, float* y,
                          void* stream) {
  return guard([&] {
    WB_REQUIRE(mh && vc && u && y, WB_EINVAL, "NULL argument");
    WB_REQUIRE(u != y, WB_EINVAL, "in-place apply is not allowed");
    WB_REQUIRE(prec == WB_FP32 || prec == WB_BF16 || prec == WB_BF16X1, WB_EINVAL,
               "prec must be WB_FP32, WB_BF16 or WB_BF16X1");
    const Mesh& m = mh->m;
    wb_visc* v = const_cast<wb_visc*>(vc);
    const size_t nq = (size_t)m.E * m.n * m.n * m.n;
    if (!v->mu_q_f) {
      WB_HIP(hipMalloc(&v->mu_q_f, sizeof(float) * nq));
      launch_cast<double, float>(S(stream), nq, v->mu_q, v->mu_q_f);
    }
    const int mf = prec == WB_BF16 ? F_MF3 : (prec == WB_BF16X1 ? F_MF : 0);
    launch_op<float>(S(stream), F_A | F_DIR | mf, 3, m.N, m.k, u, y,
                     v->mu_q_f, nullptr, nullptr, nullptr, false, mesh_work(mh));
    check_launch();
    return WB_OK;
  });
}

namespace {
int lowp_flag(int prec, int k) {
  WB_REQUIRE(prec == WB_FP32 || prec == WB_BF16 || prec == WB_BF16X1, WB_EINVAL,
             "prec must be WB_FP32, WB_BF16 or WB_BF16X1");
  WB_REQUIRE(k >= 2, WB_EUNSUPPORTED, "B and B^T need k >= 2");
  WB_REQUIRE(prec == WB_FP32 || k <= 4, WB_EUNSUPPORTED, "the BF16 forms are built for k <= 4");
  return prec == WB_BF16 ? F_MF3 : (prec == WB_BF16X1 ? F_MF : 0);
}
}  // namespace

wb_status wb_apply_B_lowp(const wb_mesh* mh, int prec, const float* u, float* p, void* stream) {
  return guard([&] {
    WB_REQUIRE(mh && u && p, WB_EINVAL, "NULL argument");
    const Mesh& m = mh->m;
    const int mf = lowp_flag(prec, m.k);
    launch_op<float>(S(stream), F_B | F_DIR | mf, 3, m.N, m.k, u, nullptr, nullptr, nullptr, p,
                     nullptr, false, nullptr);
    check_launch();
    return WB_OK;
  });
}

wb_status wb_apply_BT_lowp(const wb_mesh* mh, int prec, const float* p, float* u, void* stream) {
  return guard([&] {
    WB_REQUIRE(mh && u && p, WB_EINVAL, "NULL argument");
    const Mesh& m = mh->m;
    const int mf = lowp_flag(prec, m.k);
    launch_op<float>(S(stream), F_BT | F_DIR | mf, 3, m.N, m.k, nullptr, u, nullptr, p, nullptr,
                     nullptr, false, mesh_work(mh));
    check_launch();
    return WB_OK;
  });
}

wb_status wb_solver_create(const wb_mesh* mh, const wb_visc* v, const wb_opts* opts, void* stream,
                           wb_solver** out) {
  return guard([&] {
    WB_REQUIRE(mh && v && out, WB_EINVAL, "NULL argument");
    wb_opts o;
    if (opts) o = *opts;
    else wb_opts_default(&o);
    Solver* s = solver_create(mh->m, v->mu_q, v->mu_nodes, o, S(stream));
    check_launch();
    *out = reinterpret_cast<wb_solver*>(s);
    return WB_OK;
  });
}

void wb_solver_destroy(wb_solver* s) { delete reinterpret_cast<Solver*>(s); }

static Solver& SV(wb_solver* s) {
  WB_REQUIRE(s, WB_EINVAL, "solver is NULL");
  return *reinterpret_cast<Solver*>(s);
}

wb_status wb_apply_wbfbt(wb_solver* sh, const double* r, double* z, void* stream) {
  return guard([&] {
    Solver& s = SV(sh);
    WB_REQUIRE(r && z && r != z, WB_EINVAL, "bad vectors");
    s.st = S(stream);
    apply_wbfbt<double>(s, *s.pd, r, z);
    check_launch();
    return WB_OK;
  });
}

wb_status wb_apply_vcycle_A(wb_solver* sh, const double* r, double* z, void* stream) {
  return guard([&] {
    Solver& s = SV(sh);
    WB_REQUIRE(r && z && r != z, WB_EINVAL, "bad vectors");
    s.st = S(stream);
    apply_vcycle_A<double>(s, *s.pd, r, z);
    check_launch();
    return WB_OK;
  });
}

wb_status wb_apply_K(wb_solver* sh, int side, const double* p, double* y, void* stream) {
  return guard([&] {
    Solver& s = SV(sh);
    WB_REQUIRE(side == 0 || side == 1, WB_EINVAL, "side must be 0 (left) or 1 (right)");
    WB_REQUIRE(p && y && p != y, WB_EINVAL, "bad vectors");
    s.st = S(stream);
    apply_K<double>(s, *s.pd, side, p, y);
    check_launch();
    return WB_OK;
  });
}

wb_status wb_apply_vcycle_K(wb_solver* sh, int side, const double* r, double* z, void* stream) {
  return guard([&] {
    Solver& s = SV(sh);
    WB_REQUIRE(side == 0 || side == 1, WB_EINVAL, "side must be 0 (left) or 1 (right)");
    WB_REQUIRE(r && z && r != z, WB_EINVAL, "bad vectors");
    s.st = S(stream);
    apply_vcycle_K<double>(s, *s.pd, side, r, z);
    check_launch();
    return WB_OK;
  });
}

wb_status wb_apply_precond(wb_solver* sh, const double* ru, const double* rp, double* zu, double* zp,
                           void* stream) {
  return guard([&] {
    Solver& s = SV(sh);
    WB_REQUIRE(ru && rp && zu && zp, WB_EINVAL, "bad vectors");
    s.st = S(stream);
    apply_precond_any(s, ru, rp, zu, zp);
    check_launch();
    return WB_OK;
  });
}

wb_status wb_solve(wb_solver* sh, const double* f, double* u, double* p, wb_report* rep,
                   void* stream) {
  return guard([&] {
    Solver& s = SV(sh);
    WB_REQUIRE(f && u && p, WB_EINVAL, "bad vectors");
    s.st = S(stream);
    wb_status r = fgmres(s, f, u, p, rep);
    check_launch();
    if (r == WB_ENOCONV) set_error("FGMRES reached max_iter before rtol");
    return r;
  });
}

wb_status wb_subsolve(wb_solver* sh, int which, const double* b, double* x, wb_report* rep,
                      void* stream) {
  return guard([&] {
    Solver& s = SV(sh);
    WB_REQUIRE(which >= 0 && which <= 2, WB_EINVAL, "which must be 0 (A), 1 (K_l) or 2 (K_r)");
    WB_REQUIRE(b && x && b != x, WB_EINVAL, "bad vectors");
    s.st = S(stream);
    wb_status r = subsolve(s, which, b, x, rep);
    check_launch();
    if (r == WB_ENOCONV) set_error("GMRES reached max_iter before rtol");
    return r;
  });
}

wb_status wb_solver_query(wb_solver* sh, int what, int level, double* out, void* stream) {
  return guard([&] {
    Solver& s = SV(sh);
    WB_REQUIRE(out, WB_EINVAL, "out is NULL");
    hipStream_t st = S(stream);
    Precond<double>& P = *s.pd;
    const Mesh& m = s.m;
    auto cp = [&](const double* src, size_t n) {
      WB_HIP(hipMemcpyAsync(out, src, sizeof(double) * n, hipMemcpyDeviceToDevice, st));
    };
    auto lev = [&](Hierarchy<double>& H) -> Level<double>& {
      WB_REQUIRE(level >= 0 && level < (int)H.L.size(), WB_EINVAL, "level out of range");
      return H.L[level];
    };
    switch (what) {
      case 0: cp(P.winv[0], (s.o.weights == 2 ? 3 : 1) * (size_t)m.nn); break;
      case 1: cp(P.winv[1], (s.o.weights == 2 ? 3 : 1) * (size_t)m.nn); break;
      case 2: { auto& L = lev(P.A); cp(L.dinv, L.len); } break;
      case 3: { auto& L = lev(P.A); cp(L.coef, (size_t)L.E * (L.k + 1) * (L.k + 1) * (L.k + 1)); } break;
      case 4: cp(P.dk[0], (size_t)m.E * m.np); break;
      case 5: cp(P.dk[1], (size_t)m.E * m.np); break;
      case 6: { auto& L = lev(P.Pois[0]); cp(L.coef, (size_t)L.E * (L.k + 1) * (L.k + 1) * (L.k + 1)); } break;
      case 7: { auto& L = lev(P.Pois[1]); cp(L.coef, (size_t)L.E * (L.k + 1) * (L.k + 1) * (L.k + 1)); } break;
      case 8: { auto& L = lev(P.Pois[0]); cp(L.dinv, L.len); } break;
      case 9: cp(P.mpinv, (size_t)m.E * m.np); break;
      default: throw Error{WB_EINVAL, "unknown query"};
    }
    WB_HIP(hipStreamSynchronize(st));
    return WB_OK;
  });
}

wb_status wb_solver_levels(wb_solver* sh, int which, int* nlevels, int* Ns, int* ks, double* lmax) {
  return guard([&] {
    Solver& s = SV(sh);
    Precond<double>& P = *s.pd;
    if (which == 3) {
      if (nlevels) *nlevels = 2;
      for (int i = 0; i < 2; ++i) {
        if (Ns) Ns[i] = s.m.N;
        if (ks) ks[i] = s.m.k;
        if (lmax) lmax[i] = P.klmax[i];
      }
      return WB_OK;
    }
    WB_REQUIRE(which >= 0 && which <= 2, WB_EINVAL, "which must be 0..3");
    Hierarchy<double>& H = which == 0 ? P.A : P.Pois[which - 1];
    const int nl = (int)H.L.size();
    if (nlevels) *nlevels = nl;
    for (int i = 0; i < nl && i < 16; ++i) {
      if (Ns) Ns[i] = H.L[i].N;
      if (ks) ks[i] = H.L[i].k;
      if (lmax) lmax[i] = H.L[i].lmax;
    }
    return WB_OK;
  });
}

void wb_profile_enable(int on) { profile_enable(on != 0); }

double wb_set_two_pass_limit(double mb) { return set_two_pass_limit(mb); }

int wb_set_matrix_core_ops(int on) { return set_matrix_core_ops(on); }

long long wb_profile_summary(char* buf, long long len, int reset) {
  std::string s = profile_summary(reset != 0);
  if (buf && len > 0) {
    const size_t n = std::min<size_t>((size_t)len - 1, s.size());
    std::memcpy(buf, s.data(), n);
    buf[n] = 0;
  }
  return (long long)s.size();
}

wb_status wb_apply_A_add(const wb_mesh* mh, const wb_visc* v, const double* u, double* y, void* stream) {
  return guard([&] {
    WB_REQUIRE(mh && v && u && y, WB_EINVAL, "NULL argument");
    WB_REQUIRE(u != y, WB_EINVAL, "in-place apply is not allowed");
    const Mesh& m = mh->m;
    launch_op<double>(S(stream), F_A | F_DIR, 3, m.N, m.k, u, y, v->mu_q, nullptr, nullptr, nullptr,
                      true, mesh_work(mh));
    check_launch();
    return WB_OK;
  });
}

void wb_train_opts_default(wb_train_opts* o) {
  if (!o) return;
  const TrainOpts d;
  o->pairs_per_field = d.pairs_per_field;
  o->vcycles = d.vcycles;
  o->epochs = d.epochs;
  o->batch = d.batch;
  o->lr = d.lr;
  o->seed = d.seed;
  o->delta = d.delta;
  o->omega = d.omega;
  o->mu_min = d.mu_min;
  o->mu_max = d.mu_max;
  o->n_valid = d.n_valid;
}

wb_status wb_learned_train(wb_solver* sh, int n_fields, const int* n_sinkers,
                           const double* centers_host, const wb_train_opts* opts,
                           wb_train_report* rep, void* stream) {
  return guard([&] {
    Solver& s = SV(sh);
    WB_REQUIRE(opts && n_sinkers, WB_EINVAL, "NULL argument");
    s.st = S(stream);
    TrainOpts o;
    o.pairs_per_field = opts->pairs_per_field;
    o.vcycles = opts->vcycles;
    o.epochs = opts->epochs;
    o.batch = opts->batch;
    o.lr = opts->lr;
    o.seed = opts->seed;
    o.delta = opts->delta;
    o.omega = opts->omega;
    o.mu_min = opts->mu_min;
    o.mu_max = opts->mu_max;
    o.n_valid = opts->n_valid;
    TrainReport r;
    learned_train(s, n_fields, n_sinkers, centers_host, o, &r);
    check_launch();
    if (rep) {
      rep->loss_first = r.loss_first;
      rep->loss_last = r.loss_last;
      rep->valid_loss = r.valid_loss;
      rep->t_pairs_s = r.t_pairs_s;
      rep->t_train_s = r.t_train_s;
      rep->n_params = r.n_params;
      rep->n_pairs = r.n_pairs;
    }
    return WB_OK;
  });
}

wb_status wb_learned_get(wb_solver* sh, float* params, long long* n_params) {
  return guard([&] {
    Solver& s = SV(sh);
    WB_REQUIRE(s.learned, WB_EUNSUPPORTED, "no learned level (Q1 on N/2) on this mesh");
    if (n_params) *n_params = (long long)net_param_count();
    if (params) {
      WB_HIP(hipMemcpy(params, s.learned->params, sizeof(float) * net_param_count(),
                       hipMemcpyDeviceToHost));
    }
    return WB_OK;
  });
}

wb_status wb_learned_set(wb_solver* sh, const float* params, long long n_params) {
  return guard([&] {
    Solver& s = SV(sh);
    WB_REQUIRE(params, WB_EINVAL, "NULL parameters");
    WB_REQUIRE(n_params == (long long)net_param_count(), WB_EINVAL, "parameter count mismatch");
    learned_set(s, params);
    return WB_OK;
  });
}

wb_status wb_learned_info(wb_solver* sh, int* level, int* M, long long* n_params) {
  return guard([&] {
    Solver& s = SV(sh);
    WB_REQUIRE(s.learned, WB_EUNSUPPORTED, "no learned level (Q1 on N/2) on this mesh");
    if (level) *level = s.learned->lc;
    if (M) *M = s.learned->M;
    if (n_params) *n_params = (long long)net_param_count();
    return WB_OK;
  });
}

wb_status wb_learned_probe(wb_solver* sh, const double* r, double* delta, double* alpha,
                           void* stream) {
  return guard([&] {
    Solver& s = SV(sh);
    WB_REQUIRE(r && delta && alpha && r != delta, WB_EINVAL, "bad arguments");
    s.st = S(stream);
    learned_probe(s, r, delta, alpha);
    check_launch();
    return WB_OK;
  });
}

void wb_mem_trim(void) { mem_trim(); }

long long wb_net_param_count(void) { return (long long)net_param_count(); }

wb_status wb_net_eval(int M, int B, const float* params, const float* x, const float* t,
                      const float* w, float* out, float* grad, double* loss, void* stream) {
  return guard([&] {
    WB_REQUIRE(M >= 2 && M <= 1025 && B >= 1, WB_EINVAL, "bad grid or batch");
    WB_REQUIRE(params && x && out, WB_EINVAL, "NULL argument");
    WB_REQUIRE((t == nullptr) == (w == nullptr) && (grad == nullptr) == (t == nullptr), WB_EINVAL,
               "t, w and grad must be given together");
    hipStream_t st = S(stream);
    void* base = nullptr;
    WB_HIP(hipMalloc(&base, net_work_bytes(M, B)));
    double* dl = nullptr;
    if (hipMalloc(&dl, sizeof(double)) != hipSuccess) {
      (void)hipFree(base);
      throw Error{WB_ENOMEM, "hipMalloc failed"};
    }
    NetWork nw;
    net_work_carve(nw, M, B, base);
    net_forward(st, params, x, nw);
    if (t) net_backward(st, params, x, t, w, nw, grad, dl);
    const size_t n = (size_t)B * 3 * M * M * M;
    hipError_t e = hipMemcpyAsync(out, nw.z[3], sizeof(float) * n, hipMemcpyDeviceToDevice, st);
    double lh = 0.0;
    if (e == hipSuccess && t) e = hipMemcpyAsync(&lh, dl, sizeof(double), hipMemcpyDeviceToHost, st);
    if (e == hipSuccess) e = hipStreamSynchronize(st);
    (void)hipFree(base);
    (void)hipFree(dl);
    if (e != hipSuccess) throw Error{WB_EHIP, hipGetErrorString(e)};
    if (loss) *loss = lh;
    check_launch();
    return WB_OK;
  });
}

wb_status wb_net_adam(long long n, float* params, const float* grad, float* m, float* v, int step,
                      double lr, void* stream) {
  return guard([&] {
    WB_REQUIRE(n > 0 && params && grad && m && v && step >= 1 && lr > 0, WB_EINVAL, "bad arguments");
    net_adam(S(stream), (size_t)n, params, grad, m, v, step, (float)lr);
    check_launch();
    return WB_OK;
  });
}

wb_status wb_net_feature(int N, const double* coef, float* feat, void* stream) {
  return guard([&] {
    WB_REQUIRE(N >= 1 && N <= 1024 && coef && feat, WB_EINVAL, "bad arguments");
    float* tmp = nullptr;
    WB_HIP(hipMalloc(&tmp, sizeof(float) * (size_t)N * N * N));
    launch_node_feature(S(stream), N, coef, feat, tmp);
    const hipError_t e = hipStreamSynchronize(S(stream));
    (void)hipFree(tmp);
    if (e != hipSuccess) throw Error{WB_EHIP, hipGetErrorString(e)};
    check_launch();
    return WB_OK;
  });
}

}  // extern "C"
