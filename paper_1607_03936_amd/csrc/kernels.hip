// HIP kernels (gfx950) of the w-BFBT Stokes hot path.
//
// Operators are matrix-free and sum-factorized: per element the (k+1)^3 nodal
// values are interpolated to the (k+1)^3 Gauss points by three 1D contractions,
// differentiated there with the collocation derivative of the Gauss-Lagrange
// basis, multiplied by the pointwise coefficient and pulled back by the
// transposed contractions (Sec. 1.2 discretization, eq. 2).  Thread layout:
// n^2 threads per element, each holding a z-column in registers; x and y
// contractions exchange through LDS.
#include <algorithm>
#include <cmath>
#include <cstdio>
#include <map>
#include <mutex>
#include <string>
#include <vector>

#include "kernels.h"

namespace wb {

// ------------------------------------------------------------------ profiling
// Optional HIP-event timing of operator launches, keyed by kernel class.
namespace prof {
struct Rec {
  std::string key;
  hipEvent_t a, b;
};
static std::mutex mu;
static bool on = false;
static std::vector<Rec> recs;
static std::vector<hipEvent_t> pool;

static hipEvent_t get_event() {
  if (!pool.empty()) {
    hipEvent_t e = pool.back();
    pool.pop_back();
    return e;
  }
  hipEvent_t e;
  if (hipEventCreate(&e) != hipSuccess) return nullptr;
  return e;
}
}  // namespace prof

void profile_enable(bool on) {
  std::lock_guard<std::mutex> g(prof::mu);
  prof::on = on;
}

std::string profile_summary(bool reset) {
  std::lock_guard<std::mutex> g(prof::mu);
  std::map<std::string, std::pair<long, double>> agg;
  for (auto& r : prof::recs) {
    float ms = 0.f;
    if (hipEventSynchronize(r.b) == hipSuccess && hipEventElapsedTime(&ms, r.a, r.b) == hipSuccess) {
      auto& x = agg[r.key];
      x.first += 1;
      x.second += ms;
    }
  }
  std::string out;
  for (auto& kv : agg) {
    char line[256];
    snprintf(line, sizeof(line), "%s\t%ld\t%.6f\n", kv.first.c_str(), kv.second.first, kv.second.second);
    out += line;
  }
  if (reset) {
    for (auto& r : prof::recs) {
      prof::pool.push_back(r.a);
      prof::pool.push_back(r.b);
    }
    prof::recs.clear();
  }
  return out;
}

namespace {

// Per-order tables passed to kernels by value (kernel-argument memory).
template <int n, typename T>
struct KT {
  T B[n * n], D1[n * n], Dh[n * n], L[n * n], J[n * n];
  T w[n], xg[n], wl[n];
  int np;
  unsigned char ma[NPMAX], mb[NPMAX], mc[NPMAX];
};

template <int n, typename T>
KT<n, T> make_kt(int k) {
  const Tables& tb = tables(k);
  KT<n, T> o;
  for (int i = 0; i < n * n; ++i) {
    o.B[i] = (T)tb.B[i];
    o.D1[i] = (T)tb.D1[i];
    o.Dh[i] = (T)tb.Dh[i];
    o.L[i] = (T)tb.L[i];
    o.J[i] = (T)tb.J[i];
  }
  for (int i = 0; i < n; ++i) {
    o.w[i] = (T)tb.wg[i];
    o.xg[i] = (T)tb.xg[i];
    o.wl[i] = (T)tb.wl[i];
  }
  o.np = tb.np;
  for (int m = 0; m < NPMAX; ++m) {
    o.ma[m] = (unsigned char)tb.ma[m];
    o.mb[m] = (unsigned char)tb.mb[m];
    o.mc[m] = (unsigned char)tb.mc[m];
  }
  return o;
}

__device__ inline void atomic_add(double* p, double v) { unsafeAtomicAdd(p, v); }
__device__ inline void atomic_add(float* p, float v) { unsafeAtomicAdd(p, v); }

inline unsigned grid_for(size_t n, int bs) { return (unsigned)((n + bs - 1) / bs); }

// ------------------------------------------------------------------ operator
template <int n, int NC, typename T, int F>
__global__ void __launch_bounds__(256)
k_op(const KT<n, T> tb, const int N, const int k, const int M, const int E, const int nn,
     const T hh, const T* __restrict__ u, T* __restrict__ y, const T* __restrict__ coef,
     const T* __restrict__ pin, T* __restrict__ pout, const T* __restrict__ sin_,
     const T* __restrict__ sout) {
  constexpr int NN = n * n, N3 = n * n * n, EPB = 256 / NN;
  constexpr int NP = (n - 1) * n * (n + 1) / 6;
  __shared__ T sm[NC][EPB][N3];
  const int t = threadIdx.x, le = t / NN, r = t - le * NN, i = r % n, j = r / n;
  const int e = blockIdx.x * EPB + le;
  const bool valid = e < E;
  int ex = 0, ey = 0, ez = 0;
  if (valid) {
    ex = e % N;
    const int q = e / N;
    ey = q % N;
    ez = q / N;
  }
  const int gi = ex * k + i, gj = ey * k + j;
  const bool bij = (gi == 0) || (gi == M - 1) || (gj == 0) || (gj == M - 1);

  T S[NC][3][n];
  T bq[n];
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int d = 0; d < 3; ++d)
#pragma unroll
      for (int q = 0; q < n; ++q) S[c][d][q] = T(0);

  if constexpr ((F & (F_A | F_B)) != 0) {
    T U[NC][n];
#pragma unroll
    for (int l = 0; l < n; ++l) {
      const int gl = ez * k + l;
      const int g = gi + M * (gj + M * gl);
      const bool bnd = (F & F_DIR) && (bij || gl == 0 || gl == M - 1);
      T s = T(1);
      if (sin_ != nullptr && valid) s = sin_[g];
#pragma unroll
      for (int c = 0; c < NC; ++c) U[c][l] = (valid && !bnd) ? u[(size_t)c * nn + g] * s : T(0);
    }
    // interpolation to Gauss points: z in registers
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      T tmp[n];
#pragma unroll
      for (int q = 0; q < n; ++q) {
        T a = T(0);
#pragma unroll
        for (int l = 0; l < n; ++l) a += tb.B[q * n + l] * U[c][l];
        tmp[q] = a;
      }
#pragma unroll
      for (int q = 0; q < n; ++q) U[c][q] = tmp[q];
    }
    // y
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int q = 0; q < n; ++q) sm[c][le][q * NN + j * n + i] = U[c][q];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int q = 0; q < n; ++q) {
        T a = T(0);
#pragma unroll
        for (int b = 0; b < n; ++b) a += tb.B[j * n + b] * sm[c][le][q * NN + b * n + i];
        U[c][q] = a;
      }
    __syncthreads();
    // x
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int q = 0; q < n; ++q) sm[c][le][q * NN + j * n + i] = U[c][q];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int q = 0; q < n; ++q) {
        T a = T(0);
#pragma unroll
        for (int b = 0; b < n; ++b) a += tb.B[i * n + b] * sm[c][le][q * NN + j * n + b];
        U[c][q] = a;
      }
    __syncthreads();
    // collocation derivatives at the Gauss points
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int q = 0; q < n; ++q) sm[c][le][q * NN + j * n + i] = U[c][q];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int q = 0; q < n; ++q) {
        T gx = T(0), gy = T(0), gz = T(0);
#pragma unroll
        for (int b = 0; b < n; ++b) {
          gx += tb.Dh[i * n + b] * sm[c][le][q * NN + j * n + b];
          gy += tb.Dh[j * n + b] * sm[c][le][q * NN + b * n + i];
          gz += tb.Dh[q * n + b] * U[c][b];
        }
        S[c][0][q] = gx;
        S[c][1][q] = gy;
        S[c][2][q] = gz;
      }
    __syncthreads();
    // pointwise
#pragma unroll
    for (int q = 0; q < n; ++q) {
      const T w3 = tb.w[i] * tb.w[j] * tb.w[q];
      if constexpr (NC == 3) {
        if constexpr ((F & F_B) != 0) bq[q] = -hh * hh * w3 * (S[0][0][q] + S[1][1][q] + S[2][2][q]);
        if constexpr ((F & F_A) != 0) {
          const T cw = valid ? coef[(size_t)e * N3 + q * NN + j * n + i] * w3 * hh : T(0);
          const T s01 = cw * (S[0][1][q] + S[1][0][q]);
          const T s02 = cw * (S[0][2][q] + S[2][0][q]);
          const T s12 = cw * (S[1][2][q] + S[2][1][q]);
          S[0][0][q] = T(2) * cw * S[0][0][q];
          S[1][1][q] = T(2) * cw * S[1][1][q];
          S[2][2][q] = T(2) * cw * S[2][2][q];
          S[0][1][q] = S[1][0][q] = s01;
          S[0][2][q] = S[2][0][q] = s02;
          S[1][2][q] = S[2][1][q] = s12;
        } else {
#pragma unroll
          for (int c = 0; c < 3; ++c)
#pragma unroll
            for (int d = 0; d < 3; ++d) S[c][d][q] = T(0);
        }
      } else {
        const T cw = valid ? coef[(size_t)e * N3 + q * NN + j * n + i] * w3 * hh : T(0);
#pragma unroll
        for (int d = 0; d < 3; ++d) S[0][d][q] *= cw;
      }
    }
  }

  if constexpr (NC == 3 && (F & F_B) != 0) {
    // project -(h/2)^2 w3 div u onto the Legendre modes
#pragma unroll
    for (int c = 0; c < n - 1; ++c) {
      T a = T(0);
#pragma unroll
      for (int q = 0; q < n; ++q) a += tb.L[c * n + q] * bq[q];
      sm[0][le][c * NN + j * n + i] = a;
    }
    __syncthreads();
    if (valid && r < NP) {
      const int a = tb.ma[r], b = tb.mb[r], c = tb.mc[r];
      T s = T(0);
#pragma unroll
      for (int jj = 0; jj < n; ++jj)
#pragma unroll
        for (int ii = 0; ii < n; ++ii)
          s += tb.L[a * n + ii] * tb.L[b * n + jj] * sm[0][le][c * NN + jj * n + ii];
      pout[(size_t)e * NP + r] = s;
    }
    __syncthreads();
  }

  if constexpr (NC == 3 && (F & F_BT) != 0) {
    T pm[NP];
#pragma unroll
    for (int m = 0; m < NP; ++m) pm[m] = valid ? pin[(size_t)e * NP + m] : T(0);
#pragma unroll
    for (int q = 0; q < n; ++q) {
      T pq = T(0);
#pragma unroll
      for (int m = 0; m < NP; ++m)
        pq += pm[m] * tb.L[tb.ma[m] * n + i] * tb.L[tb.mb[m] * n + j] * tb.L[tb.mc[m] * n + q];
      const T v = -hh * hh * tb.w[i] * tb.w[j] * tb.w[q] * pq;
      S[0][0][q] += v;
      S[1][1][q] += v;
      S[2][2][q] += v;
    }
  }

  if constexpr ((F & (F_A | F_BT)) != 0) {
    T V[NC][n];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int q = 0; q < n; ++q) {
        T a = T(0);
#pragma unroll
        for (int m = 0; m < n; ++m) a += tb.Dh[m * n + q] * S[c][2][m];
        V[c][q] = a;
      }
    // x-derivative transpose
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int q = 0; q < n; ++q) sm[c][le][q * NN + j * n + i] = S[c][0][q];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int q = 0; q < n; ++q) {
        T a = T(0);
#pragma unroll
        for (int b = 0; b < n; ++b) a += tb.Dh[b * n + i] * sm[c][le][q * NN + j * n + b];
        V[c][q] += a;
      }
    __syncthreads();
    // y-derivative transpose
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int q = 0; q < n; ++q) sm[c][le][q * NN + j * n + i] = S[c][1][q];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int q = 0; q < n; ++q) {
        T a = T(0);
#pragma unroll
        for (int b = 0; b < n; ++b) a += tb.Dh[b * n + j] * sm[c][le][q * NN + b * n + i];
        V[c][q] += a;
      }
    __syncthreads();
    // x interpolation transpose
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int q = 0; q < n; ++q) sm[c][le][q * NN + j * n + i] = V[c][q];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int q = 0; q < n; ++q) {
        T a = T(0);
#pragma unroll
        for (int b = 0; b < n; ++b) a += tb.B[b * n + i] * sm[c][le][q * NN + j * n + b];
        V[c][q] = a;
      }
    __syncthreads();
    // y interpolation transpose
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int q = 0; q < n; ++q) sm[c][le][q * NN + j * n + i] = V[c][q];
    __syncthreads();
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int q = 0; q < n; ++q) {
        T a = T(0);
#pragma unroll
        for (int b = 0; b < n; ++b) a += tb.B[b * n + j] * sm[c][le][q * NN + b * n + i];
        V[c][q] = a;
      }
    // z interpolation transpose and scatter
#pragma unroll
    for (int l = 0; l < n; ++l) {
      const int gl = ez * k + l;
      const int g = gi + M * (gj + M * gl);
      const bool bnd = (F & F_DIR) && (bij || gl == 0 || gl == M - 1);
      if (valid && !bnd) {
        T s = T(1);
        if (sout != nullptr) s = sout[g];
#pragma unroll
        for (int c = 0; c < NC; ++c) {
          T a = T(0);
#pragma unroll
          for (int q = 0; q < n; ++q) a += tb.B[q * n + l] * V[c][q];
          atomic_add(&y[(size_t)c * nn + g], a * s);
        }
      }
    }
  }
}

template <int n, int NC, typename T, int F>
void op_launch(hipStream_t st, int N, int k, const T* u, T* y, const T* coef, const T* pin, T* pout,
               const T* sin, const T* sout) {
  constexpr int NN = n * n, EPB = 256 / NN;
  const int M = k * N + 1, E = N * N * N, nn = M * M * M;
  const T hh = (T)(0.5 / N);
  const KT<n, T> tb = make_kt<n, T>(k);
  hipEvent_t ea = nullptr, eb = nullptr;
  if (prof::on) {
    std::lock_guard<std::mutex> g(prof::mu);
    ea = prof::get_event();
    eb = prof::get_event();
    if (ea) (void)hipEventRecord(ea, st);
  }
  hipLaunchKernelGGL((k_op<n, NC, T, F>), dim3(grid_for(E, EPB)), dim3(EPB * NN), 0, st, tb, N, k,
                     M, E, nn, hh, u, y, coef, pin, pout, sin, sout);
  if (ea && eb) {
    std::lock_guard<std::mutex> g(prof::mu);
    (void)hipEventRecord(eb, st);
    char key[160];
    snprintf(key, sizeof(key), "op nc=%d k=%d N=%d flags=%s%s%s%s%s %s", NC, k, N,
             (F & F_A) ? "A" : "", (F & F_BT) ? "+BT" : "", (F & F_B) ? "+B" : "",
             (F & F_DIR) ? "+dir" : "", sin ? "+scale" : "", sizeof(T) == 8 ? "f64" : "f32");
    prof::recs.push_back({key, ea, eb});
  }
}

template <int n, typename T>
void op_dispatch_n(hipStream_t st, int flags, int NC, int N, int k, const T* u, T* y, const T* coef,
                   const T* pin, T* pout, const T* sin, const T* sout) {
  if (NC == 1) {
    if (flags == F_A)
      return op_launch<n, 1, T, F_A>(st, N, k, u, y, coef, pin, pout, sin, sout);
    if (flags == (F_A | F_DIR))
      return op_launch<n, 1, T, F_A | F_DIR>(st, N, k, u, y, coef, pin, pout, sin, sout);
  } else {
    switch (flags) {
      case F_A | F_DIR:
        return op_launch<n, 3, T, F_A | F_DIR>(st, N, k, u, y, coef, pin, pout, sin, sout);
      case F_A | F_BT | F_B | F_DIR:
        return op_launch<n, 3, T, F_A | F_BT | F_B | F_DIR>(st, N, k, u, y, coef, pin, pout, sin,
                                                             sout);
      case F_B | F_DIR:
        return op_launch<n, 3, T, F_B | F_DIR>(st, N, k, u, y, coef, pin, pout, sin, sout);
      case F_BT | F_DIR:
        return op_launch<n, 3, T, F_BT | F_DIR>(st, N, k, u, y, coef, pin, pout, sin, sout);
      default:
        break;
    }
  }
  throw Error{WB_EUNSUPPORTED, "operator flag combination not built"};
}

// ------------------------------------------------------------------ diagonals
template <int n, int NC>
__global__ void k_diag(const KT<n, double> tb, int N, int k, int M, int E, int nn, double hh, int dir,
                       const double* __restrict__ coef, double* __restrict__ diag) {
  constexpr int NN = n * n, N3 = NN * n;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)E * N3) return;
  const int e = (int)(idx / N3), li = (int)(idx % N3);
  const int a = li % n, b = (li / n) % n, c = li / NN;
  const int ex = e % N, ey = (e / N) % N, ez = e / (N * N);
  const int gi = ex * k + a, gj = ey * k + b, gl = ez * k + c;
  if (dir && (gi == 0 || gi == M - 1 || gj == 0 || gj == M - 1 || gl == 0 || gl == M - 1)) return;
  double sall = 0, sx = 0, sy = 0, sz = 0;
  for (int qz = 0; qz < n; ++qz)
    for (int qy = 0; qy < n; ++qy)
      for (int qx = 0; qx < n; ++qx) {
        const double cw = coef[(size_t)e * N3 + qz * NN + qy * n + qx] * tb.w[qx] * tb.w[qy] *
                          tb.w[qz] * hh;
        const double gx = tb.D1[qx * n + a] * tb.B[qy * n + b] * tb.B[qz * n + c];
        const double gy = tb.B[qx * n + a] * tb.D1[qy * n + b] * tb.B[qz * n + c];
        const double gz = tb.B[qx * n + a] * tb.B[qy * n + b] * tb.D1[qz * n + c];
        sx += cw * gx * gx;
        sy += cw * gy * gy;
        sz += cw * gz * gz;
      }
  sall = sx + sy + sz;
  const int g = gi + M * (gj + M * gl);
  if (NC == 1) {
    atomic_add(&diag[g], sall);
  } else {
    atomic_add(&diag[g], sall + sx);
    atomic_add(&diag[(size_t)nn + g], sall + sy);
    atomic_add(&diag[2 * (size_t)nn + g], sall + sz);
  }
}

__global__ void k_invert_diag(int M, int NC, int dir, double* d) {
  const long long nn = (long long)M * M * M;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nn * NC) return;
  const long long g = idx % nn;
  const int gi = (int)(g % M), gj = (int)((g / M) % M), gl = (int)(g / ((long long)M * M));
  const bool bnd = gi == 0 || gi == M - 1 || gj == 0 || gj == M - 1 || gl == 0 || gl == M - 1;
  d[idx] = (dir && bnd) ? 1.0 : 1.0 / d[idx];
}

template <int n>
__global__ void k_lumped(const KT<n, double> tb, int N, int k, int M, int E, double h3, double amp,
                         const double* __restrict__ mu_nodes, double* __restrict__ cn) {
  constexpr int NN = n * n, N3 = NN * n;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)E * N3) return;
  const int e = (int)(idx / N3), li = (int)(idx % N3);
  const int a = li % n, b = (li / n) % n, c = li / NN;
  const int ex = e % N, ey = (e / N) % N, ez = e / (N * N);
  const bool touch = ex == 0 || ex == N - 1 || ey == 0 || ey == N - 1 || ez == 0 || ez == N - 1;
  const int g = (ex * k + a) + M * ((ey * k + b) + M * (ez * k + c));
  const double ae = touch ? amp : 1.0;
  atomic_add(&cn[g], ae * sqrt(mu_nodes[g]) * tb.wl[a] * tb.wl[b] * tb.wl[c] * h3);
}

template <int n>
__global__ void k_diag_K(int N, int k, int M, int E, int np, double s2, const double* __restrict__ bhat,
                         const double* __restrict__ dinv_nodes, double* __restrict__ dk) {
  constexpr int NN = n * n, N3 = NN * n;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)E * np) return;
  const int e = (int)(idx / np), m = (int)(idx % np);
  const int ex = e % N, ey = (e / N) % N, ez = e / (N * N);
  double s = 0.0;
  for (int li = 0; li < N3; ++li) {
    const int a = li % n, b = (li / n) % n, c = li / NN;
    const int gi = ex * k + a, gj = ey * k + b, gl = ez * k + c;
    if (gi == 0 || gi == M - 1 || gj == 0 || gj == M - 1 || gl == 0 || gl == M - 1) continue;
    const int g = gi + M * (gj + M * gl);
    const double di = dinv_nodes[g];
    for (int cc = 0; cc < 3; ++cc) {
      const double v = s2 * bhat[((size_t)m * 3 + cc) * N3 + li];
      s += v * v * di;
    }
  }
  dk[idx] = 1.0 / s;
}

// ------------------------------------------------------------------ sinker
__device__ double chi_at(double x, double y, double z, const double* __restrict__ c, int ns,
                         double delta, double omega) {
  double chi = 1.0;
  for (int s = 0; s < ns; ++s) {
    const double dx = x - c[3 * s], dy = y - c[3 * s + 1], dz = z - c[3 * s + 2];
    const double d = sqrt(dx * dx + dy * dy + dz * dz);
    const double m = fmax(0.0, d - 0.5 * omega);
    chi *= 1.0 - exp(-delta * m * m);
  }
  return chi;
}

template <int n>
__global__ void k_sinker_q(const KT<n, double> tb, int N, int E, double h, const double* c, int ns,
                           double delta, double omega, double mu_min, double mu_max, double beta,
                           double* mu_q, double* f_q) {
  constexpr int NN = n * n, N3 = NN * n;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)E * N3) return;
  const int e = (int)(idx / N3), q = (int)(idx % N3);
  const int qx = q % n, qy = (q / n) % n, qz = q / NN;
  const int ex = e % N, ey = (e / N) % N, ez = e / (N * N);
  const double x = (ex + 0.5 * (tb.xg[qx] + 1.0)) * h;
  const double y = (ey + 0.5 * (tb.xg[qy] + 1.0)) * h;
  const double z = (ez + 0.5 * (tb.xg[qz] + 1.0)) * h;
  const double chi = chi_at(x, y, z, c, ns, delta, omega);
  if (mu_q) mu_q[idx] = (mu_max - mu_min) * (1.0 - chi) + mu_min;
  if (f_q) f_q[idx] = beta * (chi - 1.0);
}

__global__ void k_sinker_nodes(int M, const double* __restrict__ x1, const double* c, int ns,
                               double delta, double omega, double mu_min, double mu_max,
                               double* mu_nodes) {
  const long long nn = (long long)M * M * M;
  const long long g = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nn) return;
  const int gi = (int)(g % M), gj = (int)((g / M) % M), gl = (int)(g / ((long long)M * M));
  const double chi = chi_at(x1[gi], x1[gj], x1[gl], c, ns, delta, omega);
  mu_nodes[g] = (mu_max - mu_min) * (1.0 - chi) + mu_min;
}

template <int n>
__global__ void k_load(const KT<n, double> tb, int N, int k, int M, int E, double h3,
                       const double* __restrict__ f_q, double* __restrict__ F) {
  constexpr int NN = n * n, N3 = NN * n;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)E * N3) return;
  const int e = (int)(idx / N3), li = (int)(idx % N3);
  const int a = li % n, b = (li / n) % n, c = li / NN;
  const int ex = e % N, ey = (e / N) % N, ez = e / (N * N);
  const int gi = ex * k + a, gj = ey * k + b, gl = ez * k + c;
  if (gi == 0 || gi == M - 1 || gj == 0 || gj == M - 1 || gl == 0 || gl == M - 1) return;
  double s = 0.0;
  for (int qz = 0; qz < n; ++qz)
    for (int qy = 0; qy < n; ++qy)
      for (int qx = 0; qx < n; ++qx)
        s += f_q[(size_t)e * N3 + qz * NN + qy * n + qx] * tb.w[qx] * tb.w[qy] * tb.w[qz] *
             tb.B[qx * n + a] * tb.B[qy * n + b] * tb.B[qz * n + c];
  const long long nn = (long long)M * M * M;
  atomic_add(&F[2 * nn + gi + (long long)M * (gj + (long long)M * gl)], s * h3);
}

__global__ void k_poisson_coef(int N, int n3, int E, double amp, const double* __restrict__ mu_q,
                               double* __restrict__ c) {
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)E * n3) return;
  const int e = (int)(idx / n3);
  const int ex = e % N, ey = (e / N) % N, ez = e / (N * N);
  const bool touch = ex == 0 || ex == N - 1 || ey == 0 || ey == N - 1 || ez == 0 || ez == N - 1;
  c[idx] = 1.0 / ((touch ? amp : 1.0) * sqrt(mu_q[idx]));
}

// ------------------------------------------------------------------ transfers
template <typename T>
__global__ void k_kron(int Mo, int Mi, int NC, int W, const int* __restrict__ cnt,
                       const int* __restrict__ col, const double* __restrict__ val, int dir, int add,
                       const T* __restrict__ in, T* __restrict__ out) {
  const long long no = (long long)Mo * Mo * Mo, ni = (long long)Mi * Mi * Mi;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= no * NC) return;
  const int c = (int)(idx / no);
  const long long o = idx % no;
  const int oi = (int)(o % Mo), oj = (int)((o / Mo) % Mo), ol = (int)(o / ((long long)Mo * Mo));
  if (dir && (oi == 0 || oi == Mo - 1 || oj == 0 || oj == Mo - 1 || ol == 0 || ol == Mo - 1)) {
    if (!add) out[idx] = T(0);
    return;
  }
  double s = 0.0;
  const T* inc = in + (size_t)c * ni;
  for (int tc = 0; tc < cnt[ol]; ++tc) {
    const double vc = val[ol * W + tc];
    const long long bc = (long long)col[ol * W + tc] * Mi * Mi;
    for (int tb = 0; tb < cnt[oj]; ++tb) {
      const double vb = vc * val[oj * W + tb];
      const long long bb = bc + (long long)col[oj * W + tb] * Mi;
      for (int ta = 0; ta < cnt[oi]; ++ta) s += vb * val[oi * W + ta] * (double)inc[bb + col[oi * W + ta]];
    }
  }
  out[idx] = add ? out[idx] + (T)s : (T)s;
}

template <int n, typename T>
__global__ void k_modal_I(const KT<n, T> tb, int N, int k, int M, int E, const T* __restrict__ u,
                          T* __restrict__ p, int add) {
  constexpr int NN = n * n, N3 = NN * n, NP = (n - 1) * n * (n + 1) / 6;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)E * NP) return;
  const int e = (int)(idx / NP), m = (int)(idx % NP);
  const int ex = e % N, ey = (e / N) % N, ez = e / (N * N);
  const int ma = tb.ma[m], mb = tb.mb[m], mc = tb.mc[m];
  T s = T(0);
  for (int li = 0; li < N3; ++li) {
    const int a = li % n, b = (li / n) % n, c = li / NN;
    const int g = (ex * k + a) + M * ((ey * k + b) + M * (ez * k + c));
    s += tb.J[ma * n + a] * tb.J[mb * n + b] * tb.J[mc * n + c] * u[g];
  }
  p[idx] = add ? p[idx] + s : s;
}

template <int n, typename T>
__global__ void k_modal_IT(const KT<n, T> tb, int N, int k, int M, int E, const T* __restrict__ p,
                           T* __restrict__ u) {
  constexpr int NN = n * n, N3 = NN * n, NP = (n - 1) * n * (n + 1) / 6;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)E * N3) return;
  const int e = (int)(idx / N3), li = (int)(idx % N3);
  const int a = li % n, b = (li / n) % n, c = li / NN;
  const int ex = e % N, ey = (e / N) % N, ez = e / (N * N);
  T s = T(0);
  for (int m = 0; m < NP; ++m)
    s += tb.J[tb.ma[m] * n + a] * tb.J[tb.mb[m] * n + b] * tb.J[tb.mc[m] * n + c] *
         p[(size_t)e * NP + m];
  const int g = (ex * k + a) + M * ((ey * k + b) + M * (ez * k + c));
  atomic_add(&u[g], s);
}

__global__ void k_coarsen_p(int E, int nf, int nc, const double* __restrict__ Q,
                            const double* __restrict__ in, double* __restrict__ out) {
  const int nf3 = nf * nf * nf, nc3 = nc * nc * nc;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)E * nc3) return;
  const int e = (int)(idx / nc3), q = (int)(idx % nc3);
  const int cx = q % nc, cy = (q / nc) % nc, cz = q / (nc * nc);
  const double* f = in + (size_t)e * nf3;
  double s = 0.0, mn = 1e300;
  for (int fz = 0; fz < nf; ++fz)
    for (int fy = 0; fy < nf; ++fy)
      for (int fx = 0; fx < nf; ++fx) {
        const double v = f[fz * nf * nf + fy * nf + fx];
        s += Q[cz * nf + fz] * Q[cy * nf + fy] * Q[cx * nf + fx] * v;
        mn = fmin(mn, v);
      }
  out[idx] = fmax(s, mn);
}

__global__ void k_coarsen_h(int Nf, int n, const double* __restrict__ Q, const double* __restrict__ in,
                            double* __restrict__ out) {
  const int Nc = Nf / 2, n3 = n * n * n, W = 2 * n;
  const long long Ec = (long long)Nc * Nc * Nc;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= Ec * n3) return;
  const int ce = (int)(idx / n3), q = (int)(idx % n3);
  const int cx = q % n, cy = (q / n) % n, cz = q / (n * n);
  const int ex = ce % Nc, ey = (ce / Nc) % Nc, ez = ce / (Nc * Nc);
  double s = 0.0, mn = 1e300;
  for (int sz = 0; sz < 2; ++sz)
    for (int sy = 0; sy < 2; ++sy)
      for (int sx = 0; sx < 2; ++sx) {
        const int fe = (2 * ex + sx) + Nf * ((2 * ey + sy) + Nf * (2 * ez + sz));
        const double* f = in + (size_t)fe * n3;
        for (int fz = 0; fz < n; ++fz)
          for (int fy = 0; fy < n; ++fy)
            for (int fx = 0; fx < n; ++fx) {
              const double v = f[fz * n * n + fy * n + fx];
              s += Q[cz * W + sz * n + fz] * Q[cy * W + sy * n + fy] * Q[cx * W + sx * n + fx] * v;
              mn = fmin(mn, v);
            }
      }
  out[idx] = fmax(s, mn);
}

template <typename T>
__global__ void k_dense(int nd, const double* __restrict__ G, const int* __restrict__ idx,
                        const T* __restrict__ x, T* __restrict__ y) {
  const int r = blockIdx.x * blockDim.x + threadIdx.x;
  if (r >= nd) return;
  double s = 0.0;
  for (int c = 0; c < nd; ++c) s += G[(size_t)r * nd + c] * (double)x[idx[c]];
  y[idx[r]] = (T)s;
}

// ------------------------------------------------------------------ vectors
template <typename T>
__global__ void k_fill(T* x, T v, size_t n) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] = v;
}
template <typename T>
__global__ void k_axpby(size_t n, T a, const T* __restrict__ x, T b, T* __restrict__ y) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i] + b * y[i];
}
template <typename Ta, typename Tb>
__global__ void k_cast(size_t n, const Ta* __restrict__ a, Tb* __restrict__ b) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) b[i] = (Tb)a[i];
}
template <typename T>
__global__ void k_scale_nodes(size_t nn, int NC, const T* __restrict__ s, const T* __restrict__ x,
                              T* __restrict__ y) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < nn * NC) y[i] = s[i % nn] * x[i];
}
template <typename T>
__global__ void k_cheb_first(size_t n, const T* __restrict__ b, const T* __restrict__ t,
                             const T* __restrict__ dinv, T inv_theta, T* __restrict__ d,
                             T* __restrict__ x, T* __restrict__ r, int xzero) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const T ri = t ? b[i] - t[i] : b[i];
  const T di = inv_theta * dinv[i] * ri;
  r[i] = ri;
  d[i] = di;
  x[i] = xzero ? di : x[i] + di;
}
template <typename T>
__global__ void k_cheb_step(size_t n, const T* __restrict__ t, const T* __restrict__ dinv, T alpha,
                            T beta, T* __restrict__ d, T* __restrict__ x, T* __restrict__ r) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const T ri = r[i] - t[i];
  const T di = alpha * d[i] + beta * dinv[i] * ri;
  r[i] = ri;
  d[i] = di;
  x[i] += di;
}
template <typename T>
__global__ void k_scal(size_t n, T a, const T* __restrict__ x, T* __restrict__ y) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) y[i] = a * x[i];
}
template <typename T>
__global__ void k_mask_boundary(int M, int NC, T* __restrict__ x) {
  const long long nn = (long long)M * M * M;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nn * NC) return;
  const long long g = idx % nn;
  const int gi = (int)(g % M), gj = (int)((g / M) % M), gl = (int)(g / ((long long)M * M));
  if (gi == 0 || gi == M - 1 || gj == 0 || gj == M - 1 || gl == 0 || gl == M - 1) x[idx] = T(0);
}
template <typename T>
__global__ void k_mul(size_t n, const T* __restrict__ a, const T* __restrict__ b, T* __restrict__ c) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) c[i] = a[i] * b[i];
}
template <typename T>
__global__ void k_sub(size_t n, const T* __restrict__ b, const T* __restrict__ t, T* __restrict__ r) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) r[i] = b[i] - t[i];
}

// block reduction of a double over 256 threads (wavefront 64)
__device__ inline double block_sum(double v) {
  __shared__ double red[4];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
  if (lane == 0) red[wid] = v;
  __syncthreads();
  double s = 0.0;
  if (threadIdx.x == 0) s = red[0] + red[1] + red[2] + red[3];
  __syncthreads();
  return s;
}

template <typename T>
__global__ void __launch_bounds__(256) k_dot_partial(size_t n, const T* __restrict__ x,
                                                     const T* __restrict__ y, double* partial) {
  double s = 0.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    s += (double)x[i] * (double)y[i];
  s = block_sum(s);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

__global__ void __launch_bounds__(256) k_final_sum(int nb, const double* __restrict__ partial,
                                                   double* out) {
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) s += partial[i];
  s = block_sum(s);
  if (threadIdx.x == 0) *out = s;
}

template <typename T>
__global__ void __launch_bounds__(256) k_mode0_partial(int E, int np, const T* __restrict__ p,
                                                       double* partial) {
  double s = 0.0;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < E; e += gridDim.x * blockDim.x)
    s += (double)p[(size_t)e * np];
  s = block_sum(s);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}

template <typename T>
__global__ void k_mode0_sub(int E, int np, T* __restrict__ p, const double* __restrict__ sum) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < E) p[(size_t)e * np] -= (T)(*sum / E);
}

__global__ void __launch_bounds__(256) k_mdot_partial(size_t n, int nv, const double* __restrict__ V,
                                                      size_t ld, const double* __restrict__ w,
                                                      double* partial) {
  for (int v = 0; v < nv; ++v) {
    const double* Vv = V + (size_t)v * ld;
    double s = 0.0;
    for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
      s += Vv[i] * w[i];
    s = block_sum(s);
    if (threadIdx.x == 0) partial[(size_t)v * gridDim.x + blockIdx.x] = s;
  }
}

__global__ void __launch_bounds__(256) k_rows_sum(int nb, const double* __restrict__ partial,
                                                  double* __restrict__ out) {
  double s = 0.0;
  const double* p = partial + (size_t)blockIdx.x * nb;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) s += p[i];
  s = block_sum(s);
  if (threadIdx.x == 0) out[blockIdx.x] = s;
}

__global__ void k_gemv(size_t n, int nv, const double* __restrict__ V, size_t ld,
                       const double* __restrict__ h, double sign, double* __restrict__ w) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int v = 0; v < nv; ++v) s += V[(size_t)v * ld + i] * h[v];
  w[i] += sign * s;
}

}  // namespace

// ================================================================== launchers
template <typename T>
void launch_op(hipStream_t st, int flags, int NC, int N, int k, const T* u, T* y, const T* coef,
               const T* pin, T* pout, const T* sin, const T* sout) {
  switch (k + 1) {
    case 2: return op_dispatch_n<2, T>(st, flags, NC, N, k, u, y, coef, pin, pout, sin, sout);
    case 3: return op_dispatch_n<3, T>(st, flags, NC, N, k, u, y, coef, pin, pout, sin, sout);
    case 4: return op_dispatch_n<4, T>(st, flags, NC, N, k, u, y, coef, pin, pout, sin, sout);
    case 5: return op_dispatch_n<5, T>(st, flags, NC, N, k, u, y, coef, pin, pout, sin, sout);
    default: throw Error{WB_EUNSUPPORTED, "order not built"};
  }
}
template void launch_op<double>(hipStream_t, int, int, int, int, const double*, double*,
                                const double*, const double*, double*, const double*, const double*);
template void launch_op<float>(hipStream_t, int, int, int, int, const float*, float*, const float*,
                               const float*, float*, const float*, const float*);

#define WB_BY_ORDER(k, ...)                                       \
  switch ((k) + 1) {                                              \
    case 2: { constexpr int n = 2; __VA_ARGS__; } break;          \
    case 3: { constexpr int n = 3; __VA_ARGS__; } break;          \
    case 4: { constexpr int n = 4; __VA_ARGS__; } break;          \
    case 5: { constexpr int n = 5; __VA_ARGS__; } break;          \
    default: throw Error{WB_EUNSUPPORTED, "order not built"};     \
  }

void launch_diag(hipStream_t st, int NC, int N, int k, bool dir, const double* coef, double* diag) {
  const int M = k * N + 1, E = N * N * N, nn = M * M * M, n3 = (k + 1) * (k + 1) * (k + 1);
  const size_t tot = (size_t)E * n3;
  WB_BY_ORDER(k, {
    auto tb = make_kt<n, double>(k);
    if (NC == 1)
      hipLaunchKernelGGL((k_diag<n, 1>), dim3(grid_for(tot, 256)), dim3(256), 0, st, tb, N, k, M, E,
                         nn, 0.5 / N, (int)dir, coef, diag);
    else
      hipLaunchKernelGGL((k_diag<n, 3>), dim3(grid_for(tot, 256)), dim3(256), 0, st, tb, N, k, M, E,
                         nn, 0.5 / N, (int)dir, coef, diag);
  });
}

void launch_invert_diag(hipStream_t st, int NC, int N, int k, bool dir, double* d) {
  const int M = k * N + 1;
  const size_t tot = (size_t)M * M * M * NC;
  hipLaunchKernelGGL(k_invert_diag, dim3(grid_for(tot, 256)), dim3(256), 0, st, M, NC, (int)dir, d);
}

void launch_lumped_mass(hipStream_t st, int N, int k, double amp, const double* mu_nodes,
                        double* cn) {
  const int M = k * N + 1, E = N * N * N, n3 = (k + 1) * (k + 1) * (k + 1);
  const double h = 1.0 / N;
  WB_BY_ORDER(k, {
    auto tb = make_kt<n, double>(k);
    hipLaunchKernelGGL((k_lumped<n>), dim3(grid_for((size_t)E * n3, 256)), dim3(256), 0, st, tb, N,
                       k, M, E, h * h * h / 8.0, amp, mu_nodes, cn);
  });
}

void launch_diag_K(hipStream_t st, int N, int k, const double* bhat, const double* dinv_nodes,
                   double* dk) {
  const int M = k * N + 1, E = N * N * N, np = tables(k).np;
  const double hh = 0.5 / N;
  WB_BY_ORDER(k, {
    hipLaunchKernelGGL((k_diag_K<n>), dim3(grid_for((size_t)E * np, 256)), dim3(256), 0, st, N, k,
                       M, E, np, hh * hh, bhat, dinv_nodes, dk);
  });
}

void launch_sinker_q(hipStream_t st, int N, int k, const double* centers, int ns, double delta,
                     double omega, double mu_min, double mu_max, double beta, double* mu_q,
                     double* f_q) {
  const int E = N * N * N, n3 = (k + 1) * (k + 1) * (k + 1);
  WB_BY_ORDER(k, {
    auto tb = make_kt<n, double>(k);
    hipLaunchKernelGGL((k_sinker_q<n>), dim3(grid_for((size_t)E * n3, 256)), dim3(256), 0, st, tb,
                       N, E, 1.0 / N, centers, ns, delta, omega, mu_min, mu_max, beta, mu_q, f_q);
  });
}

void launch_sinker_nodes(hipStream_t st, int N, int k, const double* x1, const double* centers,
                         int ns, double delta, double omega, double mu_min, double mu_max,
                         double* mu_nodes) {
  const int M = k * N + 1;
  hipLaunchKernelGGL(k_sinker_nodes, dim3(grid_for((size_t)M * M * M, 256)), dim3(256), 0, st, M,
                     x1, centers, ns, delta, omega, mu_min, mu_max, mu_nodes);
}

void launch_load(hipStream_t st, int N, int k, const double* f_q, double* F) {
  const int M = k * N + 1, E = N * N * N, n3 = (k + 1) * (k + 1) * (k + 1);
  const double h = 1.0 / N;
  WB_BY_ORDER(k, {
    auto tb = make_kt<n, double>(k);
    hipLaunchKernelGGL((k_load<n>), dim3(grid_for((size_t)E * n3, 256)), dim3(256), 0, st, tb, N, k,
                       M, E, h * h * h / 8.0, f_q, F);
  });
}

void launch_poisson_coef(hipStream_t st, int N, int k, double amp, const double* mu_q, double* c_q) {
  const int E = N * N * N, n3 = (k + 1) * (k + 1) * (k + 1);
  hipLaunchKernelGGL(k_poisson_coef, dim3(grid_for((size_t)E * n3, 256)), dim3(256), 0, st, N, n3,
                     E, amp, mu_q, c_q);
}

template <typename T>
void launch_kron(hipStream_t st, const Rows1D& R, int NC, bool dir, bool add, const T* in, T* out) {
  const size_t tot = (size_t)R.rows * R.rows * R.rows * NC;
  hipLaunchKernelGGL((k_kron<T>), dim3(grid_for(tot, 256)), dim3(256), 0, st, R.rows, R.cols, NC,
                     R.W, R.cnt, R.col, R.val, (int)dir, (int)add, in, out);
}
template void launch_kron<double>(hipStream_t, const Rows1D&, int, bool, bool, const double*, double*);
template void launch_kron<float>(hipStream_t, const Rows1D&, int, bool, bool, const float*, float*);

template <typename T>
void launch_modal_I(hipStream_t st, int N, int k, const T* u, T* p, bool add) {
  const int M = k * N + 1, E = N * N * N, np = tables(k).np;
  WB_BY_ORDER(k, {
    auto tb = make_kt<n, T>(k);
    hipLaunchKernelGGL((k_modal_I<n, T>), dim3(grid_for((size_t)E * np, 256)), dim3(256), 0, st, tb,
                       N, k, M, E, u, p, (int)add);
  });
}
template <typename T>
void launch_modal_IT(hipStream_t st, int N, int k, const T* p, T* u) {
  const int M = k * N + 1, E = N * N * N, n3 = (k + 1) * (k + 1) * (k + 1);
  WB_BY_ORDER(k, {
    auto tb = make_kt<n, T>(k);
    hipLaunchKernelGGL((k_modal_IT<n, T>), dim3(grid_for((size_t)E * n3, 256)), dim3(256), 0, st, tb,
                       N, k, M, E, p, u);
  });
}
template void launch_modal_I<double>(hipStream_t, int, int, const double*, double*, bool);
template void launch_modal_I<float>(hipStream_t, int, int, const float*, float*, bool);
template void launch_modal_IT<double>(hipStream_t, int, int, const double*, double*);
template void launch_modal_IT<float>(hipStream_t, int, int, const float*, float*);

void launch_coarsen_p(hipStream_t st, int E, int nf, int nc, const double* Q, const double* in,
                      double* out) {
  hipLaunchKernelGGL(k_coarsen_p, dim3(grid_for((size_t)E * nc * nc * nc, 256)), dim3(256), 0, st, E,
                     nf, nc, Q, in, out);
}
void launch_coarsen_h(hipStream_t st, int Nf, int n, const double* Q, const double* in, double* out) {
  const size_t Ec = (size_t)(Nf / 2) * (Nf / 2) * (Nf / 2);
  hipLaunchKernelGGL(k_coarsen_h, dim3(grid_for(Ec * n * n * n, 256)), dim3(256), 0, st, Nf, n, Q,
                     in, out);
}

template <typename T>
void launch_dense(hipStream_t st, int nd, const double* G, const int* idx, const T* x, T* y) {
  hipLaunchKernelGGL((k_dense<T>), dim3(grid_for(nd, 64)), dim3(64), 0, st, nd, G, idx, x, y);
}
template void launch_dense<double>(hipStream_t, int, const double*, const int*, const double*, double*);
template void launch_dense<float>(hipStream_t, int, const double*, const int*, const float*, float*);

template <typename T>
void launch_fill(hipStream_t st, T* x, T v, size_t n) {
  if (n) hipLaunchKernelGGL((k_fill<T>), dim3(grid_for(n, 256)), dim3(256), 0, st, x, v, n);
}
template <typename T>
void launch_axpby(hipStream_t st, size_t n, T a, const T* x, T b, T* y) {
  hipLaunchKernelGGL((k_axpby<T>), dim3(grid_for(n, 256)), dim3(256), 0, st, n, a, x, b, y);
}
template <typename Ta, typename Tb>
void launch_cast(hipStream_t st, size_t n, const Ta* a, Tb* b) {
  hipLaunchKernelGGL((k_cast<Ta, Tb>), dim3(grid_for(n, 256)), dim3(256), 0, st, n, a, b);
}
template <typename T>
void launch_scale_nodes(hipStream_t st, int nn, int NC, const T* s, const T* x, T* y) {
  hipLaunchKernelGGL((k_scale_nodes<T>), dim3(grid_for((size_t)nn * NC, 256)), dim3(256), 0, st,
                     (size_t)nn, NC, s, x, y);
}
template <typename T>
void launch_cheb_first(hipStream_t st, size_t n, const T* b, const T* t, const T* dinv, T inv_theta,
                       T* d, T* x, T* r, bool xzero) {
  hipLaunchKernelGGL((k_cheb_first<T>), dim3(grid_for(n, 256)), dim3(256), 0, st, n, b, t, dinv,
                     inv_theta, d, x, r, (int)xzero);
}
template <typename T>
void launch_cheb_step(hipStream_t st, size_t n, const T* t, const T* dinv, T alpha, T beta, T* d,
                      T* x, T* r) {
  hipLaunchKernelGGL((k_cheb_step<T>), dim3(grid_for(n, 256)), dim3(256), 0, st, n, t, dinv, alpha,
                     beta, d, x, r);
}
template <typename T>
void launch_sub(hipStream_t st, size_t n, const T* b, const T* t, T* r) {
  hipLaunchKernelGGL((k_sub<T>), dim3(grid_for(n, 256)), dim3(256), 0, st, n, b, t, r);
}
template <typename T>
void launch_scal(hipStream_t st, size_t n, T a, const T* x, T* y) {
  hipLaunchKernelGGL((k_scal<T>), dim3(grid_for(n, 256)), dim3(256), 0, st, n, a, x, y);
}
template <typename T>
void launch_mask_boundary(hipStream_t st, int M, int NC, T* x) {
  hipLaunchKernelGGL((k_mask_boundary<T>), dim3(grid_for((size_t)M * M * M * NC, 256)), dim3(256), 0,
                     st, M, NC, x);
}
template <typename T>
void launch_mul(hipStream_t st, size_t n, const T* a, const T* b, T* c) {
  hipLaunchKernelGGL((k_mul<T>), dim3(grid_for(n, 256)), dim3(256), 0, st, n, a, b, c);
}
template <typename T>
void launch_dot(hipStream_t st, size_t n, const T* x, const T* y, double* partial, double* out) {
  int nb = (int)std::min<size_t>(RED_BLOCKS, grid_for(n, 256));
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL((k_dot_partial<T>), dim3(nb), dim3(256), 0, st, n, x, y, partial);
  hipLaunchKernelGGL(k_final_sum, dim3(1), dim3(256), 0, st, nb, partial, out);
}
template <typename T>
void launch_remove_mean(hipStream_t st, int E, int np, T* p, double* partial, double* scratch) {
  int nb = (int)std::min<size_t>(RED_BLOCKS, grid_for(E, 256));
  hipLaunchKernelGGL((k_mode0_partial<T>), dim3(nb), dim3(256), 0, st, E, np, p, partial);
  hipLaunchKernelGGL(k_final_sum, dim3(1), dim3(256), 0, st, nb, partial, scratch);
  hipLaunchKernelGGL((k_mode0_sub<T>), dim3(grid_for(E, 256)), dim3(256), 0, st, E, np, p, scratch);
}

#define WB_INST_VEC(T)                                                                            \
  template void launch_fill<T>(hipStream_t, T*, T, size_t);                                       \
  template void launch_axpby<T>(hipStream_t, size_t, T, const T*, T, T*);                         \
  template void launch_scale_nodes<T>(hipStream_t, int, int, const T*, const T*, T*);             \
  template void launch_cheb_first<T>(hipStream_t, size_t, const T*, const T*, const T*, T, T*, T*, \
                                     T*, bool);                                                    \
  template void launch_cheb_step<T>(hipStream_t, size_t, const T*, const T*, T, T, T*, T*, T*);   \
  template void launch_sub<T>(hipStream_t, size_t, const T*, const T*, T*);                       \
  template void launch_mul<T>(hipStream_t, size_t, const T*, const T*, T*);                       \
  template void launch_scal<T>(hipStream_t, size_t, T, const T*, T*);                             \
  template void launch_mask_boundary<T>(hipStream_t, int, int, T*);                               \
  template void launch_dot<T>(hipStream_t, size_t, const T*, const T*, double*, double*);         \
  template void launch_remove_mean<T>(hipStream_t, int, int, T*, double*, double*);
WB_INST_VEC(double)
WB_INST_VEC(float)
template void launch_fill<int>(hipStream_t, int*, int, size_t);
template void launch_cast<double, float>(hipStream_t, size_t, const double*, float*);
template void launch_cast<float, double>(hipStream_t, size_t, const float*, double*);
template void launch_cast<double, double>(hipStream_t, size_t, const double*, double*);

void launch_mdot(hipStream_t st, size_t n, int nv, const double* V, size_t ld, const double* w,
                 double* partial, double* h) {
  int nb = (int)std::min<size_t>(256, grid_for(n, 256));
  hipLaunchKernelGGL(k_mdot_partial, dim3(nb), dim3(256), 0, st, n, nv, V, ld, w, partial);
  hipLaunchKernelGGL(k_rows_sum, dim3(nv), dim3(256), 0, st, nb, partial, h);
}
void launch_gemv_sub(hipStream_t st, size_t n, int nv, const double* V, size_t ld, const double* h,
                     double* w) {
  hipLaunchKernelGGL(k_gemv, dim3(grid_for(n, 256)), dim3(256), 0, st, n, nv, V, ld, h, -1.0, w);
}
void launch_gemv_add(hipStream_t st, size_t n, int nv, const double* Z, size_t ld, const double* y,
                     double* x) {
  hipLaunchKernelGGL(k_gemv, dim3(grid_for(n, 256)), dim3(256), 0, st, n, nv, Z, ld, y, 1.0, x);
}

}  // namespace wb
