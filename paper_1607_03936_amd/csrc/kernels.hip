// HIP kernels (gfx950) of the w-BFBT Stokes hot path.
//
// Operators are matrix-free and sum-factorized: per element the (k+1)^3 nodal
// values are interpolated to the (k+1)^3 Gauss points by three 1D contractions,
// differentiated there with the collocation derivative of the Gauss-Lagrange
// basis, multiplied by the pointwise coefficient and pulled back by the
// transposed contractions (Sec. 1.2 discretization, eq. 2).  Thread layout:
// n^2 threads per element, each holding a z-column in registers; x and y
// contractions exchange through LDS.  The divergence and the gradient alone
// use the precomputed tensor-product element matrix of the uniform mesh
// (k_div_elem, k_grad_line).
#include <algorithm>
#include <atomic>
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

// XCD-aware block order: workgroups are dealt round-robin to the eight XCDs (id % 8), so block id
// takes the work item (start of its XCD's range) + id / 8; each XCD then owns a contiguous run of
// work items, and the cache lines that neighbouring items share stay in one L2.  A bijection of
// [0, nb).
__device__ __forceinline__ int xcd_order(const int id, const int nb) {
  const int r = id & 7;
  return r * (nb >> 3) + min(r, nb & 7) + (id >> 3);
}

// ------------------------------------------------------------------ operator
// All threads of one element live in one wavefront, so the exchanges inside an element need
// only a wavefront-scope barrier (LDS operations of a wave complete in order).
__device__ inline void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}

// Elements per wavefront and the lane mapping: lane -> (element slot, thread in element).
template <int n>
struct WaveMap {
  static constexpr int NN = n * n, EPW = 64 / NN;
  static __device__ inline void map(int t, int& slot, int& r, bool& lane_ok) {
    const int wave = t >> 6, lane = t & 63;
    const int le = lane / NN;
    lane_ok = le < EPW;
    r = lane_ok ? lane - le * NN : 0;
    slot = lane_ok ? wave * EPW + le : -1;
  }
};

// 1D tables are centro-symmetric: B(n-1-q, n-1-l) = B(q, l) and Dh(n-1-q, n-1-m) = -Dh(q, m)
// (symmetric Gauss points, symmetric GLL nodes); Dh vanishes at the middle of an odd rule.
// The element kernels read the compile-time tables CT<n> with compile-time indices (after
// unrolling), so every entry is a literal; referencing only the first half of each table keeps
// the distinct constants at about half and lets sign modifiers supply the rest.
template <int n, typename T>
__device__ __forceinline__ T Bm(int q, int l) {
  constexpr int H = n / 2;
  if (q < H) return (T)CT<n>::t.B[q * n + l];
  if (q >= n - H) return (T)CT<n>::t.B[(n - 1 - q) * n + (n - 1 - l)];
  return (T)CT<n>::t.B[q * n + (l <= H ? l : n - 1 - l)];  // middle row of an odd rule
}
template <int n, typename T>
__device__ __forceinline__ T Dm(int q, int m) {
  constexpr int H = n / 2;
  if (q < H) return (T)CT<n>::t.Dh[q * n + m];
  if (q >= n - H) return -(T)CT<n>::t.Dh[(n - 1 - q) * n + (n - 1 - m)];
  if (m == H) return T(0);
  return m < H ? (T)CT<n>::t.Dh[q * n + m] : -(T)CT<n>::t.Dh[q * n + (n - 1 - m)];
}
template <int n, typename T>
__device__ __forceinline__ T Wg(int q) {
  return (T)CT<n>::t.wg[q < n / 2 ? q : n - 1 - q];
}
template <int n, typename T>
__device__ __forceinline__ T Lg(int a, int q) {
  return (T)CT<n>::t.L[a * n + q];
}

// ------------------------------------------------------------ line contractions
// A lane applies one 1D table to the n values of its line: out[q] = sum_m M[q][m] v[m], with
// M = B (interpolation to Gauss points), Dh (collocation derivative), or their transposes.
enum : int { C_B = 0, C_D = 1, C_BT = 2, C_DT = 3, C_NT = 4 };

template <int n, typename T, int C>
__device__ __forceinline__ T ctab(int q, int m) {
  if constexpr (C == C_B) return Bm<n, T>(q, m);
  else if constexpr (C == C_D) return Dm<n, T>(q, m);
  else if constexpr (C == C_BT) return Bm<n, T>(m, q);
  else return Dm<n, T>(m, q);
}

typedef __bf16 bf16x4 __attribute__((ext_vector_type(4)));
typedef float f32x4 __attribute__((ext_vector_type(4)));

// BF16 form: the leading 4x4 block of every table goes through the matrix cores.  With the
// 16-block 4x4x4 BF16 MFMA, lane l supplies row (l % 4) of the table as its A fragment and its
// own 4-vector as B; each lane then receives the table times its own vector, accumulated in
// FP32 (lanes do not mix, so any lane-to-line assignment works).  Lines of n < 4 values are
// zero-padded; for n = 5 the fifth row and column are applied on the VALU in FP32.
// MF = 1: one product of the BF16-rounded table and line (relative error ~2^-8 per contraction).
// MF = 3: table and line split into BF16 high and low parts, t = t_h + t_l, v = v_h + v_l, and
// t_h v_h + t_l v_h + t_h v_l accumulated in FP32 (~2^-16 per contraction).
struct Frags {
  bf16x4 f[C_NT];  // high parts
  bf16x4 g[C_NT];  // low parts
};

template <int n>
__device__ inline Frags make_frags() {
  Frags fr;
  const int row = (int)(threadIdx.x & 3);
#pragma unroll
  for (int c = 0; c < C_NT; ++c)
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      float v = 0.f;
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        float t = 0.f;
        if (q < n && m < n) {
          if (c == C_B) t = ctab<n, float, C_B>(q, m);
          else if (c == C_D) t = ctab<n, float, C_D>(q, m);
          else if (c == C_BT) t = ctab<n, float, C_BT>(q, m);
          else t = ctab<n, float, C_DT>(q, m);
        }
        v = (row == q) ? t : v;
      }
      const __bf16 hi = (__bf16)v;
      fr.f[c][m] = hi;
      fr.g[c][m] = (__bf16)(v - (float)hi);
    }
  return fr;
}

template <int n, typename T, int MF, int C>
__device__ __forceinline__ void ctr(const Frags& fr, const T (&v)[n], T (&out)[n]) {
  if constexpr (MF == 0) {
#pragma unroll
    for (int q = 0; q < n; ++q) {
      T acc = T(0);
#pragma unroll
      for (int m = 0; m < n; ++m) acc += ctab<n, T, C>(q, m) * v[m];
      out[q] = acc;
    }
  } else {
    static_assert(sizeof(T) == 4, "the BF16 form accumulates in FP32");
    bf16x4 bh, bl;
#pragma unroll
    for (int m = 0; m < 4; ++m) {
      const float x = m < n ? v[m] : 0.f;
      const __bf16 h = (__bf16)x;
      bh[m] = h;
      bl[m] = (__bf16)(x - (float)h);
    }
    f32x4 d = {0.f, 0.f, 0.f, 0.f};
    if constexpr (n == 5) {
#pragma unroll
      for (int q = 0; q < 4; ++q) d[q] = ctab<5, float, C>(q, 4) * v[4];
    }
    d = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(fr.f[C], bh, d, 0, 0, 0);
    if constexpr (MF == 3) {
      d = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(fr.g[C], bh, d, 0, 0, 0);
      d = __builtin_amdgcn_mfma_f32_4x4x4bf16_1k(fr.f[C], bl, d, 0, 0, 0);
    }
#pragma unroll
    for (int q = 0; q < (n < 4 ? n : 4); ++q) out[q] = d[q];
    if constexpr (n == 5) {
      float acc = 0.f;
#pragma unroll
      for (int m = 0; m < 5; ++m) acc += ctab<5, float, C>(4, m) * v[m];
      out[4] = acc;
    }
  }
}

// LDS layout of an element's scratch for element size ES: value (x, y, z) at x + SY y + SZ z,
// slots SL apart.  Padded strides spread the three line roles of a wavefront (z-, y- and
// x-lines) over the banks; the Q3 FP64 strides were chosen by measured bank-conflict counts.
template <int n, int ES> struct Lds;
template <int ES> struct Lds<2, ES> { static constexpr int SY = 2, SZ = 4, SL = 8; };
template <int ES> struct Lds<3, ES> { static constexpr int SY = 3, SZ = 9, SL = 27; };
template <> struct Lds<4, 8> { static constexpr int SY = 4, SZ = 19, SL = 88; };
template <> struct Lds<4, 4> { static constexpr int SY = 4, SZ = 18, SL = 71; };
template <int ES> struct Lds<5, ES> { static constexpr int SY = 5, SZ = 25, SL = 125; };
template <int ES> struct Lds<6, ES> { static constexpr int SY = 6, SZ = 37, SL = 222; };

// Element computation shared by the operator kernels.  The n^2 lanes of an element take three
// roles, always with a = r % n, b = r / n: the z-line (a, b, .), the y-line (a, ., b) or the
// x-line (., a, b).  A lane contracts a whole line with compile-time table indices; lines move
// between roles through the element's LDS scratch s, s2 (layout of Lds<n>).
// Components are processed one after the other.  For F_A / F_BT the contribution of the
// element to its local node (x, y, z) of component c is handed to sink(c, x, y, z, value);
// F_B hands each of the element's n_p pressure modes to psink(e n_p + m, value).
// Contains wavefront barriers: every lane of the wavefront must call it.
// Global inputs of one element in the z-line role (a, b): the node column of every component
// (masked: 0 on Dirichlet nodes and for idle lanes) and the coefficient at the Gauss points.
template <int n, int NC, typename T>
struct ElemIn {
  T uz[NC][n];
  T cq[n];
};

// Loads of one element, issued up front from in-bounds addresses (index 0 for idle lanes);
// masked values are selected away afterwards.
// ZIN: the input is ugain uscale u entry by entry (the zero-start Chebyshev direction).
template <int n, int NC, typename T, int F, bool ZIN = false>
__device__ inline void element_load(const bool valid, const int e, const int ex, const int ey,
                                    const int ez, const int k, const int M, const int nn,
                                    const T* __restrict__ u, const T* __restrict__ coef,
                                    const T* __restrict__ sin_, const int r, ElemIn<n, NC, T>& in,
                                    const T* __restrict__ uscale = nullptr, const T ugain = T(0)) {
  constexpr int NN = n * n, N3 = n * n * n;
  if constexpr ((F & (F_A | F_B)) != 0) {
    const int a = r % n, b = r / n;
    const int gi = ex * k + a, gj = ey * k + b;
    const bool bij = (gi == 0) || (gi == M - 1) || (gj == 0) || (gj == M - 1);
    int gidx[n];
    bool live[n];
#pragma unroll
    for (int l = 0; l < n; ++l) {
      const int gl = ez * k + l;
      const bool bnd = (F & F_DIR) && (bij || gl == 0 || gl == M - 1);
      live[l] = valid && !bnd;
      gidx[l] = valid ? gi + M * (gj + M * gl) : 0;
    }
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int l = 0; l < n; ++l) {
        const size_t j = (size_t)c * nn + gidx[l];
        if constexpr (ZIN) in.uz[c][l] = ugain * uscale[j] * u[j];
        else in.uz[c][l] = u[j];
      }
    if constexpr ((F & F_A) != 0) {
      const size_t eb = (size_t)(valid ? e : 0) * N3 + b * n + a;
#pragma unroll
      for (int q = 0; q < n; ++q) in.cq[q] = coef[eb + q * NN];
    }
    if (sin_ != nullptr) {
#pragma unroll
      for (int l = 0; l < n; ++l) {
        const T sl = sin_[gidx[l]];
#pragma unroll
        for (int c = 0; c < NC; ++c) in.uz[c][l] *= sl;
      }
    }
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int l = 0; l < n; ++l) in.uz[c][l] = live[l] ? in.uz[c][l] : T(0);
  }
}

template <int n, int NC, typename T, int F, int MF, typename PSink, typename Sink>
__device__ inline void element_op(const bool valid, const int e, const int k, const T hh,
                                  const ElemIn<n, NC, T>& in, const T* __restrict__ pin,
                                  PSink&& psink, T* s, T* s2, const int r, Sink&& sink) {
  constexpr int NP = (n - 1) * n * (n + 1) / 6;
  constexpr int SY = Lds<n, sizeof(T)>::SY, SZ = Lds<n, sizeof(T)>::SZ;
  const int a = r % n, b = r / n;
  Frags fr;
  if constexpr (MF) fr = make_frags<n>();
  constexpr int FC = F & (F_A | F_B | F_BT);

  if constexpr (NC == 3 && FC == F_B) {
    // Divergence alone: component c needs only its derivative in direction c, taken right after
    // the interpolation in that direction; the sum is formed in the x-line role (x Gauss point
    // q, y Gauss point a, z Gauss point b), then projected onto the Legendre modes.
    T dv[n];
#pragma unroll
    for (int q = 0; q < n; ++q) dv[q] = T(0);
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      T v[n], w[n];
      ctr<n, T, MF, C_B>(fr, in.uz[c], w);
      if (c == 2) {
        ctr<n, T, MF, C_D>(fr, w, v);
#pragma unroll
        for (int q = 0; q < n; ++q) w[q] = v[q];
      }
#pragma unroll
      for (int q = 0; q < n; ++q) s[a + SY * b + SZ * q] = w[q];
      wave_sync();
      // y-line (a, ., b), in place
#pragma unroll
      for (int m = 0; m < n; ++m) v[m] = s[a + SY * m + SZ * b];
      ctr<n, T, MF, C_B>(fr, v, w);
      if (c == 1) {
        ctr<n, T, MF, C_D>(fr, w, v);
#pragma unroll
        for (int q = 0; q < n; ++q) w[q] = v[q];
      }
#pragma unroll
      for (int q = 0; q < n; ++q) s[a + SY * q + SZ * b] = w[q];
      wave_sync();
      // x-line (., a, b)
#pragma unroll
      for (int m = 0; m < n; ++m) v[m] = s[m + SY * a + SZ * b];
      ctr<n, T, MF, C_B>(fr, v, w);
      if (c == 0) {
        ctr<n, T, MF, C_D>(fr, w, v);
#pragma unroll
        for (int q = 0; q < n; ++q) w[q] = v[q];
      }
#pragma unroll
      for (int q = 0; q < n; ++q) dv[q] += w[q];
      wave_sync();
    }
    // project -(h/2)^2 w3 div u onto the Legendre modes: x first (mode ma), then y and z
    const T wab = Wg<n, T>(a) * Wg<n, T>(b);
#pragma unroll
    for (int q = 0; q < n; ++q) dv[q] = -hh * hh * wab * Wg<n, T>(q) * dv[q];
#pragma unroll
    for (int c = 0; c < n - 1; ++c) {
      T acc = T(0);
#pragma unroll
      for (int q = 0; q < n; ++q) acc += Lg<n, T>(c, q) * dv[q];
      s[c + SY * a + SZ * b] = acc;
    }
    wave_sync();
    if (valid && r < NP) {
      const int ma = CT<n>::t.ma[r], mb = CT<n>::t.mb[r], mc = CT<n>::t.mc[r];
      T acc = T(0);
#pragma unroll
      for (int kk = 0; kk < n; ++kk)
#pragma unroll
        for (int jj = 0; jj < n; ++jj)
          acc += Lg<n, T>(mb, jj) * Lg<n, T>(mc, kk) * s[ma + SY * jj + SZ * kk];
      psink((size_t)e * NP + r, acc);
    }
    wave_sync();
    return;
  }

  if constexpr (NC == 3 && FC == F_BT) {
    // Gradient alone: the weighted pressure vv at the Gauss points is shared by the three
    // components, u_c = (B^T Dh^T)_c (B^T)_others vv, so the transposed contractions are
    // factored: z: A = B^T vv, Z = B^T Dh^T vv; y: from A both B^T and B^T Dh^T, from Z B^T;
    // x: the last factor of each component.
    T La[n - 1], Lb[n - 1];
#pragma unroll
    for (int m = 0; m < n - 1; ++m) {
      La[m] = Lg<n, T>(m, a);
      Lb[m] = Lg<n, T>(m, b);
    }
    const T wab = Wg<n, T>(a) * Wg<n, T>(b);
    T vv[n];
#pragma unroll
    for (int q = 0; q < n; ++q) {
      T pq = T(0);
#pragma unroll
      for (int m = 0; m < NP; ++m) {
        const T pmv = valid ? pin[(size_t)e * NP + m] : T(0);
        pq += pmv * La[CT<n>::t.ma[m]] * Lb[CT<n>::t.mb[m]] * Lg<n, T>(CT<n>::t.mc[m], q);
      }
      vv[q] = -hh * hh * wab * Wg<n, T>(q) * pq;
    }
    T v[n], w[n], A[n];
    // z-line (a, b, .): Gauss points -> z nodes
    ctr<n, T, MF, C_BT>(fr, vv, A);
    ctr<n, T, MF, C_DT>(fr, vv, w);
    ctr<n, T, MF, C_BT>(fr, w, v);
#pragma unroll
    for (int l = 0; l < n; ++l) {
      s[a + SY * b + SZ * l] = A[l];
      s2[a + SY * b + SZ * l] = v[l];
    }
    wave_sync();
    // y-line (a, ., b) with a the x Gauss point and b the z node, in place
    T by[n];
#pragma unroll
    for (int m = 0; m < n; ++m) v[m] = s[a + SY * m + SZ * b];
    ctr<n, T, MF, C_BT>(fr, v, A);
    ctr<n, T, MF, C_DT>(fr, v, w);
    ctr<n, T, MF, C_BT>(fr, w, by);
#pragma unroll
    for (int m = 0; m < n; ++m) v[m] = s2[a + SY * m + SZ * b];
    ctr<n, T, MF, C_BT>(fr, v, w);
#pragma unroll
    for (int l = 0; l < n; ++l) {
      s[a + SY * l + SZ * b] = A[l];
      s2[a + SY * l + SZ * b] = w[l];
    }
    wave_sync();
    // x-line (., a, b) with a the y node and b the z node: u_x and u_z
#pragma unroll
    for (int m = 0; m < n; ++m) v[m] = s[m + SY * a + SZ * b];
    ctr<n, T, MF, C_DT>(fr, v, w);
    ctr<n, T, MF, C_BT>(fr, w, v);
#pragma unroll
    for (int q = 0; q < n; ++q) sink(0, q, a, b, v[q]);
#pragma unroll
    for (int m = 0; m < n; ++m) v[m] = s2[m + SY * a + SZ * b];
    ctr<n, T, MF, C_BT>(fr, v, w);
#pragma unroll
    for (int q = 0; q < n; ++q) sink(2, q, a, b, w[q]);
    wave_sync();
    // u_y from the y-line result kept in registers
#pragma unroll
    for (int l = 0; l < n; ++l) s[a + SY * l + SZ * b] = by[l];
    wave_sync();
#pragma unroll
    for (int m = 0; m < n; ++m) v[m] = s[m + SY * a + SZ * b];
    ctr<n, T, MF, C_BT>(fr, v, w);
#pragma unroll
    for (int q = 0; q < n; ++q) sink(1, q, a, b, w[q]);
    wave_sync();
    return;
  }

  T S[NC][3][n];  // z-line role: gradients, then stresses, at (a, b, q)
  T bq[n];
  const T* cq = in.cq;  // coefficient at (a, b, q)

  if constexpr ((F & (F_A | F_B)) != 0) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      T v[n], w[n];
      // z: interpolate the node column to the Gauss points
      ctr<n, T, MF, C_B>(fr, in.uz[c], w);
#pragma unroll
      for (int q = 0; q < n; ++q) s[a + SY * b + SZ * q] = w[q];
      wave_sync();
      // y-line (a, ., b): interpolate in y, in place
#pragma unroll
      for (int m = 0; m < n; ++m) v[m] = s[a + SY * m + SZ * b];
      ctr<n, T, MF, C_B>(fr, v, w);
#pragma unroll
      for (int q = 0; q < n; ++q) s[a + SY * q + SZ * b] = w[q];
      wave_sync();
      // x-line (., a, b): interpolate in x, then differentiate in x
#pragma unroll
      for (int m = 0; m < n; ++m) v[m] = s[m + SY * a + SZ * b];
      ctr<n, T, MF, C_B>(fr, v, w);
      ctr<n, T, MF, C_D>(fr, w, v);
#pragma unroll
      for (int q = 0; q < n; ++q) {
        s[q + SY * a + SZ * b] = w[q];
        s2[q + SY * a + SZ * b] = v[q];
      }
      wave_sync();
      // y-line: differentiate in y (kept); z-line: differentiate in z
#pragma unroll
      for (int m = 0; m < n; ++m) v[m] = s[a + SY * m + SZ * b];
      ctr<n, T, MF, C_D>(fr, v, w);
#pragma unroll
      for (int m = 0; m < n; ++m) v[m] = s[a + SY * b + SZ * m];
      ctr<n, T, MF, C_D>(fr, v, S[c][2]);
      wave_sync();
#pragma unroll
      for (int q = 0; q < n; ++q) s[a + SY * q + SZ * b] = w[q];
      wave_sync();
#pragma unroll
      for (int q = 0; q < n; ++q) {
        S[c][0][q] = s2[a + SY * b + SZ * q];
        S[c][1][q] = s[a + SY * b + SZ * q];
      }
      wave_sync();
    }
    // pointwise at (a, b, q)
    const T wab = Wg<n, T>(a) * Wg<n, T>(b);
#pragma unroll
    for (int q = 0; q < n; ++q) {
      const T w3 = wab * Wg<n, T>(q);
      if constexpr (NC == 3) {
        if constexpr ((F & F_B) != 0) bq[q] = -hh * hh * w3 * (S[0][0][q] + S[1][1][q] + S[2][2][q]);
        if constexpr ((F & F_A) != 0) {
          const T cw = valid ? cq[q] * w3 * hh : T(0);
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
        const T cw = valid ? cq[q] * w3 * hh : T(0);
#pragma unroll
        for (int d = 0; d < 3; ++d) S[0][d][q] *= cw;
      }
    }
  } else {
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int d = 0; d < 3; ++d)
#pragma unroll
        for (int q = 0; q < n; ++q) S[c][d][q] = T(0);
  }

  if constexpr (NC == 3 && (F & F_B) != 0) {
    // project -(h/2)^2 w3 div u onto the Legendre modes
#pragma unroll
    for (int c = 0; c < n - 1; ++c) {
      T acc = T(0);
#pragma unroll
      for (int q = 0; q < n; ++q) acc += Lg<n, T>(c, q) * bq[q];
      s[a + SY * b + SZ * c] = acc;
    }
    wave_sync();
    if (valid && r < NP) {
      const int ma = CT<n>::t.ma[r], mb = CT<n>::t.mb[r], mc = CT<n>::t.mc[r];
      T acc = T(0);
#pragma unroll
      for (int jj = 0; jj < n; ++jj)
#pragma unroll
        for (int ii = 0; ii < n; ++ii)
          acc += Lg<n, T>(ma, ii) * Lg<n, T>(mb, jj) * s[ii + SY * jj + SZ * mc];
      psink((size_t)e * NP + r, acc);
    }
    wave_sync();
  }

  if constexpr (NC == 3 && (F & F_BT) != 0) {
    T La[n - 1], Lb[n - 1];
#pragma unroll
    for (int m = 0; m < n - 1; ++m) {
      La[m] = Lg<n, T>(m, a);
      Lb[m] = Lg<n, T>(m, b);
    }
    const T wab = Wg<n, T>(a) * Wg<n, T>(b);
#pragma unroll
    for (int q = 0; q < n; ++q) {
      T pq = T(0);
#pragma unroll
      for (int m = 0; m < NP; ++m) {
        const T pmv = valid ? pin[(size_t)e * NP + m] : T(0);
        pq += pmv * La[CT<n>::t.ma[m]] * Lb[CT<n>::t.mb[m]] * Lg<n, T>(CT<n>::t.mc[m], q);
      }
      const T vv = -hh * hh * wab * Wg<n, T>(q) * pq;
      S[0][0][q] += vv;
      S[1][1][q] += vv;
      S[2][2][q] += vv;
    }
  }

  if constexpr ((F & (F_A | F_BT)) != 0) {
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      T V[n], v[n], w[n];
      ctr<n, T, MF, C_DT>(fr, S[c][2], V);
#pragma unroll
      for (int q = 0; q < n; ++q) {
        s[a + SY * b + SZ * q] = S[c][0][q];
        s2[a + SY * b + SZ * q] = S[c][1][q];
      }
      wave_sync();
      // x-line: transposed x-derivative of S_cx; y-line: transposed y-derivative of S_cy
#pragma unroll
      for (int m = 0; m < n; ++m) v[m] = s[m + SY * a + SZ * b];
      ctr<n, T, MF, C_DT>(fr, v, w);
#pragma unroll
      for (int q = 0; q < n; ++q) s[q + SY * a + SZ * b] = w[q];
#pragma unroll
      for (int m = 0; m < n; ++m) v[m] = s2[a + SY * m + SZ * b];
      ctr<n, T, MF, C_DT>(fr, v, w);
#pragma unroll
      for (int q = 0; q < n; ++q) s2[a + SY * q + SZ * b] = w[q];
      wave_sync();
      // z-line: sum, then transposed z-interpolation to the nodes
#pragma unroll
      for (int q = 0; q < n; ++q) V[q] += s[a + SY * b + SZ * q] + s2[a + SY * b + SZ * q];
      wave_sync();
      ctr<n, T, MF, C_BT>(fr, V, w);
#pragma unroll
      for (int l = 0; l < n; ++l) s[a + SY * b + SZ * l] = w[l];
      wave_sync();
      // y-line (a, ., b = z node): transposed y-interpolation, in place
#pragma unroll
      for (int m = 0; m < n; ++m) v[m] = s[a + SY * m + SZ * b];
      ctr<n, T, MF, C_BT>(fr, v, w);
#pragma unroll
      for (int q = 0; q < n; ++q) s[a + SY * q + SZ * b] = w[q];
      wave_sync();
      // x-line (., a = y node, b = z node): transposed x-interpolation to the nodes
#pragma unroll
      for (int m = 0; m < n; ++m) v[m] = s[m + SY * a + SZ * b];
      ctr<n, T, MF, C_BT>(fr, v, w);
#pragma unroll
      for (int q = 0; q < n; ++q) sink(c, q, a, b, w[q]);
      wave_sync();
    }
  }
}

// What happens to a finished output value v of index j (see Epi in kernels.h); the mode is
// a template constant, so a plain store carries none of the epilogue's arguments.  The loads the
// epilogue needs (epi_load) and the update itself (epi_store) are separate steps, so that a
// kernel can issue the loads early; emit does both at once.
template <typename T>
struct EpiIn {
  T b = T(0), r = T(0), dold = T(0), dinv = T(0), x = T(0);
};
template <int EP, typename T>
__device__ __forceinline__ EpiIn<T> epi_load(const Epi<T>& e, const size_t j,
                                             const T* __restrict__ y, const int add) {
  EpiIn<T> q;
  if constexpr (EP == EPI_RESID) {
    q.b = e.b[j];
  } else if constexpr (EP == EPI_CHEB_FIRST || EP == EPI_CHEB_ZERO) {
    q.b = e.b[j];
    q.dinv = e.dinv[j];
  } else if constexpr (EP == EPI_CHEB_STEP) {
    q.r = e.r[j];
    q.dold = e.dold[j];
    q.dinv = e.dinv[j];
    q.x = e.x[j];
  }
  return q;   // the plain store reads y (when it adds) in epi_store
}
template <int EP, typename T>
__device__ __forceinline__ void epi_store(const Epi<T>& e, const size_t j, const T v,
                                          const EpiIn<T>& q, T* __restrict__ y, const int add) {
  if constexpr (EP == EPI_RESID) {
    e.r[j] = q.b - v;
  } else if constexpr (EP == EPI_CHEB_FIRST) {
    const T ri = q.b - v;
    e.r[j] = ri;
    e.dnew[j] = e.alpha * q.dinv * ri;
  } else if constexpr (EP == EPI_CHEB_ZERO) {
    const T d0 = e.gamma * q.dinv * q.b;
    const T ri = q.b - v;
    e.r[j] = ri;
    const T dn = e.alpha * d0 + e.beta * q.dinv * ri;
    e.dnew[j] = dn;
    e.x[j] = d0 + dn;
  } else if constexpr (EP == EPI_CHEB_STEP) {
    const T ri = q.r - v;
    e.r[j] = ri;
    const T d0 = q.dold;
    const T dn = e.alpha * d0 + e.beta * q.dinv * ri;
    e.dnew[j] = dn;
    e.x[j] = q.x + (e.add_old ? d0 + dn : dn);
  } else {
    y[j] = add ? y[j] + v : v;
  }
}
template <int EP, typename T>
__device__ __forceinline__ void emit(const Epi<T>& e, const size_t j, const T v, T* __restrict__ y,
                                     const int add) {
  epi_store<EP>(e, j, v, epi_load<EP>(e, j, y, add), y, add);
}

// Brick geometry of the scatter kernel: a block owns a BX x BY tile of elements and marches
// through a chunk of Bz element layers in z.
template <int n> struct Tile;
template <> struct Tile<2> { static constexpr int BX = 8, BY = 8; };
template <> struct Tile<3> { static constexpr int BX = 8, BY = 4; };
template <> struct Tile<4> { static constexpr int BX = 8, BY = 4; };
template <> struct Tile<5> { static constexpr int BX = 4, BY = 4; };
template <> struct Tile<6> { static constexpr int BX = 4, BY = 2; };

struct BrickGeom {
  int N, k, M, nn, E;
  int BX, BY, Bz;        // tile and chunk sizes (elements)
  int nbx, nby, nbz;     // bricks per direction
  size_t plane;          // M * M
  size_t fx, fy, fz;     // offsets (elements of T) of the x/y/z face arrays per component
  size_t per_comp;       // face-array elements per component
};

// The two-pass form (k_op_elem + k_node_sum) is used while the element contributions take at
// most two_pass_limit bytes in FP64 (at most TWO_PASS_MAX_BYTES; 96 MiB by default); larger
// problems use the brick scatter (no element buffer in HBM).  The choice does not depend on the
// data type, so a workspace sized for FP64 serves FP32 too, and workspaces are sized for both
// forms up to TWO_PASS_MAX_BYTES, so the limit may change while solvers exist.  With the 96 MiB
// default the order-3 Poisson operator on 64^3 elements (a 128 MiB buffer) takes the matrix-core
// brick form, about 10 ms faster per 64^3 Q3 solve than the two-pass form.
constexpr size_t TWO_PASS_MAX_BYTES = 128u << 20;
std::atomic<size_t> two_pass_limit{96u << 20};
// Order-3 brick applies of A and the Poisson operator (FP64, and the FP32 data of the FP32
// precision form) on the FP64 matrix cores (k_op_mfma), or with line contractions in LDS
// (k_op_brick).
std::atomic<int> matrix_core_ops{1};
inline size_t elem_buf_bytes(int NC, int N, int k) {
  return sizeof(double) * NC * (size_t)N * N * N * (size_t)(k + 1) * (k + 1) * (k + 1);
}
// Per-thread cap on the two-pass element buffer (the caller's workspace size; unlimited by
// default), set for the duration of a call by WorkspaceCap.
thread_local size_t two_pass_cap = ~(size_t)0;
inline bool two_pass(int NC, int N, int k) {
  const size_t b = elem_buf_bytes(NC, N, k);
  return b <= two_pass_limit.load(std::memory_order_relaxed) && b <= two_pass_cap;
}

inline BrickGeom brick_geom(int N, int k, int BX, int BY) {
  BrickGeom g;
  g.N = N;
  g.k = k;
  g.M = k * N + 1;
  g.nn = g.M * g.M * g.M;
  g.E = N * N * N;
  g.BX = BX;
  g.BY = BY;
  g.nbx = (N + BX - 1) / BX;
  g.nby = (N + BY - 1) / BY;
  const int tiles = g.nbx * g.nby;
  g.Bz = std::max(1, std::min(N, (N * tiles) / 512));
  g.nbz = (N + g.Bz - 1) / g.Bz;
  g.plane = (size_t)g.M * g.M;
  g.fx = 0;
  g.fy = 8 * (size_t)(g.nbx - 1) * g.plane;
  g.fz = g.fy + 8 * (size_t)(g.nby - 1) * g.plane;
  g.per_comp = g.fz + 8 * (size_t)(g.nbz - 1) * g.plane;
  return g;
}

// Kernel-side copy of the brick geometry: the order and the tile shape are template constants,
// the face array starts with the x planes; 32-bit fields (3 n_nodes < 2^31, face arrays smaller).
struct BrickDev {
  int N, M, nn, Bz, nbx, nby, nbz, fy, fz, per_comp;
};
inline BrickDev brick_dev(const BrickGeom& g) {
  BrickDev d;
  d.N = g.N;
  d.M = g.M;
  d.nn = g.nn;
  d.Bz = g.Bz;
  d.nbx = g.nbx;
  d.nby = g.nby;
  d.nbz = g.nbz;
  d.fy = (int)g.fy;
  d.fz = (int)g.fz;
  d.per_comp = (int)g.per_comp;
  return d;
}

// Store one finished node value: direct when the node is owned by this brick alone, else into
// the face array of the first internal brick plane it lies on, slot s = sx + 2 sy + 4 sz
// (s_d = 1 when this brick lies above that plane).  Dirichlet nodes emit 0.
template <int n, int NC, typename T, bool DIR, int EP>
__device__ inline void store_node(const BrickDev& G, const int gx, const int gy, const int gz,
                                  const int X0, const int Y0, const int Z0, const int X1,
                                  const int Y1, const int Z1, const T (&val)[NC],
                                  T* __restrict__ y, T* __restrict__ face, const int add,
                                  const Epi<T>& ep) {
  constexpr int k = n - 1, KX = k * Tile<n>::BX, KY = k * Tile<n>::BY;
  const int M = G.M;
  const size_t g = (size_t)gx + (size_t)M * (gy + (size_t)M * gz);
  if (DIR && (gx == 0 || gx == M - 1 || gy == 0 || gy == M - 1 || gz == 0 || gz == M - 1)) {
    // a Dirichlet node on an internal brick plane is visited by every adjacent brick: only the
    // one for which it lies on no internal lower plane emits
    if ((gx == X0 && X0 > 0) || (gy == Y0 && Y0 > 0) || (gz == Z0 && Z0 > 0)) return;
#pragma unroll
    for (int c = 0; c < NC; ++c) emit<EP>(ep, (size_t)c * G.nn + g, T(0), y, add);
    return;
  }
  const bool lx = gx == X0 && X0 > 0, ux = gx == X1 && X1 < M - 1;
  const bool ly = gy == Y0 && Y0 > 0, uy = gy == Y1 && Y1 < M - 1;
  const bool lz = gz == Z0 && Z0 > 0, uz = gz == Z1 && Z1 < M - 1;
  if (!(lx || ux || ly || uy || lz || uz)) {
#pragma unroll
    for (int c = 0; c < NC; ++c) emit<EP>(ep, (size_t)c * G.nn + g, val[c], y, add);
    return;
  }
  const int s = (lx ? 1 : 0) + 2 * (ly ? 1 : 0) + 4 * (lz ? 1 : 0);
  int off;
  if (lx || ux) {
    const int b = gx / KX - 1;
    off = ((s * (G.nbx - 1) + b) * M + gz) * M + gy;
  } else if (ly || uy) {
    const int b = gy / KY - 1;
    off = G.fy + ((s * (G.nby - 1) + b) * M + gz) * M + gx;
  } else {
    const int b = gz / (k * G.Bz) - 1;
    off = G.fz + ((s * (G.nbz - 1) + b) * M + gy) * M + gx;
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) face[(size_t)c * G.per_comp + off] = val[c];
}

// Strides of the LDS accumulation window (row, plane) for element size ES: padding spreads the
// accumulations of neighbouring elements over the banks.
template <int n, int ES>
struct WinPad {
  static constexpr int WX = (n - 1) * Tile<n>::BX + 1, WY = (n - 1) * Tile<n>::BY + 1;
  static constexpr int WXS = WX, WPS = WX * WY;
};

// Divergence only (no scatter) with the sum-factorized element machinery, element-parallel; the
// pressure modes go through the epilogue.  Used by the BF16 forms (their contractions on the
// matrix cores); the other forms use k_div_elem.
template <int n, typename T, int F, int MF, int EP>
__global__ void __launch_bounds__(256)
k_op_gather(const int N, const int k, const int M, const int E, const int nn, const T hh,
            const T* __restrict__ u, T* __restrict__ pout, const T* __restrict__ sin_,
            const int add, const Epi<T> ep) {
  constexpr int EPW = WaveMap<n>::EPW, SLOTS = 4 * EPW, SL = Lds<n, sizeof(T)>::SL;
  __shared__ T sm[2 * (SLOTS + 1) * SL];
  int slot, r;
  bool lane_ok;
  WaveMap<n>::map(threadIdx.x, slot, r, lane_ok);
  const int e = blockIdx.x * SLOTS + slot;
  const bool valid = lane_ok && e < E;
  int ex = 0, ey = 0, ez = 0;
  if (valid) {
    ex = e % N;
    const int q = e / N;
    ey = q % N;
    ez = q / N;
  }
  T* s0 = sm + (lane_ok ? slot : SLOTS) * SL;
  ElemIn<n, 3, T> in;
  element_load<n, 3, T, F>(valid, e, ex, ey, ez, k, M, nn, u, nullptr, sin_, r, in);
  element_op<n, 3, T, F, MF>(valid, e, k, hh, in, nullptr,
                             [&](size_t j, T v) { emit<EP>(ep, j, v, pout, add); }, s0,
                             s0 + (SLOTS + 1) * SL, r, [](int, int, int, int, T) {});
}

// Two-pass form of the node-scattering operators (A, Poisson) for problems small enough that the
// element contributions fit in a modest buffer: every element runs in parallel (no brick march,
// no LDS window) and stores its NC n^3 contributions; then each node sums those of
// the at most eight elements containing it, in a fixed order, and goes through the epilogue.
// The buffer is [NC][n^3][E] (element index fastest): the node sums of a wavefront, which walk
// along x through consecutive elements, then read contiguous runs.
template <int n, int NC, typename T, int F, int MF, int EP>
__global__ void __launch_bounds__(256)
k_op_elem(const int N, const int k, const int M, const int E, const int nn, const T hh,
          const T* __restrict__ u, const T* __restrict__ coef, const T* __restrict__ sin_,
          T* __restrict__ buf, const Epi<T> ep) {
  constexpr int EPW = WaveMap<n>::EPW, SLOTS = 4 * EPW, SL = Lds<n, sizeof(T)>::SL;
  constexpr int N3 = n * n * n;
  __shared__ T sm[2 * (SLOTS + 1) * SL];
  int slot, r;
  bool lane_ok;
  WaveMap<n>::map(threadIdx.x, slot, r, lane_ok);
  const int e = blockIdx.x * SLOTS + slot;
  const bool valid = lane_ok && e < E;
  int ex = 0, ey = 0, ez = 0;
  if (valid) {
    ex = e % N;
    const int q = e / N;
    ey = q % N;
    ez = q / N;
  }
  T* s0 = sm + (lane_ok ? slot : SLOTS) * SL;
  ElemIn<n, NC, T> in;
  if constexpr (EP == EPI_CHEB_ZERO)
    element_load<n, NC, T, F, true>(valid, e, ex, ey, ez, k, M, nn, ep.b, coef, sin_, r, in, ep.dinv,
                                    ep.gamma);
  else
    element_load<n, NC, T, F>(valid, e, ex, ey, ez, k, M, nn, u, coef, sin_, r, in);
  element_op<n, NC, T, F, MF>(valid, e, k, hh, in, nullptr, [](size_t, T) {}, s0,
                              s0 + (SLOTS + 1) * SL, r, [&](int c, int x, int yy, int z, T v) {
                                if (valid)
                                  buf[(size_t)(c * N3 + x + n * (yy + n * z)) * E + e] = v;
                              });
}

template <int n, int NC, typename T, bool DIR, int EP>
__global__ void __launch_bounds__(256)
k_node_sum(const int N, const int M, const int nn, const T* __restrict__ buf, T* __restrict__ y,
           const int add, const Epi<T> ep) {
  constexpr int k = n - 1, N3 = n * n * n;
  const int g = blockIdx.x * blockDim.x + threadIdx.x;
  if (g >= nn) return;
  const int gc[3] = {g % M, (g / M) % M, g / (M * M)};
  T val[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) val[c] = T(0);
  const bool bnd = DIR && (gc[0] == 0 || gc[0] == M - 1 || gc[1] == 0 || gc[1] == M - 1 ||
                           gc[2] == 0 || gc[2] == M - 1);
  if (!bnd) {
    // per direction: element of the first candidate and its local index, and whether the second
    // candidate (the next element, local index 0) exists
    int e0[3], l0[3];
    bool has0[3], has1[3];
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      const int rr = gc[d] % k, q = gc[d] / k;
      const bool vert = rr == 0;
      has0[d] = !vert || q > 0;
      has1[d] = vert && q < N;
      e0[d] = vert ? q - 1 : q;
      l0[d] = vert ? k : rr;
    }
#pragma unroll
    for (int sz = 0; sz < 2; ++sz)
#pragma unroll
      for (int sy = 0; sy < 2; ++sy)
#pragma unroll
        for (int sx = 0; sx < 2; ++sx) {
          if (!((sx ? has1[0] : has0[0]) && (sy ? has1[1] : has0[1]) && (sz ? has1[2] : has0[2])))
            continue;
          const int ex = sx ? e0[0] + 1 : e0[0], ey = sy ? e0[1] + 1 : e0[1], ez = sz ? e0[2] + 1 : e0[2];
          const int lx = sx ? 0 : l0[0], ly = sy ? 0 : l0[1], lz = sz ? 0 : l0[2];
          const size_t E = (size_t)N * N * N;
          const T* be = buf + (size_t)(lx + n * (ly + n * lz)) * E + (size_t)ex +
                        (size_t)N * (ey + (size_t)N * ez);
#pragma unroll
          for (int c = 0; c < NC; ++c) val[c] += be[(size_t)c * N3 * E];
        }
  }
#pragma unroll
  for (int c = 0; c < NC; ++c) emit<EP>(ep, (size_t)c * nn + g, val[c], y, add);
}

// Scatter operator: y = op(u) (or y += op(u)), F_B output as well when requested.
template <int n>
struct BrickThreads {
  static constexpr int NE = Tile<n>::BX * Tile<n>::BY;
  static constexpr int WAVES = (NE + WaveMap<n>::EPW - 1) / WaveMap<n>::EPW;
  static constexpr int NT = 64 * WAVES;
};

template <int n, int NC, typename T, int F, int MF, int EP>
__global__ void __launch_bounds__(BrickThreads<n>::NT)
k_op_brick(const BrickDev G, const T hh, const T* __restrict__ u,
           T* __restrict__ y, const T* __restrict__ coef, const T* __restrict__ pin,
           T* __restrict__ pout, const T* __restrict__ sin_, T* __restrict__ face, const int add,
           const Epi<T> ep) {
  constexpr int BX = Tile<n>::BX, BY = Tile<n>::BY, NE = BX * BY;
  constexpr int N3 = n * n * n, k = n - 1;
  constexpr int WX = k * BX + 1, WY = k * BY + 1, WP = WX * WY;   // window plane (logical)
  // padded strides of the window in LDS (row WXS, plane WPS)
  constexpr int WXS = WinPad<n, sizeof(T)>::WXS, WPS = WinPad<n, sizeof(T)>::WPS;
  static_assert(WXS >= WX && WPS >= WXS * WY, "window padding");
  constexpr int NT = BrickThreads<n>::NT, SLOTS = BrickThreads<n>::WAVES * WaveMap<n>::EPW;
  constexpr int SL = Lds<n, sizeof(T)>::SL;
  __shared__ T sm[2 * (SLOTS + 1) * SL];
  __shared__ T win[NC * (k + 1) * WPS];
  const int N = G.N, M = G.M;
  const int t = threadIdx.x;
  int le, r;
  bool lane_ok;
  WaveMap<n>::map(t, le, r, lane_ok);
  const bool slot_ok = lane_ok && le < NE;
  const int lx = slot_ok ? le % BX : 0, ly = slot_ok ? le / BX : 0;
  const int tx = blockIdx.x % G.nbx, ty = blockIdx.x / G.nbx, bz = blockIdx.y;
  const int ex = tx * BX + lx, ey = ty * BY + ly;
  const int X0 = tx * BX * k, Y0 = ty * BY * k;
  const int X1 = X0 + k * BX, Y1 = Y0 + k * BY;
  const int ez0 = bz * G.Bz, ez1 = min(N, ez0 + G.Bz);
  const int Z0 = ez0 * k, Z1 = ez1 * k;
  for (int idx = t; idx < NC * (k + 1) * WPS; idx += NT) win[idx] = T(0);
  const bool valid = slot_ok && ex < N && ey < N;
  __syncthreads();
  for (int ez = ez0; ez < ez1; ++ez) {
    const int e = ex + N * (ey + N * ez);
    T* wbase = win + (ly * k) * WXS + lx * k;
    T* s0 = sm + (lane_ok ? le : SLOTS) * SL;
    // (loading the next layer before the plane flush raises the register peak of the Q3
    // operator past 128 and costs a wave per SIMD: loads stay at the top of the layer)
    ElemIn<n, NC, T> in;
    if constexpr (EP == EPI_CHEB_ZERO)
      element_load<n, NC, T, F, true>(valid, e, ex, ey, ez, k, M, G.nn, ep.b, coef, sin_, r, in,
                                      ep.dinv, ep.gamma);
    else
      element_load<n, NC, T, F>(valid, e, ex, ey, ez, k, M, G.nn, u, coef, sin_, r, in);
    element_op<n, NC, T, F, MF>(valid, e, k, hh, in, pin, [&](size_t j, T v) { pout[j] = v; }, s0,
                                s0 + (SLOTS + 1) * SL, r,
                                [&](int c, int x, int yy, int z, T v) {
                                  if (valid)
                                    atomicAdd(wbase + (c * (k + 1) + z) * WPS + yy * WXS + x, v);
                                });
    __syncthreads();
    // planes z = ez k .. ez k + k - 1 are complete
    for (int idx = t; idx < k * WP; idx += NT) {
      const int l = idx / WP, w = idx - l * WP;
      const int wx = w % WX, wy = w / WX;
      const int gx = X0 + wx, gy = Y0 + wy, gz = ez * k + l;
      if (gx >= M || gy >= M) continue;
      T val[NC];
#pragma unroll
      for (int c = 0; c < NC; ++c) val[c] = win[(c * (k + 1) + l) * WPS + wy * WXS + wx];
      store_node<n, NC, T, (F & F_DIR) != 0, EP>(G, gx, gy, gz, X0, Y0, Z0, X1, Y1, Z1, val, y, face, add, ep);
    }
    __syncthreads();
    // shift the window: plane k becomes plane 0, the others restart at zero
    for (int idx = t; idx < NC * WP; idx += NT) {
      const int c = idx / WP, w = idx - c * WP;
      const int ws = (w / WX) * WXS + w % WX;
      win[(c * (k + 1)) * WPS + ws] = win[(c * (k + 1) + k) * WPS + ws];
#pragma unroll
      for (int l = 1; l <= k; ++l) win[(c * (k + 1) + l) * WPS + ws] = T(0);
    }
    __syncthreads();
  }
  // last plane of the chunk (z = Z1)
  for (int w = t; w < WP; w += NT) {
    const int wx = w % WX, wy = w / WX;
    const int gx = X0 + wx, gy = Y0 + wy;
    if (gx >= M || gy >= M) continue;
    T val[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) val[c] = win[(c * (k + 1)) * WPS + wy * WXS + wx];
    store_node<n, NC, T, (F & F_DIR) != 0, EP>(G, gx, gy, Z1, X0, Y0, Z0, X1, Y1, Z1, val, y, face, add, ep);
  }
}

// ------------------------------------------------------------ matrix-core FP64 operator, order 3
// The node-scattering operators (A, Poisson) at order 3 with FP64 data, brick geometry and face
// array as k_op_brick, but with the 1D contractions in x and y on the FP64 matrix cores.
// v_mfma_f64_4x4x4_4b computes four independent 4x4x4 products D = A B + C, one double of A, B
// and D per lane.  Lane layout (measured on gfx950), lane l = f0 + 4 f1 + 16 f2:
//   A[i][k] at (f0, f2) = (i, k), B[k][j] at (f0, f2) = (j, k), D[i][j] at (f0, f2) = (j, i),
// f1 the block.  A wave holds four elements (f1 = element slot, consecutive in x); for each
// element and component, lane (f0, f2) keeps a column of four values along z in registers, so
// contractions in z are register FMAs, and a contraction over f2 is one instruction per z value:
//   mf_keep: table as A, data as B: contracts f2, the result index replaces f2, f0 kept;
//   mf_swap: data as A, table as B: contracts f2, the result index goes to f0 and f0 to f2.
// In both the lane supplies the table entry T[f0][f2] (T[q][m]: output q, input m).  Starting
// from (f0, f2) = (x, y): y then x by mf_swap give the Gauss values with (f0, f2) = (qx, qy);
// the x-derivative is mf_swap with the node-to-Gauss derivative table, the y-derivative mf_keep
// with the Gauss-point derivative, the z-derivative a register contraction, so the gradient
// components all end in one layout and the stress is pointwise.  The transposed contractions
// run the same two swaps backwards, accumulating in the matrix cores' C operand.
// Element contributions leave in z columns: the top value of a column is the bottom value of the
// next element layer (same lane), kept in a register; node sums over the elements of a layer
// go through a small LDS exchange in fixed order (deterministic, no atomics).
__device__ __forceinline__ double mf_keep(double t, double v, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(t, v, c, 0, 0, 0);
}
__device__ __forceinline__ double mf_swap(double t, double v, double c) {
  return __builtin_amdgcn_mfma_f64_4x4x4f64(v, t, c, 0, 0, 0);
}

enum : int { MT_B = 0, MT_D1 = 1, MT_DH = 2, MT_BT = 3, MT_D1T = 4 };
// Entry (q, m) of an order-3 table with compile-time indices.
template <int C>
__device__ __forceinline__ double mt_entry(int q, int m) {
  if constexpr (C == MT_B) return Bm<4, double>(q, m);
  else if constexpr (C == MT_D1) return CT<4>::t.D1[q * 4 + m];
  else if constexpr (C == MT_DH) return Dm<4, double>(q, m);
  else if constexpr (C == MT_BT) return Bm<4, double>(m, q);
  else return CT<4>::t.D1[m * 4 + q];
}
// The lane's entry T[f0][f2] of table C (selected among the 16 compile-time values).
template <int C>
__device__ inline double mt_lane(int f0, int f2) {
  double v = 0.0;
#pragma unroll
  for (int q = 0; q < 4; ++q)
#pragma unroll
    for (int m = 0; m < 4; ++m) v = (q == f0 && m == f2) ? mt_entry<C>(q, m) : v;
  return v;
}

// Tile of k_op_mfma: 8 x 4 elements; a tile row is two waves of four elements consecutive in x
// (f1 = element slot); eight waves.
constexpr int MF_PX = 2, MF_BX = 4 * MF_PX, MF_BY = 8 / MF_PX, MF_NT = 512;

// Neighbour exchange of k_op_mfma through LDS, per plane and component: the top row (f2 = 3) of
// every wave's elements (16 values) for the row above, and the right column (f0 = 3) of the last
// element of the left wave of a tile row (4 values) for the right wave.
template <int NC>
struct MfLds {
  static constexpr int YW = NC * 3 * 16, XW = NC * 3 * 4;    // per wave
  static constexpr int XOFF = 8 * YW, BUF = XOFF + 8 * XW;
};

// Value of lane - 1 within the lane's row of 16 (DPP row shift right by one).
__device__ __forceinline__ double from_left(double v) {
  const long long b = __builtin_bit_cast(long long, v);
  const int lo = __builtin_amdgcn_update_dpp(0, (int)(b & 0xffffffff), 0x111, 0xf, 0xf, false);
  const int hi = __builtin_amdgcn_update_dpp(0, (int)(b >> 32), 0x111, 0xf, 0xf, false);
  return __builtin_bit_cast(double, ((long long)hi << 32) | (unsigned int)lo);
}

// T is the storage type of the vectors, the coefficient and the face array (FP64, or FP32 for the
// FP32 precision form); the arithmetic is FP64 throughout (matrix cores and registers).  EP is an
// output epilogue, or EPI_ZERO_IN: plain stores of the operator applied to d0 = gamma D^-1 b,
// formed as it is read (the operator half of EPI_CHEB_ZERO, whose epilogue then runs apart).
constexpr int EPI_ZERO_IN = 5;
template <int NC, typename T, int F, int EP>
__global__ void __launch_bounds__(MF_NT, NC == 1 ? 4 : 2)
k_op_mfma(const BrickDev G, const double hh, const T* __restrict__ u,
          T* __restrict__ y, const T* __restrict__ coef,
          const T* __restrict__ sin_, T* __restrict__ face, const int add,
          const Epi<T> ep) {
  static_assert(Tile<4>::BX == MF_BX && Tile<4>::BY == MF_BY, "brick tile of order 3");
  constexpr int k = 3, YW = MfLds<NC>::YW, XW = MfLds<NC>::XW, XOFF = MfLds<NC>::XOFF;
  constexpr int BUF = MfLds<NC>::BUF;
  constexpr bool DIR = (F & F_DIR) != 0;
  constexpr int EO = EP == EPI_ZERO_IN ? EPI_STORE : EP;   // output epilogue
  __shared__ double ybuf[2 * BUF];
  const int N = G.N, M = G.M, nn = G.nn;
  const int t = threadIdx.x, lane = t & 63, wave = t >> 6, px = wave % MF_PX, ly = wave / MF_PX;
  const int f0 = lane & 3, f1 = (lane >> 2) & 3, f2 = lane >> 4;
  // XCD-aware tile order (tiles numbered x fastest)
  int tx, ty, bz;
  {
    const int L = xcd_order(blockIdx.x, G.nbx * G.nby * G.nbz);
    tx = L % G.nbx;
    ty = (L / G.nbx) % G.nby;
    bz = L / (G.nbx * G.nby);
  }
  const int ex = tx * MF_BX + 4 * px + f1, ey = ty * MF_BY + ly;
  const int X0 = tx * MF_BX * k, Y0 = ty * MF_BY * k;
  const int X1 = X0 + k * MF_BX, Y1 = Y0 + k * MF_BY;
  const int ez0 = bz * G.Bz, ez1 = min(N, ez0 + G.Bz);
  const int Z0 = ez0 * k, Z1 = ez1 * k;
  const bool valid = ex < N && ey < N;
  const int gi = ex * k + f0, gj = ey * k + f2;       // node column of this lane
  const bool bij = gi == 0 || gi == M - 1 || gj == 0 || gj == M - 1;
  const int col = valid ? gi + M * gj : 0;
  const double tB = mt_lane<MT_B>(f0, f2), tD1 = mt_lane<MT_D1>(f0, f2);
  const double tDh = mt_lane<MT_DH>(f0, f2), tBT = mt_lane<MT_BT>(f0, f2);
  const double tD1T = mt_lane<MT_D1T>(f0, f2);
  const double w_out = Wg<4, double>(0), w_in = Wg<4, double>(1);  // Gauss weights, outer / inner
  const double wxy = (f0 == 0 || f0 == 3 ? w_out : w_in) * (f2 == 0 || f2 == 3 ? w_out : w_in) * hh;

  // Node sums.  A node column of the tile gets the contributions of at most four elements of the
  // layer.  Within a wave, the lane in the element with the larger x (f0 = 0) adds its left
  // neighbour's value (f0 = 3, previous slot: lane - 1 of the same row of 16).  Through LDS, the
  // first element of the right wave of a tile row adds the right column of the left wave's last
  // element, and the lane in the element with the larger y (f2 = 0) adds the row below (f2 = 3,
  // summed within its wave); the one node column that joins four elements of two waves and two
  // rows also adds the corner of the left wave below.  The lane that ends up with a column's sum
  // owns it: f0 < 3 or the tile's last slot, f2 < 3 or the tile's last row.
  const bool xrecv = f0 == 0 && f1 > 0;
  const bool xsend = px < MF_PX - 1 && f0 == 3 && f1 == 3, xcross = px > 0 && f0 == 0 && f1 == 0;
  const bool ysend = f2 == 3 && ly < MF_BY - 1, yrecv = f2 == 0 && ly > 0;
  const bool diag = xcross && f2 == 0 && ly > 0;
  const bool owner = (f0 < 3 || (px == MF_PX - 1 && f1 == 3)) && (f2 < 3 || ly == MF_BY - 1) &&
                     gi < M && gj < M;
  const int yoff = wave * YW + f0 + 4 * f1;                 // this wave's top row
  const int xoff = XOFF + wave * XW + f2;                   // this (left) wave's right column
  // destination of the owner's values on planes inside the chunk and off the domain boundary in
  // z: a node store (with the epilogue), a brick-face slot, a Dirichlet zero, or nothing (another
  // brick emits it); the chunk's first and last planes take the general store_node
  enum { K_NODE = 0, K_FACE = 1, K_ZERO = 2, K_SKIP = 3 };
  int kind = K_SKIP, base = 0;
  {
    constexpr int KX = k * MF_BX, KY = k * MF_BY;
    const bool lx = gi == X0 && X0 > 0, ux = gi == X1 && X1 < M - 1;
    const bool lyb = gj == Y0 && Y0 > 0, uyb = gj == Y1 && Y1 < M - 1;
    if (!owner) kind = K_SKIP;
    else if (DIR && bij) kind = (lx || lyb) ? K_SKIP : K_ZERO;
    else if (!(lx || ux || lyb || uyb)) kind = K_NODE;
    else {
      kind = K_FACE;
      const int sl = (lx ? 1 : 0) + 2 * (lyb ? 1 : 0);
      if (lx || ux) base = (sl * (G.nbx - 1) + gi / KX - 1) * M * M + gj;
      else base = G.fy + (sl * (G.nby - 1) + gj / KY - 1) * M * M + gi;
    }
  }
  const int colg = gi + M * gj;
  // plain stores (no add): node, face slot and Dirichlet zero are one store sequence per lane,
  // with a per-lane destination, component stride and plane stride (no divergent branches)
  T* const dptr = kind == K_FACE ? face + base : y + colg;
  const size_t cstr = kind == K_FACE ? G.per_comp : (size_t)nn;
  const size_t zstr = kind == K_FACE ? (size_t)M : (size_t)M * M;
  auto store = [&](const double (&vd)[NC], int gz, bool general) {
    T val[NC];
#pragma unroll
    for (int c = 0; c < NC; ++c) val[c] = (T)vd[c];
    if (general) {
      if (owner)
        store_node<4, NC, T, DIR, EO>(G, gi, gj, gz, X0, Y0, Z0, X1, Y1, Z1, val, y, face, add, ep);
    } else if (EO == EPI_STORE && !add) {
      if (kind != K_SKIP) {
#pragma unroll
        for (int c = 0; c < NC; ++c)
          dptr[(size_t)c * cstr + zstr * gz] = kind == K_ZERO ? T(0) : val[c];
      }
    } else if (kind == K_NODE) {
#pragma unroll
      for (int c = 0; c < NC; ++c)
        emit<EO>(ep, (size_t)c * nn + (size_t)colg + (size_t)M * M * gz, val[c], y, add);
    } else if (kind == K_FACE) {
#pragma unroll
      for (int c = 0; c < NC; ++c) face[(size_t)c * G.per_comp + base + (size_t)M * gz] = val[c];
    } else if (kind == K_ZERO) {
#pragma unroll
      for (int c = 0; c < NC; ++c)
        emit<EO>(ep, (size_t)c * nn + (size_t)colg + (size_t)M * M * gz, T(0), y, add);
    }
  };
  // sums the np planes of v across the tile (v holds this lane's element contributions) and stores
  // them at z = zb + l; the first plane through store_node when first_general
  auto node_sums = [&](double (&v)[NC][3], int np, int zb, bool first_general, double* buf) {
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int l = 0; l < 3; ++l)
        if (l < np) {
          const double w = from_left(v[c][l]);
          if (xrecv) v[c][l] += w;
        }
    if (ysend) {
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int l = 0; l < 3; ++l)
          if (l < np) buf[yoff + (c * 3 + l) * 16] = v[c][l];
    }
    if (xsend) {
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int l = 0; l < 3; ++l)
          if (l < np) buf[xoff + (c * 3 + l) * 4] = v[c][l];
    }
    __syncthreads();
    if (xcross) {
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int l = 0; l < 3; ++l)
          if (l < np) v[c][l] += buf[xoff - XW + (c * 3 + l) * 4];
    }
    if (yrecv) {
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int l = 0; l < 3; ++l)
          if (l < np) v[c][l] += buf[yoff - MF_PX * YW + (c * 3 + l) * 16];
    }
    if (diag) {
#pragma unroll
      for (int c = 0; c < NC; ++c)
#pragma unroll
        for (int l = 0; l < 3; ++l)
          if (l < np) v[c][l] += buf[xoff - XW - MF_PX * XW + 3 + (c * 3 + l) * 4];
    }
#pragma unroll
    for (int l = 0; l < 3; ++l)
      if (l < np) {
        double val[NC];
#pragma unroll
        for (int c = 0; c < NC; ++c) val[c] = v[c][l];
        store(val, zb + l, l == 0 && first_general);
      }
  };

  double uc[NC][4];         // node columns of the current layer (masked)
  double carry[NC];         // contributions of the previous layer to its top plane
#pragma unroll
  for (int c = 0; c < NC; ++c) carry[c] = 0.0;
  // raw loads of node z-index gl of this lane's column (in-bounds for idle lanes: column 0),
  // masked afterwards (Dirichlet nodes and idle lanes: 0)
  auto raw_node = [&](int c, int gl) -> double {
    const size_t j = (size_t)c * nn + (size_t)col + (size_t)M * M * gl;
    if constexpr (EP == EPI_CHEB_ZERO || EP == EPI_ZERO_IN)
      return (double)(ep.gamma * ep.dinv[j] * ep.b[j]);
    else
      return (double)u[j];
  };
  auto live_node = [&](int gl) -> bool { return valid && !(DIR && (bij || gl == 0 || gl == M - 1)); };
  double cq[4];             // coefficient of the current layer at the lane's Gauss points
  // loads of one layer (nodes 1..3 of the column, coefficient); two sets, so that the loads of
  // the layer after next are in flight during a whole layer
  struct LBuf {
    double u[NC][3], c[4];
  };
  auto load_layer = [&](int ez, LBuf& b) {
    const size_t eb = (size_t)(valid ? ex + N * (ey + N * ez) : 0) * 64 + f0 + 4 * f2;
#pragma unroll
    for (int r = 0; r < 4; ++r) b.c[r] = (double)coef[eb + 16 * r];
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int r = 1; r < 4; ++r) b.u[c][r - 1] = raw_node(c, ez * k + r);
  };
  auto take_layer = [&](int ez, const LBuf& b) {
#pragma unroll
    for (int r = 0; r < 4; ++r) cq[r] = b.c[r];
#pragma unroll
    for (int r = 1; r < 4; ++r) {
      const int gl = ez * k + r;
      const double sc = sin_ != nullptr ? (double)sin_[(size_t)col + (size_t)M * M * gl] : 1.0;
      const bool lv = live_node(gl);
#pragma unroll
      for (int c = 0; c < NC; ++c) uc[c][r] = lv ? b.u[c][r - 1] * sc : 0.0;
    }
  };
#pragma unroll
  for (int c = 0; c < NC; ++c) {
    const double sc = sin_ != nullptr ? (double)sin_[(size_t)col + (size_t)M * M * Z0] : 1.0;
    uc[c][0] = live_node(Z0) ? raw_node(c, Z0) * sc : 0.0;
  }
  LBuf lb0, lb1;
  load_layer(ez0, lb0);
  take_layer(ez0, lb0);
  if (ez0 + 1 < ez1) load_layer(ez0 + 1, lb0);

  // one element layer: `next` holds the loads of layer ez + 1 (in flight), `fill` receives those
  // of layer ez + 2
  auto layer = [&](const int ez, const LBuf& next, LBuf& fill) {
    if (ez + 2 < ez1) load_layer(ez + 2, fill);
    double cw[4];
#pragma unroll
    for (int r = 0; r < 4; ++r) cw[r] = valid ? cq[r] * wxy * Wg<4, double>(r) : 0.0;

    // stresses at the lane's Gauss points (qx, qy) = (f0, f2), qz = register index
    double sg[NC == 3 ? 6 : 3][4];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      double w[4], gx_[4], gy_[4], gz_[4];
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        double a = 0.0;
#pragma unroll
        for (int l = 0; l < 4; ++l) a += Bm<4, double>(q, l) * uc[c][l];
        w[q] = a;
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        const double p = mf_swap(tB, w[r], 0.0);          // (qy, x)
        w[r] = mf_swap(tB, p, 0.0);                        // (qx, qy): Gauss values
        gx_[r] = mf_swap(tD1, p, 0.0);                     // x-derivative
      }
#pragma unroll
      for (int r = 0; r < 4; ++r) gy_[r] = mf_keep(tDh, w[r], 0.0);
#pragma unroll
      for (int q = 0; q < 4; ++q) {
        double a = 0.0;
#pragma unroll
        for (int m = 0; m < 4; ++m) a += Dm<4, double>(q, m) * w[m];
        gz_[q] = a;
      }
      if constexpr (NC == 1) {
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          sg[0][r] = cw[r] * gx_[r];
          sg[1][r] = cw[r] * gy_[r];
          sg[2][r] = cw[r] * gz_[r];
        }
      } else {
        // sg: 0 xx, 1 yy, 2 zz, 3 xy, 4 xz, 5 yz (symmetric gradient times 2 mu w |J| (2/h)^2)
#pragma unroll
        for (int r = 0; r < 4; ++r) {
          if (c == 0) {
            sg[0][r] = 2.0 * cw[r] * gx_[r];
            sg[3][r] = cw[r] * gy_[r];
            sg[4][r] = cw[r] * gz_[r];
          } else if (c == 1) {
            sg[3][r] += cw[r] * gx_[r];
            sg[1][r] = 2.0 * cw[r] * gy_[r];
            sg[5][r] = cw[r] * gz_[r];
          } else {
            sg[4][r] += cw[r] * gx_[r];
            sg[5][r] += cw[r] * gy_[r];
            sg[2][r] = 2.0 * cw[r] * gz_[r];
          }
        }
      }
    }
    // the bottom plane of the next layer is the top plane of this one
#pragma unroll
    for (int c = 0; c < NC; ++c) uc[c][0] = uc[c][3];

    double v3[NC][3];
#pragma unroll
    for (int c = 0; c < NC; ++c) {
      constexpr int SX[3] = {0, 3, 4}, SY[3] = {3, 1, 5}, SZ[3] = {4, 5, 2};
      const double* sx = sg[NC == 3 ? SX[c] : 0];
      const double* sy = sg[NC == 3 ? SY[c] : 1];
      const double* sz = sg[NC == 3 ? SZ[c] : 2];
      double o[4];
#pragma unroll
      for (int r = 0; r < 4; ++r) {
        double tz = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) tz += Dm<4, double>(q, r) * sz[q];
        const double a = mf_swap(tBT, sx[r], 0.0);          // (y, qx)
        double b = mf_swap(tD1T, sy[r], 0.0);
        b = mf_swap(tBT, tz, b);
        double oo = mf_swap(tD1T, a, 0.0);                   // (x, y)
        o[r] = mf_swap(tBT, b, oo);
      }
      double v[4];
#pragma unroll
      for (int l = 0; l < 4; ++l) {
        double a = 0.0;
#pragma unroll
        for (int q = 0; q < 4; ++q) a += Bm<4, double>(q, l) * o[q];
        v[l] = a;
      }
      v3[c][0] = v[0] + carry[c];
      v3[c][1] = v[1];
      v3[c][2] = v[2];
      carry[c] = v[3];
    }
    node_sums(v3, 3, ez * k, ez == ez0, ybuf + (ez & 1) * BUF);
    if (ez + 1 < ez1) take_layer(ez + 1, next);
  };
  for (int ez = ez0; ez < ez1; ez += 2) {
    layer(ez, lb0, lb1);
    if (ez + 1 < ez1) layer(ez + 1, lb1, lb0);
  }
  // top plane of the chunk
  double vt[NC][3];
#pragma unroll
  for (int c = 0; c < NC; ++c) vt[c][0] = vt[c][1] = vt[c][2] = carry[c];
  node_sums(vt, 1, Z1, true, ybuf + (ez1 & 1) * BUF);
}

// Gradient alone (B^T p) node by node.  On the uniform brick mesh every element carries the same
// gradient matrix: the tensor product of the 1D integrals GM[a][i] = int P_a l_i and
// GX[a][i] = int P_a l_i' (exact under the (k+1)-point Gauss rule), times -(h/2)^2 (eq. 2,
// B = -div).  A velocity node therefore gathers the pressure modes of the at most eight elements
// that contain it: no LDS, no face pass, every node written once.
struct GradTab {
  double GM[NMAX * NMAX], GX[NMAX * NMAX];  // [a n + i]
};

template <int n>
constexpr GradTab build_gradtab() {
  GradTab g{};
  const Tables& t = CT<n>::t;
  for (int a = 0; a < n - 1; ++a)
    for (int i = 0; i < n; ++i) {
      double m = 0.0, d = 0.0;
      for (int q = 0; q < n; ++q) {
        m += t.wg[q] * t.L[a * n + q] * t.B[q * n + i];
        d += t.wg[q] * t.L[a * n + q] * t.D1[q * n + i];
      }
      g.GM[a * n + i] = m;
      g.GX[a * n + i] = d;
    }
  return g;
}

template <int n>
struct CG {
  static constexpr GradTab t = build_gradtab<n>();
};

// Elements around a node coordinate g in one direction: the node lies in one element (local
// index 1..k-1) or, on an element boundary plane, in two (local index k in the lower, 0 in the
// upper).  The first candidate is e0 with weights GM/GX[.][i0], the second e1 with local index 0;
// an absent candidate gets zero weights and repeats a valid element index, so loads stay in bounds.
template <int n, typename T>
__device__ __forceinline__ void node_cands(const int g, const int N, int& e0, int& e1,
                                           T (&fm)[2][n - 1], T (&fd)[2][n - 1]) {
  constexpr int k = n - 1;
  const int r = g % k, q = g / k;
  const bool vert = r == 0;
  const bool v0 = !vert || q > 0, v1 = vert && q < N;
  const int i0 = vert ? k : r;
  e0 = vert ? (q > 0 ? q - 1 : 0) : q;
  e1 = v1 ? q : e0;
#pragma unroll
  for (int a = 0; a < k; ++a) {
    T m0 = T(0), d0 = T(0);
#pragma unroll
    for (int ii = 1; ii <= k; ++ii) {
      m0 = (i0 == ii) ? (T)CG<n>::t.GM[a * n + ii] : m0;
      d0 = (i0 == ii) ? (T)CG<n>::t.GX[a * n + ii] : d0;
    }
    fm[0][a] = v0 ? m0 : T(0);
    fd[0][a] = v0 ? d0 : T(0);
    fm[1][a] = v1 ? (T)CG<n>::t.GM[a * n] : T(0);
    fd[1][a] = v1 ? (T)CG<n>::t.GX[a * n] : T(0);
  }
}

// GM/GX[a][i] with a runtime local index i (selects over the compile-time table).
template <int n, typename T>
__device__ __forceinline__ void local_weights(const int i, T (&gm)[n - 1], T (&gx)[n - 1]) {
#pragma unroll
  for (int a = 0; a < n - 1; ++a) {
    T m = T(0), d = T(0);
#pragma unroll
    for (int ii = 0; ii < n; ++ii) {
      m = (i == ii) ? (T)CG<n>::t.GM[a * n + ii] : m;
      d = (i == ii) ? (T)CG<n>::t.GX[a * n + ii] : d;
    }
    gm[a] = m;
    gx[a] = d;
  }
}

// Gradient with the Dirichlet mask, one thread per x-line segment: thread (ex, gy, gz) writes the
// nodes gx = ex k .. ex k + k - 1 of the line (gy, gz), and the thread with ex = N - 1 also the
// boundary node gx = M - 1.  The pressure modes of the elements around the line (x elements ex - 1
// and ex, times the y and z candidates) are first contracted over y and z into Q[X][c][a] (x-mode
// a, component c), shared by the k nodes; each node then takes a k-term sum per x element.
template <int n, typename T>
__global__ void __launch_bounds__(256)
k_grad_line(const int N, const int M, const int nn, const T hh, const T* __restrict__ p,
            T* __restrict__ y, const int add) {
  constexpr int k = n - 1, NP = (n - 1) * n * (n + 1) / 6;
  // each thread contracts the modes of its own x element (ex) over y and z; the element on its
  // left (ex - 1) is its left neighbour thread's, read from LDS.  Blocks overlap by one: thread 0
  // only contracts the element left of the block's first output, threads 1..255 write outputs.
  __shared__ T qs[3 * k][256];
  const int t = xcd_order(blockIdx.x, gridDim.x) * (blockDim.x - 1) + (int)threadIdx.x - 1;
  const bool valid = t >= 0 && t < N * M * M;
  const int tt = valid ? t : 0;
  const int ex = tt % N, gy = (tt / N) % M, gz = tt / (N * M);
  const bool inner = valid && gy > 0 && gy < M - 1 && gz > 0 && gz < M - 1;
  int y0, y1, z0, z1;
  T fmy[2][k], fdy[2][k], fmz[2][k], fdz[2][k];
  node_cands<n, T>(gy, N, y0, y1, fmy, fdy);
  node_cands<n, T>(gz, N, z0, z1, fmz, fdz);
  auto contract = [&](const int X, T (&Q)[3][k]) {
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int a = 0; a < k; ++a) Q[c][a] = T(0);
#pragma unroll
    for (int sz = 0; sz < 2; ++sz)
#pragma unroll
      for (int sy = 0; sy < 2; ++sy) {
        const T* pe = p + ((size_t)N * ((sy ? y1 : y0) + (size_t)N * (sz ? z1 : z0)) + X) * NP;
#pragma unroll
        for (int m = 0; m < NP; ++m) {
          const int a = CT<n>::t.ma[m], b = CT<n>::t.mb[m], c = CT<n>::t.mc[m];
          const T pm = pe[m];
          Q[0][a] += pm * (fmy[sy][b] * fmz[sz][c]);
          Q[1][a] += pm * (fdy[sy][b] * fmz[sz][c]);
          Q[2][a] += pm * (fmy[sy][b] * fdz[sz][c]);
        }
      }
  };
  T Q1[3][k], Q0[3][k];
  if (inner) {
    contract(ex, Q1);
  } else {
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int a = 0; a < k; ++a) Q1[c][a] = T(0);
  }
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int a = 0; a < k; ++a) qs[c * k + a][threadIdx.x] = Q1[c][a];
  __syncthreads();
  if (!valid || threadIdx.x == 0) return;
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int a = 0; a < k; ++a) Q0[c][a] = (inner && ex > 0) ? qs[c * k + a][threadIdx.x - 1] : T(0);
  T v[k][3];
  const T h2 = -hh * hh;
#pragma unroll
  for (int i = 0; i < k; ++i)
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      T acc = T(0);
#pragma unroll
      for (int a = 0; a < k; ++a) {
        acc += Q1[c][a] * (T)(c == 0 ? CG<n>::t.GX[a * n + i] : CG<n>::t.GM[a * n + i]);
        if (i == 0) acc += Q0[c][a] * (T)(c == 0 ? CG<n>::t.GX[a * n + k] : CG<n>::t.GM[a * n + k]);
      }
      v[i][c] = (!inner || (i == 0 && ex == 0)) ? T(0) : acc * h2;
    }
  const size_t base = (size_t)ex * k + (size_t)M * (gy + (size_t)M * gz);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
#pragma unroll
    for (int i = 0; i < k; ++i) {
      const size_t j = (size_t)c * nn + base + i;
      y[j] = add ? y[j] + v[i][c] : v[i][c];
    }
    if (ex == N - 1) {
      const size_t j = (size_t)c * nn + base + k;
      y[j] = add ? y[j] : T(0);
    }
  }
}

// Divergence with the Dirichlet mask (and an optional per-node input scaling).  A block holds n
// wavefronts on the same 64 consecutive elements (lane = element, consecutive in x, so each load
// instruction covers a contiguous run of nodes and the n loads of a node line reuse its cache
// lines); wavefront l takes the node lines (j, l), j = 0..k, of its element: it contracts each
// line's nodes in x into R_c[a] and adds the line's share of every mode.  The n partial sums of
// an element are added in LDS in the order l = 0..k and go out through the epilogue (pressure
// outputs e n_p + m).
template <int n, typename T, int EP, bool SCALE>
__global__ void __launch_bounds__(64 * n)
k_div_elem(const int N, const int M, const int E, const int nn, const T hh,
           const T* __restrict__ u, const T* __restrict__ sin_, T* __restrict__ pout,
           const int add, const Epi<T> ep) {
  constexpr int k = n - 1, NP = (n - 1) * n * (n + 1) / 6;
  __shared__ T red[NP * 64];
  const int lane = threadIdx.x & 63, l = threadIdx.x >> 6;
  const int e = xcd_order(blockIdx.x, gridDim.x) * 64 + lane;
  const bool valid = e < E;
  const int ee = valid ? e : E - 1;   // idle lanes load in bounds and are masked
  const int ex = ee % N, ey = (ee / N) % N, ez = ee / (N * N);
  const int gz = ez * k + l;
  const bool zin = valid && gz > 0 && gz < M - 1;
  T gml[k], gxl[k];
  local_weights<n, T>(l, gml, gxl);
  T acc[NP];
#pragma unroll
  for (int m = 0; m < NP; ++m) acc[m] = T(0);
  // all lines' loads in flight at once up to order 3; one line at a time above (registers)
#pragma unroll(n <= 4 ? n : 1)
  for (int j = 0; j < n; ++j) {
    const int gy = ey * k + j;
    const bool row = zin && gy > 0 && gy < M - 1;
    const size_t gyz = (size_t)M * (gy + (size_t)M * gz);
    T uv[n][3], sv[n];
#pragma unroll
    for (int i = 0; i < n; ++i) {
      const size_t gn = (size_t)ex * k + i + gyz;
#pragma unroll
      for (int c = 0; c < 3; ++c) uv[i][c] = u[(size_t)c * nn + gn];
      if constexpr (SCALE) sv[i] = sin_[gn];   // a template flag: no branch between the loads
      else sv[i] = T(1);
    }
    T R[3][k];
#pragma unroll
    for (int c = 0; c < 3; ++c)
#pragma unroll
      for (int a = 0; a < k; ++a) R[c][a] = T(0);
#pragma unroll
    for (int i = 0; i < n; ++i) {
      const int gx = ex * k + i;
      const T sc = (row && gx > 0 && gx < M - 1) ? sv[i] : T(0);
#pragma unroll
      for (int a = 0; a < k; ++a) {
        const T mi = (T)CG<n>::t.GM[a * n + i], di = (T)CG<n>::t.GX[a * n + i];
        R[0][a] += di * (sc * uv[i][0]);
        R[1][a] += mi * (sc * uv[i][1]);
        R[2][a] += mi * (sc * uv[i][2]);
      }
    }
    T gmj[k], gxj[k];
    local_weights<n, T>(j, gmj, gxj);
#pragma unroll
    for (int m = 0; m < NP; ++m) {
      const int a = CT<n>::t.ma[m], b = CT<n>::t.mb[m], c = CT<n>::t.mc[m];
      acc[m] += R[0][a] * (gmj[b] * gml[c]) + R[1][a] * (gxj[b] * gml[c]) +
                R[2][a] * (gmj[b] * gxl[c]);
    }
  }
  // the epilogue's loads of this thread's outputs (modes l, l + n, ...) go out before the sums,
  // so that their latency overlaps the reduction instead of following it
  constexpr int MO = (NP + n - 1) / n;
  EpiIn<T> pre[MO];
#pragma unroll
  for (int i = 0; i < MO; ++i) {
    const int m = l + n * i;
    if (valid && m < NP) pre[i] = epi_load<EP>(ep, (size_t)e * NP + m, pout, add);
  }
  for (int w = 0; w < n; ++w) {
    if (l == w) {
#pragma unroll
      for (int m = 0; m < NP; ++m) red[m * 64 + lane] = (w == 0 ? T(0) : red[m * 64 + lane]) + acc[m];
    }
    __syncthreads();
  }
#pragma unroll
  for (int i = 0; i < MO; ++i) {
    const int m = l + n * i;
    if (valid && m < NP)
      epi_store<EP>(ep, (size_t)e * NP + m, -hh * hh * red[m * 64 + lane], pre[i], pout, add);
  }
}

// Sum the partial values on internal brick planes into y (x planes, then y planes not on an
// x plane, then z planes on neither).
template <int n, int NC, typename T, bool DIR, int EP>
__global__ void k_face_sum(const BrickDev G, const T* __restrict__ face, T* __restrict__ y,
                           const int add, const Epi<T> ep) {
  // 32-bit index arithmetic: the face nodes number (nbx + nby + nbz - 3) M^2 < 2^31
  const int M = G.M, MM = M * M;
  const int nx = (G.nbx - 1) * MM, ny = (G.nby - 1) * MM, nz = (G.nbz - 1) * MM;
  int idx = blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= nx + ny + nz) return;
  constexpr int k = n - 1, KX = k * Tile<n>::BX, KY = k * Tile<n>::BY;
  const int KZ = k * G.Bz;
  int gx, gy, gz, cat, b;
  if (idx < nx) {
    cat = 0;
    b = idx / MM;
    const int rem = idx - b * MM;
    gz = rem / M;
    gy = rem - gz * M;
    gx = (b + 1) * KX;
  } else if (idx < nx + ny) {
    idx -= nx;
    cat = 1;
    b = idx / MM;
    const int rem = idx - b * MM;
    gz = rem / M;
    gx = rem - gz * M;
    gy = (b + 1) * KY;
  } else {
    idx -= nx + ny;
    cat = 2;
    b = idx / MM;
    const int rem = idx - b * MM;
    gy = rem / M;
    gx = rem - gy * M;
    gz = (b + 1) * KZ;
  }
  const bool on_x = gx % KX == 0 && gx > 0 && gx < M - 1;
  const bool on_y = gy % KY == 0 && gy > 0 && gy < M - 1;
  const bool on_z = gz % KZ == 0 && gz > 0 && gz < M - 1;
  if (cat == 1 && on_x) return;
  if (cat == 2 && (on_x || on_y)) return;
  if (DIR && (gx == 0 || gx == M - 1 || gy == 0 || gy == M - 1 || gz == 0 || gz == M - 1)) return;
  T val[NC];
#pragma unroll
  for (int c = 0; c < NC; ++c) val[c] = T(0);
  for (int sz = 0; sz <= (on_z ? 1 : 0); ++sz)
    for (int sy = 0; sy <= (on_y ? 1 : 0); ++sy)
      for (int sx = 0; sx <= (on_x ? 1 : 0); ++sx) {
        const int s = sx + 2 * sy + 4 * sz;
        size_t off;
        if (cat == 0) off = ((size_t)(s * (G.nbx - 1) + b) * M + gz) * M + gy;
        else if (cat == 1) off = G.fy + ((size_t)(s * (G.nby - 1) + b) * M + gz) * M + gx;
        else off = G.fz + ((size_t)(s * (G.nbz - 1) + b) * M + gy) * M + gx;
#pragma unroll
        for (int c = 0; c < NC; ++c) val[c] += face[(size_t)c * G.per_comp + off];
      }
  const size_t g = (size_t)gx + (size_t)M * (gy + (size_t)M * gz);
#pragma unroll
  for (int c = 0; c < NC; ++c) emit<EP>(ep, (size_t)c * G.nn + g, val[c], y, add);
}

// The epilogue of an operator apply as a pass of its own: t holds the operator's output, and
// t is the buffer the epilogue overwrites only after reading it at the same index (r for the
// residual, the new search direction otherwise), so t carries no restrict qualifier.
template <typename T, int EP>
__global__ void __launch_bounds__(256) k_epi_apply(const size_t n, const T* t, const Epi<T> ep) {
  const size_t j = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j < n) {
    const T v = t[j];
    emit<EP>(ep, j, v, static_cast<T*>(nullptr), 0);
  }
}

template <int EP, typename T>
T* epi_target(const Epi<T>& ep) {
  return EP == EPI_RESID ? ep.r : ep.dnew;
}

struct ProfScope {
  hipEvent_t a = nullptr, b = nullptr;
  hipStream_t st;
  std::string key;
  ProfScope(hipStream_t s, std::string k) : st(s), key(std::move(k)) {
    if (!prof::on) return;
    hipStreamCaptureStatus cs = hipStreamCaptureStatusNone;
    if (hipStreamIsCapturing(st, &cs) != hipSuccess || cs != hipStreamCaptureStatusNone) return;
    std::lock_guard<std::mutex> g(prof::mu);
    a = prof::get_event();
    b = prof::get_event();
    if (a) (void)hipEventRecord(a, st);
  }
  ~ProfScope() {
    if (!a || !b) return;
    std::lock_guard<std::mutex> g(prof::mu);
    (void)hipEventRecord(b, st);
    prof::recs.push_back({key, a, b});
  }
};

std::string op_key(int NC, int k, int N, int F, bool scale, size_t es, const char* part) {
  char key[160];
  snprintf(key, sizeof(key), "op%s nc=%d k=%d N=%d flags=%s%s%s%s%s %s", part, NC, k, N,
           (F & F_A) ? "A" : "", (F & F_BT) ? "+BT" : "", (F & F_B) ? "+B" : "",
           (F & F_DIR) ? "+dir" : "", scale ? "+scale" : "",
           es == 8 ? "f64" : ((F & F_MF3) ? "f32+bf16x3mfma" : ((F & F_MF) ? "f32+bf16mfma" : "f32")));
  return key;
}

template <int n, int NC, typename T, int F, int MF, int EP>
void op_launch_ep(hipStream_t st, int N, int k, const T* u, T* y, const T* coef, const T* pin,
                  T* pout, const T* sin, bool add, void* work, const Epi<T>& ep) {
  const int M = k * N + 1, E = N * N * N, nn = M * M * M;
  const T hh = (T)(0.5 / N);
  const int Fk = F | (MF == 1 ? F_MF : 0) | (MF == 3 ? F_MF3 : 0);
  if constexpr ((F & (F_A | F_BT)) == 0) {
    constexpr int SLOTS = 4 * WaveMap<n>::EPW;
    ProfScope ps(st, op_key(NC, k, N, Fk, sin != nullptr, sizeof(T), ""));
    if constexpr (MF == 0 && (F & F_DIR) != 0)
      if (sin != nullptr)
        hipLaunchKernelGGL((k_div_elem<n, T, EP, true>), dim3(grid_for(E, 64)), dim3(64 * n), 0, st, N,
                           M, E, nn, hh, u, sin, pout, (int)add, ep);
      else
        hipLaunchKernelGGL((k_div_elem<n, T, EP, false>), dim3(grid_for(E, 64)), dim3(64 * n), 0, st,
                           N, M, E, nn, hh, u, sin, pout, (int)add, ep);
    else
      hipLaunchKernelGGL((k_op_gather<n, T, F, MF, EP>), dim3(grid_for(E, SLOTS)), dim3(256), 0, st,
                         N, k, M, E, nn, hh, u, pout, sin, (int)add, ep);
  } else if constexpr ((F & (F_A | F_B)) == 0 && (F & F_DIR) != 0 && NC == 3 && MF == 0 &&
                       EP == EPI_STORE) {
    ProfScope ps(st, op_key(NC, k, N, Fk, sin != nullptr, sizeof(T), ""));
    hipLaunchKernelGGL((k_grad_line<n, T>), dim3(grid_for((size_t)N * M * M, 255)), dim3(256), 0, st,
                       N, M, nn, hh, pin, y, (int)add);
  } else {
    if constexpr ((F & (F_BT | F_B)) == 0) {
      if (two_pass(NC, N, k)) {
        constexpr int SLOTS = 4 * WaveMap<n>::EPW;
        T* buf = static_cast<T*>(work);
        {
          ProfScope ps(st, op_key(NC, k, N, Fk, sin != nullptr, sizeof(T), ""));
          hipLaunchKernelGGL((k_op_elem<n, NC, T, F, MF, EP>), dim3(grid_for(E, SLOTS)), dim3(256), 0,
                             st, N, k, M, E, nn, hh, u, coef, sin, buf, ep);
        }
        ProfScope ps(st, op_key(NC, k, N, Fk, sin != nullptr, sizeof(T), "-faces"));
        hipLaunchKernelGGL((k_node_sum<n, NC, T, (F & F_DIR) != 0, EP>), dim3(grid_for(nn, 256)),
                           dim3(256), 0, st, N, M, nn, buf, y, (int)add, ep);
        return;
      }
    }
    constexpr int BX = Tile<n>::BX, BY = Tile<n>::BY;
    const BrickGeom G = brick_geom(N, k, BX, BY);
    const BrickDev D = brick_dev(G);
    T* face = static_cast<T*>(work);
    {
      ProfScope ps(st, op_key(NC, k, N, Fk, sin != nullptr, sizeof(T), ""));
      bool done = false;
      if constexpr (n == 4 && MF == 0 && (F & (F_BT | F_B)) == 0) {
        if (matrix_core_ops.load(std::memory_order_relaxed)) {
          if constexpr (EP == EPI_STORE) {
            hipLaunchKernelGGL((k_op_mfma<NC, T, F, EPI_STORE>), dim3(G.nbx * G.nby * G.nbz),
                               dim3(MF_NT), 0, st, D, (double)hh, u, y, coef, sin, face, (int)add,
                               ep);
            done = true;
          } else {
            // The epilogue runs as a separate streaming pass: fused into this kernel, its loads
            // wait behind the layer prefetch and stall every layer.  The operator output goes
            // to the buffer the epilogue overwrites last (bit-identical results).
            constexpr int EK = EP == EPI_CHEB_ZERO ? EPI_ZERO_IN : EPI_STORE;
            T* t = epi_target<EP>(ep);
            hipLaunchKernelGGL((k_op_mfma<NC, T, F, EK>), dim3(G.nbx * G.nby * G.nbz),
                               dim3(MF_NT), 0, st, D, (double)hh, u, t, coef, sin, face, 0, ep);
            const size_t tot = (size_t)(G.nbx + G.nby + G.nbz - 3) * G.plane;
            if (tot > 0)
              hipLaunchKernelGGL((k_face_sum<n, NC, T, (F & F_DIR) != 0, EPI_STORE>),
                                 dim3(grid_for(tot, 256)), dim3(256), 0, st, D, face, t, 0, ep);
            const size_t len = (size_t)NC * nn;
            hipLaunchKernelGGL((k_epi_apply<T, EP>), dim3(grid_for(len, 256)), dim3(256), 0, st,
                               len, (const T*)t, ep);
            return;
          }
        }
      }
      if (!done)
        hipLaunchKernelGGL((k_op_brick<n, NC, T, F, MF, EP>), dim3(G.nbx * G.nby, G.nbz),
                           dim3(BrickThreads<n>::NT), 0, st, D, hh, u, y, coef, pin, pout, sin, face,
                           (int)add, ep);
    }
    const size_t tot = (size_t)(G.nbx + G.nby + G.nbz - 3) * G.plane;
    if (tot > 0) {
      ProfScope ps(st, op_key(NC, k, N, Fk, sin != nullptr, sizeof(T), "-faces"));
      hipLaunchKernelGGL((k_face_sum<n, NC, T, (F & F_DIR) != 0, EP>), dim3(grid_for(tot, 256)),
                         dim3(256), 0, st, D, face, y, (int)add, ep);
    }
  }
}

// Epilogues other than the plain store exist for the level operators (A with or without the
// Dirichlet mask) and for the divergence alone (its pressure output: Chebyshev steps on K_w).
template <int n, int NC, typename T, int F, int MF>
void op_launch(hipStream_t st, int N, int k, const T* u, T* y, const T* coef, const T* pin, T* pout,
               const T* sin, bool add, void* work, const Epi<T>& ep) {
  if constexpr (F == F_A || F == (F_A | F_DIR) || F == (F_B | F_DIR)) {
    switch (ep.mode) {
      case EPI_RESID:
        return op_launch_ep<n, NC, T, F, MF, EPI_RESID>(st, N, k, u, y, coef, pin, pout, sin, add,
                                                        work, ep);
      case EPI_CHEB_FIRST:
        return op_launch_ep<n, NC, T, F, MF, EPI_CHEB_FIRST>(st, N, k, u, y, coef, pin, pout, sin,
                                                             add, work, ep);
      case EPI_CHEB_ZERO:
        if constexpr ((F & F_A) != 0)
          return op_launch_ep<n, NC, T, F, MF, EPI_CHEB_ZERO>(st, N, k, u, y, coef, pin, pout, sin,
                                                              add, work, ep);
        break;
      case EPI_CHEB_STEP:
        return op_launch_ep<n, NC, T, F, MF, EPI_CHEB_STEP>(st, N, k, u, y, coef, pin, pout, sin,
                                                            add, work, ep);
      default:
        break;
    }
  } else {
    WB_REQUIRE(ep.mode == EPI_STORE, WB_EUNSUPPORTED, "epilogue not built for this operator");
  }
  op_launch_ep<n, NC, T, F, MF, EPI_STORE>(st, N, k, u, y, coef, pin, pout, sin, add, work, ep);
}

template <int n, typename T, int MF>
void op_dispatch_mf(hipStream_t st, int flags, int NC, int N, int k, const T* u, T* y,
                    const T* coef, const T* pin, T* pout, const T* sin, bool add, void* work,
                    const Epi<T>& ep) {
  if (NC == 1) {
    if (flags == F_A)
      return op_launch<n, 1, T, F_A, MF>(st, N, k, u, y, coef, pin, pout, sin, add, work, ep);
  } else {
    switch (flags) {
      case F_A | F_DIR:
        return op_launch<n, 3, T, F_A | F_DIR, MF>(st, N, k, u, y, coef, pin, pout, sin, add, work, ep);
      case F_A | F_BT | F_B | F_DIR:
        if constexpr (MF == 0) {
          // at order 5 the fused kernel spills, and at order 3 above the two-pass size the
          // matrix-core A with the line kernels of B^T and B is faster than the fused LDS-line
          // kernel: A, then B^T added, then B (same results up to rounding order)
          bool split = n == 6;
          if constexpr (n == 4)
            split = matrix_core_ops.load(std::memory_order_relaxed) && !two_pass(3, N, k) &&
                    ep.mode == EPI_STORE && sin == nullptr;
          if (split) {
            WB_REQUIRE(ep.mode == EPI_STORE && sin == nullptr, WB_EUNSUPPORTED,
                       "fused Stokes operator: plain store only");
            op_launch<n, 3, T, F_A | F_DIR, MF>(st, N, k, u, y, coef, nullptr, nullptr, nullptr, add,
                                                work, ep);
            op_launch<n, 3, T, F_BT | F_DIR, MF>(st, N, k, nullptr, y, nullptr, pin, nullptr, nullptr,
                                                 true, work, ep);
            return op_launch<n, 3, T, F_B | F_DIR, MF>(st, N, k, u, nullptr, nullptr, nullptr, pout,
                                                       nullptr, false, work, ep);
          } else if constexpr (n != 6) {
            return op_launch<n, 3, T, F_A | F_BT | F_B | F_DIR, MF>(st, N, k, u, y, coef, pin, pout,
                                                                    sin, add, work, ep);
          }
        }
        break;
      case F_B | F_DIR:
        return op_launch<n, 3, T, F_B | F_DIR, MF>(st, N, k, u, y, coef, pin, pout, sin, add, work, ep);
      case F_BT | F_DIR:
        return op_launch<n, 3, T, F_BT | F_DIR, MF>(st, N, k, u, y, coef, pin, pout, sin, add, work, ep);
      default:
        break;
    }
  }
  throw Error{WB_EUNSUPPORTED, "operator flag combination not built"};
}

template <int n, typename T>
void op_dispatch_n(hipStream_t st, int flags, int NC, int N, int k, const T* u, T* y, const T* coef,
                   const T* pin, T* pout, const T* sin, bool add, void* work, const Epi<T>& ep) {
  if ((flags & (F_MF | F_MF3)) != 0) {
    if constexpr (sizeof(T) == 4 && n <= 5) {
      if ((flags & F_MF3) != 0)
        return op_dispatch_mf<n, T, 3>(st, flags & ~(F_MF | F_MF3), NC, N, k, u, y, coef, pin, pout,
                                       sin, add, work, ep);
      return op_dispatch_mf<n, T, 1>(st, flags & ~F_MF, NC, N, k, u, y, coef, pin, pout, sin, add,
                                     work, ep);
    }
    throw Error{WB_EUNSUPPORTED, "BF16 contractions are built for FP32 data and k <= 4 only"};
  }
  return op_dispatch_mf<n, T, 0>(st, flags, NC, N, k, u, y, coef, pin, pout, sin, add, work, ep);
}

// ------------------------------------------------------------------ assembled Q1 levels
// Element matrices of the Q1 level operator, taken from the element kernel itself: column
// (j, d) is the element operator applied to the unit vector of local node j = jx + 2 jy + 4 jz,
// component d (the zero vector when that node is a Dirichlet node of a masked operator).
// ae[e][j NC + d][i NC + c]; rows of Dirichlet nodes are dropped by the gather.
template <int NC, bool DIR>
__global__ void __launch_bounds__(256)
k_elem_matrix(const int N, const double hh, const double* __restrict__ coef, double* __restrict__ ae) {
  constexpr int n = 2, EPW = WaveMap<n>::EPW, SLOTS = 4 * EPW, SL = Lds<n, 8>::SL, ND = 8 * NC;
  __shared__ double sm[2 * (SLOTS + 1) * SL];
  int slot, r;
  bool lane_ok;
  WaveMap<n>::map(threadIdx.x, slot, r, lane_ok);
  const int E = N * N * N, M = N + 1;
  const int e = blockIdx.x * SLOTS + slot;
  const bool valid = lane_ok && e < E;
  int ex = 0, ey = 0, ez = 0;
  if (valid) {
    ex = e % N;
    ey = (e / N) % N;
    ez = e / (N * N);
  }
  double* s0 = sm + (lane_ok ? slot : SLOTS) * SL;
  const int a = r % n, b = r / n;
  ElemIn<n, NC, double> in;
  const size_t eb = (size_t)(valid ? e : 0) * 8 + b * 2 + a;  // in bounds for idle lanes
#pragma unroll
  for (int q = 0; q < n; ++q) in.cq[q] = coef[eb + q * 4];
  for (int col = 0; col < ND; ++col) {
    const int j = col / NC, d = col % NC;
    const int jx = j & 1, jy = (j >> 1) & 1, jz = j >> 2;
    const int gx = ex + jx, gy = ey + jy, gz = ez + jz;
    const bool dead = DIR && (gx == 0 || gx == M - 1 || gy == 0 || gy == M - 1 || gz == 0 || gz == M - 1);
#pragma unroll
    for (int c = 0; c < NC; ++c)
#pragma unroll
      for (int l = 0; l < n; ++l)
        in.uz[c][l] = (!dead && c == d && a == jx && b == jy && l == jz) ? 1.0 : 0.0;
    double* out = ae + ((size_t)(valid ? e : 0) * ND + col) * ND;
    element_op<n, NC, double, F_A, 0>(valid, e, 1, hh, in, nullptr, [](size_t, double) {}, s0,
                                      s0 + (SLOTS + 1) * SL, r,
                                      [&](int c, int x, int yy, int z, double v) {
                                        if (valid) out[(x + 2 * yy + 4 * z) * NC + c] = v;
                                      });
  }
}

// 27-point stencil of an assembled Q1 level: S[((o NC + c) NC + d) nn + i] couples component c
// of node i with component d of node i + offset o, o = (ox+1) + 3 (oy+1) + 9 (oz+1); it sums
// the element-matrix entries of the elements holding both nodes.  Entries reaching outside the
// mesh, rows of Dirichlet nodes (DIR) and columns of Dirichlet nodes are zero.
template <int NC, bool DIR>
__global__ void k_stencil_gather(const int N, const double* __restrict__ ae, double* __restrict__ S) {
  constexpr int ND = 8 * NC;
  const int M = N + 1, nn = M * M * M;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= 27LL * nn) return;
  const int o = (int)(idx / nn), i = (int)(idx % nn);
  const int ix = i % M, iy = (i / M) % M, iz = i / (M * M);
  const int jx = ix + o % 3 - 1, jy = iy + (o / 3) % 3 - 1, jz = iz + o / 9 - 1;
  double acc[NC][NC];
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int d = 0; d < NC; ++d) acc[c][d] = 0.0;
  const bool row_dead = DIR && (ix == 0 || ix == M - 1 || iy == 0 || iy == M - 1 || iz == 0 || iz == M - 1);
  const bool in_mesh = jx >= 0 && jx < M && jy >= 0 && jy < M && jz >= 0 && jz < M;
  if (in_mesh && !row_dead) {
    for (int ez = iz - 1; ez <= iz; ++ez) {
      if (ez < 0 || ez >= N || jz < ez || jz > ez + 1) continue;
      for (int ey = iy - 1; ey <= iy; ++ey) {
        if (ey < 0 || ey >= N || jy < ey || jy > ey + 1) continue;
        for (int ex = ix - 1; ex <= ix; ++ex) {
          if (ex < 0 || ex >= N || jx < ex || jx > ex + 1) continue;
          const size_t e = (size_t)ex + (size_t)N * (ey + (size_t)N * ez);
          const int il = (ix - ex) + 2 * (iy - ey) + 4 * (iz - ez);
          const int jl = (jx - ex) + 2 * (jy - ey) + 4 * (jz - ez);
          const double* m = ae + e * ND * ND;
#pragma unroll
          for (int c = 0; c < NC; ++c)
#pragma unroll
            for (int d = 0; d < NC; ++d) acc[c][d] += m[(jl * NC + d) * ND + il * NC + c];
        }
      }
    }
  }
#pragma unroll
  for (int c = 0; c < NC; ++c)
#pragma unroll
    for (int d = 0; d < NC; ++d) S[((size_t)(o * NC + c) * NC + d) * nn + i] = acc[c][d];
}

// y = S u for an assembled Q1 level (one thread per output component c and node i), with the
// same epilogues as the element kernels.  One-wave blocks spread the small grids of the coarse
// levels over more compute units.
constexpr int STENCIL_BLOCK = 64;
template <int NC, typename T, int EP>
__global__ void __launch_bounds__(STENCIL_BLOCK)
k_stencil(const int M, const T* __restrict__ S, const T* __restrict__ u, T* __restrict__ y,
          const int add, const Epi<T> ep) {
  const int nn = M * M * M;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)NC * nn) return;
  const int c = (int)(idx / nn), i = (int)(idx % nn);
  const int ix = i % M, iy = (i / M) % M, iz = i / (M * M);
  // loads without branches (neighbours outside the mesh read node i and are selected away), so
  // that a whole plane of offsets is in flight at once
  bool inx[3], iny[3];
#pragma unroll
  for (int t = 0; t < 3; ++t) {
    inx[t] = ix + t - 1 >= 0 && ix + t - 1 < M;
    iny[t] = iy + t - 1 >= 0 && iy + t - 1 < M;
  }
  T acc = T(0);
#pragma unroll
  for (int oz = 0; oz < 3; ++oz) {
    const bool inz = iz + oz - 1 >= 0 && iz + oz - 1 < M;
    T sv[9][NC], uv[9][NC];
#pragma unroll
    for (int oy = 0; oy < 3; ++oy)
#pragma unroll
      for (int ox = 0; ox < 3; ++ox) {
        const int p = ox + 3 * oy, o = p + 9 * oz;
        const bool in = inz && iny[oy] && inx[ox];
        const int j = in ? i + (ox - 1) + M * ((oy - 1) + M * (oz - 1)) : i;
#pragma unroll
        for (int d = 0; d < NC; ++d) {
          const size_t jd = (size_t)d * nn + j;
          sv[p][d] = S[((size_t)(o * NC + c) * NC + d) * nn + i];
          if constexpr (EP == EPI_CHEB_ZERO) uv[p][d] = ep.gamma * ep.dinv[jd] * ep.b[jd];
          else uv[p][d] = u[jd];
        }
      }
#pragma unroll
    for (int oy = 0; oy < 3; ++oy)
#pragma unroll
      for (int ox = 0; ox < 3; ++ox) {
        const int p = ox + 3 * oy;
        const bool in = inz && iny[oy] && inx[ox];
#pragma unroll
        for (int d = 0; d < NC; ++d) acc += in ? sv[p][d] * uv[p][d] : T(0);
      }
  }
  emit<EP>(ep, (size_t)c * nn + i, acc, y, add);
}

// Coarse tail of a scalar (Neumann) V-cycle in one workgroup: Chebyshev-Jacobi smoothing on an
// assembled Q1 level of at most TAIL_MAX nodes, residual, restriction (linear 2:1), the coarsest
// dense solve, prolongation and post-smoothing, with every vector in LDS and thread t owning
// node t (its 27 stencil entries held in registers).  The steps are those of the per-kernel path
// (k_cheb_first, k_stencil with its epilogues, k_lin21, k_dense); the coarsest product sums each
// row over eight lanes instead of a wavefront, so it differs from k_dense by rounding order.
template <typename T>
__device__ inline T tail_apply(const int M, const int t, const int ix, const int iy, const int iz,
                               const T (&sr)[27], const T* v) {
  T acc = T(0);
#pragma unroll
  for (int o = 0; o < 27; ++o) {
    const int ox = o % 3 - 1, oy = (o / 3) % 3 - 1, oz = o / 9 - 1;
    const bool in = ix + ox >= 0 && ix + ox < M && iy + oy >= 0 && iy + oy < M && iz + oz >= 0 &&
                    iz + oz < M;
    const T vj = v[in ? t + ox + M * (oy + M * oz) : t];
    acc += in ? sr[o] * vj : T(0);
  }
  return acc;
}

template <typename T>
__global__ void __launch_bounds__(TAIL_THREADS)
k_vcycle_tail(const TailArgs<T> a, const T* __restrict__ bg, T* __restrict__ xg) {
  __shared__ T b[TAIL_MAX], x[TAIL_MAX], r[TAIL_MAX], dv[2][TAIL_MAX], bc[TAIL_MAX], xc[TAIL_MAX];
  const int t = threadIdx.x, M = a.M, nn = M * M * M, Mc = a.Mc, nc = Mc * Mc * Mc;
  const bool own = t < nn;
  const int tt = own ? t : 0, ix = tt % M, iy = (tt / M) % M, iz = tt / (M * M);
  T sr[27];
#pragma unroll
  for (int o = 0; o < 27; ++o) sr[o] = own ? a.S[(size_t)o * nn + t] : T(0);
  const T dinv = own ? a.dinv[t] : T(0);
  // pre-smoothing from x = 0
  int cur = 0;
  if (own) {
    const T bt = bg[t];
    const T di = a.inv_theta * dinv * bt;
    b[t] = bt;
    r[t] = bt;
    dv[0][t] = di;
    x[t] = di;
  }
  __syncthreads();
  for (int it = 1; it < a.deg; ++it) {
    const T v = tail_apply<T>(M, tt, ix, iy, iz, sr, dv[cur]);
    if (own) {
      const T ri = r[t] - v;
      const T dn = a.alpha[it] * dv[cur][t] + a.beta[it] * dinv * ri;
      r[t] = ri;
      dv[cur ^ 1][t] = dn;
      x[t] += dn;
    }
    __syncthreads();
    cur ^= 1;
  }
  // residual and restriction
  {
    const T v = tail_apply<T>(M, tt, ix, iy, iz, sr, x);
    if (own) r[t] = b[t] - v;
  }
  __syncthreads();
  if (t < nc) {
    const int ox = t % Mc, oy = (t / Mc) % Mc, oz = t / (Mc * Mc);
    int xs[3], ys[3], zs[3];
    double wx[3], wy[3], wz[3];
#pragma unroll
    for (int q = 0; q < 3; ++q) {
      const int fx = 2 * ox + q - 1, fy = 2 * oy + q - 1, fz = 2 * oz + q - 1;
      const double w = q == 1 ? 1.0 : 0.5;
      wx[q] = (fx >= 0 && fx < M) ? w : 0.0;
      wy[q] = (fy >= 0 && fy < M) ? w : 0.0;
      wz[q] = (fz >= 0 && fz < M) ? w : 0.0;
      xs[q] = min(max(fx, 0), M - 1);
      ys[q] = min(max(fy, 0), M - 1);
      zs[q] = min(max(fz, 0), M - 1);
    }
    double s = 0.0;
#pragma unroll
    for (int qz = 0; qz < 3; ++qz) {
      double sz = 0.0;
#pragma unroll
      for (int q = 0; q < 9; ++q)
        sz += wy[q / 3] * wx[q % 3] * (double)r[xs[q % 3] + M * (ys[q / 3] + M * zs[qz])];
      s += wz[qz] * sz;
    }
    bc[t] = (T)s;
  }
  __syncthreads();
  // coarsest: xc[idx[row]] = sum_c G[row, c] bc[idx[c]]
  // eight lanes per row (row t / 8), lane t % 8 holding columns t % 8 + 8 c, all loads of a lane
  // issued together
  constexpr int GCH = 16;
  const bool gfast = a.nd <= TAIL_THREADS / 8 && a.nd <= 8 * GCH;
  const int grow = t >> 3, gpart = t & 7;
  const bool grow_ok = gfast && grow < a.nd;
  double gv[GCH];
#pragma unroll
  for (int c = 0; c < GCH; ++c) {
    const int col = gpart + 8 * c;
    gv[c] = (grow_ok && col < a.nd) ? a.G[(size_t)grow * a.nd + col] : 0.0;
  }
  const int grow_dst = grow_ok ? a.gidx[grow] : 0;
  const int gsel = (gfast && t < a.nd) ? a.gidx[t] : 0;
  if (gfast) {
    // gather the right-hand side in row order into r (free until the post-smoothing)
    if (t < a.nd) r[t] = bc[gsel];
    __syncthreads();
    double s = 0.0;
#pragma unroll
    for (int c = 0; c < GCH; ++c) {
      const int col = gpart + 8 * c;
      if (col < a.nd) s += gv[c] * (double)r[col];
    }
#pragma unroll
    for (int off = 4; off > 0; off >>= 1) s += __shfl_xor(s, off, 64);
    if (grow_ok && gpart == 0) xc[grow_dst] = (T)s;
  } else {
    const int lane = t & 63, wave = t >> 6;
    for (int row = wave; row < a.nd; row += TAIL_THREADS / 64) {
      double s = 0.0;
      for (int c = lane; c < a.nd; c += 64) s += a.G[(size_t)row * a.nd + c] * (double)bc[a.gidx[c]];
#pragma unroll
      for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
      if (lane == 0) xc[a.gidx[row]] = (T)s;
    }
  }
  __syncthreads();
  // prolongation x += P xc
  if (own) {
    const int fx = t % M, fy = (t / M) % M, fz = t / (M * M);
    const int x0 = fx >> 1, y0 = fy >> 1, z0 = fz >> 1;
    const int xs[2] = {x0, x0 + (fx & 1)}, ys[2] = {y0, y0 + (fy & 1)}, zs[2] = {z0, z0 + (fz & 1)};
    double v[8];
#pragma unroll
    for (int q = 0; q < 8; ++q) v[q] = (double)xc[xs[q & 1] + Mc * (ys[(q >> 1) & 1] + Mc * zs[q >> 2])];
    const double a0 = 0.5 * (v[0] + v[1]), a1 = 0.5 * (v[2] + v[3]);
    const double a2 = 0.5 * (v[4] + v[5]), a3 = 0.5 * (v[6] + v[7]);
    x[t] = x[t] + (T)(0.5 * (0.5 * (a0 + a1) + 0.5 * (a2 + a3)));
  }
  __syncthreads();
  // post-smoothing from x: the first correction is added to x by the next step
  cur = 0;
  {
    const T v = tail_apply<T>(M, tt, ix, iy, iz, sr, x);
    if (own) {
      const T ri = b[t] - v;
      r[t] = ri;
      dv[0][t] = a.inv_theta * dinv * ri;
    }
  }
  __syncthreads();
  bool pending = true;
  for (int it = 1; it < a.deg; ++it) {
    const T v = tail_apply<T>(M, tt, ix, iy, iz, sr, dv[cur]);
    if (own) {
      const T ri = r[t] - v;
      const T d0 = dv[cur][t];
      const T dn = a.alpha[it] * d0 + a.beta[it] * dinv * ri;
      r[t] = ri;
      dv[cur ^ 1][t] = dn;
      x[t] += pending ? d0 + dn : dn;
    }
    __syncthreads();
    cur ^= 1;
    pending = false;
  }
  if (own) xg[t] = pending ? x[t] + dv[cur][t] : x[t];
}

template <int NC, typename T, int EP>
void stencil_launch(hipStream_t st, int N, const T* S, const T* u, T* y, bool add, const Epi<T>& ep) {
  const int M = N + 1;
  const size_t tot = (size_t)NC * M * M * M;
  char key[96];
  snprintf(key, sizeof(key), "stencil nc=%d k=1 N=%d %s", NC, N, sizeof(T) == 8 ? "f64" : "f32");
  ProfScope ps(st, key);
  hipLaunchKernelGGL((k_stencil<NC, T, EP>), dim3(grid_for(tot, STENCIL_BLOCK)), dim3(STENCIL_BLOCK),
                     0, st, M, S, u, y, (int)add, ep);
}

template <int NC, typename T>
void stencil_dispatch(hipStream_t st, int N, const T* S, const T* u, T* y, bool add, const Epi<T>& ep) {
  switch (ep.mode) {
    case EPI_STORE: return stencil_launch<NC, T, EPI_STORE>(st, N, S, u, y, add, ep);
    case EPI_RESID: return stencil_launch<NC, T, EPI_RESID>(st, N, S, u, y, add, ep);
    case EPI_CHEB_FIRST: return stencil_launch<NC, T, EPI_CHEB_FIRST>(st, N, S, u, y, add, ep);
    case EPI_CHEB_STEP: return stencil_launch<NC, T, EPI_CHEB_STEP>(st, N, S, u, y, add, ep);
    case EPI_CHEB_ZERO: return stencil_launch<NC, T, EPI_CHEB_ZERO>(st, N, S, u, y, add, ep);
    default: throw Error{WB_EINVAL, "unknown epilogue"};
  }
}

// Inverse of the diagonal of the inverse viscosity-weighted pressure mass M_p(1/mu) (eq. 4):
// out[e n_p + m] = 1 / sum_q W_q |J| psi_m(x_q)^2 / mu_q, one thread per (element, mode).
template <int n>
__global__ void k_pmass_inv(const int E, const double hh, const double* __restrict__ mu_q,
                            double* __restrict__ out) {
  constexpr int NP = (n - 1) * n * (n + 1) / 6, N3 = n * n * n;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)E * NP) return;
  const int e = (int)(idx / NP), r = (int)(idx % NP);
  const int ma = CT<n>::t.ma[r], mb = CT<n>::t.mb[r], mc = CT<n>::t.mc[r];
  const double* mu = mu_q + (size_t)e * N3;
  double s = 0.0;
  for (int qz = 0; qz < n; ++qz)
    for (int qy = 0; qy < n; ++qy)
      for (int qx = 0; qx < n; ++qx) {
        const double psi = CT<n>::t.L[ma * n + qx] * CT<n>::t.L[mb * n + qy] * CT<n>::t.L[mc * n + qz];
        s += CT<n>::t.wg[qx] * CT<n>::t.wg[qy] * CT<n>::t.wg[qz] * psi * psi / mu[qx + n * (qy + n * qz)];
      }
  out[idx] = 1.0 / (hh * hh * hh * s);
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
                         const double* __restrict__ dinv_nodes, const int cstride,
                         double* __restrict__ dk) {
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
    for (int cc = 0; cc < 3; ++cc) {
      const double v = s2 * bhat[((size_t)m * 3 + cc) * N3 + li];
      s += v * v * dinv_nodes[(size_t)cc * cstride + g];
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

// Viscosity-gradient weights w = (mu^2 + |grad mu|^2)^(1/4), grad mu of the element's Q_k
// interpolant of mu_nodes.  Lumped mass: per element node, accumulated as in k_lumped.
template <int n>
__global__ void k_lumped_grad(int N, int M, int E, double h3, double s, double amp,
                              const double* __restrict__ mu_nodes, double* __restrict__ cn) {
  constexpr int NN = n * n, N3 = NN * n, k = n - 1;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)E * N3) return;
  const int e = (int)(idx / N3), li = (int)(idx % N3);
  const int a = li % n, b = (li / n) % n, c = li / NN;
  const int ex = e % N, ey = (e / N) % N, ez = e / (N * N);
  const bool touch = ex == 0 || ex == N - 1 || ey == 0 || ey == N - 1 || ez == 0 || ez == N - 1;
  auto mu = [&](int i, int j, int l) {
    return mu_nodes[(ex * k + i) + M * ((ey * k + j) + M * (ez * k + l))];
  };
  double gx = 0.0, gy = 0.0, gz = 0.0;
  for (int l = 0; l < n; ++l) {
    gx += CT<n>::t.DN[a * n + l] * mu(l, b, c);
    gy += CT<n>::t.DN[b * n + l] * mu(a, l, c);
    gz += CT<n>::t.DN[c * n + l] * mu(a, b, l);
  }
  const double m0 = mu(a, b, c);
  const double w = sqrt(sqrt(m0 * m0 + s * s * (gx * gx + gy * gy + gz * gz)));
  const int g = (ex * k + a) + M * ((ey * k + b) + M * (ez * k + c));
  atomic_add(&cn[g], (touch ? amp : 1.0) * w * CT<n>::t.wl[a] * CT<n>::t.wl[b] * CT<n>::t.wl[c] * h3);
}

// Poisson coefficient 1/(a_e w) at the Gauss points with the gradient weights.
template <int n>
__global__ void k_poisson_coef_grad(int N, int M, int E, double s, double amp,
                                    const double* __restrict__ mu_q, const double* __restrict__ mu_nodes,
                                    double* __restrict__ c) {
  constexpr int NN = n * n, N3 = NN * n, k = n - 1;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= (long long)E * N3) return;
  const int e = (int)(idx / N3), q = (int)(idx % N3);
  const int qx = q % n, qy = (q / n) % n, qz = q / NN;
  const int ex = e % N, ey = (e / N) % N, ez = e / (N * N);
  const bool touch = ex == 0 || ex == N - 1 || ey == 0 || ey == N - 1 || ez == 0 || ez == N - 1;
  double gx = 0.0, gy = 0.0, gz = 0.0;
  for (int l3 = 0; l3 < n; ++l3)
    for (int l2 = 0; l2 < n; ++l2)
      for (int l1 = 0; l1 < n; ++l1) {
        const double v = mu_nodes[(ex * k + l1) + M * ((ey * k + l2) + M * (ez * k + l3))];
        const double bx = CT<n>::t.B[qx * n + l1], by = CT<n>::t.B[qy * n + l2], bz = CT<n>::t.B[qz * n + l3];
        gx += CT<n>::t.D1[qx * n + l1] * by * bz * v;
        gy += bx * CT<n>::t.D1[qy * n + l2] * bz * v;
        gz += bx * by * CT<n>::t.D1[qz * n + l3] * v;
      }
  const double m0 = mu_q[idx];
  const double w = sqrt(sqrt(m0 * m0 + s * s * (gx * gx + gy * gy + gz * gz)));
  c[idx] = 1.0 / ((touch ? amp : 1.0) * w);
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

// The same transfer with at most WM entries per 1D row (the same 1D rows serve the three
// directions).  The block first copies the rows into LDS (padded entries repeat a valid column
// with weight 0), so that the per-output row lookups cost no memory instructions; every input
// load is unconditional, and each output sums x first, then weights by its y and z entries.
// Grid: (plane of Mo^2 outputs, groups of zb of the Mo NC z-planes); 32-bit index arithmetic;
// dynamic LDS of Mo WM (int + double).
template <typename T, int WM>
__global__ void __launch_bounds__(256)
k_kron_fixed(int Mo, int Mi, int NC, int W, const int* __restrict__ cnt, const int* __restrict__ col,
             const double* __restrict__ val, int dir, int add, int zb, const T* __restrict__ in,
             T* __restrict__ out) {
  extern __shared__ double kron_lds[];
  double* lv = kron_lds;                                // [Mo][WM] weights
  int* lc = reinterpret_cast<int*>(lv + Mo * WM);       // [Mo][WM] columns
  for (int q = threadIdx.x; q < Mo * WM; q += blockDim.x) {
    const int r = q / WM, t = q % WM, nr = cnt[r];
    const int tt = min(t, max(nr - 1, 0));
    lc[q] = col[r * W + tt];
    lv[q] = t < nr ? val[r * W + tt] : 0.0;
  }
  __syncthreads();
  const int pl = blockIdx.x * blockDim.x + threadIdx.x;
  if (pl >= Mo * Mo) return;
  const int oi = pl % Mo, oj = pl / Mo;
  const size_t ni = (size_t)Mi * Mi * Mi;
  const int z1 = min((int)(blockIdx.y + 1) * zb, Mo * NC);
  for (int zc = blockIdx.y * zb; zc < z1; ++zc) {
    const int c = zc / Mo, ol = zc % Mo;
    const size_t idx = ((size_t)zc * Mo) * Mo + pl;
    if (dir && (oi == 0 || oi == Mo - 1 || oj == 0 || oj == Mo - 1 || ol == 0 || ol == Mo - 1)) {
      if (!add) out[idx] = T(0);
      continue;
    }
    const T* inc = in + (size_t)c * ni;
    double s = 0.0;
#pragma unroll
    for (int tc = 0; tc < WM; ++tc)
#pragma unroll
      for (int tb = 0; tb < WM; ++tb) {
        const T* line = inc + ((size_t)lc[ol * WM + tc] * Mi + lc[oj * WM + tb]) * Mi;
        double sx = 0.0;
#pragma unroll
        for (int ta = 0; ta < WM; ++ta) sx += lv[oi * WM + ta] * (double)line[lc[oi * WM + ta]];
        s += (lv[ol * WM + tc] * lv[oj * WM + tb]) * sx;
      }
    out[idx] = add ? out[idx] + (T)s : (T)s;
  }
}

// Linear interpolation between nested node grids, M_fine = 2 M_coarse - 1, and its transpose.
// Prolongation: the fine node value is the mean of the coarse values at the 8 corners
// (x0|x1) x (y0|y1) x (z0|z1), x0 = fx / 2, x1 = x0 + (fx odd): 1 at shared nodes, 1/2 along a
// midpoint direction.  Restriction: weights (1/2, 1, 1/2) on the fine nodes 2c-1, 2c, 2c+1 of each
// direction (inside the grid).  Dirichlet outputs (dir) are zeroed when !add, left alone when add.
template <typename T, bool PROLONG>
__global__ void __launch_bounds__(256)
k_lin21(const int Mo, const int Mi, const int NC, const int dir, const int add,
        const T* __restrict__ in, T* __restrict__ out) {
  const long long no = (long long)Mo * Mo * Mo, ni = (long long)Mi * Mi * Mi;
  const long long idx = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (idx >= no * NC) return;
  const int c = (int)(idx / no);
  const long long o = idx % no;
  const int ox = (int)(o % Mo), oy = (int)((o / Mo) % Mo), oz = (int)(o / ((long long)Mo * Mo));
  if (dir && (ox == 0 || ox == Mo - 1 || oy == 0 || oy == Mo - 1 || oz == 0 || oz == Mo - 1)) {
    if (!add) out[idx] = T(0);
    return;
  }
  const T* inc = in + (size_t)c * ni;
  double s = 0.0;
  if constexpr (PROLONG) {
    const int x0 = ox >> 1, y0 = oy >> 1, z0 = oz >> 1;
    const int xs[2] = {x0, x0 + (ox & 1)}, ys[2] = {y0, y0 + (oy & 1)}, zs[2] = {z0, z0 + (oz & 1)};
    double v[8];
#pragma unroll
    for (int t = 0; t < 8; ++t)
      v[t] = (double)inc[xs[t & 1] + (size_t)Mi * (ys[(t >> 1) & 1] + (size_t)Mi * zs[t >> 2])];
    // pairwise means (exact where a pair is one node)
    const double a0 = 0.5 * (v[0] + v[1]), a1 = 0.5 * (v[2] + v[3]);
    const double a2 = 0.5 * (v[4] + v[5]), a3 = 0.5 * (v[6] + v[7]);
    s = 0.5 * (0.5 * (a0 + a1) + 0.5 * (a2 + a3));
  } else {
    int xs[3], ys[3], zs[3];
    double wx[3], wy[3], wz[3];
#pragma unroll
    for (int t = 0; t < 3; ++t) {
      const int fx = 2 * ox + t - 1, fy = 2 * oy + t - 1, fz = 2 * oz + t - 1;
      const double w = t == 1 ? 1.0 : 0.5;
      wx[t] = (fx >= 0 && fx < Mi) ? w : 0.0;
      wy[t] = (fy >= 0 && fy < Mi) ? w : 0.0;
      wz[t] = (fz >= 0 && fz < Mi) ? w : 0.0;
      xs[t] = min(max(fx, 0), Mi - 1);
      ys[t] = min(max(fy, 0), Mi - 1);
      zs[t] = min(max(fz, 0), Mi - 1);
    }
#pragma unroll
    for (int tz = 0; tz < 3; ++tz) {
      double v[9];
#pragma unroll
      for (int t = 0; t < 9; ++t)
        v[t] = (double)inc[xs[t % 3] + (size_t)Mi * (ys[t / 3] + (size_t)Mi * zs[tz])];
      double sz = 0.0;
#pragma unroll
      for (int t = 0; t < 9; ++t) sz += wy[t / 3] * wx[t % 3] * v[t];
      s += wz[tz] * sz;
    }
  }
  out[idx] = add ? out[idx] + (T)s : (T)s;
}

template <int n, typename T>
__global__ void __launch_bounds__(256)
k_modal_I(const int N, const int M, const int E, const T* __restrict__ u, T* __restrict__ p,
          const int add) {
  // one thread per element, consecutive threads on consecutive elements in x (each load
  // instruction covers a contiguous run of nodes); per node line (b, c) the x contraction
  // R[a'] = sum_a J[a'][a] u[a, b, c] first, then each mode takes J[mb][b] J[mc][c] R[ma]
  constexpr int k = n - 1, NP = (n - 1) * n * (n + 1) / 6;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  const int ex = e % N, ey = (e / N) % N, ez = e / (N * N);
  T acc[NP];
#pragma unroll
  for (int m = 0; m < NP; ++m) acc[m] = T(0);
#pragma unroll
  for (int c = 0; c < n; ++c)
#pragma unroll
    for (int b = 0; b < n; ++b) {
      const T* row = u + (size_t)ex * k + (size_t)M * ((size_t)(ey * k + b) + (size_t)M * (ez * k + c));
      T uv[n];
#pragma unroll
      for (int a = 0; a < n; ++a) uv[a] = row[a];
      T R[k];
#pragma unroll
      for (int ma = 0; ma < k; ++ma) {
        T r = T(0);
#pragma unroll
        for (int a = 0; a < n; ++a) r += (T)CT<n>::t.J[ma * n + a] * uv[a];
        R[ma] = r;
      }
#pragma unroll
      for (int m = 0; m < NP; ++m)
        acc[m] += (T)CT<n>::t.J[CT<n>::t.mb[m] * n + b] * (T)CT<n>::t.J[CT<n>::t.mc[m] * n + c] *
                  R[CT<n>::t.ma[m]];
    }
#pragma unroll
  for (int m = 0; m < NP; ++m) {
    const size_t j = (size_t)e * NP + m;
    p[j] = add ? p[j] + acc[m] : acc[m];
  }
}

// Transpose of the element-wise projection onto the Legendre modes, u = I^T p on the continuous
// Q_k nodes (no boundary mask), gathered node by node: thread (ex, gy, gz) writes the nodes
// gx = ex k .. ex k + k - 1 of the line (gy, gz) and the thread with ex = N - 1 also gx = M - 1.
// The modes of the elements around the line are contracted over y and z first (J weights of the
// y and z candidates), then each node takes a k-term sum per neighbouring x element.
template <int n, typename T>
__global__ void __launch_bounds__(256)
k_modal_IT(const int N, const int M, const T* __restrict__ p, T* __restrict__ u) {
  constexpr int k = n - 1, NP = (n - 1) * n * (n + 1) / 6;
  // each thread contracts the modes of its own x element over y and z; the left element's
  // contraction is the left neighbour thread's, read from LDS.  Blocks overlap by one: thread 0
  // only contracts the element left of the block's first output, threads 1..255 write outputs.
  __shared__ T qs[k][256];
  const int t = xcd_order(blockIdx.x, gridDim.x) * (blockDim.x - 1) + (int)threadIdx.x - 1;
  const bool valid = t >= 0 && t < N * M * M;
  const int tt = valid ? t : 0;
  const int ex = tt % N, gy = (tt / N) % M, gz = tt / (N * M);
  int yc[2], zc[2];
  T jy[2][k], jz[2][k];
  const int gc[2] = {gy, gz};
#pragma unroll
  for (int d = 0; d < 2; ++d) {
    const int r = gc[d] % k, q = gc[d] / k;
    const bool vert = r == 0;
    const bool v0 = !vert || q > 0, v1 = vert && q < N;
    const int i0 = vert ? k : r;
    const int e0 = vert ? (q > 0 ? q - 1 : 0) : q;
    (d ? zc : yc)[0] = e0;
    (d ? zc : yc)[1] = v1 ? q : e0;
#pragma unroll
    for (int a = 0; a < k; ++a) {
      T w0 = T(0);
#pragma unroll
      for (int ii = 1; ii <= k; ++ii) w0 = (i0 == ii) ? (T)CT<n>::t.J[a * n + ii] : w0;
      (d ? jz : jy)[0][a] = v0 ? w0 : T(0);
      (d ? jz : jy)[1][a] = v1 ? (T)CT<n>::t.J[a * n] : T(0);
    }
  }
  auto contract = [&](const int X, T (&Q)[k]) {
#pragma unroll
    for (int a = 0; a < k; ++a) Q[a] = T(0);
#pragma unroll
    for (int sz = 0; sz < 2; ++sz)
#pragma unroll
      for (int sy = 0; sy < 2; ++sy) {
        const T* pe = p + ((size_t)N * (yc[sy] + (size_t)N * zc[sz]) + X) * NP;
#pragma unroll
        for (int m = 0; m < NP; ++m)
          Q[CT<n>::t.ma[m]] += pe[m] * (jy[sy][CT<n>::t.mb[m]] * jz[sz][CT<n>::t.mc[m]]);
      }
  };
  T Q1[k], Q0[k];
  if (valid) {
    contract(ex, Q1);
  } else {
#pragma unroll
    for (int a = 0; a < k; ++a) Q1[a] = T(0);
  }
#pragma unroll
  for (int a = 0; a < k; ++a) qs[a][threadIdx.x] = Q1[a];
  __syncthreads();
  if (!valid || threadIdx.x == 0) return;
#pragma unroll
  for (int a = 0; a < k; ++a) Q0[a] = ex > 0 ? qs[a][threadIdx.x - 1] : T(0);
  const size_t base = (size_t)ex * k + (size_t)M * (gy + (size_t)M * gz);
#pragma unroll
  for (int i = 0; i < k; ++i) {
    T acc = T(0);
#pragma unroll
    for (int a = 0; a < k; ++a) {
      acc += Q1[a] * (T)CT<n>::t.J[a * n + i];
      if (i == 0) acc += Q0[a] * (T)CT<n>::t.J[a * n + k];
    }
    u[base + i] = acc;
  }
  if (ex == N - 1) {
    T acc = T(0);
#pragma unroll
    for (int a = 0; a < k; ++a) acc += Q1[a] * (T)CT<n>::t.J[a * n + k];
    u[base + k] = acc;
  }
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
__global__ void __launch_bounds__(256) k_dense(int nd, const double* __restrict__ G,
                                               const int* __restrict__ idx,
                                               const T* __restrict__ x, T* __restrict__ y) {
  // one wavefront per row: coalesced reads of the row, wavefront sum
  const int lane = threadIdx.x & 63, row = blockIdx.x * 4 + (threadIdx.x >> 6);
  if (row >= nd) return;  // whole wavefronts leave together
  double s = 0.0;
  for (int c = lane; c < nd; c += 64) s += G[(size_t)row * nd + c] * (double)x[idx[c]];
#pragma unroll
  for (int off = 32; off > 0; off >>= 1) s += __shfl_down(s, off, 64);
  if (lane == 0) y[idx[row]] = (T)s;
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

__global__ void __launch_bounds__(256) k_final_sum(int nb, const double* __restrict__ partial,
                                                   double* out) {
  double s = 0.0;
  for (int i = threadIdx.x; i < nb; i += blockDim.x) s += partial[i];
  s = block_sum(s);
  if (threadIdx.x == 0) *out = s;
}

// Second stage of a block reduction inside the same launch: each block publishes its partial
// (thread 0, value s), the block that completes the count sums all partials in block order
// into *out and re-arms the counter (partial[RED_BLOCKS], zero between launches).
__device__ inline void finish_by_last_block(double s, double* partial, double* out) {
  __shared__ int last;
  unsigned* count = reinterpret_cast<unsigned*>(partial + RED_BLOCKS);
  if (threadIdx.x == 0) {
    partial[blockIdx.x] = s;
    __threadfence();  // the partial is visible device-wide before the count says so
    last = atomicAdd(count, 1u) == gridDim.x - 1 ? 1 : 0;
  }
  __syncthreads();
  if (!last) return;
  __threadfence();  // and the partials of the other blocks are seen here
  double t = 0.0;
  for (int i = threadIdx.x; i < (int)gridDim.x; i += blockDim.x) t += partial[i];
  t = block_sum(t);
  if (threadIdx.x == 0) {
    *out = t;
    *count = 0u;
  }
}

template <typename T, bool LAST>
__global__ void __launch_bounds__(256) k_dot_partial(size_t n, const T* __restrict__ x,
                                                     const T* __restrict__ y, double* partial,
                                                     double* out) {
  double s = 0.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    s += (double)x[i] * (double)y[i];
  s = block_sum(s);
  if constexpr (LAST) {
    finish_by_last_block(s, partial, out);
  } else {
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
  }
}

template <typename T>
__global__ void __launch_bounds__(256) k_mode0_sum(int E, int np, const T* __restrict__ p,
                                                   double* partial, double* out) {
  double s = 0.0;
  for (int e = blockIdx.x * blockDim.x + threadIdx.x; e < E; e += gridDim.x * blockDim.x)
    s += (double)p[(size_t)e * np];
  finish_by_last_block(block_sum(s), partial, out);
}

template <typename T>
__global__ void k_mode0_sub(int E, int np, T* __restrict__ p, const double* __restrict__ sum) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e < E) p[(size_t)e * np] -= (T)(*sum / E);
}

// h[v] partials for a group of MDOT_VG basis vectors: block (bx, g) covers the rows
// bx*256 + t, stepping gridDim.x*256, for vectors g*MDOT_VG ...; every row of w is read once per
// group and MDOT_VG independent streams are in flight per thread.
constexpr int MDOT_VG = 8;
__global__ void __launch_bounds__(256) k_mdot_partial(size_t n, int nv, const double* __restrict__ V,
                                                      size_t ld, const double* __restrict__ w,
                                                      double* partial) {
  __shared__ double red[4][MDOT_VG];
  const int v0 = blockIdx.y * MDOT_VG;
  const int cnt = min(MDOT_VG, nv - v0);
  double acc[MDOT_VG];
#pragma unroll
  for (int j = 0; j < MDOT_VG; ++j) acc[j] = 0.0;
  const double* Vb = V + (size_t)v0 * ld;
  const size_t stride = (size_t)gridDim.x * 256;
  size_t i = (size_t)blockIdx.x * 256 + threadIdx.x;
  // two rows per pass: twice the loads in flight
  for (; i + stride < n; i += 2 * stride) {
    const double w0 = w[i], w1 = w[i + stride];
#pragma unroll
    for (int j = 0; j < MDOT_VG; ++j)
      if (j < cnt) acc[j] += Vb[(size_t)j * ld + i] * w0 + Vb[(size_t)j * ld + i + stride] * w1;
  }
  if (i < n) {
    const double wi = w[i];
#pragma unroll
    for (int j = 0; j < MDOT_VG; ++j)
      if (j < cnt) acc[j] += Vb[(size_t)j * ld + i] * wi;
  }
  const int lane = threadIdx.x & 63, wid = threadIdx.x >> 6;
#pragma unroll
  for (int j = 0; j < MDOT_VG; ++j) {
    double v = acc[j];
#pragma unroll
    for (int off = 32; off > 0; off >>= 1) v += __shfl_down(v, off, 64);
    if (lane == 0) red[wid][j] = v;
  }
  __syncthreads();
  if (threadIdx.x < cnt) {
    const int j = threadIdx.x;
    partial[(size_t)(v0 + j) * gridDim.x + blockIdx.x] = red[0][j] + red[1][j] + red[2][j] + red[3][j];
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

// The update of the first classical Gram-Schmidt sweep fused with the projections of the
// second: w -= V h, then partials of V[v] . w for the updated w, from one read of V.  Rows go in
// chunks of GS_ROWS staged in LDS ([nv][GS_ROWS + 1], padded against bank conflicts), the loads
// of the next chunk in registers while the current one is worked on: each row is summed over
// the vectors in four interleaved partial sums (wave q takes v = q mod 4), added in a fixed
// order; then TPV threads per vector accumulate V[v] . w over interleaved rows.
// partial[v * gridDim.x + block], as k_mdot_partial.
// PER: the vectors per wave the kernel is built for (nv <= 4 PER); loads are unconditional, with
// clamped indices, so that none waits behind a branch.
constexpr int GS_ROWS = 64, GS_MAX_NV = 120;
template <int PER>
__global__ void __launch_bounds__(256) k_gs_sub_dot(size_t n, int nv, const double* __restrict__ V,
                                                    size_t ld, const double* __restrict__ h,
                                                    double* __restrict__ w,
                                                    double* __restrict__ partial) {
  extern __shared__ double sh[];
  constexpr int LS = GS_ROWS + 1;
  double* vs = sh;                                  // [nv][LS]
  double* ws = vs + (size_t)nv * LS;                // [GS_ROWS] updated w of the chunk
  double* ps = ws + GS_ROWS;                        // [4][GS_ROWS] row partial sums
  double* hs = ps + 4 * GS_ROWS;                    // [nv]
  const int t = threadIdx.x, r = t % GS_ROWS, q = t / GS_ROWS;
  for (int v = t; v < nv; v += blockDim.x) hs[v] = h[v];
  // dot: TPV threads per vector (all 256 threads busy up to nv = 256 / TPV), thread dq of vector
  // dv taking the rows dq, dq + TPV, ...
  constexpr int TPV = PER <= 2 ? 32 : PER <= 4 ? 16 : PER <= 8 ? 8 : PER <= 16 ? 4 : 2;
  static_assert(TPV * 4 * PER <= 256 && GS_ROWS % TPV == 0, "dot threads");
  const int dv = t / TPV, dq = t % TPV;
  const bool dact = dv < nv;
  double acc = 0.0;
  double pre[PER];
  double wpre = 0.0;
  auto load = [&](size_t c0) {
    const size_t i = min(c0 + r, n - 1);
#pragma unroll
    for (int s = 0; s < PER; ++s) pre[s] = V[(size_t)min(q + 4 * s, nv - 1) * ld + i];
    wpre = w[i];
  };
  const size_t step = (size_t)gridDim.x * GS_ROWS;
  size_t c0 = (size_t)blockIdx.x * GS_ROWS;
  if (c0 < n) load(c0);
  for (; c0 < n; c0 += step) {
    __syncthreads();  // the previous chunk's LDS reads are done (and hs is written)
    const size_t i = c0 + r;
#pragma unroll
    for (int s = 0; s < PER; ++s) {
      const int v = q + 4 * s;
      if (v < nv) vs[v * LS + r] = i < n ? pre[s] : 0.0;
    }
    const double wcur = wpre;
    __syncthreads();
    if (c0 + step < n) load(c0 + step);
    double sum = 0.0;
    for (int v = q; v < nv; v += 4) sum += vs[v * LS + r] * hs[v];
    ps[q * GS_ROWS + r] = sum;
    __syncthreads();
    if (q == 0) {
      const double wn =
          wcur - (((ps[r] + ps[GS_ROWS + r]) + ps[2 * GS_ROWS + r]) + ps[3 * GS_ROWS + r]);
      if (i < n) w[i] = wn;
      ws[r] = i < n ? wn : 0.0;
    }
    __syncthreads();
    if (dact) {
      const double* row = vs + dv * LS + dq;
#pragma unroll
      for (int rr = 0; rr < GS_ROWS / TPV; ++rr) acc += row[rr * TPV] * ws[rr * TPV + dq];
    }
  }
  __syncthreads();
  if (dact) ps[t] = acc;
  __syncthreads();
  if (t < nv) {
    double sum = 0.0;
#pragma unroll
    for (int q = 0; q < TPV; ++q) sum += ps[t * TPV + q];
    partial[(size_t)t * gridDim.x + blockIdx.x] = sum;
  }
}

__global__ void k_gemv(size_t n, int nv, const double* __restrict__ V, size_t ld,
                       const double* __restrict__ h, double sign, double* __restrict__ w) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  double s = 0.0;
  for (int v = 0; v < nv; ++v) s += V[(size_t)v * ld + i] * h[v];
  w[i] += sign * s;
}

// Jacobi-CG steps with device scalars (eigenvalue estimate): alpha = rz / pq, r -= alpha q,
// z = dinv r; then beta = rz_new / rz, p = z + beta p.  Non-positive denominators give 0 (the
// host reads the scalars afterwards and stops the recurrence there).
// (grid-stride; with LAST the block partials of r . z are finished by the last block, else
// they are left in partial for k_final_sum)
template <bool LAST>
__global__ void __launch_bounds__(256)
k_cg_r(size_t n, const double* __restrict__ q, const double* __restrict__ dinv,
       double* __restrict__ r, double* __restrict__ z, const double* __restrict__ rz,
       const double* __restrict__ pq, double* partial, double* rz_new) {
  const double a = (*pq > 0.0 && *rz > 0.0) ? *rz / *pq : 0.0;
  double s = 0.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x) {
    const double ri = r[i] - a * q[i];
    const double zi = dinv[i] * ri;
    r[i] = ri;
    z[i] = zi;
    s += ri * zi;
  }
  s = block_sum(s);
  if constexpr (LAST) {
    finish_by_last_block(s, partial, rz_new);
  } else {
    if (threadIdx.x == 0) partial[blockIdx.x] = s;
  }
}
// y = x / sqrt(*d) (zero when *d <= 0): a normalization whose norm is still on the device.
__global__ void k_scal_rnorm(size_t n, const double* __restrict__ d, const double* __restrict__ x,
                             double* __restrict__ y) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double s = *d > 0.0 ? 1.0 / sqrt(*d) : 0.0;
  y[i] = s * x[i];
}
__global__ void k_cg_p(size_t n, const double* __restrict__ z, double* __restrict__ p,
                       const double* __restrict__ rz_new, const double* __restrict__ rz_old) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  const double b = *rz_old > 0.0 ? *rz_new / *rz_old : 0.0;
  p[i] = z[i] + b * p[i];
}
// Counter-based splitmix64 uniform in [-1, 1): x_i = 2 U(mix(seed * 2^32 + i)) - 1; with
// M > 0 the entries on boundary nodes of an [NC][M^3] nodal vector are zeroed.
__global__ void k_splitmix_vec(size_t n, unsigned long long seed, int M, double* __restrict__ x) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n) return;
  unsigned long long z = (seed << 32) + (unsigned long long)i + 0x9E3779B97F4A7C15ULL;
  z = (z ^ (z >> 30)) * 0xBF58476D1CE4E5B9ULL;
  z = (z ^ (z >> 27)) * 0x94D049BB133111EBULL;
  z = z ^ (z >> 31);
  double v = 2.0 * ((double)(z >> 11) * (1.0 / 9007199254740992.0)) - 1.0;
  if (M > 0) {
    const size_t nn = (size_t)M * M * M, g = i % nn;
    const int gi = (int)(g % M), gj = (int)((g / M) % M), gl = (int)(g / ((size_t)M * M));
    if (gi == 0 || gi == M - 1 || gj == 0 || gj == M - 1 || gl == 0 || gl == M - 1) v = 0.0;
  }
  x[i] = v;
}
__global__ void __launch_bounds__(256) k_sum_partial(size_t n, const double* __restrict__ x,
                                                     double* partial) {
  double s = 0.0;
  for (size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x; i < n; i += (size_t)gridDim.x * blockDim.x)
    s += x[i];
  s = block_sum(s);
  if (threadIdx.x == 0) partial[blockIdx.x] = s;
}
__global__ void k_sub_mean(size_t n, double* __restrict__ x, const double* __restrict__ sum) {
  const size_t i = (size_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) x[i] -= *sum / (double)n;
}

}  // namespace

// ================================================================== launchers
int set_matrix_core_ops(int on) { return matrix_core_ops.exchange(on ? 1 : 0); }

double set_two_pass_limit(double mb) {
  const double prev = (double)two_pass_limit.load() / 1e6;
  const double b = std::min(std::max(mb, 0.0) * 1e6, (double)TWO_PASS_MAX_BYTES);
  two_pass_limit.store((size_t)b);
  return prev;
}

size_t op_workspace_bytes_capped(int NC, int N, int k, size_t elem_size, size_t cap) {
  int BX = 8, BY = 8;
  switch (k + 1) {
    case 2: BX = Tile<2>::BX; BY = Tile<2>::BY; break;
    case 3: BX = Tile<3>::BX; BY = Tile<3>::BY; break;
    case 4: BX = Tile<4>::BX; BY = Tile<4>::BY; break;
    case 5: BX = Tile<5>::BX; BY = Tile<5>::BY; break;
    case 6: BX = Tile<6>::BX; BY = Tile<6>::BY; break;
    default: break;
  }
  const size_t b = elem_buf_bytes(NC, N, k);
  if (b <= two_pass_limit.load(std::memory_order_relaxed) && b <= cap)
    return b / sizeof(double) * elem_size;
  const BrickGeom G = brick_geom(N, k, BX, BY);
  return elem_size * NC * std::max<size_t>(G.per_comp, 1);
}

WorkspaceCap::WorkspaceCap(size_t bytes) : prev(two_pass_cap) { two_pass_cap = bytes; }
WorkspaceCap::~WorkspaceCap() { two_pass_cap = prev; }

size_t op_workspace_bytes(int NC, int N, int k, size_t elem_size) {
  const size_t elem_buf = elem_buf_bytes(NC, N, k) <= TWO_PASS_MAX_BYTES
                              ? elem_buf_bytes(NC, N, k) / sizeof(double) * elem_size
                              : 0;
  int BX = 8, BY = 8;
  switch (k + 1) {
    case 2: BX = Tile<2>::BX; BY = Tile<2>::BY; break;
    case 3: BX = Tile<3>::BX; BY = Tile<3>::BY; break;
    case 4: BX = Tile<4>::BX; BY = Tile<4>::BY; break;
    case 5: BX = Tile<5>::BX; BY = Tile<5>::BY; break;
    case 6: BX = Tile<6>::BX; BY = Tile<6>::BY; break;
    default: break;
  }
  const BrickGeom G = brick_geom(N, k, BX, BY);
  return std::max(elem_buf, elem_size * NC * std::max<size_t>(G.per_comp, 1));
}

template <typename T>
void launch_op_epi(hipStream_t st, int flags, int NC, int N, int k, const T* u, T* y, const T* coef,
                   const T* pin, T* pout, const T* sin, bool add, void* work, const Epi<T>& ep) {
  switch (k + 1) {
    case 2: return op_dispatch_n<2, T>(st, flags, NC, N, k, u, y, coef, pin, pout, sin, add, work, ep);
    case 3: return op_dispatch_n<3, T>(st, flags, NC, N, k, u, y, coef, pin, pout, sin, add, work, ep);
    case 4: return op_dispatch_n<4, T>(st, flags, NC, N, k, u, y, coef, pin, pout, sin, add, work, ep);
    case 5: return op_dispatch_n<5, T>(st, flags, NC, N, k, u, y, coef, pin, pout, sin, add, work, ep);
    case 6: return op_dispatch_n<6, T>(st, flags, NC, N, k, u, y, coef, pin, pout, sin, add, work, ep);
    default: throw Error{WB_EUNSUPPORTED, "order not built"};
  }
}
template void launch_op_epi<double>(hipStream_t, int, int, int, int, const double*, double*,
                                    const double*, const double*, double*, const double*, bool, void*,
                                    const Epi<double>&);
template void launch_op_epi<float>(hipStream_t, int, int, int, int, const float*, float*,
                                   const float*, const float*, float*, const float*, bool, void*,
                                   const Epi<float>&);

template <typename T>
void launch_op(hipStream_t st, int flags, int NC, int N, int k, const T* u, T* y, const T* coef,
               const T* pin, T* pout, const T* sin, bool add, void* work) {
  launch_op_epi<T>(st, flags, NC, N, k, u, y, coef, pin, pout, sin, add, work, Epi<T>{});
}
template void launch_op<double>(hipStream_t, int, int, int, int, const double*, double*,
                                const double*, const double*, double*, const double*, bool, void*);
template void launch_op<float>(hipStream_t, int, int, int, int, const float*, float*, const float*,
                               const float*, float*, const float*, bool, void*);

size_t q1_elem_matrix_len(int NC, int N) { return (size_t)N * N * N * 64 * NC * NC; }
size_t q1_stencil_len(int NC, int N) { return (size_t)27 * NC * NC * (N + 1) * (N + 1) * (N + 1); }

void assemble_q1(hipStream_t st, int NC, int N, bool dir, const double* coef, double* ae, double* S) {
  WB_REQUIRE(NC == 1 || NC == 3, WB_EINVAL, "assemble_q1: NC must be 1 or 3");
  const double hh = 0.5 / N;
  const int E = N * N * N, M = N + 1;
  const unsigned eg = grid_for(E, 4 * WaveMap<2>::EPW);
  const unsigned sg = grid_for((size_t)27 * M * M * M, 256);
  if (NC == 1) {
    WB_REQUIRE(!dir, WB_EUNSUPPORTED, "assemble_q1: scalar levels are Neumann");
    hipLaunchKernelGGL((k_elem_matrix<1, false>), dim3(eg), dim3(256), 0, st, N, hh, coef, ae);
    hipLaunchKernelGGL((k_stencil_gather<1, false>), dim3(sg), dim3(256), 0, st, N, ae, S);
  } else {
    WB_REQUIRE(dir, WB_EUNSUPPORTED, "assemble_q1: vector levels are Dirichlet");
    hipLaunchKernelGGL((k_elem_matrix<3, true>), dim3(eg), dim3(256), 0, st, N, hh, coef, ae);
    hipLaunchKernelGGL((k_stencil_gather<3, true>), dim3(sg), dim3(256), 0, st, N, ae, S);
  }
  WB_HIP(hipGetLastError());
}

template <typename T>
void launch_stencil_epi(hipStream_t st, int NC, int N, const T* S, const T* u, T* y, bool add,
                        const Epi<T>& ep) {
  if (NC == 1) return stencil_dispatch<1, T>(st, N, S, u, y, add, ep);
  if (NC == 3) return stencil_dispatch<3, T>(st, N, S, u, y, add, ep);
  throw Error{WB_EINVAL, "launch_stencil_epi: NC must be 1 or 3"};
}
template void launch_stencil_epi<double>(hipStream_t, int, int, const double*, const double*,
                                         double*, bool, const Epi<double>&);
template void launch_stencil_epi<float>(hipStream_t, int, int, const float*, const float*, float*,
                                        bool, const Epi<float>&);

template <typename T>
void launch_vcycle_tail(hipStream_t st, const TailArgs<T>& a, const T* b, T* x) {
  WB_REQUIRE(a.M >= 2 && a.M * a.M * a.M <= TAIL_MAX && 2 * a.Mc - 1 == a.M, WB_EINVAL,
             "vcycle tail: level sizes out of range");
  WB_REQUIRE(a.nd == a.Mc * a.Mc * a.Mc, WB_EINVAL, "vcycle tail: coarsest must be dense over all nodes");
  WB_REQUIRE(a.deg >= 1 && a.deg <= TAIL_MAXDEG, WB_EINVAL, "vcycle tail: Chebyshev degree out of range");
  char key[64];
  snprintf(key, sizeof(key), "vcycle tail M=%d %s", a.M, sizeof(T) == 8 ? "f64" : "f32");
  ProfScope ps(st, key);
  hipLaunchKernelGGL((k_vcycle_tail<T>), dim3(1), dim3(TAIL_THREADS), 0, st, a, b, x);
}
template void launch_vcycle_tail<double>(hipStream_t, const TailArgs<double>&, const double*, double*);
template void launch_vcycle_tail<float>(hipStream_t, const TailArgs<float>&, const float*, float*);

#define WB_BY_ORDER(k, ...)                                       \
  switch ((k) + 1) {                                              \
    case 2: { constexpr int n = 2; __VA_ARGS__; } break;          \
    case 3: { constexpr int n = 3; __VA_ARGS__; } break;          \
    case 4: { constexpr int n = 4; __VA_ARGS__; } break;          \
    case 5: { constexpr int n = 5; __VA_ARGS__; } break;          \
    case 6: { constexpr int n = 6; __VA_ARGS__; } break;          \
    default: throw Error{WB_EUNSUPPORTED, "order not built"};     \
  }

void launch_lumped_mass_grad(hipStream_t st, int N, int k, double amp, const double* mu_nodes,
                             double* cnodes) {
  const int M = k * N + 1, E = N * N * N, n3 = (k + 1) * (k + 1) * (k + 1);
  const double h = 1.0 / N, h3 = 0.125 * h * h * h, s = 2.0 / h;
  WB_BY_ORDER(k, {
    hipLaunchKernelGGL((k_lumped_grad<n>), dim3(grid_for((size_t)E * n3, 256)), dim3(256), 0, st, N,
                       M, E, h3, s, amp, mu_nodes, cnodes);
  });
}

void launch_poisson_coef_grad(hipStream_t st, int N, int k, double amp, const double* mu_q,
                              const double* mu_nodes, double* c_q) {
  const int M = k * N + 1, E = N * N * N, n3 = (k + 1) * (k + 1) * (k + 1);
  const double s = 2.0 * N;
  WB_BY_ORDER(k, {
    hipLaunchKernelGGL((k_poisson_coef_grad<n>), dim3(grid_for((size_t)E * n3, 256)), dim3(256), 0,
                       st, N, M, E, s, amp, mu_q, mu_nodes, c_q);
  });
}

void launch_pmass_inv(hipStream_t st, int N, int k, const double* mu_q, double* out) {
  const int E = N * N * N, np = tables(k).np;
  const double hh = 0.5 / N;
  WB_BY_ORDER(k, {
    hipLaunchKernelGGL((k_pmass_inv<n>), dim3(grid_for((size_t)E * np, 256)), dim3(256), 0, st, E,
                       hh, mu_q, out);
  });
  WB_HIP(hipGetLastError());
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
                   double* dk, bool per_component) {
  const int M = k * N + 1, E = N * N * N, np = tables(k).np;
  const double hh = 0.5 / N;
  const int cstride = per_component ? M * M * M : 0;
  WB_BY_ORDER(k, {
    hipLaunchKernelGGL((k_diag_K<n>), dim3(grid_for((size_t)E * np, 256)), dim3(256), 0, st, N, k,
                       M, E, np, hh * hh, bhat, dinv_nodes, cstride, dk);
  });
}

// diag(A)-BFBT Poisson coefficient: per element the mean over its nodes of m_i / w_i with
// w_i = (diag_0 + diag_1 + diag_2)(i) / 3 the component mean of the unmasked diag(A) and m_i the
// unweighted lumped mass (so 1/w_eff, w_eff = diag(A) / m), divided by a_e; constant on the element.
template <int n>
__global__ void k_diag_a_coef(int N, int M, int E, double amp, const double* __restrict__ diag3,
                              const double* __restrict__ mass, double* __restrict__ c) {
  constexpr int N3 = n * n * n, k = n - 1;
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  if (e >= E) return;
  const int ex = e % N, ey = (e / N) % N, ez = e / (N * N);
  const bool touch = ex == 0 || ex == N - 1 || ey == 0 || ey == N - 1 || ez == 0 || ez == N - 1;
  const size_t nn = (size_t)M * M * M;
  double s = 0.0;
  for (int li = 0; li < N3; ++li) {
    const int a = li % n, b = (li / n) % n, cc = li / (n * n);
    const size_t g = (size_t)(ex * k + a) + M * ((size_t)(ey * k + b) + M * (size_t)(ez * k + cc));
    s += 3.0 * mass[g] / (diag3[g] + diag3[nn + g] + diag3[2 * nn + g]);
  }
  const double ce = s / N3 / (touch ? amp : 1.0);
  for (int q = 0; q < N3; ++q) c[(size_t)e * N3 + q] = ce;
}

void launch_diag_a_coef(hipStream_t st, int N, int k, double amp, const double* diag3,
                        const double* mass, double* c_q) {
  const int M = k * N + 1, E = N * N * N;
  WB_BY_ORDER(k, {
    hipLaunchKernelGGL((k_diag_a_coef<n>), dim3(grid_for((size_t)E, 256)), dim3(256), 0, st, N, M, E,
                       amp, diag3, mass, c_q);
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
  if (R.lin21) {
    if (R.rows > R.cols)
      hipLaunchKernelGGL((k_lin21<T, true>), dim3(grid_for(tot, 256)), dim3(256), 0, st, R.rows,
                         R.cols, NC, (int)dir, (int)add, in, out);
    else
      hipLaunchKernelGGL((k_lin21<T, false>), dim3(grid_for(tot, 256)), dim3(256), 0, st, R.rows,
                         R.cols, NC, (int)dir, (int)add, in, out);
    return;
  }
  // z-planes per block: up to 8 (fewer table copies), while the grid keeps >= 4096 blocks
  const size_t pb = grid_for((size_t)R.rows * R.rows, 256), planes = (size_t)R.rows * NC;
  const int zb = (int)std::max<size_t>(1, std::min<size_t>(8, pb * planes / 4096));
  const dim3 g(pb, grid_for(planes, zb)), b(256);
  const int wm = R.W <= 2 ? 2 : R.W <= 3 ? 3 : R.W <= 4 ? 4 : R.W <= 7 ? 7 : 0;
  const size_t lds = (size_t)R.rows * wm * (sizeof(double) + sizeof(int));
  if (wm == 0 || lds > 48u * 1024u) {
    hipLaunchKernelGGL((k_kron<T>), dim3(grid_for(tot, 256)), b, 0, st, R.rows, R.cols, NC, R.W,
                       R.cnt, R.col, R.val, (int)dir, (int)add, in, out);
    return;
  }
#define WB_KRON(WMV)                                                                               \
  hipLaunchKernelGGL((k_kron_fixed<T, WMV>), g, b, lds, st, R.rows, R.cols, NC, R.W, R.cnt, R.col, \
                     R.val, (int)dir, (int)add, zb, in, out)
  if (wm == 2) WB_KRON(2);
  else if (wm == 3) WB_KRON(3);
  else if (wm == 4) WB_KRON(4);
  else WB_KRON(7);
#undef WB_KRON
}
template void launch_kron<double>(hipStream_t, const Rows1D&, int, bool, bool, const double*, double*);
template void launch_kron<float>(hipStream_t, const Rows1D&, int, bool, bool, const float*, float*);

template <typename T>
void launch_modal_I(hipStream_t st, int N, int k, const T* u, T* p, bool add) {
  const int M = k * N + 1, E = N * N * N;
  WB_BY_ORDER(k, {
    hipLaunchKernelGGL((k_modal_I<n, T>), dim3(grid_for((size_t)E, 256)), dim3(256), 0, st, N, M, E,
                       u, p, (int)add);
  });
}
template <typename T>
void launch_modal_IT(hipStream_t st, int N, int k, const T* p, T* u) {
  const int M = k * N + 1;
  WB_BY_ORDER(k, {
    hipLaunchKernelGGL((k_modal_IT<n, T>), dim3(grid_for((size_t)N * M * M, 255)), dim3(256), 0, st,
                       N, M, p, u);
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
  hipLaunchKernelGGL((k_dense<T>), dim3(grid_for(nd, 4)), dim3(256), 0, st, nd, G, idx, x, y);
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
  // short vectors: one launch finished by the last block; long ones: the full-bandwidth partial
  // pass, then one block (a device-wide fence in each of many blocks measured slower)
  int nb = (int)std::min<size_t>(RED_BLOCKS, grid_for(n, 256));
  if (nb < 1) nb = 1;
  if (nb <= RED_LAST_BLOCKS) {
    hipLaunchKernelGGL((k_dot_partial<T, true>), dim3(nb), dim3(256), 0, st, n, x, y, partial, out);
    return;
  }
  hipLaunchKernelGGL((k_dot_partial<T, false>), dim3(nb), dim3(256), 0, st, n, x, y, partial, out);
  hipLaunchKernelGGL(k_final_sum, dim3(1), dim3(256), 0, st, nb, partial, out);
}
template <typename T>
void launch_remove_mean(hipStream_t st, int E, int np, T* p, double* partial, double* scratch) {
  // one launch for the sum: few blocks, since each block's completion carries a device-wide fence
  int nb = (int)std::min<size_t>(RED_LAST_BLOCKS, grid_for(E, 256));
  if (nb < 1) nb = 1;
  hipLaunchKernelGGL((k_mode0_sum<T>), dim3(nb), dim3(256), 0, st, E, np, p, partial, scratch);
  hipLaunchKernelGGL((k_mode0_sub<T>), dim3(grid_for(E, 256)), dim3(256), 0, st, E, np, p, scratch);
}

#define WB_INST_VEC(T)                                                                            \
  template void launch_fill<T>(hipStream_t, T*, T, size_t);                                       \
  template void launch_axpby<T>(hipStream_t, size_t, T, const T*, T, T*);                         \
  template void launch_scale_nodes<T>(hipStream_t, int, int, const T*, const T*, T*);             \
  template void launch_cheb_first<T>(hipStream_t, size_t, const T*, const T*, const T*, T, T*, T*, \
                                     T*, bool);                                                    \
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
  // up to MDOT_BLOCKS row blocks, at least about 4 rows per thread
  const int nb = (int)std::min<size_t>(MDOT_BLOCKS, std::max<size_t>(1, grid_for(n, 1024)));
  const int ng = (nv + MDOT_VG - 1) / MDOT_VG;
  hipLaunchKernelGGL(k_mdot_partial, dim3(nb, ng), dim3(256), 0, st, n, nv, V, ld, w, partial);
  hipLaunchKernelGGL(k_rows_sum, dim3(nv), dim3(256), 0, st, nb, partial, h);
}
bool launch_gs_sub_dot(hipStream_t st, size_t n, int nv, const double* V, size_t ld,
                       const double* h, double* w, double* partial, double* h2) {
  if (nv > GS_MAX_NV || nv < 1 || n < 1) return false;
  const size_t lds = sizeof(double) * ((size_t)nv * (GS_ROWS + 1) + 5 * GS_ROWS + nv);
  // as many blocks as are resident at once (the LDS bounds them), at most MDOT_BLOCKS
  int dev = 0, cus = 0, per_cu = 0;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || cus < 1)
    return false;
  // the smallest build with 4 PER >= nv (padded loads repeat the last vector)
  using K = void (*)(size_t, int, const double*, size_t, const double*, double*, double*);
  static const K tiers[] = {k_gs_sub_dot<2>,  k_gs_sub_dot<4>,  k_gs_sub_dot<6>,  k_gs_sub_dot<8>,
                            k_gs_sub_dot<10>, k_gs_sub_dot<12>, k_gs_sub_dot<14>, k_gs_sub_dot<16>,
                            k_gs_sub_dot<20>, k_gs_sub_dot<24>, k_gs_sub_dot<30>};
  static const int per[] = {2, 4, 6, 8, 10, 12, 14, 16, 20, 24, 30};
  int ti = 0;
  while (4 * per[ti] < nv) ++ti;
  const K kern = tiers[ti];
  if (hipOccupancyMaxActiveBlocksPerMultiprocessor(&per_cu, kern, 256, lds) != hipSuccess ||
      per_cu < 1)
    return false;
  const int nb = (int)std::min<size_t>({(size_t)MDOT_BLOCKS, (size_t)cus * per_cu,
                                        std::max<size_t>(1, grid_for(n, GS_ROWS))});
  hipLaunchKernelGGL(kern, dim3(nb), dim3(256), lds, st, n, nv, V, ld, h, w, partial);
  hipLaunchKernelGGL(k_rows_sum, dim3(nv), dim3(256), 0, st, nb, partial, h2);
  return true;
}
void launch_gemv_sub(hipStream_t st, size_t n, int nv, const double* V, size_t ld, const double* h,
                     double* w) {
  hipLaunchKernelGGL(k_gemv, dim3(grid_for(n, 256)), dim3(256), 0, st, n, nv, V, ld, h, -1.0, w);
}
void launch_gemv_add(hipStream_t st, size_t n, int nv, const double* Z, size_t ld, const double* y,
                     double* x) {
  hipLaunchKernelGGL(k_gemv, dim3(grid_for(n, 256)), dim3(256), 0, st, n, nv, Z, ld, y, 1.0, x);
}

void launch_cg_r(hipStream_t st, size_t n, const double* q, const double* dinv, double* r, double* z,
                 const double* rz, const double* pq, double* partial, double* rz_new) {
  const int nb = (int)std::max<size_t>(1, std::min<size_t>(RED_BLOCKS, grid_for(n, 256)));
  if (nb <= RED_LAST_BLOCKS) {
    hipLaunchKernelGGL((k_cg_r<true>), dim3(nb), dim3(256), 0, st, n, q, dinv, r, z, rz, pq, partial,
                       rz_new);
  } else {
    hipLaunchKernelGGL((k_cg_r<false>), dim3(nb), dim3(256), 0, st, n, q, dinv, r, z, rz, pq,
                       partial, rz_new);
    hipLaunchKernelGGL(k_final_sum, dim3(1), dim3(256), 0, st, nb, partial, rz_new);
  }
}
void launch_cg_p(hipStream_t st, size_t n, const double* z, double* p, const double* rz_new,
                 const double* rz_old) {
  hipLaunchKernelGGL(k_cg_p, dim3(grid_for(n, 256)), dim3(256), 0, st, n, z, p, rz_new, rz_old);
}
void launch_scal_rnorm(hipStream_t st, size_t n, const double* d, const double* x, double* y) {
  hipLaunchKernelGGL(k_scal_rnorm, dim3(grid_for(n, 256)), dim3(256), 0, st, n, d, x, y);
}

void launch_splitmix_vec(hipStream_t st, size_t n, unsigned long long seed, int M, double* x) {
  hipLaunchKernelGGL(k_splitmix_vec, dim3(grid_for(n, 256)), dim3(256), 0, st, n, seed, M, x);
}
void launch_remove_global_mean(hipStream_t st, size_t n, double* x, double* partial, double* scratch) {
  const int nb = (int)std::min<size_t>(RED_BLOCKS, grid_for(n, 256));
  hipLaunchKernelGGL(k_sum_partial, dim3(nb), dim3(256), 0, st, n, x, partial);
  hipLaunchKernelGGL(k_final_sum, dim3(1), dim3(256), 0, st, nb, partial, scratch);
  hipLaunchKernelGGL(k_sub_mean, dim3(grid_for(n, 256)), dim3(256), 0, st, n, x, scratch);
}

}  // namespace wb
