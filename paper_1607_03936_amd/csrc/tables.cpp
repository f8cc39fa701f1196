// Host-side 1D quadrature rules and polynomial tables for the Q_k x P_{k-1}
// discretization: Gauss-Legendre quadrature, Gauss-Lobatto-Legendre nodes,
// Lagrange and Legendre bases (Sec. 1.2 discretization; node set and
// quadrature rule as documented in the header of wbfbt.h).
#include <cmath>
#include <cstring>
#include <mutex>

#include "wb_internal.h"

namespace wb {

namespace {
// P_N(x) and P_N'(x) by the three-term recurrence.
void legendre_pd(int N, double x, double* p, double* dp) {
  double p0 = 1.0, p1 = x;
  if (N == 0) {
    *p = 1.0;
    *dp = 0.0;
    return;
  }
  for (int j = 2; j <= N; ++j) {
    double p2 = ((2.0 * j - 1.0) * x * p1 - (j - 1.0) * p0) / j;
    p0 = p1;
    p1 = p2;
  }
  *p = p1;
  // derivative from (x^2 - 1) P_N' = N (x P_N - P_{N-1})
  if (std::fabs(std::fabs(x) - 1.0) < 1e-15)
    *dp = (x > 0 ? 1.0 : (N % 2 ? 1.0 : -1.0)) * 0.5 * N * (N + 1.0);
  else
    *dp = N * (x * p1 - p0) / (x * x - 1.0);
}
}  // namespace

double legendre(int a, double x) {
  double p, dp;
  legendre_pd(a, x, &p, &dp);
  return p;
}

void gauss_rule(int n, double* x, double* w) {
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < n; ++i) {
    double z = std::cos(pi * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p, dp;
      legendre_pd(n, z, &p, &dp);
      double dz = p / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    double p, dp;
    legendre_pd(n, z, &p, &dp);
    x[n - 1 - i] = z;  // ascending order
    w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

void gll_rule(int n, double* x, double* w) {
  const double pi = 3.14159265358979323846;
  const int N = n - 1;
  x[0] = -1.0;
  x[N] = 1.0;
  for (int i = 1; i < N; ++i) {
    // interior nodes: roots of P_N'; Newton on P_N' with P_N'' from Legendre's equation
    double z = -std::cos(pi * i / N);
    for (int it = 0; it < 100; ++it) {
      double p, dp;
      legendre_pd(N, z, &p, &dp);
      double d2p = (2.0 * z * dp - N * (N + 1.0) * p) / (1.0 - z * z);
      double dz = dp / d2p;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = z;
  }
  for (int i = 0; i < n; ++i) {
    double p, dp;
    legendre_pd(N, x[i], &p, &dp);
    w[i] = 2.0 / (N * (N + 1.0) * p * p);
  }
}

void lagrange(int n, const double* nodes, int m, const double* x, double* V, double* D) {
  for (int i = 0; i < m; ++i) {
    for (int a = 0; a < n; ++a) {
      double v = 1.0, d = 0.0;
      for (int j = 0; j < n; ++j) {
        if (j == a) continue;
        v *= (x[i] - nodes[j]) / (nodes[a] - nodes[j]);
      }
      for (int j = 0; j < n; ++j) {
        if (j == a) continue;
        double t = 1.0 / (nodes[a] - nodes[j]);
        for (int l = 0; l < n; ++l) {
          if (l == a || l == j) continue;
          t *= (x[i] - nodes[l]) / (nodes[a] - nodes[l]);
        }
        d += t;
      }
      if (V) V[i * n + a] = v;
      if (D) D[i * n + a] = d;
    }
  }
}

int modes(int k, int* ma, int* mb, int* mc) {
  int m = 0;
  for (int c = 0; c < k; ++c)
    for (int b = 0; b < k - c; ++b)
      for (int a = 0; a < k - b - c; ++a) {
        if (ma) {
          ma[m] = a;
          mb[m] = b;
          mc[m] = c;
        }
        ++m;
      }
  return m;
}

static Tables build_tables(int k) {
  Tables t;
  std::memset(&t, 0, sizeof(t));
  const int n = k + 1;
  t.n = n;
  t.k = k;
  gauss_rule(n, t.xg, t.wg);
  gll_rule(n, t.xl, t.wl);
  lagrange(n, t.xl, n, t.xg, t.B, t.D1);
  double Vg[NMAX * NMAX];
  lagrange(n, t.xg, n, t.xg, Vg, t.Dh);
  for (int a = 0; a < n; ++a)
    for (int q = 0; q < n; ++q) t.L[a * n + q] = legendre(a, t.xg[q]);
  for (int a = 0; a < n; ++a)
    for (int i = 0; i < n; ++i) {
      double s = 0.0;
      for (int q = 0; q < n; ++q) s += t.wg[q] * t.L[a * n + q] * t.B[q * n + i];
      t.J[a * n + i] = s * (2.0 * a + 1.0) / 2.0;
    }
  t.np = modes(k, t.ma, t.mb, t.mc);
  return t;
}

const Tables& tables(int k) {
  static Tables tab[NMAX + 1];
  static std::once_flag once;
  std::call_once(once, [] {
    for (int kk = 1; kk <= NMAX - 1; ++kk) tab[kk] = build_tables(kk);
  });
  return tab[k];
}

}  // namespace wb
