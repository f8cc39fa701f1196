// 1D quadrature rules and polynomial tables of the Q_k x P_{k-1} discretization (Sec. 1.2):
// Gauss-Legendre quadrature, Gauss-Lobatto-Legendre nodes, Lagrange and Legendre bases.
// Everything here is constexpr, so the element kernels see the tables of their order as
// compile-time constants and the host reads the very same numbers.
#pragma once

namespace wb {

constexpr int NMAX = 6;   // n = k+1 <= 6
constexpr int NPMAX = 35; // modes for k = 5

// All 1D tables of one order k (n = k+1), double precision.
struct Tables {
  int n, k, np;
  double xg[NMAX], wg[NMAX];           // Gauss points / weights
  double xl[NMAX], wl[NMAX];           // GLL nodes / weights
  double B[NMAX * NMAX];               // B[q*n+a] = l_a(xg_q), GLL Lagrange at Gauss points
  double D1[NMAX * NMAX];              // D1[q*n+a] = l_a'(xg_q)
  double DN[NMAX * NMAX];              // DN[p*n+a] = l_a'(xl_p), GLL Lagrange at GLL nodes
  double Dh[NMAX * NMAX];              // Dh[q*n+p] = derivative at xg_q of Gauss-Lagrange l^G_p
  double L[NMAX * NMAX];               // L[a*n+q] = P_a(xg_q)
  double J[NMAX * NMAX];               // J[a*n+i] = sum_q wg_q P_a(xg_q) B[q,i] / (2/(2a+1))
  int ma[NPMAX], mb[NPMAX], mc[NPMAX]; // pressure modes
};

namespace rules {

constexpr double cabs(double x) { return x < 0 ? -x : x; }

// cos(x) for |x| <= pi by its Taylor series (initial Newton guesses only).
constexpr double ccos(double x) {
  double s = 1.0, t = 1.0;
  for (int i = 1; i < 40; ++i) {
    t *= -x * x / ((2.0 * i - 1.0) * (2.0 * i));
    s += t;
  }
  return s;
}

constexpr double kPi = 3.14159265358979323846;

// P_N(x) and P_N'(x) by the three-term recurrence.
constexpr void legendre_pd(int N, double x, double* p, double* dp) {
  double p0 = 1.0, p1 = x;
  if (N == 0) {
    *p = 1.0;
    *dp = 0.0;
    return;
  }
  for (int j = 2; j <= N; ++j) {
    const double p2 = ((2.0 * j - 1.0) * x * p1 - (j - 1.0) * p0) / j;
    p0 = p1;
    p1 = p2;
  }
  *p = p1;
  // derivative from (x^2 - 1) P_N' = N (x P_N - P_{N-1})
  if (cabs(cabs(x) - 1.0) < 1e-15)
    *dp = (x > 0 ? 1.0 : (N % 2 ? 1.0 : -1.0)) * 0.5 * N * (N + 1.0);
  else
    *dp = N * (x * p1 - p0) / (x * x - 1.0);
}

constexpr double legendre(int a, double x) {
  double p = 0, dp = 0;
  legendre_pd(a, x, &p, &dp);
  return p;
}

// Gauss-Legendre rule with n points, ascending: Newton on P_n.
constexpr void gauss_rule(int n, double* x, double* w) {
  for (int i = 0; i < n; ++i) {
    double z = ccos(kPi * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double p = 0, dp = 0;
      legendre_pd(n, z, &p, &dp);
      const double dz = p / dp;
      z -= dz;
      if (cabs(dz) < 1e-16) break;
    }
    double p = 0, dp = 0;
    legendre_pd(n, z, &p, &dp);
    x[n - 1 - i] = z;
    w[n - 1 - i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

// Gauss-Lobatto-Legendre nodes (+-1 and the roots of P_N', N = n-1) and weights.
constexpr void gll_rule(int n, double* x, double* w) {
  const int N = n - 1;
  x[0] = -1.0;
  x[N] = 1.0;
  for (int i = 1; i < N; ++i) {
    // Newton on P_N' with P_N'' from Legendre's equation
    double z = -ccos(kPi * i / N);
    for (int it = 0; it < 100; ++it) {
      double p = 0, dp = 0;
      legendre_pd(N, z, &p, &dp);
      const double d2p = (2.0 * z * dp - N * (N + 1.0) * p) / (1.0 - z * z);
      const double dz = dp / d2p;
      z -= dz;
      if (cabs(dz) < 1e-16) break;
    }
    x[i] = z;
  }
  for (int i = 0; i < n; ++i) {
    double p = 0, dp = 0;
    legendre_pd(N, x[i], &p, &dp);
    w[i] = 2.0 / (N * (N + 1.0) * p * p);
  }
}

// Lagrange basis through nodes[0..n) evaluated at x[0..m): V[i*n+a] = l_a(x_i),
// D[i*n+a] = l_a'(x_i) (product rule).
constexpr void lagrange(int n, const double* nodes, int m, const double* x, double* V, double* D) {
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

// Pressure modes (a, b, c) with a+b+c <= k-1, c slowest, a fastest.
constexpr int modes(int k, int* ma, int* mb, int* mc) {
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

constexpr Tables build_tables(int k) {
  Tables t{};
  const int n = k + 1;
  t.n = n;
  t.k = k;
  gauss_rule(n, t.xg, t.wg);
  gll_rule(n, t.xl, t.wl);
  lagrange(n, t.xl, n, t.xg, t.B, t.D1);
  double Vl[NMAX * NMAX] = {};
  lagrange(n, t.xl, n, t.xl, Vl, t.DN);
  double Vg[NMAX * NMAX] = {};
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

}  // namespace rules

// Tables of order k = n-1 as a compile-time constant.
template <int n>
struct CT {
  static constexpr Tables t = rules::build_tables(n - 1);
};

}  // namespace wb
