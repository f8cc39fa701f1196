// Internal declarations of the w-BFBT Stokes library (not part of the C-ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/wbfbt.h"

namespace wb {

// ---------------------------------------------------------------- errors
void set_error(const std::string& msg);

struct Error {
  wb_status code;
  std::string msg;
};

#define WB_HIP(call)                                                                  \
  do {                                                                                \
    hipError_t e_ = (call);                                                           \
    if (e_ != hipSuccess)                                                             \
      throw ::wb::Error{WB_EHIP, std::string(#call) + ": " + hipGetErrorString(e_)};  \
  } while (0)

#define WB_REQUIRE(cond, code, msg)                  \
  do {                                               \
    if (!(cond)) throw ::wb::Error{code, msg};       \
  } while (0)

// --------------------------------------------------------- 1D tables (host)
// Gauss-Legendre rule with n points on [-1,1].
void gauss_rule(int n, double* x, double* w);
// Gauss-Lobatto-Legendre points and weights with n points.
void gll_rule(int n, double* x, double* w);
// Lagrange basis through nodes[0..n): V[i*n+a] = l_a(x_i), D[i*n+a] = l_a'(x_i).
void lagrange(int n, const double* nodes, int m, const double* x, double* V, double* D);
// Unnormalized Legendre polynomial P_a(x).
double legendre(int a, double x);
// Modes (a,b,c) with a+b+c <= k-1, c slowest, a fastest.
int modes(int k, int* ma, int* mb, int* mc);

constexpr int NMAX = 5;   // n = k+1 <= 5
constexpr int NPMAX = 20; // modes for k = 4

// All 1D tables of one order k (n = k+1), double precision; kernels receive a
// per-order copy by value.
struct Tables {
  int n, k, np;
  double xg[NMAX], wg[NMAX];           // Gauss points / weights
  double xl[NMAX], wl[NMAX];           // GLL nodes / weights
  double B[NMAX * NMAX];               // B[q*n+a] = l_a(xg_q), GLL Lagrange at Gauss points
  double D1[NMAX * NMAX];              // D1[q*n+a] = l_a'(xg_q)
  double Dh[NMAX * NMAX];              // Dh[q*n+p] = derivative at xg_q of Gauss-Lagrange l^G_p
  double L[NMAX * NMAX];               // L[a*n+q] = P_a(xg_q)
  double J[NMAX * NMAX];               // J[a*n+i] = sum_q wg_q P_a(xg_q) B[q,i] / (2/(2a+1))
  int ma[NPMAX], mb[NPMAX], mc[NPMAX]; // pressure modes
};
const Tables& tables(int k);

// --------------------------------------------------------------- handles
struct Mesh {
  int N, k, n, M;
  int nn;      // nodes (kN+1)^3
  int E;       // elements N^3
  int np;      // pressure modes
  double h;
};

}  // namespace wb

struct wb_mesh {
  wb::Mesh m;
  mutable void* work = nullptr;  // face-array workspace of standalone operator applies
};

struct wb_visc {
  wb::Mesh m;
  double* mu_q = nullptr;      // [E][n^3]
  double* mu_nodes = nullptr;  // [nn]
  float* mu_q_f = nullptr;     // FP32 copy (lazily created)
};
