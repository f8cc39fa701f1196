// Internal declarations of the w-BFBT Stokes library (not part of the C-ABI).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "../../include/wbfbt.h"
#include "rules.h"

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

// All 1D tables of one order k (n = k+1) and the compile-time copy CT<n>: see rules.h.
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
