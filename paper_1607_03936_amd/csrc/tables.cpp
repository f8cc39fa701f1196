// Host access to the 1D tables of rules.h (Sec. 1.2 discretization; node set and quadrature
// rule as documented in the header of wbfbt.h).
#include "wb_internal.h"

namespace wb {

double legendre(int a, double x) { return rules::legendre(a, x); }
void gauss_rule(int n, double* x, double* w) { rules::gauss_rule(n, x, w); }
void gll_rule(int n, double* x, double* w) { rules::gll_rule(n, x, w); }
void lagrange(int n, const double* nodes, int m, const double* x, double* V, double* D) {
  rules::lagrange(n, nodes, m, x, V, D);
}
int modes(int k, int* ma, int* mb, int* mc) { return rules::modes(k, ma, mb, mc); }

const Tables& tables(int k) {
  static constexpr Tables tab[NMAX] = {rules::build_tables(1), rules::build_tables(1),
                                       rules::build_tables(2), rules::build_tables(3),
                                       rules::build_tables(4), rules::build_tables(5)};
  return tab[k];
}

}  // namespace wb
