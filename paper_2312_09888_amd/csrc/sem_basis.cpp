// GLL nodes, weights and collocation derivative matrix for the kernels.
//
// Standard spectral-element basis (Deville, Fischer & Mund 2002, ch. 2);
// the paper (section 1) only names the spectral element method.  Computed
// here in x87 extended precision and rounded once to double, so the tables
// the kernels read are correctly rounded to within an ulp.
//
// * nodes: -1, +1 and the roots of P_N', found by Newton's method on the
//   function (1 - x^2) P_N'(x) = N (P_{N-1}(x) - x P_N(x)), whose derivative
//   is -N(N+1) P_N(x) by Legendre's equation; starting guesses are the
//   Chebyshev-Gauss-Lobatto points.
// * weights: 2 / (N (N+1) P_N(xi)^2).
// * D[i][m] = l_m'(xi_i) = P_N(xi_i) / (P_N(xi_m) (xi_i - xi_m)), i != m;
//   D[i][i] = -sum_{m != i} D[i][m] (the derivative of a constant is 0).
#include <cmath>

#include "sem_internal.h"

namespace sem {
namespace {

using ld = long double;

// P_N(x) and P_{N-1}(x) by Bonnet's recurrence.
void legendre_pair(int n, ld x, ld* pn, ld* pnm1) {
  ld a = 1.0L, b = x;  // P_0, P_1
  if (n == 0) { *pn = a; *pnm1 = 0.0L; return; }
  for (int k = 1; k < n; ++k) {
    ld c = ((2 * k + 1) * x * b - k * a) / (k + 1);
    a = b;
    b = c;
  }
  *pn = b;
  *pnm1 = a;
}

}  // namespace

bool gll_basis(int n, double* nodes, double* weights, double* dmat) {
  if (n < 1 || n > kMaxBasisOrder) return false;
  const int p = n + 1;
  ld xi[kMaxBasisOrder + 1];
  ld pn[kMaxBasisOrder + 1];
  const ld pi = 3.141592653589793238462643383279502884L;
  xi[0] = -1.0L;
  xi[n] = 1.0L;
  for (int j = 1; j < n; ++j) {
    ld x = -std::cos(pi * j / n);
    for (int it = 0; it < 60; ++it) {
      ld a, b;
      legendre_pair(n, x, &a, &b);
      ld g = n * (b - x * a);          // (1 - x^2) P_N'
      ld dg = -(ld)n * (n + 1) * a;    // its derivative
      ld step = g / dg;
      x -= step;
      if (std::fabs(step) < 1e-21L) break;
    }
    xi[j] = x;
  }
  // exact symmetry about the midpoint
  for (int j = 0; j < p / 2; ++j) {
    ld s = 0.5L * (xi[n - j] - xi[j]);
    xi[j] = -s;
    xi[n - j] = s;
  }
  if (n % 2 == 0) xi[n / 2] = 0.0L;
  for (int j = 0; j < p; ++j) {
    ld b;
    legendre_pair(n, xi[j], &pn[j], &b);
  }
  if (nodes)
    for (int j = 0; j < p; ++j) nodes[j] = (double)xi[j];
  if (weights)
    for (int j = 0; j < p; ++j) weights[j] = (double)(2.0L / (n * (n + 1) * pn[j] * pn[j]));
  if (dmat) {
    for (int i = 0; i < p; ++i) {
      ld diag = 0.0L;
      for (int m = 0; m < p; ++m) {
        if (m == i) continue;
        ld v = pn[i] / (pn[m] * (xi[i] - xi[m]));
        dmat[i * p + m] = (double)v;
        diag -= v;
      }
      dmat[i * p + i] = (double)diag;
    }
  }
  return true;
}

}  // namespace sem
