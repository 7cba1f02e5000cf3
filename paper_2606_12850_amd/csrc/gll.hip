// GLL nodes, weights, Lagrange basis and differentiation matrix for the
// library (host, FP64).  Sec. II-B: the interpolation points of an element
// are tensor products of the N+1 one-dimensional Gauss-Lobatto-Legendre
// points; the basis is the Lagrange polynomials on them, and reference
// derivatives at the nodes are products with D_ab = l'_b(xi_a).
#include <cmath>
#include <vector>

#include "semx_internal.hpp"

namespace semx {

namespace {
// P_N(x) and P'_N(x) via the Bonnet recurrence.
void legendre_pd(int N, double x, double& p, double& dp) {
  double pm1 = 1.0, pc = x;
  if (N == 0) { p = 1.0; dp = 0.0; return; }
  for (int m = 2; m <= N; ++m) {
    double pn = ((2 * m - 1) * x * pc - (m - 1) * pm1) / m;
    pm1 = pc;
    pc = pn;
  }
  p = pc;
  // P'_N(x) = N (x P_N - P_{N-1}) / (x^2 - 1) away from the end points
  if (std::fabs(std::fabs(x) - 1.0) < 1e-300) dp = (x > 0 ? 1.0 : (N % 2 ? 1.0 : -1.0)) * 0.5 * N * (N + 1);
  else dp = N * (x * pc - pm1) / (x * x - 1.0);
}
}  // namespace

void gll_nodes_weights(int n, std::vector<double>& xi, std::vector<double>& w) {
  const int N = n - 1;
  xi.assign(n, 0.0);
  w.assign(n, 0.0);
  xi[0] = -1.0;
  xi[N] = 1.0;
  // interior nodes: zeros of P'_N; Newton on q(x) = (1 - x^2) P'_N(x), whose
  // derivative is -N(N+1) P_N(x) by Legendre's equation.
  for (int a = 1; a < N; ++a) {
    double x = -std::cos(M_PI * a / N);
    for (int it = 0; it < 60; ++it) {
      double p, dp;
      legendre_pd(N, x, p, dp);
      double q = (1.0 - x * x) * dp;
      double dq = -N * (N + 1.0) * p;
      double step = q / dq;
      x -= step;
      if (std::fabs(step) < 1e-17) break;
    }
    xi[a] = x;
  }
  for (int a = 0; a < n / 2; ++a) {
    double s = 0.5 * (xi[N - a] - xi[a]);
    xi[a] = -s;
    xi[N - a] = s;
  }
  if (n % 2) xi[N / 2] = 0.0;
  for (int a = 0; a < n; ++a) {
    double p, dp;
    legendre_pd(N, xi[a], p, dp);
    w[a] = 2.0 / (N * (N + 1.0) * p * p);
  }
}

void lagrange_at(int n, const std::vector<double>& xi, double x, double* l) {
  for (int a = 0; a < n; ++a) {
    double v = 1.0;
    for (int m = 0; m < n; ++m)
      if (m != a) v *= (x - xi[m]) / (xi[a] - xi[m]);
    l[a] = v;
  }
}

// Closed form of the GLL differentiation matrix: off the diagonal
// D_ab = P_N(xi_a) / (P_N(xi_b) (xi_a - xi_b)); the diagonal makes every row
// sum to zero (derivative of a constant), which fixes D_00 = -N(N+1)/4,
// D_NN = N(N+1)/4 and 0 elsewhere up to rounding.
void deriv_matrix(int n, const std::vector<double>& xi, std::vector<double>& D) {
  const int N = n - 1;
  std::vector<double> P(n);
  for (int a = 0; a < n; ++a) {
    double dp;
    legendre_pd(N, xi[a], P[a], dp);
  }
  D.assign(n * n, 0.0);
  for (int a = 0; a < n; ++a) {
    double row = 0.0;
    for (int b = 0; b < n; ++b) {
      if (a == b) continue;
      D[a * n + b] = P[a] / (P[b] * (xi[a] - xi[b]));
      row += D[a * n + b];
    }
    D[a * n + a] = -row;
  }
}

}  // namespace semx
