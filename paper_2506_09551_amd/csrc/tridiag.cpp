// Lowest eigenpair of a symmetric tridiagonal matrix (host).
//
// Used by the ground-state Lanczos: the Lanczos coefficients define
// T = tridiag(b, a, b); its lowest eigenvalue is found by bisection on the
// Sturm sequence count (the number of negative pivots of T - x I equals the
// number of eigenvalues below x), and the eigenvector by inverse iteration
// with a tridiagonal LU factorisation with partial pivoting.
#include <algorithm>
#include <cmath>
#include <vector>

#include "msb_internal.h"

namespace msb {

static int sturm_count(const std::vector<double>& a, const std::vector<double>& b, double x) {
  const size_t n = a.size();
  int count = 0;
  double q = a[0] - x;
  const double tiny = 1e-300;
  if (q < 0) ++count;
  for (size_t i = 1; i < n; ++i) {
    if (std::fabs(q) < tiny) q = -tiny;
    q = (a[i] - x) - b[i - 1] * b[i - 1] / q;
    if (q < 0) ++count;
  }
  return count;
}

// Solve (T - lam I) x = rhs by Gaussian elimination with partial pivoting on
// the tridiagonal band (fill-in of one extra super-diagonal).
static void tridiag_solve(const std::vector<double>& a, const std::vector<double>& b, double lam,
                          std::vector<double>& x) {
  const size_t n = a.size();
  std::vector<double> d(n), du(n, 0.0), du2(n, 0.0), dl(n, 0.0);
  for (size_t i = 0; i < n; ++i) d[i] = a[i] - lam;
  for (size_t i = 0; i + 1 < n; ++i) { du[i] = b[i]; dl[i] = b[i]; }
  std::vector<double> rhs = x;
  // LU with partial pivoting (LAPACK dgttrf-like, written out).
  for (size_t i = 0; i + 1 < n; ++i) {
    if (std::fabs(d[i]) >= std::fabs(dl[i])) {
      double piv = d[i];
      if (piv == 0.0) piv = d[i] = 1e-300;
      const double f = dl[i] / piv;
      d[i + 1] -= f * du[i];
      if (i + 2 < n) du2[i] = 0.0;
      rhs[i + 1] -= f * rhs[i];
      dl[i] = f;
    } else {
      // swap rows i and i+1
      const double f = d[i] / dl[i];
      d[i] = dl[i];
      const double tmp = d[i + 1];
      d[i + 1] = du[i] - f * tmp;
      du[i] = tmp;
      if (i + 2 < n) {
        du2[i] = du[i + 1];
        du[i + 1] = -f * du2[i];
      }
      std::swap(rhs[i], rhs[i + 1]);
      rhs[i + 1] -= f * rhs[i];
      dl[i] = f;
    }
  }
  if (d[n - 1] == 0.0) d[n - 1] = 1e-300;
  // back substitution
  x[n - 1] = rhs[n - 1] / d[n - 1];
  if (n > 1) x[n - 2] = (rhs[n - 2] - du[n - 2] * x[n - 1]) / d[n - 2];
  for (size_t k = n - 2; k-- > 0;) {
    x[k] = (rhs[k] - du[k] * x[k + 1] - du2[k] * x[k + 2]) / d[k];
  }
}

double tridiag_lowest(const std::vector<double>& a, const std::vector<double>& b,
                      std::vector<double>& y) {
  const size_t n = a.size();
  y.assign(n, 0.0);
  if (n == 0) return 0.0;
  if (n == 1) {
    y[0] = 1.0;
    return a[0];
  }
  // Gershgorin interval.
  double lo = a[0], hi = a[0];
  for (size_t i = 0; i < n; ++i) {
    const double r = (i > 0 ? std::fabs(b[i - 1]) : 0.0) + (i + 1 < n ? std::fabs(b[i]) : 0.0);
    lo = std::min(lo, a[i] - r);
    hi = std::max(hi, a[i] + r);
  }
  // Bisection for the smallest eigenvalue: count(x) >= 1 iff x > lambda_min.
  for (int it = 0; it < 200; ++it) {
    const double mid = 0.5 * (lo + hi);
    if (mid <= lo || mid >= hi) break;
    if (sturm_count(a, b, mid) >= 1) hi = mid; else lo = mid;
  }
  const double lam = 0.5 * (lo + hi);
  // Inverse iteration.
  std::vector<double> x(n, 1.0);
  for (size_t i = 0; i < n; ++i) x[i] = 1.0 + 1e-3 * (double)((i * 7919) % 97);
  for (int it = 0; it < 4; ++it) {
    tridiag_solve(a, b, lam, x);
    double nrm = 0.0;
    for (double v : x) nrm += v * v;
    nrm = std::sqrt(nrm);
    for (double& v : x) v /= nrm;
  }
  y = x;
  return lam;
}

}  // namespace msb
