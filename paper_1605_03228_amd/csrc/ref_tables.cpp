// Host construction of the 1-D reference tables: GLL nodes and weights,
// Gauss-Legendre points and weights, and the Lagrange basis on the GLL nodes.
//
// GLL nodes are +-1 and the roots of P_p'; Gauss points are the roots of
// P_{p+2}.  Both are found by Newton's method on the Legendre recurrence.
#include <cmath>

#include "common.hpp"
#include "internal.hpp"

namespace ihdg {

// P_n(x) and P_n'(x) by the three-term recurrence.
static void legendre(int n, double x, double* P, double* dP) {
  double p0 = 1.0, p1 = x;
  if (n == 0) {
    *P = 1.0;
    *dP = 0.0;
    return;
  }
  for (int k = 2; k <= n; ++k) {
    double p2 = ((2 * k - 1) * x * p1 - (k - 1) * p0) / k;
    p0 = p1;
    p1 = p2;
  }
  *P = p1;
  if (std::fabs(std::fabs(x) - 1.0) < 1e-15) {
    *dP = (x > 0 ? 1.0 : (n % 2 ? 1.0 : -1.0)) * 0.5 * n * (n + 1);
  } else {
    *dP = n * (p0 - x * p1) / (1.0 - x * x);
  }
}

static void gauss_rule(int n, double* x, double* w) {
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < n; ++i) {
    double t = -std::cos(pi * (i + 0.75) / (n + 0.5));
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(n, t, &P, &dP);
      double dt = P / dP;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    double P, dP;
    legendre(n, t, &P, &dP);
    x[i] = t;
    w[i] = 2.0 / ((1.0 - t * t) * dP * dP);
  }
}

static void gll_rule(int p, double* x, double* w) {
  const double pi = 3.14159265358979323846;
  for (int i = 0; i <= p; ++i) x[i] = -std::cos(pi * i / p);
  for (int i = 1; i < p; ++i) {
    double t = x[i];
    for (int it = 0; it < 100; ++it) {
      double P, dP;
      legendre(p, t, &P, &dP);
      // q = (1 - t^2) P_p'(t);  q' = -p(p+1) P_p(t)
      double q = (1 - t * t) * dP, dq = -p * (p + 1) * P;
      double dt = q / dq;
      t -= dt;
      if (std::fabs(dt) < 1e-16) break;
    }
    x[i] = t;
  }
  x[0] = -1.0;
  x[p] = 1.0;
  for (int i = 0; i <= p; ++i) {
    double P, dP;
    legendre(p, x[i], &P, &dP);
    w[i] = 2.0 / (p * (p + 1) * P * P);
  }
}

static void lagrange_at(const double* r, int n1, double t, double* L, double* dL) {
  for (int j = 0; j < n1; ++j) {
    double den = 1.0, val = 1.0, der = 0.0;
    for (int m = 0; m < n1; ++m) {
      if (m == j) continue;
      den *= r[j] - r[m];
    }
    for (int m = 0; m < n1; ++m) {
      if (m == j) continue;
      double prod = 1.0;
      for (int k = 0; k < n1; ++k)
        if (k != j && k != m) prod *= t - r[k];
      der += prod;
      val *= t - r[m];
    }
    L[j] = val / den;
    dL[j] = der / den;
  }
}

RefTab make_reftab(int p, int dim) {
  RefTab t{};
  t.p = p;
  t.n1 = p + 1;
  t.nq1 = p + 2;
  t.dim = dim;
  gll_rule(p, t.r, t.wgll);
  gauss_rule(t.nq1, t.q, t.wq);
  for (int a = 0; a < t.nq1; ++a) lagrange_at(t.r, t.n1, t.q[a], t.L[a], t.dL[a]);
  double dummy[kMax1];
  lagrange_at(t.r, t.n1, -1.0, t.Lend[0], dummy);
  lagrange_at(t.r, t.n1, 1.0, t.Lend[1], dummy);
  return t;
}

}  // namespace ihdg
