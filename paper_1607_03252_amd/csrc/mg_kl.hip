// Host-side Karhunen-Loeve tables of the separable exponential covariance.
//
// Per axis the covariance exp(-|s-t|/lambda) on [0,1] (Section 3.2,
// eq. def:expcov, taken per coordinate) has eigenpairs
//   theta = 2 lambda / (1 + lambda^2 w^2),  phi(s) ~ sin(w s) + lambda w cos(w s),
// with w the positive roots of tan(w) = 2 lambda w / (lambda^2 w^2 - 1), one in
// each interval (m pi, (m+1) pi).  Roots are found here by a bracketed
// Newton iteration on g(w) = (lambda^2 w^2 - 1) sin w - 2 lambda w cos w, and
// the normalisation by Gauss-Legendre quadrature of phi^2.
#include <cmath>
#include <vector>

#include "mg_kl.h"

namespace mg {

namespace {

double g_fun(double lam, double w) {
  return (lam * lam * w * w - 1.0) * std::sin(w) - 2.0 * lam * w * std::cos(w);
}

double g_der(double lam, double w) {
  // d/dw [(l^2 w^2 - 1) sin w - 2 l w cos w]
  return 2.0 * lam * lam * w * std::sin(w) + (lam * lam * w * w - 1.0) * std::cos(w) -
         2.0 * lam * std::cos(w) + 2.0 * lam * w * std::sin(w);
}

// Gauss-Legendre nodes/weights on [-1,1] by Newton iteration on P_q.
void gauss_legendre(int q, std::vector<double>& x, std::vector<double>& w) {
  x.assign(q, 0.0);
  w.assign(q, 0.0);
  const double pi = 3.14159265358979323846;
  for (int i = 0; i < q; ++i) {
    double z = std::cos(pi * (i + 0.75) / (q + 0.5));
    double dp = 1.0;
    for (int it = 0; it < 100; ++it) {
      double p0 = 1.0, p1 = z;
      for (int k = 2; k <= q; ++k) {
        const double p2 = ((2.0 * k - 1.0) * z * p1 - (k - 1.0) * p0) / k;
        p0 = p1;
        p1 = p2;
      }
      dp = q * (z * p1 - p0) / (z * z - 1.0);
      const double dz = p1 / dp;
      z -= dz;
      if (std::fabs(dz) < 1e-16) break;
    }
    x[i] = z;
    w[i] = 2.0 / ((1.0 - z * z) * dp * dp);
  }
}

}  // namespace

bool kl_1d_modes(double lambda, int nmodes, double* omega, double* theta, double* scale) {
  if (!(lambda > 0.0) || nmodes < 1) return false;
  const double pi = 3.14159265358979323846;
  std::vector<double> gx, gw;
  gauss_legendre(16, gx, gw);
  for (int m = 0; m < nmodes; ++m) {
    double a = m * pi, b = (m + 1) * pi;
    // sign of g just right of m*pi is -(-1)^m; the root is the unique sign change
    const double sa = (m % 2 == 0) ? -1.0 : 1.0;
    double w = 0.5 * (a + b);
    for (int it = 0; it < 200; ++it) {
      const double gv = g_fun(lambda, w);
      if (gv == 0.0) break;
      if ((gv < 0.0) == (sa < 0.0)) a = w; else b = w;
      const double d = g_der(lambda, w);
      double wn = (d != 0.0) ? w - gv / d : 0.5 * (a + b);
      if (!(wn > a && wn < b)) wn = 0.5 * (a + b);  // keep Newton inside the bracket
      if (std::fabs(wn - w) <= 1e-15 * w) { w = wn; break; }
      w = wn;
    }
    omega[m] = w;
    theta[m] = 2.0 * lambda / (1.0 + lambda * lambda * w * w);
    // || sin(w s) + lambda w cos(w s) ||^2 on [0,1]: 64 panels x 16-point Gauss
    double nrm = 0.0;
    const int panels = 64;
    for (int p = 0; p < panels; ++p) {
      const double lo = (double)p / panels, hi = (double)(p + 1) / panels;
      for (int q = 0; q < 16; ++q) {
        const double s = 0.5 * (lo + hi) + 0.5 * (hi - lo) * gx[q];
        const double f = std::sin(w * s) + lambda * w * std::cos(w * s);
        nrm += 0.5 * (hi - lo) * gw[q] * f * f;
      }
    }
    scale[m] = 1.0 / std::sqrt(nrm);
  }
  return true;
}

void kl_phi_table(double lambda, int nmodes, const double* omega, const double* scale, int n,
                  double* table) {
  for (int m = 0; m < nmodes; ++m)
    for (int i = 0; i < n; ++i) {
      const double s = (double)i / (double)(n - 1);
      table[m * n + i] = scale[m] * (std::sin(omega[m] * s) + lambda * omega[m] * std::cos(omega[m] * s));
    }
}

}  // namespace mg
