// Host-side Karhunen-Loeve tables (separable exponential covariance).
#pragma once

namespace mg {

// Roots omega[m], eigenvalues theta[m] and normalisation factors scale[m]
// (phi_m = scale[m] (sin(omega s) + lambda omega cos(omega s))) for m < nmodes.
bool kl_1d_modes(double lambda, int nmodes, double* omega, double* theta, double* scale);

// table[m*n + i] = phi_m(i/(n-1)) for m < nmodes, i < n.
void kl_phi_table(double lambda, int nmodes, const double* omega, const double* scale, int n,
                  double* table);

}  // namespace mg
