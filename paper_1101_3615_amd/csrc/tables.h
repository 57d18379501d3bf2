// Host-side FP64 tables of the discretisation: stencil weights, wavelet,
// damping profile, stability bound.  The device needs no transcendental
// functions: everything here is computed once on the host and uploaded.
#pragma once
#include <cmath>
#include <vector>

namespace mp {

// 8th-order central second-difference weights w0, w1..w4.
static const double FD8[5] = {-205.0 / 72.0, 8.0 / 5.0, -1.0 / 5.0, 8.0 / 315.0, -1.0 / 560.0};

// Largest stable c dt / h of the undamped leapfrog with this Laplacian:
// 2 / sqrt(ndim * 2048/315) (the Nyquist symbol of each axis is -2048/315 h^-2).
inline double cfl_limit(int ndim) {
  double lam = -FD8[0];
  for (int j = 1; j <= 4; ++j) lam -= 2.0 * FD8[j] * ((j & 1) ? -1.0 : 1.0);
  return 2.0 / std::sqrt(ndim * lam);
}

// Ricker wavelet (second derivative of a Gaussian) at t_n = n dt, delayed by t0.
inline std::vector<double> ricker(double f, double t0, double dt, int nt) {
  std::vector<double> w(nt);
  const double pi = 3.14159265358979323846;
  for (int n = 0; n < nt; ++n) {
    const double a = (pi * f * (n * dt - t0)) * (pi * f * (n * dt - t0));
    w[n] = (1.0 - 2.0 * a) * std::exp(-a);
  }
  return w;
}

// Peak damping of the layer: eta_max = 3 c_max ln(1/R) / (2 nb h).
inline double sponge_max(int nb, double cmax, double h, double R) {
  return 3.0 * cmax * std::log(1.0 / R) / (2.0 * nb * h);
}

// Damping eta along one axis of n model cells with nb layer cells each side:
// eta_max (d / nb)^2, d = distance into the layer in cells.
inline std::vector<double> sponge_profile(int n, int nb, double cmax, double h, double R) {
  std::vector<double> e(n + 2 * nb, 0.0);
  if (nb <= 0) return e;
  const double emax = sponge_max(nb, cmax, h, R);
  for (int i = 0; i < n + 2 * nb; ++i) {
    int d = nb - i;
    const int d2 = i - (n + nb - 1);
    if (d2 > d) d = d2;
    if (d < 0) d = 0;
    const double r = (double)d / nb;
    e[i] = emax * r * r;
  }
  return e;
}

}  // namespace mp
