// Device code shared by the direct-sum and the particle-mesh trace kernels:
// the background a(t) and the geodesic right-hand side in z.  Not part of the
// public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "rt_internal.h"

namespace rt {

// ---------------------------------------------------------------------------
// Background: a(t) of eq. scalefac2 (t = lookback time) and da/dt.
// ---------------------------------------------------------------------------
__device__ __forceinline__ void scale_factor(const DevCosmo& c, double t, double& a, double& adot) {
  const double rate = 1.5 * c.sqrt_ol * c.H0;
  const double u = rate * (c.t0 - t);
  const double e = exp(u);
  const double ie = 1.0 / e;
  const double sh = 0.5 * (e - ie), ch = 0.5 * (e + ie);
  a = cbrt(c.ratio * sh * sh);
  // a^3 = ratio sh^2  =>  3 a^2 da/dt = -2 ratio sh ch rate
  adot = -(2.0 / 3.0) * rate * c.ratio * sh * ch / (a * a);
}

// ---------------------------------------------------------------------------
// Geodesic right-hand side (Sec. 3.4, eq. geodesiceqn), Christoffel symbols
// differentiated exactly from eq. expandingmetric with psi = phi / a.  The
// z-form (x^3 as independent variable) integrates Y = (t, x, y, kt, kx, ky, kz).
// ---------------------------------------------------------------------------
struct State {
  double t, x, y, kt, kx, ky, kz;
};

// The contraction A^mu = Gamma^mu_ab k^a k^b at lookback time t for wave vector
// (kt, kx, ky, kz), comoving potential phi and gradient g; a_out = a(t).
__device__ __forceinline__ void accel(const DevCosmo& c, double t, double kt, double kx, double ky, double kz,
                                      double phi, double gx, double gy, double gz, double& a_out, double& At,
                                      double& Ax, double& Ay, double& Az) {
  double a, adot;
  scale_factor(c, t, a, adot);
  a_out = a;
  const double inv_a = 1.0 / a;
  const double invE = 1.0 / (1.0 + 2.0 * phi * inv_a);
  const double invF = 1.0 / (a * a - 2.0 * a * phi);
  const double gk = gx * kx + gy * ky + gz * kz;
  const double k2 = kx * kx + ky * ky + kz * kz;
  const double kt2 = kt * kt;
  const double hub = adot * (a - phi);
  At = (-adot * phi * inv_a * inv_a * kt2 + 2.0 * kt * inv_a * gk + hub * k2) * invE;
  const double c1 = kt2 * inv_a, c2 = 2.0 * hub * kt;
  Ax = (gx * c1 + c2 * kx + a * (gx * k2 - 2.0 * kx * gk)) * invF;
  Ay = (gy * c1 + c2 * ky + a * (gy * k2 - 2.0 * ky * gk)) * invF;
  Az = (gz * c1 + c2 * kz + a * (gz * k2 - 2.0 * kz * gk)) * invF;
}

// dY/dz = (dY/dlambda) / k^z.
__device__ __forceinline__ State rhs(const DevCosmo& c, const State& Y, double phi, double gx, double gy, double gz,
                                     double& a_out) {
  double At, Ax, Ay, Az;
  accel(c, Y.t, Y.kt, Y.kx, Y.ky, Y.kz, phi, gx, gy, gz, a_out, At, Ax, Ay, Az);
  const double iz = 1.0 / Y.kz;
  return State{Y.kt * iz, Y.kx * iz, Y.ky * iz, -At * iz, -Ax * iz, -Ay * iz, -Az * iz};
}

__device__ __forceinline__ State axpy(const State& Y, double h, const State& k) {
  return State{Y.t + h * k.t, Y.x + h * k.x, Y.y + h * k.y, Y.kt + h * k.kt, Y.kx + h * k.kx, Y.ky + h * k.ky,
               Y.kz + h * k.kz};
}

}  // namespace rt
