/*
 * Plain FP64 CPU oracle for three-dimensional ray-bundle lensing
 * (Killedar, Lasky, Lewis & Fluke 2011, "Gravitational lensing with
 * three-dimensional ray tracing").
 *
 * TEST INFRASTRUCTURE ONLY: it exists to check the GPU library.  Only the
 * tests, the smoke check and the CPU-baseline leg of the benchmark load it.
 * It shares no code, header, table or constant generator with the product.
 *
 * Everything here is written for a reader holding the paper: each function
 * names the section or equation it follows.  Sums run in natural order, one
 * particle after another, with no blocking or reordering.  No fast-math.
 *
 * Parity pins: every function is pinned by tests/test_oracle_*.py against
 * closed forms, printed values, brute force or independent quadrature.
 */
#include "oracle.h"

#include <math.h>
#include <stdlib.h>
#include <string.h>
#ifdef _OPENMP
#include <omp.h>
#endif

/* ------------------------------------------------------------------------ */
/* Constants (published values, chosen here; the paper states none).        */
/*   GM_sun: IAU 2012 nominal heliocentric gravitational parameter.         */
/*   c: exact SI value.  1 pc = 3.0856775814913673e16 m (IAU 2015, exact).  */
/* ------------------------------------------------------------------------ */
static const double GM_SUN_SI = 1.32712440018e20;      /* m^3 s^-2 */
static const double C_SI = 299792458.0;                /* m s^-1   */
static const double MPC_SI = 3.0856775814913673e22;    /* m        */
static const double C_KM_S = 299792.458;               /* km s^-1  */

double or_G_over_c2(void) { return GM_SUN_SI / (C_SI * C_SI) / MPC_SI; }

/* H0 = 100 h km/s/Mpc expressed in Mpc^-1 with c = 1. */
double or_H0(const or_cosmo* c) { return 100.0 * c->h / C_KM_S; }

/* eq. critdens at t = 0: rho_c = 3 H0^2 / (8 pi G), here in Msun / Mpc^3. */
double or_rho_crit0(const or_cosmo* c) {
  double H = or_H0(c);
  return 3.0 * H * H / (8.0 * M_PI * or_G_over_c2());
}

/* ------------------------------------------------------------------------ */
/* Background cosmology: Sec. 3.5 (eq. scalefac2, lookbacksingularity),      */
/* Sec. 5.1 (eq. raytracedistance), App. E (eq. angularDD12, DRempty).       */
/* ------------------------------------------------------------------------ */

/* H(z)/H0 for the flat Lemaitre model (Omega_m + Omega_Lambda = 1). */
double or_E(const or_cosmo* c, double z) {
  double zp = 1.0 + z;
  return sqrt(c->omega_m * zp * zp * zp + c->omega_lambda);
}

typedef double (*or_integrand)(const or_cosmo*, double);

static double inv_E(const or_cosmo* c, double z) { return 1.0 / or_E(c, z); }
static double inv_E_zp2(const or_cosmo* c, double z) {
  double zp = 1.0 + z;
  return 1.0 / (zp * zp * or_E(c, z));
}

/* Adaptive Simpson with Richardson correction. */
static double simpson(or_integrand f, const or_cosmo* c, double a, double b, double fa, double fm,
                      double fb, double whole, double tol, int depth) {
  double m = 0.5 * (a + b), lm = 0.5 * (a + m), rm = 0.5 * (m + b);
  double flm = f(c, lm), frm = f(c, rm);
  double left = (m - a) / 6.0 * (fa + 4.0 * flm + fm);
  double right = (b - m) / 6.0 * (fm + 4.0 * frm + fb);
  double delta = left + right - whole;
  if (depth <= 0 || fabs(delta) <= 15.0 * tol) return left + right + delta / 15.0;
  return simpson(f, c, a, m, fa, flm, fm, left, 0.5 * tol, depth - 1) +
         simpson(f, c, m, b, fm, frm, fb, right, 0.5 * tol, depth - 1);
}

static double integrate(or_integrand f, const or_cosmo* c, double a, double b) {
  const int panels = 64;
  double total = 0.0;
  for (int i = 0; i < panels; ++i) {
    double x0 = a + (b - a) * i / panels, x1 = a + (b - a) * (i + 1) / panels;
    double f0 = f(c, x0), f1 = f(c, x1), fm = f(c, 0.5 * (x0 + x1));
    double whole = (x1 - x0) / 6.0 * (f0 + 4.0 * fm + f1);
    total += simpson(f, c, x0, x1, f0, fm, f1, whole, 1e-15 * fabs(whole) + 1e-300, 30);
  }
  return total;
}

/* eq. raytracedistance: D_C = c * int_0^z dz / H(z). */
double or_comoving_distance(const or_cosmo* c, double z) {
  if (z <= 0.0) return 0.0;
  return integrate(inv_E, c, 0.0, z) / or_H0(c);
}

/* eq. DRempty: D_eb = c * int_0^z dz / ((1+z)^2 H(z)). */
double or_empty_beam_distance(const or_cosmo* c, double z) {
  if (z <= 0.0) return 0.0;
  return integrate(inv_E_zp2, c, 0.0, z) / or_H0(c);
}

/* eq. lookbacksingularity, read with the square root that a(0) = 1 requires:
 * t0 = 2 / (3 H0 sqrt(OL)) * asinh(sqrt(OL / OM)). */
double or_t0(const or_cosmo* c) {
  return 2.0 / (3.0 * or_H0(c) * sqrt(c->omega_lambda)) * asinh(sqrt(c->omega_lambda / c->omega_m));
}

/* eq. scalefac2 with t the lookback time, and its exact t-derivative. */
void or_scale_factor(const or_cosmo* c, double t, double* a, double* adot) {
  double H0 = or_H0(c), sl = sqrt(c->omega_lambda);
  double u = 1.5 * sl * H0 * (or_t0(c) - t);
  double sh = sinh(u), ch = cosh(u);
  double ratio = c->omega_m / c->omega_lambda;
  double av = cbrt(ratio * sh * sh);
  *a = av;
  /* d(a^3)/dt = ratio * 2 sh ch * du/dt, du/dt = -1.5 sl H0 */
  *adot = -(ratio * sh * ch * sl * H0) / (av * av);
}

/* ------------------------------------------------------------------------ */
/* Potential of a uniform rectangular cuboid (the mean density that Sec. 3.3 */
/* subtracts, eq. perturbation and meanmatterdens).                          */
/* U(p) = int over the cuboid of d^3x' / |p - x'|; gradU = dU/dp.            */
/* Closed form from the antiderivative of 1/R in three variables, evaluated  */
/* at the eight corners with alternating signs.                              */
/* ------------------------------------------------------------------------ */

/* coef * ln(w + R), R = sqrt(w^2 + other2); written without cancellation for
 * w < 0, and zero when coef is zero. */
static double coef_log(double coef, double w, double R, double other2) {
  if (coef == 0.0) return 0.0;
  double s = (w >= 0.0) ? (w + R) : other2 / (R - w);
  return coef * log(s);
}

/* coef * atan(num / den), zero when coef is zero. */
static double coef_atan(double coef, double num, double den) {
  if (coef == 0.0) return 0.0;
  return coef * atan(num / den);
}

/* F(X,Y,Z) with d^3F/dXdYdZ = 1/R. */
static double prism_F(double X, double Y, double Z) {
  double X2 = X * X, Y2 = Y * Y, Z2 = Z * Z;
  double R = sqrt(X2 + Y2 + Z2);
  if (R == 0.0) return 0.0;
  return coef_log(X * Y, Z, R, X2 + Y2) + coef_log(Y * Z, X, R, Y2 + Z2) + coef_log(Z * X, Y, R, Z2 + X2) -
         coef_atan(0.5 * X2, Y * Z, X * R) - coef_atan(0.5 * Y2, Z * X, Y * R) - coef_atan(0.5 * Z2, X * Y, Z * R);
}

/* G(A; B, C) = int int dB dC / R at fixed A, the face integral used for dU/dp_A. */
static double prism_G(double A, double B, double C) {
  double A2 = A * A, B2 = B * B, C2 = C * C;
  double R = sqrt(A2 + B2 + C2);
  if (R == 0.0) return 0.0;
  return coef_log(B, C, R, A2 + B2) + coef_log(C, B, R, A2 + C2) - coef_atan(A, B * C, A * R);
}

void or_prism(const double lo[3], const double hi[3], const double p[3], double* U, double gradU[3]) {
  double X[2] = {lo[0] - p[0], hi[0] - p[0]};
  double Y[2] = {lo[1] - p[1], hi[1] - p[1]};
  double Z[2] = {lo[2] - p[2], hi[2] - p[2]};
  double u = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
  for (int i = 0; i < 2; ++i)
    for (int j = 0; j < 2; ++j)
      for (int k = 0; k < 2; ++k) {
        /* sign = product over the axes of (+1 upper limit, -1 lower limit) */
        double s = (i ? 1.0 : -1.0) * (j ? 1.0 : -1.0) * (k ? 1.0 : -1.0);
        u += s * prism_F(X[i], Y[j], Z[k]);
        /* the limits depend on p with d(limit)/dp = -1 */
        gx -= s * prism_G(X[i], Y[j], Z[k]);
        gy -= s * prism_G(Y[j], Z[k], X[i]);
        gz -= s * prism_G(Z[k], X[i], Y[j]);
      }
  *U = u;
  gradU[0] = gx;
  gradU[1] = gy;
  gradU[2] = gz;
}

/* ------------------------------------------------------------------------ */
/* Field of one particle set, Sec. 3.3 (eq. psi, derivs, phicotophys), with   */
/* the Green's-function prefactor G/c^2 and the integrand at x' (the printed */
/* 4 pi and delta(x) are read as typos).  The density of point masses with   */
/* Plummer softening eps gives                                               */
/*   phi(p)   = -(G/c^2) [ sum_j m_j / sqrt(r_j^2 + eps^2) - rho_bar U(p) ]   */
/*   dphi/dp  =  (G/c^2) [ sum_j m_j (p - x_j) / (r_j^2 + eps^2)^(3/2)       */
/*                         - rho_bar dU/dp ]                                */
/* where the U term appears only for sets with a background cuboid and      */
/* rho_bar = Omega_m rho_c0 is the comoving mean density (eq. meanmatterdens)*/
/* ------------------------------------------------------------------------ */
void or_field_at(const or_cosmo* c, const or_set* s, const double p[3], double* phi, double grad[3]) {
  double eps2 = s->softening * s->softening;
  double sum_phi = 0.0, sx = 0.0, sy = 0.0, sz = 0.0;
  for (int64_t j = 0; j < s->n; ++j) {
    double dx = p[0] - s->x[j], dy = p[1] - s->y[j], dz = p[2] - s->z[j];
    double r2 = dx * dx + dy * dy + dz * dz + eps2;
    double r = sqrt(r2);
    double w = s->m[j] / r;      /* m / r        */
    double w3 = w / r2;          /* m / r^3      */
    sum_phi += w;
    sx += w3 * dx;
    sy += w3 * dy;
    sz += w3 * dz;
  }
  double G = or_G_over_c2();
  double ph = -G * sum_phi, gx = G * sx, gy = G * sy, gz = G * sz;
  if (s->background) {
    double U, gU[3];
    double rho_bar = c->omega_m * or_rho_crit0(c);
    or_prism(s->lo, s->hi, p, &U, gU);
    /* minus the field of the uniform cuboid, whose potential is -G rho U */
    ph += G * rho_bar * U;
    gx += G * rho_bar * gU[0];
    gy += G * rho_bar * gU[1];
    gz += G * rho_bar * gU[2];
  }
  *phi = ph;
  grad[0] = gx;
  grad[1] = gy;
  grad[2] = gz;
}

/* ------------------------------------------------------------------------ */
/* Geodesic equation (Sec. 3.4, eq. geodesiceqn) for the metric of eq.       */
/* expandingmetric with psi = phi / a (eq. phicotophys):                     */
/*   g_tt = -(1 + 2 phi/a) = -E,   g_ij = (a^2 - 2 a phi) delta_ij = F delta_ij */
/* Christoffel symbols differentiated exactly from these components          */
/* (App. A lists them to first order in phi):                                */
/*   G^t_tt = -adot phi / (a^2 E)       G^t_ti = g_i / (a E)                  */
/*   G^t_ij = delta_ij adot (a - phi) / E                                     */
/*   G^i_tt = g_i / (a F)               G^i_tj = delta_ij adot (a - phi) / F  */
/*   G^i_jk = a (g_i delta_jk - g_j delta_ik - g_k delta_ij) / F              */
/* A^alpha = G^alpha_beta_gamma k^beta k^gamma.                               */
/* ------------------------------------------------------------------------ */
void or_accel(const or_cosmo* c, double t, const double k[4], double phi, const double g[3], double A[4]) {
  double a, adot;
  or_scale_factor(c, t, &a, &adot);
  double E = 1.0 + 2.0 * phi / a;
  double F = a * a - 2.0 * a * phi;
  double kt = k[0];
  double gk = g[0] * k[1] + g[1] * k[2] + g[2] * k[3];
  double k2 = k[1] * k[1] + k[2] * k[2] + k[3] * k[3];
  /* time component */
  double Gtt = -adot * phi / (a * a);
  A[0] = (Gtt * kt * kt + 2.0 * (kt / a) * gk + adot * (a - phi) * k2) / E;
  /* spatial components */
  for (int i = 0; i < 3; ++i) {
    A[1 + i] = ((g[i] / a) * kt * kt + 2.0 * adot * (a - phi) * kt * k[1 + i] +
                a * (g[i] * k2 - 2.0 * k[1 + i] * gk)) / F;
  }
}

/* The same geodesic with x^3 = z as the independent variable: for
 * Y = (t, x, y, kt, kx, ky, kz),  dY/dz = (kt, kx, ky, -A^t, -A^x, -A^y, -A^z) / kz. */
void or_derivs(const or_cosmo* c, const double Y[7], double phi, const double g[3], double dY[7]) {
  double k[4] = {Y[3], Y[4], Y[5], Y[6]};
  double A[4];
  or_accel(c, Y[0], k, phi, g, A);
  double inv = 1.0 / Y[6];
  dY[0] = Y[3] * inv;
  dY[1] = Y[4] * inv;
  dY[2] = Y[5] * inv;
  dY[3] = -A[0] * inv;
  dY[4] = -A[1] * inv;
  dY[5] = -A[2] * inv;
  dY[6] = -A[3] * inv;
}

/* ------------------------------------------------------------------------ */
/* Step schedule (Sec. 3.4 fixes the RK4 step; here the nodes are explicit). */
/* n_fine equal steps over [z_lo, z_hi]; outside it, steps grow by q away    */
/* from the interval until 0 and chi_s; a final step shorter than half its   */
/* nominal length is merged into the one before it.                          */
/* ------------------------------------------------------------------------ */
int or_make_schedule(double chi_s, double z_lo, double z_hi, int32_t n_fine, double q, double* nodes,
                     int32_t capacity, int32_t* n_steps) {
  if (!(chi_s > 0.0) || !(z_lo >= 0.0) || !(z_hi > z_lo) || !(z_hi <= chi_s) || n_fine < 1 || !(q >= 1.0))
    return -1;
  double h = (z_hi - z_lo) / n_fine;
  /* lower outer nodes, generated downward from z_lo */
  int32_t n_low = 0;
  double* low = NULL;
  if (z_lo > 0.0) {
    low = (double*)malloc(sizeof(double) * (size_t)capacity);
    double r = z_lo, hk = h;
    for (;;) {
      hk *= q;
      if (n_low >= capacity) { free(low); return -2; }
      if (r - hk < 0.5 * hk) { low[n_low++] = 0.0; break; }
      r -= hk;
      low[n_low++] = r;
    }
  }
  int32_t n = 0;
  for (int32_t i = n_low - 1; i >= 0; --i) {
    if (n >= capacity) { free(low); return -2; }
    nodes[n++] = low[i];
  }
  free(low);
  for (int32_t i = 0; i < n_fine; ++i) {
    if (n >= capacity) return -2;
    nodes[n++] = z_lo + (double)i * h;
  }
  if (n >= capacity) return -2;
  nodes[n++] = z_hi;
  if (z_hi < chi_s) {
    double r = z_hi, hk = h;
    for (;;) {
      hk *= q;
      if (n >= capacity) return -2;
      if (chi_s - (r + hk) < 0.5 * hk) { nodes[n++] = chi_s; break; }
      r += hk;
      nodes[n++] = r;
    }
  }
  *n_steps = n - 1;
  return 0;
}

/* Box replicas stacked along the line of sight, replica r covering
 * [r L, (r+1) L): each step uses the replica containing its midpoint. */
int or_replica_step_sets(const double* nodes, int32_t n_steps, double box, int32_t n_replicas, int32_t* step_set) {
  if (!(box > 0.0) || n_replicas < 1) return -1;
  for (int32_t s = 0; s < n_steps; ++s) {
    double mid = 0.5 * (nodes[s] + nodes[s + 1]);
    int32_t r = (int32_t)floor(mid / box);
    if (r < 0) r = 0;
    if (r > n_replicas - 1) r = n_replicas - 1;
    step_set[s] = r;
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Ray bundles (Sec. 3.1: a central ray and 8 rays on a regular        */
/* polygon).  Ring ray k sits at angle pi k / 4, counter-clockwise from +x.  */
/* Directions are gnomonic, n ~ (theta_x, theta_y, 1), so that straight rays */
/* reach the plane z = chi_s at theta * chi_s.  At the observer t = 0,       */
/* x = 0, kt = 1 and k = n sqrt(E0 / F0), which is exactly null.             */
/* ------------------------------------------------------------------------ */
static const double RING_C[8] = {1.0, 0.70710678118654752440, 0.0, -0.70710678118654752440,
                                 -1.0, -0.70710678118654752440, 0.0, 0.70710678118654752440};
static const double RING_S[8] = {0.0, 0.70710678118654752440, 1.0, 0.70710678118654752440,
                                 0.0, -0.70710678118654752440, -1.0, -0.70710678118654752440};

static double observer_potential(const or_cosmo* c, const or_field* f) {
  if (f->n_steps < 1) return 0.0;
  int32_t S = f->step_set[0];
  if (S < 0) return 0.0;
  double p[3] = {0.0, 0.0, 0.0}, phi, g[3];
  or_field_at(c, &f->sets[S], p, &phi, g);
  return phi;
}

int or_build_bundles(const or_cosmo* c, const or_field* fields, int32_t n_fields, int64_t n_bundles,
                     const double* theta, double radius, double* rays) {
  int64_t n_rays = 9 * n_bundles;
  double a0, adot0;
  or_scale_factor(c, 0.0, &a0, &adot0);
  for (int64_t b = 0; b < n_bundles; ++b) {
    double phi_obs = 0.0;
    for (int32_t f = 0; f < n_fields; ++f)
      if (b >= fields[f].bundle_offset && b < fields[f].bundle_offset + fields[f].n_bundles)
        phi_obs = observer_potential(c, &fields[f]);
    double E0 = 1.0 + 2.0 * phi_obs / a0, F0 = a0 * a0 - 2.0 * a0 * phi_obs;
    double norm = sqrt(E0 / F0);
    for (int k = 0; k < 9; ++k) {
      double tx = theta[b], ty = theta[n_bundles + b];
      if (k > 0) {
        tx += radius * RING_C[k - 1];
        ty += radius * RING_S[k - 1];
      }
      double len = sqrt(tx * tx + ty * ty + 1.0);
      int64_t i = 9 * b + k;
      rays[0 * n_rays + i] = 0.0;
      rays[1 * n_rays + i] = 0.0;
      rays[2 * n_rays + i] = 0.0;
      rays[3 * n_rays + i] = 0.0;
      rays[4 * n_rays + i] = 1.0;
      rays[5 * n_rays + i] = norm * tx / len;
      rays[6 * n_rays + i] = norm * ty / len;
      rays[7 * n_rays + i] = norm * 1.0 / len;
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Fixed-step classical RK4 (Sec. 3.4) in z between the schedule's nodes.   */
/* All four stages of step s use the particle set step_set[s].               */
/* Flags: 1 non-finite state, 2 kz <= 0 (the ray turned back), 4 |phi|/a >   */
/* 1e-2 (outside the weak-field regime of Sec. 3.2).  A ray whose step ends  */
/* non-finite or with kz <= 0 keeps its last good state and stops.           */
/* ------------------------------------------------------------------------ */
static void field_at(const or_cosmo* c, const or_field* f, int32_t S, double x, double y, double z, double* phi,
                     double g[3]) {
  if (S < 0) {
    *phi = 0.0;
    g[0] = g[1] = g[2] = 0.0;
    return;
  }
  double p[3] = {x, y, z};
  or_field_at(c, &f->sets[S], p, phi, g);
}

static uint8_t trace_one(const or_cosmo* c, const or_field* f, int32_t sb, int32_t se, double st[8]) {
  double Y[7] = {st[0], st[1], st[2], st[4], st[5], st[6], st[7]};
  double z = st[3];
  uint8_t flag = 0;
  for (int32_t s = sb; s < se; ++s) {
    double Z0 = f->z_nodes[s], Z1 = f->z_nodes[s + 1], h = Z1 - Z0;
    int32_t S = f->step_set[s];
    double k1[7], k2[7], k3[7], k4[7], Yt[7], phi, g[3], a, adot;
    field_at(c, f, S, Y[1], Y[2], Z0, &phi, g);
    or_scale_factor(c, Y[0], &a, &adot);
    if (fabs(phi) / a > 1e-2) flag |= 4;
    or_derivs(c, Y, phi, g, k1);
    for (int i = 0; i < 7; ++i) Yt[i] = Y[i] + 0.5 * h * k1[i];
    field_at(c, f, S, Yt[1], Yt[2], Z0 + 0.5 * h, &phi, g);
    or_derivs(c, Yt, phi, g, k2);
    for (int i = 0; i < 7; ++i) Yt[i] = Y[i] + 0.5 * h * k2[i];
    field_at(c, f, S, Yt[1], Yt[2], Z0 + 0.5 * h, &phi, g);
    or_derivs(c, Yt, phi, g, k3);
    for (int i = 0; i < 7; ++i) Yt[i] = Y[i] + h * k3[i];
    field_at(c, f, S, Yt[1], Yt[2], Z1, &phi, g);
    or_derivs(c, Yt, phi, g, k4);
    double Yn[7];
    int finite = 1;
    for (int i = 0; i < 7; ++i) {
      Yn[i] = Y[i] + h / 6.0 * (k1[i] + 2.0 * k2[i] + 2.0 * k3[i] + k4[i]);
      if (!isfinite(Yn[i])) finite = 0;
    }
    if (!finite) { flag |= 1; break; }
    if (!(Yn[6] > 0.0)) { flag |= 2; break; }
    memcpy(Y, Yn, sizeof(Y));
    z = Z1;
  }
  st[0] = Y[0]; st[1] = Y[1]; st[2] = Y[2]; st[3] = z;
  st[4] = Y[3]; st[5] = Y[4]; st[6] = Y[5]; st[7] = Y[6];
  return flag;
}

int or_trace(const or_cosmo* c, const or_field* fields, int32_t n_fields, int32_t step_begin, int32_t step_end,
             int64_t n_rays, double* rays, uint8_t* flags, int32_t n_threads) {
#ifdef _OPENMP
  if (n_threads > 0) omp_set_num_threads(n_threads);
#else
  (void)n_threads;
#endif
  for (int32_t fi = 0; fi < n_fields; ++fi) {
    const or_field* f = &fields[fi];
    int32_t sb = step_begin < 0 ? 0 : step_begin;
    int32_t se = step_end > f->n_steps ? f->n_steps : step_end;
    int64_t r0 = 9 * f->bundle_offset, r1 = 9 * (f->bundle_offset + f->n_bundles);
#pragma omp parallel for schedule(dynamic, 1)
    for (int64_t i = r0; i < r1; ++i) {
      double st[8];
      for (int cc = 0; cc < 8; ++cc) st[cc] = rays[cc * n_rays + i];
      uint8_t fl = trace_one(c, f, sb, se, st);
      for (int cc = 0; cc < 8; ++cc) rays[cc * n_rays + i] = st[cc];
      if (flags) flags[i] |= fl;
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Magnification from the bundle at the source plane (Sec. 3.1 and      */
/* eq. lensmap, magnification).  Offsets D_k = x_k - x_anchor at z = chi_s.  */
/* mu = (area of the homogeneous octagon) / (signed area of the traced one); */
/* the Jacobian is the least-squares linear map from the ring offsets u_k    */
/* (radians) to D_k / chi_s:  A = sum_k D_k u_k^T / (4 r_b^2 chi_s).          */
/* jac[0..3][b] = kappa, gamma1, gamma2, omega.                              */
/* ------------------------------------------------------------------------ */
int or_magnification(double chi_s, int64_t n_bundles, double radius, const double* rays, double* mu, double* jac) {
  int64_t n_rays = 9 * n_bundles;
  const double* X = rays + 1 * n_rays;
  const double* Yv = rays + 2 * n_rays;
  double area_hom = 0.0;
  for (int k = 0; k < 8; ++k) {
    int kn = (k + 1) % 8;
    area_hom += 0.5 * (RING_C[k] * RING_S[kn] - RING_S[k] * RING_C[kn]);
  }
  area_hom *= radius * radius * chi_s * chi_s;
  for (int64_t b = 0; b < n_bundles; ++b) {
    double dx[8], dy[8];
    for (int k = 0; k < 8; ++k) {
      dx[k] = X[9 * b + 1 + k] - X[9 * b];
      dy[k] = Yv[9 * b + 1 + k] - Yv[9 * b];
    }
    double area = 0.0;
    for (int k = 0; k < 8; ++k) {
      int kn = (k + 1) % 8;
      area += 0.5 * (dx[k] * dy[kn] - dy[k] * dx[kn]);
    }
    mu[b] = area_hom / area;
    if (jac) {
      double a11 = 0, a12 = 0, a21 = 0, a22 = 0;
      for (int k = 0; k < 8; ++k) {
        double ux = radius * RING_C[k], uy = radius * RING_S[k];
        a11 += dx[k] * ux;
        a12 += dx[k] * uy;
        a21 += dy[k] * ux;
        a22 += dy[k] * uy;
      }
      double nrm = 4.0 * radius * radius * chi_s;
      a11 /= nrm; a12 /= nrm; a21 /= nrm; a22 /= nrm;
      jac[0 * n_bundles + b] = 1.0 - 0.5 * (a11 + a22);
      jac[1 * n_bundles + b] = 0.5 * (a22 - a11);
      jac[2 * n_bundles + b] = -0.5 * (a12 + a21);
      jac[3 * n_bundles + b] = 0.5 * (a21 - a12);
    }
  }
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Source-weighted magnification PDF (Sec. 5.3, eq. weighthisto): each       */
/* bundle with mu > 0 has weight 1/mu; bins are uniform in log10 mu over     */
/* [log_lo, log_hi]; P_i = sum_{b in i} w_b / (sum_b w_b * width_i) with     */
/* width_i the bin width in mu.  moments = {sum w, <mu>_w, sigma_w,          */
/* n(mu <= 0), n below range, n above range}.                                */
/* ------------------------------------------------------------------------ */
int or_mu_histogram(int64_t n, const double* mu, int32_t n_bins, double log_lo, double log_hi, double* pdf,
                    double* moments) {
  if (n_bins < 1 || !(log_hi > log_lo)) return -1;
  double* acc = (double*)calloc((size_t)n_bins, sizeof(double));
  double sw = 0.0, swm = 0.0;
  double n_bad = 0, n_under = 0, n_over = 0;
  for (int64_t b = 0; b < n; ++b) {
    double m = mu[b];
    if (!(m > 0.0)) { n_bad += 1; continue; }
    double w = 1.0 / m;
    sw += w;
    swm += w * m;
    double lm = log10(m);
    if (lm < log_lo) { n_under += 1; continue; }
    if (lm >= log_hi) { n_over += 1; continue; }
    int32_t i = (int32_t)floor((lm - log_lo) / (log_hi - log_lo) * n_bins);
    if (i >= n_bins) i = n_bins - 1;
    acc[i] += w;
  }
  double mean = sw > 0 ? swm / sw : 0.0;
  double var = 0.0;
  for (int64_t b = 0; b < n; ++b) {
    double m = mu[b];
    if (!(m > 0.0)) continue;
    var += (1.0 / m) * (m - mean) * (m - mean);
  }
  for (int32_t i = 0; i < n_bins; ++i) {
    double e0 = log_lo + (log_hi - log_lo) * i / n_bins, e1 = log_lo + (log_hi - log_lo) * (i + 1) / n_bins;
    double width = pow(10.0, e1) - pow(10.0, e0);
    pdf[i] = sw > 0 ? acc[i] / (sw * width) : 0.0;
  }
  moments[0] = sw;
  moments[1] = mean;
  moments[2] = sw > 0 ? sqrt(var / sw) : 0.0;
  moments[3] = n_bad;
  moments[4] = n_under;
  moments[5] = n_over;
  free(acc);
  return 0;
}

/* ------------------------------------------------------------------------ */
/* Source-weighted shear PDF (Sec. 5.4, the shear distribution that the     */
/* paper compares between methods; Sec. 5.3 weights every bundle statistic */
/* by 1/mu).  |gamma| = hypot(gamma1, gamma2) from the Jacobian; bins       */
/* uniform in |gamma| over [lo, hi); pdf_i = sum_{b in i} w_b / (sum w dg). */
/* moments = {sum w, <|gamma|>_w, sigma_w, n(mu <= 0), n below, n above}.   */
/* ------------------------------------------------------------------------ */
int or_shear_histogram(int64_t n, const double* mu, const double* jac, int32_t n_bins, double lo, double hi,
                       double* pdf, double* moments) {
  if (n_bins < 1 || !(hi > lo)) return -1;
  double* acc = (double*)calloc((size_t)n_bins, sizeof(double));
  double sw = 0.0, swg = 0.0, n_bad = 0, n_under = 0, n_over = 0;
  for (int64_t b = 0; b < n; ++b) {
    if (!(mu[b] > 0.0)) { n_bad += 1; continue; }
    double w = 1.0 / mu[b];
    double gm = hypot(jac[1 * n + b], jac[2 * n + b]);
    sw += w;
    swg += w * gm;
    if (gm < lo) { n_under += 1; continue; }
    if (gm >= hi) { n_over += 1; continue; }
    int32_t i = (int32_t)floor((gm - lo) / (hi - lo) * n_bins);
    if (i >= n_bins) i = n_bins - 1;
    acc[i] += w;
  }
  double mean = sw > 0 ? swg / sw : 0.0;
  double var = 0.0;
  for (int64_t b = 0; b < n; ++b) {
    if (!(mu[b] > 0.0)) continue;
    double gm = hypot(jac[1 * n + b], jac[2 * n + b]);
    var += (1.0 / mu[b]) * (gm - mean) * (gm - mean);
  }
  double width = (hi - lo) / n_bins;
  for (int32_t i = 0; i < n_bins; ++i) pdf[i] = sw > 0 ? acc[i] / (sw * width) : 0.0;
  moments[0] = sw;
  moments[1] = mean;
  moments[2] = sw > 0 ? sqrt(var / sw) : 0.0;
  moments[3] = n_bad;
  moments[4] = n_under;
  moments[5] = n_over;
  free(acc);
  return 0;
}
