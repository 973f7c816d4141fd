/*
 * Plain FP64 CPU oracle for three-dimensional ray-bundle lensing through a
 * weakly perturbed flat FLRW metric (Killedar, Lasky, Lewis & Fluke 2011).
 *
 * TEST INFRASTRUCTURE ONLY.  Only the test-suite, the smoke check and the
 * CPU-baseline leg of the benchmark may load this library.  The product
 * library never links, loads or calls it, and shares no code with it.
 *
 * Units: comoving Mpc for lengths, c = 1 (times in Mpc), masses in Msun.
 * Ray state, per ray, is 8 doubles: t (lookback time), x, y, z (comoving),
 * kt, kx, ky, kz (derivatives with respect to the affine parameter).
 * Arrays of rays are structure-of-arrays: rays[c * n_rays + i], c = 0..7.
 * A bundle b owns rays 9b (anchor) and 9b+1 .. 9b+8 (ring, counter-clockwise
 * from +x).
 */
#ifndef RT_ORACLE_H
#define RT_ORACLE_H
#include <stdint.h>

typedef struct { double omega_m, omega_lambda, h; } or_cosmo;

typedef struct {
  int64_t n;                /* number of point masses                        */
  const double* x;          /* [n] comoving Mpc, observer frame              */
  const double* y;
  const double* z;
  const double* m;          /* [n] Msun                                      */
  double softening;         /* Plummer softening, comoving Mpc               */
  int32_t background;       /* 1: subtract a uniform cuboid at the mean density */
  double lo[3], hi[3];      /* the cuboid, comoving Mpc                      */
} or_set;

typedef struct {
  int32_t n_sets; const or_set* sets;
  int32_t n_steps; const double* z_nodes;   /* [n_steps + 1]                 */
  const int32_t* step_set;                  /* [n_steps], -1 = no field      */
  int64_t bundle_offset, n_bundles;
} or_field;

/* constants */
double or_G_over_c2(void);                  /* Mpc / Msun                    */
double or_H0(const or_cosmo* c);            /* Mpc^-1                        */
double or_rho_crit0(const or_cosmo* c);     /* Msun / Mpc^3                  */

/* background cosmology */
double or_E(const or_cosmo* c, double z);
double or_comoving_distance(const or_cosmo* c, double z);
double or_empty_beam_distance(const or_cosmo* c, double z);
double or_t0(const or_cosmo* c);
void   or_scale_factor(const or_cosmo* c, double t, double* a, double* adot);

/* field of one particle set at a point */
void or_prism(const double lo[3], const double hi[3], const double p[3], double* U, double gradU[3]);
void or_field_at(const or_cosmo* c, const or_set* s, const double p[3], double* phi, double grad[3]);

/* derivative of Y = (t, x, y, kt, kx, ky, kz) with respect to z */
void or_derivs(const or_cosmo* c, const double Y[7], double phi, const double g[3], double dY[7]);
void or_accel(const or_cosmo* c, double t, const double k[4], double phi, const double g[3], double A[4]);

/* schedule and replica selection */
int or_make_schedule(double chi_s, double z_lo, double z_hi, int32_t n_fine, double q,
                     double* nodes, int32_t capacity, int32_t* n_steps);
int or_replica_step_sets(const double* nodes, int32_t n_steps, double box, int32_t n_replicas, int32_t* step_set);

/* the hot path */
int or_build_bundles(const or_cosmo* c, const or_field* fields, int32_t n_fields, int64_t n_bundles,
                     const double* theta, double radius, double* rays);
int or_trace(const or_cosmo* c, const or_field* fields, int32_t n_fields, int32_t step_begin, int32_t step_end,
             int64_t n_rays, double* rays, uint8_t* flags, int32_t n_threads);
int or_magnification(double chi_s, int64_t n_bundles, double radius, const double* rays, double* mu, double* jac);
int or_mu_histogram(int64_t n, const double* mu, int32_t n_bins, double log_lo, double log_hi,
                    double* pdf, double* moments);
int or_shear_histogram(int64_t n, const double* mu, const double* jac, int32_t n_bins, double lo, double hi,
                       double* pdf, double* moments);

#endif
