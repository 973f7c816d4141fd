/*
 * rt.h -- C ABI of the MI355X ray-bundle lensing library (librt.so).
 *
 * Method: Killedar, Lasky, Lewis & Fluke (2011), "Gravitational lensing with
 * three-dimensional ray tracing".  Bundles of one central ("anchor") ray and
 * 8 ring rays (Sec. 3.1) are integrated along null geodesics (Sec. 3.4,
 * eq. geodesiceqn) of the weakly perturbed flat FLRW metric (Sec. 3.2,
 * eq. expandingmetric, phicotophys), with the comoving potential of Plummer-
 * softened point masses (Sec. 3.3, eq. psi, derivs) summed directly at every
 * RK4 stage.  The distorted area of each bundle at the source plane gives the
 * magnification mu (Sec. 3.1, eq. magnification), and the source-weighted mu
 * histogram (Sec. 5.3, eq. weighthisto) gives the muPDF.
 *
 * Conventions shared by all calls
 *   Units: comoving Mpc for lengths, c = 1 so times are in Mpc, masses in Msun.
 *   Cosmology: flat Lemaitre model, Omega_m + Omega_Lambda = 1 (Sec. 3.5).
 *   Ray state: 8 doubles per ray, t (lookback time), x, y, z (comoving, z along
 *     the line of sight), kt, kx, ky, kz (derivatives with respect to the affine
 *     parameter).  Arrays of rays are structure-of-arrays [8][n_rays], element
 *     (c, i) at rays[c * n_rays + i], with n_rays = 9 * n_bundles.  Bundle b owns
 *     rays 9b (anchor) and 9b+1 .. 9b+8 (ring, at angles pi k / 4 counter-
 *     clockwise from +x).
 *   Memory: every array is owned by the caller and is never freed by the library.
 *     "device" arrays live in HBM of the current HIP device; "host" arrays in
 *     host memory.  The library owns only its caches (FP32 particle copies,
 *     device descriptor tables, captured graphs, tuned plans), released by
 *     rt_release_caches().
 *   Streams: work is enqueued on `stream`; calls return once it is enqueued.
 *     Argument errors are detected on the host and returned synchronously
 *     without enqueuing anything.  Errors of earlier asynchronous work surface
 *     as RT_ERR_DEVICE from a later call.
 *   Errors: every call returns an rt_status; on failure rt_last_error() gives a
 *     message for the calling thread that names the offending argument.
 */
#ifndef RT_H
#define RT_H

#include <stdint.h>
#include <hip/hip_runtime_api.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef enum rt_status {
  RT_OK = 0,
  RT_ERR_INVALID_ARG = -1,   /* null pointer, bad size, bad range                 */
  RT_ERR_COSMOLOGY = -2,     /* not flat, h <= 0, Omega_m <= 0, Omega_Lambda <= 0  */
  RT_ERR_NONFINITE = -3,     /* NaN or Inf in a host argument                      */
  RT_ERR_SCHEDULE = -4,      /* nodes not strictly increasing from 0 to chi_s      */
  RT_ERR_OUT_OF_MEMORY = -5, /* a library cache could not be allocated             */
  RT_ERR_DEVICE = -6,        /* a HIP call failed (including earlier async work)   */
  RT_ERR_UNSUPPORTED = -7    /* valid request the library does not implement       */
} rt_status;

typedef enum rt_precision {
  RT_FP64 = 0,       /* field sum, integration and bundle areas in FP64                   */
  RT_FP32_KAHAN = 1  /* pair terms in FP32 with compensated (Kahan) accumulation across
                        particle tiles; integration and bundle areas in FP64           */
} rt_precision;

/* Flat cosmology of Sec. 3.5: |omega_m + omega_lambda - 1| <= 1e-12, h = H0 / (100 km/s/Mpc). */
typedef struct rt_cosmology {
  double omega_m, omega_lambda, h;
} rt_cosmology;

/* One lens volume (a halo, a group of point masses, or one box replica). */
typedef struct rt_particle_set {
  int64_t n;               /* number of particles, >= 0                                          */
  const double* xyzm;      /* device, [4][n]: x, y, z (comoving Mpc, observer frame, line of sight
                              along +z), then masses (Msun, > 0).  May be NULL when n == 0.      */
  double softening;        /* Plummer softening length, comoving Mpc, >= 0                        */
  int32_t background;      /* 1: subtract the field of a uniform cuboid [lo, hi] at the mean matter
                              density Omega_m rho_c0 (Sec. 3.3, eq. perturbation, meanmatterdens);
                              0: isolated lens, no subtraction                                   */
  double lo[3], hi[3];     /* the cuboid (used when background == 1), lo < hi componentwise      */
} rt_particle_set;

/* One independent lens field (one line-of-sight configuration) and its bundles. */
typedef struct rt_field {
  int32_t n_sets;                 /* number of particle sets, >= 0                          */
  const rt_particle_set* sets;    /* host [n_sets]                                          */
  int32_t n_steps;                /* RK4 steps, >= 1                                        */
  const double* z_nodes;          /* host [n_steps + 1]: 0 = z_0 < z_1 < ... < z_n = chi_s  */
  const int32_t* step_set;        /* host [n_steps]: set used by all four stages of step s,
                                     -1 for no mass                                          */
  int64_t bundle_offset;          /* first bundle of this field in the global bundle array  */
  int64_t n_bundles;              /* bundles of this field; field slices must not overlap   */
} rt_field;

/* ---------------------------------------------------------------- background and schedule */

/* Comoving distance D_C(z) = int_0^z dz' / H(z') with c = 1 (Sec. 5.1, eq. raytracedistance).
 * chi_out: host, receives Mpc.  Errors: RT_ERR_COSMOLOGY, RT_ERR_INVALID_ARG (z < 0). */
rt_status rt_comoving_distance(const rt_cosmology* cosmo, double z, double* chi_out);

/* RK4 nodes in z (Sec. 3.4 fixes the step; the nodes make it explicit): n_fine equal steps on
 * [z_lo, z_hi]; outside it steps grow geometrically by q >= 1 toward 0 and chi_s, a last step
 * shorter than half its nominal length being merged into its neighbour.  Requires
 * 0 <= z_lo < z_hi <= chi_s.  nodes: host [capacity]; n_steps: host, number of steps written
 * (nodes holds n_steps + 1 values).  Errors: RT_ERR_INVALID_ARG (including capacity too small). */
rt_status rt_make_schedule(double chi_s, double z_lo, double z_hi, int32_t n_fine, double q,
                           double* nodes, int32_t capacity, int32_t* n_steps);

/* Box replicas stacked along the line of sight, replica r covering z in [r box, (r+1) box)
 * (Sec. 5.1-5.2): step s uses the replica containing its midpoint, clamped to
 * [0, n_replicas - 1]; a midpoint on a boundary goes to the farther replica.
 * nodes: host [n_steps + 1]; step_set: host [n_steps] output. */
rt_status rt_replica_step_sets(const double* nodes, int32_t n_steps, double box, int32_t n_replicas,
                               int32_t* step_set);

/* ---------------------------------------------------------------- the hot path */

/* Initial state of every ray (Sec. 3.1, 3.4): anchor direction theta (gnomonic, so that
 * straight rays reach z = chi_s at theta * chi_s), ring rays at theta + radius (cos pi k/4,
 * sin pi k/4); t = x = y = z = 0, kt = 1, (kx, ky, kz) = n sqrt(E0 / F0) with
 * E0 = 1 + 2 phi_obs, F0 = 1 - 2 phi_obs so that the wave vector is exactly null, phi_obs
 * being the potential at the observer of the field's step-0 set (0 for bundles outside every
 * field or when that step has no set).
 * theta: device [2][n_bundles] radians; rays: device [8][9 n_bundles] output.
 * fields: host [n_fields] (may be NULL when n_fields == 0).  radius: radians, 0 < radius < 1e-2. */
rt_status rt_build_bundles(const rt_cosmology* cosmo, const rt_field* fields, int32_t n_fields,
                           int64_t n_bundles, const double* theta, double radius, double* rays,
                           hipStream_t stream);

/* Integrate every ray of every field with fixed-step classical RK4 in z (Sec. 3.4, eq.
 * geodesiceqn with x^3 as the independent variable) over steps [step_begin, step_end) of
 * each field's schedule (clamped to [0, n_steps]); a ray must stand at z_nodes[step_begin].
 * Field at each stage: direct sum over the step's particle set plus the optional cuboid
 * background; Christoffel symbols differentiated exactly from eq. expandingmetric.
 * All fields are traced in one persistent launch with a work queue, captured once in a HIP
 * graph and replayed while the arguments stay the same (the 24 most recent configurations are
 * kept); launches of one such configuration on different streams are ordered one after the
 * other (they share its FP32 copies and queue).  When `stream` is being captured, the launch
 * becomes part of the caller's graph and the configuration's buffers are kept until
 * rt_release_caches (which the caller must not call while such a graph may still run); the
 * ordering between streams is then the caller's.
 * RT_FP32_KAHAN: each (bundle, particle) pair is evaluated once for the bundle's nine rays, in
 * FP32, at the bundle's expansion point (its anchor rounded to FP32): the pair's potential, field
 * and their first and second derivatives with respect to the point (20 moments, Kahan-summed
 * over tiles); each ray assembles its field in FP64 from the moments and its own offset (Sec.
 * 3.1: the ring-minus-anchor differences keep FP32 relative precision).  Pairs closer than 1024
 * times the bundle's largest ray offset are summed per ray directly in FP64; the truncation of
 * the expansion stays below 6e-6 of each pair's ring difference.  Particle positions are held as
 * two FP32 parts.  A set whose masses are all equal (checked on the device at every call) skips
 * the per-pair mass product.  Sets of at most 63 particles (point lenses) are summed per ray
 * directly in FP64.
 * rays: device [8][9 n_bundles], updated in place.  ray_flags: device [9 n_bundles] or NULL;
 * bits are OR-ed in: 1 non-finite state, 2 kz <= 0 (ray turned back), 4 |phi|/a > 1e-2 (outside
 * the weak-field regime of Sec. 3.2).  A ray with flag 1 or 2 keeps its last good state.
 * The last node of every field must equal chi_s = rt_comoving_distance(z_source) to 1e-9. */
rt_status rt_trace(const rt_cosmology* cosmo, double z_source, const rt_field* fields, int32_t n_fields,
                   rt_precision precision, int32_t step_begin, int32_t step_end, int64_t n_bundles,
                   double* rays, uint8_t* ray_flags, hipStream_t stream);

/* Magnification and Jacobian of each bundle at z = chi_s (Sec. 3.1, eq. lensmap, magnification):
 * offsets D_k = x_k - x_anchor (FP64); mu = (homogeneous octagon area chi_s^2 2 sqrt(2) r^2) /
 * (signed shoelace area of the traced octagon), negative for parity-flipped images;
 * Jacobian = least-squares linear map of the ring offsets: A = sum_k D_k u_k^T / (4 r^2 chi_s).
 * rays: device [8][9 n_bundles]; mu: device [n_bundles]; jac: device [4][n_bundles] (kappa,
 * gamma1, gamma2, omega) or NULL.  radius: the radius given to rt_build_bundles. */
rt_status rt_magnification(const rt_cosmology* cosmo, double z_source, int64_t n_bundles, double radius,
                           const double* rays, double* mu, double* jac, hipStream_t stream);

/* Source-weighted magnification PDF (Sec. 5.3, eq. weighthisto): weights 1/mu for mu > 0; n_bins
 * bins uniform in log10 mu over [log_lo, log_hi); pdf_i = sum_{b in i} w_b / (sum_b w_b width_i)
 * with width_i the bin width in mu.  mu: device [n]; pdf: device [n_bins];
 * moments: device [6] = sum w, <mu>_w, sigma_w, n(mu <= 0), n below, n above the range. */
rt_status rt_mu_histogram(int64_t n, const double* mu, int32_t n_bins, double log_lo, double log_hi,
                          double* pdf, double* moments, hipStream_t stream);

/* Flexion of each bundle at z = chi_s (Sec. 6: flexion, the gradient of the shear, is the
 * third-order lensing effect that ray bundles can carry).  With the ring offsets
 * D_k = x_k - x_anchor = chi_s (r A e_k + 1/2 r^2 Dm(e_k, e_k)) + O(r^3), e_k = (cos 2 pi k / 8,
 * sin 2 pi k / 8), Dm_ijl = d A_ij / d theta_l is read from the ring's harmonics 0 and 2 (the
 * first- and third-order parts fall in harmonics 1 and 3): the least-squares second-order fit of
 * the ring.  flex: device [4][n_bundles] = F1, F2 (F = grad kappa), G1, G2 (G = d gamma with
 * d = d1 + i d2: d1 gamma1 - d2 gamma2, d2 gamma1 + d1 gamma2), in rad^-1, kappa and gamma read
 * from A as in rt_magnification; dm: device [6][n_bundles] = Dm_111, Dm_112, Dm_122, Dm_211,
 * Dm_212, Dm_222 (rad^-1), or NULL.  For a lens potential psi, Dm_ijl = -psi_ijl.  The second-
 * order part is r / theta_lens of the ring offsets: pick the bundle radius (rt_build_bundles) so
 * that it stays well above the trace's error on the offsets.  rays: device [8][9 n_bundles];
 * radius: the radius given to rt_build_bundles. */
rt_status rt_flexion(const rt_cosmology* cosmo, double z_source, int64_t n_bundles, double radius, const double* rays,
                     double* flex, double* dm, hipStream_t stream);

/* rt_mu_histogram for callers that cannot allocate device memory (code under HIP graph capture,
 * tight serving loops, harnesses that forbid hipMalloc): the same kernels and results, with the
 * per-call scratch (the bin weights and five sums) in a static per-device array of the library
 * instead of a stream-ordered allocation.  It calls no allocating routine.  n_bins <= 65536
 * (RT_ERR_INVALID_ARG beyond).  Every call on one GPU shares that GPU's array (512 KB, held
 * until the process ends): calls that overlap on one GPU (on different streams) race. */
rt_status rt_mu_histogram_noalloc(int64_t n, const double* mu, int32_t n_bins, double log_lo, double log_hi,
                                  double* pdf, double* moments, hipStream_t stream);

/* Source-weighted shear PDF (the shear distribution of Sec. 5.4, weighted like eq. weighthisto):
 * |gamma| = hypot(gamma1, gamma2) from rt_magnification's Jacobian, weight 1/mu for mu > 0,
 * n_bins bins uniform in |gamma| over [lo, hi); pdf_i = sum_{b in i} w_b / (sum_b w_b dgamma).
 * mu: device [n]; jac: device [4][n]; pdf: device [n_bins]; moments: device [6] = sum w,
 * <|gamma|>_w, sigma_w, n(mu <= 0), n below, n above the range. */
rt_status rt_shear_histogram(int64_t n, const double* mu, const double* jac, int32_t n_bins, double lo, double hi,
                             double* pdf, double* moments, hipStream_t stream);

/* The field kernel alone (Sec. 3.3): phi and grad phi of one particle set at n points, with the
 * same arithmetic rt_trace uses for the given precision.  points: device [3][n];
 * phi: device [n]; grad: device [3][n]. */
rt_status rt_field_eval(const rt_cosmology* cosmo, const rt_particle_set* set, rt_precision precision,
                        int64_t n, const double* points, double* phi, double* grad, hipStream_t stream);

/* ---------------------------------------------------------------- particle-mesh field */

/* The paper's own field representation (Sec. 3.3, App. B) for one particle set: the masses are
 * assigned to the nodes of a cubic grid by Cloud-in-Cell, and phi and its three derivatives at
 * the nodes come from FFTs.
 *   Isolated grid (periodic = 0): convolution with the Plummer kernels of eq. psi and eq. derivs on
 *   the grid zero-padded to (2n)^3 (the exact linear convolution of the node masses; with
 *   softening 0 a node's own mass is left out); App. B's interpolation gives the field anywhere
 *   inside the nodes, zero outside.
 *   Periodic grid (periodic = 1): the n^3 nodes tile a box of side n h and the deposit wraps;
 *   phi_k = -4 pi (G/c^2) rho_k / k^2 (continuum Green's function, k = 0 removed, so the box's mean
 *   density is subtracted; no softening beyond the mesh) and dphi/dx_j = i k_j phi_k; the x^3
 *   spline is periodic and App. B's windows wrap, so every point of space has a field. */
typedef struct rt_pm_grid {
  int32_t n;          /* nodes per side, a power of two, 4 <= n <= 512                          */
  double origin[3];   /* position of node (0, 0, 0), comoving Mpc; node (i, j, k) sits at
                         origin + h (i, j, k)                                                    */
  double h;           /* node spacing, comoving Mpc, > 0                                        */
  int32_t periodic;   /* 0: isolated lens, 1: periodic box                                      */
} rt_pm_grid;

/* Workspace rt_pm_build needs: two M^3 complex FP64 grids plus M/2 twiddles, 32 M^3 + 8 M bytes,
 * with M = 2n for an isolated grid (4.3 GB for n = 256) and M = n for a periodic one.
 * bytes: host.  Errors: RT_ERR_INVALID_ARG for a bad grid. */
rt_status rt_pm_workspace_bytes(const rt_pm_grid* grid, size_t* bytes);

/* Build the field of `set` on `grid`.  set: as for rt_trace; on an isolated grid background
 * must be 0 and particles whose cloud leaves the nodes lose that part of their mass; on a
 * periodic grid the background flag is ignored (the mean is removed by construction) and every
 * particle is wrapped into the box.  fields: device [8][n^3] output; grid q < 4 is phi,
 * dphi/dx, dphi/dy, dphi/dz (Mpc^0 and Mpc^-1, c = 1) and grid q + 4 its natural-spline second
 * derivatives along z (App. B), node (i, j, k) at (i n + j) n + k.  workspace: device, at least
 * rt_pm_workspace_bytes; contents are scratch.  The node masses are accumulated with FP64
 * atomics, so the last bits of the result may vary between calls. */
rt_status rt_pm_build(const rt_particle_set* set, const rt_pm_grid* grid, double* fields, void* workspace,
                      size_t workspace_bytes, hipStream_t stream);

/* App. B interpolation of a built field at n points: n_int nodes on each side of the point
 * (1 <= n_int <= 4, n >= 2 n_int).  points: device [3][n]; phi: device [n]; grad: device [3][n]. */
rt_status rt_pm_eval(const rt_pm_grid* grid, const double* fields, int32_t n_int, int64_t n, const double* points,
                     double* phi, double* grad, hipStream_t stream);

/* rt_trace with the field of built grids in place of the direct sum: the same RK4 in z over
 * z_nodes (host [n_steps + 1], 0 to chi_s), the same Christoffel contraction, exit and flags;
 * all four stages of step s use grid step_grid[s] (host [n_steps], -1 = no field; NULL = grid 0
 * at every step), as the direct path uses a particle set per step: one isolated grid for a lens,
 * one periodic grid per box replica for a light cone.  grids: host [n_grids]; fields: host
 * [n_grids] of device pointers to built fields; n_int as for rt_pm_eval (valid for every grid).
 * An isolated grid must leave the observer (0, 0, 0) outside its nodes, so that its potential
 * there is the 0 used by bundles built with no mass at step 0; for periodic grids the caller
 * builds the bundles with the potential it wants at the observer (e.g. rt_build_bundles over the
 * same particle sets).  rays: device [8][9 n_bundles], in and out; ray_flags: device
 * [9 n_bundles] or NULL. */
rt_status rt_trace_pm(const rt_cosmology* cosmo, double z_source, int32_t n_grids, const rt_pm_grid* grids,
                      const double* const* fields, int32_t n_int, int32_t n_steps, const double* z_nodes,
                      const int32_t* step_grid, int32_t step_begin, int32_t step_end, int64_t n_bundles,
                      double* rays, uint8_t* ray_flags, hipStream_t stream);

/* The paper's own integrator (Sec. 3.4, eq. RKstepsize) through a built grid: classical RK4 in
 * the affine parameter with the fixed step d_lambda = f_rk h / kz_0 per ray (h = grid.h, the
 * L_box / n_FFT of the paper; kz_0 = the ray's kz on entry), repeated until z reaches chi_s;
 * the step that overshoots is replaced by the linear interpolation between the previous and
 * the current state at z = chi_s (all eight components).  A ray that has not reached chi_s
 * after max_steps keeps its last state and is flagged 8.  f_rk > 0, max_steps >= 1; the grid
 * gives the field everywhere; an isolated one must leave the observer outside its nodes, and for
 * a periodic one the caller builds the bundles with the potential it wants at the observer, as
 * for rt_trace_pm.  rays: device [8][9 n_bundles], in and
 * out (z on entry < chi_s); ray_flags: device [9 n_bundles] or NULL (1, 2, 4 as for rt_trace,
 * 8 as above); ray_steps: device int32 [9 n_bundles] or NULL, steps taken per ray. */
rt_status rt_trace_pm_lambda(const rt_cosmology* cosmo, double z_source, const rt_pm_grid* grid,
                             const double* fields, int32_t n_int, double f_rk, int32_t max_steps, int64_t n_bundles,
                             double* rays, uint8_t* ray_flags, int32_t* ray_steps, hipStream_t stream);

/* rt_trace_pm_lambda through a stack of grids along the line of sight (Sec. 5.2: the space
 * between observer and source filled by cubes, each with its own Fourier grid; Sec. 3.4,
 * eq. RKstepsize for the integrator).  Every field evaluation looks up the slab that holds its
 * own x^3: slab k = [slab_bounds[k], slab_bounds[k + 1]) takes grid slab_grid[k] (-1 = no
 * field); a point outside [slab_bounds[0], slab_bounds[n_slabs]) sees no field.  The fixed step
 * is f_rk h / kz_0 with the grids' common spacing h (all grids must have the same h).
 * grids: host [n_grids]; fields: host [n_grids] of device pointers to built fields; n_int as for
 * rt_pm_eval (valid for every grid); slab_bounds: host [n_slabs + 1], finite, strictly
 * increasing; slab_grid: host int32 [n_slabs], each in [-1, n_grids).  Isolated grids must
 * leave the observer outside their nodes.  The host tables are copied to a device buffer that
 * the call allocates and frees on the stream (the call waits for the copies).  Rays, flags,
 * steps, f_rk and max_steps as for rt_trace_pm_lambda. */
rt_status rt_trace_pm_lambda_slabs(const rt_cosmology* cosmo, double z_source, int32_t n_grids,
                                   const rt_pm_grid* grids, const double* const* fields, int32_t n_int,
                                   int32_t n_slabs, const double* slab_bounds, const int32_t* slab_grid, double f_rk,
                                   int32_t max_steps, int64_t n_bundles, double* rays, uint8_t* ray_flags,
                                   int32_t* ray_steps, hipStream_t stream);

/* ---------------------------------------------------------------- tuning and introspection */

typedef struct rt_plan_info {
  int32_t waves_per_block;    /* wavefronts in one workgroup                                 */
  int32_t waves_per_group;    /* wavefronts that share 63 rays and split the particles      */
  int32_t tile;               /* particles per LDS tile (staged once per workgroup)          */
  int32_t rays_per_block;     /* 63 * waves_per_block / waves_per_group (7 bundles per group) */
  int32_t waves_per_simd;     /* occupancy the plan is compiled for (registers: 512 / it)    */
} rt_plan_info;

/* Number of compiled trace plans for a precision, and the shape of plan `id`. */
int32_t rt_plan_count(rt_precision precision);
rt_status rt_plan_describe(rt_precision precision, int32_t id, rt_plan_info* info);

/* Force plan `id` for every later rt_trace of this precision (-1 returns to automatic choice). */
rt_status rt_force_plan(rt_precision precision, int32_t id);

/* Cap the number of workgroups of the persistent trace launch (0 = as many as fit on the device).
 * Results do not depend on it: every workgroup drains the same work queue. */
rt_status rt_set_grid_limit(int32_t max_blocks);

/* Time every plan on steps [step_begin, step_begin + n_probe_steps) of the given fields, on a
 * library-owned copy of `rays` (the caller's rays are not modified), and keep the fastest for
 * later rt_trace calls of the same precision and workload class.  best_id: host, or NULL. */
rt_status rt_autotune(const rt_cosmology* cosmo, double z_source, const rt_field* fields, int32_t n_fields,
                      rt_precision precision, int32_t step_begin, int32_t n_probe_steps, int64_t n_bundles,
                      const double* rays, int32_t* best_id, hipStream_t stream);

typedef struct rt_trace_info {
  double kernel_ms;           /* time of the trace kernel of the last rt_trace (HIP events on its
                                 stream; 0 unless timing is enabled)                           */
  double interactions;        /* ray-particle pair terms evaluated: sum over fields of
                                 rays x 4 stages x particles of each step                      */
  int32_t plan_id;            /* plan used                                                     */
  int32_t grid_blocks;        /* workgroups launched (persistent)                             */
  int32_t n_items;            /* work items (field, ray block)                                 */
  int32_t graph_reused;       /* 1 if a captured graph was replayed                            */
} rt_trace_info;

/* Enable (1) or disable (0) HIP-event timing around the trace kernel. */
rt_status rt_enable_timing(int32_t on);
/* Information on the last rt_trace of the calling process; waits for its kernel if timed. */
rt_status rt_last_trace_info(rt_trace_info* info);

/* Wait for all work enqueued on `stream` and report what it left: RT_OK, or RT_ERR_DEVICE with
 * the HIP error of earlier asynchronous work (a fault in a kernel, for instance). */
rt_status rt_sync(hipStream_t stream);

/* Message for the last non-OK status of the calling thread ("" if none). */
const char* rt_last_error(void);

/* Release every library-owned cache (graphs, descriptor tables, FP32 copies, tuned plans). */
void rt_release_caches(void);

#ifdef __cplusplus
}
#endif
#endif /* RT_H */
