// Internal declarations shared by the host API (rt_api.hip) and the gfx950
// kernels (rt_kernels.hip).  Not part of the public ABI.
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>

#include "../../include/rt.h"

namespace rt {

// Background cosmology handed to kernels by value (Sec. 3.5, eq. scalefac2).
struct DevCosmo {
  double H0;        // Mpc^-1 (c = 1)
  double t0;        // lookback time of the big bang, Mpc
  double sqrt_ol;   // sqrt(Omega_Lambda)
  double ratio;     // Omega_m / Omega_Lambda
  double G;         // G / c^2, Mpc / Msun
  double G_rho;     // G / c^2 * Omega_m * rho_c0 (mean-density term), Mpc^-2
};

// One particle set as the kernels see it.
struct DevSet {
  const double* p64;   // caller's [4][n] (x, y, z, m)
  float4* p32;         // library copy, [2][n] float4: (x - org, y - org, z - org, m / mref) rounded to
                       // FP32, then the rounding residuals of the three coordinates (and 0)
  int32_t* equal_mass; // n > 0: 1 when every mass equals mass (set on the device), shared by the sets of one array
  int64_t n;
  double eps2;         // softening^2, FP64
  float eps2f;         // softening^2, FP32
  int32_t background;
  double mass;         // the first particle's mass (filled on the device)
  double mref;         // unit of the FP32 copy's masses: mass, or 1 when that is 0 (filled on the device)
  double org[3];       // frame origin of p32 (filled on the device)
  double lo[3], hi[3]; // background cuboid
};

// One lens field: its rays and the slices of the node / step-set / set tables.
struct DevField {
  int64_t ray_begin, n_rays;
  int32_t n_steps, node_off, step_off, set_off;
};

// One unit of work of the persistent trace kernel: a block of rays of one field.
struct WorkItem {
  int32_t field, block;
};

struct TraceParams {
  DevCosmo cosmo;
  const DevField* fields;
  const DevSet* sets;
  const double* nodes;
  const int32_t* step_set;
  const WorkItem* items;
  int32_t n_items;
  int32_t* queue;
  int32_t step_begin, step_end;
  double* rays;
  int64_t n_rays;
  uint8_t* flags;
};

// Plans of the trace kernel (compile-time shapes).
int plan_count(bool fp64);
rt_plan_info plan_info(bool fp64, int id);
hipError_t plan_occupancy(bool fp64, int id, int* blocks_per_cu);
hipError_t launch_trace(bool fp64, int id, const TraceParams& p, int grid, hipStream_t s);

hipError_t launch_reset_queue(int32_t* q, hipStream_t s);
hipError_t launch_prepare_sets(DevSet* sets, int32_t n_sets, hipStream_t s);
hipError_t launch_convert_set(const DevSet* set_dev, const double* p64, float4* p32, int64_t n, hipStream_t s);
hipError_t launch_bundles(DevCosmo c, const double* phi_obs, int64_t b0, int64_t nb_range, int64_t n_bundles,
                          const double* theta, double radius, double* rays, hipStream_t s);
hipError_t launch_field_eval(DevCosmo c, const DevSet* set, bool fp64, int64_t n, const double* pts, double* phi,
                             double* grad, hipStream_t s);
hipError_t launch_magnification(double chi_s, int64_t nb, double radius, const double* rays, double* mu,
                                double* jac, hipStream_t s);
hipError_t launch_flexion(double chi_s, int64_t nb, double radius, const double* rays, double* flex, double* dm,
                          hipStream_t s);
// The static scratch of rt_mu_histogram_noalloc on the current device (its address is
// looked up once per device) and the largest bin count it holds.
hipError_t noalloc_scratch(double** out, int32_t* max_bins);
hipError_t launch_histogram(int64_t n, const double* mu, const double* jac, int mode, int32_t n_bins, double lo,
                            double hi, double* pdf, double* moments, double* work, hipStream_t s);

// Particle-mesh field (rt_pm.hip).
struct DevPmGrid {
  int32_t n;
  double origin[3];
  double h;
  int32_t periodic;
  const double* fields;   // [8][n^3]
};
int64_t pm_workspace_bytes(int n, int periodic);
hipError_t launch_pm_build(const double* xyzm, int64_t np, double eps, const double origin[3], double h, int n,
                           int periodic, double G, double* fields, void* workspace, hipStream_t s);
hipError_t launch_pm_eval(const double origin[3], double h, int n, int periodic, const double* fields, int n_int,
                          int64_t np, const double* pts, double* phi, double* grad, hipStream_t s);
hipError_t launch_pm_trace(DevCosmo c, const DevPmGrid* grids, const int32_t* step_grid, int n_int,
                           const double* nodes, int32_t step_begin, int32_t step_end, double* rays, int64_t n_rays,
                           uint8_t* flags, hipStream_t s);
hipError_t launch_pm_trace_lambda(DevCosmo c, const double origin[3], double h, int n, int periodic,
                                  const double* fields, int n_int, double chi_s, double f_rk, int32_t max_steps,
                                  double* rays, int64_t n_rays, uint8_t* flags, int32_t* steps, hipStream_t s);
hipError_t launch_pm_trace_lambda_slabs(DevCosmo c, const DevPmGrid* grids, const double* bounds,
                                        const int32_t* slab_grid, int32_t n_slabs, double h_rk, int n_int,
                                        double chi_s, double f_rk, int32_t max_steps, double* rays, int64_t n_rays,
                                        uint8_t* flags, int32_t* steps, hipStream_t s);

}  // namespace rt
