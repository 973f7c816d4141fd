// gfx950 kernels of the particle-mesh field (Sec. 3.3) and of its
// interpolation scheme (App. B), and a trace kernel that integrates rays
// through that field.
//
// Field build for an isolated lens (the zero-padded case of Sec. 3.3):
//   * Cloud-in-Cell deposit of the particle masses onto the n^3 nodes, into the
//     real part of a complex (2n)^3 grid (FP64 atomics; mass whose cloud falls
//     outside the nodes is dropped);
//   * 3-D complex FFTs, one LDS-resident radix-2 line per workgroup per axis;
//   * product with the transforms of the Plummer kernels of eq. psi and
//     eq. derivs on the padded grid, which makes the cyclic convolution the exact
//     linear one;  phi = -(G/c^2) sum M (d^2 + eps^2)^(-1/2) and
//     dphi/dx = (G/c^2) sum M d_x (d^2 + eps^2)^(-3/2) at every node;
//   * natural cubic-spline second derivatives of each of the four grids along
//     the line of sight x^3 (computed once per grid, App. B).
// Periodic boxes: the deposit wraps, the node masses' transform is multiplied
// by the continuum Green's function of Poisson's equation (and i k_j for the
// derivatives), and the x^3 spline is the periodic one.
// Evaluation at a point (App. B, n_int nodes on each side): (2 n_int)^2 spline
// evaluations along x^3, 2 n_int local natural splines along x^1, one local
// natural spline along x^2; zero outside the node range.
//
// HBM layout of the field: fields[8][n^3], grid q in [0, 4) = phi, dphi/dx^1,
// dphi/dx^2, dphi/dx^3 and q + 4 = its x^3 spline second derivatives; node
// (i, j, k) at (i n + j) n + k, so every x^3 line is contiguous.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>

#include "rt_geodesic.h"
#include "rt_internal.h"

namespace rt {

namespace {

constexpr int kMaxLine = 1024;   // longest FFT line (2n for n = 512)

// ------------------------------------------------------------------ build
__global__ void pm_clear_kernel(double2* buf, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < count) buf[i] = make_double2(0.0, 0.0);
}

__global__ void pm_twiddle_kernel(double2* tw, int M) {
  const int k = blockIdx.x * blockDim.x + threadIdx.x;
  if (k >= M / 2) return;
  double s, c;
  sincospi(2.0 * (double)k / (double)M, &s, &c);
  tw[k] = make_double2(c, -s);   // exp(-2 pi i k / M)
}

__global__ void pm_cic_kernel(const double* __restrict__ xyzm, int64_t np, double ox, double oy, double oz, double h,
                              int n, int M, int periodic, double2* buf) {
  const int64_t p = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (p >= np) return;
  const double u[3] = {(xyzm[p] - ox) / h, (xyzm[np + p] - oy) / h, (xyzm[2 * np + p] - oz) / h};
  const double m = xyzm[3 * np + p];
  int64_t i0[3];
  double f[3];
  for (int d = 0; d < 3; ++d) {
    const double fl = floor(u[d]);
    i0[d] = (int64_t)fl;
    f[d] = u[d] - fl;
  }
#pragma unroll
  for (int corner = 0; corner < 8; ++corner) {
    const int a = corner >> 2, b = (corner >> 1) & 1, c = corner & 1;
    int64_t i = i0[0] + a, j = i0[1] + b, k = i0[2] + c;
    if (periodic) {
      i = ((i % n) + n) % n;
      j = ((j % n) + n) % n;
      k = ((k % n) + n) % n;
    } else if (i < 0 || i >= n || j < 0 || j >= n || k < 0 || k >= n) {
      continue;
    }
    const double w = (a ? f[0] : 1.0 - f[0]) * (b ? f[1] : 1.0 - f[1]) * (c ? f[2] : 1.0 - f[2]);
    atomicAdd(&buf[(i * M + j) * M + k].x, m * w);
  }
}

// One line of M points per workgroup: bit-reversed load into LDS, log2 M
// radix-2 stages, store.  axis 2 is contiguous, axis 1 has stride M, axis 0 M^2.
__global__ __launch_bounds__(256) void pm_fft_kernel(double2* buf, int M, int log2M, int axis, int inverse,
                                                     const double2* __restrict__ tw) {
  __shared__ double2 line[kMaxLine];
  const int64_t l = blockIdx.x;
  const int64_t MM = (int64_t)M * M;
  int64_t base, stride;
  if (axis == 2) {
    base = l * M;
    stride = 1;
  } else if (axis == 1) {
    base = (l / M) * MM + (l % M);
    stride = M;
  } else {
    base = l;
    stride = MM;
  }
  const int nt = blockDim.x;
  for (int t = threadIdx.x; t < M; t += nt) {
    const int r = (int)(__brev((unsigned)t) >> (32 - log2M));
    line[r] = buf[base + (int64_t)t * stride];
  }
  __syncthreads();
  for (int s = 1; s <= log2M; ++s) {
    const int half = 1 << (s - 1);
    const int tstep = M >> s;   // twiddle index step: exp(-2 pi i pos / (2 half)) = tw[pos * tstep]
    for (int b = threadIdx.x; b < M / 2; b += nt) {
      const int pos = b & (half - 1);
      const int i0 = ((b >> (s - 1)) << s) + pos;
      const int i1 = i0 + half;
      double2 w = tw[pos * tstep];
      if (inverse) w.y = -w.y;
      const double2 x1 = line[i1];
      const double2 t = make_double2(w.x * x1.x - w.y * x1.y, w.x * x1.y + w.y * x1.x);
      const double2 x0 = line[i0];
      line[i0] = make_double2(x0.x + t.x, x0.y + t.y);
      line[i1] = make_double2(x0.x - t.x, x0.y - t.y);
    }
    __syncthreads();
  }
  for (int t = threadIdx.x; t < M; t += nt) buf[base + (int64_t)t * stride] = line[t];
}

// Kernel q on the padded grid: displacement of index i is i h for i < n and
// (i - M) h otherwise.
__global__ void pm_greens_kernel(double2* buf, int n, int M, double h, double eps2, int q, double G) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t MM = (int64_t)M * M;
  if (idx >= MM * M) return;
  const int i = (int)(idx / MM), j = (int)((idx / M) % M), k = (int)(idx % M);
  const double dx = (i < n ? i : i - M) * h, dy = (j < n ? j : j - M) * h, dz = (k < n ? k : k - M) * h;
  const double r2 = dx * dx + dy * dy + dz * dz + eps2;
  const double k1 = r2 > 0.0 ? 1.0 / sqrt(r2) : 0.0;
  const double k3 = k1 * k1 * k1;
  double v;
  if (q == 0) v = -G * k1;
  else v = G * (q == 1 ? dx : (q == 2 ? dy : dz)) * k3;
  buf[idx] = make_double2(v, 0.0);
}

__global__ void pm_mul_kernel(double2* b, const double2* __restrict__ a, int64_t count) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= count) return;
  const double2 x = a[i], y = b[i];
  b[i] = make_double2(x.x * y.x - x.y * y.y, x.x * y.y + x.y * y.x);
}

__global__ void pm_extract_kernel(const double2* __restrict__ buf, double* out, int n, int M, double scale) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nn = (int64_t)n * n;
  if (idx >= nn * n) return;
  const int64_t i = idx / nn, j = (idx / n) % n, k = idx % n;
  out[idx] = buf[(i * M + j) * M + k].x * scale;
}

// Natural-spline second derivatives along each contiguous x^3 line: the
// tridiagonal system y2[k-1] + 4 y2[k] + y2[k+1] = 6 (y[k+1] - 2 y[k] + y[k-1]) / h^2
// with y2 = 0 at both ends, by elimination (its pivots are the same for every
// line and are kept in LDS).
__global__ __launch_bounds__(256) void pm_spline_z_kernel(const double* __restrict__ F, double* F2, int n, double h,
                                                          int64_t n_lines) {
  __shared__ double cp[kMaxLine];
  if (threadIdx.x == 0) {
    double c = 0.0;
    for (int k = 1; k < n - 1; ++k) {
      c = 1.0 / (4.0 - (k > 1 ? c : 0.0));
      cp[k] = c;
    }
  }
  __syncthreads();
  const int64_t line = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (line >= n_lines) return;
  const double* y = F + line * n;
  double* y2 = F2 + line * n;
  y2[0] = 0.0;
  y2[n - 1] = 0.0;
  if (n < 3) return;
  const double s = 6.0 / (h * h);
  double d = 0.0;
  for (int k = 1; k < n - 1; ++k) {
    const double r = s * (y[k + 1] - 2.0 * y[k] + y[k - 1]);
    d = (r - (k > 1 ? d : 0.0)) * cp[k];
    y2[k] = d;
  }
  for (int k = n - 3; k >= 1; --k) y2[k] = y2[k] - cp[k] * y2[k + 1];
}

// Periodic box: b = G_q(k) a for the node masses' transform a, with the
// continuum Green's function of Poisson's equation, phi_k = -4 pi G rho_k / k^2
// (rho = mass / h^3, k = 0 removed, which also removes the mean density), and
// dphi/dx_j = i k_j phi_k.  Frequencies in the FFT's order: index i means
// i / (n h) for i < n/2 and (i - n) / (n h) otherwise.
__global__ void pm_poisson_kernel(double2* b, const double2* __restrict__ a, int n, double h, int q, double G) {
  const int64_t idx = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  const int64_t nn = (int64_t)n * n;
  if (idx >= nn * n) return;
  const int i = (int)(idx / nn), j = (int)((idx / n) % n), k = (int)(idx % n);
  const double w = 2.0 * M_PI / (n * h);
  const double kx = (i < n / 2 ? i : i - n) * w, ky = (j < n / 2 ? j : j - n) * w, kz = (k < n / 2 ? k : k - n) * w;
  const double k2 = kx * kx + ky * ky + kz * kz;
  double2 out = make_double2(0.0, 0.0);
  if (k2 > 0.0) {
    const double g = -4.0 * M_PI * G / (h * h * h) / k2;
    const double2 phik = make_double2(g * a[idx].x, g * a[idx].y);
    if (q == 0) {
      out = phik;
    } else {
      const double kq = q == 1 ? kx : (q == 2 ? ky : kz);
      out = make_double2(-kq * phik.y, kq * phik.x);   // i k_q phi_k
    }
  }
  b[idx] = out;
}

// Periodic cubic-spline second derivatives along each x^3 line: the cyclic
// system y2[k-1] + 4 y2[k] + y2[k+1] = 6 (y[k+1] - 2 y[k] + y[k-1]) / h^2,
// indices mod n, by the Sherman-Morrison form of elimination: the tridiagonal
// part with modified corner pivots is solved for the right-hand side and for
// the corner vector (the latter, like the pivots, is the same for every line
// and is kept in LDS).
__global__ __launch_bounds__(256) void pm_spline_z_periodic_kernel(const double* __restrict__ F, double* F2, int n,
                                                                   double h, int64_t n_lines) {
  __shared__ double piv[kMaxLine];   // 1 / (diagonal - previous multiplier)
  __shared__ double zc[kMaxLine];    // solution for the corner vector
  __shared__ double fz;              // 1 + z[0] + z[n-1] / gamma
  constexpr double gamma = -4.0;
  if (threadIdx.x == 0) {
    double c = 0.0;
    for (int k = 0; k < n; ++k) {
      const double diag = (k == 0) ? 4.0 - gamma : ((k == n - 1) ? 4.0 - 1.0 / gamma : 4.0);
      const double pk = 1.0 / (diag - (k > 0 ? c : 0.0));
      piv[k] = pk;
      c = pk;                         // super-diagonal 1 times the pivot inverse
    }
    // corner vector u = (gamma, 0, ..., 0, 1)
    double d = 0.0;
    for (int k = 0; k < n; ++k) {
      const double r = (k == 0) ? gamma : ((k == n - 1) ? 1.0 : 0.0);
      d = (r - (k > 0 ? d : 0.0)) * piv[k];
      zc[k] = d;
    }
    for (int k = n - 2; k >= 0; --k) zc[k] = zc[k] - piv[k] * zc[k + 1];
    fz = 1.0 + zc[0] + zc[n - 1] / gamma;
  }
  __syncthreads();
  const int64_t line = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (line >= n_lines) return;
  const double* y = F + line * n;
  double* y2 = F2 + line * n;
  const double s = 6.0 / (h * h);
  double d = 0.0;
  for (int k = 0; k < n; ++k) {
    const double r = s * (y[(k + 1) % n] - 2.0 * y[k] + y[(k + n - 1) % n]);
    d = (r - (k > 0 ? d : 0.0)) * piv[k];
    y2[k] = d;
  }
  for (int k = n - 2; k >= 0; --k) y2[k] = y2[k] - piv[k] * y2[k + 1];
  const double fact = (y2[0] + y2[n - 1] / gamma) / fz;
  for (int k = 0; k < n; ++k) y2[k] = y2[k] - fact * zc[k];
}

// ------------------------------------------------------------------ App. B evaluation
__device__ __forceinline__ double spline_eval(double yk, double yk1, double y2k, double y2k1, double A, double h) {
  const double B = 1.0 - A;
  return A * yk + B * yk1 + ((A * A * A - A) * y2k + (B * B * B - B) * y2k1) * (h * h) / 6.0;
}

// Natural spline through m = 2 NI values at unit-spaced nodes node0 + a (spacing h),
// evaluated at u (in node units).
template <int NI>
__device__ __forceinline__ double local_spline(const double (&v)[2 * NI], int node0, double u, double h) {
  constexpr int m = 2 * NI;
  double y2[m];
  y2[0] = 0.0;
  y2[m - 1] = 0.0;
  if constexpr (m >= 3) {
    const double s = 6.0 / (h * h);
    double cp[m];
    double c = 0.0, d = 0.0;
#pragma unroll
    for (int k = 1; k < m - 1; ++k) {
      c = 1.0 / (4.0 - (k > 1 ? c : 0.0));
      cp[k] = c;
      d = (s * (v[k + 1] - 2.0 * v[k] + v[k - 1]) - (k > 1 ? d : 0.0)) * c;
      y2[k] = d;
    }
#pragma unroll
    for (int k = m - 3; k >= 1; --k) y2[k] = y2[k] - cp[k] * y2[k + 1];
  }
  int kl = (int)floor(u) - node0;
  kl = kl < 0 ? 0 : (kl > m - 2 ? m - 2 : kl);
  const double A = (double)(node0 + kl + 1) - u;
  double yk = v[0], yk1 = v[1], s2k = y2[0], s2k1 = y2[1];
#pragma unroll
  for (int a = 1; a < m - 1; ++a)
    if (a == kl) {
      yk = v[a];
      yk1 = v[a + 1];
      s2k = y2[a];
      s2k1 = y2[a + 1];
    }
  return spline_eval(yk, yk1, s2k, s2k1, A, h);
}

__device__ __forceinline__ int window_start(double u, int n, int NI) {
  int k = (int)floor(u);
  k = k < 0 ? 0 : (k > n - 2 ? n - 2 : k);
  int st = k - NI + 1;
  st = st < 0 ? 0 : (st > n - 2 * NI ? n - 2 * NI : st);
  return st;
}

struct PmGrid {
  int n;
  double ox, oy, oz, h;
  int periodic;
};

__device__ __forceinline__ int wrap(int i, int n) { return ((i % n) + n) % n; }

// App. B on a periodic grid: the point is brought into the box (fmod, then + n
// for negative values), the x^3 segment and the x^1, x^2 windows are taken
// modulo n; the local splines see the unwrapped window nodes.
template <int NI>
__device__ void pm_field_periodic(const PmGrid& g, const double* __restrict__ fields, double x, double y, double z,
                                  double& phi, double& gx, double& gy, double& gz) {
  const int n = g.n;
  const double dn = (double)n;
  double ux = fmod((x - g.ox) / g.h, dn), uy = fmod((y - g.oy) / g.h, dn), uz = fmod((z - g.oz) / g.h, dn);
  phi = gx = gy = gz = 0.0;
  if (!(isfinite(ux) && isfinite(uy) && isfinite(uz))) return;
  if (ux < 0.0) ux += dn;
  if (uy < 0.0) uy += dn;
  if (uz < 0.0) uz += dn;
  const int fx = (int)floor(ux), fy = (int)floor(uy), fz = (int)floor(uz);
  const int wx = fx - NI + 1, wy = fy - NI + 1;
  const int kz0 = wrap(fz, n), kz1 = wrap(fz + 1, n);
  const double Az = (double)(fz + 1) - uz;
  const int64_t n3 = (int64_t)n * n * n;
  double out[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double* F = fields + q * n3;
    const double* F2 = fields + (q + 4) * n3;
    double w[2 * NI];
#pragma unroll
    for (int b = 0; b < 2 * NI; ++b) {
      const int j = wrap(wy + b, n);
      double v[2 * NI];
#pragma unroll
      for (int a = 0; a < 2 * NI; ++a) {
        const int64_t row = ((int64_t)wrap(wx + a, n) * n + j) * n;
        v[a] = spline_eval(F[row + kz0], F[row + kz1], F2[row + kz0], F2[row + kz1], Az, g.h);
      }
      w[b] = local_spline<NI>(v, wx, ux, g.h);
    }
    out[q] = local_spline<NI>(w, wy, uy, g.h);
  }
  phi = out[0];
  gx = out[1];
  gy = out[2];
  gz = out[3];
}

// The four grid quantities at (x, y, z): phi and its gradient.
template <int NI>
__device__ void pm_field(const PmGrid& g, const double* __restrict__ fields, double x, double y, double z, double& phi,
                         double& gx, double& gy, double& gz) {
  if (g.periodic) {
    pm_field_periodic<NI>(g, fields, x, y, z, phi, gx, gy, gz);
    return;
  }
  const int n = g.n;
  const double ux = (x - g.ox) / g.h, uy = (y - g.oy) / g.h, uz = (z - g.oz) / g.h;
  phi = gx = gy = gz = 0.0;
  if (!(ux >= 0.0 && uy >= 0.0 && uz >= 0.0 && ux <= n - 1 && uy <= n - 1 && uz <= n - 1)) return;
  const int wx = window_start(ux, n, NI), wy = window_start(uy, n, NI);
  int kz = (int)floor(uz);
  kz = kz > n - 2 ? n - 2 : kz;
  const double Az = (double)(kz + 1) - uz;
  const int64_t n3 = (int64_t)n * n * n;
  double out[4];
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const double* F = fields + q * n3;
    const double* F2 = fields + (q + 4) * n3;
    double w[2 * NI];
#pragma unroll
    for (int b = 0; b < 2 * NI; ++b) {
      double v[2 * NI];
#pragma unroll
      for (int a = 0; a < 2 * NI; ++a) {
        const int64_t at = ((int64_t)(wx + a) * n + (wy + b)) * n + kz;
        v[a] = spline_eval(F[at], F[at + 1], F2[at], F2[at + 1], Az, g.h);
      }
      w[b] = local_spline<NI>(v, wx, ux, g.h);
    }
    out[q] = local_spline<NI>(w, wy, uy, g.h);
  }
  phi = out[0];
  gx = out[1];
  gy = out[2];
  gz = out[3];
}

template <int NI>
__global__ __launch_bounds__(256) void pm_eval_kernel(PmGrid g, const double* __restrict__ fields, int64_t np,
                                                      const double* __restrict__ pts, double* phi, double* grad) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= np) return;
  double p, gx, gy, gz;
  pm_field<NI>(g, fields, pts[i], pts[np + i], pts[2 * np + i], p, gx, gy, gz);
  phi[i] = p;
  grad[i] = gx;
  grad[np + i] = gy;
  grad[2 * np + i] = gz;
}

// ------------------------------------------------------------------ trace through the PM field
// One ray per thread; the same RK4 in z, Christoffel contraction and flags as
// the direct-sum trace kernel, with the field of step s taken from grid
// step_grid[s] (none for -1): one isolated grid for a lens, one periodic grid
// per box replica for a light cone.
template <int NI>
__global__ __launch_bounds__(256) void pm_trace_kernel(DevCosmo cz, const DevPmGrid* __restrict__ grids,
                                                       const int32_t* __restrict__ step_grid,
                                                       const double* __restrict__ nodes, int32_t step_begin,
                                                       int32_t step_end, double* rays, int64_t N, uint8_t* flags) {
  const int64_t ri = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ri >= N) return;
  State Y{rays[ri], rays[N + ri], rays[2 * N + ri], rays[4 * N + ri], rays[5 * N + ri], rays[6 * N + ri],
          rays[7 * N + ri]};
  double zpos = rays[3 * N + ri];
  uint8_t flag = 0;
  bool live = true;
  for (int s = step_begin; s < step_end && live; ++s) {
    const double Z0 = nodes[s], Z1 = nodes[s + 1];
    const double h = Z1 - Z0, hh = 0.5 * h;
    const int gi = step_grid[s];
    PmGrid g{0, 0.0, 0.0, 0.0, 1.0, 0};
    const double* fields = nullptr;
    if (gi >= 0) {
      const DevPmGrid d = grids[gi];
      g = PmGrid{d.n, d.origin[0], d.origin[1], d.origin[2], d.h, d.periodic};
      fields = d.fields;
    }
    State acc, Ys, k;
    double a;
#pragma unroll 1
    for (int stage = 0; stage < 4; ++stage) {
      const State& Yin = (stage == 0) ? Y : Ys;
      const double zs = (stage == 0) ? Z0 : ((stage == 3) ? Z1 : Z0 + hh);
      double phi = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
      if (gi >= 0) pm_field<NI>(g, fields, Yin.x, Yin.y, zs, phi, gx, gy, gz);
      k = rhs(cz, Yin, phi, gx, gy, gz, a);
      if (stage == 0) {
        if (fabs(phi) / a > 1e-2) flag |= 4;
        acc = k;
        Ys = axpy(Y, hh, k);
      } else if (stage == 1) {
        acc = axpy(acc, 2.0, k);
        Ys = axpy(Y, hh, k);
      } else if (stage == 2) {
        acc = axpy(acc, 2.0, k);
        Ys = axpy(Y, h, k);
      } else {
        acc = axpy(acc, 1.0, k);
      }
    }
    const State Yn = axpy(Y, h / 6.0, acc);
    const bool finite = isfinite(Yn.t) && isfinite(Yn.x) && isfinite(Yn.y) && isfinite(Yn.kt) && isfinite(Yn.kx) &&
                        isfinite(Yn.ky) && isfinite(Yn.kz);
    if (!finite) {
      flag |= 1;
      live = false;
    } else if (!(Yn.kz > 0.0)) {
      flag |= 2;
      live = false;
    } else {
      Y = Yn;
      zpos = Z1;
    }
  }
  rays[ri] = Y.t;
  rays[N + ri] = Y.x;
  rays[2 * N + ri] = Y.y;
  rays[3 * N + ri] = zpos;
  rays[4 * N + ri] = Y.kt;
  rays[5 * N + ri] = Y.kx;
  rays[6 * N + ri] = Y.ky;
  rays[7 * N + ri] = Y.kz;
  if (flags && flag) flags[ri] |= flag;
}

// The paper's own integrator (Sec. 3.4, eq. RKstepsize): classical RK4 in the
// affine parameter with the fixed step f_RK h / kz_0 (h: the Fourier-grid
// spacing, kz_0: the ray's dz/dlambda at the start), repeated until z reaches
// chi_s; the step that overshoots is replaced by the linear interpolation
// between the previous and the current state at z = chi_s.  One ray per
// thread; a ray that has not reached chi_s after max_steps is flagged 8.  The
// field is a functor of the evaluation point: one grid everywhere, or the grid
// of the slab along x^3 that holds the point (Sec. 5.2's stack of cubes).
struct State8 {
  double t, x, y, z, kt, kx, ky, kz;
};

__device__ __forceinline__ State8 axpy8(const State8& Y, double h, const State8& k) {
  return State8{Y.t + h * k.t,   Y.x + h * k.x,   Y.y + h * k.y,   Y.z + h * k.z,
                Y.kt + h * k.kt, Y.kx + h * k.kx, Y.ky + h * k.ky, Y.kz + h * k.kz};
}

template <int NI>
struct OneGridField {
  PmGrid g;
  const double* fields;
  __device__ __forceinline__ void operator()(double x, double y, double z, double& phi, double& gx, double& gy,
                                             double& gz) const {
    pm_field<NI>(g, fields, x, y, z, phi, gx, gy, gz);
  }
};

// bounds [n_slabs + 1] strictly increasing; slab k = [bounds[k], bounds[k + 1])
// takes grid slab_grid[k] (none for -1); no field outside [bounds[0],
// bounds[n_slabs]) (a NaN z included).
template <int NI>
struct SlabField {
  const DevPmGrid* grids;
  const double* bounds;
  const int32_t* slab_grid;
  int32_t n_slabs;
  __device__ __forceinline__ void operator()(double x, double y, double z, double& phi, double& gx, double& gy,
                                             double& gz) const {
    phi = gx = gy = gz = 0.0;
    if (!(z >= bounds[0] && z < bounds[n_slabs])) return;
    int lo = 0, hi = n_slabs;   // bounds[lo] <= z < bounds[hi]
    while (hi - lo > 1) {
      const int mid = (lo + hi) >> 1;
      if (z >= bounds[mid])
        lo = mid;
      else
        hi = mid;
    }
    const int gi = slab_grid[lo];
    if (gi < 0) return;
    const DevPmGrid d = grids[gi];
    pm_field<NI>(PmGrid{d.n, d.origin[0], d.origin[1], d.origin[2], d.h, d.periodic}, d.fields, x, y, z, phi, gx, gy,
                 gz);
  }
};

template <class FieldAt>
__device__ __forceinline__ State8 rhs_lambda(const DevCosmo& c, const FieldAt& field, const State8& Y, double& phi,
                                             double& a) {
  double gx, gy, gz, At, Ax, Ay, Az;
  field(Y.x, Y.y, Y.z, phi, gx, gy, gz);
  accel(c, Y.t, Y.kt, Y.kx, Y.ky, Y.kz, phi, gx, gy, gz, a, At, Ax, Ay, Az);
  return State8{Y.kt, Y.kx, Y.ky, Y.kz, -At, -Ax, -Ay, -Az};
}

template <class FieldAt>
__global__ __launch_bounds__(256) void pm_trace_lambda_kernel(DevCosmo cz, FieldAt field, double h_rk, double chi_s,
                                                              double f_rk, int32_t max_steps, double* rays, int64_t N,
                                                              uint8_t* flags, int32_t* steps_out) {
  const int64_t ri = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (ri >= N) return;
  State8 Y{rays[ri],         rays[N + ri],     rays[2 * N + ri], rays[3 * N + ri],
           rays[4 * N + ri], rays[5 * N + ri], rays[6 * N + ri], rays[7 * N + ri]};
  const double dl = f_rk * h_rk / Y.kz;
  uint8_t flag = 0;
  bool done = !(Y.z < chi_s);
  int32_t s = 0;
  for (; s < max_steps && !done; ++s) {
    double phi, a, unused_phi, unused_a;
    const State8 k1 = rhs_lambda(cz, field, Y, phi, a);
    if (fabs(phi) / a > 1e-2) flag |= 4;
    const State8 k2 = rhs_lambda(cz, field, axpy8(Y, 0.5 * dl, k1), unused_phi, unused_a);
    const State8 k3 = rhs_lambda(cz, field, axpy8(Y, 0.5 * dl, k2), unused_phi, unused_a);
    const State8 k4 = rhs_lambda(cz, field, axpy8(Y, dl, k3), unused_phi, unused_a);
    State8 sum = axpy8(k1, 2.0, k2);
    sum = axpy8(sum, 2.0, k3);
    sum = axpy8(sum, 1.0, k4);
    const State8 Yn = axpy8(Y, dl / 6.0, sum);
    const bool finite = isfinite(Yn.t) && isfinite(Yn.x) && isfinite(Yn.y) && isfinite(Yn.z) && isfinite(Yn.kt) &&
                        isfinite(Yn.kx) && isfinite(Yn.ky) && isfinite(Yn.kz);
    if (!finite) {
      flag |= 1;
      done = true;
    } else if (!(Yn.kz > 0.0)) {
      flag |= 2;
      done = true;
    } else if (Yn.z >= chi_s) {
      const double w = (chi_s - Y.z) / (Yn.z - Y.z);
      Y = State8{Y.t + w * (Yn.t - Y.t),     Y.x + w * (Yn.x - Y.x),     Y.y + w * (Yn.y - Y.y),
                 Y.z + w * (Yn.z - Y.z),     Y.kt + w * (Yn.kt - Y.kt),  Y.kx + w * (Yn.kx - Y.kx),
                 Y.ky + w * (Yn.ky - Y.ky), Y.kz + w * (Yn.kz - Y.kz)};
      done = true;
    } else {
      Y = Yn;
    }
  }
  if (!done) flag |= 8;
  rays[ri] = Y.t;
  rays[N + ri] = Y.x;
  rays[2 * N + ri] = Y.y;
  rays[3 * N + ri] = Y.z;
  rays[4 * N + ri] = Y.kt;
  rays[5 * N + ri] = Y.kx;
  rays[6 * N + ri] = Y.ky;
  rays[7 * N + ri] = Y.kz;
  if (flags && flag) flags[ri] |= flag;
  if (steps_out) steps_out[ri] = s;
}

inline unsigned blocks_for(int64_t count, int threads) { return (unsigned)((count + threads - 1) / threads); }

}  // namespace

int64_t pm_workspace_bytes(int n, int periodic) {
  const int64_t M = periodic ? (int64_t)n : 2 * (int64_t)n;
  return 2 * M * M * M * (int64_t)sizeof(double2) + (M / 2) * (int64_t)sizeof(double2);
}

hipError_t launch_pm_build(const double* xyzm, int64_t np, double eps, const double origin[3], double h, int n,
                           int periodic, double G, double* fields, void* workspace, hipStream_t s) {
  const int M = periodic ? n : 2 * n;
  int log2M = 0;
  while ((1 << log2M) < M) ++log2M;
  const int64_t M3 = (int64_t)M * M * M;
  double2* A = static_cast<double2*>(workspace);
  double2* B = A + M3;
  double2* tw = B + M3;
  const int64_t n3 = (int64_t)n * n * n;
  const int fft_threads = M / 2 < 256 ? M / 2 : 256;
  hipLaunchKernelGGL(pm_twiddle_kernel, dim3(blocks_for(M / 2, 256)), dim3(256), 0, s, tw, M);
  hipLaunchKernelGGL(pm_clear_kernel, dim3(blocks_for(M3, 256)), dim3(256), 0, s, A, M3);
  if (np > 0)
    hipLaunchKernelGGL(pm_cic_kernel, dim3(blocks_for(np, 256)), dim3(256), 0, s, xyzm, np, origin[0], origin[1],
                       origin[2], h, n, M, periodic, A);
  auto fft3 = [&](double2* buf, int inverse) {
    for (int axis = 2; axis >= 0; --axis)
      hipLaunchKernelGGL(pm_fft_kernel, dim3((unsigned)((int64_t)M * M)), dim3(fft_threads), 0, s, buf, M, log2M,
                         axis, inverse, (const double2*)tw);
  };
  fft3(A, 0);
  for (int q = 0; q < 4; ++q) {
    if (periodic) {
      hipLaunchKernelGGL(pm_poisson_kernel, dim3(blocks_for(M3, 256)), dim3(256), 0, s, B, (const double2*)A, n, h, q,
                         G);
    } else {
      hipLaunchKernelGGL(pm_greens_kernel, dim3(blocks_for(M3, 256)), dim3(256), 0, s, B, n, M, h, eps * eps, q, G);
      fft3(B, 0);
      hipLaunchKernelGGL(pm_mul_kernel, dim3(blocks_for(M3, 256)), dim3(256), 0, s, B, (const double2*)A, M3);
    }
    fft3(B, 1);
    hipLaunchKernelGGL(pm_extract_kernel, dim3(blocks_for(n3, 256)), dim3(256), 0, s, (const double2*)B,
                       fields + q * n3, n, M, 1.0 / (double)M3);
  }
  const int64_t lines = 4 * (int64_t)n * n;
  if (periodic)
    hipLaunchKernelGGL(pm_spline_z_periodic_kernel, dim3(blocks_for(lines, 256)), dim3(256), 0, s,
                       (const double*)fields, fields + 4 * n3, n, h, lines);
  else
    hipLaunchKernelGGL(pm_spline_z_kernel, dim3(blocks_for(lines, 256)), dim3(256), 0, s, (const double*)fields,
                       fields + 4 * n3, n, h, lines);
  return hipGetLastError();
}

hipError_t launch_pm_eval(const double origin[3], double h, int n, int periodic, const double* fields, int n_int, int64_t np,
                          const double* pts, double* phi, double* grad, hipStream_t s) {
  const PmGrid g{n, origin[0], origin[1], origin[2], h, periodic};
  const dim3 grid(blocks_for(np, 256)), block(256);
  switch (n_int) {
    case 1: hipLaunchKernelGGL(pm_eval_kernel<1>, grid, block, 0, s, g, fields, np, pts, phi, grad); break;
    case 2: hipLaunchKernelGGL(pm_eval_kernel<2>, grid, block, 0, s, g, fields, np, pts, phi, grad); break;
    case 3: hipLaunchKernelGGL(pm_eval_kernel<3>, grid, block, 0, s, g, fields, np, pts, phi, grad); break;
    default: hipLaunchKernelGGL(pm_eval_kernel<4>, grid, block, 0, s, g, fields, np, pts, phi, grad); break;
  }
  return hipGetLastError();
}

hipError_t launch_pm_trace(DevCosmo c, const DevPmGrid* grids, const int32_t* step_grid, int n_int,
                           const double* nodes, int32_t step_begin, int32_t step_end, double* rays, int64_t n_rays,
                           uint8_t* flags, hipStream_t s) {
  const dim3 grid(blocks_for(n_rays, 256)), block(256);
  switch (n_int) {
    case 1:
      hipLaunchKernelGGL(pm_trace_kernel<1>, grid, block, 0, s, c, grids, step_grid, nodes, step_begin, step_end,
                         rays, n_rays, flags);
      break;
    case 2:
      hipLaunchKernelGGL(pm_trace_kernel<2>, grid, block, 0, s, c, grids, step_grid, nodes, step_begin, step_end,
                         rays, n_rays, flags);
      break;
    case 3:
      hipLaunchKernelGGL(pm_trace_kernel<3>, grid, block, 0, s, c, grids, step_grid, nodes, step_begin, step_end,
                         rays, n_rays, flags);
      break;
    default:
      hipLaunchKernelGGL(pm_trace_kernel<4>, grid, block, 0, s, c, grids, step_grid, nodes, step_begin, step_end,
                         rays, n_rays, flags);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_pm_trace_lambda(DevCosmo c, const double origin[3], double h, int n, int periodic, const double* fields,
                                  int n_int, double chi_s, double f_rk, int32_t max_steps, double* rays,
                                  int64_t n_rays, uint8_t* flags, int32_t* steps, hipStream_t s) {
  const PmGrid g{n, origin[0], origin[1], origin[2], h, periodic};
  const dim3 grid(blocks_for(n_rays, 256)), block(256);
  switch (n_int) {
    case 1:
      hipLaunchKernelGGL(pm_trace_lambda_kernel<OneGridField<1>>, grid, block, 0, s, c, OneGridField<1>{g, fields}, h,
                         chi_s, f_rk, max_steps, rays, n_rays, flags, steps);
      break;
    case 2:
      hipLaunchKernelGGL(pm_trace_lambda_kernel<OneGridField<2>>, grid, block, 0, s, c, OneGridField<2>{g, fields}, h,
                         chi_s, f_rk, max_steps, rays, n_rays, flags, steps);
      break;
    case 3:
      hipLaunchKernelGGL(pm_trace_lambda_kernel<OneGridField<3>>, grid, block, 0, s, c, OneGridField<3>{g, fields}, h,
                         chi_s, f_rk, max_steps, rays, n_rays, flags, steps);
      break;
    default:
      hipLaunchKernelGGL(pm_trace_lambda_kernel<OneGridField<4>>, grid, block, 0, s, c, OneGridField<4>{g, fields}, h,
                         chi_s, f_rk, max_steps, rays, n_rays, flags, steps);
      break;
  }
  return hipGetLastError();
}

hipError_t launch_pm_trace_lambda_slabs(DevCosmo c, const DevPmGrid* grids, const double* bounds,
                                        const int32_t* slab_grid, int32_t n_slabs, double h_rk, int n_int,
                                        double chi_s, double f_rk, int32_t max_steps, double* rays, int64_t n_rays,
                                        uint8_t* flags, int32_t* steps, hipStream_t s) {
  const dim3 grid(blocks_for(n_rays, 256)), block(256);
  switch (n_int) {
    case 1:
      hipLaunchKernelGGL(pm_trace_lambda_kernel<SlabField<1>>, grid, block, 0, s, c,
                         SlabField<1>{grids, bounds, slab_grid, n_slabs}, h_rk, chi_s, f_rk, max_steps, rays, n_rays,
                         flags, steps);
      break;
    case 2:
      hipLaunchKernelGGL(pm_trace_lambda_kernel<SlabField<2>>, grid, block, 0, s, c,
                         SlabField<2>{grids, bounds, slab_grid, n_slabs}, h_rk, chi_s, f_rk, max_steps, rays, n_rays,
                         flags, steps);
      break;
    case 3:
      hipLaunchKernelGGL(pm_trace_lambda_kernel<SlabField<3>>, grid, block, 0, s, c,
                         SlabField<3>{grids, bounds, slab_grid, n_slabs}, h_rk, chi_s, f_rk, max_steps, rays, n_rays,
                         flags, steps);
      break;
    default:
      hipLaunchKernelGGL(pm_trace_lambda_kernel<SlabField<4>>, grid, block, 0, s, c,
                         SlabField<4>{grids, bounds, slab_grid, n_slabs}, h_rk, chi_s, f_rk, max_steps, rays, n_rays,
                         flags, steps);
      break;
  }
  return hipGetLastError();
}

}  // namespace rt
