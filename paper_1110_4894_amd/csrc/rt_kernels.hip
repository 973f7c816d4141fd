// gfx950 kernels of the ray-bundle lensing path.
//
// Method: Killedar, Lasky, Lewis & Fluke (2011).  The hot kernel is the
// persistent trace kernel: every wavefront owns 7 whole bundles (63 rays, one
// per lane) and integrates them through all RK4 steps; at every stage the
// rays' field is the direct sum over the step's particle set (Sec. 3.3,
// eq. psi, derivs), streamed in tiles through the wavefront's own LDS slice.
// Several wavefronts may share the same rays and split the particles between
// them, combining their partial sums through LDS in a fixed order.
//
// Design notes for CDNA4:
//   * pair terms are plain VALU work: 13 FP32 VALU operations per pair with one
//     v_rsq_f32 among them, 12 for sets of equal masses (whose copies hold
//     positions only, four particles in three float4).  (A matrix-core form of the sum exists, but the FP32 frame of
//     a bundle can be shared by at most the 4 rays of a 4x4x1 block, and that
//     MFMA shape runs slower than the VALU loop on gfx950.)
//   * the FP32 path works in a frame per bundle: each 64-particle tile is
//     staged in LDS once per bundle as particle - anchor, and each lane holds
//     its ray's small offset from its anchor, so the differences between the
//     rays of a bundle keep full FP32 resolution;
//   * plain FP32 partial sums over each 64-particle tile are added with Kahan
//     compensation; FP64 is kept for the ray state and the integration;
//   * work items (field, block of rays) are pulled from an atomic queue so that
//     fields of very different particle counts share one launch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <type_traits>

#include "rt_geodesic.h"
#include "rt_internal.h"

namespace rt {

namespace {


__device__ __forceinline__ void wave_sync() {
  __builtin_amdgcn_fence(__ATOMIC_RELEASE, "wavefront");
  __builtin_amdgcn_wave_barrier();
  __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "wavefront");
}


__device__ __forceinline__ void kahan_add(float& s, float& c, float v) {
  float y = v - c;
  float t = s + y;
  c = (t - s) - y;
  s = t;
}

// FP64 reciprocal square root of a finite x > 0: the hardware estimate r
// (relative error about 2^-24) refined with the second-order expansion of
// (1 - e)^(-1/2), where e = 1 - x r^2:  r (1 + e/2 + 3 e^2/8).  The neglected
// term is 5 e^3 / 16, far below 2^-53.  The input is r^2 + eps^2 of a pair;
// it is zero only for a ray exactly on an unsoftened particle, where the
// field is singular anyway (the result is then NaN and the ray is flagged).
__device__ __forceinline__ double rsqrt_f64(double x) {
  const double r = __builtin_amdgcn_rsq(x);
  const double e = fma(-(x * r), r, 1.0);
  return fma(r * e, fma(0.375, e, 0.5), r);
}

// ---------------------------------------------------------------------------
// Uniform cuboid of unit density: U = int d^3x'/|p - x'| and dU/dp, from the
// antiderivative of 1/R evaluated at the eight corners (mean-density term of
// Sec. 3.3).  Each corner's three logarithms and three arctangents serve both
// U and its gradient; terms whose coefficient vanishes are skipped, which
// keeps faces, edges and corners finite (the observer sits on a face of the
// first box replica).
// ---------------------------------------------------------------------------
__device__ __forceinline__ double log_w_plus_r(double w, double R, double other2) {
  if (other2 == 0.0) return 0.0;      // every coefficient of this log is zero then
  return (w >= 0.0) ? log(w + R) : log(other2 / (R - w));
}

__device__ void cuboid_field(const double lo[3], const double hi[3], double px, double py, double pz, double& U,
                             double& gx, double& gy, double& gz) {
  U = gx = gy = gz = 0.0;
  const double xs[2] = {lo[0] - px, hi[0] - px};
  const double ys[2] = {lo[1] - py, hi[1] - py};
  const double zs[2] = {lo[2] - pz, hi[2] - pz};
#pragma unroll
  for (int corner = 0; corner < 8; ++corner) {
    const int i = corner & 1, j = (corner >> 1) & 1, k = (corner >> 2) & 1;
    const double X = xs[i], Y = ys[j], Z = zs[k];
    // sign = product over the axes of (+1 upper limit, -1 lower limit)
    const double s = ((i + j + k) & 1) ? 1.0 : -1.0;
    const double X2 = X * X, Y2 = Y * Y, Z2 = Z * Z;
    const double R = sqrt(X2 + Y2 + Z2);
    if (R == 0.0) continue;
    const double LX = log_w_plus_r(X, R, Y2 + Z2);
    const double LY = log_w_plus_r(Y, R, Z2 + X2);
    const double LZ = log_w_plus_r(Z, R, X2 + Y2);
    const double AX = (X != 0.0) ? atan(Y * Z / (X * R)) : 0.0;
    const double AY = (Y != 0.0) ? atan(Z * X / (Y * R)) : 0.0;
    const double AZ = (Z != 0.0) ? atan(X * Y / (Z * R)) : 0.0;
    const double F = X * Y * LZ + Y * Z * LX + Z * X * LY - 0.5 * (X2 * AX + Y2 * AY + Z2 * AZ);
    U += s * F;
    // the limits move with p (d limit / dp = -1)
    gx -= s * (Y * LZ + Z * LY - X * AX);
    gy -= s * (Z * LX + X * LZ - Y * AY);
    gz -= s * (X * LY + Y * LX - Z * AZ);
  }
}

// ---------------------------------------------------------------------------
// Field sums over one wavefront's share of a particle set.
//
// A wavefront holds 7 whole bundles: lane l < 63 owns ray l of the group
// (bundle l / 9, ray l % 9 of it, the anchor first); lane 63 only helps.
// Raw sums returned: S0 = sum m / r,  S = sum m (x_j - x) / r^3.
// ---------------------------------------------------------------------------
constexpr int kLanes = 63;              // rays per wavefront
constexpr int kSeg = 7;                 // bundles per wavefront
constexpr int kTile32 = 64;             // particles per FP32 tile (one per lane)
constexpr int kCopyStride = kTile32 + 1;  // float4 per bundle copy (+1 spreads the copies over LDS banks)

__device__ __forceinline__ int lane_segment(int lane) { return lane < kLanes ? lane / 9 : kSeg - 1; }

// FP32 path, equal masses: the staged copies hold positions only, four
// particles in three float4 (x0 y0 z0 x1 | y1 z1 x2 y2 | z2 x3 y3 z3), so the
// pair loop issues three LDS reads per four particles instead of four (the
// loop is bound by VALU issue and LDS returns together); the caller multiplies
// the unit-mass sums by the common mass.
constexpr int kPackedStride = 3 * kTile32 / 4 + 1;   // float4 per bundle copy
static_assert(kPackedStride <= kCopyStride, "the packed copies fit in the general tile");

// Four packed particles (three float4) against the lane's ray, unit masses.
__device__ __forceinline__ void pairs_equal4(const float4* g, float rx, float ry, float rz, float e2, float& p0,
                                             float& p1, float& p2, float& p3) {
  const float4 P0 = g[0], P1 = g[1], P2 = g[2];
  const float px[4] = {P0.x, P0.w, P1.z, P2.y};
  const float py[4] = {P0.y, P1.x, P1.w, P2.z};
  const float pz[4] = {P0.z, P1.y, P2.x, P2.w};
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const float ex = px[v] - rx, ey = py[v] - ry, ez = pz[v] - rz;
    float r2 = fmaf(ex, ex, e2);
    r2 = fmaf(ey, ey, r2);
    r2 = fmaf(ez, ez, r2);
    const float ri = __builtin_amdgcn_rsqf(r2);
    p0 += ri;
    const float r3 = ri * ri * ri;
    p1 = fmaf(r3, ex, p1);
    p2 = fmaf(r3, ey, p2);
    p3 = fmaf(r3, ez, p3);
  }
}

// Plain FP32 partial sums over one tile, added to the running sums with Kahan
// compensation.  A set's last tile runs only over its particles (to the next
// group of four), which is what a set of a few particles costs.
template <int WPR>
__device__ __forceinline__ void sum_fp32_equal(const DevSet& s, float4* tile, int q, int lane,
                                               const float (&A)[kSeg][3], float rx, float ry, float rz, double& S0,
                                               double& Sx, double& Sy, double& Sz) {
  float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
  float c0 = 0.f, c1 = 0.f, c2 = 0.f, c3 = 0.f;
  const int64_t n = s.n;
  const float e2 = s.eps2f;
  const int64_t n_chunks = (n + kTile32 - 1) / kTile32;
  const float4* __restrict__ src = s.p32;
  float* tf = reinterpret_cast<float*>(tile);
  const float4* mine = tile + lane_segment(lane) * kPackedStride;
  for (int64_t ch = q; ch < n_chunks; ch += WPR) {
    const int64_t j = ch * kTile32 + lane;
    // Padding past the end sits so far away that r^2 overflows to +inf, whose
    // reciprocal square root is +0: it adds exactly nothing.
    const float4 p = (j < n) ? src[j] : make_float4(1e30f, 1e30f, 1e30f, 0.f);
#pragma unroll
    for (int b = 0; b < kSeg; ++b) {
      float* d = tf + 4 * b * kPackedStride + 3 * lane;
      d[0] = p.x - A[b][0];
      d[1] = p.y - A[b][1];
      d[2] = p.z - A[b][2];
    }
    wave_sync();
    const int64_t left = n - ch * kTile32;
    float p0 = 0.f, p1 = 0.f, p2 = 0.f, p3 = 0.f;
    if (left >= kTile32) {
#pragma unroll
      for (int u = 0; u < kTile32 / 4; ++u) pairs_equal4(mine + 3 * u, rx, ry, rz, e2, p0, p1, p2, p3);
    } else {
      const int groups = (int)((left + 3) / 4);
#pragma unroll 1
      for (int u = 0; u < groups; ++u) pairs_equal4(mine + 3 * u, rx, ry, rz, e2, p0, p1, p2, p3);
    }
    kahan_add(s0, c0, p0);
    kahan_add(s1, c1, p1);
    kahan_add(s2, c2, p2);
    kahan_add(s3, c3, p3);
    wave_sync();
  }
  const double m = s.mass;
  S0 = m * ((double)s0 - (double)c0);
  Sx = m * ((double)s1 - (double)c1);
  Sy = m * ((double)s2 - (double)c2);
  Sz = m * ((double)s3 - (double)c3);
}

// One (x, y, z, m) particle against the lane's ray.
__device__ __forceinline__ void pair_general(const float4 c, float rx, float ry, float rz, float e2, float& p0,
                                             float& p1, float& p2, float& p3) {
  const float ex = c.x - rx, ey = c.y - ry, ez = c.z - rz;
  float r2 = fmaf(ex, ex, e2);
  r2 = fmaf(ey, ey, r2);
  r2 = fmaf(ez, ez, r2);
  const float ri = __builtin_amdgcn_rsqf(r2);
  const float mr = c.w * ri;
  p0 += mr;
  const float mr3 = mr * ri * ri;
  p1 = fmaf(mr3, ex, p1);
  p2 = fmaf(mr3, ey, p2);
  p3 = fmaf(mr3, ez, p3);
}

// FP32 path.  Each tile of 64 particles is staged once per bundle of the
// wavefront, as particle - anchor (7 copies); each lane then subtracts only its
// ray's small offset from its anchor.  The anchor-relative part is rounded
// identically for the 9 rays of a bundle, so the differences between ring rays
// and anchor that carry the lensing signal keep full FP32 resolution wherever
// the bundles are on the sky.
template <int WPR>
__device__ __forceinline__ void sum_fp32(const DevSet& s, float4* tile, int q, int lane, const float (&A)[kSeg][3],
                                         float rx, float ry, float rz, double& S0, double& Sx, double& Sy,
                                         double& Sz) {
  float s0 = 0.f, s1 = 0.f, s2 = 0.f, s3 = 0.f;
  float c0 = 0.f, c1 = 0.f, c2 = 0.f, c3 = 0.f;
  const int64_t n = s.n;
  const float e2 = s.eps2f;
  const int64_t n_chunks = (n + kTile32 - 1) / kTile32;
  const float4* __restrict__ src = s.p32;
  const float4* mine = tile + lane_segment(lane) * kCopyStride;
  for (int64_t ch = q; ch < n_chunks; ch += WPR) {
    const int64_t j = ch * kTile32 + lane;
    const float4 p = (j < n) ? src[j] : make_float4(1e15f, 1e15f, 1e15f, 0.f);
#pragma unroll
    for (int b = 0; b < kSeg; ++b)
      tile[b * kCopyStride + lane] = make_float4(p.x - A[b][0], p.y - A[b][1], p.z - A[b][2], p.w);
    wave_sync();
    const int64_t left = n - ch * kTile32;
    float p0 = 0.f, p1 = 0.f, p2 = 0.f, p3 = 0.f;
    if (left >= kTile32) {
#pragma unroll
      for (int u = 0; u < kTile32; ++u) pair_general(mine[u], rx, ry, rz, e2, p0, p1, p2, p3);
    } else {
#pragma unroll 1
      for (int u = 0; u < (int)left; ++u) pair_general(mine[u], rx, ry, rz, e2, p0, p1, p2, p3);
    }
    kahan_add(s0, c0, p0);
    kahan_add(s1, c1, p1);
    kahan_add(s2, c2, p2);
    kahan_add(s3, c3, p3);
    wave_sync();
  }
  S0 = (double)s0 - (double)c0;
  Sx = (double)s1 - (double)c1;
  Sy = (double)s2 - (double)c2;
  Sz = (double)s3 - (double)c3;
}

__device__ __forceinline__ void pair_fp64(const double4 c, double x, double y, double z, double e2, double& a0,
                                          double& a1, double& a2, double& a3) {
  const double ex = c.x - x, ey = c.y - y, ez = c.z - z;
  double r2 = fma(ex, ex, e2);
  r2 = fma(ey, ey, r2);
  r2 = fma(ez, ez, r2);
  const double ri = rsqrt_f64(r2);
  const double mr = c.w * ri;
  a0 += mr;
  const double mr3 = mr * ri * ri;
  a1 = fma(mr3, ex, a1);
  a2 = fma(mr3, ey, a2);
  a3 = fma(mr3, ez, a3);
}

// The same with unit mass (sets of equal masses: the caller scales the sums).
__device__ __forceinline__ void pair_fp64_unit(const double4 c, double x, double y, double z, double e2,
                                               double& a0, double& a1, double& a2, double& a3) {
  const double ex = c.x - x, ey = c.y - y, ez = c.z - z;
  double r2 = fma(ex, ex, e2);
  r2 = fma(ey, ey, r2);
  r2 = fma(ez, ez, r2);
  const double ri = rsqrt_f64(r2);
  a0 += ri;
  const double r3 = ri * ri * ri;
  a1 = fma(r3, ex, a1);
  a2 = fma(r3, ey, a2);
  a3 = fma(r3, ez, a3);
}

// FP64 path: tiles of the caller's FP64 particles, broadcast to every lane.
// UNIT: every mass equals s.mass, which multiplies the finished sums.
template <int T, int WPR, bool UNIT>
__device__ __forceinline__ void sum_fp64(const DevSet& s, double4* tile, int q, int lane, double x, double y,
                                         double z, double& S0, double& Sx, double& Sy, double& Sz) {
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  const int64_t n = s.n;
  const double e2 = s.eps2;
  const int64_t n_chunks = (n + T - 1) / T;
  const double* __restrict__ px = s.p64;
  for (int64_t ch = q; ch < n_chunks; ch += WPR) {
    const int64_t base = ch * T;
#pragma unroll
    for (int k = lane; k < T; k += 64) {
      const int64_t j = base + k;
      tile[k] = (j < n) ? make_double4(px[j], px[n + j], px[2 * n + j], px[3 * n + j])
                        : make_double4(1e100, 1e100, 1e100, 0.0);
    }
    wave_sync();
    const int64_t left = n - base;   // the set's last tile runs only over its particles
    if (left >= T) {
#pragma unroll 8
      for (int k = 0; k < T; ++k) {
        if constexpr (UNIT) pair_fp64_unit(tile[k], x, y, z, e2, a0, a1, a2, a3);
        else pair_fp64(tile[k], x, y, z, e2, a0, a1, a2, a3);
      }
    } else {
#pragma unroll 1
      for (int k = 0; k < (int)left; ++k) {
        if constexpr (UNIT) pair_fp64_unit(tile[k], x, y, z, e2, a0, a1, a2, a3);
        else pair_fp64(tile[k], x, y, z, e2, a0, a1, a2, a3);
      }
    }
    wave_sync();
  }
  const double m = UNIT ? s.mass : 1.0;
  S0 = m * a0;
  Sx = m * a1;
  Sy = m * a2;
  Sz = m * a3;
}

// LDS needed by one wavefront's tiles.
template <bool F64, int T>
struct TileSpace {
  static constexpr int kElems = F64 ? T : kSeg * kCopyStride;
  using Elem = typename std::conditional<F64, double4, float4>::type;
};

// Field of one set at the lane's point for a group of WPR wavefronts holding
// the same rays: each sums its share of the tiles and the shares meet in LDS
// in a fixed order, so every wavefront of the group gets identical results.
template <bool F64, int T, int WPR>
struct FieldEval {
  using Tile = typename TileSpace<F64, T>::Elem;

  // red_in_tiles: red lives in the LDS tiles of the workgroup, so every wavefront must have
  // finished its pair loop before the partial sums are written.
  __device__ static void eval(const DevCosmo& c, const DevSet& s, Tile* tile, double* red, int q, int lane, double x,
                              double y, double z, double& phi, double& gx, double& gy, double& gz,
                              bool red_in_tiles = false) {
    double S0, Sx, Sy, Sz;
    if constexpr (F64) {
      if (s.equal_mass && *s.equal_mass)
        sum_fp64<T, WPR, true>(s, tile, q, lane, x, y, z, S0, Sx, Sy, Sz);
      else
        sum_fp64<T, WPR, false>(s, tile, q, lane, x, y, z, S0, Sx, Sy, Sz);
    } else {
      // positions in the set's frame (FP64), each bundle's anchor rounded to FP32
      const double X = x - s.org[0], Yv = y - s.org[1], Z = z - s.org[2];
      const int anchor = 9 * lane_segment(lane);
      const double AX = __shfl(X, anchor), AY = __shfl(Yv, anchor), AZ = __shfl(Z, anchor);
      const float ax = (float)AX, ay = (float)AY, az = (float)AZ;
      float A[kSeg][3];
#pragma unroll
      for (int b = 0; b < kSeg; ++b) {
        A[b][0] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ax), 9 * b));
        A[b][1] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(ay), 9 * b));
        A[b][2] = __int_as_float(__builtin_amdgcn_readlane(__float_as_int(az), 9 * b));
      }
      const float rx = (float)(X - (double)ax), ry = (float)(Yv - (double)ay), rz = (float)(Z - (double)az);
      if (s.equal_mass && *s.equal_mass)
        sum_fp32_equal<WPR>(s, tile, q, lane, A, rx, ry, rz, S0, Sx, Sy, Sz);
      else
        sum_fp32<WPR>(s, tile, q, lane, A, rx, ry, rz, S0, Sx, Sy, Sz);
    }
    if constexpr (WPR > 1) {
      // red: [WPR][4][64] for this group
      if (red_in_tiles) __syncthreads();
      red[(q * 4 + 0) * 64 + lane] = S0;
      red[(q * 4 + 1) * 64 + lane] = Sx;
      red[(q * 4 + 2) * 64 + lane] = Sy;
      red[(q * 4 + 3) * 64 + lane] = Sz;
      __syncthreads();
      S0 = Sx = Sy = Sz = 0.0;
#pragma unroll
      for (int w = 0; w < WPR; ++w) {
        S0 += red[(w * 4 + 0) * 64 + lane];
        Sx += red[(w * 4 + 1) * 64 + lane];
        Sy += red[(w * 4 + 2) * 64 + lane];
        Sz += red[(w * 4 + 3) * 64 + lane];
      }
      __syncthreads();
    }
    phi = -c.G * S0;
    gx = -c.G * Sx;
    gy = -c.G * Sy;
    gz = -c.G * Sz;
    if (s.background) {
      double U, ux, uy, uz;
      cuboid_field(s.lo, s.hi, x, y, z, U, ux, uy, uz);
      phi += c.G_rho * U;
      gx += c.G_rho * ux;
      gy += c.G_rho * uy;
      gz += c.G_rho * uz;
    }
  }
};

__device__ __forceinline__ void store_state(double* st, int lane, int at, const State& v) {
  st[(at + 0) * 64 + lane] = v.t;
  st[(at + 1) * 64 + lane] = v.x;
  st[(at + 2) * 64 + lane] = v.y;
  st[(at + 3) * 64 + lane] = v.kt;
  st[(at + 4) * 64 + lane] = v.kx;
  st[(at + 5) * 64 + lane] = v.ky;
  st[(at + 6) * 64 + lane] = v.kz;
}

__device__ __forceinline__ State load_state(const double* st, int lane, int at) {
  return State{st[(at + 0) * 64 + lane], st[(at + 1) * 64 + lane], st[(at + 2) * 64 + lane],
               st[(at + 3) * 64 + lane], st[(at + 4) * 64 + lane], st[(at + 5) * 64 + lane],
               st[(at + 6) * 64 + lane]};
}

// ---------------------------------------------------------------------------
// The persistent trace kernel.
// NW wavefronts per workgroup; WPR of them share 63 rays (7 bundles) and split
// the particles; T particles per FP64 tile.  Four wavefronts per SIMD are
// requested: the FP64 state stays in registers through the pair loop, and
// the compiler spills only inside the rarely used cuboid-background code.
// ---------------------------------------------------------------------------
template <bool F64, int NW, int WPR, int T>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(4, 4))) void trace_kernel(TraceParams P) {
  constexpr int NG = NW / WPR;
  using FE = FieldEval<F64, T, WPR>;
  using Tile = typename FE::Tile;
  // When the WPR wavefronts of a group share rays, one copy of the group's FP64
  // RK4 state (Y, the stage input and the accumulator: 21 values per ray) waits
  // in LDS while the field is summed, instead of 128-VGPR wavefronts spilling
  // their identical copies to scratch.  The reduction buffer then shares the
  // tiles' LDS, so that the state fits beside them at two workgroups per CU.
  constexpr int kStateWords = 21 * 64;
  constexpr int kTileBytes = NW * TileSpace<F64, T>::kElems * (int)sizeof(Tile);
  // (FP32 path only: the FP64 path measured 4% slower with the extra barriers.)
  constexpr bool kLdsState = !F64 && WPR >= 2 && kTileBytes + NG * kStateWords * 8 <= 80 * 1024 &&
                             kTileBytes >= NG * WPR * 4 * 64 * 8;
  __shared__ Tile tiles[NW][TileSpace<F64, T>::kElems];
  __shared__ double red_own[NG][(WPR > 1 && !kLdsState) ? WPR * 4 * 64 : 1];
  __shared__ double state_lds[kLdsState ? NG : 1][kLdsState ? kStateWords : 1];
  __shared__ int s_item;

  // the wavefront index is uniform: keep it (and the tile loop counters) in SGPRs
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int g = wave / WPR, q = wave % WPR;
  const DevCosmo& cz = P.cosmo;
  double* red = kLdsState ? reinterpret_cast<double*>(&tiles[0][0]) + g * (WPR * 4 * 64) : &red_own[g][0];
  double* st = &state_lds[kLdsState ? g : 0][0];

  for (;;) {
    if (threadIdx.x == 0) s_item = atomicAdd(P.queue, 1);
    __syncthreads();
    const int item = s_item;
    __syncthreads();
    if (item >= P.n_items) break;

    const WorkItem wi = P.items[item];
    const DevField f = P.fields[wi.field];
    const int64_t rend = f.ray_begin + f.n_rays;
    int64_t ri = f.ray_begin + (int64_t)wi.block * (kLanes * NG) + g * kLanes + (lane < kLanes ? lane : kLanes - 1);
    const bool valid = lane < kLanes && ri < rend;
    if (ri >= rend) ri = rend - 1;
    const int64_t N = P.n_rays;
    State Y{P.rays[ri], P.rays[N + ri], P.rays[2 * N + ri], P.rays[4 * N + ri], P.rays[5 * N + ri],
            P.rays[6 * N + ri], P.rays[7 * N + ri]};
    double zpos = P.rays[3 * N + ri];
    uint8_t flag = 0;
    bool live = true;
    const int sb = P.step_begin < 0 ? 0 : P.step_begin;
    const int se = P.step_end > f.n_steps ? f.n_steps : P.step_end;

    for (int s = sb; s < se; ++s) {
      const double Z0 = P.nodes[f.node_off + s], Z1 = P.nodes[f.node_off + s + 1];
      const double h = Z1 - Z0, hh = 0.5 * h;
      const int S = P.step_set[f.step_off + s];
      State acc{}, Ys{}, k;
      double a;
#pragma unroll 1
      for (int stage = 0; stage < 4; ++stage) {
        const double xin = (stage == 0) ? Y.x : Ys.x, yin = (stage == 0) ? Y.y : Ys.y;
        const double zs = (stage == 0) ? Z0 : ((stage == 3) ? Z1 : Z0 + hh);
        if constexpr (kLdsState) {
          if (q == 0) {
            store_state(st, lane, 0, Y);
            store_state(st, lane, 7, acc);
            store_state(st, lane, 14, Ys);
          }
        }
        double phi = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
        if (S >= 0) {
          const DevSet& set = P.sets[f.set_off + S];
          FE::eval(cz, set, tiles[wave], red, q, lane, xin, yin, zs, phi, gx, gy, gz, kLdsState);
        }
        if constexpr (kLdsState) {
          if (S < 0) __syncthreads();   // the field sum's barriers order the stores otherwise
          Y = load_state(st, lane, 0);
          acc = load_state(st, lane, 7);
          Ys = load_state(st, lane, 14);
          __syncthreads();              // every wavefront has its copy before the next stores
        }
        const State& Yin = (stage == 0) ? Y : Ys;
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
      if (live) {
        const State Yn = axpy(Y, h / 6.0, acc);
        const bool finite = isfinite(Yn.t) && isfinite(Yn.x) && isfinite(Yn.y) && isfinite(Yn.kt) &&
                            isfinite(Yn.kx) && isfinite(Yn.ky) && isfinite(Yn.kz);
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
    }
    if (valid) {
      P.rays[ri] = Y.t;
      P.rays[N + ri] = Y.x;
      P.rays[2 * N + ri] = Y.y;
      P.rays[3 * N + ri] = zpos;
      P.rays[4 * N + ri] = Y.kt;
      P.rays[5 * N + ri] = Y.kx;
      P.rays[6 * N + ri] = Y.ky;
      P.rays[7 * N + ri] = Y.kz;
      if (P.flags && flag) P.flags[ri] |= flag;
    }
  }
}

// Field at arbitrary points: one wavefront = 63 points, no particle split.
// In the FP32 path every group of 9 consecutive points shares the frame of its
// first point, as the rays of a bundle do in the trace kernel.
template <bool F64, int T>
__global__ __launch_bounds__(256) void field_eval_kernel(DevCosmo c, const DevSet* set_p, int64_t n,
                                                         const double* pts, double* phi, double* grad) {
  using FE = FieldEval<F64, T, 1>;
  using Tile = typename FE::Tile;
  __shared__ Tile tiles[4][TileSpace<F64, T>::kElems];
  // the wavefront index is uniform: keep it (and the tile loop counters) in SGPRs
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int64_t w0 = ((int64_t)blockIdx.x * 4 + wave) * kLanes;
  if (w0 >= n) return;   // whole wavefront idle
  int64_t i = w0 + (lane < kLanes ? lane : kLanes - 1);
  const bool valid = lane < kLanes && i < n;
  if (i >= n) i = n - 1;
  const DevSet set = *set_p;
  double p, gx, gy, gz;
  FE::eval(c, set, tiles[wave], nullptr, 0, lane, pts[i], pts[n + i], pts[2 * n + i], p, gx, gy, gz);
  if (valid) {
    phi[i] = p;
    grad[i] = gx;
    grad[n + i] = gy;
    grad[2 * n + i] = gz;
  }
}

// ---------------------------------------------------------------------------
// Small kernels: queue reset, set frames, FP32 copies.
// ---------------------------------------------------------------------------
__global__ void reset_queue_kernel(int32_t* q) {
  if (threadIdx.x == 0 && blockIdx.x == 0) *q = 0;
}

// Frame origin of each set: the cuboid centre for sets with a background,
// otherwise the first particle.
__global__ void prepare_sets_kernel(DevSet* sets, int32_t n_sets) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= n_sets) return;
  DevSet& s = sets[i];
  s.mass = (s.n > 0) ? s.p64[3 * s.n] : 0.0;
  if (s.equal_mass) *s.equal_mass = 1;   // cleared by the FP32 conversion at the first other mass
  if (s.background) {
    for (int d = 0; d < 3; ++d) s.org[d] = 0.5 * (s.lo[d] + s.hi[d]);
  } else if (s.n > 0) {
    for (int d = 0; d < 3; ++d) s.org[d] = s.p64[d * s.n];
  } else {
    for (int d = 0; d < 3; ++d) s.org[d] = 0.0;
  }
}

__global__ void convert_set_kernel(const DevSet* set, const double* p64, float4* p32, int64_t n) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const double ox = set->org[0], oy = set->org[1], oz = set->org[2];
  const double m = p64[3 * n + j];
  if (p32)   // (FP64 sets have no copy: only their masses are checked)
    p32[j] = make_float4((float)(p64[j] - ox), (float)(p64[n + j] - oy), (float)(p64[2 * n + j] - oz), (float)m);
  if (!(m == p64[3 * n])) *set->equal_mass = 0;   // (a NaN mass also takes the general path)
}

// ---------------------------------------------------------------------------
// Bundle construction (Sec. 2.4, 3.1): one thread per ray.
// ---------------------------------------------------------------------------
__constant__ double kRingCos[8] = {1.0, 0.70710678118654752440, 0.0, -0.70710678118654752440,
                                   -1.0, -0.70710678118654752440, 0.0, 0.70710678118654752440};
__constant__ double kRingSin[8] = {0.0, 0.70710678118654752440, 1.0, 0.70710678118654752440,
                                   0.0, -0.70710678118654752440, -1.0, -0.70710678118654752440};

__global__ void bundles_kernel(DevCosmo c, const double* phi_obs, int64_t b0, int64_t nb_range, int64_t n_bundles,
                               const double* theta, double radius, double* rays) {
  const int64_t i = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= 9 * nb_range) return;
  const int64_t b = b0 + i / 9;
  const int k = (int)(i % 9);
  double tx = theta[b], ty = theta[n_bundles + b];
  if (k > 0) {
    tx += radius * kRingCos[k - 1];
    ty += radius * kRingSin[k - 1];
  }
  double a0, adot0;
  scale_factor(c, 0.0, a0, adot0);
  const double ph = phi_obs ? *phi_obs : 0.0;
  const double E0 = 1.0 + 2.0 * ph / a0, F0 = a0 * a0 - 2.0 * a0 * ph;
  const double norm = sqrt(E0 / F0) / sqrt(tx * tx + ty * ty + 1.0);
  const int64_t N = 9 * n_bundles, r = 9 * b + k;
  rays[r] = 0.0;
  rays[N + r] = 0.0;
  rays[2 * N + r] = 0.0;
  rays[3 * N + r] = 0.0;
  rays[4 * N + r] = 1.0;
  rays[5 * N + r] = norm * tx;
  rays[6 * N + r] = norm * ty;
  rays[7 * N + r] = norm;
}

// ---------------------------------------------------------------------------
// Bundle reduction (Sec. 2.4, eq. lensmap, magnification): 9 consecutive lanes
// hold one bundle (7 bundles per wavefront, lane 63 idle); offsets from the
// anchor and the neighbour's offsets arrive by lane shuffles, and the five
// sums are reduced within each 9-lane segment.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void magnification_kernel(double chi_s, int64_t nb, double radius, const double* rays,
                                                            double* mu, double* jac) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int seg = lane / 9, k = lane % 9;
  const int64_t b = ((int64_t)blockIdx.x * 4 + wave) * 7 + seg;
  const bool valid = (seg < 7) && (b < nb);
  const int64_t N = 9 * nb;
  const int64_t r = valid ? 9 * b + k : 0;
  const double x = rays[N + r], y = rays[2 * N + r];
  const int anchor = seg * 9;
  const double dx = x - __shfl(x, anchor), dy = y - __shfl(y, anchor);
  const int nxt = anchor + (k == 8 ? 1 : k + 1);
  const double dxn = __shfl(dx, nxt), dyn = __shfl(dy, nxt);
  double v[5] = {0.0, 0.0, 0.0, 0.0, 0.0};
  if (k > 0) {
    const double ux = radius * kRingCos[k - 1], uy = radius * kRingSin[k - 1];
    v[0] = 0.5 * (dx * dyn - dy * dxn);
    v[1] = dx * ux;
    v[2] = dx * uy;
    v[3] = dy * ux;
    v[4] = dy * uy;
  }
#pragma unroll
  for (int off = 1; off < 9; off <<= 1) {
    const int src = (k + off < 9) ? lane + off : lane;
#pragma unroll
    for (int m = 0; m < 5; ++m) {
      const double o = __shfl(v[m], src);
      if (k + off < 9) v[m] += o;
    }
  }
  if (valid && k == 0) {
    const double hom = 2.0 * sqrt(2.0) * radius * radius * chi_s * chi_s;
    mu[b] = hom / v[0];
    if (jac) {
      const double nrm = 1.0 / (4.0 * radius * radius * chi_s);
      const double a11 = v[1] * nrm, a12 = v[2] * nrm, a21 = v[3] * nrm, a22 = v[4] * nrm;
      jac[b] = 1.0 - 0.5 * (a11 + a22);
      jac[nb + b] = 0.5 * (a22 - a11);
      jac[2 * nb + b] = -0.5 * (a12 + a21);
      jac[3 * nb + b] = 0.5 * (a21 - a12);
    }
  }
}

// ---------------------------------------------------------------------------
// Source-weighted histograms (Sec. 5.3, eq. weighthisto; the same weighting
// for the shear distribution of Sec. 5.4): every bundle with mu > 0 has
// weight 1/mu.  mode 0: value log10 mu, bins of width in mu; mode 1: value
// |gamma| from the Jacobian, bins of width in |gamma|.  Deterministic: every
// sum runs in a fixed order (strided per thread, then a tree in LDS).
// work layout: [n_bins] bin weights, then sum w, sum w v, n_bad, n_under, n_over.
// ---------------------------------------------------------------------------
__device__ __forceinline__ double hist_value(int mode, const double* mu, const double* jac, int64_t n, int64_t i) {
  return mode == 0 ? log10(mu[i]) : hypot(jac[n + i], jac[2 * n + i]);
}

__device__ __forceinline__ int value_bin(double v, double lo, double hi, int nb) {
  if (v < lo) return -1;
  if (v >= hi) return nb;
  int i = (int)floor((v - lo) / (hi - lo) * nb);
  return i >= nb ? nb - 1 : i;
}

template <int NT>
__device__ __forceinline__ double block_sum(double v, double* sh) {
  sh[threadIdx.x] = v;
  __syncthreads();
#pragma unroll
  for (int o = NT / 2; o > 0; o >>= 1) {
    if ((int)threadIdx.x < o) sh[threadIdx.x] += sh[threadIdx.x + o];
    __syncthreads();
  }
  const double r = sh[0];
  __syncthreads();
  return r;
}

__global__ __launch_bounds__(256) void hist_bins_kernel(int64_t n, const double* mu, const double* jac, int mode,
                                                        int32_t nb, double lo, double hi, double* work) {
  __shared__ double sh[256];
  const int bin = blockIdx.x;
  if (bin < nb) {
    double acc = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
      const double m = mu[i];
      if (m > 0.0 && value_bin(hist_value(mode, mu, jac, n, i), lo, hi, nb) == bin) acc += 1.0 / m;
    }
    const double t = block_sum<256>(acc, sh);
    if (threadIdx.x == 0) work[bin] = t;
  } else {
    double sw = 0.0, swv = 0.0, bad = 0.0, under = 0.0, over = 0.0;
    for (int64_t i = threadIdx.x; i < n; i += 256) {
      const double m = mu[i];
      if (!(m > 0.0)) {
        bad += 1.0;
        continue;
      }
      const double w = 1.0 / m;
      const double v = hist_value(mode, mu, jac, n, i);
      sw += w;
      swv += w * (mode == 0 ? m : v);
      const int b = value_bin(v, lo, hi, nb);
      if (b < 0) under += 1.0;
      if (b >= nb) over += 1.0;
    }
    const double t0 = block_sum<256>(sw, sh), t1 = block_sum<256>(swv, sh), t2 = block_sum<256>(bad, sh);
    const double t3 = block_sum<256>(under, sh), t4 = block_sum<256>(over, sh);
    if (threadIdx.x == 0) {
      work[nb] = t0;
      work[nb + 1] = t1;
      work[nb + 2] = t2;
      work[nb + 3] = t3;
      work[nb + 4] = t4;
    }
  }
}

__global__ __launch_bounds__(256) void hist_final_kernel(int64_t n, const double* mu, const double* jac, int mode,
                                                         int32_t nb, double lo, double hi, const double* work,
                                                         double* pdf, double* moments) {
  __shared__ double sh[256];
  const double sw = work[nb];
  const double mean = sw > 0.0 ? work[nb + 1] / sw : 0.0;
  double acc = 0.0;
  for (int64_t i = threadIdx.x; i < n; i += 256) {
    const double m = mu[i];
    if (m > 0.0) {
      const double v = mode == 0 ? m : hist_value(mode, mu, jac, n, i);
      acc += (1.0 / m) * (v - mean) * (v - mean);
    }
  }
  const double var = block_sum<256>(acc, sh);
  for (int i = threadIdx.x; i < nb; i += 256) {
    const double e0 = lo + (hi - lo) * i / nb, e1 = lo + (hi - lo) * (i + 1) / nb;
    const double width = mode == 0 ? pow(10.0, e1) - pow(10.0, e0) : (hi - lo) / nb;
    pdf[i] = sw > 0.0 ? work[i] / (sw * width) : 0.0;
  }
  if (threadIdx.x == 0) {
    moments[0] = sw;
    moments[1] = mean;
    moments[2] = sw > 0.0 ? sqrt(var / sw) : 0.0;
    moments[3] = work[nb + 2];
    moments[4] = work[nb + 3];
    moments[5] = work[nb + 4];
  }
}

// ---------------------------------------------------------------------------
// Plan table.
// ---------------------------------------------------------------------------
struct PlanShape {
  int nw, wpr, tile;
};

constexpr PlanShape kPlans32[] = {{8, 1, 64}, {8, 2, 64}, {8, 4, 64}, {8, 8, 64}, {4, 1, 64}, {4, 4, 64}};
constexpr PlanShape kPlans64[] = {{8, 1, 128}, {8, 2, 128}, {8, 4, 128}, {8, 8, 64}, {4, 1, 128}, {4, 4, 128}};
constexpr int kNumPlans = 6;

template <bool F64, int I>
struct PlanKernel;

#define RT_PLAN(F64, I, TABLE)                                                                   \
  template <>                                                                                    \
  struct PlanKernel<F64, I> {                                                                    \
    static constexpr PlanShape S = TABLE[I];                                                     \
    static const void* fn() { return (const void*)&trace_kernel<F64, S.nw, S.wpr, S.tile>; }      \
    static hipError_t launch(const TraceParams& p, int grid, hipStream_t st) {                  \
      hipLaunchKernelGGL((trace_kernel<F64, S.nw, S.wpr, S.tile>), dim3(grid), dim3(S.nw * 64), 0, st, p); \
      return hipGetLastError();                                                                  \
    }                                                                                            \
  };

RT_PLAN(false, 0, kPlans32)
RT_PLAN(false, 1, kPlans32)
RT_PLAN(false, 2, kPlans32)
RT_PLAN(false, 3, kPlans32)
RT_PLAN(false, 4, kPlans32)
RT_PLAN(false, 5, kPlans32)
RT_PLAN(true, 0, kPlans64)
RT_PLAN(true, 1, kPlans64)
RT_PLAN(true, 2, kPlans64)
RT_PLAN(true, 3, kPlans64)
RT_PLAN(true, 4, kPlans64)
RT_PLAN(true, 5, kPlans64)
#undef RT_PLAN

template <bool F64>
const void* plan_fn(int id) {
  switch (id) {
    case 0: return PlanKernel<F64, 0>::fn();
    case 1: return PlanKernel<F64, 1>::fn();
    case 2: return PlanKernel<F64, 2>::fn();
    case 3: return PlanKernel<F64, 3>::fn();
    case 4: return PlanKernel<F64, 4>::fn();
    default: return PlanKernel<F64, 5>::fn();
  }
}

template <bool F64>
hipError_t plan_launch(int id, const TraceParams& p, int grid, hipStream_t st) {
  switch (id) {
    case 0: return PlanKernel<F64, 0>::launch(p, grid, st);
    case 1: return PlanKernel<F64, 1>::launch(p, grid, st);
    case 2: return PlanKernel<F64, 2>::launch(p, grid, st);
    case 3: return PlanKernel<F64, 3>::launch(p, grid, st);
    case 4: return PlanKernel<F64, 4>::launch(p, grid, st);
    default: return PlanKernel<F64, 5>::launch(p, grid, st);
  }
}

}  // namespace

int plan_count(bool) { return kNumPlans; }

rt_plan_info plan_info(bool fp64, int id) {
  const PlanShape s = fp64 ? kPlans64[id] : kPlans32[id];
  rt_plan_info r;
  r.waves_per_block = s.nw;
  r.waves_per_group = s.wpr;
  r.tile = s.tile;
  r.rays_per_block = kLanes * s.nw / s.wpr;
  return r;
}

hipError_t plan_occupancy(bool fp64, int id, int* blocks_per_cu) {
  const PlanShape s = fp64 ? kPlans64[id] : kPlans32[id];
  const void* fn = fp64 ? plan_fn<true>(id) : plan_fn<false>(id);
  return hipOccupancyMaxActiveBlocksPerMultiprocessor(blocks_per_cu, fn, s.nw * 64, 0);
}

hipError_t launch_trace(bool fp64, int id, const TraceParams& p, int grid, hipStream_t s) {
  return fp64 ? plan_launch<true>(id, p, grid, s) : plan_launch<false>(id, p, grid, s);
}

hipError_t launch_reset_queue(int32_t* q, hipStream_t s) {
  hipLaunchKernelGGL(reset_queue_kernel, dim3(1), dim3(64), 0, s, q);
  return hipGetLastError();
}

hipError_t launch_prepare_sets(DevSet* sets, int32_t n_sets, hipStream_t s) {
  if (n_sets <= 0) return hipSuccess;
  hipLaunchKernelGGL(prepare_sets_kernel, dim3((n_sets + 63) / 64), dim3(64), 0, s, sets, n_sets);
  return hipGetLastError();
}

hipError_t launch_convert_set(const DevSet* set_dev, const double* p64, float4* p32, int64_t n, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  hipLaunchKernelGGL(convert_set_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, set_dev, p64, p32, n);
  return hipGetLastError();
}

hipError_t launch_bundles(DevCosmo c, const double* phi_obs, int64_t b0, int64_t nb_range, int64_t n_bundles,
                          const double* theta, double radius, double* rays, hipStream_t s) {
  if (nb_range <= 0) return hipSuccess;
  const int64_t n = 9 * nb_range;
  hipLaunchKernelGGL(bundles_kernel, dim3((unsigned)((n + 255) / 256)), dim3(256), 0, s, c, phi_obs, b0, nb_range,
                     n_bundles, theta, radius, rays);
  return hipGetLastError();
}

hipError_t launch_field_eval(DevCosmo c, const DevSet* set, bool fp64, int64_t n, const double* pts, double* phi,
                             double* grad, hipStream_t s) {
  if (n <= 0) return hipSuccess;
  const unsigned grid = (unsigned)((n + 4 * kLanes - 1) / (4 * kLanes));
  if (fp64)
    hipLaunchKernelGGL((field_eval_kernel<true, kPlans64[0].tile>), dim3(grid), dim3(256), 0, s, c, set, n, pts, phi,
                       grad);
  else
    hipLaunchKernelGGL((field_eval_kernel<false, kPlans32[0].tile>), dim3(grid), dim3(256), 0, s, c, set, n, pts,
                       phi, grad);
  return hipGetLastError();
}

hipError_t launch_magnification(double chi_s, int64_t nb, double radius, const double* rays, double* mu,
                                double* jac, hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  const int64_t waves = (nb + 6) / 7;
  hipLaunchKernelGGL(magnification_kernel, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, chi_s, nb, radius,
                     rays, mu, jac);
  return hipGetLastError();
}

hipError_t launch_histogram(int64_t n, const double* mu, const double* jac, int mode, int32_t n_bins, double lo,
                            double hi, double* pdf, double* moments, double* work, hipStream_t s) {
  hipLaunchKernelGGL(hist_bins_kernel, dim3(n_bins + 1), dim3(256), 0, s, n, mu, jac, mode, n_bins, lo, hi, work);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  hipLaunchKernelGGL(hist_final_kernel, dim3(1), dim3(256), 0, s, n, mu, jac, mode, n_bins, lo, hi, work, pdf,
                     moments);
  return hipGetLastError();
}

}  // namespace rt
