// gfx950 kernels of the ray-bundle lensing path.
//
// Method: Killedar, Lasky, Lewis & Fluke (2011).  The hot kernel is the
// persistent trace kernel: every wavefront owns 7 whole bundles (63 rays, one
// per lane) and integrates them through all RK4 steps in FP64; at every stage
// the rays' field is the direct sum over the step's particle set (Sec. 3.3,
// eq. psi, derivs), streamed in tiles through the wavefront's own LDS slice.
//
// Design notes for CDNA4:
//   * FP32 field sums work per bundle (Sec. 3.1: an anchor and a ring of 8
//     rays a few parsecs away).  The nine lanes of a bundle split the
//     particles; each (bundle, particle) pair is evaluated once, at the
//     bundle's expansion point, as the pair's potential and field and their
//     first and second derivatives (20 moments, 37 VALU instructions per pair
//     of a set of equal masses including one v_rsq_f32, i.e. 4.1 per
//     ray-particle interaction).  Every ray
//     assembles its own field in FP64 from the moments and its exact offset.
//     Ring-minus-anchor field differences, which carry the lensing signal,
//     so keep FP32 relative precision: rounding each particle-ray
//     displacement to FP32 instead would quantise the ring offset to the ulp
//     of a Mpc-scale distance, identically for every particle of a binade;
//   * plain FP32 partial sums over 256 rounds of a bundle's nine lanes (one
//     or more tiles; one tile when the nearness test runs) are added with
//     Kahan compensation; FP64 is kept for the ray state, the integration and
//     the assembly of each ray's field;
//   * the pairwise sum is not a dense contraction: no matrix cores;
//   * work items (field, block of rays) are pulled from an atomic queue so that
//     fields of very different particle counts share one launch.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdint>
#include <map>
#include <mutex>
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
// Lane layout shared by every kernel that holds bundles: a wavefront holds 7
// whole bundles, lane l < 63 owns ray l of the group (bundle l / 9, ray l % 9
// of it, the anchor first); lane 63 only helps to stage tiles.
// ---------------------------------------------------------------------------
constexpr int kLanes = 63;              // rays per wavefront
constexpr int kSeg = 7;                 // bundles per wavefront

__device__ __forceinline__ int lane_segment(int lane) { return lane < kLanes ? lane / 9 : kSeg - 1; }

// ===========================================================================
// FP32 field sums: bundle moments.
//
// A ray of a bundle sits at e + delta, where e is the bundle's expansion point
// (its anchor rounded to FP32 in the set's frame, at the stage's z) and delta
// = (dx, dy, 0) its own offset, a few parsecs (all rays of a field share z).
// With D = x_j - e and s = |D|^2 + eps^2, one particle's terms at the ray,
// m (s - 2 D.delta + |delta|^2)^(-1/2) and m (D - delta) (...)^(-3/2), expand
// in delta; to second order the sums over the particles are
//
//   S0(delta) = Phi + G.delta - |delta|^2 W / 2 + 3/2 delta.T.delta
//   S(delta)  = G + 3 T.delta - W delta - 3/2 |delta|^2 V - 3 delta (V.delta)
//               + 15/2 U(delta, delta)
//
// with the moments (w = s^-3/2, q = s^-5/2, r = s^-7/2, sums over j of m_j x)
//   Phi = m s^-1/2, G_i = m w D_i, W = m w, V_i = m q D_i, T_il = m q D_i D_l,
//   U_ilk = m r D_i D_l D_k   (l, k over x and y only, as delta_z = 0).
//
// The expansion variable u = (|delta|^2 - 2 D.delta) / s has |u| <= 2 |delta|
// / sqrt(s) + |delta|^2 / s; the first neglected terms are 35/16 u^3 of the
// pair's field and 5/16 u^3 of its potential, i.e. about 1.5 u^2 and 0.6 u^2 of
// the pair's ring-minus-anchor difference (its first-order term).  A pair is
// summed this way only when sqrt(s) >= 1024 |delta|max of its bundle
// (|u| < 0.002: the neglected terms stay below 6e-6 of the pair's ring
// difference and 1e-8 of the pair term); closer pairs, and pairs within 1e-4
// Mpc of the expansion point (where s^-7/2 would leave the FP32 range), are
// left out of the moments and summed per ray directly in FP64.  Softened sets
// whose softening exceeds 1024 |delta|max for every bundle of a wavefront
// (boxes: 71 kpc against a few parsecs) skip the nearness test altogether.
// ===========================================================================
constexpr int kMom = 20;
constexpr int kKahanRounds = 256;        // rounds of plain FP32 sums between compensated adds (unguarded sums)
constexpr float kNearRatio2 = 1048576.f;   // (1024)^2
constexpr float kNearFloor2 = 1e-8f;     // (1e-4 Mpc)^2
// LDS bytes per wavefront of the FP32 path: its tile, and at least what its
// share of the moment reduction needs ([20][64] floats, [4][64] doubles, and
// the group's [20][7] double totals).
// LDS of the FP32 path, per workgroup: WPR tiles (one per wavefront index q of
// the ray groups; the NG groups of a workgroup share them), each TP float4
// (x, y in the set's frame, z relative to the stage, m, or z^2 + eps^2 for a
// set of equal masses) followed by TP float2
// (the rounding residuals of x and y).  After the last tile the same bytes hold
// the moment reduction: per wavefront [20][64] floats, [4][64] doubles and, per
// group, [20][7] double totals.
constexpr int kRedBytes = kMom * 64 * 4 + 4 * 64 * 8 + kMom * kSeg * 8;
static_assert(kRedBytes % 16 == 0, "reduction areas stay 16-byte aligned");
template <int NW, int WPR, int TP>
struct Lds32 {
  static_assert(TP % 9 == 0, "a tile holds whole rounds of the nine lanes of a bundle");
  static_assert(TP % 2 == 0, "the residuals start 16-byte aligned");
  static constexpr int kTileElems = TP * 24 / 16;                    // float4 per tile
  static constexpr int kTileBytes = WPR * TP * 24;
  static constexpr int kRed = NW * kRedBytes;
  static constexpr int kElems = ((kTileBytes > kRed) ? kTileBytes : kRed) / 16;
};

// LDS elements of a kernel's FP32 workgroup tiles (none for FP64 kernels).
template <bool F64, int NW, int WPR, int TP>
struct Lds32Elems {
  static constexpr int v = 1;
};
template <int NW, int WPR, int TP>
struct Lds32Elems<false, NW, WPR, TP> {
  static constexpr int v = Lds32<NW, WPR, TP>::kElems;
};

// Moment indices.
enum : int {
  M_PHI = 0, M_GX, M_GY, M_GZ, M_W, M_VX, M_VY, M_VZ, M_TXX, M_TXY, M_TYY, M_TZX, M_TZY,
  M_UXXX, M_UXXY, M_UXYY, M_UYYY, M_UZXX, M_UZXY, M_UZYY
};

// One (bundle, particle) pair.  p = (x, y, z relative to e, w) with x, y still
// in the set's frame and w = m / mref, or for a set of equal masses (whose pairs
// need no mass) w = z^2 + eps^2, staged once per particle; lo = the residuals of
// x and y; (ex, ey) = e.  DETECT: return whether the pair is near (s < thr);
// EXCLUDE: also leave a near pair out of the moments.
template <bool EQUAL>
__device__ __forceinline__ float pair_s(const float4 p, float Dx, float Dy, float e2) {
  const float sz = EQUAL ? p.w : fmaf(p.z, p.z, e2);
  return fmaf(Dx, Dx, fmaf(Dy, Dy, sz));
}

template <bool EQUAL, bool DETECT, bool EXCLUDE>
__device__ __forceinline__ bool moment_terms(const float4 p, const float2 lo, float ex, float ey, float e2,
                                             float thr, float (&a)[kMom]) {
  const float Dx = (p.x - ex) + lo.x, Dy = (p.y - ey) + lo.y, Dz = p.z;
  const float s = pair_s<EQUAL>(p, Dx, Dy, e2);
  float ia = __builtin_amdgcn_rsqf(s);
  const bool near = (DETECT || EXCLUDE) && s < thr;
  if constexpr (EXCLUDE) ia = near ? 0.f : ia;
  const float ia2 = ia * ia;
  const float mia = EQUAL ? ia : p.w * ia;
  a[M_PHI] += mia;
  const float w = mia * ia2;
  a[M_GX] = fmaf(w, Dx, a[M_GX]);
  a[M_GY] = fmaf(w, Dy, a[M_GY]);
  a[M_GZ] = fmaf(w, Dz, a[M_GZ]);
  a[M_W] += w;
  const float q = w * ia2;
  const float qx = q * Dx, qy = q * Dy;
  a[M_VX] += qx;
  a[M_VY] += qy;
  a[M_VZ] = fmaf(q, Dz, a[M_VZ]);
  a[M_TXX] = fmaf(Dx, qx, a[M_TXX]);
  a[M_TXY] = fmaf(Dx, qy, a[M_TXY]);
  a[M_TYY] = fmaf(Dy, qy, a[M_TYY]);
  a[M_TZX] = fmaf(Dz, qx, a[M_TZX]);
  a[M_TZY] = fmaf(Dz, qy, a[M_TZY]);
  // m s^-7/2 (Dx, Dy), from the s^-5/2 products
  const float rx = qx * ia2, ry = qy * ia2;
  const float rxx = rx * Dx, rxy = rx * Dy, ryy = ry * Dy;
  a[M_UXXX] = fmaf(Dx, rxx, a[M_UXXX]);
  a[M_UXXY] = fmaf(Dx, rxy, a[M_UXXY]);
  a[M_UXYY] = fmaf(Dx, ryy, a[M_UXYY]);
  a[M_UYYY] = fmaf(Dy, ryy, a[M_UYYY]);
  a[M_UZXX] = fmaf(Dz, rxx, a[M_UZXX]);
  a[M_UZXY] = fmaf(Dz, rxy, a[M_UZXY]);
  a[M_UZYY] = fmaf(Dz, ryy, a[M_UZYY]);
  return near;
}

// A near pair, summed directly at the ray e + (dx, dy, 0), in FP64 (such pairs
// are rare).  The nearness test repeats moment_terms' FP32 arithmetic exactly,
// so the bundle's nine lanes and the lane that left the pair out of the moments
// agree on every pair.
// (dz is the ray's height above the staged z: zero in the trace kernel, whose
// rays share z; points of a field evaluation may differ.)
template <bool EQUAL>
__device__ __forceinline__ void near_direct(const float4 p, const float2 lo, float ex, float ey, float e2,
                                            float thr, float dx, float dy, float dz, double (&d)[4]) {
  const float Dx = (p.x - ex) + lo.x, Dy = (p.y - ey) + lo.y, Dz = p.z;
  const float s = pair_s<EQUAL>(p, Dx, Dy, e2);
  if (!(s < thr)) return;
  // FP64 from here: the displacement from the particle's two-part position is
  // exact, and the term's rounding stays far below its ring-minus-anchor difference
  const double rx = (((double)p.x - ex) + lo.x) - dx, ry = (((double)p.y - ey) + lo.y) - dy;
  const double rz = (double)Dz - dz;
  const double s2 = fma(rz, rz, fma(ry, ry, fma(rx, rx, (double)e2)));
  const double ia = rsqrt_f64(s2);
  const double mia = EQUAL ? ia : (double)p.w * ia;
  const double w = mia * ia * ia;
  d[0] += mia;
  d[1] += w * rx;
  d[2] += w * ry;
  d[3] += w * rz;
}

__device__ __forceinline__ void kahan_add(float& s, float& c, float v) {
  float y = v - c;
  float t = s + y;
  c = (t - s) - y;
  s = t;
}

// This wavefront's share of the tiles of one set: Kahan-compensated moments
// (plain FP32 sums over each tile, then added with compensation) and, for a
// guarded sum, the near pairs' direct terms of the lane's own ray.  A guarded
// tile is first summed with the nearness test only; a tile that holds a near
// pair for some bundle of the wavefront is summed again with those pairs left
// out, and its near pairs are then added per ray.
template <bool EQUAL, bool DETECT, bool EXCLUDE>
__device__ __forceinline__ bool tile_moments(const float4* tile, const float2* tlo, int rounds, int l, float ex,
                                             float ey, float e2, float thr, float (&a)[kMom]) {
  bool any_near = false;
#pragma unroll 8
  for (int i = 0; i < rounds; ++i)
    any_near |= moment_terms<EQUAL, DETECT, EXCLUDE>(tile[9 * i + l], tlo[9 * i + l], ex, ey, e2, thr, a);
  return any_near;
}

// The tiles of one set, walked by all wavefronts of the workgroup in the same
// number of rounds: in round it, the NG wavefronts of index q stage tile
// q + it WPR together and each sums it for its own bundles.
template <int TP, int WPR, int NG, bool EQUAL, bool GUARD>
__device__ __forceinline__ void moment_tiles(const DevSet& s, float4* tile, int q, int g, int lane, float ex, float ey, float thr,
                             float dx, float dy, float dz, double zrel, float (&ks)[kMom], float (&kc)[kMom],
                             double (&dir)[4]) {
  const int64_t n = s.n;
  const float e2 = s.eps2f;
  const int l = lane < kLanes ? lane % 9 : 0;
  const int64_t n_tiles = (n + TP - 1) / TP;
  const int64_t n_rounds = (n_tiles + WPR - 1) / WPR;
  const float4* __restrict__ src = s.p32;
  const float4* __restrict__ src_lo = s.p32 + n;
  float2* tlo = reinterpret_cast<float2*>(tile + TP);
  // the stage's z in two FP32 parts
  const float zr_hi = (float)zrel, zr_lo = (float)(zrel - (double)zr_hi);
  // unguarded sums: plain FP32 over kKahanRounds rounds (whatever the tile size), then Kahan
  constexpr int kTilesPerKahan = (kKahanRounds * 9 + TP - 1) / TP;
  float acc[kMom];
#pragma unroll
  for (int k = 0; k < kMom; ++k) acc[k] = 0.f;
  int since = 0;
  for (int64_t it = 0; it < n_rounds; ++it) {
    const int64_t ch = q + it * WPR;
    const int64_t base = ch * TP;
    // Stage: positions in the set's frame (two parts for x and y), z relative
    // to the stage's z, and for equal masses z^2 + eps^2 in place of the mass.
    // Padding past the end lies so far away that s overflows to +inf, whose
    // reciprocal square root is +0.
    if (ch < n_tiles) {
#pragma unroll
      for (int k = 0; k < (TP + NG * 64 - 1) / (NG * 64); ++k) {
        const int j = g * 64 + lane + NG * 64 * k;
        if (j < TP) {
          float4 v = make_float4(1e30f, 1e30f, 1e30f, EQUAL ? __builtin_inff() : 0.f);
          float2 vl = make_float2(0.f, 0.f);
          if (base + j < n) {
            const float4 p = src[base + j], r = src_lo[base + j];
            const float zs = (p.z - zr_hi) + (r.z - zr_lo);
            v = make_float4(p.x, p.y, zs, EQUAL ? fmaf(zs, zs, e2) : p.w);
            vl = make_float2(r.x, r.y);
          }
          tile[j] = v;
          tlo[j] = vl;
        }
      }
    }
    __syncthreads();
    if (ch < n_tiles) {
      const int64_t left = n - base;
      // a set's last tile runs only over its particles
      const int rounds = left >= TP ? TP / 9 : (int)((left + 8) / 9);
      if constexpr (GUARD) {
        // per tile: a tile holding a near pair is summed again without it
        float a[kMom];
#pragma unroll
        for (int k = 0; k < kMom; ++k) a[k] = 0.f;
        const bool near = tile_moments<EQUAL, true, false>(tile, tlo, rounds, l, ex, ey, e2, thr, a);
        if (__any(near)) {
#pragma unroll
          for (int k = 0; k < kMom; ++k) a[k] = 0.f;
          tile_moments<EQUAL, false, true>(tile, tlo, rounds, l, ex, ey, e2, thr, a);
          const int cnt = left >= TP ? TP : (int)left;
#pragma unroll 1
          for (int j = 0; j < cnt; ++j) near_direct<EQUAL>(tile[j], tlo[j], ex, ey, e2, thr, dx, dy, dz, dir);
        }
#pragma unroll
        for (int k = 0; k < kMom; ++k) kahan_add(ks[k], kc[k], a[k]);
      } else {
        // plain sums over kKahanRounds rounds of the nine lanes, then one compensated add
        tile_moments<EQUAL, false, false>(tile, tlo, rounds, l, ex, ey, e2, thr, acc);
        if (++since >= kTilesPerKahan || ch + WPR >= n_tiles) {
#pragma unroll
          for (int k = 0; k < kMom; ++k) {
            kahan_add(ks[k], kc[k], acc[k]);
            acc[k] = 0.f;
          }
          since = 0;
        }
      }
    }
    __syncthreads();   // before the tile is staged again
  }
}

// A set of at most kSmallSet particles (point-mass lenses) is summed directly at
// every ray in FP64, with the particles read by every lane from the caller's
// array: a few FP64 pair terms per stage cost less than the moments'
// reduction, and are exact.  (Every wavefront of a workgroup takes this path for
// the same set, so it needs no barrier.)
constexpr int64_t kSmallSet = 63;

__device__ __forceinline__ void small_set_fp64(const DevCosmo& c, const DevSet& s, double x, double y, double z,
                                               double& phi, double& gx, double& gy, double& gz);

// (Every device function on the trace path is inlined into its kernel: a large
// called function reaches its far blocks through long branches, and the
// compiler builds their targets in the register pair that holds the function's
// return address.)
//
// Field of one set at the lane's ray (FP32 pair terms).  The WPR wavefronts of
// a group hold the same rays and split the tiles; all wavefronts of the
// workgroup share the staged tiles.  The group's partial moments meet in LDS
// in a fixed order, so that every wavefront of the group gets identical
// results.  Every wavefront of the workgroup must call this for the same set.
template <int NW, int WPR, int TP>
struct FieldEval32 {
  static constexpr int NG = NW / WPR;
  using L = Lds32<NW, WPR, TP>;

  __device__ __forceinline__ static void eval(const DevCosmo& c, const DevSet& s, float4* lds, int g, int q, int lane,
                                              double x, double y, double z, double& phi, double& gx, double& gy,
                                              double& gz) {
    if (s.n <= kSmallSet) {
      small_set_fp64(c, s, x, y, z, phi, gx, gy, gz);
      return;
    }
    // positions in the set's frame (FP64); each bundle's expansion point is its
    // anchor rounded to FP32; each ray's offset from it in FP32
    const double X = x - s.org[0], Yv = y - s.org[1], Zl = z - s.org[2];
    const int seg = lane_segment(lane), anchor = 9 * seg;
    const float ex = (float)__shfl(X, anchor), ey = (float)__shfl(Yv, anchor);
    const float dx = (float)(X - (double)ex), dy = (float)(Yv - (double)ey);
    // Tiles are staged with z relative to one height for the whole workgroup.
    // The expansion needs every point at that height (always so in the trace
    // kernel, whose work items are rays of one field); a wavefront with other
    // heights sums every pair directly.
    const double zrel = __shfl(Zl, 0);
    __shared__ double zshared;
    if (threadIdx.x == 0) zshared = zrel;
    __syncthreads();
    const double zwg = zshared;
    __syncthreads();
    const float dz = (float)(Zl - zwg);
    const bool level = !__any(Zl != zwg);
    // largest offset in the bundle -> nearness threshold on s
    const int l = lane < kLanes ? lane % 9 : 0;
    float m2 = lane < kLanes ? fmaf(dx, dx, dy * dy) : 0.f;
#pragma unroll
    for (int off = 1; off < 9; off <<= 1) {
      const float o = __shfl(m2, (l + off < 9) ? lane + off : lane);
      m2 = fmaxf(m2, o);
    }
    m2 = __shfl(m2, anchor);
    const float thr = level ? fmaxf(kNearRatio2 * m2, kNearFloor2) : __builtin_inff();
    // Every pair has s >= eps^2: if no bundle's threshold exceeds it, no pair can
    // be near and the unguarded loop runs.
    const bool guard = __any(thr > s.eps2f);
    float ks[kMom], kc[kMom];
#pragma unroll
    for (int k = 0; k < kMom; ++k) ks[k] = kc[k] = 0.f;
    double dir[4] = {0.0, 0.0, 0.0, 0.0};
    const bool equal = s.equal_mass && *s.equal_mass;
    float4* tile = lds + q * L::kTileElems;
    if (s.n > 0) {
      if (equal) {
        if (guard) moment_tiles<TP, WPR, NG, true, true>(s, tile, q, g, lane, ex, ey, thr, dx, dy, dz, zwg, ks, kc, dir);
        else moment_tiles<TP, WPR, NG, true, false>(s, tile, q, g, lane, ex, ey, thr, dx, dy, dz, zwg, ks, kc, dir);
      } else {
        if (guard) moment_tiles<TP, WPR, NG, false, true>(s, tile, q, g, lane, ex, ey, thr, dx, dy, dz, zwg, ks, kc, dir);
        else moment_tiles<TP, WPR, NG, false, false>(s, tile, q, g, lane, ex, ey, thr, dx, dy, dz, zwg, ks, kc, dir);
      }
    }
    // ---- reduction over the nine lanes of each bundle and the group's wavefronts
    // (the tiles are free: moment_tiles ends with a barrier)
    char* area = reinterpret_cast<char*>(lds) + g * WPR * kRedBytes;
    float* red = reinterpret_cast<float*>(area);                                   // [WPR][20][64]
    double* dred = reinterpret_cast<double*>(area + WPR * kMom * 64 * 4);          // [WPR][4][64]
    double* tot = reinterpret_cast<double*>(area + WPR * (kMom * 64 * 4 + 4 * 64 * 8));   // [20][7]
#pragma unroll
    for (int k = 0; k < kMom; ++k) red[(q * kMom + k) * 64 + lane] = ks[k] - kc[k];
#pragma unroll
    for (int k = 0; k < 4; ++k) dred[(q * 4 + k) * 64 + lane] = dir[k];
    __syncthreads();
    for (int t = q * 64 + lane; t < kMom * kSeg; t += WPR * 64) {
      const int k = t / kSeg, b = t - k * kSeg;
      double acc = 0.0;
#pragma unroll
      for (int w = 0; w < WPR; ++w)
#pragma unroll
        for (int j = 0; j < 9; ++j) acc += (double)red[(w * kMom + k) * 64 + 9 * b + j];
      tot[t] = acc;
    }
    __syncthreads();
    double M[kMom];
#pragma unroll
    for (int k = 0; k < kMom; ++k) M[k] = tot[k * kSeg + seg];
    double D0 = 0.0, D1 = 0.0, D2 = 0.0, D3 = 0.0;
#pragma unroll
    for (int w = 0; w < WPR; ++w) {
      D0 += dred[(w * 4 + 0) * 64 + lane];
      D1 += dred[(w * 4 + 1) * 64 + lane];
      D2 += dred[(w * 4 + 2) * 64 + lane];
      D3 += dred[(w * 4 + 3) * 64 + lane];
    }
    __syncthreads();   // before the tiles are staged again
    // ---- the lane's own field from the moments (FP64)
    const double ddx = dx, ddy = dy;
    const double d2 = ddx * ddx + ddy * ddy;
    const double Tx = M[M_TXX] * ddx + M[M_TXY] * ddy;
    const double Ty = M[M_TXY] * ddx + M[M_TYY] * ddy;
    const double Tz = M[M_TZX] * ddx + M[M_TZY] * ddy;
    const double Vd = M[M_VX] * ddx + M[M_VY] * ddy;
    const double xx = ddx * ddx, xy = 2.0 * ddx * ddy, yy = ddy * ddy;
    const double Ux = M[M_UXXX] * xx + M[M_UXXY] * xy + M[M_UXYY] * yy;
    const double Uy = M[M_UXXY] * xx + M[M_UXYY] * xy + M[M_UYYY] * yy;
    const double Uz = M[M_UZXX] * xx + M[M_UZXY] * xy + M[M_UZYY] * yy;
    const double W = M[M_W];
    const double S0 = M[M_PHI] + M[M_GX] * ddx + M[M_GY] * ddy - 0.5 * d2 * W + 1.5 * (ddx * Tx + ddy * Ty) + D0;
    const double Sx = M[M_GX] + 3.0 * Tx - W * ddx - 1.5 * d2 * M[M_VX] - 3.0 * ddx * Vd + 7.5 * Ux + D1;
    const double Sy = M[M_GY] + 3.0 * Ty - W * ddy - 1.5 * d2 * M[M_VY] - 3.0 * ddy * Vd + 7.5 * Uy + D2;
    const double Sz = M[M_GZ] + 3.0 * Tz - 1.5 * d2 * M[M_VZ] + 7.5 * Uz + D3;
    // the FP32 copy holds masses in units of mref; the equal-mass loop sums unit masses
    const double gm = -c.G * (equal ? s.mass : s.mref);
    phi = gm * S0;
    gx = gm * Sx;
    gy = gm * Sy;
    gz = gm * Sz;
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

// ===========================================================================
// FP64 field sums: the direct sum at each ray, tiles of the caller's FP64
// particles broadcast to every lane.
// ===========================================================================
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

__device__ __forceinline__ void small_set_fp64(const DevCosmo& c, const DevSet& s, double x, double y, double z,
                                               double& phi, double& gx, double& gy, double& gz) {
  double a0 = 0.0, a1 = 0.0, a2 = 0.0, a3 = 0.0;
  const int64_t n = s.n;
  const double* __restrict__ px = s.p64;
#pragma unroll 1
  for (int64_t j = 0; j < n; ++j)
    pair_fp64(make_double4(px[j], px[n + j], px[2 * n + j], px[3 * n + j]), x, y, z, s.eps2, a0, a1, a2, a3);
  phi = -c.G * a0;
  gx = -c.G * a1;
  gy = -c.G * a2;
  gz = -c.G * a3;
  if (s.background) {
    double U, ux, uy, uz;
    cuboid_field(s.lo, s.hi, x, y, z, U, ux, uy, uz);
    phi += c.G_rho * U;
    gx += c.G_rho * ux;
    gy += c.G_rho * uy;
    gz += c.G_rho * uz;
  }
}

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

// Field of one set at the lane's point for a group of WPR wavefronts holding
// the same rays: each sums its share of the tiles and the shares meet in LDS
// in a fixed order, so every wavefront of the group gets identical results.
// UNIT selects the loop of sets whose masses are all equal; the caller picks it
// from the set's device flag.
template <int T, int WPR>
struct FieldEval64 {
  __device__ __forceinline__ static void eval(const DevCosmo& c, const DevSet& s, double4* tile, double* red, int q,
                                              int lane, double x, double y, double z, double& phi, double& gx,
                                              double& gy, double& gz) {
    double S0, Sx, Sy, Sz;
    if (s.equal_mass && *s.equal_mass)
      sum_fp64<T, WPR, true>(s, tile, q, lane, x, y, z, S0, Sx, Sy, Sz);
    else
      sum_fp64<T, WPR, false>(s, tile, q, lane, x, y, z, S0, Sx, Sy, Sz);
    if constexpr (WPR > 1) {
      // red: [WPR][4][64] for this group
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

// ---------------------------------------------------------------------------
// The persistent trace kernel.
// NW wavefronts per workgroup; WPR of them share 63 rays (7 bundles) and split
// the particles; T particles per tile; OCC wavefronts per SIMD requested (the
// register budget is 512 / OCC per lane).
// ---------------------------------------------------------------------------
template <bool F64, int NW, int WPR, int T, int OCC>
__global__ __launch_bounds__(NW * 64) __attribute__((amdgpu_waves_per_eu(OCC, OCC))) void trace_kernel(TraceParams P) {
  constexpr int NG = NW / WPR;
  // FP64: a tile per wavefront; FP32: workgroup tiles (Lds32)
  __shared__ double4 tiles64[F64 ? NW : 1][F64 ? T : 1];
  __shared__ double red_own[NG][(F64 && WPR > 1) ? WPR * 4 * 64 : 1];
  __shared__ float4 lds32[Lds32Elems<F64, NW, WPR, T>::v];
  __shared__ int s_item;

  // the wavefront index is uniform: keep it (and the tile loop counters) in SGPRs
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int g = wave / WPR, q = wave % WPR;
  const DevCosmo& cz = P.cosmo;

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
        double phi = 0.0, gx = 0.0, gy = 0.0, gz = 0.0;
        if (S >= 0) {
          const DevSet& set = P.sets[f.set_off + S];
          if constexpr (F64)
            FieldEval64<T, WPR>::eval(cz, set, tiles64[wave], &red_own[g][0], q, lane, xin, yin, zs, phi, gx, gy,
                                      gz);
          else
            FieldEval32<NW, WPR, T>::eval(cz, set, lds32, g, q, lane, xin, yin, zs, phi, gx, gy, gz);
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
// Every group of 9 consecutive points is treated as a bundle: FP32 sums expand
// about the first point of the group (rounded to FP32), as the trace kernel
// does about a bundle's anchor, when the points of the workgroup share z
// (otherwise each point's sum is direct).  Wavefronts past the last point still
// take part in the workgroup's tile rounds, on a copy of the last point.
template <bool F64, int T>
__global__ __launch_bounds__(256) void field_eval_kernel(DevCosmo c, const DevSet* set_p, int64_t n,
                                                         const double* pts, double* phi, double* grad) {
  __shared__ double4 tiles64[F64 ? 4 : 1][F64 ? T : 1];
  __shared__ float4 lds32[Lds32Elems<F64, 4, 1, T>::v];
  // the wavefront index is uniform: keep it (and the tile loop counters) in SGPRs
  const int wave = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6), lane = threadIdx.x & 63;
  const int64_t w0 = ((int64_t)blockIdx.x * 4 + wave) * kLanes;
  int64_t i = w0 + (lane < kLanes ? lane : kLanes - 1);
  const bool valid = lane < kLanes && i < n;
  if (i >= n) i = n - 1;
  const DevSet set = *set_p;
  double p, gx, gy, gz;
  if constexpr (F64) {
    if (w0 >= n) return;   // whole wavefront idle (no workgroup barriers in this path)
    FieldEval64<T, 1>::eval(c, set, tiles64[wave], nullptr, 0, lane, pts[i], pts[n + i], pts[2 * n + i], p, gx, gy,
                            gz);
  } else {
    FieldEval32<4, 1, T>::eval(c, set, lds32, wave, 0, lane, pts[i], pts[n + i], pts[2 * n + i], p, gx, gy, gz);
  }
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
  s.mref = (s.mass != 0.0 && isfinite(s.mass)) ? s.mass : 1.0;
  if (s.equal_mass) *s.equal_mass = 1;   // cleared by the FP32 conversion at the first other mass
  if (s.background) {
    for (int d = 0; d < 3; ++d) s.org[d] = 0.5 * (s.lo[d] + s.hi[d]);
  } else if (s.n > 0) {
    for (int d = 0; d < 3; ++d) s.org[d] = s.p64[d * s.n];
  } else {
    for (int d = 0; d < 3; ++d) s.org[d] = 0.0;
  }
}

// The FP32 copy: positions relative to the set's frame origin as an FP32 value
// and its FP32 rounding residual (so that the FP32 displacement from a ray is
// rounded once relative to the particle-ray distance, not to the particle's
// distance from the frame origin), masses in units of the set's first mass (1 if
// that is 0), which multiplies the finished sums, so that the moments' powers of
// 1/r stay inside the FP32 range for any mass scale.
__global__ void convert_set_kernel(const DevSet* set, const double* p64, float4* p32, int64_t n) {
  const int64_t j = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  if (j >= n) return;
  const double ox = set->org[0], oy = set->org[1], oz = set->org[2];
  const double m = p64[3 * n + j];
  if (p32) {   // (FP64 sets have no copy: only their masses are checked)
    const double x = p64[j] - ox, y = p64[n + j] - oy, z = p64[2 * n + j] - oz;
    const float xh = (float)x, yh = (float)y, zh = (float)z;
    p32[j] = make_float4(xh, yh, zh, (float)(m / set->mref));
    p32[n + j] = make_float4((float)(x - (double)xh), (float)(y - (double)yh), (float)(z - (double)zh), 0.f);
  }
  if (!(m == p64[3 * n])) *set->equal_mass = 0;   // (a NaN mass also takes the general path)
}

// ---------------------------------------------------------------------------
// Bundle construction (Sec. 3.1): one thread per ray.
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
// Bundle reduction (Sec. 3.1, eq. lensmap, magnification): 9 consecutive lanes
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
// Bundle flexion (Sec. 6: flexion, the gradient of the shear, through ray
// bundles).  About the anchor, the ring offsets are
//   D_k = chi_s (r A e_k + 1/2 r^2 Dm(e_k, e_k)) + O(r^3),
// e_k = (cos 2 pi k / 8, sin 2 pi k / 8), Dm_ijl = d A_ij / d theta_l.  Over the
// eight ring rays the first- and third-order parts live in the harmonics 1 and
// 3 only, so the harmonics 0 and 2 hold Dm alone:
//   sum_k D_ik = 2 r^2 chi_s (Dm_i11 + Dm_i22),
//   sum_k D_ik cos 2 phi_k = r^2 chi_s (Dm_i11 - Dm_i22),
//   sum_k D_ik sin 2 phi_k = 2 r^2 chi_s Dm_i12
// (cos 2 phi_k and sin 2 phi_k are exactly 0 or +-1).  F = grad kappa and
// G = (d1 gamma1 - d2 gamma2, d2 gamma1 + d1 gamma2) with kappa, gamma read from
// A as in magnification_kernel.  Same 9-lane layout as magnification_kernel.
// ---------------------------------------------------------------------------
__global__ __launch_bounds__(256) void flexion_kernel(double chi_s, int64_t nb, double radius, const double* rays,
                                                      double* flex, double* dm) {
  const int wave = threadIdx.x >> 6, lane = threadIdx.x & 63;
  const int seg = lane / 9, k = lane % 9;
  const int64_t b = ((int64_t)blockIdx.x * 4 + wave) * 7 + seg;
  const bool valid = (seg < 7) && (b < nb);
  const int64_t N = 9 * nb;
  const int64_t r = valid ? 9 * b + k : 0;
  const double x = rays[N + r], y = rays[2 * N + r];
  const int anchor = seg * 9;
  const double dx = x - __shfl(x, anchor), dy = y - __shfl(y, anchor);
  double v[6] = {0.0, 0.0, 0.0, 0.0, 0.0, 0.0};
  if (k > 0) {
    const int q = (k - 1) & 3;   // 2 phi_k = q pi / 2 (mod 2 pi)
    const double c2 = q == 0 ? 1.0 : (q == 2 ? -1.0 : 0.0);
    const double s2 = q == 1 ? 1.0 : (q == 3 ? -1.0 : 0.0);
    v[0] = dx;
    v[1] = dy;
    v[2] = dx * c2;
    v[3] = dy * c2;
    v[4] = dx * s2;
    v[5] = dy * s2;
  }
#pragma unroll
  for (int off = 1; off < 9; off <<= 1) {
    const int src = (k + off < 9) ? lane + off : lane;
#pragma unroll
    for (int m = 0; m < 6; ++m) {
      const double o = __shfl(v[m], src);
      if (k + off < 9) v[m] += o;
    }
  }
  if (valid && k == 0) {
    const double u = 1.0 / (radius * radius * chi_s);
    const double tx = 0.5 * v[0] * u, ty = 0.5 * v[1] * u;   // Dm_x11 + Dm_x22, Dm_y11 + Dm_y22
    const double ex = v[2] * u, ey = v[3] * u;               // Dm_x11 - Dm_x22, Dm_y11 - Dm_y22
    const double d111 = 0.5 * (tx + ex), d122 = 0.5 * (tx - ex), d112 = 0.5 * v[4] * u;
    const double d211 = 0.5 * (ty + ey), d222 = 0.5 * (ty - ey), d212 = 0.5 * v[5] * u;
    // kappa = 1 - (A11 + A22) / 2, gamma1 = (A22 - A11) / 2, gamma2 = -(A12 + A21) / 2
    const double dk1 = -0.5 * (d111 + d212), dk2 = -0.5 * (d112 + d222);
    const double dg1_1 = 0.5 * (d212 - d111), dg1_2 = 0.5 * (d222 - d112);
    const double dg2_1 = -0.5 * (d112 + d211), dg2_2 = -0.5 * (d122 + d212);
    flex[b] = dk1;
    flex[nb + b] = dk2;
    flex[2 * nb + b] = dg1_1 - dg2_2;
    flex[3 * nb + b] = dg1_2 + dg2_1;
    if (dm) {
      dm[b] = d111;
      dm[nb + b] = d112;
      dm[2 * nb + b] = d122;
      dm[3 * nb + b] = d211;
      dm[4 * nb + b] = d212;
      dm[5 * nb + b] = d222;
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
  int nw, wpr, tile, occ;
};

// FP32: the workgroup's tiles and reduction area take at most 66 KB of LDS, so
// two workgroups of 8 wavefronts (four per SIMD, 128 registers) or three of 4
// (three per SIMD, 168 registers) fit a compute unit.
constexpr PlanShape kPlans32[] = {{8, 1, 576, 4}, {8, 2, 576, 4}, {8, 4, 576, 4}, {8, 8, 288, 4},
                                  {8, 1, 1152, 4}, {8, 2, 1152, 4}, {4, 1, 576, 3}, {4, 4, 288, 3},
                                  {8, 1, 2304, 4}};
constexpr PlanShape kPlans64[] = {{8, 1, 128, 4}, {8, 2, 128, 4}, {8, 4, 128, 4},
                                  {8, 8, 64, 4},  {4, 1, 128, 4}, {4, 4, 128, 4}};
constexpr int kNumPlans32 = sizeof(kPlans32) / sizeof(kPlans32[0]);
constexpr int kNumPlans64 = sizeof(kPlans64) / sizeof(kPlans64[0]);

template <bool F64, int I>
struct PlanKernel {
  static constexpr PlanShape S = F64 ? kPlans64[I] : kPlans32[I];
  static const void* fn() { return (const void*)&trace_kernel<F64, S.nw, S.wpr, S.tile, S.occ>; }
  static hipError_t launch(const TraceParams& p, int grid, hipStream_t st) {
    hipLaunchKernelGGL((trace_kernel<F64, S.nw, S.wpr, S.tile, S.occ>), dim3(grid), dim3(S.nw * 64), 0, st, p);
    return hipGetLastError();
  }
};

template <bool F64, int I = 0>
const void* plan_fn(int id) {
  constexpr int n = F64 ? kNumPlans64 : kNumPlans32;
  if constexpr (I + 1 < n) {
    if (id != I) return plan_fn<F64, I + 1>(id);
  }
  return PlanKernel<F64, I>::fn();
}

template <bool F64, int I = 0>
hipError_t plan_launch(int id, const TraceParams& p, int grid, hipStream_t st) {
  constexpr int n = F64 ? kNumPlans64 : kNumPlans32;
  if constexpr (I + 1 < n) {
    if (id != I) return plan_launch<F64, I + 1>(id, p, grid, st);
  }
  return PlanKernel<F64, I>::launch(p, grid, st);
}

}  // namespace

int plan_count(bool fp64) { return fp64 ? kNumPlans64 : kNumPlans32; }

rt_plan_info plan_info(bool fp64, int id) {
  const PlanShape s = fp64 ? kPlans64[id] : kPlans32[id];
  rt_plan_info r;
  r.waves_per_block = s.nw;
  r.waves_per_group = s.wpr;
  r.tile = s.tile;
  r.rays_per_block = kLanes * s.nw / s.wpr;
  r.waves_per_simd = s.occ;
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

hipError_t launch_flexion(double chi_s, int64_t nb, double radius, const double* rays, double* flex, double* dm,
                          hipStream_t s) {
  if (nb <= 0) return hipSuccess;
  const int64_t waves = (nb + 6) / 7;
  hipLaunchKernelGGL(flexion_kernel, dim3((unsigned)((waves + 3) / 4)), dim3(256), 0, s, chi_s, nb, radius, rays,
                     flex, dm);
  return hipGetLastError();
}

// ---------------------------------------------------------------------------
// Scratch of the histogram entry point that allocates nothing
// (rt_mu_histogram_noalloc): the bin weights and the five sums of one call,
// for at most kNoAllocBins bins.  Each GPU holds its own copy of the array;
// host code uses the per-device address from hipGetSymbolAddress, never the
// array's name.
// ---------------------------------------------------------------------------
constexpr int kNoAllocBins = 65536;
static __device__ __align__(256) double scratch[kNoAllocBins + 8];

hipError_t noalloc_scratch(double** out, int32_t* max_bins) {
  static std::mutex mu;
  static std::map<int, void*> addr;   // device -> address of its copy of scratch
  int dev;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  std::lock_guard<std::mutex> lk(mu);
  auto it = addr.find(dev);
  if (it == addr.end()) {
    void* ptr = nullptr;
    e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    it = addr.emplace(dev, ptr).first;
  }
  *out = static_cast<double*>(it->second);
  *max_bins = kNoAllocBins;
  return hipSuccess;
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
