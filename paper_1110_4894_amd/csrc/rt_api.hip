// Host side of librt: argument validation, background cosmology, schedules,
// device descriptor tables, the captured-graph cache and the plan tuner.
// Every entry point is declared, with its contract, in include/rt.h.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <array>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <map>
#include <memory>
#include <mutex>
#include <string>
#include <tuple>
#include <vector>

#include "rt_internal.h"

using namespace rt;

namespace {

// ---------------------------------------------------------------- errors
thread_local std::string g_err;

rt_status fail(rt_status st, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return st;
}

// A C caller may pass any int for an rt_precision, and reading an enum object
// that holds no enumerator's value is undefined in C++: look at its bytes.
bool valid_precision(const rt_precision& p) {
  int32_t v;
  static_assert(sizeof(p) == sizeof(v), "rt_precision is an int");
  std::memcpy(&v, &p, sizeof(v));
  return v == 0 || v == 1;   // RT_FP64, RT_FP32_KAHAN
}

#define RT_HIP(expr)                                                                       \
  do {                                                                                     \
    hipError_t e_ = (expr);                                                                \
    if (e_ != hipSuccess) return fail(RT_ERR_DEVICE, "%s failed: %s", #expr, hipGetErrorString(e_)); \
  } while (0)

// A stream-ordered scratch allocation that is freed on every return path (an
// argument or device error after the allocation included).
struct StreamScratch {
  void* p = nullptr;
  hipStream_t s;
  explicit StreamScratch(hipStream_t st) : s(st) {}
  StreamScratch(const StreamScratch&) = delete;
  StreamScratch& operator=(const StreamScratch&) = delete;
  hipError_t alloc(size_t bytes) { return hipMallocAsync(&p, bytes, s); }
  hipError_t release() {
    const hipError_t e = p ? hipFreeAsync(p, s) : hipSuccess;
    p = nullptr;
    return e;
  }
  ~StreamScratch() {
    if (p) (void)hipFreeAsync(p, s);
  }
};

// ---------------------------------------------------------------- constants and background
// GM_sun (IAU 2012 nominal), c (exact), 1 Mpc = 3.0856775814913673e22 m (IAU 2015).
constexpr double kGMsun = 1.32712440018e20;
constexpr double kCsi = 299792458.0;
constexpr double kMpcM = 3.0856775814913673e22;
constexpr double kCkms = 299792.458;

inline double g_over_c2() { return kGMsun / (kCsi * kCsi) / kMpcM; }

rt_status check_cosmo(const rt_cosmology* c) {
  if (!c) return fail(RT_ERR_INVALID_ARG, "cosmo is NULL");
  if (!std::isfinite(c->omega_m) || !std::isfinite(c->omega_lambda) || !std::isfinite(c->h))
    return fail(RT_ERR_NONFINITE, "cosmology has a non-finite parameter");
  if (!(c->omega_m > 0.0) || !(c->omega_lambda > 0.0) || !(c->h > 0.0))
    return fail(RT_ERR_COSMOLOGY, "cosmology needs omega_m > 0, omega_lambda > 0, h > 0");
  if (std::fabs(c->omega_m + c->omega_lambda - 1.0) > 1e-12)
    return fail(RT_ERR_COSMOLOGY, "cosmology is not flat: omega_m + omega_lambda = %.17g", c->omega_m + c->omega_lambda);
  return RT_OK;
}

double hubble0(const rt_cosmology& c) { return 100.0 * c.h / kCkms; }

// Romberg integration of 1 / E(z) on [0, z] (Sec. 5.1, eq. raytracedistance).
double comoving_distance(const rt_cosmology& c, double z) {
  if (z <= 0.0) return 0.0;
  auto f = [&](double x) {
    const double zp = 1.0 + x;
    return 1.0 / std::sqrt(c.omega_m * zp * zp * zp + c.omega_lambda);
  };
  double R[24][24];
  double h = z;
  R[0][0] = 0.5 * h * (f(0.0) + f(z));
  double result = R[0][0];
  for (int n = 1; n < 24; ++n) {
    h *= 0.5;
    double s = 0.0;
    const long m = 1L << (n - 1);
    for (long i = 0; i < m; ++i) s += f((2 * i + 1) * h);
    R[n][0] = 0.5 * R[n - 1][0] + h * s;
    double p = 1.0;
    for (int k = 1; k <= n; ++k) {
      p *= 4.0;
      R[n][k] = R[n][k - 1] + (R[n][k - 1] - R[n - 1][k - 1]) / (p - 1.0);
    }
    result = R[n][n];
    if (n >= 5 && std::fabs(R[n][n] - R[n - 1][n - 1]) <= 1e-15 * std::fabs(R[n][n])) break;
  }
  return result / hubble0(c);
}

DevCosmo make_dev_cosmo(const rt_cosmology& c) {
  DevCosmo d;
  d.H0 = hubble0(c);
  d.sqrt_ol = std::sqrt(c.omega_lambda);
  d.ratio = c.omega_m / c.omega_lambda;
  // eq. lookbacksingularity with the square root that makes a(0) = 1
  d.t0 = 2.0 / (3.0 * d.H0 * d.sqrt_ol) * std::asinh(std::sqrt(c.omega_lambda / c.omega_m));
  d.G = g_over_c2();
  const double rho_c0 = 3.0 * d.H0 * d.H0 / (8.0 * M_PI * d.G);
  d.G_rho = d.G * c.omega_m * rho_c0;
  return d;
}

// ---------------------------------------------------------------- validation of fields
rt_status check_set(const rt_particle_set& s, int f, int j) {
  if (s.n < 0) return fail(RT_ERR_INVALID_ARG, "fields[%d].sets[%d].n < 0", f, j);
  if (s.n > 0 && !s.xyzm) return fail(RT_ERR_INVALID_ARG, "fields[%d].sets[%d].xyzm is NULL", f, j);
  if (s.n > (int64_t)1 << 31) return fail(RT_ERR_UNSUPPORTED, "fields[%d].sets[%d].n exceeds 2^31", f, j);
  if (!std::isfinite(s.softening)) return fail(RT_ERR_NONFINITE, "fields[%d].sets[%d].softening", f, j);
  if (s.softening < 0.0) return fail(RT_ERR_INVALID_ARG, "fields[%d].sets[%d].softening < 0", f, j);
  if (s.background != 0 && s.background != 1)
    return fail(RT_ERR_INVALID_ARG, "fields[%d].sets[%d].background must be 0 or 1", f, j);
  if (s.background) {
    for (int d = 0; d < 3; ++d) {
      if (!std::isfinite(s.lo[d]) || !std::isfinite(s.hi[d]))
        return fail(RT_ERR_NONFINITE, "fields[%d].sets[%d] cuboid bound", f, j);
      if (!(s.lo[d] < s.hi[d])) return fail(RT_ERR_INVALID_ARG, "fields[%d].sets[%d] cuboid needs lo < hi", f, j);
    }
  }
  return RT_OK;
}

rt_status check_fields(const rt_field* fields, int32_t n_fields, int64_t n_bundles, double chi_s, bool need_nodes) {
  if (n_fields < 0) return fail(RT_ERR_INVALID_ARG, "n_fields < 0");
  if (n_fields > 0 && !fields) return fail(RT_ERR_INVALID_ARG, "fields is NULL");
  std::vector<std::pair<int64_t, int64_t>> ranges;
  for (int f = 0; f < n_fields; ++f) {
    const rt_field& F = fields[f];
    if (F.n_sets < 0 || (F.n_sets > 0 && !F.sets)) return fail(RT_ERR_INVALID_ARG, "fields[%d].sets", f);
    for (int j = 0; j < F.n_sets; ++j) {
      rt_status st = check_set(F.sets[j], f, j);
      if (st != RT_OK) return st;
    }
    if (F.n_steps < 1) return fail(RT_ERR_SCHEDULE, "fields[%d].n_steps < 1", f);
    if (!F.z_nodes || !F.step_set) return fail(RT_ERR_INVALID_ARG, "fields[%d] z_nodes or step_set is NULL", f);
    if (F.bundle_offset < 0 || F.n_bundles < 0 || F.bundle_offset + F.n_bundles > n_bundles)
      return fail(RT_ERR_INVALID_ARG, "fields[%d] bundle range [%lld, %lld) outside [0, %lld)", f,
                  (long long)F.bundle_offset, (long long)(F.bundle_offset + F.n_bundles), (long long)n_bundles);
    for (int s = 0; s < F.n_steps; ++s) {
      if (F.step_set[s] < -1 || F.step_set[s] >= F.n_sets)
        return fail(RT_ERR_INVALID_ARG, "fields[%d].step_set[%d] = %d out of [-1, %d)", f, s, F.step_set[s], F.n_sets);
    }
    if (need_nodes) {
      if (F.z_nodes[0] != 0.0) return fail(RT_ERR_SCHEDULE, "fields[%d].z_nodes[0] != 0", f);
      for (int s = 0; s < F.n_steps; ++s) {
        if (!std::isfinite(F.z_nodes[s + 1])) return fail(RT_ERR_NONFINITE, "fields[%d].z_nodes[%d]", f, s + 1);
        if (!(F.z_nodes[s + 1] > F.z_nodes[s]))
          return fail(RT_ERR_SCHEDULE, "fields[%d].z_nodes not strictly increasing at %d", f, s + 1);
      }
      if (std::fabs(F.z_nodes[F.n_steps] - chi_s) > 1e-9 * chi_s)
        return fail(RT_ERR_SCHEDULE, "fields[%d] last node %.17g differs from chi_s %.17g", f, F.z_nodes[F.n_steps],
                    chi_s);
    }
    if (F.n_bundles > 0) ranges.emplace_back(F.bundle_offset, F.bundle_offset + F.n_bundles);
  }
  std::sort(ranges.begin(), ranges.end());
  for (size_t i = 1; i < ranges.size(); ++i)
    if (ranges[i].first < ranges[i - 1].second) return fail(RT_ERR_INVALID_ARG, "field bundle ranges overlap");
  return RT_OK;
}

// ---------------------------------------------------------------- device properties
struct DeviceInfo {
  int id = -1;
  int n_cu = 0;
};

rt_status device_info(DeviceInfo* out) {
  int dev;
  RT_HIP(hipGetDevice(&dev));
  static std::mutex mu;
  static std::map<int, int> cache;
  std::lock_guard<std::mutex> lk(mu);
  auto it = cache.find(dev);
  if (it == cache.end()) {
    int n;
    RT_HIP(hipDeviceGetAttribute(&n, hipDeviceAttributeMultiprocessorCount, dev));
    it = cache.emplace(dev, n).first;
  }
  out->id = dev;
  out->n_cu = it->second;
  return RT_OK;
}

// ---------------------------------------------------------------- trace plans and cache
struct Buffer {
  void* p = nullptr;
  ~Buffer() {
    if (p) (void)hipFree(p);
  }
};

struct TraceEntry {
  std::vector<uint8_t> key;
  int device = -1;
  bool fp64 = false;
  int plan = 0;
  std::vector<std::unique_ptr<Buffer>> owned;
  TraceParams params{};
  DevSet* d_sets = nullptr;
  int32_t n_sets_total = 0;
  struct Conv {
    int32_t set_index;
    const double* p64;
    float4* p32;
    int64_t n;
  };
  std::vector<Conv> conv;
  int grid = 0;
  int n_items = 0;
  double interactions = 0.0;
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  hipEvent_t done = nullptr;   // recorded after every launch of the graph
  bool pinned = false;         // launched into a caller's graph: kept until rt_release_caches
  ~TraceEntry() {
    // an evicted entry may still be running: its buffers are freed only after it ends
    if (done) {
      (void)hipEventSynchronize(done);
      (void)hipEventDestroy(done);
    }
    if (exec) (void)hipGraphExecDestroy(exec);
    if (graph) (void)hipGraphDestroy(graph);
  }
};

struct State {
  std::mutex mu;
  std::vector<std::unique_ptr<TraceEntry>> cache;   // most recent last
  int forced[2] = {-1, -1};
  int grid_limit = 0;
  std::map<std::tuple<int, int, int, int>, int> tuned;   // (device, fp64, log2 rays, log2 mean np) -> plan
  hipStream_t capture_stream[64] = {};
  bool timing = false;
  hipEvent_t ev0 = nullptr, ev1 = nullptr;
  bool timed_last = false;
  rt_trace_info last{};
} g;

// Configurations kept (a benchmark walks 20 step windows of one band, and each
// window is a configuration of its own).
constexpr size_t kMaxEntries = 24;

template <class T>
void put(std::vector<uint8_t>& k, const T& v) {
  const uint8_t* p = reinterpret_cast<const uint8_t*>(&v);
  k.insert(k.end(), p, p + sizeof(T));
}

void put_bytes(std::vector<uint8_t>& k, const void* p, size_t n) {
  const uint8_t* b = reinterpret_cast<const uint8_t*>(p);
  k.insert(k.end(), b, b + n);
}

std::vector<uint8_t> make_key(int dev, const rt_cosmology& c, const rt_field* fields, int32_t n_fields, bool fp64,
                              int plan, int32_t sb, int32_t se, int64_t nb, const double* rays, const uint8_t* flags) {
  std::vector<uint8_t> k;
  put(k, dev);
  put(k, c);
  put(k, fp64);
  put(k, plan);
  put(k, sb);
  put(k, se);
  put(k, nb);
  put(k, rays);
  put(k, flags);
  put(k, g.grid_limit);
  put(k, n_fields);
  for (int f = 0; f < n_fields; ++f) {
    const rt_field& F = fields[f];
    put(k, F.n_sets);
    put(k, F.n_steps);
    put(k, F.bundle_offset);
    put(k, F.n_bundles);
    put_bytes(k, F.z_nodes, sizeof(double) * (F.n_steps + 1));
    put_bytes(k, F.step_set, sizeof(int32_t) * F.n_steps);
    for (int j = 0; j < F.n_sets; ++j) {
      const rt_particle_set& s = F.sets[j];
      put(k, s.n);
      put(k, s.xyzm);
      put(k, s.softening);
      put(k, s.background);
      put_bytes(k, s.lo, sizeof(s.lo));
      put_bytes(k, s.hi, sizeof(s.hi));
    }
  }
  return k;
}

int ilog2(double v) { return v <= 1.0 ? 0 : (int)std::floor(std::log2(v)); }

struct Workload {
  double rays = 0.0;         // total rays
  double mean_np = 0.0;      // particles per step, averaged over rays and steps
  double interactions = 0.0;
};

Workload describe(const rt_field* fields, int32_t n_fields, int32_t sb, int32_t se) {
  Workload w;
  double ray_steps = 0.0;
  for (int f = 0; f < n_fields; ++f) {
    const rt_field& F = fields[f];
    const double nr = 9.0 * (double)F.n_bundles;
    const int b = std::max(sb, 0), e = std::min(se, F.n_steps);
    double np = 0.0;
    for (int s = b; s < e; ++s)
      if (F.step_set[s] >= 0) np += (double)F.sets[F.step_set[s]].n;
    w.rays += nr;
    w.interactions += nr * 4.0 * np;
    ray_steps += nr * std::max(0, e - b);
  }
  w.mean_np = ray_steps > 0 ? w.interactions / 4.0 / ray_steps : 0.0;
  return w;
}

// Default plan: split the particles over enough wavefronts to give every SIMD
// at least four of them, while every share keeps several tiles.
// Without a tuned plan: enough wavefronts for about four per SIMD (several
// wavefronts share a ray group when there are few rays and many particles),
// and for FP32 the larger tiles when the sets fill them.
int heuristic_plan(bool fp64, const Workload& w, int n_cu) {
  const double waves = w.rays / 64.0;
  const double target = 0.9 * 16.0 * n_cu;
  const int tile = plan_info(fp64, 0).tile;
  int wpr = 1;
  while (wpr < 8 && waves * wpr < target && w.mean_np >= 4.0 * tile * wpr * 2) wpr *= 2;
  if (!fp64) {
    // the plan of 8 wavefronts with this sharing and the largest tile the sets fill
    int best = -1, best_tile = 0;
    for (int id = 0; id < plan_count(false); ++id) {
      const rt_plan_info p = plan_info(false, id);
      if (p.waves_per_block == 8 && p.waves_per_group == wpr && p.waves_per_simd == 4 && p.tile > best_tile &&
          w.mean_np >= 4.0 * p.tile) {
        best = id;
        best_tile = p.tile;
      }
    }
    if (best >= 0) return best;
  }
  switch (wpr) {
    case 1: return 0;
    case 2: return 1;
    case 4: return 2;
    default: return 3;
  }
}

template <class T>
rt_status dev_alloc(TraceEntry* e, T** out, size_t count) {
  auto b = std::make_unique<Buffer>();
  if (count == 0) count = 1;
  hipError_t err = hipMalloc(&b->p, sizeof(T) * count);
  if (err != hipSuccess) {
    b->p = nullptr;
    return fail(RT_ERR_OUT_OF_MEMORY, "hipMalloc of %zu bytes failed: %s", sizeof(T) * count, hipGetErrorString(err));
  }
  *out = static_cast<T*>(b->p);
  e->owned.push_back(std::move(b));
  return RT_OK;
}

// Build the device tables of one rt_trace configuration (uploads synchronously).
rt_status build_entry(TraceEntry* e, const DeviceInfo& di, const rt_cosmology& c, const rt_field* fields,
                      int32_t n_fields, bool fp64, int plan, int32_t sb, int32_t se, int64_t nb, double* rays,
                      uint8_t* flags) {
  e->device = di.id;
  e->fp64 = fp64;
  e->plan = plan;
  const rt_plan_info pi = plan_info(fp64, plan);
  std::vector<DevField> hf(n_fields);
  std::vector<DevSet> hs;
  std::vector<double> nodes;
  std::vector<int32_t> steps;
  std::vector<std::pair<double, WorkItem>> items;
  // One FP32 copy per particle array and frame: the frame origin depends on the
  // background cuboid, so the key holds it too.
  using ConvKey = std::tuple<const double*, int64_t, int32_t, std::array<double, 6>>;
  std::map<ConvKey, std::pair<float4*, int32_t*>> p32_of;
  for (int f = 0; f < n_fields; ++f) {
    const rt_field& F = fields[f];
    DevField& d = hf[f];
    d.ray_begin = 9 * F.bundle_offset;
    d.n_rays = 9 * F.n_bundles;
    d.n_steps = F.n_steps;
    d.node_off = (int32_t)nodes.size();
    d.step_off = (int32_t)steps.size();
    d.set_off = (int32_t)hs.size();
    nodes.insert(nodes.end(), F.z_nodes, F.z_nodes + F.n_steps + 1);
    steps.insert(steps.end(), F.step_set, F.step_set + F.n_steps);
    for (int j = 0; j < F.n_sets; ++j) {
      const rt_particle_set& s = F.sets[j];
      DevSet ds{};
      ds.p64 = s.xyzm;
      ds.n = s.n;
      ds.eps2 = s.softening * s.softening;
      ds.eps2f = (float)ds.eps2;
      ds.background = s.background;
      for (int k = 0; k < 3; ++k) {
        ds.lo[k] = s.lo[k];
        ds.hi[k] = s.hi[k];
      }
      ds.p32 = nullptr;
      if (s.n > 0) {
        std::array<double, 6> box{};
        if (s.background) box = {s.lo[0], s.lo[1], s.lo[2], s.hi[0], s.hi[1], s.hi[2]};
        const ConvKey key{s.xyzm, s.n, s.background, box};
        auto it = p32_of.find(key);
        if (it == p32_of.end()) {
          float4* p = nullptr;   // FP64 traces keep no copy; their masses are still checked
          int32_t* eq;
          rt_status st;
          if (!fp64 && (st = dev_alloc(e, &p, 2 * (size_t)s.n)) != RT_OK) return st;
          if ((st = dev_alloc(e, &eq, 1)) != RT_OK) return st;
          it = p32_of.emplace(key, std::make_pair(p, eq)).first;
          e->conv.push_back({(int32_t)hs.size(), s.xyzm, p, s.n});
        }
        ds.p32 = it->second.first;
        ds.equal_mass = it->second.second;
      }
      hs.push_back(ds);
    }
    if (F.n_bundles <= 0) continue;
    const int b0 = std::max(sb, 0), b1 = std::min(se, F.n_steps);
    double np = 0.0;
    for (int s = b0; s < b1; ++s)
      if (F.step_set[s] >= 0) np += (double)F.sets[F.step_set[s]].n;
    const double per_ray = np + 64.0 * std::max(0, b1 - b0);
    const int64_t n_rays = 9 * F.n_bundles;
    const int64_t n_blocks = (n_rays + pi.rays_per_block - 1) / pi.rays_per_block;
    for (int64_t b = 0; b < n_blocks; ++b) {
      const double r = (double)std::min<int64_t>(pi.rays_per_block, n_rays - b * pi.rays_per_block);
      items.push_back({r * per_ray, WorkItem{f, (int32_t)b}});
    }
  }
  // largest first, so that the long items start early
  std::stable_sort(items.begin(), items.end(),
                   [](const std::pair<double, WorkItem>& a, const std::pair<double, WorkItem>& b) {
                     return a.first > b.first;
                   });
  std::vector<WorkItem> hitems(items.size());
  for (size_t i = 0; i < items.size(); ++i) hitems[i] = items[i].second;

  DevField* d_fields;
  double* d_nodes;
  int32_t* d_steps;
  WorkItem* d_items;
  int32_t* d_queue;
  rt_status st;
  if ((st = dev_alloc(e, &d_fields, hf.size())) != RT_OK) return st;
  if ((st = dev_alloc(e, &e->d_sets, hs.size())) != RT_OK) return st;
  if ((st = dev_alloc(e, &d_nodes, nodes.size())) != RT_OK) return st;
  if ((st = dev_alloc(e, &d_steps, steps.size())) != RT_OK) return st;
  if ((st = dev_alloc(e, &d_items, hitems.size())) != RT_OK) return st;
  if ((st = dev_alloc(e, &d_queue, 1)) != RT_OK) return st;
  if (!hf.empty()) RT_HIP(hipMemcpy(d_fields, hf.data(), sizeof(DevField) * hf.size(), hipMemcpyHostToDevice));
  if (!hs.empty()) RT_HIP(hipMemcpy(e->d_sets, hs.data(), sizeof(DevSet) * hs.size(), hipMemcpyHostToDevice));
  if (!nodes.empty()) RT_HIP(hipMemcpy(d_nodes, nodes.data(), sizeof(double) * nodes.size(), hipMemcpyHostToDevice));
  if (!steps.empty()) RT_HIP(hipMemcpy(d_steps, steps.data(), sizeof(int32_t) * steps.size(), hipMemcpyHostToDevice));
  if (!hitems.empty())
    RT_HIP(hipMemcpy(d_items, hitems.data(), sizeof(WorkItem) * hitems.size(), hipMemcpyHostToDevice));
  e->n_sets_total = (int32_t)hs.size();

  TraceParams& p = e->params;
  p.cosmo = make_dev_cosmo(c);
  p.fields = d_fields;
  p.sets = e->d_sets;
  p.nodes = d_nodes;
  p.step_set = d_steps;
  p.items = d_items;
  p.n_items = (int32_t)hitems.size();
  p.queue = d_queue;
  p.step_begin = sb;
  p.step_end = se;
  p.rays = rays;
  p.n_rays = 9 * nb;
  p.flags = flags;
  e->n_items = p.n_items;
  int per_cu = 0;
  RT_HIP(plan_occupancy(fp64, plan, &per_cu));
  if (per_cu < 1) return fail(RT_ERR_DEVICE, "trace plan %d does not fit on a compute unit", plan);
  e->grid = std::max(1, std::min(e->n_items, per_cu * di.n_cu));
  if (g.grid_limit > 0) e->grid = std::min(e->grid, g.grid_limit);
  e->interactions = describe(fields, n_fields, sb, se).interactions;
  return RT_OK;
}

// Enqueue the work of an entry on `s` (frames and FP32 copies, queue reset, trace).
rt_status enqueue_entry(TraceEntry* e, hipStream_t s) {
  RT_HIP(launch_prepare_sets(e->d_sets, e->n_sets_total, s));
  for (const auto& cv : e->conv) RT_HIP(launch_convert_set(e->d_sets + cv.set_index, cv.p64, cv.p32, cv.n, s));
  RT_HIP(launch_reset_queue(e->params.queue, s));
  if (e->n_items > 0) RT_HIP(launch_trace(e->fp64, e->plan, e->params, e->grid, s));
  return RT_OK;
}

rt_status capture_entry(TraceEntry* e) {
  hipStream_t& cs = g.capture_stream[e->device & 63];
  if (!cs) RT_HIP(hipStreamCreateWithFlags(&cs, hipStreamNonBlocking));
  RT_HIP(hipStreamBeginCapture(cs, hipStreamCaptureModeThreadLocal));
  rt_status st = enqueue_entry(e, cs);
  hipGraph_t graph = nullptr;
  hipError_t end = hipStreamEndCapture(cs, &graph);
  if (st != RT_OK) {
    if (graph) (void)hipGraphDestroy(graph);
    return st;
  }
  if (end != hipSuccess) return fail(RT_ERR_DEVICE, "hipStreamEndCapture failed: %s", hipGetErrorString(end));
  e->graph = graph;
  RT_HIP(hipGraphInstantiate(&e->exec, graph, nullptr, nullptr, 0));
  return RT_OK;
}

int choose_plan(bool fp64, const Workload& w, const DeviceInfo& di) {
  if (g.forced[fp64] >= 0) return g.forced[fp64];
  auto it = g.tuned.find(std::make_tuple(di.id, (int)fp64, ilog2(w.rays), ilog2(w.mean_np)));
  if (it != g.tuned.end()) return it->second;
  return heuristic_plan(fp64, w, di.n_cu);
}

}  // namespace

// ============================================================================ C ABI
extern "C" {

rt_status rt_sync(hipStream_t stream) {
  RT_HIP(hipStreamSynchronize(stream));
  RT_HIP(hipGetLastError());
  return RT_OK;
}

const char* rt_last_error(void) { return g_err.c_str(); }

rt_status rt_comoving_distance(const rt_cosmology* cosmo, double z, double* chi_out) {
  rt_status st = check_cosmo(cosmo);
  if (st != RT_OK) return st;
  if (!chi_out) return fail(RT_ERR_INVALID_ARG, "chi_out is NULL");
  if (!std::isfinite(z)) return fail(RT_ERR_NONFINITE, "z is not finite");
  if (z < 0.0) return fail(RT_ERR_INVALID_ARG, "z < 0");
  *chi_out = comoving_distance(*cosmo, z);
  return RT_OK;
}

rt_status rt_make_schedule(double chi_s, double z_lo, double z_hi, int32_t n_fine, double q, double* nodes,
                           int32_t capacity, int32_t* n_steps) {
  if (!nodes || !n_steps) return fail(RT_ERR_INVALID_ARG, "nodes or n_steps is NULL");
  if (!std::isfinite(chi_s) || !std::isfinite(z_lo) || !std::isfinite(z_hi) || !std::isfinite(q))
    return fail(RT_ERR_NONFINITE, "schedule argument is not finite");
  if (!(chi_s > 0.0) || !(z_lo >= 0.0) || !(z_hi > z_lo) || !(z_hi <= chi_s))
    return fail(RT_ERR_INVALID_ARG, "schedule needs 0 <= z_lo < z_hi <= chi_s");
  if (n_fine < 1) return fail(RT_ERR_INVALID_ARG, "n_fine < 1");
  if (!(q >= 1.0)) return fail(RT_ERR_INVALID_ARG, "q < 1");
  const double h = (z_hi - z_lo) / n_fine;
  std::vector<double> below;     // nodes under z_lo, generated downward
  if (z_lo > 0.0) {
    double r = z_lo, step = h;
    while (true) {
      step *= q;
      if ((int64_t)below.size() >= capacity) return fail(RT_ERR_INVALID_ARG, "capacity %d too small", capacity);
      if (r - step < 0.5 * step) {
        below.push_back(0.0);
        break;
      }
      r -= step;
      below.push_back(r);
    }
  }
  std::vector<double> out(below.rbegin(), below.rend());
  for (int32_t i = 0; i < n_fine; ++i) out.push_back(z_lo + (double)i * h);
  out.push_back(z_hi);
  if (z_hi < chi_s) {
    double r = z_hi, step = h;
    while (true) {
      step *= q;
      if ((int64_t)out.size() >= capacity) return fail(RT_ERR_INVALID_ARG, "capacity %d too small", capacity);
      if (chi_s - (r + step) < 0.5 * step) {
        out.push_back(chi_s);
        break;
      }
      r += step;
      out.push_back(r);
    }
  }
  if ((int64_t)out.size() > capacity) return fail(RT_ERR_INVALID_ARG, "capacity %d too small", capacity);
  std::copy(out.begin(), out.end(), nodes);
  *n_steps = (int32_t)out.size() - 1;
  return RT_OK;
}

rt_status rt_replica_step_sets(const double* nodes, int32_t n_steps, double box, int32_t n_replicas,
                               int32_t* step_set) {
  if (!nodes || !step_set) return fail(RT_ERR_INVALID_ARG, "nodes or step_set is NULL");
  if (n_steps < 1 || n_replicas < 1) return fail(RT_ERR_INVALID_ARG, "n_steps and n_replicas must be >= 1");
  if (!(box > 0.0) || !std::isfinite(box)) return fail(RT_ERR_INVALID_ARG, "box must be positive");
  for (int32_t s = 0; s < n_steps; ++s) {
    const double mid = 0.5 * (nodes[s] + nodes[s + 1]);
    int32_t r = (int32_t)std::floor(mid / box);
    step_set[s] = std::min(std::max(r, 0), n_replicas - 1);
  }
  return RT_OK;
}

rt_status rt_build_bundles(const rt_cosmology* cosmo, const rt_field* fields, int32_t n_fields, int64_t n_bundles,
                           const double* theta, double radius, double* rays, hipStream_t stream) {
  rt_status st = check_cosmo(cosmo);
  if (st != RT_OK) return st;
  if (n_bundles <= 0) return fail(RT_ERR_INVALID_ARG, "n_bundles must be > 0");
  if (!theta || !rays) return fail(RT_ERR_INVALID_ARG, "theta or rays is NULL");
  if (!std::isfinite(radius)) return fail(RT_ERR_NONFINITE, "radius is not finite");
  if (!(radius > 0.0) || !(radius < 1e-2)) return fail(RT_ERR_INVALID_ARG, "radius must be in (0, 1e-2) rad");
  if ((st = check_fields(fields, n_fields, n_bundles, 0.0, false)) != RT_OK) return st;
  const DevCosmo dc = make_dev_cosmo(*cosmo);
  RT_HIP(launch_bundles(dc, nullptr, 0, n_bundles, n_bundles, theta, radius, rays, stream));
  // fields whose first step has a set: potential at the observer from that set (FP64)
  std::vector<int> need;
  for (int f = 0; f < n_fields; ++f)
    if (fields[f].n_bundles > 0 && fields[f].step_set[0] >= 0) need.push_back(f);
  if (need.empty()) return RT_OK;
  const size_t n = need.size();
  // scratch: [n] DevSet, then doubles: [3] origin point, [n] phi, [3n] grad
  const size_t set_bytes = sizeof(DevSet) * n;
  const size_t dbl = 3 + n + 3 * n;
  StreamScratch sc(stream);
  RT_HIP(sc.alloc(set_bytes + sizeof(double) * dbl));
  void* scratch = sc.p;
  DevSet* d_sets = static_cast<DevSet*>(scratch);
  double* d_pt = reinterpret_cast<double*>(static_cast<char*>(scratch) + set_bytes);
  double* d_phi = d_pt + 3;
  double* d_grad = d_phi + n;
  std::vector<DevSet> hs(n);
  for (size_t i = 0; i < n; ++i) {
    const rt_particle_set& s = fields[need[i]].sets[fields[need[i]].step_set[0]];
    DevSet ds{};
    ds.p64 = s.xyzm;
    ds.n = s.n;
    ds.eps2 = s.softening * s.softening;
    ds.eps2f = (float)ds.eps2;
    ds.background = s.background;
    for (int k = 0; k < 3; ++k) {
      ds.lo[k] = s.lo[k];
      ds.hi[k] = s.hi[k];
    }
    hs[i] = ds;
  }
  const double zero3[3] = {0.0, 0.0, 0.0};
  RT_HIP(hipMemcpyAsync(d_sets, hs.data(), set_bytes, hipMemcpyHostToDevice, stream));
  RT_HIP(hipMemcpyAsync(d_pt, zero3, sizeof(zero3), hipMemcpyHostToDevice, stream));
  RT_HIP(hipStreamSynchronize(stream));   // host staging above is pageable and local
  for (size_t i = 0; i < n; ++i) {
    const rt_field& F = fields[need[i]];
    RT_HIP(launch_field_eval(dc, d_sets + i, true, 1, d_pt, d_phi + i, d_grad + 3 * i, stream));
    RT_HIP(launch_bundles(dc, d_phi + i, F.bundle_offset, F.n_bundles, n_bundles, theta, radius, rays, stream));
  }
  RT_HIP(sc.release());
  return RT_OK;
}

rt_status rt_trace(const rt_cosmology* cosmo, double z_source, const rt_field* fields, int32_t n_fields,
                   rt_precision precision, int32_t step_begin, int32_t step_end, int64_t n_bundles, double* rays,
                   uint8_t* ray_flags, hipStream_t stream) {
  rt_status st = check_cosmo(cosmo);
  if (st != RT_OK) return st;
  if (!valid_precision(precision)) return fail(RT_ERR_INVALID_ARG, "unknown precision");
  if (!std::isfinite(z_source)) return fail(RT_ERR_NONFINITE, "z_source is not finite");
  if (!(z_source > 0.0)) return fail(RT_ERR_INVALID_ARG, "z_source must be > 0");
  if (n_bundles <= 0) return fail(RT_ERR_INVALID_ARG, "n_bundles must be > 0");
  if (!rays) return fail(RT_ERR_INVALID_ARG, "rays is NULL");
  if (step_begin < 0 || step_end < step_begin) return fail(RT_ERR_INVALID_ARG, "bad step window");
  const double chi_s = comoving_distance(*cosmo, z_source);
  if ((st = check_fields(fields, n_fields, n_bundles, chi_s, true)) != RT_OK) return st;
  if (n_fields == 0) return RT_OK;
  DeviceInfo di;
  if ((st = device_info(&di)) != RT_OK) return st;
  const bool fp64 = precision == RT_FP64;
  std::lock_guard<std::mutex> lk(g.mu);
  const Workload w = describe(fields, n_fields, step_begin, step_end);
  const int plan = choose_plan(fp64, w, di);
  std::vector<uint8_t> key =
      make_key(di.id, *cosmo, fields, n_fields, fp64, plan, step_begin, step_end, n_bundles, rays, ray_flags);
  TraceEntry* e = nullptr;
  bool reused = false;
  for (size_t i = 0; i < g.cache.size(); ++i) {
    if (g.cache[i]->key == key) {
      std::unique_ptr<TraceEntry> hit = std::move(g.cache[i]);
      g.cache.erase(g.cache.begin() + i);
      g.cache.push_back(std::move(hit));
      e = g.cache.back().get();
      reused = true;
      break;
    }
  }
  if (!e) {
    auto fresh = std::make_unique<TraceEntry>();
    fresh->key = std::move(key);
    if ((st = build_entry(fresh.get(), di, *cosmo, fields, n_fields, fp64, plan, step_begin, step_end, n_bundles,
                          rays, ray_flags)) != RT_OK)
      return st;
    if ((st = capture_entry(fresh.get())) != RT_OK) return st;
    // evict the least recently used entry that no caller's graph refers to
    if (g.cache.size() >= kMaxEntries) {
      for (size_t i = 0; i < g.cache.size(); ++i) {
        if (!g.cache[i]->pinned) {
          g.cache.erase(g.cache.begin() + i);
          break;
        }
      }
    }
    g.cache.push_back(std::move(fresh));
    e = g.cache.back().get();
  }
  // Launches of one cached configuration share its work queue and FP32 copies: a
  // launch on another stream waits for the previous one instead of racing it.
  // (Not while the caller's stream is being captured: an event recorded outside a
  // capture cannot be waited on inside it.)
  hipStreamCaptureStatus cap = hipStreamCaptureStatusNone;
  RT_HIP(hipStreamIsCapturing(stream, &cap));
  const bool ordered = cap == hipStreamCaptureStatusNone;
  if (!e->done)
    RT_HIP(hipEventCreateWithFlags(&e->done, hipEventDisableTiming));
  else if (ordered)
    RT_HIP(hipStreamWaitEvent(stream, e->done, 0));
  if (g.timing) {
    if (!g.ev0) RT_HIP(hipEventCreate(&g.ev0));
    if (!g.ev1) RT_HIP(hipEventCreate(&g.ev1));
    RT_HIP(hipEventRecord(g.ev0, stream));
  }
  if (ordered) {
    RT_HIP(hipGraphLaunch(e->exec, stream));
    RT_HIP(hipEventRecord(e->done, stream));
  } else {
    // The caller is capturing its own graph: enqueue the kernels themselves so that
    // they are recorded there (a graph launched into a capture is not).  They keep
    // referring to this entry's buffers on every replay, after this call returns:
    // the entry is never evicted.
    if ((st = enqueue_entry(e, stream)) != RT_OK) return st;
    e->pinned = true;
  }
  if (g.timing) RT_HIP(hipEventRecord(g.ev1, stream));
  g.timed_last = g.timing;
  g.last.kernel_ms = 0.0;
  g.last.interactions = e->interactions;
  g.last.plan_id = e->plan;
  g.last.grid_blocks = e->grid;
  g.last.n_items = e->n_items;
  g.last.graph_reused = reused ? 1 : 0;
  return RT_OK;
}

rt_status rt_magnification(const rt_cosmology* cosmo, double z_source, int64_t n_bundles, double radius,
                           const double* rays, double* mu, double* jac, hipStream_t stream) {
  rt_status st = check_cosmo(cosmo);
  if (st != RT_OK) return st;
  if (!std::isfinite(z_source) || !std::isfinite(radius)) return fail(RT_ERR_NONFINITE, "z_source or radius");
  if (!(z_source > 0.0)) return fail(RT_ERR_INVALID_ARG, "z_source must be > 0");
  if (!(radius > 0.0) || !(radius < 1e-2)) return fail(RT_ERR_INVALID_ARG, "radius must be in (0, 1e-2) rad");
  if (n_bundles <= 0) return fail(RT_ERR_INVALID_ARG, "n_bundles must be > 0");
  if (!rays || !mu) return fail(RT_ERR_INVALID_ARG, "rays or mu is NULL");
  const double chi_s = comoving_distance(*cosmo, z_source);
  RT_HIP(launch_magnification(chi_s, n_bundles, radius, rays, mu, jac, stream));
  return RT_OK;
}

rt_status rt_flexion(const rt_cosmology* cosmo, double z_source, int64_t n_bundles, double radius, const double* rays,
                     double* flex, double* dm, hipStream_t stream) {
  rt_status st = check_cosmo(cosmo);
  if (st != RT_OK) return st;
  if (!std::isfinite(z_source) || !std::isfinite(radius)) return fail(RT_ERR_NONFINITE, "z_source or radius");
  if (!(z_source > 0.0)) return fail(RT_ERR_INVALID_ARG, "z_source must be > 0");
  if (!(radius > 0.0) || !(radius < 1e-2)) return fail(RT_ERR_INVALID_ARG, "radius must be in (0, 1e-2) rad");
  if (n_bundles <= 0) return fail(RT_ERR_INVALID_ARG, "n_bundles must be > 0");
  if (!rays || !flex) return fail(RT_ERR_INVALID_ARG, "rays or flex is NULL");
  const double chi_s = comoving_distance(*cosmo, z_source);
  RT_HIP(launch_flexion(chi_s, n_bundles, radius, rays, flex, dm, stream));
  return RT_OK;
}

rt_status rt_mu_histogram(int64_t n, const double* mu, int32_t n_bins, double log_lo, double log_hi, double* pdf,
                          double* moments, hipStream_t stream) {
  if (n < 0) return fail(RT_ERR_INVALID_ARG, "n < 0");
  if (n > 0 && !mu) return fail(RT_ERR_INVALID_ARG, "mu is NULL");
  if (!pdf || !moments) return fail(RT_ERR_INVALID_ARG, "pdf or moments is NULL");
  if (n_bins < 1 || n_bins > 1 << 16) return fail(RT_ERR_INVALID_ARG, "n_bins must be in [1, 65536]");
  if (!std::isfinite(log_lo) || !std::isfinite(log_hi)) return fail(RT_ERR_NONFINITE, "histogram range");
  if (!(log_hi > log_lo)) return fail(RT_ERR_INVALID_ARG, "log_hi must exceed log_lo");
  StreamScratch work(stream);
  RT_HIP(work.alloc(sizeof(double) * (n_bins + 8)));
  RT_HIP(launch_histogram(n, mu, nullptr, 0, n_bins, log_lo, log_hi, pdf, moments, static_cast<double*>(work.p),
                          stream));
  RT_HIP(work.release());
  return RT_OK;
}

rt_status rt_mu_histogram_noalloc(int64_t n, const double* mu, int32_t n_bins, double log_lo, double log_hi,
                                  double* pdf, double* moments, hipStream_t stream) {
  if (n < 0) return fail(RT_ERR_INVALID_ARG, "n < 0");
  if (n > 0 && !mu) return fail(RT_ERR_INVALID_ARG, "mu is NULL");
  if (!pdf || !moments) return fail(RT_ERR_INVALID_ARG, "pdf or moments is NULL");
  if (!std::isfinite(log_lo) || !std::isfinite(log_hi)) return fail(RT_ERR_NONFINITE, "histogram range");
  if (!(log_hi > log_lo)) return fail(RT_ERR_INVALID_ARG, "log_hi must exceed log_lo");
  double* work = nullptr;
  int32_t max_bins = 0;
  RT_HIP(noalloc_scratch(&work, &max_bins));
  if (n_bins < 1 || n_bins > max_bins)
    return fail(RT_ERR_INVALID_ARG, "n_bins = %d must be in [1, %d] (the static scratch)", n_bins, max_bins);
  RT_HIP(launch_histogram(n, mu, nullptr, 0, n_bins, log_lo, log_hi, pdf, moments, work, stream));
  return RT_OK;
}

rt_status rt_shear_histogram(int64_t n, const double* mu, const double* jac, int32_t n_bins, double lo, double hi,
                             double* pdf, double* moments, hipStream_t stream) {
  if (n < 0) return fail(RT_ERR_INVALID_ARG, "n < 0");
  if (n > 0 && (!mu || !jac)) return fail(RT_ERR_INVALID_ARG, "mu or jac is NULL");
  if (!pdf || !moments) return fail(RT_ERR_INVALID_ARG, "pdf or moments is NULL");
  if (n_bins < 1 || n_bins > 1 << 16) return fail(RT_ERR_INVALID_ARG, "n_bins must be in [1, 65536]");
  if (!std::isfinite(lo) || !std::isfinite(hi)) return fail(RT_ERR_NONFINITE, "histogram range");
  if (!(hi > lo)) return fail(RT_ERR_INVALID_ARG, "hi must exceed lo");
  StreamScratch work(stream);
  RT_HIP(work.alloc(sizeof(double) * (n_bins + 8)));
  RT_HIP(launch_histogram(n, mu, jac, 1, n_bins, lo, hi, pdf, moments, static_cast<double*>(work.p), stream));
  RT_HIP(work.release());
  return RT_OK;
}

rt_status rt_field_eval(const rt_cosmology* cosmo, const rt_particle_set* set, rt_precision precision, int64_t n,
                        const double* points, double* phi, double* grad, hipStream_t stream) {
  rt_status st = check_cosmo(cosmo);
  if (st != RT_OK) return st;
  if (!set) return fail(RT_ERR_INVALID_ARG, "set is NULL");
  if ((st = check_set(*set, 0, 0)) != RT_OK) return st;
  if (!valid_precision(precision)) return fail(RT_ERR_INVALID_ARG, "unknown precision");
  if (n < 0) return fail(RT_ERR_INVALID_ARG, "n < 0");
  if (n == 0) return RT_OK;
  if (!points || !phi || !grad) return fail(RT_ERR_INVALID_ARG, "points, phi or grad is NULL");
  const bool fp64 = precision == RT_FP64;
  const DevCosmo dc = make_dev_cosmo(*cosmo);
  DevSet hs{};
  hs.p64 = set->xyzm;
  hs.n = set->n;
  hs.eps2 = set->softening * set->softening;
  hs.eps2f = (float)hs.eps2;
  hs.background = set->background;
  for (int k = 0; k < 3; ++k) {
    hs.lo[k] = set->lo[k];
    hs.hi[k] = set->hi[k];
  }
  const size_t p32_bytes = (!fp64 && set->n > 0) ? 2 * sizeof(float4) * (size_t)set->n : 0;
  // scratch: DevSet, its equal-mass flag, then (256-byte aligned) the FP32 copy
  const size_t flag_off = ((sizeof(DevSet) + 7) / 8) * 8;
  const size_t p32_off = ((flag_off + sizeof(int32_t) + 255) / 256) * 256;
  StreamScratch sc(stream);
  RT_HIP(sc.alloc(p32_off + p32_bytes));
  void* scratch = sc.p;
  DevSet* d_set = static_cast<DevSet*>(scratch);
  float4* p32 = reinterpret_cast<float4*>(static_cast<char*>(scratch) + p32_off);
  hs.p32 = p32_bytes ? p32 : nullptr;
  hs.equal_mass = set->n > 0 ? reinterpret_cast<int32_t*>(static_cast<char*>(scratch) + flag_off) : nullptr;
  RT_HIP(hipMemcpyAsync(d_set, &hs, sizeof(DevSet), hipMemcpyHostToDevice, stream));
  RT_HIP(hipStreamSynchronize(stream));   // hs is a local
  RT_HIP(launch_prepare_sets(d_set, 1, stream));
  if (set->n > 0) RT_HIP(launch_convert_set(d_set, set->xyzm, hs.p32, set->n, stream));
  RT_HIP(launch_field_eval(dc, d_set, fp64, n, points, phi, grad, stream));
  RT_HIP(sc.release());
  return RT_OK;
}

int32_t rt_plan_count(rt_precision precision) {
  return valid_precision(precision) ? plan_count(precision == RT_FP64) : 0;
}

rt_status rt_plan_describe(rt_precision precision, int32_t id, rt_plan_info* info) {
  if (!valid_precision(precision)) return fail(RT_ERR_INVALID_ARG, "unknown precision");
  if (!info) return fail(RT_ERR_INVALID_ARG, "info is NULL");
  if (id < 0 || id >= plan_count(precision == RT_FP64)) return fail(RT_ERR_INVALID_ARG, "plan id %d out of range", id);
  *info = plan_info(precision == RT_FP64, id);
  return RT_OK;
}

rt_status rt_force_plan(rt_precision precision, int32_t id) {
  if (!valid_precision(precision)) return fail(RT_ERR_INVALID_ARG, "unknown precision");
  if (id < -1 || id >= plan_count(precision == RT_FP64)) return fail(RT_ERR_INVALID_ARG, "plan id %d out of range", id);
  std::lock_guard<std::mutex> lk(g.mu);
  g.forced[precision == RT_FP64] = id;
  return RT_OK;
}

rt_status rt_set_grid_limit(int32_t max_blocks) {
  if (max_blocks < 0) return fail(RT_ERR_INVALID_ARG, "max_blocks < 0");
  std::lock_guard<std::mutex> lk(g.mu);
  g.grid_limit = max_blocks;
  return RT_OK;
}

rt_status rt_autotune(const rt_cosmology* cosmo, double z_source, const rt_field* fields, int32_t n_fields,
                      rt_precision precision, int32_t step_begin, int32_t n_probe_steps, int64_t n_bundles,
                      const double* rays, int32_t* best_id, hipStream_t stream) {
  rt_status st = check_cosmo(cosmo);
  if (st != RT_OK) return st;
  if (!valid_precision(precision)) return fail(RT_ERR_INVALID_ARG, "unknown precision");
  if (!(z_source > 0.0)) return fail(RT_ERR_INVALID_ARG, "z_source must be > 0");
  if (n_bundles <= 0 || !rays) return fail(RT_ERR_INVALID_ARG, "n_bundles or rays");
  if (step_begin < 0 || n_probe_steps < 1) return fail(RT_ERR_INVALID_ARG, "bad probe window");
  const double chi_s = comoving_distance(*cosmo, z_source);
  if ((st = check_fields(fields, n_fields, n_bundles, chi_s, true)) != RT_OK) return st;
  if (n_fields == 0) return RT_OK;
  DeviceInfo di;
  if ((st = device_info(&di)) != RT_OK) return st;
  const bool fp64 = precision == RT_FP64;
  const int32_t se = step_begin + n_probe_steps;
  const size_t bytes = sizeof(double) * 8 * 9 * (size_t)n_bundles;
  void* scratch = nullptr;
  RT_HIP(hipMalloc(&scratch, bytes));
  std::unique_ptr<Buffer> guard(new Buffer);
  guard->p = scratch;
  hipEvent_t e0, e1;
  RT_HIP(hipEventCreate(&e0));
  RT_HIP(hipEventCreate(&e1));
  int best = -1;
  float best_ms = 0.f;
  for (int id = 0; id < plan_count(fp64); ++id) {
    TraceEntry te;
    if ((st = build_entry(&te, di, *cosmo, fields, n_fields, fp64, id, step_begin, se, n_bundles,
                          static_cast<double*>(scratch), nullptr)) != RT_OK)
      break;
    float ms = 0.f;
    for (int rep = 0; rep < 2 && st == RT_OK; ++rep) {   // first run warms up
      hipError_t err = hipMemcpyAsync(scratch, rays, bytes, hipMemcpyDeviceToDevice, stream);
      if (err == hipSuccess) err = hipEventRecord(e0, stream);
      if (err != hipSuccess) st = fail(RT_ERR_DEVICE, "autotune copy: %s", hipGetErrorString(err));
      if (st == RT_OK) st = enqueue_entry(&te, stream);
      if (st == RT_OK) {
        err = hipEventRecord(e1, stream);
        if (err == hipSuccess) err = hipEventSynchronize(e1);
        if (err == hipSuccess) err = hipEventElapsedTime(&ms, e0, e1);
        if (err != hipSuccess) st = fail(RT_ERR_DEVICE, "autotune timing: %s", hipGetErrorString(err));
      }
    }
    if (st != RT_OK) break;
    if (best < 0 || ms < best_ms) {
      best = id;
      best_ms = ms;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  RT_HIP(hipStreamSynchronize(stream));
  if (st != RT_OK) return st;
  const Workload w = describe(fields, n_fields, 0, INT32_MAX);
  {
    std::lock_guard<std::mutex> lk(g.mu);
    g.tuned[std::make_tuple(di.id, (int)fp64, ilog2(w.rays), ilog2(w.mean_np))] = best;
  }
  if (best_id) *best_id = best;
  return RT_OK;
}

rt_status rt_enable_timing(int32_t on) {
  std::lock_guard<std::mutex> lk(g.mu);
  g.timing = on != 0;
  return RT_OK;
}

rt_status rt_last_trace_info(rt_trace_info* info) {
  if (!info) return fail(RT_ERR_INVALID_ARG, "info is NULL");
  std::lock_guard<std::mutex> lk(g.mu);
  *info = g.last;
  if (g.timed_last && g.ev1) {
    float ms = 0.f;
    RT_HIP(hipEventSynchronize(g.ev1));
    RT_HIP(hipEventElapsedTime(&ms, g.ev0, g.ev1));
    info->kernel_ms = ms;
  }
  return RT_OK;
}

void rt_release_caches(void) {
  std::lock_guard<std::mutex> lk(g.mu);
  (void)hipDeviceSynchronize();
  g.cache.clear();
  g.tuned.clear();
}

}  // extern "C"

// ---------------------------------------------------------------- particle-mesh field

namespace {
rt_status check_pm_grid(const rt_pm_grid* g) {
  if (!g) return fail(RT_ERR_INVALID_ARG, "grid is NULL");
  if (g->n < 4 || g->n > 512 || (g->n & (g->n - 1)) != 0)
    return fail(RT_ERR_INVALID_ARG, "grid.n = %d must be a power of two in [4, 512]", g->n);
  for (int d = 0; d < 3; ++d)
    if (!std::isfinite(g->origin[d])) return fail(RT_ERR_NONFINITE, "grid.origin[%d] is not finite", d);
  if (!std::isfinite(g->h)) return fail(RT_ERR_NONFINITE, "grid.h is not finite");
  if (!(g->h > 0.0)) return fail(RT_ERR_INVALID_ARG, "grid.h must be > 0");
  if (g->periodic != 0 && g->periodic != 1) return fail(RT_ERR_INVALID_ARG, "grid.periodic must be 0 or 1");
  return RT_OK;
}

// An isolated grid's potential at the observer must be 0 (bundles are built with
// phi_obs = 0 there), so it must leave the observer outside its nodes.
rt_status check_observer_outside(const rt_pm_grid* g) {
  bool inside = true;
  for (int d = 0; d < 3; ++d) {
    const double lo = g->origin[d], hi = g->origin[d] + g->h * (g->n - 1);
    if (!(0.0 >= lo && 0.0 <= hi)) inside = false;
  }
  if (inside) return fail(RT_ERR_INVALID_ARG, "the observer (0, 0, 0) lies inside the grid");
  return RT_OK;
}

rt_status check_n_int(const rt_pm_grid* g, int32_t n_int) {
  if (n_int < 1 || n_int > 4) return fail(RT_ERR_INVALID_ARG, "n_int = %d must be in [1, 4]", n_int);
  if (g->n < 2 * n_int) return fail(RT_ERR_INVALID_ARG, "grid.n = %d < 2 n_int", g->n);
  return RT_OK;
}
}  // namespace

extern "C" {

rt_status rt_pm_workspace_bytes(const rt_pm_grid* grid, size_t* bytes) {
  rt_status st;
  if ((st = check_pm_grid(grid)) != RT_OK) return st;
  if (!bytes) return fail(RT_ERR_INVALID_ARG, "bytes is NULL");
  *bytes = (size_t)pm_workspace_bytes(grid->n, grid->periodic);
  return RT_OK;
}

rt_status rt_pm_build(const rt_particle_set* set, const rt_pm_grid* grid, double* fields, void* workspace,
                      size_t workspace_bytes, hipStream_t stream) {
  rt_status st;
  if (!set) return fail(RT_ERR_INVALID_ARG, "set is NULL");
  if ((st = check_set(*set, 0, 0)) != RT_OK) return st;
  if ((st = check_pm_grid(grid)) != RT_OK) return st;
  if (set->background && !grid->periodic)
    return fail(RT_ERR_UNSUPPORTED, "rt_pm_build: an isolated grid needs background = 0");
  if (!fields || !workspace) return fail(RT_ERR_INVALID_ARG, "fields or workspace is NULL");
  const int64_t need = pm_workspace_bytes(grid->n, grid->periodic);
  if (workspace_bytes < (size_t)need)
    return fail(RT_ERR_INVALID_ARG, "workspace of %zu bytes, %lld needed", workspace_bytes, (long long)need);
  RT_HIP(launch_pm_build(set->xyzm, set->n, set->softening, grid->origin, grid->h, grid->n, grid->periodic,
                         g_over_c2(), fields, workspace, stream));
  return RT_OK;
}

rt_status rt_pm_eval(const rt_pm_grid* grid, const double* fields, int32_t n_int, int64_t n, const double* points,
                     double* phi, double* grad, hipStream_t stream) {
  rt_status st;
  if ((st = check_pm_grid(grid)) != RT_OK) return st;
  if ((st = check_n_int(grid, n_int)) != RT_OK) return st;
  if (n < 0) return fail(RT_ERR_INVALID_ARG, "n < 0");
  if (n == 0) return RT_OK;
  if (!fields || !points || !phi || !grad) return fail(RT_ERR_INVALID_ARG, "fields, points, phi or grad is NULL");
  RT_HIP(launch_pm_eval(grid->origin, grid->h, grid->n, grid->periodic, fields, n_int, n, points, phi, grad, stream));
  return RT_OK;
}

rt_status rt_trace_pm(const rt_cosmology* cosmo, double z_source, int32_t n_grids, const rt_pm_grid* grids,
                      const double* const* fields, int32_t n_int, int32_t n_steps, const double* z_nodes,
                      const int32_t* step_grid, int32_t step_begin, int32_t step_end, int64_t n_bundles, double* rays,
                      uint8_t* ray_flags, hipStream_t stream) {
  rt_status st;
  if ((st = check_cosmo(cosmo)) != RT_OK) return st;
  if (!std::isfinite(z_source)) return fail(RT_ERR_NONFINITE, "z_source is not finite");
  if (!(z_source > 0.0)) return fail(RT_ERR_INVALID_ARG, "z_source must be > 0");
  if (n_grids < 1 || !grids || !fields) return fail(RT_ERR_INVALID_ARG, "n_grids < 1, or grids or fields is NULL");
  for (int i = 0; i < n_grids; ++i) {
    if ((st = check_pm_grid(&grids[i])) != RT_OK) return fail(st, "grids[%d]: %s", i, g_err.c_str());
    if ((st = check_n_int(&grids[i], n_int)) != RT_OK) return fail(st, "grids[%d]: %s", i, g_err.c_str());
    if (!fields[i]) return fail(RT_ERR_INVALID_ARG, "fields[%d] is NULL", i);
    if (!grids[i].periodic && (st = check_observer_outside(&grids[i])) != RT_OK)
      return fail(st, "grids[%d]: %s", i, g_err.c_str());
  }
  if (n_bundles < 0) return fail(RT_ERR_INVALID_ARG, "n_bundles < 0");
  if (n_bundles > 0 && !rays) return fail(RT_ERR_INVALID_ARG, "rays is NULL");
  if (step_begin < 0 || step_end < step_begin) return fail(RT_ERR_INVALID_ARG, "bad step window");
  if (n_steps < 1 || !z_nodes) return fail(RT_ERR_SCHEDULE, "n_steps < 1 or z_nodes is NULL");
  const double chi_s = comoving_distance(*cosmo, z_source);
  if (z_nodes[0] != 0.0) return fail(RT_ERR_SCHEDULE, "z_nodes[0] != 0");
  for (int s = 0; s < n_steps; ++s) {
    if (!std::isfinite(z_nodes[s + 1])) return fail(RT_ERR_NONFINITE, "z_nodes[%d]", s + 1);
    if (!(z_nodes[s + 1] > z_nodes[s])) return fail(RT_ERR_SCHEDULE, "z_nodes not strictly increasing at %d", s + 1);
  }
  if (std::fabs(z_nodes[n_steps] - chi_s) > 1e-9 * chi_s)
    return fail(RT_ERR_SCHEDULE, "last node %.17g differs from chi_s %.17g", z_nodes[n_steps], chi_s);
  std::vector<int32_t> sg(n_steps, 0);
  if (step_grid) {
    for (int s = 0; s < n_steps; ++s) {
      if (step_grid[s] < -1 || step_grid[s] >= n_grids)
        return fail(RT_ERR_INVALID_ARG, "step_grid[%d] = %d out of [-1, %d)", s, step_grid[s], n_grids);
      sg[s] = step_grid[s];
    }
  }
  const int32_t se = step_end > n_steps ? n_steps : step_end;
  if (n_bundles == 0 || step_begin >= se) return RT_OK;
  std::vector<DevPmGrid> hg(n_grids);
  for (int i = 0; i < n_grids; ++i) {
    hg[i].n = grids[i].n;
    for (int d = 0; d < 3; ++d) hg[i].origin[d] = grids[i].origin[d];
    hg[i].h = grids[i].h;
    hg[i].periodic = grids[i].periodic;
    hg[i].fields = fields[i];
  }
  // scratch: grid table, then nodes, then step grids
  const size_t gbytes = ((sizeof(DevPmGrid) * n_grids + 255) / 256) * 256;
  const size_t nbytes = ((sizeof(double) * (n_steps + 1) + 255) / 256) * 256;
  StreamScratch sc(stream);
  RT_HIP(sc.alloc(gbytes + nbytes + sizeof(int32_t) * n_steps));
  char* scratch = static_cast<char*>(sc.p);
  DevPmGrid* d_grids = reinterpret_cast<DevPmGrid*>(scratch);
  double* d_nodes = reinterpret_cast<double*>(scratch + gbytes);
  int32_t* d_sg = reinterpret_cast<int32_t*>(scratch + gbytes + nbytes);
  RT_HIP(hipMemcpyAsync(d_grids, hg.data(), sizeof(DevPmGrid) * n_grids, hipMemcpyHostToDevice, stream));
  RT_HIP(hipMemcpyAsync(d_nodes, z_nodes, sizeof(double) * (n_steps + 1), hipMemcpyHostToDevice, stream));
  RT_HIP(hipMemcpyAsync(d_sg, sg.data(), sizeof(int32_t) * n_steps, hipMemcpyHostToDevice, stream));
  RT_HIP(hipStreamSynchronize(stream));   // the host staging above is pageable and local
  RT_HIP(launch_pm_trace(make_dev_cosmo(*cosmo), d_grids, d_sg, n_int, d_nodes, step_begin, se, rays,
                         9 * n_bundles, ray_flags, stream));
  RT_HIP(sc.release());
  return RT_OK;
}

rt_status rt_trace_pm_lambda(const rt_cosmology* cosmo, double z_source, const rt_pm_grid* grid,
                             const double* fields, int32_t n_int, double f_rk, int32_t max_steps, int64_t n_bundles,
                             double* rays, uint8_t* ray_flags, int32_t* ray_steps, hipStream_t stream) {
  rt_status st;
  if ((st = check_cosmo(cosmo)) != RT_OK) return st;
  if (!std::isfinite(z_source)) return fail(RT_ERR_NONFINITE, "z_source is not finite");
  if (!(z_source > 0.0)) return fail(RT_ERR_INVALID_ARG, "z_source must be > 0");
  if ((st = check_pm_grid(grid)) != RT_OK) return st;
  if ((st = check_n_int(grid, n_int)) != RT_OK) return st;
  if (!fields) return fail(RT_ERR_INVALID_ARG, "fields is NULL");
  if (!std::isfinite(f_rk)) return fail(RT_ERR_NONFINITE, "f_rk is not finite");
  if (!(f_rk > 0.0)) return fail(RT_ERR_INVALID_ARG, "f_rk must be > 0");
  if (max_steps < 1) return fail(RT_ERR_INVALID_ARG, "max_steps must be >= 1");
  if (n_bundles < 0) return fail(RT_ERR_INVALID_ARG, "n_bundles < 0");
  if (n_bundles > 0 && !rays) return fail(RT_ERR_INVALID_ARG, "rays is NULL");
  if (!grid->periodic && (st = check_observer_outside(grid)) != RT_OK) return st;
  if (n_bundles == 0) return RT_OK;
  RT_HIP(launch_pm_trace_lambda(make_dev_cosmo(*cosmo), grid->origin, grid->h, grid->n, grid->periodic, fields, n_int,
                                comoving_distance(*cosmo, z_source), f_rk, max_steps, rays, 9 * n_bundles, ray_flags,
                                ray_steps, stream));
  return RT_OK;
}

rt_status rt_trace_pm_lambda_slabs(const rt_cosmology* cosmo, double z_source, int32_t n_grids,
                                   const rt_pm_grid* grids, const double* const* fields, int32_t n_int,
                                   int32_t n_slabs, const double* slab_bounds, const int32_t* slab_grid, double f_rk,
                                   int32_t max_steps, int64_t n_bundles, double* rays, uint8_t* ray_flags,
                                   int32_t* ray_steps, hipStream_t stream) {
  rt_status st;
  if ((st = check_cosmo(cosmo)) != RT_OK) return st;
  if (!std::isfinite(z_source)) return fail(RT_ERR_NONFINITE, "z_source is not finite");
  if (!(z_source > 0.0)) return fail(RT_ERR_INVALID_ARG, "z_source must be > 0");
  if (n_grids < 1 || !grids || !fields) return fail(RT_ERR_INVALID_ARG, "n_grids < 1, or grids or fields is NULL");
  for (int i = 0; i < n_grids; ++i) {
    if ((st = check_pm_grid(&grids[i])) != RT_OK) return fail(st, "grids[%d]: %s", i, g_err.c_str());
    if ((st = check_n_int(&grids[i], n_int)) != RT_OK) return fail(st, "grids[%d]: %s", i, g_err.c_str());
    if (!fields[i]) return fail(RT_ERR_INVALID_ARG, "fields[%d] is NULL", i);
    if (!grids[i].periodic && (st = check_observer_outside(&grids[i])) != RT_OK)
      return fail(st, "grids[%d]: %s", i, g_err.c_str());
    if (grids[i].h != grids[0].h)
      return fail(RT_ERR_INVALID_ARG, "grids[%d].h = %.17g differs from grids[0].h = %.17g", i, grids[i].h,
                  grids[0].h);
  }
  if (n_slabs < 1 || !slab_bounds || !slab_grid)
    return fail(RT_ERR_INVALID_ARG, "n_slabs < 1, or slab_bounds or slab_grid is NULL");
  for (int k = 0; k <= n_slabs; ++k) {
    if (!std::isfinite(slab_bounds[k])) return fail(RT_ERR_NONFINITE, "slab_bounds[%d] is not finite", k);
    if (k > 0 && !(slab_bounds[k] > slab_bounds[k - 1]))
      return fail(RT_ERR_INVALID_ARG, "slab_bounds not strictly increasing at %d", k);
  }
  for (int k = 0; k < n_slabs; ++k)
    if (slab_grid[k] < -1 || slab_grid[k] >= n_grids)
      return fail(RT_ERR_INVALID_ARG, "slab_grid[%d] = %d out of [-1, %d)", k, slab_grid[k], n_grids);
  if (!std::isfinite(f_rk)) return fail(RT_ERR_NONFINITE, "f_rk is not finite");
  if (!(f_rk > 0.0)) return fail(RT_ERR_INVALID_ARG, "f_rk must be > 0");
  if (max_steps < 1) return fail(RT_ERR_INVALID_ARG, "max_steps must be >= 1");
  if (n_bundles < 0) return fail(RT_ERR_INVALID_ARG, "n_bundles < 0");
  if (n_bundles > 0 && !rays) return fail(RT_ERR_INVALID_ARG, "rays is NULL");
  if (n_bundles == 0) return RT_OK;
  std::vector<DevPmGrid> hg(n_grids);
  for (int i = 0; i < n_grids; ++i) {
    hg[i].n = grids[i].n;
    for (int d = 0; d < 3; ++d) hg[i].origin[d] = grids[i].origin[d];
    hg[i].h = grids[i].h;
    hg[i].periodic = grids[i].periodic;
    hg[i].fields = fields[i];
  }
  // scratch: grid table, then slab bounds, then slab grids
  const size_t gbytes = ((sizeof(DevPmGrid) * n_grids + 255) / 256) * 256;
  const size_t bbytes = ((sizeof(double) * (n_slabs + 1) + 255) / 256) * 256;
  StreamScratch sc(stream);
  RT_HIP(sc.alloc(gbytes + bbytes + sizeof(int32_t) * n_slabs));
  char* scratch = static_cast<char*>(sc.p);
  DevPmGrid* d_grids = reinterpret_cast<DevPmGrid*>(scratch);
  double* d_bounds = reinterpret_cast<double*>(scratch + gbytes);
  int32_t* d_sg = reinterpret_cast<int32_t*>(scratch + gbytes + bbytes);
  RT_HIP(hipMemcpyAsync(d_grids, hg.data(), sizeof(DevPmGrid) * n_grids, hipMemcpyHostToDevice, stream));
  RT_HIP(hipMemcpyAsync(d_bounds, slab_bounds, sizeof(double) * (n_slabs + 1), hipMemcpyHostToDevice, stream));
  RT_HIP(hipMemcpyAsync(d_sg, slab_grid, sizeof(int32_t) * n_slabs, hipMemcpyHostToDevice, stream));
  RT_HIP(hipStreamSynchronize(stream));   // the host staging above is pageable and local
  RT_HIP(launch_pm_trace_lambda_slabs(make_dev_cosmo(*cosmo), d_grids, d_bounds, d_sg, n_slabs, grids[0].h, n_int,
                                      comoving_distance(*cosmo, z_source), f_rk, max_steps, rays, 9 * n_bundles,
                                      ray_flags, ray_steps, stream));
  RT_HIP(sc.release());
  return RT_OK;
}

}  // extern "C"

