// extern "C" entry points of libhydro: argument validation and dispatch to
// the kernels.  Declarations and documentation: include/hydro.h.

#include <algorithm>
#include <atomic>
#include <cctype>
#include <cmath>
#include <cstdint>
#include <cstdio>
#include <cstdlib>
#include <map>
#include <mutex>
#include <set>
#include <string>

#include "ext_device.h"
#include "hydro.h"
#include "kernels.h"

#include <cstddef>

// the Python binding mirrors this layout with ctypes
static_assert(sizeof(hydro_level_t) == 128 && offsetof(hydro_level_t, dt) == 56 &&
                  offsetof(hydro_level_t, dt_dev) == 72 && offsetof(hydro_level_t, dt_dev_scale) == 80 &&
                  offsetof(hydro_level_t, dt_reset_dev) == 120,
              "hydro_level_t layout");

namespace {

thread_local int g_last_hip_error = 0;

// Measured defaults of the launch shapes (used when a context has no
// selection): level step XCD-blocked, column-tile order, low occupancy
// target (variant 6); fused adjoint (0); batched: one queue, high occupancy
// (0).
constexpr int kDefaultLevelVariant = 6;
constexpr int kDefaultAdjointVariant = 0;
constexpr int kDefaultBatchedVariant = 0;

}  // namespace

// A solver context: the launch-shape selections of one user of the library
// (explicitly set, or autotuned and keyed by dtype and level shape), the
// optional tuning-cache file they are loaded from and saved to, and the
// graphs captured through it.  Entry points take it as their first argument;
// NULL selects the measured defaults.
struct hydro_ctx {
  std::mutex mu;
  std::string cache_path;
  bool require_tuned = false;
  int level_sel[2][2] = {{-1, -1}, {-1, -1}};  // [dtype][with CFL epilogue], -1 = not set
  int batched_sel[2] = {-1, -1};
  int adjoint_sel[2] = {-1, -1};
  std::map<std::string, int> tuned;          // autotuned or cached selections by key
  std::set<void*> graphs;                    // hipGraphExec_t handles captured through this context
};

namespace {

const char* dtype_name(int32_t dtype) { return dtype == HYDRO_F64 ? "f64" : "f32"; }

std::string level_key(int32_t dtype, bool with_cfl, int ngx, int ngy, int ngz) {
  char b[96];
  std::snprintf(b, sizeof b, "level/%s/%s/%dx%dx%d", dtype_name(dtype), with_cfl ? "cfl" : "plain", ngx, ngy, ngz);
  return b;
}

std::string adjoint_key(int32_t dtype, int ngx, int ngy, int ngz) {
  char b[96];
  std::snprintf(b, sizeof b, "adjoint/%s/%dx%dx%d", dtype_name(dtype), ngx, ngy, ngz);
  return b;
}

std::string batched_key(int32_t dtype, const hydro_level_t* lv, int n) {
  // the kernel form with the CFL epilogue is tuned on its own
  bool cfl = false;
  for (int l = 0; l < n; ++l)
    cfl = cfl || lv[l].dt_next_dev != nullptr || lv[l].dt_patch_next_dev != nullptr || lv[l].dt_reset_dev != nullptr;
  std::string k = std::string(cfl ? "batched-cfl/" : "batched/") + dtype_name(dtype) + "/";
  for (int l = 0; l < n; ++l) {
    char b[64];
    std::snprintf(b, sizeof b, "%s%dx%dx%d", l ? "+" : "", lv[l].ngx, lv[l].ngy, lv[l].ngz);
    k += b;
  }
  return k;
}

// The shape a launch uses: a tuned selection for this key, else the one set
// explicitly, else (unless the context requires tuning) the default.
// explicit_sel points into the context and is read under its lock.
int select_shape(hydro_ctx* c, const std::string& key, const int* explicit_sel, int fallback, int* out) {
  if (c == nullptr) {
    *out = fallback;
    return HYDRO_OK;
  }
  std::lock_guard<std::mutex> lk(c->mu);
  auto it = c->tuned.find(key);
  if (it != c->tuned.end()) {
    *out = it->second;
    return HYDRO_OK;
  }
  if (*explicit_sel >= 0) {
    *out = *explicit_sel;
    return HYDRO_OK;
  }
  if (c->require_tuned) return HYDRO_ENOTUNED;
  *out = fallback;
  return HYDRO_OK;
}

// Tuning cache: a JSON object {"version": 1, "entries": {"<key>": <shape>, ...}}.
// The reader accepts exactly what the writer produces (string keys, integer
// values), so a malformed file is reported rather than half-read.
bool parse_cache(const std::string& text, std::map<std::string, int>& out) {
  size_t i = text.find("\"entries\"");
  if (i == std::string::npos) return false;
  i = text.find('{', i);
  if (i == std::string::npos) return false;
  ++i;
  for (;;) {
    while (i < text.size() && std::isspace((unsigned char)text[i])) ++i;
    if (i < text.size() && text[i] == '}') return true;
    if (i >= text.size() || text[i] != '"') return false;
    const size_t e = text.find('"', i + 1);
    if (e == std::string::npos) return false;
    std::string key = text.substr(i + 1, e - i - 1);
    i = e + 1;
    while (i < text.size() && std::isspace((unsigned char)text[i])) ++i;
    if (i >= text.size() || text[i] != ':') return false;
    ++i;
    char* end = nullptr;
    const long v = std::strtol(text.c_str() + i, &end, 10);
    if (end == text.c_str() + i || v < 0 || v > 1000) return false;
    out[key] = int(v);
    i = size_t(end - text.c_str());
    while (i < text.size() && std::isspace((unsigned char)text[i])) ++i;
    if (i < text.size() && text[i] == ',') ++i;
  }
}

int save_cache_locked(hydro_ctx* c) {
  if (c->cache_path.empty()) return HYDRO_OK;
  const std::string tmp = c->cache_path + ".tmp";
  FILE* f = std::fopen(tmp.c_str(), "w");
  if (f == nullptr) return HYDRO_EIO;
  std::fprintf(f, "{\"version\": 1, \"entries\": {");
  bool first = true;
  for (const auto& kv : c->tuned) {
    std::fprintf(f, "%s\n  \"%s\": %d", first ? "" : ",", kv.first.c_str(), kv.second);
    first = false;
  }
  std::fprintf(f, "\n}}\n");
  const bool ok = std::fclose(f) == 0;
  if (!ok || std::rename(tmp.c_str(), c->cache_path.c_str()) != 0) return HYDRO_EIO;
  return HYDRO_OK;
}

void record_tuned(hydro_ctx* c, const std::string& key, int v) {
  std::lock_guard<std::mutex> lk(c->mu);
  c->tuned[key] = v;
  (void)save_cache_locked(c);  // best effort; hydro_ctx_save reports errors
}

// Compute units of the current device (persistent-grid size), cached per device.
int device_cus() {
  static std::atomic<int> cached[64];
  int dev = 0;
  if (hipGetDevice(&dev) != hipSuccess || dev < 0 || dev >= 64) return 256;
  int v = cached[dev].load();
  if (v > 0) return v;
  if (hipDeviceGetAttribute(&v, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess || v <= 0) v = 256;
  cached[dev].store(v);
  return v;
}

int device_status(hipError_t e) {
  if (e == hipSuccess) return HYDRO_OK;
  g_last_hip_error = int(e);
  return HYDRO_EDEVICE;
}

bool finite_pos(double v) { return std::isfinite(v) && v > 0.0; }

size_t dtype_size(int32_t dtype) { return dtype == HYDRO_F64 ? 8 : 4; }

bool overlap(const void* a, size_t na, const void* b, size_t nb) {
  if (na == 0 || nb == 0) return false;
  const uintptr_t pa = reinterpret_cast<uintptr_t>(a), pb = reinterpret_cast<uintptr_t>(b);
  return pa < pb + nb && pb < pa + na;
}

bool valid_scheme(int32_t scheme, double theta) {
  if ((scheme & 0xff) != HYDRO_SCHEME_MHM_PLM_HLLC) return false;
  const int ws = (scheme >> 8) & 3;
  if (ws > 1) return false;
  if (scheme & ~(0xff | (3 << 8) | HYDRO_FIRST_ORDER)) return false;
  return std::isfinite(theta) && theta >= 1.0 && theta <= 2.0;
}

// Scheme words of hydro_advance_ext: any id, solver, limiter and
// reconstruction bit; the reconstruction must fit in the ghost zones.
bool valid_ext_scheme(int32_t scheme, double theta, int32_t ghost, gh::ExtOpts* o) {
  const int id = scheme & 0xff;
  if (id != HYDRO_SCHEME_MHM && id != HYDRO_SCHEME_CTU) return false;
  const int known =
      0xff | (3 << 8) | HYDRO_FIRST_ORDER | (3 << 11) | HYDRO_CHARACTERISTIC | HYDRO_PPM | (3 << 16) | HYDRO_DUAL_ENERGY;
  if (scheme & ~known) return false;
  o->ctu = id == HYDRO_SCHEME_CTU;
  o->ws = (scheme >> 8) & 3;
  o->first_order = (scheme & HYDRO_FIRST_ORDER) ? 1 : 0;
  o->lim = (scheme >> 11) & 3;
  o->chr = (scheme & HYDRO_CHARACTERISTIC) ? 1 : 0;
  o->ppm = (scheme & HYDRO_PPM) ? 1 : 0;
  o->solver = (scheme >> 16) & 3;
  o->de = (scheme & HYDRO_DUAL_ENERGY) ? 1 : 0;
  o->xi = 0.0;
  if (o->ws > 1 || o->solver > 2) return false;
  if (ghost < o->radius() + 1 || ghost < 2) return false;
  return std::isfinite(theta) && theta >= 1.0 && theta <= 2.0;
}

// Scheme words the fused per-group kernel computes (MHM, PLM on primitive
// variables, generalized minmod, HLLC, any wave-speed option, second or first
// order): hydro_advance_ext runs them there, with no workspace.
bool fused_ext_scheme(const gh::ExtOpts& o) {
  return !o.ctu && o.lim == 0 && !o.chr && !o.ppm && o.solver == 0 && !o.de;
}

// The other MHM + PLM words (any limiter, primitive or characteristic
// variables, HLLC / Roe / HLLE, either wave-speed option, second or first
// order; no dual energy) run in the same fused kernel with run-time options,
// also without a workspace; CTU, PPM and dual energy take the chain of
// per-cell / per-face kernels.
bool fused_plm_scheme(const gh::ExtOpts& o) { return !o.ctu && !o.ppm && !o.de; }

template <typename T>
gh::Gas<T> make_gas(double gamma, double theta, double dt, double dx) {
  gh::Gas<T> g;
  g.gamma = T(gamma);
  g.gm1 = T(gamma - 1.0);
  g.inv_gm1 = T(1.0 / (gamma - 1.0));
  g.theta = T(theta);
  g.half_theta = T(0.5 * theta);
  g.dtdx = T(dt / dx);
  g.half_dtdx = T(0.5 * (dt / dx));
  return g;
}

template <typename T>
int batched_impl(const hydro_level_t* lv, int32_t n_levels, double gamma, int32_t scheme, double theta,
                 int32_t* n_bad_dev, uint32_t* work_dev, int32_t grid, int variant, hipStream_t s) {
  gh::BatchArgs<T> a;
  a.n_levels = n_levels;
  a.cfl = 0;
  long long total = 0;
  for (int l = 0; l < n_levels; ++l) {
    gh::BatchLevel<T>& b = a.lv[l];
    b.in = static_cast<const T*>(lv[l].level_dev);
    b.out = static_cast<T*>(lv[l].level_out_dev);
    b.geo.ngx = lv[l].ngx;
    b.geo.ngy = lv[l].ngy;
    b.geo.ngz = lv[l].ngz;
    for (int i = 0; i < 6; ++i) b.geo.bc[i] = lv[l].bc[i];
    b.g_begin = total;
    const double dt = lv[l].dt_dev != nullptr ? 1.0 : lv[l].dt;
    b.dtdx = T(dt / lv[l].dx);
    b.half_dtdx = T(0.5 * (dt / lv[l].dx));
    b.dt_dev = lv[l].dt_dev;
    b.dt_scale = lv[l].dt_dev_scale == 0.0 ? 1.0 : lv[l].dt_dev_scale;
    b.dx = lv[l].dx;
    b.dt_patch = lv[l].dt_patch_next_dev;
    b.dt_min = reinterpret_cast<unsigned long long*>(lv[l].dt_next_dev);
    b.reset = reinterpret_cast<unsigned long long*>(lv[l].dt_reset_dev);
    b.c_cfl_dx = lv[l].c_cfl * lv[l].dx;
    b.fold_scale = lv[l].dt_next_scale == 0.0 ? 1.0 : lv[l].dt_next_scale;
    a.cfl = a.cfl || b.dt_patch != nullptr || b.dt_min != nullptr || b.reset != nullptr;
    total += (long long)lv[l].ngx * lv[l].ngy * lv[l].ngz;
  }
  for (int l = n_levels; l < gh::kMaxLevels; ++l) {
    a.lv[l] = a.lv[0];
    a.lv[l].reset = nullptr;
  }
  a.total = total;
  a.gamma = gamma;
  if (total == 0) return HYDRO_OK;
  const int per_cu = sizeof(T) == 8 ? 2 : 4;  // workgroups that fit in one CU's LDS
  long long g = grid > 0 ? grid : (long long)device_cus() * per_cu;
  if (g > total) g = total;
  gh::Gas<T> gas = make_gas<T>(gamma, theta, 1.0, 1.0);
  const int fo = (scheme & HYDRO_FIRST_ORDER) ? 1 : 0, ws = (scheme >> 8) & 3;
  // work_dev NULL: the allocation-free entry point (the library's own counters)
  if (work_dev == nullptr)
    return device_status(gh::launch_mhm_batched_noalloc<T>(a, gas, fo, ws, n_bad_dev, variant, int(g), s));
  return device_status(gh::launch_mhm_batched<T>(a, gas, fo, ws, n_bad_dev, work_dev, variant, int(g), s));
}

// A level of ngx x ngy x ngz groups: cell indices along each axis (plus
// ghosts) fit in 32-bit ints and group indices in 31 bits.
bool level_geom_ok(long long ngx, long long ngy, long long ngz) {
  if (ngx < 1 || ngy < 1 || ngz < 1) return false;
  if (ngx > (1ll << 26) || ngy > (1ll << 26) || ngz > (1ll << 26)) return false;
  return ngx * ngy * ngz < (1ll << 31) - 8;
}

// The level adjoint and the ghost gather also pack group indices per axis in
// 19 bits and launch 16 workgroups per group.
bool adjoint_geom_ok(long long ngx, long long ngy, long long ngz) {
  if (!level_geom_ok(ngx, ngy, ngz)) return false;
  if (ngx >= (1ll << 19) || ngy >= (1ll << 19) || ngz >= (1ll << 19)) return false;
  return ngx * ngy * ngz < (1ll << 28) - 1;
}

int validate_levels(const hydro_level_t* lv, int32_t n_levels, int32_t dtype) {
  if (lv == nullptr || n_levels < 1 || n_levels > gh::kMaxLevels) return HYDRO_EINVAL;
  const size_t es = dtype_size(dtype);
  long long total = 0;
  for (int l = 0; l < n_levels; ++l) {
    const hydro_level_t& L = lv[l];
    if (!level_geom_ok(L.ngx, L.ngy, L.ngz) || !finite_pos(L.dx)) return HYDRO_EINVAL;
    if (L.dt_dev == nullptr && !finite_pos(L.dt)) return HYDRO_EINVAL;
    for (int i = 0; i < 6; ++i)
      if (L.bc[i] != HYDRO_BC_PERIODIC && L.bc[i] != HYDRO_BC_OUTFLOW) return HYDRO_EINVAL;
    if (L.level_dev == nullptr || L.level_out_dev == nullptr) return HYDRO_EINVAL;
    if (L.dt_dev != nullptr && L.dt_dev_scale != 0.0 && !finite_pos(L.dt_dev_scale)) return HYDRO_EINVAL;
    const bool want_cfl = L.dt_next_dev != nullptr || L.dt_patch_next_dev != nullptr || L.dt_reset_dev != nullptr;
    if (want_cfl && !finite_pos(L.c_cfl)) return HYDRO_EINVAL;
    if (L.dt_next_scale != 0.0 && !finite_pos(L.dt_next_scale)) return HYDRO_EINVAL;
    for (int m = 0; m < n_levels; ++m) {
      const hydro_level_t& M = lv[m];
      if (L.dt_reset_dev != nullptr && (L.dt_reset_dev == M.dt_dev || L.dt_reset_dev == M.dt_next_dev))
        return HYDRO_EINVAL;
      if (L.dt_next_dev != nullptr && L.dt_next_dev == M.dt_dev) return HYDRO_EINVAL;
    }
    total += (long long)L.ngx * L.ngy * L.ngz;
  }
  if (total >= (1ll << 32) - (1ll << 20)) return HYDRO_EINVAL;  // the work counter is 32-bit
  // an output may not overlap any input or any other output
  for (int a = 0; a < n_levels; ++a) {
    const size_t na = size_t(lv[a].ngx) * lv[a].ngy * lv[a].ngz * 5 * 4096 * es;
    for (int b = 0; b < n_levels; ++b) {
      const size_t nb = size_t(lv[b].ngx) * lv[b].ngy * lv[b].ngz * 5 * 4096 * es;
      if (overlap(lv[a].level_out_dev, na, lv[b].level_dev, nb)) return HYDRO_EINVAL;
      if (a != b && overlap(lv[a].level_out_dev, na, lv[b].level_out_dev, nb)) return HYDRO_EINVAL;
    }
  }
  return HYDRO_OK;
}

}  // namespace

namespace {

int check_level_args(const void* level_dev, const void* level_out_dev, int32_t ngx, int32_t ngy, int32_t ngz,
                     const int32_t* bc_host, int32_t dtype, double dt, double dx, double gamma, int32_t scheme,
                     double theta, const double* dt_dev, double c_cfl, double* dt_next_dev,
                     double* dt_patch_next_dev, double* dt_reset_dev, gh::LevelGeom* geo) {
  if (!level_geom_ok(ngx, ngy, ngz) || bc_host == nullptr) return HYDRO_EINVAL;
  if (dtype != HYDRO_F64 && dtype != HYDRO_F32) return HYDRO_EINVAL;
  if (!finite_pos(dx) || !(std::isfinite(gamma) && gamma > 1.0) || !valid_scheme(scheme, theta))
    return HYDRO_EINVAL;
  if (dt_dev == nullptr && !finite_pos(dt)) return HYDRO_EINVAL;
  const bool want_cfl = dt_next_dev != nullptr || dt_patch_next_dev != nullptr || dt_reset_dev != nullptr;
  if (want_cfl && !finite_pos(c_cfl)) return HYDRO_EINVAL;
  if (dt_reset_dev != nullptr && (dt_reset_dev == dt_dev || dt_reset_dev == dt_next_dev)) return HYDRO_EINVAL;
  if (dt_next_dev != nullptr && dt_next_dev == dt_dev) return HYDRO_EINVAL;
  geo->ngx = ngx;
  geo->ngy = ngy;
  geo->ngz = ngz;
  for (int i = 0; i < 6; ++i) {
    if (bc_host[i] != HYDRO_BC_PERIODIC && bc_host[i] != HYDRO_BC_OUTFLOW) return HYDRO_EINVAL;
    geo->bc[i] = bc_host[i];
  }
  if (level_dev == nullptr || level_out_dev == nullptr) return HYDRO_EINVAL;
  const int64_t G = int64_t(ngx) * ngy * ngz;
  const size_t bytes = size_t(G) * 5 * 4096 * dtype_size(dtype);
  if (overlap(level_dev, bytes, level_out_dev, bytes)) return HYDRO_EINVAL;
  return HYDRO_OK;
}

// hydro_advance_level after argument checks, with the launch shape given.
int level_launch(const void* level_dev, void* level_out_dev, const gh::LevelGeom& geo, int32_t dtype, double dt,
                 double dx, double gamma, int32_t scheme, double theta, const double* dt_dev, int32_t* n_bad_dev,
                 double c_cfl, double* dt_next_dev, double* dt_patch_next_dev, double* dt_reset_dev, int variant,
                 hipStream_t s) {
  gh::CflOut cfl;
  cfl.dt_patch = dt_patch_next_dev;
  cfl.dt_min = reinterpret_cast<unsigned long long*>(dt_next_dev);
  cfl.reset = reinterpret_cast<unsigned long long*>(dt_reset_dev);
  const bool with_cfl = cfl.dt_min != nullptr || cfl.dt_patch != nullptr || cfl.reset != nullptr;
  cfl.c_cfl_dx = with_cfl ? c_cfl * dx : 0.0;
  cfl.gamma = gamma;
  const int first_order = (scheme & HYDRO_FIRST_ORDER) ? 1 : 0;
  const int ws = (scheme >> 8) & 3;
  const double dt_host = dt_dev != nullptr ? 1.0 : dt;
  hipError_t e;
  if (dtype == HYDRO_F64)
    e = gh::launch_mhm_level(static_cast<const double*>(level_dev), static_cast<double*>(level_out_dev), geo,
                             make_gas<double>(gamma, theta, dt_host, dx), dt_dev, dx, first_order, ws, n_bad_dev, cfl,
                             variant, s);
  else
    e = gh::launch_mhm_level(static_cast<const float*>(level_dev), static_cast<float*>(level_out_dev), geo,
                             make_gas<float>(gamma, theta, dt_host, dx), dt_dev, dx, first_order, ws, n_bad_dev, cfl,
                             variant, s);
  return device_status(e);
}

int check_level_adjoint_args(const void* level_dev, const void* g_level_out_dev, void* g_level_in_dev, int32_t ngx,
                             int32_t ngy, int32_t ngz, const int32_t* bc_host, int32_t dtype, double dt, double dx,
                             double gamma, int32_t scheme, double theta, const double* dt_dev, void* work_dev,
                             int64_t work_bytes, gh::LevelGeom* geo) {
  if (!adjoint_geom_ok(ngx, ngy, ngz) || bc_host == nullptr || (dtype != HYDRO_F64 && dtype != HYDRO_F32))
    return HYDRO_EINVAL;
  if (!finite_pos(dx) || !(std::isfinite(gamma) && gamma > 1.0) || !valid_scheme(scheme, theta)) return HYDRO_EINVAL;
  if (dt_dev == nullptr && !finite_pos(dt)) return HYDRO_EINVAL;
  geo->ngx = ngx;
  geo->ngy = ngy;
  geo->ngz = ngz;
  for (int i = 0; i < 6; ++i) {
    if (bc_host[i] != HYDRO_BC_PERIODIC && bc_host[i] != HYDRO_BC_OUTFLOW) return HYDRO_EINVAL;
    geo->bc[i] = bc_host[i];
  }
  if (level_dev == nullptr || g_level_out_dev == nullptr || g_level_in_dev == nullptr || work_dev == nullptr)
    return HYDRO_EINVAL;
  const int64_t G = int64_t(ngx) * ngy * ngz;
  const size_t es = dtype_size(dtype);
  const size_t need = gh::adjoint_workspace_elems(G, true) * es;
  if (work_bytes < 0 || size_t(work_bytes) < need) return HYDRO_EINVAL;
  const size_t lb = size_t(G) * 5 * 4096 * es;
  if (overlap(g_level_in_dev, lb, level_dev, lb) || overlap(g_level_in_dev, lb, g_level_out_dev, lb) ||
      overlap(work_dev, need, level_dev, lb) || overlap(work_dev, need, g_level_out_dev, lb) ||
      overlap(work_dev, need, g_level_in_dev, lb))
    return HYDRO_EINVAL;
  return HYDRO_OK;
}

int level_adjoint_launch(const void* level_dev, const void* g_level_out_dev, void* g_level_in_dev,
                         const gh::LevelGeom& geo, int32_t dtype, double dt, double dx, double gamma, int32_t scheme,
                         double theta, const double* dt_dev, void* work_dev, int form, hipStream_t s) {
  const int first_order = (scheme & HYDRO_FIRST_ORDER) ? 1 : 0;
  const int ws = (scheme >> 8) & 3;
  const double dt_host = dt_dev != nullptr ? 1.0 : dt;
  hipError_t e;
  if (dtype == HYDRO_F64)
    e = gh::launch_mhm_adjoint_level(static_cast<const double*>(level_dev), static_cast<const double*>(g_level_out_dev),
                                     static_cast<double*>(g_level_in_dev), geo,
                                     make_gas<double>(gamma, theta, dt_host, dx), dt_dev, dx, first_order, ws,
                                     static_cast<double*>(work_dev), form == 1, s);
  else
    e = gh::launch_mhm_adjoint_level(static_cast<const float*>(level_dev), static_cast<const float*>(g_level_out_dev),
                                     static_cast<float*>(g_level_in_dev), geo,
                                     make_gas<float>(gamma, theta, dt_host, dx), dt_dev, dx, first_order, ws,
                                     static_cast<float*>(work_dev), form == 1, s);
  return device_status(e);
}

int batched_launch(const hydro_level_t* levels_host, int32_t n_levels, int32_t dtype, double gamma, int32_t scheme,
                   double theta, int32_t* n_bad_dev, uint32_t* work_dev, int32_t grid, int variant, hipStream_t s) {
  if (dtype == HYDRO_F64)
    return batched_impl<double>(levels_host, n_levels, gamma, scheme, theta, n_bad_dev, work_dev, grid, variant, s);
  return batched_impl<float>(levels_host, n_levels, gamma, scheme, theta, n_bad_dev, work_dev, grid, variant, s);
}

// Preference among launch shapes that time as ties: XCD-blocked before
// plain order, column-tile before linear sweep, lower before higher
// occupancy target (fewer HBM bytes per step at equal speed, measured), then
// the lower shape number.
int tie_rank(int v) { return ((v & 1) << 10) | ((~v & 4) << 7) | ((~v & 2) << 7) | v; }

// Times `launch(v)` for v in [0, n): two passes of 1 untimed + reps timed
// launches each, a shape's time the smaller of its two means (so clock
// ramp-up during the first pass does not decide).  Returns the fastest v or a
// negative status; ms[n] receives the times.
template <typename F>
int time_shapes(int n, int reps, hipStream_t s, float* ms, F launch) {
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return device_status(hipGetLastError());
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return device_status(hipGetLastError());
  }
  int status = HYDRO_OK;
  for (int pass = 0; pass < 2 && status == HYDRO_OK; ++pass) {
    for (int v = 0; v < n && status == HYDRO_OK; ++v) {
      status = launch(v);
      if (status != HYDRO_OK) break;
      hipError_t he = hipEventRecord(e0, s);
      for (int r = 0; r < reps && status == HYDRO_OK && he == hipSuccess; ++r) status = launch(v);
      if (status != HYDRO_OK) break;
      if (he == hipSuccess) he = hipEventRecord(e1, s);
      if (he == hipSuccess) he = hipEventSynchronize(e1);
      float t = 0.0f;
      if (he == hipSuccess) he = hipEventElapsedTime(&t, e0, e1);
      if (he != hipSuccess) {
        status = device_status(he);
        break;
      }
      t /= float(reps);
      if (pass == 0 || t < ms[v]) ms[v] = t;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (status != HYDRO_OK) return status;
  int best = 0;
  for (int v = 1; v < n; ++v)
    if (ms[v] < ms[best]) best = v;
  return best;
}

}  // namespace

extern "C" {

int hydro_version(void) { return 5; }

int hydro_last_hip_error(void) { return g_last_hip_error; }

const char* hydro_strerror(int status) {
  switch (status) {
    case HYDRO_OK:
      return "ok";
    case HYDRO_UNPHYSICAL:
      return "unphysical cells (rho <= 0 or p <= 0) in the result";
    case HYDRO_EINVAL:
      return "invalid argument";
    case HYDRO_EDEVICE:
      return "HIP runtime error";
    case HYDRO_ENOTUNED:
      return "no tuned launch shape for this call and the context requires one";
    case HYDRO_EIO:
      return "tuning cache unreadable, malformed or not writable";
    default:
      return "unknown status";
  }
}

// ------------------------------------------------------------ context ----
int hydro_ctx_create(hydro_ctx** ctx, const char* tune_cache_json_path) {
  if (ctx == nullptr) return HYDRO_EINVAL;
  *ctx = nullptr;
  hydro_ctx* c = new (std::nothrow) hydro_ctx();
  if (c == nullptr) return HYDRO_EINVAL;
  if (tune_cache_json_path != nullptr && tune_cache_json_path[0] != '\0') {
    c->cache_path = tune_cache_json_path;
    FILE* f = std::fopen(tune_cache_json_path, "r");
    if (f != nullptr) {  // a missing file is an empty cache
      std::string text;
      char buf[4096];
      size_t n;
      while ((n = std::fread(buf, 1, sizeof buf, f)) > 0) text.append(buf, n);
      std::fclose(f);
      if (!parse_cache(text, c->tuned)) {
        delete c;
        return HYDRO_EIO;
      }
    }
  }
  *ctx = c;
  return HYDRO_OK;
}

int hydro_ctx_destroy(hydro_ctx* ctx) {
  if (ctx == nullptr) return HYDRO_EINVAL;
  int status = HYDRO_OK;
  for (void* g : ctx->graphs) {
    const hipError_t e = hipGraphExecDestroy(static_cast<hipGraphExec_t>(g));
    if (e != hipSuccess && status == HYDRO_OK) status = device_status(e);
  }
  delete ctx;
  return status;
}

int hydro_ctx_save(hydro_ctx* ctx) {
  if (ctx == nullptr) return HYDRO_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  return save_cache_locked(ctx);
}

int hydro_ctx_set_require_tuned(hydro_ctx* ctx, int32_t on) {
  if (ctx == nullptr) return HYDRO_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->require_tuned = on != 0;
  return HYDRO_OK;
}

int hydro_ctx_num_tuned(hydro_ctx* ctx) {
  if (ctx == nullptr) return HYDRO_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  return int(ctx->tuned.size());
}

int hydro_check_unphysical(const int32_t* n_bad_dev, void* stream, int32_t* n_bad_host) {
  if (n_bad_dev == nullptr) return HYDRO_EINVAL;
  int32_t v = 0;
  hipError_t e = hipStreamSynchronize(static_cast<hipStream_t>(stream));
  if (e == hipSuccess) e = hipMemcpy(&v, n_bad_dev, sizeof v, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return device_status(e);
  if (n_bad_host != nullptr) *n_bad_host = v;
  return v > 0 ? HYDRO_UNPHYSICAL : HYDRO_OK;
}

// -------------------------------------------------------- padded step ----
int hydro_advance(const void* U_pad_dev, void* U_out_dev, int64_t n_groups, int32_t ghost, int32_t dtype,
                  double dt, double dx, double gamma, int32_t scheme, double theta, const double* dt_dev,
                  int32_t* n_bad_dev, void* stream) {
  if (n_groups < 0 || ghost < 2 || ghost > 16 || (dtype != HYDRO_F64 && dtype != HYDRO_F32)) return HYDRO_EINVAL;
  if (!finite_pos(dx) || !(std::isfinite(gamma) && gamma > 1.0) || !valid_scheme(scheme, theta))
    return HYDRO_EINVAL;
  if (dt_dev == nullptr && !finite_pos(dt)) return HYDRO_EINVAL;
  if (n_groups == 0) return HYDRO_OK;
  if (U_pad_dev == nullptr || U_out_dev == nullptr) return HYDRO_EINVAL;
  const int64_t P = 16 + 2 * ghost;
  const size_t es = dtype_size(dtype);
  if (overlap(U_pad_dev, size_t(n_groups) * 5 * P * P * P * es, U_out_dev, size_t(n_groups) * 5 * 4096 * es))
    return HYDRO_EINVAL;
  const int first_order = (scheme & HYDRO_FIRST_ORDER) ? 1 : 0;
  const int ws = (scheme >> 8) & 3;
  const double dt_host = dt_dev != nullptr ? 1.0 : dt;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (dtype == HYDRO_F64)
    e = gh::launch_mhm_fwd(static_cast<const double*>(U_pad_dev), static_cast<double*>(U_out_dev), n_groups, ghost,
                           make_gas<double>(gamma, theta, dt_host, dx), dt_dev, dx, first_order, ws, n_bad_dev, s);
  else
    e = gh::launch_mhm_fwd(static_cast<const float*>(U_pad_dev), static_cast<float*>(U_out_dev), n_groups, ghost,
                           make_gas<float>(gamma, theta, dt_host, dx), dt_dev, dx, first_order, ws, n_bad_dev, s);
  return device_status(e);
}

int hydro_branch_record(const void* U_pad_dev, void* U_out_dev, int64_t n_groups, int32_t ghost, int32_t dtype,
                        double dt, double dx, double gamma, int32_t scheme, double theta, uint32_t* record_dev,
                        void* stream) {
  if (n_groups < 0 || ghost < 2 || ghost > 16 || dtype != HYDRO_F64) return HYDRO_EINVAL;
  if (!finite_pos(dx) || !(std::isfinite(gamma) && gamma > 1.0) || !valid_scheme(scheme, theta) || !finite_pos(dt))
    return HYDRO_EINVAL;
  if (n_groups == 0) return HYDRO_OK;
  if (U_pad_dev == nullptr || U_out_dev == nullptr || record_dev == nullptr) return HYDRO_EINVAL;
  const int64_t P = 16 + 2 * ghost;
  if (overlap(U_pad_dev, size_t(n_groups) * 5 * P * P * P * 8, U_out_dev, size_t(n_groups) * 5 * 4096 * 8))
    return HYDRO_EINVAL;
  const int first_order = (scheme & HYDRO_FIRST_ORDER) ? 1 : 0;
  const int ws = (scheme >> 8) & 3;
  return device_status(gh::launch_mhm_record(static_cast<const double*>(U_pad_dev), static_cast<double*>(U_out_dev),
                                             n_groups, ghost, make_gas<double>(gamma, theta, dt, dx), nullptr, dx,
                                             first_order, ws, nullptr, record_dev, static_cast<hipStream_t>(stream)));
}

// ------------------------------------------------------- other schemes ----
int64_t hydro_ext_workspace_bytes(int64_t n_groups, int32_t ghost, int32_t dtype, int32_t scheme) {
  gh::ExtOpts o;
  if (n_groups < 0 || ghost > 16 || (dtype != HYDRO_F64 && dtype != HYDRO_F32) ||
      !valid_ext_scheme(scheme, 1.5, ghost, &o))
    return HYDRO_EINVAL;
  if (fused_plm_scheme(o)) return 0;
  return gh::ext_workspace_elems(n_groups, ghost, o) * int64_t(dtype_size(dtype));
}

int hydro_advance_ext(const void* U_pad_dev, void* U_out_dev, int64_t n_groups, int32_t ghost, int32_t dtype,
                      double dt, double dx, double gamma, int32_t scheme, double theta, double xi,
                      const double* dt_dev, int32_t* n_bad_dev, void* work_dev, int64_t work_bytes,
                      void* face_flux_dev, void* stream) {
  gh::ExtOpts o;
  if (n_groups < 0 || ghost > 16 || (dtype != HYDRO_F64 && dtype != HYDRO_F32)) return HYDRO_EINVAL;
  if (!finite_pos(dx) || !(std::isfinite(gamma) && gamma > 1.0) || !valid_ext_scheme(scheme, theta, ghost, &o))
    return HYDRO_EINVAL;
  if (o.de && (!(xi >= 0.0) || std::isnan(xi) || face_flux_dev != nullptr)) return HYDRO_EINVAL;
  o.xi = xi;
  const int64_t nf = o.de ? 6 : 5;
  if (dt_dev == nullptr && !finite_pos(dt)) return HYDRO_EINVAL;
  if (n_groups == 0) return HYDRO_OK;
  const int64_t P = 16 + 2 * ghost;
  const size_t es = dtype_size(dtype);
  const double dt_host = dt_dev != nullptr ? 1.0 : dt;
  hipStream_t s = static_cast<hipStream_t>(stream);
  if (fused_plm_scheme(o)) {
    // the fused per-group kernel; the workspace is not used
    if (U_pad_dev == nullptr || U_out_dev == nullptr) return HYDRO_EINVAL;
    const size_t pad_b = size_t(n_groups) * 5 * P * P * P * es, out_b = size_t(n_groups) * 5 * 4096 * es;
    const size_t ff_b = size_t(n_groups) * 9 * 5 * 256 * es;
    if (overlap(U_pad_dev, pad_b, U_out_dev, out_b) ||
        (face_flux_dev != nullptr &&
         (overlap(face_flux_dev, ff_b, U_pad_dev, pad_b) || overlap(face_flux_dev, ff_b, U_out_dev, out_b))))
      return HYDRO_EINVAL;
    hipError_t e;
    if (fused_ext_scheme(o)) {
      if (dtype == HYDRO_F64)
        e = gh::launch_mhm_fwd(static_cast<const double*>(U_pad_dev), static_cast<double*>(U_out_dev), n_groups,
                               ghost, make_gas<double>(gamma, theta, dt_host, dx), dt_dev, dx, o.first_order, o.ws,
                               n_bad_dev, s, static_cast<double*>(face_flux_dev));
      else
        e = gh::launch_mhm_fwd(static_cast<const float*>(U_pad_dev), static_cast<float*>(U_out_dev), n_groups,
                               ghost, make_gas<float>(gamma, theta, dt_host, dx), dt_dev, dx, o.first_order, o.ws,
                               n_bad_dev, s, static_cast<float*>(face_flux_dev));
    } else if (dtype == HYDRO_F64) {
      e = gh::launch_mhm_fwd_ext(static_cast<const double*>(U_pad_dev), static_cast<double*>(U_out_dev), n_groups,
                                 ghost, make_gas<double>(gamma, theta, dt_host, dx), dt_dev, dx, o, n_bad_dev, s,
                                 static_cast<double*>(face_flux_dev));
    } else {
      e = gh::launch_mhm_fwd_ext(static_cast<const float*>(U_pad_dev), static_cast<float*>(U_out_dev), n_groups,
                                 ghost, make_gas<float>(gamma, theta, dt_host, dx), dt_dev, dx, o, n_bad_dev, s,
                                 static_cast<float*>(face_flux_dev));
    }
    return device_status(e);
  }
  if (U_pad_dev == nullptr || U_out_dev == nullptr || work_dev == nullptr) return HYDRO_EINVAL;
  const int64_t per_group = gh::ext_workspace_elems(1, ghost, o) * int64_t(es);
  if (work_bytes < per_group) return HYDRO_EINVAL;
  const size_t pad_b = size_t(n_groups) * nf * P * P * P * es, out_b = size_t(n_groups) * nf * 4096 * es;
  const int64_t chunk = std::min<int64_t>(n_groups, work_bytes / per_group);
  const size_t work_b = size_t(gh::ext_workspace_elems(chunk, ghost, o)) * es;
  if (overlap(U_pad_dev, pad_b, U_out_dev, out_b) || overlap(work_dev, work_b, U_pad_dev, pad_b) ||
      overlap(work_dev, work_b, U_out_dev, out_b))
    return HYDRO_EINVAL;
  const size_t ff_b = size_t(n_groups) * 9 * 5 * 256 * es;
  if (face_flux_dev != nullptr && (overlap(face_flux_dev, ff_b, U_pad_dev, pad_b) ||
                                   overlap(face_flux_dev, ff_b, U_out_dev, out_b) ||
                                   overlap(face_flux_dev, ff_b, work_dev, work_b)))
    return HYDRO_EINVAL;
  // groups in chunks that fit the caller's workspace, one after another on the stream
  for (int64_t g0 = 0; g0 < n_groups; g0 += chunk) {
    const int64_t G = std::min(chunk, n_groups - g0);
    hipError_t e;
    if (dtype == HYDRO_F64)
      e = gh::launch_ext_step(static_cast<const double*>(U_pad_dev) + g0 * nf * P * P * P,
                              static_cast<double*>(U_out_dev) + g0 * nf * 4096, G, ghost,
                              make_gas<double>(gamma, theta, dt_host, dx), dt_dev, dx, o, n_bad_dev,
                              static_cast<double*>(work_dev),
                              face_flux_dev ? static_cast<double*>(face_flux_dev) + g0 * 9 * 5 * 256 : nullptr, s);
    else
      e = gh::launch_ext_step(static_cast<const float*>(U_pad_dev) + g0 * nf * P * P * P,
                              static_cast<float*>(U_out_dev) + g0 * nf * 4096, G, ghost,
                              make_gas<float>(gamma, theta, dt_host, dx), dt_dev, dx, o, n_bad_dev,
                              static_cast<float*>(work_dev),
                              face_flux_dev ? static_cast<float*>(face_flux_dev) + g0 * 9 * 5 * 256 : nullptr, s);
    if (e != hipSuccess) return device_status(e);
  }
  return HYDRO_OK;
}

// ------------------------------------------------ coarse-fine coupling ----
static_assert(sizeof(hydro_amr_level_t) == 48 && offsetof(hydro_amr_level_t, n_groups) == 24 &&
                  offsetof(hydro_amr_level_t, n) == 32,
              "hydro_amr_level_t layout");

namespace {

bool amr_level_ok(const hydro_amr_level_t* L, bool need_states) {
  if (L == nullptr || L->n_groups < 0 || L->pos_dev == nullptr || L->map_dev == nullptr) return false;
  if (need_states && L->U_dev == nullptr && L->n_groups > 0) return false;
  for (int d = 0; d < 3; ++d)
    if (L->n[d] < 1 || L->n[d] > (1 << 20)) return false;
  const int64_t cells = int64_t(L->n[0]) * L->n[1] * L->n[2];
  return L->n_groups <= cells && int64_t(L->n[0]) * 16 < (1ll << 30) && int64_t(L->n[1]) * 16 < (1ll << 30) &&
         int64_t(L->n[2]) * 16 < (1ll << 30);
}

// fine lattice = 2 x coarse lattice
bool amr_pair_ok(const hydro_amr_level_t* F, const hydro_amr_level_t* C) {
  return F->n[0] == 2 * C->n[0] && F->n[1] == 2 * C->n[1] && F->n[2] == 2 * C->n[2];
}

gh::AmrLevelArgs amr_args(const hydro_amr_level_t* L) {
  gh::AmrLevelArgs a;
  a.pos = L->pos_dev;
  a.map = L->map_dev;
  a.G = L->n_groups;
  for (int d = 0; d < 3; ++d) a.n[d] = L->n[d];
  return a;
}

bool bc_ok(const int32_t* bc) {
  if (bc == nullptr) return false;
  for (int i = 0; i < 6; ++i)
    if (bc[i] != HYDRO_BC_PERIODIC && bc[i] != HYDRO_BC_OUTFLOW) return false;
  return true;
}

}  // namespace

int hydro_amr_fill_ghosts(const hydro_amr_level_t* fine, const hydro_amr_level_t* coarse, const void* coarse_old_dev,
                          const void* coarse_new_dev, double a, const int32_t* bc_host, int32_t ghost, int32_t dtype,
                          void* U_pad_dev, void* stream) {
  if (!amr_level_ok(fine, true) || !bc_ok(bc_host) || ghost < 0 || ghost > 16 || U_pad_dev == nullptr ||
      (dtype != HYDRO_F64 && dtype != HYDRO_F32))
    return HYDRO_EINVAL;
  gh::AmrLevelArgs C{};
  if (coarse != nullptr) {
    if (!amr_level_ok(coarse, false) || !amr_pair_ok(fine, coarse) || coarse_old_dev == nullptr ||
        coarse_new_dev == nullptr || !(a >= 0.0 && a <= 1.0))
      return HYDRO_EINVAL;
    C = amr_args(coarse);
  } else if (fine->n_groups != int64_t(fine->n[0]) * fine->n[1] * fine->n[2]) {
    return HYDRO_EINVAL;  // only a level covering the domain needs no coarse level
  }
  const int64_t P = 16 + 2 * ghost;
  const size_t es = dtype_size(dtype);
  if (overlap(U_pad_dev, size_t(fine->n_groups) * 5 * P * P * P * es, fine->U_dev,
              size_t(fine->n_groups) * 5 * 4096 * es))
    return HYDRO_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (dtype == HYDRO_F64)
    e = gh::launch_amr_fill(static_cast<const double*>(fine->U_dev), amr_args(fine),
                            static_cast<const double*>(coarse_old_dev), static_cast<const double*>(coarse_new_dev), C,
                            a, bc_host, ghost, static_cast<double*>(U_pad_dev), s);
  else
    e = gh::launch_amr_fill(static_cast<const float*>(fine->U_dev), amr_args(fine),
                            static_cast<const float*>(coarse_old_dev), static_cast<const float*>(coarse_new_dev), C, a,
                            bc_host, ghost, static_cast<float*>(U_pad_dev), s);
  return device_status(e);
}

int hydro_amr_flux_accumulate(const hydro_amr_level_t* fine, const void* face_flux_dev, double weight,
                              const int32_t* bc_host, int32_t dtype, void* reg_dev, void* stream) {
  if (!amr_level_ok(fine, false) || !bc_ok(bc_host) || face_flux_dev == nullptr || reg_dev == nullptr ||
      !std::isfinite(weight) || (dtype != HYDRO_F64 && dtype != HYDRO_F32))
    return HYDRO_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (dtype == HYDRO_F64)
    e = gh::launch_amr_accumulate(amr_args(fine), static_cast<const double*>(face_flux_dev), weight, bc_host,
                                  static_cast<double*>(reg_dev), s);
  else
    e = gh::launch_amr_accumulate(amr_args(fine), static_cast<const float*>(face_flux_dev), weight, bc_host,
                                  static_cast<float*>(reg_dev), s);
  return device_status(e);
}

int hydro_amr_restrict(const hydro_amr_level_t* fine, const hydro_amr_level_t* coarse, int32_t dtype, void* stream) {
  if (!amr_level_ok(fine, true) || !amr_level_ok(coarse, true) || !amr_pair_ok(fine, coarse) ||
      (dtype != HYDRO_F64 && dtype != HYDRO_F32))
    return HYDRO_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (dtype == HYDRO_F64)
    e = gh::launch_amr_restrict(static_cast<const double*>(fine->U_dev), amr_args(fine),
                                static_cast<double*>(coarse->U_dev), amr_args(coarse), s);
  else
    e = gh::launch_amr_restrict(static_cast<const float*>(fine->U_dev), amr_args(fine),
                                static_cast<float*>(coarse->U_dev), amr_args(coarse), s);
  return device_status(e);
}

int hydro_amr_fixup(const hydro_amr_level_t* coarse, const hydro_amr_level_t* fine, const void* coarse_face_flux_dev,
                    const void* reg_dev, double dt_over_dx, const int32_t* bc_host, int32_t dtype, void* stream) {
  if (!amr_level_ok(fine, false) || !amr_level_ok(coarse, true) || !amr_pair_ok(fine, coarse) || !bc_ok(bc_host) ||
      coarse_face_flux_dev == nullptr || reg_dev == nullptr || !finite_pos(dt_over_dx) ||
      (dtype != HYDRO_F64 && dtype != HYDRO_F32))
    return HYDRO_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (dtype == HYDRO_F64)
    e = gh::launch_amr_fixup(static_cast<double*>(coarse->U_dev), amr_args(coarse), amr_args(fine),
                             static_cast<const double*>(coarse_face_flux_dev), static_cast<const double*>(reg_dev),
                             dt_over_dx, bc_host, s);
  else
    e = gh::launch_amr_fixup(static_cast<float*>(coarse->U_dev), amr_args(coarse), amr_args(fine),
                             static_cast<const float*>(coarse_face_flux_dev), static_cast<const float*>(reg_dev),
                             dt_over_dx, bc_host, s);
  return device_status(e);
}

// ------------------------------------- procedure for unphysical results ----
namespace {

// Level arguments shared by the two fallback entry points (scheme: any word
// hydro_advance_ext accepts).
int check_fallback_args(const void* in, const void* out, int32_t ngx, int32_t ngy, int32_t ngz, const int32_t* bc,
                        int32_t dtype, double dx, double gamma, int32_t scheme, double theta, gh::LevelGeom* geo,
                        gh::ExtOpts* o) {
  if (!level_geom_ok(ngx, ngy, ngz) || bc == nullptr || (dtype != HYDRO_F64 && dtype != HYDRO_F32)) return HYDRO_EINVAL;
  if (!finite_pos(dx) || !(std::isfinite(gamma) && gamma > 1.0) || !valid_ext_scheme(scheme, theta, 3, o) || o->de)
    return HYDRO_EINVAL;
  geo->ngx = ngx;
  geo->ngy = ngy;
  geo->ngz = ngz;
  for (int i = 0; i < 6; ++i) {
    if (bc[i] != HYDRO_BC_PERIODIC && bc[i] != HYDRO_BC_OUTFLOW) return HYDRO_EINVAL;
    geo->bc[i] = bc[i];
  }
  if (in == nullptr || out == nullptr) return HYDRO_EINVAL;
  const size_t bytes = size_t(int64_t(ngx) * ngy * ngz) * 5 * 4096 * dtype_size(dtype);
  if (overlap(in, bytes, out, bytes)) return HYDRO_EINVAL;
  return HYDRO_OK;
}

int repair_launch(const void* in, void* out, const gh::LevelGeom& geo, int32_t dtype, double dt, double dx,
                  double gamma, const gh::ExtOpts& o, const double* dt_dev, int32_t* counts, hipStream_t s) {
  const double dt_host = dt_dev != nullptr ? 1.0 : dt;
  hipError_t e;
  if (dtype == HYDRO_F64)
    e = gh::launch_repair(static_cast<const double*>(in), static_cast<double*>(out), geo,
                          make_gas<double>(gamma, 1.5, dt_host, dx), dt_dev, dx, o, counts, s);
  else
    e = gh::launch_repair(static_cast<const float*>(in), static_cast<float*>(out), geo,
                          make_gas<float>(gamma, 1.5, dt_host, dx), dt_dev, dx, o, counts, s);
  return device_status(e);
}

constexpr int64_t kFallbackCounterBytes = 256;

int64_t fallback_pad_bytes(int64_t G, int32_t dtype) {
  return (G * 5 * 22 * 22 * 22 * int64_t(dtype_size(dtype)) + 255) / 256 * 256;
}

}  // namespace

int hydro_repair_unphysical(const void* level_in_dev, void* level_out_dev, int32_t ngx, int32_t ngy, int32_t ngz,
                            const int32_t* bc_host, int32_t dtype, double dt, double dx, double gamma, int32_t scheme,
                            const double* dt_dev, int32_t* counts_dev, void* stream) {
  gh::LevelGeom geo;
  gh::ExtOpts o;
  int st = check_fallback_args(level_in_dev, level_out_dev, ngx, ngy, ngz, bc_host, dtype, dx, gamma, scheme, 1.5,
                               &geo, &o);
  if (st != HYDRO_OK) return st;
  if (counts_dev == nullptr || (dt_dev == nullptr && !finite_pos(dt))) return HYDRO_EINVAL;
  return repair_launch(level_in_dev, level_out_dev, geo, dtype, dt, dx, gamma, o, dt_dev, counts_dev,
                       static_cast<hipStream_t>(stream));
}

int64_t hydro_fallback_workspace_bytes(int32_t ngx, int32_t ngy, int32_t ngz, int32_t dtype, int32_t scheme) {
  gh::ExtOpts o;
  if (!level_geom_ok(ngx, ngy, ngz) || (dtype != HYDRO_F64 && dtype != HYDRO_F32) ||
      !valid_ext_scheme(scheme, 1.5, 3, &o) || o.de)
    return HYDRO_EINVAL;
  if (valid_scheme(scheme, 1.5)) return kFallbackCounterBytes;  // the fused level step needs no more
  const int64_t G = int64_t(ngx) * ngy * ngz;
  return kFallbackCounterBytes + fallback_pad_bytes(G, dtype) +
         gh::ext_workspace_elems(G, 3, o) * int64_t(dtype_size(dtype));
}

int hydro_advance_level_fallback(hydro_ctx* ctx, const void* level_in_dev, void* level_out_dev, int32_t ngx,
                                 int32_t ngy, int32_t ngz, const int32_t* bc_host, int32_t dtype, double dt,
                                 double dt_min, double ratio, double dx, double gamma, int32_t scheme, double theta,
                                 void* work_dev, int64_t work_bytes, double* info_host, void* stream) {
  gh::LevelGeom geo;
  gh::ExtOpts o;
  int st = check_fallback_args(level_in_dev, level_out_dev, ngx, ngy, ngz, bc_host, dtype, dx, gamma, scheme, theta,
                               &geo, &o);
  if (st != HYDRO_OK) return st;
  if (!finite_pos(dt) || !(ratio > 0.0 && ratio < 1.0) || !(dt_min >= 0.0) || std::isnan(dt_min) ||
      work_dev == nullptr || info_host == nullptr)
    return HYDRO_EINVAL;
  const int64_t need = hydro_fallback_workspace_bytes(ngx, ngy, ngz, dtype, scheme);
  if (need < 0 || work_bytes < need) return HYDRO_EINVAL;
  const int64_t G = int64_t(ngx) * ngy * ngz;
  const size_t lb = size_t(G) * 5 * 4096 * dtype_size(dtype);
  if (overlap(work_dev, size_t(need), level_in_dev, lb) || overlap(work_dev, size_t(need), level_out_dev, lb))
    return HYDRO_EINVAL;
  const bool fused = valid_scheme(scheme, theta);
  int variant = 0;
  if (fused) {
    st = select_shape(ctx, level_key(dtype, false, ngx, ngy, ngz), ctx ? &ctx->level_sel[dtype][0] : nullptr,
                      kDefaultLevelVariant, &variant);
    if (st != HYDRO_OK) return st;
  }
  hipStream_t s = static_cast<hipStream_t>(stream);
  int32_t* cnt = static_cast<int32_t*>(work_dev);  // [0..2] repair counters, [3] unphysical count of the step
  char* pad = static_cast<char*>(work_dev) + kFallbackCounterBytes;
  char* ext_work = pad + fallback_pad_bytes(G, dtype);
  int retries = 0;
  for (;;) {
    hipError_t e = gh::launch_zero_ints(cnt, 4, s);
    if (e != hipSuccess) return device_status(e);
    if (fused) {
      st = level_launch(level_in_dev, level_out_dev, geo, dtype, dt, dx, gamma, scheme, theta, nullptr, cnt + 3, 0.0,
                        nullptr, nullptr, nullptr, variant, s);
    } else {
      e = dtype == HYDRO_F64
              ? gh::launch_fill_ghosts(static_cast<const double*>(level_in_dev), reinterpret_cast<double*>(pad), ngx,
                                       ngy, ngz, 3, geo.bc, s)
              : gh::launch_fill_ghosts(static_cast<const float*>(level_in_dev), reinterpret_cast<float*>(pad), ngx,
                                       ngy, ngz, 3, geo.bc, s);
      if (e != hipSuccess) return device_status(e);
      st = hydro_advance_ext(pad, level_out_dev, G, 3, dtype, dt, dx, gamma, scheme, theta, 0.0, nullptr, cnt + 3,
                             ext_work, need - kFallbackCounterBytes - fallback_pad_bytes(G, dtype), nullptr, stream);
    }
    if (st != HYDRO_OK) return st;
    int32_t h[4] = {0, 0, 0, 0};
    e = hipMemcpyAsync(h, cnt, sizeof h, hipMemcpyDeviceToHost, s);
    if (e == hipSuccess) e = hipStreamSynchronize(s);
    if (e != hipSuccess) return device_status(e);
    if (h[3] > 0) {
      // the step counted unphysical items: scan its output and repair
      st = repair_launch(level_in_dev, level_out_dev, geo, dtype, dt, dx, gamma, o, nullptr, cnt, s);
      if (st != HYDRO_OK) return st;
      e = hipMemcpyAsync(h, cnt, sizeof h, hipMemcpyDeviceToHost, s);
      if (e == hipSuccess) e = hipStreamSynchronize(s);
      if (e != hipSuccess) return device_status(e);
    }
    const double next = dt * ratio;
    if (h[2] == 0 || next < dt_min) {
      info_host[0] = dt;
      info_host[1] = retries;
      info_host[2] = h[0];
      info_host[3] = h[1];
      return h[2] == 0 ? HYDRO_OK : HYDRO_UNPHYSICAL;
    }
    dt = next;
    ++retries;
  }
}

// --------------------------------------------------------- level step ----
int hydro_advance_level(hydro_ctx* ctx, const void* level_dev, void* level_out_dev, int32_t ngx, int32_t ngy,
                        int32_t ngz, const int32_t* bc_host, int32_t dtype, double dt, double dx, double gamma,
                        int32_t scheme, double theta, const double* dt_dev, int32_t* n_bad_dev, double c_cfl,
                        double* dt_next_dev, double* dt_patch_next_dev, double* dt_reset_dev, void* stream) {
  gh::LevelGeom geo;
  int st = check_level_args(level_dev, level_out_dev, ngx, ngy, ngz, bc_host, dtype, dt, dx, gamma, scheme, theta,
                            dt_dev, c_cfl, dt_next_dev, dt_patch_next_dev, dt_reset_dev, &geo);
  if (st != HYDRO_OK) return st;
  const bool with_cfl = dt_next_dev != nullptr || dt_patch_next_dev != nullptr || dt_reset_dev != nullptr;
  int variant = 0;
  st = select_shape(ctx, level_key(dtype, with_cfl, ngx, ngy, ngz),
                    ctx ? &ctx->level_sel[dtype][with_cfl ? 1 : 0] : nullptr, kDefaultLevelVariant, &variant);
  if (st != HYDRO_OK) return st;
  return level_launch(level_dev, level_out_dev, geo, dtype, dt, dx, gamma, scheme, theta, dt_dev, n_bad_dev, c_cfl,
                      dt_next_dev, dt_patch_next_dev, dt_reset_dev, variant, static_cast<hipStream_t>(stream));
}

int hydro_num_variants(void) { return gh::kLevelVariants; }

int hydro_get_level_variant(hydro_ctx* ctx, int32_t dtype, int32_t with_cfl) {
  if (dtype != HYDRO_F64 && dtype != HYDRO_F32) return HYDRO_EINVAL;
  if (ctx == nullptr) return kDefaultLevelVariant;
  std::lock_guard<std::mutex> lk(ctx->mu);
  const int v = ctx->level_sel[dtype][with_cfl ? 1 : 0];
  return v >= 0 ? v : kDefaultLevelVariant;
}

int hydro_set_level_variant(hydro_ctx* ctx, int32_t dtype, int32_t with_cfl, int32_t variant) {
  if (ctx == nullptr || (dtype != HYDRO_F64 && dtype != HYDRO_F32)) return HYDRO_EINVAL;
  if (variant < 0 || variant >= gh::kLevelVariants) return HYDRO_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->level_sel[dtype][with_cfl ? 1 : 0] = variant;
  // an explicit choice overrides earlier tuned choices of this dtype and form
  const std::string prefix = std::string("level/") + dtype_name(dtype) + (with_cfl ? "/cfl/" : "/plain/");
  for (auto it = ctx->tuned.begin(); it != ctx->tuned.end();)
    it = it->first.compare(0, prefix.size(), prefix) == 0 ? ctx->tuned.erase(it) : std::next(it);
  return HYDRO_OK;
}

int hydro_get_variant(hydro_ctx* ctx, int32_t dtype) { return hydro_get_level_variant(ctx, dtype, 1); }

int hydro_set_variant(hydro_ctx* ctx, int32_t dtype, int32_t variant) {
  int st = hydro_set_level_variant(ctx, dtype, 0, variant);
  if (st == HYDRO_OK) st = hydro_set_level_variant(ctx, dtype, 1, variant);
  return st;
}

int hydro_variant_name(int32_t variant, char* buf, int32_t len) {
  if (variant < 0 || variant >= gh::kLevelVariants || buf == nullptr || len < 1) return HYDRO_EINVAL;
  std::snprintf(buf, size_t(len), "%s %s order, %s occupancy target, %s LDS rows, %s per workgroup",
                (variant & 1) ? "plain" : "xcd-blocked", (variant & 4) ? "column-tile" : "linear",
                (variant & 2) ? "low" : "high", (variant & 8) ? "padded" : "packed",
                (variant & 16) ? "2 groups (512 threads)" : "1 group (256 threads)");
  return HYDRO_OK;
}

int hydro_autotune(hydro_ctx* ctx, const void* level_dev, void* scratch_out_dev, int32_t ngx, int32_t ngy,
                   int32_t ngz, const int32_t* bc_host, int32_t dtype, double dx, double gamma, double* cfl_scratch_dev,
                   int64_t cfl_scratch_bytes, int32_t reps, float* times_ms_host, void* stream) {
  if (ctx == nullptr || reps < 1 || reps > 1000) return HYDRO_EINVAL;
  const double dt = 1e-3 * dx;  // any positive step does the same work
  const int64_t G = int64_t(ngx) * ngy * ngz;
  // the CFL form's outputs: next dt, reset scalar, 8 patch time-steps per group
  if (cfl_scratch_dev == nullptr || G < 0 || cfl_scratch_bytes < int64_t(sizeof(double)) * (3 + 8 * G))
    return HYDRO_EINVAL;
  gh::LevelGeom geo;
  int st = check_level_args(level_dev, scratch_out_dev, ngx, ngy, ngz, bc_host, dtype, dt, dx, gamma,
                            HYDRO_SCHEME_MHM_PLM_HLLC, 1.5, nullptr, 0.5, cfl_scratch_dev, cfl_scratch_dev + 3,
                            cfl_scratch_dev + 1, &geo);
  if (st != HYDRO_OK) return st;
  const size_t lb = size_t(G) * 5 * 4096 * dtype_size(dtype), cb = sizeof(double) * size_t(3 + 8 * G);
  if (overlap(cfl_scratch_dev, cb, level_dev, lb) || overlap(cfl_scratch_dev, cb, scratch_out_dev, lb))
    return HYDRO_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  float ms[2][gh::kLevelVariants] = {};
  int best[2];
  for (int form = 0; form < 2; ++form) {
    double* dt_next = form ? cfl_scratch_dev : nullptr;
    double* dt_reset = form ? cfl_scratch_dev + 1 : nullptr;
    double* dt_patch = form ? cfl_scratch_dev + 3 : nullptr;
    best[form] = time_shapes(gh::kLevelVariants, reps, s, ms[form], [&](int v) {
      return level_launch(level_dev, scratch_out_dev, geo, dtype, dt, dx, gamma, HYDRO_SCHEME_MHM_PLM_HLLC, 1.5,
                          nullptr, nullptr, 0.5, dt_next, dt_patch, dt_reset, v, s);
    });
    if (best[form] < 0) return best[form];
    // The tuner relaunches one input, which stays partly in the caches; a
    // stepping loop reads each step's fresh output, where a group order's
    // extra HBM reads (measured: plain 3x, XCD-blocked linear 1.1x the
    // XCD-blocked column-tile order's) cost more than here.  Shapes within
    // 1.5% of the fastest are ties, resolved by tie_rank.
    {
      const float tie = 1.015f * ms[form][best[form]];
      int pick = -1;
      for (int v = 0; v < gh::kLevelVariants; ++v)
        if (ms[form][v] <= tie && (pick < 0 || tie_rank(v) < tie_rank(pick))) pick = v;
      best[form] = pick;
    }
  }
  if (times_ms_host != nullptr)
    for (int form = 0; form < 2; ++form)
      for (int v = 0; v < gh::kLevelVariants; ++v) times_ms_host[form * gh::kLevelVariants + v] = ms[form][v];
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->tuned[level_key(dtype, false, ngx, ngy, ngz)] = best[0];
    ctx->tuned[level_key(dtype, true, ngx, ngy, ngz)] = best[1];
    ctx->level_sel[dtype][0] = best[0];
    ctx->level_sel[dtype][1] = best[1];
    (void)save_cache_locked(ctx);
  }
  return best[1];
}

// ------------------------------------------------------------ batched ----
int hydro_advance_batched(hydro_ctx* ctx, const hydro_level_t* levels_host, int32_t n_levels, int32_t dtype,
                          double gamma, int32_t scheme, double theta, int32_t* n_bad_dev, uint32_t* work_dev,
                          int32_t grid, void* stream) {
  if ((dtype != HYDRO_F64 && dtype != HYDRO_F32) || !(std::isfinite(gamma) && gamma > 1.0) ||
      !valid_scheme(scheme, theta) || work_dev == nullptr || grid < 0)
    return HYDRO_EINVAL;
  int st = validate_levels(levels_host, n_levels, dtype);
  if (st != HYDRO_OK) return st;
  int variant = 0;
  st = select_shape(ctx, batched_key(dtype, levels_host, n_levels), ctx ? &ctx->batched_sel[dtype] : nullptr,
                    kDefaultBatchedVariant, &variant);
  if (st != HYDRO_OK) return st;
  return batched_launch(levels_host, n_levels, dtype, gamma, scheme, theta, n_bad_dev, work_dev, grid, variant,
                        static_cast<hipStream_t>(stream));
}

int hydro_advance_batched_noalloc(hydro_ctx* ctx, const hydro_level_t* levels_host, int32_t n_levels,
                                  int32_t dtype, double gamma, int32_t scheme, double theta, int32_t* n_bad_dev,
                                  int32_t grid, void* stream) {
  if ((dtype != HYDRO_F64 && dtype != HYDRO_F32) || !(std::isfinite(gamma) && gamma > 1.0) ||
      !valid_scheme(scheme, theta) || grid < 0)
    return HYDRO_EINVAL;
  int st = validate_levels(levels_host, n_levels, dtype);
  if (st != HYDRO_OK) return st;
  int variant = 0;
  st = select_shape(ctx, batched_key(dtype, levels_host, n_levels), ctx ? &ctx->batched_sel[dtype] : nullptr,
                    kDefaultBatchedVariant, &variant);
  if (st != HYDRO_OK) return st;
  return batched_launch(levels_host, n_levels, dtype, gamma, scheme, theta, n_bad_dev, nullptr, grid, variant,
                        static_cast<hipStream_t>(stream));
}

int hydro_set_batched_variant(hydro_ctx* ctx, int32_t dtype, int32_t variant) {
  if (ctx == nullptr || (dtype != HYDRO_F64 && dtype != HYDRO_F32)) return HYDRO_EINVAL;
  if (variant < 0 || variant >= gh::kBatchedVariants) return HYDRO_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->batched_sel[dtype] = variant;
  const std::string prefix = std::string("batched/") + dtype_name(dtype) + "/";
  for (auto it = ctx->tuned.begin(); it != ctx->tuned.end();)
    it = it->first.compare(0, prefix.size(), prefix) == 0 ? ctx->tuned.erase(it) : std::next(it);
  return HYDRO_OK;
}

int hydro_get_batched_variant(hydro_ctx* ctx, int32_t dtype) {
  if (dtype != HYDRO_F64 && dtype != HYDRO_F32) return HYDRO_EINVAL;
  if (ctx == nullptr) return kDefaultBatchedVariant;
  std::lock_guard<std::mutex> lk(ctx->mu);
  return ctx->batched_sel[dtype] >= 0 ? ctx->batched_sel[dtype] : kDefaultBatchedVariant;
}

int hydro_autotune_batched(hydro_ctx* ctx, const hydro_level_t* levels_host, int32_t n_levels, int32_t dtype,
                           double gamma, uint32_t* work_dev, int32_t reps, float* times_ms_host, void* stream) {
  if (ctx == nullptr || reps < 1 || reps > 1000 || (dtype != HYDRO_F64 && dtype != HYDRO_F32) ||
      work_dev == nullptr || !(std::isfinite(gamma) && gamma > 1.0))
    return HYDRO_EINVAL;
  const int v = validate_levels(levels_host, n_levels, dtype);
  if (v != HYDRO_OK) return v;
  hipStream_t s = static_cast<hipStream_t>(stream);
  float ms[gh::kBatchedVariants] = {};
  const int best = time_shapes(gh::kBatchedVariants, reps, s, ms, [&](int var) {
    return batched_launch(levels_host, n_levels, dtype, gamma, HYDRO_SCHEME_MHM_PLM_HLLC, 1.5, nullptr, work_dev, 0,
                          var, s);
  });
  if (best < 0) return best;
  if (times_ms_host != nullptr)
    for (int var = 0; var < gh::kBatchedVariants; ++var) times_ms_host[var] = ms[var];
  record_tuned(ctx, batched_key(dtype, levels_host, n_levels), best);
  return best;
}

// ------------------------------------------------------------- graphs ----
int hydro_graph_begin(void* stream) {
  if (stream == nullptr) return HYDRO_EINVAL;  // the null stream cannot be captured
  return device_status(hipStreamBeginCapture(static_cast<hipStream_t>(stream), hipStreamCaptureModeThreadLocal));
}

int hydro_graph_end(hydro_ctx* ctx, void* stream, void** graph_exec) {
  if (stream == nullptr || graph_exec == nullptr) return HYDRO_EINVAL;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(static_cast<hipStream_t>(stream), &g);
  if (e != hipSuccess) return device_status(e);
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return device_status(e);
  if (ctx != nullptr) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->graphs.insert(x);
  }
  *graph_exec = x;
  return HYDRO_OK;
}

int hydro_graph_launch(void* graph_exec, void* stream) {
  if (graph_exec == nullptr) return HYDRO_EINVAL;
  return device_status(hipGraphLaunch(static_cast<hipGraphExec_t>(graph_exec), static_cast<hipStream_t>(stream)));
}

int hydro_graph_destroy(hydro_ctx* ctx, void* graph_exec) {
  if (graph_exec == nullptr) return HYDRO_EINVAL;
  if (ctx != nullptr) {
    std::lock_guard<std::mutex> lk(ctx->mu);
    if (ctx->graphs.erase(graph_exec) == 0) return HYDRO_EINVAL;  // not captured through this context
  }
  return device_status(hipGraphExecDestroy(static_cast<hipGraphExec_t>(graph_exec)));
}

// ------------------------------------------------------------ adjoint ----
int64_t hydro_adjoint_workspace_bytes(int64_t n_groups, int32_t dtype, int32_t level) {
  if (n_groups < 0 || (dtype != HYDRO_F64 && dtype != HYDRO_F32)) return HYDRO_EINVAL;
  return int64_t(gh::adjoint_workspace_elems(n_groups, level != 0) * dtype_size(dtype));
}

int hydro_advance_adjoint(hydro_ctx* ctx, const void* U_pad_dev, const void* gU_out_dev, void* gU_pad_dev,
                          int64_t n_groups, int32_t ghost, int32_t dtype, double dt, double dx, double gamma,
                          int32_t scheme, double theta, void* work_dev, int64_t work_bytes, void* stream) {
  if (n_groups < 0 || ghost < 2 || ghost > 16 || (dtype != HYDRO_F64 && dtype != HYDRO_F32)) return HYDRO_EINVAL;
  if (!finite_pos(dt) || !finite_pos(dx) || !(std::isfinite(gamma) && gamma > 1.0) || !valid_scheme(scheme, theta))
    return HYDRO_EINVAL;
  if (n_groups == 0) return HYDRO_OK;
  if (U_pad_dev == nullptr || gU_out_dev == nullptr || gU_pad_dev == nullptr) return HYDRO_EINVAL;
  const size_t es = dtype_size(dtype);
  const size_t need = gh::adjoint_workspace_elems(n_groups, false) * es;
  if (work_bytes < 0 || size_t(work_bytes) < need || (need > 0 && work_dev == nullptr)) return HYDRO_EINVAL;
  const int64_t P = 16 + 2 * ghost;
  const size_t pad = size_t(n_groups) * 5 * P * P * P * es, out = size_t(n_groups) * 5 * 4096 * es;
  if (overlap(gU_pad_dev, pad, U_pad_dev, pad) || overlap(gU_pad_dev, pad, gU_out_dev, out) ||
      overlap(work_dev, need, U_pad_dev, pad) || overlap(work_dev, need, gU_out_dev, out) ||
      overlap(work_dev, need, gU_pad_dev, pad))
    return HYDRO_EINVAL;
  int form = 0;
  // the padded form has no tuned entry: it follows the explicit selection
  int st = select_shape(ctx, "adjoint/padded", ctx ? &ctx->adjoint_sel[dtype] : nullptr, kDefaultAdjointVariant, &form);
  if (st != HYDRO_OK) return st;
  const int first_order = (scheme & HYDRO_FIRST_ORDER) ? 1 : 0;
  const int ws = (scheme >> 8) & 3;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (dtype == HYDRO_F64)
    e = gh::launch_mhm_adjoint_padded(static_cast<const double*>(U_pad_dev), static_cast<const double*>(gU_out_dev),
                                      static_cast<double*>(gU_pad_dev), n_groups, ghost,
                                      make_gas<double>(gamma, theta, dt, dx), first_order, ws,
                                      static_cast<double*>(work_dev), form == 1, s);
  else
    e = gh::launch_mhm_adjoint_padded(static_cast<const float*>(U_pad_dev), static_cast<const float*>(gU_out_dev),
                                      static_cast<float*>(gU_pad_dev), n_groups, ghost,
                                      make_gas<float>(gamma, theta, dt, dx), first_order, ws,
                                      static_cast<float*>(work_dev), form == 1, s);
  return device_status(e);
}

int hydro_advance_level_adjoint(hydro_ctx* ctx, const void* level_dev, const void* g_level_out_dev,
                                void* g_level_in_dev, int32_t ngx, int32_t ngy, int32_t ngz, const int32_t* bc_host,
                                int32_t dtype, double dt, double dx, double gamma, int32_t scheme, double theta,
                                const double* dt_dev, void* work_dev, int64_t work_bytes, void* stream) {
  gh::LevelGeom geo;
  int st = check_level_adjoint_args(level_dev, g_level_out_dev, g_level_in_dev, ngx, ngy, ngz, bc_host, dtype, dt, dx,
                                    gamma, scheme, theta, dt_dev, work_dev, work_bytes, &geo);
  if (st != HYDRO_OK) return st;
  int form = 0;
  st = select_shape(ctx, adjoint_key(dtype, ngx, ngy, ngz), ctx ? &ctx->adjoint_sel[dtype] : nullptr,
                    kDefaultAdjointVariant, &form);
  if (st != HYDRO_OK) return st;
  return level_adjoint_launch(level_dev, g_level_out_dev, g_level_in_dev, geo, dtype, dt, dx, gamma, scheme, theta,
                              dt_dev, work_dev, form, static_cast<hipStream_t>(stream));
}

int hydro_autotune_adjoint(hydro_ctx* ctx, const void* level_dev, const void* g_level_out_dev, void* g_level_in_dev,
                           int32_t ngx, int32_t ngy, int32_t ngz, const int32_t* bc_host, int32_t dtype, double dx,
                           double gamma, void* work_dev, int64_t work_bytes, int32_t reps, float* times_ms_host,
                           void* stream) {
  if (ctx == nullptr || reps < 1 || reps > 1000) return HYDRO_EINVAL;
  const double dt = 1e-3 * dx;  // any positive step does the same work
  gh::LevelGeom geo;
  const int st = check_level_adjoint_args(level_dev, g_level_out_dev, g_level_in_dev, ngx, ngy, ngz, bc_host, dtype,
                                          dt, dx, gamma, HYDRO_SCHEME_MHM_PLM_HLLC, 1.5, nullptr, work_dev,
                                          work_bytes, &geo);
  if (st != HYDRO_OK) return st;
  hipStream_t s = static_cast<hipStream_t>(stream);
  float ms[2] = {};
  const int best = time_shapes(2, reps, s, ms, [&](int form) {
    return level_adjoint_launch(level_dev, g_level_out_dev, g_level_in_dev, geo, dtype, dt, dx, gamma,
                                HYDRO_SCHEME_MHM_PLM_HLLC, 1.5, nullptr, work_dev, form, s);
  });
  if (best < 0) return best;
  if (times_ms_host != nullptr) {
    times_ms_host[0] = ms[0];
    times_ms_host[1] = ms[1];
  }
  {
    std::lock_guard<std::mutex> lk(ctx->mu);
    ctx->tuned[adjoint_key(dtype, ngx, ngy, ngz)] = best;
    ctx->adjoint_sel[dtype] = best;
    (void)save_cache_locked(ctx);
  }
  return best;
}

int hydro_set_adjoint_variant(hydro_ctx* ctx, int32_t dtype, int32_t variant) {
  if (ctx == nullptr || (dtype != HYDRO_F64 && dtype != HYDRO_F32)) return HYDRO_EINVAL;
  if (variant != 0 && variant != 1) return HYDRO_EINVAL;
  std::lock_guard<std::mutex> lk(ctx->mu);
  ctx->adjoint_sel[dtype] = variant;
  const std::string prefix = std::string("adjoint/") + dtype_name(dtype) + "/";
  for (auto it = ctx->tuned.begin(); it != ctx->tuned.end();)
    it = it->first.compare(0, prefix.size(), prefix) == 0 ? ctx->tuned.erase(it) : std::next(it);
  return HYDRO_OK;
}

int hydro_get_adjoint_variant(hydro_ctx* ctx, int32_t dtype) {
  if (dtype != HYDRO_F64 && dtype != HYDRO_F32) return HYDRO_EINVAL;
  if (ctx == nullptr) return kDefaultAdjointVariant;
  std::lock_guard<std::mutex> lk(ctx->mu);
  return ctx->adjoint_sel[dtype] >= 0 ? ctx->adjoint_sel[dtype] : kDefaultAdjointVariant;
}

int hydro_dt(const void* U_pad_dev, int64_t n_groups, int32_t ghost, int32_t dtype, double dx, double gamma,
             double c_cfl, double* dt_patch_dev, double* dt_min_dev, void* stream) {
  if (n_groups < 0 || ghost < 0 || ghost > 16 || (dtype != HYDRO_F64 && dtype != HYDRO_F32)) return HYDRO_EINVAL;
  if (!finite_pos(dx) || !finite_pos(c_cfl) || !(std::isfinite(gamma) && gamma > 1.0)) return HYDRO_EINVAL;
  if (n_groups > 0 && (U_pad_dev == nullptr || dt_patch_dev == nullptr)) return HYDRO_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (dtype == HYDRO_F64)
    e = gh::launch_cfl_dt(static_cast<const double*>(U_pad_dev), n_groups, ghost, dx, gamma, c_cfl, dt_patch_dev,
                          dt_min_dev, s);
  else
    e = gh::launch_cfl_dt(static_cast<const float*>(U_pad_dev), n_groups, ghost, dx, gamma, c_cfl, dt_patch_dev,
                          dt_min_dev, s);
  return device_status(e);
}

int hydro_fill_ghosts(const void* level_dev, void* U_pad_dev, int32_t ngx, int32_t ngy, int32_t ngz, int32_t ghost,
                      int32_t dtype, const int32_t* bc_host, void* stream) {
  if (!level_geom_ok(ngx, ngy, ngz) || ghost < 0 || ghost > 16 || bc_host == nullptr) return HYDRO_EINVAL;
  if (dtype != HYDRO_F64 && dtype != HYDRO_F32) return HYDRO_EINVAL;
  int bc[6];
  for (int i = 0; i < 6; ++i) {
    if (bc_host[i] != HYDRO_BC_PERIODIC && bc_host[i] != HYDRO_BC_OUTFLOW) return HYDRO_EINVAL;
    bc[i] = bc_host[i];
  }
  if (level_dev == nullptr || U_pad_dev == nullptr) return HYDRO_EINVAL;
  const int64_t G = int64_t(ngx) * ngy * ngz, P = 16 + 2 * ghost;
  const size_t es = dtype_size(dtype);
  if (overlap(level_dev, size_t(G) * 5 * 4096 * es, U_pad_dev, size_t(G) * 5 * P * P * P * es)) return HYDRO_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (dtype == HYDRO_F64)
    e = gh::launch_fill_ghosts(static_cast<const double*>(level_dev), static_cast<double*>(U_pad_dev), ngx, ngy, ngz,
                               ghost, bc, s);
  else
    e = gh::launch_fill_ghosts(static_cast<const float*>(level_dev), static_cast<float*>(U_pad_dev), ngx, ngy, ngz,
                               ghost, bc, s);
  return device_status(e);
}

int hydro_gather_ghost_adjoint(const void* g_pad_dev, void* g_level_dev, int32_t ngx, int32_t ngy, int32_t ngz,
                               int32_t ghost, int32_t dtype, const int32_t* bc_host, void* stream) {
  if (!adjoint_geom_ok(ngx, ngy, ngz) || ghost < 0 || ghost > 16 || bc_host == nullptr) return HYDRO_EINVAL;
  if (dtype != HYDRO_F64 && dtype != HYDRO_F32) return HYDRO_EINVAL;
  gh::LevelGeom geo;
  geo.ngx = ngx;
  geo.ngy = ngy;
  geo.ngz = ngz;
  for (int i = 0; i < 6; ++i) {
    if (bc_host[i] != HYDRO_BC_PERIODIC && bc_host[i] != HYDRO_BC_OUTFLOW) return HYDRO_EINVAL;
    geo.bc[i] = bc_host[i];
  }
  if (g_pad_dev == nullptr || g_level_dev == nullptr) return HYDRO_EINVAL;
  const int64_t G = int64_t(ngx) * ngy * ngz, P = 16 + 2 * ghost;
  const size_t es = dtype_size(dtype);
  if (overlap(g_level_dev, size_t(G) * 5 * 4096 * es, g_pad_dev, size_t(G) * 5 * P * P * P * es)) return HYDRO_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (dtype == HYDRO_F64)
    e = gh::launch_gather_ghost_adjoint(static_cast<const double*>(g_pad_dev), static_cast<double*>(g_level_dev), geo,
                                        ghost, s);
  else
    e = gh::launch_gather_ghost_adjoint(static_cast<const float*>(g_pad_dev), static_cast<float*>(g_level_dev), geo,
                                        ghost, s);
  return device_status(e);
}

}  // extern "C"
