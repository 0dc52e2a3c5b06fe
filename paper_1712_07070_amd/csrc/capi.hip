// extern "C" entry points of libhydro: argument validation and dispatch to
// the kernels.  Declarations and documentation: include/hydro.h.

#include <atomic>
#include <cmath>
#include <cstdint>
#include <cstdio>

#include "hydro.h"
#include "kernels.h"

#include <cstddef>

// the Python binding mirrors this layout with ctypes
static_assert(sizeof(hydro_level_t) == 80 && offsetof(hydro_level_t, dt) == 56 &&
                  offsetof(hydro_level_t, dt_dev) == 72,
              "hydro_level_t layout");

namespace {

thread_local int g_last_hip_error = 0;

// Launch shape of the level step per dtype (index into the variants of
// mhm_fwd.hip); set by hydro_set_variant or hydro_autotune, process-wide.
// [dtype][with CFL epilogue]: the two kernels differ in register needs, so
// each gets its own shape.
std::atomic<int> g_level_variant[2][2] = {{{1}, {1}}, {{1}, {1}}};  // measured defaults: plain order, high occupancy
// Form of the step adjoint per dtype: 0 fused single sweep, 1 two kernels
// with a face workspace.
std::atomic<int> g_adjoint_variant[2] = {{0}, {0}};  // measured: fused faster in both dtypes
// Launch shape of the batched kernel per dtype (bit 0: item order, bit 1:
// occupancy target, bit 2: per-XCD queues).
std::atomic<int> g_batched_variant[2] = {{0}, {0}};  // one queue, high occupancy

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
    b.dx = lv[l].dx;
    total += (long long)lv[l].ngx * lv[l].ngy * lv[l].ngz;
  }
  for (int l = n_levels; l < gh::kMaxLevels; ++l) a.lv[l] = a.lv[0];
  a.total = total;
  if (total == 0) return HYDRO_OK;
  const int per_cu = sizeof(T) == 8 ? 2 : 4;  // workgroups that fit in one CU's LDS
  long long g = grid > 0 ? grid : (long long)device_cus() * per_cu;
  if (g > total) g = total;
  gh::Gas<T> gas = make_gas<T>(gamma, theta, 1.0, 1.0);
  return device_status(gh::launch_mhm_batched<T>(a, gas, (scheme & HYDRO_FIRST_ORDER) ? 1 : 0, (scheme >> 8) & 3,
                                                 n_bad_dev, work_dev, variant, int(g), s));
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

extern "C" {

int hydro_version(void) { return 4; }

int hydro_last_hip_error(void) { return g_last_hip_error; }

const char* hydro_strerror(int status) {
  switch (status) {
    case HYDRO_OK:
      return "ok";
    case HYDRO_EINVAL:
      return "invalid argument";
    case HYDRO_EDEVICE:
      return "HIP runtime error";
    default:
      return "unknown status";
  }
}

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

int hydro_advance_level(const void* level_dev, void* level_out_dev, int32_t ngx, int32_t ngy, int32_t ngz,
                        const int32_t* bc_host, int32_t dtype, double dt, double dx, double gamma, int32_t scheme,
                        double theta, const double* dt_dev, int32_t* n_bad_dev, double c_cfl, double* dt_next_dev,
                        double* dt_patch_next_dev, double* dt_reset_dev, void* stream) {
  if (!level_geom_ok(ngx, ngy, ngz) || bc_host == nullptr) return HYDRO_EINVAL;
  if (dtype != HYDRO_F64 && dtype != HYDRO_F32) return HYDRO_EINVAL;
  if (!finite_pos(dx) || !(std::isfinite(gamma) && gamma > 1.0) || !valid_scheme(scheme, theta))
    return HYDRO_EINVAL;
  if (dt_dev == nullptr && !finite_pos(dt)) return HYDRO_EINVAL;
  const bool want_cfl = dt_next_dev != nullptr || dt_patch_next_dev != nullptr || dt_reset_dev != nullptr;
  if (want_cfl && !finite_pos(c_cfl)) return HYDRO_EINVAL;
  if (dt_reset_dev != nullptr && (dt_reset_dev == dt_dev || dt_reset_dev == dt_next_dev)) return HYDRO_EINVAL;
  if (dt_next_dev != nullptr && dt_next_dev == dt_dev) return HYDRO_EINVAL;
  gh::LevelGeom geo;
  geo.ngx = ngx;
  geo.ngy = ngy;
  geo.ngz = ngz;
  for (int i = 0; i < 6; ++i) {
    if (bc_host[i] != HYDRO_BC_PERIODIC && bc_host[i] != HYDRO_BC_OUTFLOW) return HYDRO_EINVAL;
    geo.bc[i] = bc_host[i];
  }
  if (level_dev == nullptr || level_out_dev == nullptr) return HYDRO_EINVAL;
  const int64_t G = int64_t(ngx) * ngy * ngz;
  const size_t bytes = size_t(G) * 5 * 4096 * dtype_size(dtype);
  if (overlap(level_dev, bytes, level_out_dev, bytes)) return HYDRO_EINVAL;
  gh::CflOut cfl;
  cfl.dt_patch = dt_patch_next_dev;
  cfl.dt_min = reinterpret_cast<unsigned long long*>(dt_next_dev);
  cfl.reset = reinterpret_cast<unsigned long long*>(dt_reset_dev);
  cfl.c_cfl_dx = want_cfl ? c_cfl * dx : 0.0;
  cfl.gamma = gamma;
  const int first_order = (scheme & HYDRO_FIRST_ORDER) ? 1 : 0;
  const int ws = (scheme >> 8) & 3;
  const double dt_host = dt_dev != nullptr ? 1.0 : dt;
  const bool with_cfl = cfl.dt_min != nullptr || cfl.dt_patch != nullptr || cfl.reset != nullptr;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (dtype == HYDRO_F64)
    e = gh::launch_mhm_level(static_cast<const double*>(level_dev), static_cast<double*>(level_out_dev), geo,
                             make_gas<double>(gamma, theta, dt_host, dx), dt_dev, dx, first_order, ws, n_bad_dev, cfl,
                             g_level_variant[0][with_cfl ? 1 : 0].load(), s);
  else
    e = gh::launch_mhm_level(static_cast<const float*>(level_dev), static_cast<float*>(level_out_dev), geo,
                             make_gas<float>(gamma, theta, dt_host, dx), dt_dev, dx, first_order, ws, n_bad_dev, cfl,
                             g_level_variant[1][with_cfl ? 1 : 0].load(), s);
  return device_status(e);
}

int hydro_num_variants(void) { return gh::kLevelVariants; }

int hydro_get_level_variant(int32_t dtype, int32_t with_cfl) {
  if (dtype != HYDRO_F64 && dtype != HYDRO_F32) return HYDRO_EINVAL;
  return g_level_variant[dtype][with_cfl ? 1 : 0].load();
}

int hydro_set_level_variant(int32_t dtype, int32_t with_cfl, int32_t variant) {
  if (dtype != HYDRO_F64 && dtype != HYDRO_F32) return HYDRO_EINVAL;
  if (variant < 0 || variant >= gh::kLevelVariants) return HYDRO_EINVAL;
  g_level_variant[dtype][with_cfl ? 1 : 0].store(variant);
  return HYDRO_OK;
}

int hydro_get_variant(int32_t dtype) { return hydro_get_level_variant(dtype, 1); }

int hydro_set_variant(int32_t dtype, int32_t variant) {
  int st = hydro_set_level_variant(dtype, 0, variant);
  if (st == HYDRO_OK) st = hydro_set_level_variant(dtype, 1, variant);
  return st;
}

int hydro_variant_name(int32_t variant, char* buf, int32_t len) {
  if (variant < 0 || variant >= gh::kLevelVariants || buf == nullptr || len < 1) return HYDRO_EINVAL;
  std::snprintf(buf, size_t(len), "%s order, %s occupancy target", (variant & 1) ? "plain" : "xcd-blocked",
                (variant & 2) ? "low" : "high");
  return HYDRO_OK;
}

int hydro_autotune(const void* level_dev, void* scratch_out_dev, int32_t ngx, int32_t ngy, int32_t ngz,
                   const int32_t* bc_host, int32_t dtype, double dx, double gamma, int32_t reps, float* times_ms_host,
                   void* stream) {
  if (reps < 1 || reps > 1000 || (dtype != HYDRO_F64 && dtype != HYDRO_F32)) return HYDRO_EINVAL;
  if (!level_geom_ok(ngx, ngy, ngz)) return HYDRO_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int saved[2] = {g_level_variant[dtype][0].load(), g_level_variant[dtype][1].load()};
  // CFL outputs of the timed CFL-epilogue launches: 3 scalars + 8 per group
  const int64_t G = int64_t(ngx) * ngy * ngz;
  double* cfl_buf = nullptr;
  if (hipMalloc(&cfl_buf, sizeof(double) * size_t(3 + 8 * G)) != hipSuccess) return device_status(hipGetLastError());
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) {
    (void)hipFree(cfl_buf);
    return device_status(hipGetLastError());
  }
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    (void)hipFree(cfl_buf);
    return device_status(hipGetLastError());
  }
  int best[2] = {-1, -1}, status = HYDRO_OK;
  float best_ms[2] = {0.0f, 0.0f};
  float ms_min[2][gh::kLevelVariants] = {};
  const double dt = 1e-3 * dx;  // any positive step does the same work
  // two passes over every (form, shape); a shape's time is the smaller of its
  // two, so clock ramp-up or drift during the first pass does not decide
  for (int pass = 0; pass < 2 && status == HYDRO_OK; ++pass) {
    for (int form = 0; form < 2 && status == HYDRO_OK; ++form) {
      double* dt_next = form ? cfl_buf : nullptr;
      double* dt_reset = form ? cfl_buf + 1 : nullptr;
      double* dt_patch = form ? cfl_buf + 3 : nullptr;
      for (int v = 0; v < gh::kLevelVariants && status == HYDRO_OK; ++v) {
        g_level_variant[dtype][form].store(v);
        auto launch = [&]() {
          return hydro_advance_level(level_dev, scratch_out_dev, ngx, ngy, ngz, bc_host, dtype, dt, dx, gamma,
                                     HYDRO_SCHEME_MHM_PLM_HLLC, 1.5, nullptr, nullptr, 0.5, dt_next, dt_patch,
                                     dt_reset, stream);
        };
        // one untimed launch, then `reps` timed ones
        status = launch();
        if (status != HYDRO_OK) break;
        hipError_t he = hipEventRecord(e0, s);
        for (int r = 0; r < reps && status == HYDRO_OK && he == hipSuccess; ++r) status = launch();
        if (status != HYDRO_OK) break;
        if (he == hipSuccess) he = hipEventRecord(e1, s);
        if (he == hipSuccess) he = hipEventSynchronize(e1);
        float ms = 0.0f;
        if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
        if (he != hipSuccess) {
          status = device_status(he);
          break;
        }
        ms /= float(reps);
        if (pass == 0 || ms < ms_min[form][v]) ms_min[form][v] = ms;
      }
    }
  }
  for (int form = 0; form < 2 && status == HYDRO_OK; ++form) {
    for (int v = 0; v < gh::kLevelVariants; ++v) {
      if (times_ms_host != nullptr) times_ms_host[form * gh::kLevelVariants + v] = ms_min[form][v];
      if (best[form] < 0 || ms_min[form][v] < best_ms[form]) {
        best[form] = v;
        best_ms[form] = ms_min[form][v];
      }
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  (void)hipStreamSynchronize(s);
  (void)hipFree(cfl_buf);
  if (status != HYDRO_OK) {
    g_level_variant[dtype][0].store(saved[0]);
    g_level_variant[dtype][1].store(saved[1]);
    return status;
  }
  g_level_variant[dtype][0].store(best[0]);
  g_level_variant[dtype][1].store(best[1]);
  return best[1];
}

int hydro_advance_batched(const hydro_level_t* levels_host, int32_t n_levels, int32_t dtype, double gamma,
                          int32_t scheme, double theta, int32_t* n_bad_dev, uint32_t* work_dev, int32_t grid,
                          void* stream) {
  if ((dtype != HYDRO_F64 && dtype != HYDRO_F32) || !(std::isfinite(gamma) && gamma > 1.0) ||
      !valid_scheme(scheme, theta) || work_dev == nullptr || grid < 0)
    return HYDRO_EINVAL;
  const int v = validate_levels(levels_host, n_levels, dtype);
  if (v != HYDRO_OK) return v;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int variant = g_batched_variant[dtype].load();
  if (dtype == HYDRO_F64)
    return batched_impl<double>(levels_host, n_levels, gamma, scheme, theta, n_bad_dev, work_dev, grid, variant, s);
  return batched_impl<float>(levels_host, n_levels, gamma, scheme, theta, n_bad_dev, work_dev, grid, variant, s);
}

int hydro_set_batched_variant(int32_t dtype, int32_t variant) {
  if (dtype != HYDRO_F64 && dtype != HYDRO_F32) return HYDRO_EINVAL;
  if (variant < 0 || variant >= gh::kBatchedVariants) return HYDRO_EINVAL;
  g_batched_variant[dtype].store(variant);
  return HYDRO_OK;
}

int hydro_get_batched_variant(int32_t dtype) {
  if (dtype != HYDRO_F64 && dtype != HYDRO_F32) return HYDRO_EINVAL;
  return g_batched_variant[dtype].load();
}

int hydro_autotune_batched(const hydro_level_t* levels_host, int32_t n_levels, int32_t dtype, double gamma,
                           uint32_t* work_dev, int32_t reps, float* times_ms_host, void* stream) {
  if (reps < 1 || reps > 1000 || (dtype != HYDRO_F64 && dtype != HYDRO_F32) || work_dev == nullptr)
    return HYDRO_EINVAL;
  const int v = validate_levels(levels_host, n_levels, dtype);
  if (v != HYDRO_OK) return v;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int saved = g_batched_variant[dtype].load();
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return device_status(hipGetLastError());
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return device_status(hipGetLastError());
  }
  int best = -1, status = HYDRO_OK;
  float best_ms = 0.0f;
  float ms_min[gh::kBatchedVariants] = {};
  // two passes, a shape's time is the smaller of its two (as hydro_autotune)
  for (int pass = 0; pass < 2 && status == HYDRO_OK; ++pass) {
    for (int var = 0; var < gh::kBatchedVariants && status == HYDRO_OK; ++var) {
      g_batched_variant[dtype].store(var);
      status = hydro_advance_batched(levels_host, n_levels, dtype, gamma, HYDRO_SCHEME_MHM_PLM_HLLC, 1.5, nullptr,
                                     work_dev, 0, stream);
      if (status != HYDRO_OK) break;
      hipError_t he = hipEventRecord(e0, s);
      for (int r = 0; r < reps && status == HYDRO_OK && he == hipSuccess; ++r)
        status = hydro_advance_batched(levels_host, n_levels, dtype, gamma, HYDRO_SCHEME_MHM_PLM_HLLC, 1.5, nullptr,
                                       work_dev, 0, stream);
      if (status != HYDRO_OK) break;
      if (he == hipSuccess) he = hipEventRecord(e1, s);
      if (he == hipSuccess) he = hipEventSynchronize(e1);
      float ms = 0.0f;
      if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
      if (he != hipSuccess) {
        status = device_status(he);
        break;
      }
      ms /= float(reps);
      if (pass == 0 || ms < ms_min[var]) ms_min[var] = ms;
    }
  }
  for (int var = 0; var < gh::kBatchedVariants && status == HYDRO_OK; ++var) {
    if (times_ms_host != nullptr) times_ms_host[var] = ms_min[var];
    if (best < 0 || ms_min[var] < best_ms) {
      best = var;
      best_ms = ms_min[var];
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (status != HYDRO_OK) {
    g_batched_variant[dtype].store(saved);
    return status;
  }
  g_batched_variant[dtype].store(best);
  return best;
}

// ------------------------------------------------------------- graphs ----
int hydro_graph_begin(void* stream) {
  if (stream == nullptr) return HYDRO_EINVAL;  // the null stream cannot be captured
  return device_status(hipStreamBeginCapture(static_cast<hipStream_t>(stream), hipStreamCaptureModeThreadLocal));
}

int hydro_graph_end(void* stream, void** graph_exec) {
  if (stream == nullptr || graph_exec == nullptr) return HYDRO_EINVAL;
  hipGraph_t g = nullptr;
  hipError_t e = hipStreamEndCapture(static_cast<hipStream_t>(stream), &g);
  if (e != hipSuccess) return device_status(e);
  hipGraphExec_t x = nullptr;
  e = hipGraphInstantiate(&x, g, nullptr, nullptr, 0);
  (void)hipGraphDestroy(g);
  if (e != hipSuccess) return device_status(e);
  *graph_exec = x;
  return HYDRO_OK;
}

int hydro_graph_launch(void* graph_exec, void* stream) {
  if (graph_exec == nullptr) return HYDRO_EINVAL;
  return device_status(hipGraphLaunch(static_cast<hipGraphExec_t>(graph_exec), static_cast<hipStream_t>(stream)));
}

int hydro_graph_destroy(void* graph_exec) {
  if (graph_exec == nullptr) return HYDRO_EINVAL;
  return device_status(hipGraphExecDestroy(static_cast<hipGraphExec_t>(graph_exec)));
}

int64_t hydro_adjoint_workspace_bytes(int64_t n_groups, int32_t dtype, int32_t level) {
  if (n_groups < 0 || (dtype != HYDRO_F64 && dtype != HYDRO_F32)) return HYDRO_EINVAL;
  return int64_t(gh::adjoint_workspace_elems(n_groups, level != 0) * dtype_size(dtype));
}

int hydro_advance_adjoint(const void* U_pad_dev, const void* gU_out_dev, void* gU_pad_dev, int64_t n_groups,
                          int32_t ghost, int32_t dtype, double dt, double dx, double gamma, int32_t scheme,
                          double theta, void* work_dev, int64_t work_bytes, void* stream) {
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
  const int first_order = (scheme & HYDRO_FIRST_ORDER) ? 1 : 0;
  const int ws = (scheme >> 8) & 3;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (dtype == HYDRO_F64)
    e = gh::launch_mhm_adjoint_padded(static_cast<const double*>(U_pad_dev), static_cast<const double*>(gU_out_dev),
                                      static_cast<double*>(gU_pad_dev), n_groups, ghost,
                                      make_gas<double>(gamma, theta, dt, dx), first_order, ws,
                                      static_cast<double*>(work_dev), g_adjoint_variant[0].load() == 1, s);
  else
    e = gh::launch_mhm_adjoint_padded(static_cast<const float*>(U_pad_dev), static_cast<const float*>(gU_out_dev),
                                      static_cast<float*>(gU_pad_dev), n_groups, ghost,
                                      make_gas<float>(gamma, theta, dt, dx), first_order, ws,
                                      static_cast<float*>(work_dev), g_adjoint_variant[1].load() == 1, s);
  return device_status(e);
}

int hydro_advance_level_adjoint(const void* level_dev, const void* g_level_out_dev, void* g_level_in_dev, int32_t ngx,
                                int32_t ngy, int32_t ngz, const int32_t* bc_host, int32_t dtype, double dt, double dx,
                                double gamma, int32_t scheme, double theta, const double* dt_dev, void* work_dev,
                                int64_t work_bytes, void* stream) {
  if (!adjoint_geom_ok(ngx, ngy, ngz) || bc_host == nullptr || (dtype != HYDRO_F64 && dtype != HYDRO_F32))
    return HYDRO_EINVAL;
  if (!finite_pos(dx) || !(std::isfinite(gamma) && gamma > 1.0) || !valid_scheme(scheme, theta)) return HYDRO_EINVAL;
  if (dt_dev == nullptr && !finite_pos(dt)) return HYDRO_EINVAL;
  gh::LevelGeom geo;
  geo.ngx = ngx;
  geo.ngy = ngy;
  geo.ngz = ngz;
  for (int i = 0; i < 6; ++i) {
    if (bc_host[i] != HYDRO_BC_PERIODIC && bc_host[i] != HYDRO_BC_OUTFLOW) return HYDRO_EINVAL;
    geo.bc[i] = bc_host[i];
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
  const int first_order = (scheme & HYDRO_FIRST_ORDER) ? 1 : 0;
  const int ws = (scheme >> 8) & 3;
  const double dt_host = dt_dev != nullptr ? 1.0 : dt;
  hipStream_t s = static_cast<hipStream_t>(stream);
  hipError_t e;
  if (dtype == HYDRO_F64)
    e = gh::launch_mhm_adjoint_level(static_cast<const double*>(level_dev), static_cast<const double*>(g_level_out_dev),
                                     static_cast<double*>(g_level_in_dev), geo,
                                     make_gas<double>(gamma, theta, dt_host, dx), dt_dev, dx, first_order, ws,
                                     static_cast<double*>(work_dev), g_adjoint_variant[0].load() == 1, s);
  else
    e = gh::launch_mhm_adjoint_level(static_cast<const float*>(level_dev), static_cast<const float*>(g_level_out_dev),
                                     static_cast<float*>(g_level_in_dev), geo,
                                     make_gas<float>(gamma, theta, dt_host, dx), dt_dev, dx, first_order, ws,
                                     static_cast<float*>(work_dev), g_adjoint_variant[1].load() == 1, s);
  return device_status(e);
}

int hydro_autotune_adjoint(const void* level_dev, const void* g_level_out_dev, void* g_level_in_dev, int32_t ngx,
                           int32_t ngy, int32_t ngz, const int32_t* bc_host, int32_t dtype, double dx, double gamma,
                           void* work_dev, int64_t work_bytes, int32_t reps, float* times_ms_host, void* stream) {
  if (reps < 1 || reps > 1000 || (dtype != HYDRO_F64 && dtype != HYDRO_F32)) return HYDRO_EINVAL;
  hipStream_t s = static_cast<hipStream_t>(stream);
  const int saved = g_adjoint_variant[dtype].load();
  const double dt = 1e-3 * dx;  // any positive step does the same work
  auto launch = [&]() {
    return hydro_advance_level_adjoint(level_dev, g_level_out_dev, g_level_in_dev, ngx, ngy, ngz, bc_host, dtype, dt,
                                       dx, gamma, HYDRO_SCHEME_MHM_PLM_HLLC, 1.5, nullptr, work_dev, work_bytes,
                                       stream);
  };
  // argument errors surface here, before any event is created
  int status = launch();
  if (status != HYDRO_OK) return status;
  hipEvent_t e0, e1;
  if (hipEventCreate(&e0) != hipSuccess) return device_status(hipGetLastError());
  if (hipEventCreate(&e1) != hipSuccess) {
    (void)hipEventDestroy(e0);
    return device_status(hipGetLastError());
  }
  float ms_min[2] = {0.0f, 0.0f};
  // two passes over both forms, each form's time the smaller of its two
  for (int pass = 0; pass < 2 && status == HYDRO_OK; ++pass) {
    for (int form = 0; form < 2 && status == HYDRO_OK; ++form) {
      g_adjoint_variant[dtype].store(form);
      status = launch();
      if (status != HYDRO_OK) break;
      hipError_t he = hipEventRecord(e0, s);
      for (int r = 0; r < reps && status == HYDRO_OK && he == hipSuccess; ++r) status = launch();
      if (status != HYDRO_OK) break;
      if (he == hipSuccess) he = hipEventRecord(e1, s);
      if (he == hipSuccess) he = hipEventSynchronize(e1);
      float ms = 0.0f;
      if (he == hipSuccess) he = hipEventElapsedTime(&ms, e0, e1);
      if (he != hipSuccess) {
        status = device_status(he);
        break;
      }
      ms /= float(reps);
      if (pass == 0 || ms < ms_min[form]) ms_min[form] = ms;
    }
  }
  (void)hipEventDestroy(e0);
  (void)hipEventDestroy(e1);
  if (status != HYDRO_OK) {
    g_adjoint_variant[dtype].store(saved);
    return status;
  }
  if (times_ms_host != nullptr) {
    times_ms_host[0] = ms_min[0];
    times_ms_host[1] = ms_min[1];
  }
  const int best = ms_min[1] < ms_min[0] ? 1 : 0;
  g_adjoint_variant[dtype].store(best);
  return best;
}

int hydro_set_adjoint_variant(int32_t dtype, int32_t variant) {
  if (dtype != HYDRO_F64 && dtype != HYDRO_F32) return HYDRO_EINVAL;
  if (variant != 0 && variant != 1) return HYDRO_EINVAL;
  g_adjoint_variant[dtype].store(variant);
  return HYDRO_OK;
}

int hydro_get_adjoint_variant(int32_t dtype) {
  if (dtype != HYDRO_F64 && dtype != HYDRO_F32) return HYDRO_EINVAL;
  return g_adjoint_variant[dtype].load();
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
