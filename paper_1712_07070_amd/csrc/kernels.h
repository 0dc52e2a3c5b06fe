// Internal launch wrappers of libhydro (not part of the public ABI).
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

#include "hydro_device.h"

namespace gh {

// Group lattice and boundary conditions of one level (bc: x-, x+, y-, y+,
// z-, z+; 0 periodic, 1 outflow).
struct LevelGeom {
  int ngx, ngy, ngz;
  int bc[6];
};

// CFL outputs of a fused step (all optional): per-patch time-steps of the
// written state, an integer-minimum target for the level time-step (the bit
// pattern of a non-negative double), and a location the kernel resets to +inf.
struct CflOut {
  double* dt_patch;
  unsigned long long* dt_min;
  unsigned long long* reset;
  double c_cfl_dx;  // C_CFL * dx, formed on the host in double
  double gamma;
};

template <typename T>
hipError_t launch_mhm_level(const T* level, T* level_out, const LevelGeom& geo, const Gas<T>& gas,
                            const double* dt_dev, double dx, int first_order, int ws, int* n_bad, const CflOut& cfl,
                            int variant, hipStream_t stream);

// One level of a batched launch: input / output level storage, geometry,
// the level's dt/dx (or a device dt), and the index of its first work item.
template <typename T>
struct BatchLevel {
  const T* in;
  T* out;
  LevelGeom geo;
  long long g_begin;  // items [g_begin, next level's g_begin) are this level's groups
  T dtdx, half_dtdx;
  const double* dt_dev;
  double dt_scale;  // with dt_dev: dt = *dt_dev * dt_scale
  double dx;
  // CFL outputs of the level's written state (launches with the epilogue)
  double* dt_patch;              // [G][8] per-patch time-steps, or null
  unsigned long long* dt_min;    // minimum x fold_scale folded in (bits of a double), or null
  unsigned long long* reset;     // set to +inf at the start of the launch, or null
  double c_cfl_dx;               // C_CFL * dx
  double fold_scale;
};

constexpr int kMaxLevels = 8;

template <typename T>
struct BatchArgs {
  BatchLevel<T> lv[kMaxLevels];
  int n_levels;
  long long total;  // number of work items (groups over all levels)
  int cfl;          // some level requests CFL outputs (the launch runs the epilogue form)
  double gamma;     // adiabatic index in double (Eq. 2 signal speeds)
};

// work: kBatchWorkWords device uint32 (kQueues ticket counters and one
// departure counter), zero before the first launch; every launch leaves them
// zero.  grid: number of persistent workgroups.
template <typename T>
hipError_t launch_mhm_batched(const BatchArgs<T>& args, const Gas<T>& gas, int first_order, int ws, int* n_bad,
                              unsigned int* work, int variant, int grid, hipStream_t stream);

// The same launch with the work counters in the library's own per-device
// array (kBatchWorkWords words), cleared before the launch in stream order.
template <typename T>
hipError_t launch_mhm_batched_noalloc(const BatchArgs<T>& args, const Gas<T>& gas, int first_order, int ws,
                                      int* n_bad, int variant, int grid, hipStream_t stream);

// Adjoint of the step (mhm_adj.hip).  Workspace in elements of T:
// adjoint_workspace_elems(G, level).
size_t adjoint_workspace_elems(int64_t n_groups, bool level);

// split: the two-kernel form (face workspace) instead of the fused one.
template <typename T>
hipError_t launch_mhm_adjoint_padded(const T* U_pad, const T* g_out, T* g_pad, int64_t G, int ghost, const Gas<T>& gas,
                                     int first_order, int ws, T* work, bool split, hipStream_t stream);

template <typename T>
hipError_t launch_mhm_adjoint_level(const T* level, const T* g_out, T* g_in, const LevelGeom& geo, const Gas<T>& gas,
                                    const double* dt_dev, double dx, int first_order, int ws, T* work, bool split,
                                    hipStream_t stream);

// Adjoint of the ghost fill: g_level[cell] = sum of g_pad over every padded
// position that copies the cell (mhm_adj.hip).
template <typename T>
hipError_t launch_gather_ghost_adjoint(const T* g_pad, T* g_level, const LevelGeom& geo, int ghost,
                                       hipStream_t stream);

// Launch shapes of the level step (all give bit-identical results):
// bit 0 set = groups in plain order instead of XCD-blocked order,
// bit 1 set = lower occupancy target for the register allocator,
// bit 2 set = groups in column-tile order (tiles of group rows, marched up in z),
// bit 3 set = LDS tiles with padded rows,
// bit 4 set = two groups per 512-thread workgroup.
constexpr int kLevelVariants = 32;
// Batched kernel: ticket queues (one per XCD of MI355X), launch-shape variants
// (bit 0 item order, bit 1 occupancy target, bits 2-3 queue mode: one queue,
// per-XCD queues, static round-robin, per-XCD column-tile queues) and the
// uint32 words of its work buffer (kQueues tickets + 1 departure counter).
constexpr int kQueues = 8;
constexpr int kBatchedVariants = 16;
constexpr int kBatchWorkWords = 16;
static_assert(kQueues + 1 <= kBatchWorkWords, "work buffer too small");

template <typename T>
hipError_t launch_mhm_fwd(const T* U_pad, T* U_out, int64_t n_groups, int ghost, const Gas<T>& gas,
                          const double* dt_dev, double dx, int first_order, int ws, int* n_bad,
                          hipStream_t stream, T* face_flux = nullptr);

// The padded step for the other MHM + PLM words (ExtOpts with ctu, ppm and
// de all 0), in the fused per-group kernel.
struct ExtOpts;
template <typename T>
hipError_t launch_mhm_fwd_ext(const T* U_pad, T* U_out, int64_t n_groups, int ghost, const Gas<T>& gas,
                              const double* dt_dev, double dx, const ExtOpts& o, int* n_bad, hipStream_t stream,
                              T* face_flux);

// The padded step that also writes every group's branch record (FP64).
hipError_t launch_mhm_record(const double* U_pad, double* U_out, int64_t n_groups, int ghost, const Gas<double>& gas,
                             const double* dt_dev, double dx, int first_order, int ws, int* n_bad, unsigned* record,
                             hipStream_t stream);

// The other schemes of the scheme word (scheme_ext.hip): workspace size in
// elements of T for G groups of ghost width `ghost`, and the step.
struct ExtOpts;
int64_t ext_workspace_elems(int64_t n_groups, int ghost, const ExtOpts& o);
// face_flux (optional): [G][9][5][256] fluxes on the patch-boundary faces.
template <typename T>
hipError_t launch_ext_step(const T* U_pad, T* U_out, int64_t G, int ghost, const Gas<T>& gas, const double* dt_dev,
                           double dx, const ExtOpts& o, int* n_bad, T* work, T* face_flux, hipStream_t stream);

// Steps (ii)-(iii) of the procedure for unphysical results on a level
// (fallback.hip); counts[3] device int32, added to: repaired unsplit,
// repaired split, still unphysical.
template <typename T>
hipError_t launch_repair(const T* level_in, T* level_out, const LevelGeom& geo, const Gas<T>& gas,
                         const double* dt_dev, double dx, const ExtOpts& o, int* counts, hipStream_t stream);
hipError_t launch_zero_ints(int* p, int n, hipStream_t stream);

// Coarse-fine coupling (amr.hip).  A level: group positions [G][3] and the
// dense map of its group lattice (n[2] x n[1] x n[0] entries, -1 if absent).
struct AmrLevelArgs {
  const int* pos;
  const int* map;
  int64_t G;
  int n[3];
};
template <typename T>
hipError_t launch_amr_fill(const T* Uf, const AmrLevelArgs& F, const T* Cold, const T* Cnew, const AmrLevelArgs& C,
                           double a, const int bc[6], int ghost, T* pad, hipStream_t stream);
template <typename T>
hipError_t launch_amr_accumulate(const AmrLevelArgs& F, const T* face_flux, double w, const int bc[6], T* R,
                                 hipStream_t stream);
template <typename T>
hipError_t launch_amr_restrict(const T* Uf, const AmrLevelArgs& F, T* Uc, const AmrLevelArgs& C, hipStream_t stream);
template <typename T>
hipError_t launch_amr_fixup(T* Uc, const AmrLevelArgs& C, const AmrLevelArgs& F, const T* cflux, const T* R,
                            double dtdx, const int bc[6], hipStream_t stream);

template <typename T>
hipError_t launch_fill_ghosts(const T* level, T* U_pad, int ngx, int ngy, int ngz, int ghost, const int bc[6],
                              hipStream_t stream);

template <typename T>
hipError_t launch_cfl_dt(const T* U_pad, int64_t n_groups, int ghost, double dx, double gamma, double c_cfl,
                         double* dt_patch, double* dt_min, hipStream_t stream);

}  // namespace gh
