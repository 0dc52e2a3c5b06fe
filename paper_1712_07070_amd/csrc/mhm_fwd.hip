// MHM step of 16^3 patch groups, one group per workgroup (GAMER-2, Sec. 2.2).
//
// Mapping on gfx950 (wave64, 160 KB LDS per CU):
//   * 256 threads = 4 waves, one per SIMD; every thread owns one interior
//     (x, y) column.  Wave 0 also owns the 64 "halo" columns one cell outside
//     the interior (x = -1, x = 16, y = -1, y = 16), whose face states feed
//     the x/y faces on the group boundary, and loads the 64 columns two cells
//     out and the 4 edge columns, which are only read as neighbours.  Wave 2
//     solves the 32 faces on the high x / y boundary from states the halo
//     columns leave in LDS.  Two workgroups share a CU in FP64, up to four
//     in FP32.
//   * The workgroup marches in z over the state planes k = -1 .. 16.  Each
//     thread keeps the primitive states of its own column at planes k-1, k,
//     k+1 in registers (the z stencil) and the conserved values of the next
//     plane in flight; plane k of all columns goes through LDS for the x/y
//     stencil.
//   * Per plane: every state cell computes its six half-step face states
//     (a2-a4) in registers; the x+ and y+ states go to LDS, the z+ state stays
//     in a register for the z-face of the next plane.  Then each interior
//     thread solves the HLLC problems of its low x and low y faces (wave 2
//     also the last faces) and its z-face k-1/2.
//   * x/y fluxes go through LDS once; the z flux stays in registers, so the
//     update of plane k-1 is completed in the iteration of plane k, summing
//     the flux differences in the order x, y, z.
// Two workgroup barriers per plane.  Every LDS buffer is single: plane k's
// primitives and states are read before the barrier after which plane k+1's
// are written, and the fluxes of plane k are read before those of k+1 are.
//
// Two sources of the input cells share this code:
//   * padded groups [G][5][P^3] whose ghost zones were filled beforehand
//     (hydro_advance), and
//   * the level storage itself [G][5][16^3] (hydro_advance_level): every cell
//     the stencil reaches outside the group is read from the neighbouring
//     group, with the periodic / outflow index map of the ghost fill.  This
//     is the ghost fill (a0) fused into the load stage: no padded copy is
//     written or read back.  Optionally the same kernel reduces the CFL
//     time-step (a8) of the cells it writes, for the next step.

#include "mhm_level.h"

namespace gh {

namespace {

// ------------------------------------------------------------- kernels ----

// kFlux: also write the fluxes of the patch-boundary faces of every group to
// face_flux [G][9][5][256] (process_group's layout).  kRec: also write every
// group's branch record to record[G] (a diagnostic).
template <typename T, int kWaves, bool kFlux, bool kRec = false>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(kWaves))) void mhm_padded_kernel(const T* __restrict__ Upad, T* __restrict__ Uout,
                                                              int gh, Gas<T> gas, const double* __restrict__ dt_dev,
                                                              double dx, int first_order, int ws,
                                                              int* __restrict__ n_bad, T* __restrict__ face_flux,
                                                              unsigned* __restrict__ record = nullptr) {
  __shared__ Smem<T> sm;
  set_dt(gas, dt_dev, dx);
  const int P = 16 + 2 * gh;
  const int64_t P3 = int64_t(P) * P * P;
  PaddedSource<T> src{Upad + int64_t(blockIdx.x) * 5 * P3, P, gh};
  T* ff = kFlux ? face_flux + int64_t(blockIdx.x) * 9 * 5 * 256 : nullptr;
  unsigned* rec = kRec ? record + blockIdx.x : nullptr;
  const int bad = process_group<T, (kWaves >= 4)>(src, Uout + int64_t(blockIdx.x) * 5 * 4096, gas, first_order, ws, sm, nullptr,
                                   0.0, threadIdx.x, ff, rec);
  if (n_bad != nullptr && bad != 0) atomicAdd(n_bad, bad);
}


template <typename T, bool kCfl, typename Off>
void launch_level_shape(const T* level, T* level_out, const LevelGeom& geo, const Gas<T>& gas,
                        const double* dt_dev, double dx, int first_order, int ws, int* n_bad, const CflOut& cfl,
                        int variant, int64_t blocks, int order, hipStream_t stream) {
  if (variant & 16)
    launch_level_shape_g2<T, kCfl, Off>(level, level_out, geo, gas, dt_dev, dx, first_order, ws, n_bad, cfl, variant,
                                        blocks, order, stream);
  else if (variant & 8)
    launch_level_lds<T, kCfl, Off, 1, 1>(level, level_out, geo, gas, dt_dev, dx, first_order, ws, n_bad, cfl,
                                         variant, blocks, order, stream);
  else
    launch_level_lds<T, kCfl, Off, 0, 1>(level, level_out, geo, gas, dt_dev, dx, first_order, ws, n_bad, cfl,
                                         variant, blocks, order, stream);
}

// Launch shapes (bit-identical results): bit 0 plain group order (else
// XCD-blocked), bit 1 low occupancy target, bit 2 column-tile order of the
// groups (else linear),
// bit 3 padded LDS rows, bit 4 two groups per 512-thread workgroup.
template <typename T, bool kCfl>
hipError_t launch_level_variant(const T* level, T* level_out, const LevelGeom& geo, const Gas<T>& gas,
                                const double* dt_dev, double dx, int first_order, int ws, int* n_bad,
                                const CflOut& cfl, int variant, hipStream_t stream) {
  const int64_t G = int64_t(geo.ngx) * geo.ngy * geo.ngz;
  const int xcd = (variant & 1) ? 0 : 1;
  const int tiled = (variant & 4) ? 1 : 0;
  const int gpw = (variant & 16) ? 2 : 1;
  const int64_t wslots = (G + gpw - 1) / gpw;
  const int64_t blocks = xcd ? ((wslots + 7) / 8) * 8 : wslots;
  const int order = xcd | (tiled << 1);
  if (blocks > (int64_t(1) << 31) - 1) return hipErrorInvalidValue;
  // 32-bit element offsets when every element of the level has one
  if (G * 5 * 4096 <= int64_t(0xffffffffu))
    launch_level_shape<T, kCfl, unsigned int>(level, level_out, geo, gas, dt_dev, dx, first_order, ws, n_bad, cfl,
                                              variant, blocks, order, stream);
  else
    launch_level_shape<T, kCfl, int64_t>(level, level_out, geo, gas, dt_dev, dx, first_order, ws, n_bad, cfl,
                                         variant, blocks, order, stream);
  return hipGetLastError();
}

}  // namespace

template <typename T>
hipError_t launch_mhm_fwd(const T* U_pad, T* U_out, int64_t n_groups, int ghost, const Gas<T>& gas,
                          const double* dt_dev, double dx, int first_order, int ws, int* n_bad,
                          hipStream_t stream, T* face_flux) {
  if (n_groups == 0) return hipSuccess;
  // one workgroup per group; very large batches go in launches of at most
  // 2^30 workgroups
  const int64_t chunk = int64_t(1) << 30;
  const int P = 16 + 2 * ghost;
  const int64_t P3 = int64_t(P) * P * P;
  // occupancy target: FP32 at the low one (two planes per loop iteration
  // without spills: 256^3 step 0.556 -> 0.540 ms, measured), FP64 at the
  // high one (the low one measured equal)
  constexpr int kW = sizeof(T) == 4 ? MinWaves<T>::lo : MinWaves<T>::hi;
  for (int64_t g0 = 0; g0 < n_groups; g0 += chunk) {
    const int64_t n = n_groups - g0 < chunk ? n_groups - g0 : chunk;
    if (face_flux != nullptr)
      hipLaunchKernelGGL((mhm_padded_kernel<T, kW, true>), dim3(unsigned(n)), dim3(kThreads), 0, stream,
                         U_pad + g0 * 5 * P3, U_out + g0 * 5 * 4096, ghost, gas, dt_dev, dx, first_order, ws, n_bad,
                         face_flux + g0 * 9 * 5 * 256);
    else
      hipLaunchKernelGGL((mhm_padded_kernel<T, kW, false>), dim3(unsigned(n)), dim3(kThreads), 0,
                         stream, U_pad + g0 * 5 * P3, U_out + g0 * 5 * 4096, ghost, gas, dt_dev, dx, first_order, ws,
                         n_bad, (T*)nullptr);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template <typename T>
hipError_t launch_mhm_level(const T* level, T* level_out, const LevelGeom& geo, const Gas<T>& gas,
                            const double* dt_dev, double dx, int first_order, int ws, int* n_bad, const CflOut& cfl,
                            int variant, hipStream_t stream) {
  const int64_t G = int64_t(geo.ngx) * geo.ngy * geo.ngz;
  if (G == 0) return hipSuccess;
  if (G > (int64_t(1) << 31) - 8) return hipErrorInvalidValue;
  const bool with_cfl = cfl.dt_min != nullptr || cfl.dt_patch != nullptr || cfl.reset != nullptr;
  if (with_cfl)
    return launch_level_variant<T, true>(level, level_out, geo, gas, dt_dev, dx, first_order, ws, n_bad, cfl, variant,
                                         stream);
  return launch_level_variant<T, false>(level, level_out, geo, gas, dt_dev, dx, first_order, ws, n_bad, cfl, variant,
                                        stream);
}


hipError_t launch_mhm_record(const double* U_pad, double* U_out, int64_t n_groups, int ghost, const Gas<double>& gas,
                             const double* dt_dev, double dx, int first_order, int ws, int* n_bad, unsigned* record,
                             hipStream_t stream) {
  if (n_groups == 0) return hipSuccess;
  if (n_groups > (int64_t(1) << 31) - 1) return hipErrorInvalidValue;
  hipLaunchKernelGGL((mhm_padded_kernel<double, MinWaves<double>::value, false, true>), dim3(unsigned(n_groups)),
                     dim3(kThreads), 0, stream, U_pad, U_out, ghost, gas, dt_dev, dx, first_order, ws, n_bad,
                     (double*)nullptr, record);
  return hipGetLastError();
}

template hipError_t launch_mhm_fwd<double>(const double*, double*, int64_t, int, const Gas<double>&,
                                           const double*, double, int, int, int*, hipStream_t, double*);
template hipError_t launch_mhm_fwd<float>(const float*, float*, int64_t, int, const Gas<float>&,
                                          const double*, double, int, int, int*, hipStream_t, float*);
template hipError_t launch_mhm_level<double>(const double*, double*, const LevelGeom&, const Gas<double>&,
                                             const double*, double, int, int, int*, const CflOut&, int, hipStream_t);
template hipError_t launch_mhm_level<float>(const float*, float*, const LevelGeom&, const Gas<float>&,
                                            const double*, double, int, int, int*, const CflOut&, int, hipStream_t);

}  // namespace gh
