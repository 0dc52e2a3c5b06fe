// The other MHM + PLM scheme words (limiters, characteristic variables,
// Roe / HLLE, wave speeds, first order) through the march of the default
// scheme (mhm_group.h), one group per workgroup on padded input.  The
// characteristic projection and the solver family (Roe, or HLLC / HLLE) are
// compile-time options of four kernel copies, the rest run time: one copy
// for every option carried the registers of all of them and spilled.

#include "mhm_group.h"

namespace gh {

namespace {

// optional patch-boundary face fluxes (kFlux) as in mhm_padded_kernel
template <typename T, int kWaves, bool kFlux, int kChr, int kRoe>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(kWaves))) void mhm_padded_ext_kernel(
    const T* __restrict__ Upad, T* __restrict__ Uout, int gh, Gas<T> gas, const double* __restrict__ dt_dev, double dx,
    ExtOpts o, int* __restrict__ n_bad, T* __restrict__ face_flux) {
  __shared__ Smem<T> sm;
  set_dt(gas, dt_dev, dx);
  const int P = 16 + 2 * gh;
  const int64_t P3 = int64_t(P) * P * P;
  PaddedSource<T> src{Upad + int64_t(blockIdx.x) * 5 * P3, P, gh};
  T* ff = kFlux ? face_flux + int64_t(blockIdx.x) * 9 * 5 * 256 : nullptr;
  const ExtSchemeT<kChr, kRoe> sch{o};
  const int bad = process_group<T, (kWaves >= 4)>(src, Uout + int64_t(blockIdx.x) * 5 * 4096, gas, o.first_order,
                                                  o.ws, sm, nullptr, 0.0, threadIdx.x, ff, nullptr, sch);
  if (n_bad != nullptr && bad != 0) atomicAdd(n_bad, bad);
}

// Occupancy target: FP32 at the low one (256 VGPRs instead of 128 with 16-41
// spilled: 256^3 steps 18-39% faster, measured), FP64 at the high one (the
// low one measured slower).
template <typename T, bool kFlux, int kChr, int kRoe>
void launch_ext_copy(const T* U_pad, T* U_out, int64_t n, int ghost, const Gas<T>& gas, const double* dt_dev,
                     double dx, const ExtOpts& o, int* n_bad, hipStream_t stream, T* face_flux) {
  constexpr int kW = sizeof(T) == 4 ? MinWaves<T>::lo : MinWaves<T>::hi;
  hipLaunchKernelGGL((mhm_padded_ext_kernel<T, kW, kFlux, kChr, kRoe>), dim3(unsigned(n)),
                     dim3(kThreads), 0, stream, U_pad, U_out, ghost, gas, dt_dev, dx, o, n_bad, face_flux);
}

template <typename T, bool kFlux>
void launch_ext(const T* U_pad, T* U_out, int64_t n, int ghost, const Gas<T>& gas, const double* dt_dev, double dx,
                const ExtOpts& o, int* n_bad, hipStream_t stream, T* face_flux) {
  const bool roe = o.solver == 1;
  if (o.chr) {
    if (roe) launch_ext_copy<T, kFlux, 1, 1>(U_pad, U_out, n, ghost, gas, dt_dev, dx, o, n_bad, stream, face_flux);
    else launch_ext_copy<T, kFlux, 1, 0>(U_pad, U_out, n, ghost, gas, dt_dev, dx, o, n_bad, stream, face_flux);
  } else {
    if (roe) launch_ext_copy<T, kFlux, 0, 1>(U_pad, U_out, n, ghost, gas, dt_dev, dx, o, n_bad, stream, face_flux);
    else launch_ext_copy<T, kFlux, 0, 0>(U_pad, U_out, n, ghost, gas, dt_dev, dx, o, n_bad, stream, face_flux);
  }
}

}  // namespace

template <typename T>
hipError_t launch_mhm_fwd_ext(const T* U_pad, T* U_out, int64_t n_groups, int ghost, const Gas<T>& gas,
                              const double* dt_dev, double dx, const ExtOpts& o, int* n_bad, hipStream_t stream,
                              T* face_flux) {
  if (n_groups == 0) return hipSuccess;
  const int64_t chunk = int64_t(1) << 30;
  const int P = 16 + 2 * ghost;
  const int64_t P3 = int64_t(P) * P * P;
  for (int64_t g0 = 0; g0 < n_groups; g0 += chunk) {
    const int64_t n = n_groups - g0 < chunk ? n_groups - g0 : chunk;
    if (face_flux != nullptr)
      launch_ext<T, true>(U_pad + g0 * 5 * P3, U_out + g0 * 5 * 4096, n, ghost, gas, dt_dev, dx, o, n_bad, stream,
                          face_flux + g0 * 9 * 5 * 256);
    else
      launch_ext<T, false>(U_pad + g0 * 5 * P3, U_out + g0 * 5 * 4096, n, ghost, gas, dt_dev, dx, o, n_bad, stream,
                           (T*)nullptr);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template hipError_t launch_mhm_fwd_ext<double>(const double*, double*, int64_t, int, const Gas<double>&, const double*,
                                               double, const ExtOpts&, int*, hipStream_t, double*);
template hipError_t launch_mhm_fwd_ext<float>(const float*, float*, int64_t, int, const Gas<float>&, const double*,
                                              double, const ExtOpts&, int*, hipStream_t, float*);

}  // namespace gh
