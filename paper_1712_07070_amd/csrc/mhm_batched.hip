// Batched multi-level MHM step: one persistent launch over the patch groups
// of several AMR levels (GAMER-2 Sec. 2.1: levels advance with their own
// time-steps, dt_l = dt_0 / 2^l in the W-cycle; the paper updates one level
// at a time, Sec. 3.3).  A work item is (level, group); workgroups take items
// from a global counter until the union of all levels is exhausted, so a
// level with few groups does not leave the GPU idle and no launch ends in a
// partial wave of workgroups.  Each item runs the same per-group code as the
// level step, so results are bit-identical to one launch per level, in any
// order of items.

#include "mhm_group.h"

namespace gh {

namespace {

template <typename T, int kWaves>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(kWaves))) void mhm_batched_kernel(
    BatchArgs<T> args, Gas<T> gas, int first_order, int ws, int* __restrict__ n_bad,
    unsigned int* __restrict__ work, int order) {
  __shared__ Smem<T> sm;
  __shared__ long long item_slot;
  for (;;) {
    if (threadIdx.x == 0) {
      const unsigned int t = atomicAdd(&work[0], 1u);
      // order 1: items dealt from the last (finest, largest) level first
      item_slot = t < args.total ? (order ? (args.total - 1 - (long long)t) : (long long)t) : -1;
    }
    __syncthreads();
    // the slot is the same for every thread: make it wave-uniform so that the
    // level lookup and everything derived from it live in scalar registers
    const long long item = (long long)__builtin_amdgcn_readfirstlane((int)(item_slot >> 32)) << 32 |
                           (unsigned int)__builtin_amdgcn_readfirstlane((int)(item_slot & 0xffffffff));
    if (item < 0) break;
    int l = 0;
    while (l + 1 < args.n_levels && item >= args.lv[l + 1].g_begin) ++l;
    const BatchLevel<T>& L = args.lv[l];
    const int64_t g = item - L.g_begin;
    Gas<T> gl = gas;
    gl.dtdx = L.dtdx;
    gl.half_dtdx = L.half_dtdx;
    if (L.dt_dev != nullptr) {
      const double dt = *L.dt_dev;
      gl.dtdx = T(dt / L.dx);
      gl.half_dtdx = T(0.5 * (dt / L.dx));
    }
    const LevelGeom& geo = L.geo;
    LevelSource<T> src{L.in, geo, int(g % geo.ngx), int((g / geo.ngx) % geo.ngy), int(g / (int64_t(geo.ngx) * geo.ngy))};
    const int bad = process_group<T>(src, L.out + g * 5 * 4096, gl, first_order, ws, sm, nullptr, 0.0);
    if (n_bad != nullptr && bad != 0) atomicAdd(n_bad, bad);
  }
  // the last workgroup to leave re-arms the queue for the next launch
  if (threadIdx.x == 0) {
    const unsigned int done = atomicAdd(&work[1], 1u);
    if (done == gridDim.x - 1) {
      atomicExch(&work[0], 0u);
      atomicExch(&work[1], 0u);
    }
  }
}

}  // namespace

template <typename T>
hipError_t launch_mhm_batched(const BatchArgs<T>& args, const Gas<T>& gas, int first_order, int ws, int* n_bad,
                              unsigned int* work, int variant, int grid, hipStream_t stream) {
  if (args.total == 0) return hipSuccess;
  const int order = variant & 1;
  if (variant & 2)
    hipLaunchKernelGGL((mhm_batched_kernel<T, MinWaves<T>::lo>), dim3(unsigned(grid)), dim3(kThreads), 0, stream,
                       args, gas, first_order, ws, n_bad, work, order);
  else
    hipLaunchKernelGGL((mhm_batched_kernel<T, MinWaves<T>::hi>), dim3(unsigned(grid)), dim3(kThreads), 0, stream,
                       args, gas, first_order, ws, n_bad, work, order);
  return hipGetLastError();
}

template hipError_t launch_mhm_batched<double>(const BatchArgs<double>&, const Gas<double>&, int, int, int*,
                                               unsigned int*, int, int, hipStream_t);
template hipError_t launch_mhm_batched<float>(const BatchArgs<float>&, const Gas<float>&, int, int, int*,
                                              unsigned int*, int, int, hipStream_t);

}  // namespace gh
