// Batched multi-level MHM step: one persistent launch over the patch groups
// of several AMR levels (GAMER-2 Sec. 2.1: levels advance with their own
// time-steps, dt_l = dt_0 / 2^l in the W-cycle; the paper updates one level
// at a time, Sec. 3.3).  A work item is (level, group); workgroups take items
// from a global counter until the union of all levels is exhausted, so a
// level with few groups does not leave the GPU idle and no launch ends in a
// partial wave of workgroups.  Each item runs the same per-group code as the
// level step, so results are bit-identical to one launch per level, in any
// order of items.

#include <mutex>

#include "mhm_group.h"
#include "mhm_level.h"

namespace gh {

// Work counters of the allocation-free entry point (hydro_advance_batched_noalloc):
// one copy per device, alive until the process ends.  In host code `scratch`
// only names the symbol; its device address comes from hipGetSymbolAddress.
static __device__ __align__(256) unsigned int scratch[kBatchWorkWords];

namespace {

// A value that is the same in every lane, moved to scalar registers.
__device__ __forceinline__ float uniform(float v) {
  return __int_as_float(__builtin_amdgcn_readfirstlane(__float_as_int(v)));
}
__device__ __forceinline__ double uniform(double v) {
  const long long b = __double_as_longlong(v);
  const long long r = (long long)(unsigned int)__builtin_amdgcn_readfirstlane((int)(b & 0xffffffff)) |
                      ((long long)__builtin_amdgcn_readfirstlane((int)(b >> 32)) << 32);
  return __longlong_as_double(r);
}

// Work counters: kQueues ticket counters, then the departure counter.
// Queue modes: 0, one queue, items in ticket order; 1, queue c serves the
// items c, c + kQueues, c + 2 kQueues, ... and workgroup b starts at queue
// b % kQueues, moving on to the next queue when its own is empty; 2, no
// queue: workgroup b takes items b, b + grid, b + 2 grid, ... (static); 3,
// tile queues: queue c serves, level by level, the c-th of kQueues
// contiguous blocks of each level's groups in column-tile order, workgroups
// starting and moving on as in mode 1.  Workgroups of a launch are dealt
// round-robin to the 8 XCDs, so modes 1 and 2 give every XCD the same
// residue class of items that a one-launch-per-level grid in plain order
// gives it, and mode 3 the range of groups the XCD-blocked column-tile level
// step gives it (half the HBM bytes of mode 0 on one 4096-group level,
// measured).  Every mode hands every item out exactly once.
//
// The ticket for the next item is taken when an item starts and decoded when
// it ends, so the atomic's return overlaps the whole group step.
//
// kCfl: levels with CFL outputs get the Eq. 2 time-steps of the state they
// write, reduced in the same pass as in the level kernel (per-patch values,
// and the level minimum times the level's fold_scale folded into a device
// word, so that the levels of a W-cycle can fold min_l 2^l dt_l, the next
// coarse step, into one word).
template <typename T, int kWaves, typename Off, bool kCfl>
__global__ __launch_bounds__(kThreads) __attribute__((amdgpu_waves_per_eu(kWaves))) void mhm_batched_kernel(
    BatchArgs<T> args, Gas<T> gas, int first_order, int ws, int* __restrict__ n_bad,
    unsigned int* __restrict__ work, int order, int queues) {
  __shared__ Smem<T> sm;
  __shared__ double cfl_slots[kCfl ? 2 * kCflHalfStride : 1];
  if (kCfl && blockIdx.x == 0 && threadIdx.x < unsigned(args.n_levels) && args.lv[threadIdx.x].reset != nullptr)
    *args.lv[threadIdx.x].reset = 0x7ff0000000000000ull;
  __shared__ long long item_slot;
  __shared__ int tried;  // queues found empty / static items taken (ticket thread only)
  const int home = int(blockIdx.x % unsigned(kQueues));
  auto queue_size = [&](int c) -> long long {
    return c < args.total ? (args.total - c + kQueues - 1) / kQueues : 0;
  };
  // the queue the next ticket comes from (mode 0: the only one)
  auto cur_queue = [&]() { return (queues == 1 || queues == 3) ? (home + tried) % kQueues : 0; };
  // mode 3: entry t of tile queue c (levels finest first with order 1)
  auto tile_item = [&](int c, long long t) -> long long {
    for (int k = 0; k < args.n_levels; ++k) {
      const int l = order ? args.n_levels - 1 - k : k;
      const LevelGeom& geo = args.lv[l].geo;
      const long long G = (long long)geo.ngx * geo.ngy * geo.ngz;
      const long long per = (G + kQueues - 1) / kQueues, b0 = c * per;
      const long long n = b0 >= G ? 0 : (G - b0 < per ? G - b0 : per);
      if (t < n) return args.lv[l].g_begin + tile_group(b0 + t, geo);
      t -= n;
    }
    return -1;
  };
  // ticket t of the current queue -> item (or -1 if that queue is exhausted)
  auto decode = [&](unsigned int t) -> long long {
    if (queues == 0) return t < args.total ? (long long)t : -1;
    const int c = cur_queue();
    if (queues == 3) return tile_item(c, (long long)t);
    return (long long)t < queue_size(c) ? c + (long long)kQueues * t : -1;
  };
  // take a ticket (thread 0); for mode 2 the "ticket" is the static index
  auto take = [&]() -> unsigned int {
    if (queues == 2) return unsigned(tried++);
    return atomicAdd(&work[cur_queue()], 1u);
  };
  // resolve a taken ticket into the next item, moving on through exhausted queues
  auto resolve = [&](unsigned int t) -> long long {
    long long i;
    if (queues == 2) {
      const long long c = (long long)blockIdx.x + (long long)t * gridDim.x;
      i = c < args.total ? c : -1;
    } else {
      i = decode(t);
      while (i < 0 && (queues == 1 || queues == 3) && ++tried < kQueues) i = decode(atomicAdd(&work[cur_queue()], 1u));
      if (queues == 3) return i;  // the level order is taken in tile_item
    }
    // order 1 deals items from the last (finest, largest) level first
    return i < 0 ? -1 : (order ? args.total - 1 - i : i);
  };
  // dt / dx of every level, once per workgroup (the same expression as the
  // level kernel's, kept out of the item loop's registers)
  __shared__ T lv_dtdx[kMaxLevels], lv_half_dtdx[kMaxLevels];
  if (threadIdx.x < unsigned(args.n_levels)) {
    const BatchLevel<T>& L = args.lv[threadIdx.x];
    T dtdx = L.dtdx, half_dtdx = L.half_dtdx;
    if (L.dt_dev != nullptr) {
      const double dt = *L.dt_dev * L.dt_scale;  // exact for a power-of-two scale
      dtdx = T(dt / L.dx);
      half_dtdx = T(0.5 * (dt / L.dx));
    }
    lv_dtdx[threadIdx.x] = dtdx;
    lv_half_dtdx[threadIdx.x] = half_dtdx;
  }
  // tickets are taken and resolved by the first lane of the last wave: the
  // atomic's return then holds up a wave without halo roles (the halo wave
  // sets the pace of every plane)
  const bool taker = threadIdx.x == kThreads - 64;
  if (taker) {
    tried = 0;
    item_slot = resolve(take());
  }
  __syncthreads();
  for (;;) {
    // the item is the same for every thread: make it wave-uniform so that the
    // level lookup and everything derived from it live in scalar registers
    const long long it = item_slot;
    const long long item = (long long)__builtin_amdgcn_readfirstlane((int)(it >> 32)) << 32 |
                           (unsigned int)__builtin_amdgcn_readfirstlane((int)(it & 0xffffffff));
    if (item < 0) break;
    unsigned int ticket = 0;
    if (taker) ticket = take();
    int l = 0;
    while (l + 1 < args.n_levels && item >= args.lv[l + 1].g_begin) ++l;
    const BatchLevel<T>& L = args.lv[l];
    const int g = int(item - L.g_begin);  // < 2^31 groups per level
    Gas<T> gl = gas;
    gl.dtdx = uniform(lv_dtdx[l]);
    gl.half_dtdx = uniform(lv_half_dtdx[l]);
    const LevelGeom& geo = L.geo;
    const unsigned int gu = unsigned(g), nx = unsigned(geo.ngx), ny = unsigned(geo.ngy);
    LevelSource<T, Off> src{L.in, geo, int(gu % nx), int((gu / nx) % ny), int(gu / nx / ny)};
    // an opaque thread index per item keeps thread-derived addresses from
    // being hoisted out of the item loop (they would stay live across the
    // whole group step and cost registers / occupancy)
    int tid = threadIdx.x;
    asm volatile("" : "+v"(tid));
    double* smax = nullptr;
    if (kCfl && (L.dt_min != nullptr || L.dt_patch != nullptr)) {
      // the previous item's epilogue read the slots before the item barrier
      smax = cfl_slots + cfl_slot(tid);
      smax[0] = 0.0;
      smax[kCflHalfStride] = 0.0;
    }
    const int bad = process_group<T, (kWaves >= 4)>(src, L.out + int64_t(g) * 5 * 4096, gl, first_order, ws, sm, smax,
                                                    args.gamma, tid);
    if (n_bad != nullptr && bad != 0) atomicAdd(n_bad, bad);
    if (kCfl && smax != nullptr)
      cfl_epilogue(cfl_slots, L.c_cfl_dx, L.dt_patch != nullptr ? L.dt_patch + int64_t(g) * 8 : nullptr, L.dt_min,
                   L.fold_scale, tid);
    // every thread has read item_slot (first barrier of the group step)
    if (taker) item_slot = resolve(ticket);
    __syncthreads();
  }
  // the last workgroup to leave re-arms the queues for the next launch
  if (threadIdx.x == 0) {
    const unsigned int done = atomicAdd(&work[kQueues], 1u);
    if (done == gridDim.x - 1) {
      for (int c = 0; c <= kQueues; ++c) atomicExch(&work[c], 0u);
    }
  }
}

template <typename T, typename Off, bool kCfl>
void launch_batched_cfl(const BatchArgs<T>& args, const Gas<T>& gas, int first_order, int ws, int* n_bad,
                        unsigned int* work, int variant, int grid, hipStream_t stream) {
  const int order = variant & 1, queues = (variant >> 2) & 3;
  if (variant & 2)
    hipLaunchKernelGGL((mhm_batched_kernel<T, MinWaves<T>::lo, Off, kCfl>), dim3(unsigned(grid)), dim3(kThreads), 0,
                       stream, args, gas, first_order, ws, n_bad, work, order, queues);
  else
    hipLaunchKernelGGL((mhm_batched_kernel<T, MinWaves<T>::hi, Off, kCfl>), dim3(unsigned(grid)), dim3(kThreads), 0,
                       stream, args, gas, first_order, ws, n_bad, work, order, queues);
}

}  // namespace

template <typename T>
hipError_t launch_mhm_batched(const BatchArgs<T>& args, const Gas<T>& gas, int first_order, int ws, int* n_bad,
                              unsigned int* work, int variant, int grid, hipStream_t stream) {
  if (args.total == 0) return hipSuccess;
  // 32-bit element offsets when every level's elements have one
  bool small = true;
  for (int l = 0; l < args.n_levels; ++l) {
    const LevelGeom& g = args.lv[l].geo;
    small = small && int64_t(g.ngx) * g.ngy * g.ngz * 5 * 4096 <= int64_t(0xffffffffu);
  }
  if (small) {
    if (args.cfl)
      launch_batched_cfl<T, unsigned int, true>(args, gas, first_order, ws, n_bad, work, variant, grid, stream);
    else
      launch_batched_cfl<T, unsigned int, false>(args, gas, first_order, ws, n_bad, work, variant, grid, stream);
  } else {
    if (args.cfl)
      launch_batched_cfl<T, int64_t, true>(args, gas, first_order, ws, n_bad, work, variant, grid, stream);
    else
      launch_batched_cfl<T, int64_t, false>(args, gas, first_order, ws, n_bad, work, variant, grid, stream);
  }
  return hipGetLastError();
}

namespace {

__global__ void clear_words_kernel(unsigned int* __restrict__ p, int n) {
  if (int(threadIdx.x) < n) p[threadIdx.x] = 0u;
}

constexpr int kMaxDevices = 64;
std::mutex g_scratch_mu;
unsigned int* g_scratch_addr[kMaxDevices] = {};

// Device address of `scratch` on the current device, looked up once per
// device (with that device current) and kept.
hipError_t scratch_address(unsigned int** out) {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lk(g_scratch_mu);
  if (g_scratch_addr[dev] == nullptr) {
    void* p = nullptr;
    e = hipGetSymbolAddress(&p, HIP_SYMBOL(scratch));
    if (e != hipSuccess) return e;
    g_scratch_addr[dev] = static_cast<unsigned int*>(p);
  }
  *out = g_scratch_addr[dev];
  return hipSuccess;
}

}  // namespace

template <typename T>
hipError_t launch_mhm_batched_noalloc(const BatchArgs<T>& args, const Gas<T>& gas, int first_order, int ws,
                                      int* n_bad, int variant, int grid, hipStream_t stream) {
  if (args.total == 0) return hipSuccess;
  unsigned int* work = nullptr;
  hipError_t e = scratch_address(&work);
  if (e != hipSuccess) return e;
  // the counters must start at zero: clear them in stream order (a kernel,
  // not a memset, so that the call can be captured into a graph)
  hipLaunchKernelGGL(clear_words_kernel, dim3(1), dim3(64), 0, stream, work, kBatchWorkWords);
  e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_mhm_batched<T>(args, gas, first_order, ws, n_bad, work, variant, grid, stream);
}

template hipError_t launch_mhm_batched_noalloc<double>(const BatchArgs<double>&, const Gas<double>&, int, int, int*,
                                                       int, int, hipStream_t);
template hipError_t launch_mhm_batched_noalloc<float>(const BatchArgs<float>&, const Gas<float>&, int, int, int*, int,
                                                      int, hipStream_t);

template hipError_t launch_mhm_batched<double>(const BatchArgs<double>&, const Gas<double>&, int, int, int*,
                                               unsigned int*, int, int, hipStream_t);
template hipError_t launch_mhm_batched<float>(const BatchArgs<float>&, const Gas<float>&, int, int, int*,
                                              unsigned int*, int, int, hipStream_t);

}  // namespace gh
