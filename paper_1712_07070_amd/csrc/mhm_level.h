// The level step's kernel (GAMER-2 Sec. 2.2 MHM on every group of a level,
// ghost cells read from the neighbouring groups, Sec. 3.4), shared by the
// translation units that instantiate its launch shapes.
#pragma once

#include "mhm_group.h"

namespace gh {

namespace {

// Groups are assigned to workgroups so that each XCD (workgroups are dealt
// to the 8 XCDs round-robin) sweeps a contiguous range of groups: halo cells
// read from a neighbouring group then mostly hit the same XCD's L2.
__device__ __forceinline__ int64_t xcd_group(int64_t b, int64_t G) {
  const int64_t per = (G + 7) / 8;
  const int64_t g = (b & 7) * per + (b >> 3);
  return g;
}

// Column-tile order of the groups of a level: the lattice is cut into tiles
// of kTileGroups / ngx rows of groups (at least one row; full in x), and the
// groups are visited tile by tile, within a tile layer by layer upward (z),
// within a layer x fastest.  With the XCD blocking each XCD then marches one
// tile upward: the group that replaces a finished one is usually the one
// above it, which reads as its lower ghost planes the planes the finished
// group read last, and reads first the planes that group read as its upper
// ghost planes -- so both still sit in the XCD's L2.  In the linear order
// the groups of a tile layer run together too, but the layer above runs
// several tile layers later, and every group fetches its 4 ghost planes
// (with their halo rows) from HBM.
constexpr int kTileGroups = 64;
__device__ __forceinline__ int64_t tile_slots(const LevelGeom& geo) {
  return int64_t(geo.ngx) * geo.ngy * geo.ngz;
}
__device__ __forceinline__ int64_t tile_group(int64_t s, const LevelGeom& geo) {
  const int ty = geo.ngx >= kTileGroups ? 1 : (kTileGroups / geo.ngx < geo.ngy ? kTileGroups / geo.ngx : geo.ngy);
  const int64_t full_tiles = geo.ngy / ty, tile = int64_t(ty) * geo.ngx * geo.ngz;
  int64_t t, rows, r;
  if (s < full_tiles * tile) {
    t = s / tile;
    rows = ty;
    r = s - t * tile;
  } else {
    t = full_tiles;
    rows = geo.ngy - full_tiles * ty;
    r = s - full_tiles * tile;
  }
  const int64_t layer = rows * geo.ngx;
  const int gz = int(r / layer), rem = int(r % layer);
  const int gx = rem % geo.ngx, gy = int(t * ty) + rem / geo.ngx;
  return (int64_t(gz) * geo.ngy + gy) * geo.ngx + gx;
}

// order: bit 0 XCD-blocked (else plain), bit 1 brick order of the groups.
// kGpw groups per workgroup (256 threads each; 2: a 512-thread workgroup
// whose halves march two groups side by side, each in its own LDS, passing
// the same barriers).  Workgroup w takes the group slots kGpw w + h, mapped
// through the group order; a half whose slot holds no group (an odd slot
// count, a partial brick) recomputes the other half's group and writes the
// same bits to the same places, keeping its barriers, but leaves the
// unphysical count and the CFL outputs to that half.  In the second half
// local wave w acts as wave w ^ 1, so that its halo and last-faces waves
// land on the SIMDs (1, 3) the first half's plain waves use (the waves of a
// workgroup are dealt round-robin over the 4 SIMDs).
template <typename T, bool kCfl, int kWaves, typename Off, int kL, int kGpw>
__global__ __launch_bounds__(kThreads * kGpw) __attribute__((amdgpu_waves_per_eu(kWaves))) void mhm_level_kernel(
    const T* __restrict__ level, T* __restrict__ level_out, LevelGeom geo, Gas<T> gas,
    const double* __restrict__ dt_dev, double dx, int first_order, int ws, int* __restrict__ n_bad, CflOut cfl,
    int order) {
  __shared__ Smem<T, kL> sm[kGpw];
  set_dt(gas, dt_dev, dx);
  if (kCfl && cfl.reset != nullptr && blockIdx.x == 0 && threadIdx.x == 0) *cfl.reset = 0x7ff0000000000000ull;
  const int half = kGpw == 2 ? __builtin_amdgcn_readfirstlane(int(threadIdx.x) >> 8) : 0;
  const int tid = kGpw == 2 ? (int(threadIdx.x) & 255) ^ (half << 6) : int(threadIdx.x);
  const int64_t G = int64_t(geo.ngx) * geo.ngy * geo.ngz;
  const int64_t slots = (order & 2) ? tile_slots(geo) : G;
  const int64_t wslots = (slots + kGpw - 1) / kGpw;
  const int64_t w = (order & 1) ? xcd_group(blockIdx.x, wslots) : int64_t(blockIdx.x);
  if (w >= wslots) return;  // the whole workgroup leaves together (w is uniform)
  int64_t gs[kGpw];
#pragma unroll
  for (int h = 0; h < kGpw; ++h) {
    const int64_t sl = w * kGpw + h;
    gs[h] = sl >= slots ? -1 : ((order & 2) ? tile_group(sl, geo) : sl);
  }
  bool any = false;
#pragma unroll
  for (int h = 0; h < kGpw; ++h) any = any || gs[h] >= 0;
  if (!any) return;  // uniform
  int64_t g = gs[half];
  const bool dup = g < 0;
  if (dup) g = gs[kGpw - 1 - half];
  LevelSource<T, Off> src{level, geo, int(g % geo.ngx), int((g / geo.ngx) % geo.ngy),
                          int(g / (int64_t(geo.ngx) * geo.ngy))};
  __shared__ double cfl_slots[kGpw][kCfl ? 2 * kCflHalfStride : 1];
  double* smax = nullptr;
  if (kCfl) {
    smax = cfl_slots[half] + cfl_slot(tid);
    smax[0] = 0.0;
    smax[kCflHalfStride] = 0.0;
  }
  const int bad = process_group<T, (kWaves >= 4)>(src, level_out + g * 5 * 4096, gas, first_order, ws, sm[half],
                                                  smax, cfl.gamma, tid);
  if (n_bad != nullptr && bad != 0 && !dup) atomicAdd(n_bad, bad);
  if (kCfl)
    cfl_epilogue(cfl_slots[half], cfl.c_cfl_dx, (cfl.dt_patch != nullptr && !dup) ? cfl.dt_patch + g * 8 : nullptr,
                 dup ? nullptr : cfl.dt_min, 1.0, tid);
}

template <typename T, bool kCfl, typename Off, int kL, int kGpw>
void launch_level_lds(const T* level, T* level_out, const LevelGeom& geo, const Gas<T>& gas, const double* dt_dev,
                      double dx, int first_order, int ws, int* n_bad, const CflOut& cfl, int variant, int64_t blocks,
                      int order, hipStream_t stream) {
  if (variant & 2)
    hipLaunchKernelGGL((mhm_level_kernel<T, kCfl, MinWaves<T>::lo, Off, kL, kGpw>), dim3(unsigned(blocks)),
                       dim3(kThreads * kGpw), 0, stream, level, level_out, geo, gas, dt_dev, dx, first_order, ws, n_bad,
                       cfl, order);
  else
    hipLaunchKernelGGL((mhm_level_kernel<T, kCfl, MinWaves<T>::hi, Off, kL, kGpw>), dim3(unsigned(blocks)),
                       dim3(kThreads * kGpw), 0, stream, level, level_out, geo, gas, dt_dev, dx, first_order, ws, n_bad,
                       cfl, order);
}

}  // namespace

// Shapes with two groups per workgroup (instantiated in mhm_fwd_g2.hip).
template <typename T, bool kCfl, typename Off>
void launch_level_shape_g2(const T* level, T* level_out, const LevelGeom& geo, const Gas<T>& gas,
                           const double* dt_dev, double dx, int first_order, int ws, int* n_bad, const CflOut& cfl,
                           int variant, int64_t blocks, int order, hipStream_t stream);

}  // namespace gh
