// Procedure for unphysical results (GAMER-2, Sec. 2.2), steps (ii)-(iii):
// after a step of a level, every cell whose new state has rho <= 0 or p <= 0
// is recomputed from the step's input, first with a first-order,
// dimensionally unsplit update (Riemann fluxes of the cell averages on its
// six faces), and if that is still unphysical with a first-order,
// dimensionally split update (x, then y, then z sweeps over the 3x3x3 block
// around the cell).  Only failed cells are touched; the level retries of
// steps (iv)-(v) are driven by the host (capi.hip).
//
// One thread per level cell.  The scan reads the five fields of each output
// cell once (40 B per cell in FP64); a failed cell reads its 7 (unsplit) or
// 27 (split) neighbours from the input level through the ghost-fill index
// map (periodic / outflow).  Counters (device int32, added to): [0] cells
// repaired unsplit, [1] repaired split, [2] still unphysical.

#include <algorithm>

#include "ext_device.h"
#include "kernels.h"

namespace gh {

namespace {

struct LevelCells {
  int nx, ny, nz;  // cells per axis
  int bc[6];
  int ngx, ngy;
  __device__ __forceinline__ static int map(int i, int n, int lo, int hi) {
    if (i < 0) return lo == 0 ? i + n : 0;
    if (i >= n) return hi == 0 ? i - n : n - 1;
    return i;
  }
  __device__ __forceinline__ int64_t offset(int X, int Y, int Z) const {
    X = map(X, nx, bc[0], bc[1]);
    Y = map(Y, ny, bc[2], bc[3]);
    Z = map(Z, nz, bc[4], bc[5]);
    const int64_t g = (int64_t(Z >> 4) * ngy + (Y >> 4)) * ngx + (X >> 4);
    return g * 5 * 4096 + ((Z & 15) * 16 + (Y & 15)) * 16 + (X & 15);
  }
};

template <typename T>
__device__ __forceinline__ void load5(const T* __restrict__ L, int64_t o, T U[5]) {
#pragma unroll
  for (int q = 0; q < 5; ++q) U[q] = L[o + q * 4096];
}

template <int D, typename T>
__device__ __forceinline__ void sweep(const T Um[5], const T U0[5], const T Up[5], const Gas<T>& g, const ExtOpts& o,
                                      T out[5]) {
  T Fm[5], Fp[5];
  riemann_any<D>(Um, U0, g, o, Fm);
  riemann_any<D>(U0, Up, g, o, Fp);
#pragma unroll
  for (int q = 0; q < 5; ++q) out[q] = U0[q] - g.dtdx * (Fp[q] - Fm[q]);
}

template <typename T>
__global__ __launch_bounds__(256) void repair_kernel(const T* __restrict__ in, T* __restrict__ out, LevelCells lc,
                                                     Gas<T> gas, const double* __restrict__ dt_dev, double dx,
                                                     ExtOpts o, int* __restrict__ counts) {
  if (dt_dev != nullptr) {
    const double dt = *dt_dev;
    gas.dtdx = T(dt / dx);
  }
  const int64_t n_cells = int64_t(lc.nx) * lc.ny * lc.nz;
  int nu = 0, ns = 0, nl = 0;
  for (int64_t c = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; c < n_cells; c += int64_t(gridDim.x) * blockDim.x) {
    // c enumerates the level storage: group-major, x fastest within a group
    const int64_t g = c >> 12;
    const int w = int(c & 4095);
    T U[5];
    load5(out, g * 5 * 4096 + w, U);
    if (!unphysical(U, gas)) continue;
    const int gx = int(g % lc.ngx), gy = int((g / lc.ngx) % lc.ngy), gz = int(g / (int64_t(lc.ngx) * lc.ngy));
    const int X = gx * 16 + (w & 15), Y = gy * 16 + ((w >> 4) & 15), Z = gz * 16 + (w >> 8);
    T R[5];
    {
      // first order, unsplit: U0 - dt/dx sum_d (F(U0, U+) - F(U-, U0)), summed x, y, z
      T U0[5], Um[5], Up[5], Fm[5], Fp[5], acc[5];
      load5(in, lc.offset(X, Y, Z), U0);
      load5(in, lc.offset(X - 1, Y, Z), Um);
      load5(in, lc.offset(X + 1, Y, Z), Up);
      riemann_any<0>(Um, U0, gas, o, Fm);
      riemann_any<0>(U0, Up, gas, o, Fp);
#pragma unroll
      for (int q = 0; q < 5; ++q) acc[q] = Fp[q] - Fm[q];
      load5(in, lc.offset(X, Y - 1, Z), Um);
      load5(in, lc.offset(X, Y + 1, Z), Up);
      riemann_any<1>(Um, U0, gas, o, Fm);
      riemann_any<1>(U0, Up, gas, o, Fp);
#pragma unroll
      for (int q = 0; q < 5; ++q) acc[q] = acc[q] + (Fp[q] - Fm[q]);
      load5(in, lc.offset(X, Y, Z - 1), Um);
      load5(in, lc.offset(X, Y, Z + 1), Up);
      riemann_any<2>(Um, U0, gas, o, Fm);
      riemann_any<2>(U0, Up, gas, o, Fp);
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        acc[q] = acc[q] + (Fp[q] - Fm[q]);
        R[q] = U0[q] - gas.dtdx * acc[q];
      }
    }
    if (!unphysical(R, gas)) {
      ++nu;
    } else {
      // first order, split: x sweeps of the 9 lines through the block's
      // centre column, y sweeps at the three z planes, z sweep at the cell
      T C[3][3][5];
      for (int k = 0; k < 3; ++k)
        for (int j = 0; j < 3; ++j) {
          T a[5], b[5], d[5];
          load5(in, lc.offset(X - 1, Y + j - 1, Z + k - 1), a);
          load5(in, lc.offset(X, Y + j - 1, Z + k - 1), b);
          load5(in, lc.offset(X + 1, Y + j - 1, Z + k - 1), d);
          sweep<0>(a, b, d, gas, o, C[k][j]);
        }
      T Dz[3][5];
      for (int k = 0; k < 3; ++k) sweep<1>(C[k][0], C[k][1], C[k][2], gas, o, Dz[k]);
      sweep<2>(Dz[0], Dz[1], Dz[2], gas, o, R);
      if (!unphysical(R, gas)) ++ns;
      else ++nl;
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) out[g * 5 * 4096 + q * 4096 + w] = R[q];
  }
  if (nu) atomicAdd(&counts[0], nu);
  if (ns) atomicAdd(&counts[1], ns);
  if (nl) atomicAdd(&counts[2], nl);
}

__global__ void zero_ints_kernel(int* __restrict__ p, int n) {
  if (int(threadIdx.x) < n) p[threadIdx.x] = 0;
}

}  // namespace

template <typename T>
hipError_t launch_repair(const T* level_in, T* level_out, const LevelGeom& geo, const Gas<T>& gas,
                         const double* dt_dev, double dx, const ExtOpts& o, int* counts, hipStream_t stream) {
  LevelCells lc;
  lc.nx = geo.ngx * 16;
  lc.ny = geo.ngy * 16;
  lc.nz = geo.ngz * 16;
  lc.ngx = geo.ngx;
  lc.ngy = geo.ngy;
  for (int i = 0; i < 6; ++i) lc.bc[i] = geo.bc[i];
  const int64_t n = int64_t(lc.nx) * lc.ny * lc.nz;
  const int64_t blocks = std::min<int64_t>((n + 255) / 256, 256 * 64);
  hipLaunchKernelGGL(repair_kernel<T>, dim3(unsigned(blocks)), dim3(256), 0, stream, level_in, level_out, lc, gas,
                     dt_dev, dx, o, counts);
  return hipGetLastError();
}

hipError_t launch_zero_ints(int* p, int n, hipStream_t stream) {
  hipLaunchKernelGGL(zero_ints_kernel, dim3(1), dim3(64), 0, stream, p, n);
  return hipGetLastError();
}

template hipError_t launch_repair<double>(const double*, double*, const LevelGeom&, const Gas<double>&, const double*,
                                          double, const ExtOpts&, int*, hipStream_t);
template hipError_t launch_repair<float>(const float*, float*, const LevelGeom&, const Gas<float>&, const double*,
                                         double, const ExtOpts&, int*, hipStream_t);

}  // namespace gh
