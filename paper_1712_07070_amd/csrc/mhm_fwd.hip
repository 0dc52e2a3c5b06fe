// Fused MHM step of one 16^3 patch group per workgroup (GAMER-2, Sec. 2.2).
//
// Mapping on gfx950 (wave64, 160 KB LDS per CU):
//   * 320 threads = 5 waves.  Waves 0-3 own the 256 interior (x, y) columns
//     of the group; wave 4 owns the 64 "halo" columns one cell outside the
//     interior (x = -1, x = 16, y = -1, y = 16), whose face states feed the
//     x/y faces on the group boundary.  Wave 4 also loads the 64 columns two
//     cells out and the 4 edge columns, which are only read as neighbours.
//   * The workgroup marches in z over the state planes k = -1 .. 16.  Each
//     thread keeps the primitive states of its own column at planes k-1, k,
//     k+1 in registers (the z stencil); plane k of all columns goes through
//     LDS for the x/y stencil.
//   * Per plane: every state cell computes its six half-step face states
//     (a2-a4) in registers; the x+ and y+ states go to LDS, the z+ state stays
//     in a register for the z-face of the next plane.  Then each interior
//     thread solves the HLLC problems of its low x and low y faces (the halo
//     threads at x = 16 / y = 16 solve the last face) and its z-face k-1/2.
//   * x/y fluxes go through LDS once; the z flux stays in registers, so the
//     update of plane k-1 is completed in the iteration of plane k, summing
//     the flux differences in the order x, y, z.
// Two workgroup barriers per plane.  Every LDS buffer is single: plane k's
// primitives and states are read before the barrier after which plane k+1's
// are written, and the fluxes of plane k are read before those of k+1 are.
//
// HBM traffic per group: the padded input planes -2..17 (read once, the
// z stencil re-uses registers) and the 16^3 x 5 output.

#include "hydro_device.h"
#include "kernels.h"

namespace gh {

namespace {

constexpr int kThreads = 320;
constexpr int kPW = 20;  // primitive plane tile: x, y in [-2, 17]
constexpr int kSW = 18;  // state tile: x, y in [-1, 16]

__device__ __forceinline__ int pidx(int x, int y) { return (y + 2) * kPW + (x + 2); }
__device__ __forceinline__ int sidx(int x, int y) { return (y + 1) * kSW + (x + 1); }
__device__ __forceinline__ int fxidx(int i, int j) { return j * 17 + i; }  // x-face i: between i-1 and i
__device__ __forceinline__ int fyidx(int i, int j) { return j * 16 + i; }  // y-face j: between j-1 and j

template <typename T>
__device__ __forceinline__ void load_prim(const T* __restrict__ Ug, int64_t P3, int P, int gh, int x, int y,
                                          int z, const Gas<T>& g, T W[5]) {
  const int64_t o = (int64_t(z + gh) * P + (y + gh)) * P + (x + gh);
  T U[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) U[q] = Ug[q * P3 + o];
  cons_to_prim(U, g, W);
}

template <typename T>
__global__ __launch_bounds__(kThreads) void mhm_fwd_kernel(const T* __restrict__ Upad, T* __restrict__ Uout,
                                                           int gh, Gas<T> gas, const double* __restrict__ dt_dev,
                                                           double dx, int first_order, int ws,
                                                           int* __restrict__ n_bad) {
  __shared__ T sP[5][kPW * kPW];     // primitive plane k
  __shared__ T sS[2][5][kSW * kSW];  // x+ and y+ half-step states of plane k
  __shared__ T sF[2][5][17 * 16];    // x and y fluxes of plane k

  if (dt_dev != nullptr) {
    const double dt = *dt_dev;
    gas.dtdx = T(dt / dx);
    gas.half_dtdx = T(0.5 * (dt / dx));
  }

  const int tid = threadIdx.x;
  const int P = 16 + 2 * gh;
  const int64_t P3 = int64_t(P) * P * P;
  const T* __restrict__ Ug = Upad + int64_t(blockIdx.x) * 5 * P3;
  T* __restrict__ Og = Uout + int64_t(blockIdx.x) * 5 * 4096;

  // roles
  const bool interior = tid < 256;
  int cx, cy;        // own state column
  int ox = 0, oy = 0;  // wave 4: the column two cells out
  int ex = 0, ey = 0;  // wave 4, lanes 0..3: one of the 4 edge columns
  if (interior) {
    cx = tid & 15;
    cy = tid >> 4;
  } else {
    const int l = tid - 256, side = l >> 4, k = l & 15;
    cx = side == 0 ? -1 : side == 1 ? 16 : k;
    cy = side == 2 ? -1 : side == 3 ? 16 : k;
    ox = side == 0 ? -2 : side == 1 ? 17 : k;
    oy = side == 2 ? -2 : side == 3 ? 17 : k;
    ex = (l & 1) ? 16 : -1;
    ey = (l & 2) ? 16 : -1;
  }
  const bool has_edge = !interior && (tid - 256) < 4;
  const bool xface16 = !interior && cx == 16;  // solves x-face 16 (between 15 and 16)
  const bool yface16 = !interior && cy == 16;  // solves y-face 16

  // register ring of the own column's primitive states
  T Wm[5], Wc[5], Wp[5];
  if (interior) load_prim(Ug, P3, P, gh, cx, cy, -2, gas, Wm);
  load_prim(Ug, P3, P, gh, cx, cy, -1, gas, Wc);

  T Uz[5];    // z+ face state of the previous plane (interior)
  T Fz0[5];   // z flux at the low face of the previous plane (interior)
  T Ux[5], Uy[5];  // own x- and y- face states of the current plane
  int bad = 0;

  for (int k = -1; k <= 16; ++k) {
    // ---- B: next plane of the own column, publish plane k to LDS
    if (interior || k + 1 <= 16) load_prim(Ug, P3, P, gh, cx, cy, k + 1, gas, Wp);
#pragma unroll
    for (int q = 0; q < 5; ++q) sP[q][pidx(cx, cy)] = Wc[q];
    if (!interior && k >= 0 && k <= 15) {
      T Wo[5];
      load_prim(Ug, P3, P, gh, ox, oy, k, gas, Wo);
#pragma unroll
      for (int q = 0; q < 5; ++q) sP[q][pidx(ox, oy)] = Wo[q];
      if (has_edge) {
        load_prim(Ug, P3, P, gh, ex, ey, k, gas, Wo);
#pragma unroll
        for (int q = 0; q < 5; ++q) sP[q][pidx(ex, ey)] = Wo[q];
      }
    }
    __syncthreads();

    // ---- H: x/y flux differences of plane k-1 (fluxes written last iteration)
    T acc[5];
    if (interior && k >= 1) {
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        acc[q] = sF[0][q][fxidx(cx + 1, cy)] - sF[0][q][fxidx(cx, cy)];
        acc[q] = acc[q] + (sF[1][q][fyidx(cx, cy + 1)] - sF[1][q][fyidx(cx, cy)]);
      }
    }

    // ---- D: half-step face states of the own state cell at plane k
    if (interior || (k >= 0 && k <= 15)) {
      T Wn[3][2][5];
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        Wn[0][0][q] = sP[q][pidx(cx - 1, cy)];
        Wn[0][1][q] = sP[q][pidx(cx + 1, cy)];
        Wn[1][0][q] = sP[q][pidx(cx, cy - 1)];
        Wn[1][1][q] = sP[q][pidx(cx, cy + 1)];
        Wn[2][0][q] = Wm[q];
        Wn[2][1][q] = Wp[q];
      }
      T Ut[3][2][5];
      hancock_states(Wc, Wn, gas, first_order != 0, Ut);
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        sS[0][q][sidx(cx, cy)] = Ut[0][1][q];
        sS[1][q][sidx(cx, cy)] = Ut[1][1][q];
        Ux[q] = Ut[0][0][q];
        Uy[q] = Ut[1][0][q];
      }
      if (interior) {
        if (k >= 0) {
          T Fz1[5];
          bad += hllc_flux<2>(Uz, Ut[2][0], gas, ws, Fz1);
          if (k >= 1) {
            // complete plane k-1: U^{n+1} = U^n - dt/dx [(x) + (y) + (z)]
            const int64_t o = (int64_t(k - 1 + gh) * P + (cy + gh)) * P + (cx + gh);
            T Un[5];
#pragma unroll
            for (int q = 0; q < 5; ++q) {
              const T a = acc[q] + (Fz1[q] - Fz0[q]);
              Un[q] = Ug[q * P3 + o] - gas.dtdx * a;
              Og[q * 4096 + ((k - 1) * 16 + cy) * 16 + cx] = Un[q];
            }
            bad += unphysical(Un, gas);
          }
#pragma unroll
          for (int q = 0; q < 5; ++q) Fz0[q] = Fz1[q];
        }
#pragma unroll
        for (int q = 0; q < 5; ++q) Uz[q] = Ut[2][1][q];
      }
    }
    __syncthreads();

    // ---- F: x and y faces of plane k
    if (k >= 0 && k <= 15) {
      if (interior || xface16) {
        T L[5], F[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) L[q] = sS[0][q][sidx(cx - 1, cy)];
        bad += hllc_flux<0>(L, Ux, gas, ws, F);
#pragma unroll
        for (int q = 0; q < 5; ++q) sF[0][q][fxidx(cx, cy)] = F[q];
      }
      if (interior || yface16) {
        T L[5], F[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) L[q] = sS[1][q][sidx(cx, cy - 1)];
        bad += hllc_flux<1>(L, Uy, gas, ws, F);
#pragma unroll
        for (int q = 0; q < 5; ++q) sF[1][q][fyidx(cx, cy)] = F[q];
      }
    }

#pragma unroll
    for (int q = 0; q < 5; ++q) {
      Wm[q] = Wc[q];
      Wc[q] = Wp[q];
    }
  }

  if (n_bad != nullptr && bad != 0) atomicAdd(n_bad, bad);
}

}  // namespace

template <typename T>
hipError_t launch_mhm_fwd(const T* U_pad, T* U_out, int64_t n_groups, int ghost, const Gas<T>& gas,
                          const double* dt_dev, double dx, int first_order, int ws, int* n_bad,
                          hipStream_t stream) {
  if (n_groups == 0) return hipSuccess;
  // one workgroup per group; split very large batches into launches of at
  // most 2^30 workgroups
  const int64_t chunk = int64_t(1) << 30;
  const int P = 16 + 2 * ghost;
  const int64_t P3 = int64_t(P) * P * P;
  for (int64_t g0 = 0; g0 < n_groups; g0 += chunk) {
    const int64_t n = n_groups - g0 < chunk ? n_groups - g0 : chunk;
    hipLaunchKernelGGL(mhm_fwd_kernel<T>, dim3(unsigned(n)), dim3(kThreads), 0, stream, U_pad + g0 * 5 * P3,
                       U_out + g0 * 5 * 4096, ghost, gas, dt_dev, dx, first_order, ws, n_bad);
    const hipError_t e = hipGetLastError();
    if (e != hipSuccess) return e;
  }
  return hipSuccess;
}

template hipError_t launch_mhm_fwd<double>(const double*, double*, int64_t, int, const Gas<double>&,
                                           const double*, double, int, int, int*, hipStream_t);
template hipError_t launch_mhm_fwd<float>(const float*, float*, int64_t, int, const Gas<float>&,
                                          const double*, double, int, int, int*, hipStream_t);

}  // namespace gh
