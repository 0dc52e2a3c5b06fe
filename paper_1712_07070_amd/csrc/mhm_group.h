// Per-group device code of the MHM step shared by the level kernels
// (mhm_fwd.hip) and the batched persistent kernel (mhm_batched.hip): input
// sources, the LDS layout, and the z-marching routine that advances one
// 16^3 patch group with one 320-thread workgroup.  See mhm_fwd.hip for the
// mapping of threads to columns.
#pragma once

#include "hydro_device.h"
#include "kernels.h"

namespace gh {

constexpr int kThreads = 320;
constexpr int kPW = 20;  // primitive plane tile: x, y in [-2, 17]
constexpr int kSW = 18;  // state tile: x, y in [-1, 16]

__device__ __forceinline__ int pidx(int x, int y) { return (y + 2) * kPW + (x + 2); }
__device__ __forceinline__ int sidx(int x, int y) { return (y + 1) * kSW + (x + 1); }
__device__ __forceinline__ int fxidx(int i, int j) { return j * 17 + i; }  // x-face i: between i-1 and i
__device__ __forceinline__ int fyidx(int i, int j) { return j * 16 + i; }  // y-face j: between j-1 and j

// ------------------------------------------------------------- sources ----
// A source maps group-relative cell coordinates to element offsets:
// offset(f, x, y, z) = col(x, y) + plane(z) + f * fstride.

template <typename T>
struct PaddedSource {
  const T* base;  // this group's padded block
  int P, gh;
  __device__ int64_t col(int x, int y) const { return int64_t(y + gh) * P + (x + gh); }
  __device__ int64_t plane(int z) const { return int64_t(z + gh) * P * P; }
  __device__ int64_t fstride() const { return int64_t(P) * P * P; }
};

__device__ __forceinline__ int bc_wrap(int i, int n, int lo, int hi) {
  if (i < 0) return lo == 0 ? i + n : 0;
  if (i >= n) return hi == 0 ? i - n : n - 1;
  return i;
}

template <typename T>
struct LevelSource {
  const T* base;  // the level storage [G][5][16^3]
  LevelGeom geo;
  int gx, gy, gz;
  __device__ int64_t col(int x, int y) const {
    const int X = bc_wrap(gx * 16 + x, geo.ngx * 16, geo.bc[0], geo.bc[1]);
    const int Y = bc_wrap(gy * 16 + y, geo.ngy * 16, geo.bc[2], geo.bc[3]);
    return int64_t((Y >> 4) * geo.ngx + (X >> 4)) * (5 * 4096) + (Y & 15) * 16 + (X & 15);
  }
  __device__ int64_t plane(int z) const {
    const int Z = bc_wrap(gz * 16 + z, geo.ngz * 16, geo.bc[4], geo.bc[5]);
    return int64_t(Z >> 4) * geo.ngx * geo.ngy * (5 * 4096) + (Z & 15) * 256;
  }
  __device__ int64_t fstride() const { return 4096; }
};

template <typename T, class Src>
__device__ __forceinline__ void load_cons(const Src& src, int64_t col, int z, T U[5]) {
  const int64_t o = col + src.plane(z);
  const int64_t fs = src.fstride();
#pragma unroll
  for (int q = 0; q < 5; ++q) U[q] = src.base[o + q * fs];
}

template <typename T, class Src>
__device__ __forceinline__ void load_prim(const Src& src, int64_t col, int z, const Gas<T>& g, T W[5]) {
  T U[5];
  load_cons(src, col, z, U);
  cons_to_prim(U, g, W);
}

template <typename T>
struct Smem {
  T P[5][kPW * kPW];     // primitive plane k
  T S[2][5][kSW * kSW];  // x+ and y+ half-step states of plane k
  T F[2][5][17 * 16];    // x and y fluxes of plane k
};

// ---------------------------------------------------- one patch group ----
// Advance one group: read through `src`, write the 16^3 x 5 interior to `out`
// (field stride 4096).  Returns this thread's unphysical count.  If smax is
// non-null, also returns (interior threads) the maximum CFL signal speed of
// the thread's cells in patch-z halves 0..7 and 8..15.  `tid` is the thread's
// index in the workgroup (a loop over groups passes it opaque, so that the
// compiler keeps thread-derived addresses out of the loop's live set).
template <typename T, class Src>
__device__ __forceinline__ int process_group(const Src& src, T* __restrict__ out, const Gas<T>& gas,
                                             int first_order, int ws, Smem<T>& sm, double* smax,
                                             double gamma_d, int tid = threadIdx.x) {
  const bool interior = tid < 256;
  int cx, cy;          // own state column
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
  const int64_t col_own = src.col(cx, cy);
  const int64_t col_out = interior ? 0 : src.col(ox, oy);
  const int64_t col_edge = has_edge ? src.col(ex, ey) : 0;
  const int64_t fs = src.fstride();

  // register ring of the own column's primitive states; the conserved
  // values of the next plane to convert are loaded one iteration ahead
  // (software prefetch: the load latency overlaps a whole plane's work)
  T Wm[5], Wc[5], Wp[5];
  T Un[5];           // own column, plane k+1 (in flight during iteration k-1)
  T Uo[5], Ue[5];    // wave 4: 2-deep and edge column, plane k
  if (interior) load_prim(src, col_own, -2, gas, Wm);
  load_prim(src, col_own, -1, gas, Wc);
  load_cons(src, col_own, 0, Un);
  if (!interior) {
    load_cons(src, col_out, 0, Uo);
    if (has_edge) load_cons(src, col_edge, 0, Ue);
  }

  T Uz[5];         // z+ face state of the previous plane (interior)
  T Fz0[5];        // z flux at the low face of the previous plane (interior)
  T Ux[5], Uy[5];  // own x- and y- face states of the current plane
  int bad = 0;

  for (int k = -1; k <= 16; ++k) {
    // ---- next plane of the own column (prefetched); publish plane k to LDS
    if (interior || k + 1 <= 16) {
      cons_to_prim(Un, gas, Wp);
      if (k + 2 <= (interior ? 17 : 16)) load_cons(src, col_own, k + 2, Un);
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) sm.P[q][pidx(cx, cy)] = Wc[q];
    if (!interior && k >= 0 && k <= 15) {
      T Wo[5];
      cons_to_prim(Uo, gas, Wo);
      if (k + 1 <= 15) load_cons(src, col_out, k + 1, Uo);
#pragma unroll
      for (int q = 0; q < 5; ++q) sm.P[q][pidx(ox, oy)] = Wo[q];
      if (has_edge) {
        cons_to_prim(Ue, gas, Wo);
        if (k + 1 <= 15) load_cons(src, col_edge, k + 1, Ue);
#pragma unroll
        for (int q = 0; q < 5; ++q) sm.P[q][pidx(ex, ey)] = Wo[q];
      }
    }
    __syncthreads();

    // ---- x/y flux differences of plane k-1 (fluxes written last iteration)
    T acc[5];
    if (interior && k >= 1) {
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        acc[q] = sm.F[0][q][fxidx(cx + 1, cy)] - sm.F[0][q][fxidx(cx, cy)];
        acc[q] = acc[q] + (sm.F[1][q][fyidx(cx, cy + 1)] - sm.F[1][q][fyidx(cx, cy)]);
      }
    }

    // ---- half-step face states of the own state cell at plane k
    if (interior || (k >= 0 && k <= 15)) {
      T Wn[3][2][5];
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        Wn[0][0][q] = sm.P[q][pidx(cx - 1, cy)];
        Wn[0][1][q] = sm.P[q][pidx(cx + 1, cy)];
        Wn[1][0][q] = sm.P[q][pidx(cx, cy - 1)];
        Wn[1][1][q] = sm.P[q][pidx(cx, cy + 1)];
        Wn[2][0][q] = Wm[q];
        Wn[2][1][q] = Wp[q];
      }
      T Ut[3][2][5];
      hancock_states(Wc, Wn, gas, first_order != 0, Ut);
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        sm.S[0][q][sidx(cx, cy)] = Ut[0][1][q];
        sm.S[1][q][sidx(cx, cy)] = Ut[1][1][q];
        Ux[q] = Ut[0][0][q];
        Uy[q] = Ut[1][0][q];
      }
      if (interior) {
        if (k >= 0) {
          T Fz1[5];
          bad += hllc_flux<2>(Uz, Ut[2][0], gas, ws, Fz1);
          if (k >= 1) {
            // complete plane k-1: U^{n+1} = U^n - dt/dx [(x) + (y) + (z)]
            const int64_t o = col_own + src.plane(k - 1);
            T Un[5];
#pragma unroll
            for (int q = 0; q < 5; ++q) {
              const T a = acc[q] + (Fz1[q] - Fz0[q]);
              Un[q] = src.base[o + q * fs] - gas.dtdx * a;
              out[q * 4096 + ((k - 1) * 16 + cy) * 16 + cx] = Un[q];
            }
            bad += unphysical(Un, gas);
            if (smax != nullptr) {
              const double s = cfl_signal_speed(double(Un[0]), double(Un[1]), double(Un[2]), double(Un[3]),
                                                double(Un[4]), gamma_d);
              double& m = smax[(k - 1) >> 3];
              if (s > m) m = s;
            }
          }
#pragma unroll
          for (int q = 0; q < 5; ++q) Fz0[q] = Fz1[q];
        }
#pragma unroll
        for (int q = 0; q < 5; ++q) Uz[q] = Ut[2][1][q];
      }
    }
    __syncthreads();

    // ---- x and y faces of plane k
    if (k >= 0 && k <= 15) {
      if (interior || xface16) {
        T L[5], F[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) L[q] = sm.S[0][q][sidx(cx - 1, cy)];
        bad += hllc_flux<0>(L, Ux, gas, ws, F);
#pragma unroll
        for (int q = 0; q < 5; ++q) sm.F[0][q][fxidx(cx, cy)] = F[q];
      }
      if (interior || yface16) {
        T L[5], F[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) L[q] = sm.S[1][q][sidx(cx, cy - 1)];
        bad += hllc_flux<1>(L, Uy, gas, ws, F);
#pragma unroll
        for (int q = 0; q < 5; ++q) sm.F[1][q][fyidx(cx, cy)] = F[q];
      }
    }

#pragma unroll
    for (int q = 0; q < 5; ++q) {
      Wm[q] = Wc[q];
      Wc[q] = Wp[q];
    }
  }
  return bad;
}

// Reduce the per-thread signal-speed maxima of one group to its 8 patch
// time-steps (patch p = (pz*2 + py)*2 + px); LDS scratch `red` >= 512 doubles.
// Optionally stores dt_patch[8] and folds the minimum into *dt_min (integer
// minimum of non-negative doubles: exact and order-independent).
__device__ __forceinline__ void cfl_epilogue(const double smax[2], double* red, double c_cfl_dx,
                                             double* __restrict__ dt_patch, unsigned long long* __restrict__ dt_min) {
  const int tid = threadIdx.x;
  __syncthreads();
  if (tid < 256) {
    const int x = tid & 15, y = tid >> 4;
    const int pxy = (y >> 3) * 2 + (x >> 3), col = (y & 7) * 8 + (x & 7);
    red[(0 * 4 + pxy) * 64 + col] = smax[0];
    red[(1 * 4 + pxy) * 64 + col] = smax[1];
  }
  __syncthreads();
  if (tid < 8) {
    double m = 0.0;
    for (int i = 0; i < 64; ++i) {
      const double s = red[((tid >> 2) * 4 + (tid & 3)) * 64 + i];
      if (s > m) m = s;
    }
    const double dt = c_cfl_dx / m;
    if (dt_patch != nullptr) dt_patch[tid] = dt;
    if (dt_min != nullptr) atomicMin(dt_min, (unsigned long long)__double_as_longlong(dt));
  }
}

template <typename T>
__device__ __forceinline__ void set_dt(Gas<T>& gas, const double* dt_dev, double dx) {
  if (dt_dev != nullptr) {
    const double dt = *dt_dev;
    gas.dtdx = T(dt / dx);
    gas.half_dtdx = T(0.5 * (dt / dx));
  }
}

// Waves per SIMD the register allocation must allow: with 5-wave workgroups,
// 3 (FP64, <= 168 VGPRs) lets two workgroups share a CU (the LDS of two FP64
// workgroups fits in 160 KB); 5 (FP32, <= 102 VGPRs) lets four share it.
// The lower settings leave the allocator room for the prefetched plane (one
// FP64 or three FP32 workgroups per CU); `value` is the padded step's choice.
template <typename T> struct MinWaves;
template <> struct MinWaves<double> { static constexpr int hi = 3, lo = 2; static constexpr int value = lo; };
template <> struct MinWaves<float> { static constexpr int hi = 5, lo = 4; static constexpr int value = lo; };

}  // namespace gh
