// Per-group device code of the MHM step shared by the level kernels
// (mhm_fwd.hip) and the batched persistent kernel (mhm_batched.hip): input
// sources, the LDS layout, and the z-marching routine that advances one
// 16^3 patch group with one 256-thread workgroup (the mapping of threads to
// columns and roles is described at "one patch group" below).
#pragma once

#include <type_traits>

#include "ext_device.h"
#include "hydro_device.h"
#include "kernels.h"

namespace gh {

constexpr int kThreads = 256;
constexpr int kPW = 20;  // primitive plane tile: x, y in [-2, 17]
constexpr int kSW = 18;  // state tile: x, y in [-1, 16]

__device__ __forceinline__ int pidx(int x, int y) { return (y + 2) * kPW + (x + 2); }
__device__ __forceinline__ int sidx(int x, int y) { return (y + 1) * kSW + (x + 1); }
__device__ __forceinline__ int fxidx(int i, int j) { return j * 17 + i; }  // x-face i: between i-1 and i
__device__ __forceinline__ int fyidx(int i, int j) { return j * 16 + i; }  // y-face j: between j-1 and j

// ------------------------------------------------------------- sources ----
// A source maps group-relative cell coordinates to element offsets:
// offset(f, x, y, z) = col(x, y) + plane(z) + f * fstride, in the source's
// offset type Off.  A 32-bit unsigned offset lets every load take the
// scalar-base + 32-bit-vector-offset address form (no 64-bit address adds in
// the march, fewer registers: measured 1-5% per step); sources that can hold
// 2^32 elements or more use 64-bit offsets.

template <typename T>
struct PaddedSource {
  using Off = unsigned int;  // one group's padded block: 5 P^3 elements
  const T* base;  // this group's padded block
  int P, gh;
  __device__ Off col(int x, int y) const { return Off(y + gh) * P + (x + gh); }
  __device__ Off plane(int z) const { return Off(z + gh) * P * P; }
  __device__ Off fstride() const { return Off(P) * P * P; }
};

__device__ __forceinline__ int bc_wrap(int i, int n, int lo, int hi) {
  if (i < 0) return lo == 0 ? i + n : 0;
  if (i >= n) return hi == 0 ? i - n : n - 1;
  return i;
}

template <typename T, typename OffT = int64_t>
struct LevelSource {
  using Off = OffT;  // unsigned int only for levels of fewer than 2^32 elements
  const T* base;  // the level storage [G][5][16^3]
  LevelGeom geo;
  int gx, gy, gz;
  __device__ Off col(int x, int y) const {
    const int X = bc_wrap(gx * 16 + x, geo.ngx * 16, geo.bc[0], geo.bc[1]);
    const int Y = bc_wrap(gy * 16 + y, geo.ngy * 16, geo.bc[2], geo.bc[3]);
    return Off((Y >> 4) * geo.ngx + (X >> 4)) * (5 * 4096) + (Y & 15) * 16 + (X & 15);
  }
  __device__ Off plane(int z) const {
    const int Z = bc_wrap(gz * 16 + z, geo.ngz * 16, geo.bc[4], geo.bc[5]);
    return Off(Z >> 4) * geo.ngx * geo.ngy * (5 * 4096) + (Z & 15) * 256;
  }
  __device__ Off fstride() const { return 4096; }
};

template <typename T, class Src>
__device__ __forceinline__ void load_cons(const Src& src, typename Src::Off col, int z, T U[5]) {
  const typename Src::Off o = col + src.plane(z);
  const typename Src::Off fs = src.fstride();
#pragma unroll
  for (int q = 0; q < 5; ++q) U[q] = src.base[o + q * fs];
}

template <typename T, class Src>
__device__ __forceinline__ void load_prim(const Src& src, typename Src::Off col, int z, const Gas<T>& g, T W[5]) {
  T U[5];
  load_cons(src, col, z, U);
  cons_to_prim(U, g, W);
}

// LDS of one group's march.  kL pads the rows of the primitive and state
// tiles by kL elements (an LDS-layout option of the launch shapes: the same
// values at other addresses, so results are bit-identical).
template <typename T, int kL = 0>
struct Smem {
  static constexpr int PW = kPW + kL, SW = kSW + kL;
  static __device__ __forceinline__ int pi(int x, int y) { return (y + 2) * PW + (x + 2); }
  static __device__ __forceinline__ int si(int x, int y) { return (y + 1) * SW + (x + 1); }
  T P[5][PW * PW];       // primitive plane k
  T S[2][5][SW * SW];    // x+ and y+ half-step states of plane k
  T F[2][5][17 * 16];    // x and y fluxes of plane k
  T H[5][32];            // high-side states of the last faces: x = 16 (slot y), y = 16 (slot 16 + x)
};

// ------------------------------------------------------------- schemes ----
// The march computes one of two families of MHM + PLM steps:
//   DefaultScheme  generalized minmod on primitive variables and HLLC (the
//                  limiter specialized in its own inlined copy, see
//                  process_group), with the optional branch record;
//   ExtScheme      any MHM + PLM word of the other options (run-time
//                  ExtOpts: generalized minmod, van Leer, van Albada or
//                  hybrid limiter, on primitive or characteristic variables;
//                  HLLC, Roe or HLLE; either wave-speed option; first order):
//                  the same half step with the slopes of ext_slopes and the
//                  fluxes of riemann_any.
struct DefaultScheme {};
// kChr (0 / 1) fixes the characteristic projection at compile time and kRoe
// the solver family (1: Roe, 0: HLLC or HLLE); -1 leaves either to run
// time.  Each fixed combination is its own inlined copy, which carries only
// the registers of its own options.
template <int kChr = -1, int kRoe = -1>
struct ExtSchemeT {
  ExtOpts o;
  __device__ __forceinline__ ExtOpts opts() const {
    ExtOpts r = o;
    if (kChr >= 0) r.chr = kChr;
    if (kRoe == 1) r.solver = 1;
    if (kRoe == 0) r.solver = o.solver == 2 ? 2 : 0;
    return r;
  }
};
using ExtScheme = ExtSchemeT<>;

template <typename T>
__device__ __forceinline__ void scheme_half_step(const DefaultScheme&, const T Wc[5], const T Wn[3][2][5],
                                                 const Gas<T>& g, bool first_order, T Ut[3][2][5], unsigned* rec) {
  hancock_states(Wc, Wn, g, first_order, Ut, rec);
}

// The half step with full limited slopes s: face states Wc -+ s/2 (as the
// oracle's face values), then hancock_states' conserved form, fluxes and
// flux differences.
template <typename T, int kChr, int kRoe>
__device__ __forceinline__ void scheme_half_step(const ExtSchemeT<kChr, kRoe>& sch, const T Wc[5], const T Wn[3][2][5],
                                                 const Gas<T>& g, bool, T Ut[3][2][5], unsigned*) {
  const ExtOpts o = sch.opts();
  T sum[5];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    T sl[5];
    if (o.first_order) {
#pragma unroll
      for (int q = 0; q < 5; ++q) sl[q] = T(0);
    } else if (d == 0) {
      ext_slopes<0>(Wn[0][0], Wc, Wn[0][1], g, o, sl);
    } else if (d == 1) {
      ext_slopes<1>(Wn[1][0], Wc, Wn[1][1], g, o, sl);
    } else {
      ext_slopes<2>(Wn[2][0], Wc, Wn[2][1], g, o, sl);
    }
    T dF[5];
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      T W[5];
#pragma unroll
      for (int q = 0; q < 5; ++q) W[q] = side == 0 ? Wc[q] - T(0.5) * sl[q] : Wc[q] + T(0.5) * sl[q];
      T* U = Ut[d][side];
      U[0] = W[0];
      U[1] = W[0] * W[1];
      U[2] = W[0] * W[2];
      U[3] = W[0] * W[3];
      U[4] = W[4] * g.inv_gm1 + T(0.5) * W[0] * (W[1] * W[1] + W[2] * W[2] + W[3] * W[3]);
      const T un = W[1 + d];
      T F[5];
      F[0] = U[0] * un;
      F[1] = U[1] * un;
      F[2] = U[2] * un;
      F[3] = U[3] * un;
      F[1 + d] = F[1 + d] + W[4];
      F[4] = (U[4] + W[4]) * un;
#pragma unroll
      for (int q = 0; q < 5; ++q) dF[q] = side == 0 ? F[q] : dF[q] - F[q];
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) sum[q] = d == 0 ? dF[q] : sum[q] + dF[q];
  }
#pragma unroll
  for (int q = 0; q < 5; ++q) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      Ut[d][0][q] = fma_(g.half_dtdx, sum[q], Ut[d][0][q]);
      Ut[d][1][q] = fma_(g.half_dtdx, sum[q], Ut[d][1][q]);
    }
  }
}

template <int D, typename T>
__device__ __forceinline__ bool scheme_flux(const DefaultScheme&, const T L[5], const T R[5], const Gas<T>& g, int ws,
                                            T F[5], unsigned* rec) {
  return hllc_flux<D>(L, R, g, ws, F, rec);
}
template <int D, typename T, int kChr, int kRoe>
__device__ __forceinline__ bool scheme_flux(const ExtSchemeT<kChr, kRoe>& sch, const T L[5], const T R[5],
                                            const Gas<T>& g, int, T F[5], unsigned*) {
  return riemann_any<D>(L, R, g, sch.opts(), F);
}
// Two faces (normal axes D0, D1) at once; the default scheme interleaves
// their solves.
template <int D0, int D1, typename T>
__device__ __forceinline__ int scheme_flux2(const DefaultScheme&, const T L0[5], const T R0[5], const T L1[5],
                                            const T R1[5], const Gas<T>& g, int ws, T F0[5], T F1[5], unsigned* rec) {
  return hllc_flux2<D0, D1>(L0, R0, L1, R1, g, ws, F0, F1, rec);
}
template <int D0, int D1, typename T, int kChr, int kRoe>
__device__ __forceinline__ int scheme_flux2(const ExtSchemeT<kChr, kRoe>& sch, const T L0[5], const T R0[5],
                                            const T L1[5], const T R1[5], const Gas<T>& g, int, T F0[5], T F1[5],
                                            unsigned*) {
  const ExtOpts o = sch.opts();
  return int(riemann_any<D0>(L0, R0, g, o, F0)) + int(riemann_any<D1>(L1, R1, g, o, F1));
}

// ---------------------------------------------------- one patch group ----
// Workgroup of 256 threads (4 waves; the hardware gives each wave of a
// workgroup its own SIMD).  Every thread owns one interior (x, y) column; the
// 64 threads of wave 0 also own one "halo" column one cell outside the
// interior (x = -1, x = 16, y = -1, y = 16), whose half-step states feed the
// faces on the group boundary, together with the column two cells out and,
// for 4 of them, an edge column (both only read as neighbours).  Wave 0 runs
// its halo role after its interior role in every phase; wave 2 solves the 32
// faces on the high x and y boundary of the group (their high-side states
// come from the halo role through LDS) after its own faces.

// Per-column state of one role across the z-march.
template <typename T, bool kInterior, typename Off>
struct FwdCol {
  static constexpr int zhi = kInterior ? 17 : 16;  // last plane of the column that is read
  int cx, cy;
  bool xface16, yface16;  // halo columns at x = 16 / y = 16 (high side of the last x / y face)
  Off col;
  T Wm[5], Wc[5], Wp[5];  // primitive states at planes k-1, k, k+1
  T Un[5];                // conserved values of the next plane to convert (in flight)
  T Ux[5], Uy[5];         // own x- and y- face states of plane k (interior)
  T Uz[5], Fz0[5];        // interior: z+ face state of plane k-1; z flux at the low face of plane k-1
};

template <typename T, bool kI, class Src>
__device__ __forceinline__ void fwd_col_init(FwdCol<T, kI, typename Src::Off>& c, const Src& src, int cx, int cy, const Gas<T>& gas) {
  c.cx = cx;
  c.cy = cy;
  c.xface16 = !kI && cx == 16;
  c.yface16 = !kI && cy == 16;
  c.col = src.col(cx, cy);
  if (kI) load_prim(src, c.col, -2, gas, c.Wm);
  load_prim(src, c.col, -1, gas, c.Wc);
  load_cons(src, c.col, 0, c.Un);
}

// Next plane of the column (prefetched one iteration ahead); publish plane k.
template <typename T, bool kI, class Src, int kL>
__device__ __forceinline__ void fwd_col_publish(FwdCol<T, kI, typename Src::Off>& c, const Src& src, int k, const Gas<T>& gas,
                                                Smem<T, kL>& sm) {
  // Convert the plane that arrived, then issue the next one.  The load is
  // unconditional (plane index clamped to the column's last plane, re-read
  // harmlessly near the top) and issued after the conversion, so the loaded
  // registers are never merged with old values: a merge would need the data
  // and wait for the load that is meant to stay in flight.
  cons_to_prim(c.Un, gas, c.Wp);
  asm volatile("" ::: "memory");
  load_cons(src, c.col, k + 2 <= c.zhi ? k + 2 : c.zhi, c.Un);
#pragma unroll
  for (int q = 0; q < 5; ++q) sm.P[q][sm.pi(c.cx, c.cy)] = c.Wc[q];
}

// CFL signal-speed maxima of a group live in LDS as [z half][patch xy][64
// columns of the patch] (the order the epilogue reduces in): a thread's slot
// for z half 0 is cfl_slot(tid), its slot for z half 1 lies kCflHalfStride
// doubles further.  Kept in LDS rather than registers (4 VGPRs fewer through
// the march).
constexpr int kCflHalfStride = 256;
__device__ __forceinline__ int cfl_slot(int tid) {
  const int x = tid & 15, y = tid >> 4;
  return ((y >> 3) * 2 + (x >> 3)) * 64 + (y & 7) * 8 + (x & 7);
}

// Half-step face states of the column's state cell at plane k.  Interior
// columns also solve the z-face k-1/2 and complete plane k-1.
template <typename T, bool kI, class Src, int kL, class Sch>
__device__ __forceinline__ int fwd_col_states(const Sch& sch, FwdCol<T, kI, typename Src::Off>& c, const Src& src, T* __restrict__ out, int k,
                                              const Gas<T>& gas, int first_order, int ws, Smem<T, kL>& sm, double* smax,
                                              double gamma_d, T* __restrict__ ff, unsigned* rec) {
  const int cx = c.cx, cy = c.cy;
  int bad = 0;
  // U^n of plane k-1 for its update at the end of this phase, issued first
  // so that the load's latency overlaps the half step and the z-face solve
  T Uold[5];
  if (kI && k >= 1) load_cons(src, c.col, k - 1, Uold);
  // x/y flux differences of plane k-1 (fluxes written last iteration)
  T acc[5];
  if (kI && k >= 1) {
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      acc[q] = sm.F[0][q][fxidx(cx + 1, cy)] - sm.F[0][q][fxidx(cx, cy)];
      acc[q] = acc[q] + (sm.F[1][q][fyidx(cx, cy + 1)] - sm.F[1][q][fyidx(cx, cy)]);
    }
  }
  if (!kI && (k < 0 || k > 15)) return 0;
  T Wn[3][2][5];
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    Wn[0][0][q] = sm.P[q][sm.pi(cx - 1, cy)];
    Wn[0][1][q] = sm.P[q][sm.pi(cx + 1, cy)];
    Wn[1][0][q] = sm.P[q][sm.pi(cx, cy - 1)];
    Wn[1][1][q] = sm.P[q][sm.pi(cx, cy + 1)];
    Wn[2][0][q] = c.Wm[q];
    Wn[2][1][q] = c.Wp[q];
  }
  T Ut[3][2][5];
  scheme_half_step(sch, c.Wc, Wn, gas, first_order != 0, Ut, rec);
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    sm.S[0][q][sm.si(cx, cy)] = Ut[0][1][q];
    sm.S[1][q][sm.si(cx, cy)] = Ut[1][1][q];
    if (kI) {
      c.Ux[q] = Ut[0][0][q];
      c.Uy[q] = Ut[1][0][q];
    }
  }
  // halo columns at x = 16 / y = 16: their low x / y state is the high side
  // of the last face, solved by another wave after the next barrier
  if (!kI && (c.xface16 || c.yface16)) {
    const int slot = c.xface16 ? cy : 16 + cx;
#pragma unroll
    for (int q = 0; q < 5; ++q) sm.H[q][slot] = c.xface16 ? Ut[0][0][q] : Ut[1][0][q];
  }
  if (kI) {
    if (k >= 0) {
      T Fz1[5];
      bad += scheme_flux<2>(sch, c.Uz, Ut[2][0], gas, ws, Fz1, rec);
      if (ff != nullptr && (k & 7) == 0) {
        // z faces on a patch boundary (z = 0, 8, 16): plane 6 + k/8, entry y*16 + x
        T* o = ff + (6 + (k >> 3)) * 5 * 256 + cy * 16 + cx;
#pragma unroll
        for (int q = 0; q < 5; ++q) o[q * 256] = Fz1[q];
      }
      if (k >= 1) {
        // complete plane k-1: U^{n+1} = U^n - dt/dx [(x) + (y) + (z)]
        T Un[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) {
          const T a = acc[q] + (Fz1[q] - c.Fz0[q]);
          Un[q] = Uold[q] - gas.dtdx * a;
          out[q * 4096 + ((k - 1) * 16 + cy) * 16 + cx] = Un[q];
        }
        bad += unphysical(Un, gas);
        if (smax != nullptr) {
          const double s = cfl_signal_speed(double(Un[0]), double(Un[1]), double(Un[2]), double(Un[3]),
                                            double(Un[4]), gamma_d);
          double& m = smax[((k - 1) >> 3) * kCflHalfStride];
          if (s > m) m = s;
        }
      }
#pragma unroll
      for (int q = 0; q < 5; ++q) c.Fz0[q] = Fz1[q];
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) c.Uz[q] = Ut[2][1][q];
  }
  return bad;
}

// x and y faces of plane k that an interior column solves: its low x and low
// y face.
template <typename T, bool kI, typename Off, int kL, class Sch>
__device__ __forceinline__ int fwd_col_faces(const Sch& sch, FwdCol<T, kI, Off>& c, int k, const Gas<T>& gas, int ws, Smem<T, kL>& sm,
                                             T* __restrict__ ff, unsigned* rec) {
  if (!kI || k < 0 || k > 15) return 0;
  const int cx = c.cx, cy = c.cy;
  T Lx[5], Fx[5], Ly[5], Fy[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    Lx[q] = sm.S[0][q][sm.si(cx - 1, cy)];
    Ly[q] = sm.S[1][q][sm.si(cx, cy - 1)];
  }
  const int bad = scheme_flux2<0, 1>(sch, Lx, c.Ux, Ly, c.Uy, gas, ws, Fx, Fy, rec);
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    sm.F[0][q][fxidx(cx, cy)] = Fx[q];
    sm.F[1][q][fyidx(cx, cy)] = Fy[q];
  }
  if (ff != nullptr && (cx & 7) == 0) {
    // x faces at x = 0, 8: plane x/8, entry z*16 + y
    T* o = ff + (cx >> 3) * 5 * 256 + k * 16 + cy;
#pragma unroll
    for (int q = 0; q < 5; ++q) o[q * 256] = Fx[q];
  }
  if (ff != nullptr && (cy & 7) == 0) {
    // y faces at y = 0, 8: plane 3 + y/8, entry x*16 + z
    T* o = ff + (3 + (cy >> 3)) * 5 * 256 + cx * 16 + k;
#pragma unroll
    for (int q = 0; q < 5; ++q) o[q * 256] = Fy[q];
  }
  return bad;
}

// The 32 last faces of plane k (x = 16 for lanes 0..15 at y = lane, y = 16
// for lanes 16..31 at x = lane - 16), in one solver pass: a y face is solved
// in the x-normal frame with its states rotated (m_y, m_z, m_x) -> (m_x,
// m_y, m_z), the same arithmetic on the same values as the y-normal solver,
// and the flux rotated back.  The halo wave wrote the high-side states to
// H; this pass runs on another wave, which has no halo work.
template <typename T, int kL, class Sch>
__device__ __forceinline__ int last_faces(const Sch& sch, int lane, int k, const Gas<T>& gas, int ws, Smem<T, kL>& sm,
                                          T* __restrict__ ff, unsigned* rec) {
  if (k < 0 || k > 15 || lane >= 32) return 0;
  const bool yf = lane >= 16;
  const int i = lane & 15;
  const T* Sb = yf ? &sm.S[1][0][sm.si(i, 15)] : &sm.S[0][0][sm.si(15, i)];
  T L[5], R[5], Lr[5], Rr[5], F[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    L[q] = Sb[q * sm.SW * sm.SW];
    R[q] = sm.H[q][lane];
  }
  Lr[0] = L[0];
  Lr[1] = yf ? L[2] : L[1];
  Lr[2] = yf ? L[3] : L[2];
  Lr[3] = yf ? L[1] : L[3];
  Lr[4] = L[4];
  Rr[0] = R[0];
  Rr[1] = yf ? R[2] : R[1];
  Rr[2] = yf ? R[3] : R[2];
  Rr[3] = yf ? R[1] : R[3];
  Rr[4] = R[4];
  const int bad = scheme_flux<0>(sch, Lr, Rr, gas, ws, F, rec);
  T* Fb = yf ? &sm.F[1][0][fyidx(i, 16)] : &sm.F[0][0][fxidx(16, i)];
  Fb[0] = F[0];
  Fb[1 * 17 * 16] = yf ? F[3] : F[1];
  Fb[2 * 17 * 16] = yf ? F[1] : F[2];
  Fb[3 * 17 * 16] = yf ? F[2] : F[3];
  Fb[4 * 17 * 16] = F[4];
  if (ff != nullptr) {
    // x = 16: plane 2, entry z*16 + y; y = 16: plane 5, entry x*16 + z
    T* o = ff + (yf ? 5 * 5 * 256 + i * 16 + k : 2 * 5 * 256 + k * 16 + i);
    o[0] = F[0];
    o[1 * 256] = yf ? F[3] : F[1];
    o[2 * 256] = yf ? F[1] : F[2];
    o[3 * 256] = yf ? F[2] : F[3];
    o[4 * 256] = F[4];
  }
  return bad;
}

template <typename T, bool kI, typename Off>
__device__ __forceinline__ void fwd_col_shift(FwdCol<T, kI, Off>& c) {
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    c.Wm[q] = c.Wc[q];
    c.Wc[q] = c.Wp[q];
  }
}

// Roles of the waves of a workgroup beyond their interior columns.
enum WaveRole { kRoleHalo = 0, kRoleLastFaces = 1, kRolePlain = 2 };

// The z-march of one wave: interior role, plus the halo roles (kRoleHalo,
// wave 0) or the solve of the 32 last faces (kRoleLastFaces, wave 2).  Every
// instantiation passes the same barriers in the same order.
template <typename T, class Src, int kRole, int kUnroll, int kL, class Sch>
__device__ __forceinline__ int march_group(const Sch& sch, const Src& src, T* __restrict__ out, const Gas<T>& gas, int first_order,
                                           int ws, Smem<T, kL>& sm, double* smax, double gamma_d, int tid,
                                           T* __restrict__ ff, unsigned* rec) {
  // halo role: side 0..3 = x-, x+, y-, y+; the column two cells out; lanes
  // 0..3 also one of the 4 edge columns
  const int lane = tid & 63;
  const int side = lane >> 4, kk = lane & 15;
  const int hx = side == 0 ? -1 : side == 1 ? 16 : kk, hy = side == 2 ? -1 : side == 3 ? 16 : kk;
  const int ox = side == 0 ? -2 : side == 1 ? 17 : kk, oy = side == 2 ? -2 : side == 3 ? 17 : kk;
  const int ex = (lane & 1) ? 16 : -1, ey = (lane & 2) ? 16 : -1;
  constexpr bool kHalo = kRole == kRoleHalo;
  const bool has_edge = kHalo && lane < 4;

  using Off = typename Src::Off;
  FwdCol<T, true, Off> ci;
  FwdCol<T, false, Off> ch;
  fwd_col_init(ci, src, tid & 15, tid >> 4, gas);
  Off col_out = 0, col_edge = 0;
  T Uo[5], Ue[5];  // halo role: 2-deep and edge column, plane k (in flight)
  if (kHalo) {
    col_out = src.col(ox, oy);
    col_edge = src.col(has_edge ? ex : ox, has_edge ? ey : oy);  // lanes without an edge re-read their 2-deep column
    fwd_col_init(ch, src, hx, hy, gas);
    load_cons(src, col_out, 0, Uo);
    load_cons(src, col_edge, 0, Ue);
  }
  int bad = 0;

#pragma unroll kUnroll
  for (int k = -1; k <= 16; ++k) {
    // ---- next planes (prefetched); publish plane k to LDS
    fwd_col_publish(ci, src, k, gas, sm);
    if (kHalo) {
      fwd_col_publish(ch, src, k, gas, sm);
      // 2-deep and edge columns (planes 0..15; loads clamped, no merge of
      // loaded registers with old values)
      T Wo[5], We[5];
      cons_to_prim(Uo, gas, Wo);
      cons_to_prim(Ue, gas, We);
      asm volatile("" ::: "memory");
      const int kn = k + 1 < 0 ? 0 : (k + 1 > 15 ? 15 : k + 1);
      load_cons(src, col_out, kn, Uo);
      load_cons(src, col_edge, kn, Ue);
      if (k >= 0 && k <= 15) {
#pragma unroll
        for (int q = 0; q < 5; ++q) sm.P[q][sm.pi(ox, oy)] = Wo[q];
        if (has_edge) {
#pragma unroll
          for (int q = 0; q < 5; ++q) sm.P[q][sm.pi(ex, ey)] = We[q];
        }
      }
    }
    __syncthreads();

    // ---- half-step face states of plane k; z-face and update of plane k-1
    bad += fwd_col_states(sch, ci, src, out, k, gas, first_order, ws, sm, smax, gamma_d, ff, rec);
    if (kHalo) bad += fwd_col_states(sch, ch, src, out, k, gas, first_order, ws, sm, nullptr, gamma_d, (T*)nullptr, rec);
    __syncthreads();

    // ---- x and y faces of plane k
    bad += fwd_col_faces(sch, ci, k, gas, ws, sm, ff, rec);
    if (kRole == kRoleLastFaces) bad += last_faces(sch, lane, k, gas, ws, sm, ff, rec);

    fwd_col_shift(ci);
    if (kHalo) fwd_col_shift(ch);
  }
  return bad;
}

// Advance one group: read through `src`, write the 16^3 x 5 interior to `out`
// (field stride 4096).  Returns this thread's unphysical count.  If smax is
// non-null (the thread's cfl_slot in an LDS array, both halves set to 0),
// also leaves there the maximum CFL signal speed of the thread's interior
// cells in patch-z halves 0..7 and 8..15.  If ff is non-null, also writes the
// fluxes of the faces on the patch boundaries (normal coordinate 0, 8, 16 of
// each axis) to ff as [9][5][256]: plane 3 axis + k holds the faces at 8 k,
// entry b * 16 + a with (a, b) the transverse coordinates in cyclic order
// (the flux registers of coarse-fine coupling).  `tid` is the thread's index in the
// workgroup (a loop over groups passes it opaque, so that the compiler keeps
// thread-derived addresses out of the loop's live set).  Wave 0 runs the
// march with the halo roles, wave 2 with the last faces, waves 1 and 3 with
// their interior columns only (wave-uniform branches).  Two co-resident
// workgroups get their waves on SIMDs (0, 2, 1, 3) and (2, 1, 3, 0), so the
// halo waves sit on SIMDs 0 and 2 and the last-face waves on SIMDs 1 and 3.
// The second-order scheme (first_order == 0) gets its own inlined copies
// with the limiter unconditional; the first-order one keeps the runtime flag.
// kPrio: the halo wave (the most work per plane) and the last-faces wave take
// issue priority over the plain waves they share a SIMD with, so the plane's
// barrier is reached sooner.  Measured on the 256^3 shear layer: with four
// waves per SIMD (FP32, high occupancy) the step is 6-8% faster; with two
// (FP64, FP32 low occupancy) 2-5% slower, so those kernels keep equal
// priorities.
template <typename T, bool kPrio, class Src, int kL, class Sch>
__device__ __forceinline__ int march_roles(const Sch& sch, const Src& src, T* __restrict__ out, const Gas<T>& gas,
                                           int first_order, int ws, Smem<T, kL>& sm, double* smax, double gamma_d,
                                           int tid, T* __restrict__ ff, unsigned* rec) {
  const int wave = __builtin_amdgcn_readfirstlane(tid >> 6);
  // Two planes per loop iteration, so that the register rotation of a
  // column's planes (Wm <- Wc <- Wp, z-face state and flux) becomes renaming
  // instead of moves (2-3% fewer VALU instructions per plane): every role in
  // FP32 at the low occupancy target (step 2% faster), the plain and
  // last-faces roles in FP64 (step 0.5-0.8% faster; the halo role, which
  // carries a second column, would need more than 256 VGPRs).  The four-wave
  // FP32 kernels (kPrio; 128 VGPRs, where it spills) and the other scheme
  // words keep one plane.
  constexpr int kU = (sizeof(T) == 4 && !kPrio) ? 2 : 1;   // halo role
  constexpr int kU2 = !kPrio ? 2 : 1;                       // the other roles
  if constexpr (kPrio) {
    if (wave == 0) __builtin_amdgcn_s_setprio(2);
    if (wave == 2) __builtin_amdgcn_s_setprio(1);
  }
  if constexpr (!std::is_same<Sch, DefaultScheme>::value) {
    // the other words: one copy (their options are run-time anyway), one
    // plane per loop iteration
    if (wave == 0) return march_group<T, Src, kRoleHalo, 1>(sch, src, out, gas, first_order, ws, sm, smax, gamma_d, tid, ff, rec);
    if (wave == 2)
      return march_group<T, Src, kRoleLastFaces, 1>(sch, src, out, gas, first_order, ws, sm, smax, gamma_d, tid, ff, rec);
    return march_group<T, Src, kRolePlain, 1>(sch, src, out, gas, first_order, ws, sm, smax, gamma_d, tid, ff, rec);
  } else {
    if (first_order == 0) {
      if (wave == 0) return march_group<T, Src, kRoleHalo, kU>(sch, src, out, gas, 0, ws, sm, smax, gamma_d, tid, ff, rec);
      if (wave == 2)
        return march_group<T, Src, kRoleLastFaces, kU2>(sch, src, out, gas, 0, ws, sm, smax, gamma_d, tid, ff, rec);
      return march_group<T, Src, kRolePlain, kU2>(sch, src, out, gas, 0, ws, sm, smax, gamma_d, tid, ff, rec);
    }
    if (wave == 0)
      return march_group<T, Src, kRoleHalo, kU>(sch, src, out, gas, first_order, ws, sm, smax, gamma_d, tid, ff, rec);
    if (wave == 2)
      return march_group<T, Src, kRoleLastFaces, kU2>(sch, src, out, gas, first_order, ws, sm, smax, gamma_d, tid, ff, rec);
    return march_group<T, Src, kRolePlain, kU2>(sch, src, out, gas, first_order, ws, sm, smax, gamma_d, tid, ff, rec);
  }
}

// rec_out (diagnostic, optional): the group's branch record -- every
// thread's decisions hashed in its own order (record()), the threads' hashes
// combined by XOR, which is independent of the order they arrive in.
template <typename T, bool kPrio, class Src, int kL, class Sch = DefaultScheme>
__device__ __forceinline__ int process_group(const Src& src, T* __restrict__ out, const Gas<T>& gas,
                                             int first_order, int ws, Smem<T, kL>& sm, double* smax,
                                             double gamma_d, int tid = threadIdx.x, T* __restrict__ ff = nullptr,
                                             unsigned* __restrict__ rec_out = nullptr, const Sch& sch = Sch()) {
  if (rec_out == nullptr)
    return march_roles<T, kPrio>(sch, src, out, gas, first_order, ws, sm, smax, gamma_d, tid, ff, nullptr);
  __shared__ unsigned grp_rec;
  if (tid == 0) grp_rec = 0u;  // the march's first barrier orders this before any XOR
  unsigned h = 2166136261u ^ (unsigned(tid) * 0x9E3779B9u);
  const int bad = march_roles<T, kPrio>(sch, src, out, gas, first_order, ws, sm, smax, gamma_d, tid, ff, &h);
  atomicXor(&grp_rec, h);
  __syncthreads();
  if (tid == 0) *rec_out = grp_rec;
  return bad;
}

// Reduce the per-thread signal-speed maxima of one group (the LDS array
// `slots` of cfl_slot's layout, 512 doubles: patch p = (pz*2 + py)*2 + px owns
// slots [64 p, 64 p + 64)) to its 8 patch time-steps: thread p < 8 scans its
// patch's 64 slots (a maximum is exact in any order; NaN and negative speeds
// never win over the start value 0).  A butterfly of lane shuffles over the
// 4 waves (each wave two patches) was measured slower on the 256^3 step (FP64
// 0.904 vs 0.881 ms, FP32 0.553 vs 0.493 ms).  Stores dt_patch[p]
// (optional) and folds dt * fold_scale into *dt_min (optional; integer
// minimum of non-negative doubles: exact and order-independent).  Every
// thread of the workgroup must call it.
__device__ __forceinline__ void cfl_epilogue(const double* slots, double c_cfl_dx,
                                             double* __restrict__ dt_patch, unsigned long long* __restrict__ dt_min,
                                             double fold_scale = 1.0, int tid = threadIdx.x) {
  __syncthreads();
  if (tid < 8) {
    double m = 0.0;
    for (int i = 0; i < 64; ++i) {
      const double s = slots[tid * 64 + i];
      if (s > m) m = s;
    }
    const double dt = c_cfl_dx / m;
    if (dt_patch != nullptr) dt_patch[tid] = dt;
    if (dt_min != nullptr) atomicMin(dt_min, (unsigned long long)__double_as_longlong(dt * fold_scale));
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

// Waves per SIMD the register allocation must allow.  Each wave of a 4-wave
// workgroup gets its own SIMD, so this is also the number of workgroups per
// CU the registers allow: FP64 2 (<= 256 VGPRs; two workgroups' LDS fits in
// 160 KB) or 1; FP32 4 (<= 128 VGPRs) or 2.  `value` is the padded step's.
template <typename T> struct MinWaves;
template <> struct MinWaves<double> { static constexpr int hi = 2, lo = 1; static constexpr int value = hi; };
template <> struct MinWaves<float> { static constexpr int hi = 4, lo = 2; static constexpr int value = hi; };

}  // namespace gh
