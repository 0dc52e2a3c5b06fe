// Adjoint of the MHM step (reverse mode through a0-a6): given the cotangent
// gU' of the updated interiors, produce the cotangent of the step's input.
//
//   U'_c = U_c - dt/dx sum_faces (+-F_f),  F_f = HLLC(Ut_left, Ut_right),
//   Ut = Hancock(W of the cell and its 6 neighbours),  W = prim(U).
//
// Two kernels, both deterministic (no floating-point atomics):
//   fused (per group, z-march like the forward): recompute the half-step
//      face states of plane k; take the HLLC VJP at every face with
//      gF = dt/dx (gU'_right - gU'_left) (the face flux leaves the left cell
//      and enters the right one; gU' = 0 outside the interior); one plane
//      behind, reverse the Hancock predictor (fluxes, cons, limiter) of every
//      state cell into cotangents of the primitive states of the cell and its
//      6 neighbours, gather them per cell (in-plane through LDS, along z
//      through a register ring), reverse cons -> prim and add the identity
//      term gU' of interior cells.  Output: the cotangent of every
//      stencil-reachable cell of the group, on the [-2,17]^3 box (level path)
//      or in the padded layout (padded path).
//   gather (per level cell): sum the cotangents of all copies of the cell
//      that the groups read (its own interior copy and the ghost copies in
//      neighbouring groups), enumerated in closed form from the ghost-fill
//      index map -- the adjoint of the ghost fill, written as a gather.  The
//      same kernel sums padded blocks of any ghost width
//      (hydro_gather_ghost_adjoint).

#include "hydro_adjoint.h"
#include "mhm_group.h"
#include "mhm_level.h"

namespace gh {

namespace {

constexpr int kBox = 20;      // reachable box [-2, 17] per axis

__device__ __forceinline__ int b3idx(int x, int y, int z) { return ((z + 2) * kBox + (y + 2)) * kBox + (x + 2); }

// gU' (cotangent of the output interiors) of one group: [5][4096].
template <typename T>
__device__ __forceinline__ T gout(const T* __restrict__ go, int q, int x, int y, int z) {
  return (x < 0 || x > 15 || y < 0 || y > 15 || z < 0 || z > 15) ? T(0) : go[q * 4096 + (z * 16 + y) * 16 + x];
}

// ------------------------------------------------------ cell helpers ----
// Which faces of a state cell carry a cotangent (the others were not used by
// the step): interior cells all six; the halo state cells only the face they
// share with the interior; the two extra z planes only their inner z face.
__device__ __forceinline__ bool face_used(int x, int y, int z, int f) {
  const bool in_x = x >= 0 && x <= 15, in_y = y >= 0 && y <= 15, in_z = z >= 0 && z <= 15;
  if (in_x && in_y && in_z) return true;
  if (x == -1) return f == 1;
  if (x == 16) return f == 0;
  if (y == -1) return f == 3;
  if (y == 16) return f == 2;
  if (z == -1) return f == 5;
  return f == 4;  // z == 16
}

// Sink for the input cotangent of one group's reachable cells.
template <typename T>
struct BoxSink {
  T* base;  // [5][20^3]
  __device__ void put(int q, int x, int y, int z, T v) const { base[q * (kBox * kBox * kBox) + b3idx(x, y, z)] = v; }
};
template <typename T>
struct PadSink {
  T* base;  // [5][P^3]
  int P, gh;
  __device__ void put(int q, int x, int y, int z, T v) const {
    base[int64_t(q) * P * P * P + (int64_t(z + gh) * P + (y + gh)) * P + (x + gh)] = v;
  }
};

template <typename T, class Src, class Sink>
__device__ __forceinline__ void finalize_cell(const Src& src, int64_t col, int x, int y, int z, const T gW[5],
                                              const T* __restrict__ go, const Gas<T>& gas, const Sink& sink) {
  const int64_t o = col + src.plane(z);
  const int64_t fs = src.fstride();
  T U[5], gU[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    U[q] = src.base[o + q * fs];
    gU[q] = gout(go, q, x, y, z);  // identity term of the update (interior cells)
  }
  cons_to_prim_vjp(U, gas, gW, gU);
#pragma unroll
  for (int q = 0; q < 5; ++q) sink.put(q, x, y, z, gU[q]);
}

// ------------------------------------------------------- fused kernel ----
// One z-march per group that does both halves with a one-plane lag: at
// iteration k it recomputes the half-step states of plane k, takes the HLLC
// VJPs of the z-face (k-1 | k) and of the x/y faces of plane k, and reverses
// the Hancock predictor of plane k-1, whose six face cotangents are then
// complete.  Face cotangents reach the cell that owns the face state through
// registers (the faces a thread solves itself) or LDS (the x+/y+ faces, solved
// by the neighbouring thread); the cell's cotangents for its in-plane
// neighbours go through LDS, those along z stay in a register ring.
//
// Workgroup: 256 threads (4 waves, one per SIMD).  Every thread owns one
// interior column; the 64 threads of wave 0 also own one halo column each (the
// 4 x 16 columns just outside the faces, whose state cells feed the boundary
// faces) with its 2-deep neighbour and, for 4 of them, an edge column, and run
// that role after the interior one in every phase (the reverse predictor and
// finish of the halo columns run on wave 1, from LDS); wave 2 takes the VJPs of
// the 32 faces the halo columns at x = 16 and y = 16 share with the interior
// (states and cotangents through LDS) and wave 3 finishes the 2-deep and
// edge columns (their contributions are in LDS), which evens out the waves'
// work.  One wave per SIMD leaves
// the whole register file (VGPRs and AGPRs) to each wave.
constexpr int kAdjThreads = 256;
// Waves per SIMD the register allocation targets: FP64 takes the whole
// register file (one workgroup per CU, which its LDS needs anyway); FP32 fits
// two workgroups per CU (LDS 75 KB each) at a few spilled registers, which
// measured faster than one workgroup with none.
template <typename T> struct AdjWaves { static constexpr int value = sizeof(T) == 8 ? 1 : 2; };

template <typename T>
struct SmemF {
  T P[3][5][kPW * kPW];   // primitive planes, slot (k + 3) % 3
  T S[2][5][kSW * kSW];   // x+ and y+ half-step states of plane k
  T GL[2][5][kSW * kSW];  // cotangents of the x+ / y+ face states of plane k-1 cells
  T O[4][5][kSW * kSW];   // in-plane neighbour contributions of plane k-1 cells (x-, x+, y-, y+)
  T H[5][32];             // high-side states of the last faces of plane k: x = 16 (slot y), y = 16 (slot 16 + x)
  T GR[5][32];            // their cotangents (same slots), read by the halo columns one plane later
};

// Slot of a halo column at x = 16 or y = 16 in SmemF::H / GR (in range for
// every halo column; only those two sides use it).
__device__ __forceinline__ int last_slot(bool xface16, int cx, int cy) { return (xface16 ? cy : 16 + cx) & 31; }

__device__ __forceinline__ int pslot(int k) { return (k + 3) % 3; }

// finalize_cell with the cell's primitive state taken from its LDS plane
// (published by the march; the same values cons_to_prim gives, so the same
// Jacobian as from the conserved state) instead of a load from memory.
template <typename T, class Sink>
__device__ __forceinline__ void finalize_cell_lds(const SmemF<T>& sm, int x, int y, int z, const T gW[5],
                                                  const T* __restrict__ go, const Gas<T>& gas, const Sink& sink) {
  const int s = pslot(z), i = pidx(x, y);
  const T W0 = sm.P[s][0][i];
  const T inv = Fp<T>::rcp(W0);
  const T u = sm.P[s][1][i], v = sm.P[s][2][i], w = sm.P[s][3][i];
  const T gp = gW[4] * gas.gm1;
  T gU[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) gU[q] = gout(go, q, x, y, z);  // identity term of the update (interior cells)
  // the arithmetic of cons_to_prim_vjp with u = m_x / rho, ... read back
  gU[0] = gU[0] + gW[0] - (gW[1] * u + gW[2] * v + gW[3] * w) * inv + T(0.5) * gp * (u * u + v * v + w * w);
  gU[1] = gU[1] + gW[1] * inv - gp * u;
  gU[2] = gU[2] + gW[2] * inv - gp * v;
  gU[3] = gU[3] + gW[3] * inv - gp * w;
  gU[4] = gU[4] + gp;
#pragma unroll
  for (int q = 0; q < 5; ++q) sink.put(q, x, y, z, gU[q]);
}

// Is (x, y, z) a state cell (one whose half-step states the step computes)?
__device__ __forceinline__ bool in_state_plane(int x, int y, int z) {
  const bool in_x = x >= 0 && x <= 15, in_y = y >= 0 && y <= 15;
  if (in_x && in_y) return z >= -1 && z <= 16;
  const bool hx = (x == -1 || x == 16) && in_y, hy = (y == -1 || y == 16) && in_x;
  return (hx || hy) && z >= 0 && z <= 15;
}

// Per-column state of one role (interior or halo column) across the march.
// The column's primitive states of planes k-2, k-1, k are read back from the
// LDS planes (the column publishes its own values there); only W(k+1) lives
// in registers.  The face a halo column at x = 16 or y = 16 shares with the
// interior is solved by another wave: its state and cotangent go through LDS
// (SmemF::H, GR).
template <typename T, bool kInterior>
struct AdjCol {
  static constexpr bool interior = kInterior;
  static constexpr int zlo = kInterior ? -2 : -1, zhi = kInterior ? 17 : 16;  // reachable planes of the column
  int cx, cy;
  bool xface16, yface16;
  int64_t col;
  T Wp[5];                    // W(k+1) (becomes W(k) at the next publish)
  T Un[5];                    // conserved values of plane k+2 (in flight)
  T Uz[5];                    // z+ face state of plane k-1 (interior columns)
  T Ux[5], Uy[5];             // own x- and y- face states of plane k
  T gRx[5], gRy[5], gRz[5];   // cotangents of the own x-, y-, z- face states of plane k-1
  T A0[5], A1[5], A2[5];      // input cotangents of the column at planes k-2, k-1, k
};

template <typename T, bool kI, class Src>
__device__ __forceinline__ void adj_col_init(AdjCol<T, kI>& c, const Src& src, int cx, int cy, const Gas<T>& gas,
                                             SmemF<T>& sm) {
  c.cx = cx;
  c.cy = cy;
  c.xface16 = !kI && cx == 16;
  c.yface16 = !kI && cy == 16;
  c.col = src.col(cx, cy);
  if (kI) {
    T W[5];
    load_prim(src, c.col, -2, gas, W);
#pragma unroll
    for (int q = 0; q < 5; ++q) sm.P[pslot(-2)][q][pidx(cx, cy)] = W[q];
  }
  load_prim(src, c.col, -1, gas, c.Wp);  // published as plane -1 by the first iteration
  load_cons(src, c.col, 0, c.Un);
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    c.gRx[q] = c.gRy[q] = c.gRz[q] = T(0);
    c.A0[q] = c.A1[q] = c.A2[q] = T(0);
  }
}

// F1: publish plane k; convert plane k+1 (loaded one iteration ago) and
// issue the load of plane k+2 (clamped to the column's last plane, so it is
// unconditional and its registers are never merged with old values: a merge
// would wait for the load that is meant to stay in flight).  Interior columns
// publish up to plane 17 (read back by the last reverse predictor).
template <typename T, bool kI, class Src>
__device__ __forceinline__ void adj_col_publish(AdjCol<T, kI>& c, const Src& src, int k, const Gas<T>& gas,
                                                SmemF<T>& sm) {
#pragma unroll
  for (int q = 0; q < 5; ++q) sm.P[pslot(k)][q][pidx(c.cx, c.cy)] = c.Wp[q];
  cons_to_prim(c.Un, gas, c.Wp);
  asm volatile("" ::: "memory");
  load_cons(src, c.col, k + 2 <= c.zhi ? k + 2 : c.zhi, c.Un);
}

// F2: half-step states of plane k and the z-face (k-1 | k) VJP (kFwd); then
// the reverse Hancock predictor of the state cell at plane k-1 (kRev).  A
// halo column's two parts run on different waves, each with its own AdjCol
// of the column (the reverse part needs nothing the forward part keeps in
// registers: its face cotangent comes through LDS).
template <typename T, bool kI, bool kFwd = true, bool kRev = true>
__device__ __forceinline__ void adj_col_states(AdjCol<T, kI>& c, int k, const T* __restrict__ go, const Gas<T>& gas,
                                               bool fo, int ws, SmemF<T>& sm) {
  const int cx = c.cx, cy = c.cy;
  const int sk = pslot(k), sj = pslot(k - 1), si = pslot(k - 2);
  T gLz[5] = {T(0), T(0), T(0), T(0), T(0)};   // cotangent of the z+ face state of plane k-1
  T gRzn[5] = {T(0), T(0), T(0), T(0), T(0)};  // cotangent of the z- face state of plane k
  if (kFwd && k <= 16 && in_state_plane(cx, cy, k)) {
    T Wc[5], Wn[3][2][5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      Wc[q] = sm.P[sk][q][pidx(cx, cy)];
      Wn[0][0][q] = sm.P[sk][q][pidx(cx - 1, cy)];
      Wn[0][1][q] = sm.P[sk][q][pidx(cx + 1, cy)];
      Wn[1][0][q] = sm.P[sk][q][pidx(cx, cy - 1)];
      Wn[1][1][q] = sm.P[sk][q][pidx(cx, cy + 1)];
      Wn[2][0][q] = sm.P[sj][q][pidx(cx, cy)];
      Wn[2][1][q] = c.Wp[q];
    }
    T Ut[3][2][5];
    hancock_states(Wc, Wn, gas, fo, Ut);
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      sm.S[0][q][sidx(cx, cy)] = Ut[0][1][q];
      sm.S[1][q][sidx(cx, cy)] = Ut[1][1][q];
      if (kI) {
        c.Ux[q] = Ut[0][0][q];
        c.Uy[q] = Ut[1][0][q];
      }
    }
    if (!kI && (c.xface16 || c.yface16)) {
      const int slot = last_slot(c.xface16, cx, cy);
#pragma unroll
      for (int q = 0; q < 5; ++q) sm.H[q][slot] = c.xface16 ? Ut[0][0][q] : Ut[1][0][q];
    }
    if (kI) {
      if (k >= 0) {
        T gF[5];
#pragma unroll
        for (int q = 0; q < 5; ++q) gF[q] = gas.dtdx * (gout(go, q, cx, cy, k) - gout(go, q, cx, cy, k - 1));
        hllc_flux_vjp<2>(c.Uz, Ut[2][0], gas, ws, gF, gLz, gRzn);
      }
#pragma unroll
      for (int q = 0; q < 5; ++q) c.Uz[q] = Ut[2][1][q];
    }
  }

  const int j = k - 1;
  if (kRev && j >= -1 && in_state_plane(cx, cy, j)) {
    const bool u0 = face_used(cx, cy, j, 0), u1 = face_used(cx, cy, j, 1), u2 = face_used(cx, cy, j, 2);
    const bool u3 = face_used(cx, cy, j, 3), u4 = face_used(cx, cy, j, 4), u5 = face_used(cx, cy, j, 5);
    T Wj[5], gWc[5];
    const int slot = last_slot(c.xface16, cx, cy);
#pragma unroll
    for (int q = 0; q < 5; ++q) Wj[q] = sm.P[sj][q][pidx(cx, cy)];
    hancock_states_vjp_stream(
        Wj, gas, fo,
        [&](int d, int side, T W[5]) {
          if (d == 2) {
#pragma unroll
            for (int q = 0; q < 5; ++q) W[q] = sm.P[side == 0 ? si : sk][q][pidx(cx, cy)];
          } else {
            const int x = d == 0 ? cx + (side ? 1 : -1) : cx, y = d == 1 ? cy + (side ? 1 : -1) : cy;
#pragma unroll
            for (int q = 0; q < 5; ++q) W[q] = sm.P[sj][q][pidx(x, y)];
          }
        },
        [&](int d, int side, T G[5]) {
          const int f = 2 * d + side;
          const bool used = f == 0 ? u0 : f == 1 ? u1 : f == 2 ? u2 : f == 3 ? u3 : f == 4 ? u4 : u5;
#pragma unroll
          for (int q = 0; q < 5; ++q) {
            T v;
            if (f == 0) v = kI ? c.gRx[q] : sm.GR[q][slot];
            else if (f == 1) v = sm.GL[0][q][sidx(cx, cy)];
            else if (f == 2) v = kI ? c.gRy[q] : sm.GR[q][slot];
            else if (f == 3) v = sm.GL[1][q][sidx(cx, cy)];
            else if (f == 4) v = c.gRz[q];
            else v = gLz[q];
            G[q] = used ? v : T(0);
          }
        },
        [&](int d, int side, const T G[5]) {
          if (d == 2) {
#pragma unroll
            for (int q = 0; q < 5; ++q) {
              if (side == 0) c.A0[q] = c.A0[q] + G[q];
              else c.A2[q] = c.A2[q] + G[q];
            }
          } else {
#pragma unroll
            for (int q = 0; q < 5; ++q) sm.O[2 * d + side][q][sidx(cx, cy)] = G[q];
          }
        },
        gWc);
#pragma unroll
    for (int q = 0; q < 5; ++q) c.A1[q] = c.A1[q] + gWc[q];
  }
  if (kI) {
#pragma unroll
    for (int q = 0; q < 5; ++q) c.gRz[q] = gRzn[q];
  }
}

// F3a: the x and y face VJPs an interior column solves at plane k (its x-
// face and y- face).
template <typename T, bool kI>
__device__ __forceinline__ void adj_col_faces(AdjCol<T, kI>& c, int k, const T* __restrict__ go, const Gas<T>& gas,
                                              int ws, SmemF<T>& sm) {
  if (k < 0 || k > 15) return;
  const int cx = c.cx, cy = c.cy;
  if (kI) {
    {
      T L[5], gF[5], gL[5] = {T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        L[q] = sm.S[0][q][sidx(cx - 1, cy)];
        gF[q] = gas.dtdx * (gout(go, q, cx, cy, k) - gout(go, q, cx - 1, cy, k));
        c.gRx[q] = T(0);
      }
      hllc_flux_vjp<0>(L, c.Ux, gas, ws, gF, gL, c.gRx);
#pragma unroll
      for (int q = 0; q < 5; ++q) sm.GL[0][q][sidx(cx - 1, cy)] = gL[q];
    }
    {
      T L[5], gF[5], gL[5] = {T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        L[q] = sm.S[1][q][sidx(cx, cy - 1)];
        gF[q] = gas.dtdx * (gout(go, q, cx, cy, k) - gout(go, q, cx, cy - 1, k));
        c.gRy[q] = T(0);
      }
      hllc_flux_vjp<1>(L, c.Uy, gas, ws, gF, gL, c.gRy);
#pragma unroll
      for (int q = 0; q < 5; ++q) sm.GL[1][q][sidx(cx, cy - 1)] = gL[q];
    }
  }
}

// The 32 last faces of plane k (x = 16 for lanes 0..15 at y = lane, y = 16
// for lanes 16..31 at x = lane - 16), solved by a wave without halo columns
// in one pass: a y face is solved in the x-normal frame with its states and
// cotangents rotated (m_y, m_z, m_x) -> (m_x, m_y, m_z), the same arithmetic
// on the same values as the y-normal solver, and the results rotated back.
// The high-side states come from the halo columns (H); the cotangent of the
// low-side state goes to GL, that of the high-side state to GR.
template <typename T>
__device__ __forceinline__ void adj_last_faces(int lane, int k, const T* __restrict__ go, const Gas<T>& gas, int ws,
                                               SmemF<T>& sm) {
  if (k < 0 || k > 15 || lane >= 32) return;
  const bool yf = lane >= 16;
  const int i = lane & 15;
  const int hx = yf ? i : 16, hy = yf ? 16 : i;    // the halo cell on the high side
  const int lx = yf ? i : 15, ly = yf ? 15 : i;    // the interior cell on the low side
  const T* Sb = yf ? &sm.S[1][0][sidx(lx, ly)] : &sm.S[0][0][sidx(lx, ly)];
  T L[5], R[5], gF[5];
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    L[q] = Sb[q * kSW * kSW];
    R[q] = sm.H[q][lane];
    gF[q] = gas.dtdx * (gout(go, q, hx, hy, k) - gout(go, q, lx, ly, k));
  }
  auto rot = [&](const T a[5], T r[5]) {  // axis frame -> x-normal frame of this face
    r[0] = a[0];
    r[1] = yf ? a[2] : a[1];
    r[2] = yf ? a[3] : a[2];
    r[3] = yf ? a[1] : a[3];
    r[4] = a[4];
  };
  auto unrot = [&](const T r[5], T a[5]) {
    a[0] = r[0];
    a[1] = yf ? r[3] : r[1];
    a[2] = yf ? r[1] : r[2];
    a[3] = yf ? r[2] : r[3];
    a[4] = r[4];
  };
  T Lr[5], Rr[5], gFr[5];
  rot(L, Lr);
  rot(R, Rr);
  rot(gF, gFr);
  T gLr[5] = {T(0), T(0), T(0), T(0), T(0)}, gRr[5] = {T(0), T(0), T(0), T(0), T(0)};
  hllc_flux_vjp<0>(Lr, Rr, gas, ws, gFr, gLr, gRr);
  T gL[5], gR[5];
  unrot(gLr, gL);
  unrot(gRr, gR);
  T* Gb = yf ? &sm.GL[1][0][sidx(lx, ly)] : &sm.GL[0][0][sidx(lx, ly)];
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    Gb[q * kSW * kSW] = gL[q];
    sm.GR[q][lane] = gR[q];
  }
}

// In-plane gather at plane j into g: cell (x, y) receives the x+ contribution
// of (x-1, y), the x- contribution of (x+1, y), and likewise in y.
template <typename T>
__device__ __forceinline__ void adj_gather_plane(int x, int y, int j, const SmemF<T>& sm, T g[5]) {
  const bool l = in_state_plane(x - 1, y, j), r = in_state_plane(x + 1, y, j);
  const bool d = in_state_plane(x, y - 1, j), u = in_state_plane(x, y + 1, j);
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    T s = g[q];
    if (l) s = s + sm.O[1][q][sidx(x - 1, y)];
    if (r) s = s + sm.O[0][q][sidx(x + 1, y)];
    if (d) s = s + sm.O[3][q][sidx(x, y - 1)];
    if (u) s = s + sm.O[2][q][sidx(x, y + 1)];
    g[q] = s;
  }
}

// Finalize plane k-2 of the column (complete once the reverse predictor of
// plane k-1 has run).  A column whose planes another wave publishes calls this
// right after its reverse part, before the barrier that lets the publisher
// overwrite that plane's LDS slot with plane k+1.
template <typename T, bool kI, class Sink>
__device__ __forceinline__ void adj_col_finalize_prev(const AdjCol<T, kI>& c, int k, const T* __restrict__ go,
                                                      const Gas<T>& gas, const SmemF<T>& sm, const Sink& sink) {
  if (k - 2 >= c.zlo && k - 2 <= c.zhi) finalize_cell_lds(sm, c.cx, c.cy, k - 2, c.A0, go, gas, sink);
}

// F3b: in-plane gather of plane k-1 into the column; finalize the planes that
// are complete (k-2 unless kPrevDone; after the last plane also k-1 and k);
// advance the rings.
template <typename T, bool kI, class Src, class Sink, bool kPrevDone = false>
__device__ __forceinline__ void adj_col_finish(AdjCol<T, kI>& c, const Src& src, int k, const T* __restrict__ go,
                                               const Gas<T>& gas, const SmemF<T>& sm, const Sink& sink) {
  const int j = k - 1;
  if (j >= c.zlo && j <= c.zhi) adj_gather_plane(c.cx, c.cy, j, sm, c.A1);
  if (!kPrevDone) adj_col_finalize_prev(c, k, go, gas, sm, sink);
  if (k == 17) {
    if (16 <= c.zhi) finalize_cell_lds(sm, c.cx, c.cy, 16, c.A1, go, gas, sink);
    if (17 <= c.zhi) finalize_cell_lds(sm, c.cx, c.cy, 17, c.A2, go, gas, sink);
  }
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    c.A0[q] = c.A1[q];
    c.A1[q] = c.A2[q];
    c.A2[q] = T(0);
  }
}

template <typename T, class Src, class Sink>
__device__ __forceinline__ void adjoint_fused(const Src& src, const T* __restrict__ go, const Gas<T>& gas,
                                              int first_order, int ws, SmemF<T>& sm, const Sink& sink) {
  const int tid = threadIdx.x;
  const bool halo = tid < 64;                  // wave 0: halo columns, forward part
  const bool hrev = (tid >> 6) == 1;           // wave 1: halo columns, reverse part and finish
  const bool last = (tid >> 6) == 2;           // wave 2: the 32 last faces
  const bool outer = (tid >> 6) == 3;          // wave 3: finishes the 2-deep and edge columns
  const bool fo = first_order != 0;
  // FP32 (two workgroups per CU, so two waves per SIMD): the two halo waves
  // take issue priority over the other workgroup's waves on their SIMDs
  // (measured: FP32 384^3 adjoint step -2%; other assignments neutral or worse)
  if constexpr (sizeof(T) == 4) {
    // s_setprio ignores the exec mask: branch on a wave-uniform value
    if (__builtin_amdgcn_readfirstlane(tid >> 6) <= 1) __builtin_amdgcn_s_setprio(1);
  }
  // halo role of wave 0: side 0..3 = x-, x+, y-, y+; the column two cells out;
  // lanes 0..3 also one of the 4 edge columns; lane l of wave 1 takes the
  // reverse part of the halo column of lane l
  const int side = (tid & 63) >> 4, kk = tid & 15;
  const int hx = side == 0 ? -1 : side == 1 ? 16 : kk, hy = side == 2 ? -1 : side == 3 ? 16 : kk;
  const int ox = side == 0 ? -2 : side == 1 ? 17 : kk, oy = side == 2 ? -2 : side == 3 ? 17 : kk;
  const int ex = (tid & 1) ? 16 : -1, ey = (tid & 2) ? 16 : -1;
  const bool has_edge = halo && tid < 4;
  // lane l of wave 3 finishes the 2-deep (and edge) column of halo lane l
  const int ol = tid & 63, oside = ol >> 4, okk = ol & 15;
  const int fox = oside == 0 ? -2 : oside == 1 ? 17 : okk, foy = oside == 2 ? -2 : oside == 3 ? 17 : okk;
  const int fex = (ol & 1) ? 16 : -1, fey = (ol & 2) ? 16 : -1;
  const bool fedge = outer && ol < 4;
  const int64_t col_out = halo ? src.col(ox, oy) : 0;
  // lanes without an edge column re-read their 2-deep column (unconditional loads)
  const int64_t col_edge = halo ? src.col(has_edge ? ex : ox, has_edge ? ey : oy) : 0;

  AdjCol<T, true> ci;
  AdjCol<T, false> ch;  // wave 0: forward part; wave 1: reverse part of the same halo column
  adj_col_init(ci, src, tid & 15, tid >> 4, gas, sm);
  T Uo[5], Ue[5];  // halo role: 2-deep and edge column, plane k (in flight)
  if (halo || hrev) adj_col_init(ch, src, hx, hy, gas, sm);
  if (halo) {
    load_cons(src, col_out, 0, Uo);
    load_cons(src, col_edge, 0, Ue);
  }

  for (int k = -1; k <= 17; ++k) {
    const int sk = pslot(k);
    adj_col_publish(ci, src, k, gas, sm);
    if (k <= 16) {
      if (halo) {
        adj_col_publish(ch, src, k, gas, sm);
        if (k >= 0 && k <= 15) {
          T Wo[5], We[5];
          cons_to_prim(Uo, gas, Wo);
          cons_to_prim(Ue, gas, We);
          asm volatile("" ::: "memory");
          const int kn = k + 1 > 15 ? 15 : k + 1;
          load_cons(src, col_out, kn, Uo);
          load_cons(src, col_edge, kn, Ue);
#pragma unroll
          for (int q = 0; q < 5; ++q) sm.P[sk][q][pidx(ox, oy)] = Wo[q];
          if (has_edge) {
#pragma unroll
            for (int q = 0; q < 5; ++q) sm.P[sk][q][pidx(ex, ey)] = We[q];
          }
        }
      }
    }
    __syncthreads();
    adj_col_states(ci, k, go, gas, fo, ws, sm);
    if (halo) adj_col_states<T, false, true, false>(ch, k, go, gas, fo, ws, sm);
    if (hrev) {
      adj_col_states<T, false, false, true>(ch, k, go, gas, fo, ws, sm);
      // wave 0 publishes this column: plane k-2's slot is rewritten after the barrier
      adj_col_finalize_prev(ch, k, go, gas, sm, sink);
    }
    __syncthreads();
    adj_col_faces(ci, k, go, gas, ws, sm);
    if (last) adj_last_faces(tid & 63, k, go, gas, ws, sm);
    adj_col_finish(ci, src, k, go, gas, sm, sink);
    if (hrev) adj_col_finish<T, false, Src, Sink, true>(ch, src, k, go, gas, sm, sink);
    if (outer) {
      const int j = k - 1;
      if (j >= 0 && j <= 15) {
        // the 2-deep and edge columns get only in-plane contributions
        T g[5] = {T(0), T(0), T(0), T(0), T(0)};
        adj_gather_plane(fox, foy, j, sm, g);
        finalize_cell_lds(sm, fox, foy, j, g, go, gas, sink);
        if (fedge) {
          T e[5] = {T(0), T(0), T(0), T(0), T(0)};
          adj_gather_plane(fex, fey, j, sm, e);
          finalize_cell_lds(sm, fex, fey, j, e, go, gas, sink);
        }
      }
    }
    // next writes: P slot k+1 held plane k-2, read in this iteration's
    // states phase by every wave and in its finish phase only by the thread
    // that publishes the column (program order orders the two; the halo
    // columns, published by wave 0, are finalized by wave 1 in the states
    // phase); S / O / H in the next states phase (after its first barrier);
    // GL / GR in the next faces phase (after the barrier that follows their
    // reads)
  }
}

// ------------------------------------------------------- split kernels ----
// The same adjoint as two z-marches per group with a face workspace between
// them, each small enough in LDS (and registers) for two workgroups per CU:
//   faces: recompute the half-step states of plane k, take the HLLC VJP of
//      every face and store the cotangents of its two face states;
//   cells: reverse the Hancock predictor of every state cell from its six
//      face cotangents, gather in-plane (LDS) and along z (register ring),
//      and finish as the fused kernel does.
// Workspace per group: for each direction d, side s (0: the low cell's high
// face state, 1: the high cell's low face state), field q and face f,
// element ((d * 2 + s) * 5 + q) * kFaces + f.
constexpr int kFaces = 17 * 16 * 16;  // faces per direction per group
constexpr int64_t kFaceWs = 3 * 2 * 5 * int64_t(kFaces);
__device__ __forceinline__ int xface_id(int i, int y, int k) { return (k * 16 + y) * 17 + i; }    // i in [0, 16]
__device__ __forceinline__ int yface_id(int x, int j, int k) { return (k * 17 + j) * 16 + x; }    // j in [0, 16]
__device__ __forceinline__ int zface_id(int x, int y, int kz) { return (kz * 16 + y) * 16 + x; }  // kz in [0, 16]
__device__ __forceinline__ int64_t ws_at(int d, int side, int q, int f) {
  return (int64_t(d * 2 + side) * 5 + q) * kFaces + f;
}

template <typename T>
struct SmemFaces {
  T P[5][kPW * kPW];     // primitive plane k
  T S[2][5][kSW * kSW];  // x+ and y+ half-step states of plane k
};
template <typename T>
struct SmemCells {
  T P[5][kPW * kPW];     // primitive plane k
  T O[4][5][kSW * kSW];  // in-plane neighbour contributions of plane k (x-, x+, y-, y+)
};

template <typename T, bool kInterior>
struct SplitCol {
  static constexpr int zlo = kInterior ? -2 : -1, zhi = kInterior ? 17 : 16;
  int cx, cy;
  bool xface16, yface16;
  int64_t col;
  T Wm[5], Wc[5], Wp[5];  // primitive states at planes k-1, k, k+1
  T Ux[5], Uy[5], Uz[5];  // faces: own x-, y- face states of plane k; z+ state of plane k-1
  T A0[5], A1[5], A2[5];  // cells: input cotangents of the column at planes k-1, k, k+1
};

template <typename T, bool kI, class Src>
__device__ __forceinline__ void split_col_init(SplitCol<T, kI>& c, const Src& src, int cx, int cy, const Gas<T>& gas) {
  c.cx = cx;
  c.cy = cy;
  c.xface16 = !kI && cx == 16;
  c.yface16 = !kI && cy == 16;
  c.col = src.col(cx, cy);
  if (kI) load_prim(src, c.col, -2, gas, c.Wm);
  load_prim(src, c.col, -1, gas, c.Wc);
#pragma unroll
  for (int q = 0; q < 5; ++q) c.A0[q] = c.A1[q] = c.A2[q] = T(0);
}

template <typename T, bool kI, class Src>
__device__ __forceinline__ void split_col_publish(SplitCol<T, kI>& c, const Src& src, int k, const Gas<T>& gas,
                                                  T (*P)[kPW * kPW]) {
  if (k + 1 <= c.zhi) load_prim(src, c.col, k + 1, gas, c.Wp);
#pragma unroll
  for (int q = 0; q < 5; ++q) P[q][pidx(c.cx, c.cy)] = c.Wc[q];
}

template <typename T, bool kI>
__device__ __forceinline__ void split_col_shift(SplitCol<T, kI>& c) {
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    c.Wm[q] = c.Wc[q];
    c.Wc[q] = c.Wp[q];
  }
}

// The 2-deep and edge columns of the halo role: publish plane k (0..15).
template <typename T, class Src>
__device__ __forceinline__ void publish_outer(const Src& src, int k, int64_t col_out, int ox, int oy, bool has_edge,
                                              int64_t col_edge, int ex, int ey, const Gas<T>& gas,
                                              T (*P)[kPW * kPW]) {
  T Wo[5];
  load_prim(src, col_out, k, gas, Wo);
#pragma unroll
  for (int q = 0; q < 5; ++q) P[q][pidx(ox, oy)] = Wo[q];
  if (has_edge) {
    load_prim(src, col_edge, k, gas, Wo);
#pragma unroll
    for (int q = 0; q < 5; ++q) P[q][pidx(ex, ey)] = Wo[q];
  }
}

// faces kernel, states phase: half-step states of plane k; z-face (k-1 | k).
template <typename T, bool kI>
__device__ __forceinline__ void faces_col_states(SplitCol<T, kI>& c, int k, const T* __restrict__ go,
                                                 T* __restrict__ ws, const Gas<T>& gas, bool fo, int wsp,
                                                 SmemFaces<T>& sm) {
  const int cx = c.cx, cy = c.cy;
  if (k > 16 || !in_state_plane(cx, cy, k)) return;
  T Wn[3][2][5];
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    Wn[0][0][q] = sm.P[q][pidx(cx - 1, cy)];
    Wn[0][1][q] = sm.P[q][pidx(cx + 1, cy)];
    Wn[1][0][q] = sm.P[q][pidx(cx, cy - 1)];
    Wn[1][1][q] = sm.P[q][pidx(cx, cy + 1)];
    Wn[2][0][q] = c.Wm[q];
    Wn[2][1][q] = c.Wp[q];
  }
  T Ut[3][2][5];
  hancock_states(c.Wc, Wn, gas, fo, Ut);
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    sm.S[0][q][sidx(cx, cy)] = Ut[0][1][q];
    sm.S[1][q][sidx(cx, cy)] = Ut[1][1][q];
    if (kI) {
      c.Ux[q] = Ut[0][0][q];
      c.Uy[q] = Ut[1][0][q];
    } else {
      c.Ux[q] = c.xface16 ? Ut[0][0][q] : Ut[1][0][q];
    }
  }
  if (kI) {
    if (k >= 0) {
      T gF[5], gL[5] = {T(0), T(0), T(0), T(0), T(0)}, gR[5] = {T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int q = 0; q < 5; ++q) gF[q] = gas.dtdx * (gout(go, q, cx, cy, k) - gout(go, q, cx, cy, k - 1));
      hllc_flux_vjp<2>(c.Uz, Ut[2][0], gas, wsp, gF, gL, gR);
      const int f = zface_id(cx, cy, k);
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        ws[ws_at(2, 0, q, f)] = gL[q];
        ws[ws_at(2, 1, q, f)] = gR[q];
      }
    }
#pragma unroll
    for (int q = 0; q < 5; ++q) c.Uz[q] = Ut[2][1][q];
  }
}

// faces kernel, faces phase: the x / y faces the column solves at plane k.
template <typename T, bool kI>
__device__ __forceinline__ void faces_col_faces(SplitCol<T, kI>& c, int k, const T* __restrict__ go,
                                                T* __restrict__ ws, const Gas<T>& gas, int wsp, SmemFaces<T>& sm) {
  if (k < 0 || k > 15) return;
  const int cx = c.cx, cy = c.cy;
  if (kI) {
    {
      T L[5], gF[5], gL[5] = {T(0), T(0), T(0), T(0), T(0)}, gR[5] = {T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        L[q] = sm.S[0][q][sidx(cx - 1, cy)];
        gF[q] = gas.dtdx * (gout(go, q, cx, cy, k) - gout(go, q, cx - 1, cy, k));
      }
      hllc_flux_vjp<0>(L, c.Ux, gas, wsp, gF, gL, gR);
      const int f = xface_id(cx, cy, k);
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        ws[ws_at(0, 0, q, f)] = gL[q];
        ws[ws_at(0, 1, q, f)] = gR[q];
      }
    }
    {
      T L[5], gF[5], gL[5] = {T(0), T(0), T(0), T(0), T(0)}, gR[5] = {T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        L[q] = sm.S[1][q][sidx(cx, cy - 1)];
        gF[q] = gas.dtdx * (gout(go, q, cx, cy, k) - gout(go, q, cx, cy - 1, k));
      }
      hllc_flux_vjp<1>(L, c.Uy, gas, wsp, gF, gL, gR);
      const int f = yface_id(cx, cy, k);
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        ws[ws_at(1, 0, q, f)] = gL[q];
        ws[ws_at(1, 1, q, f)] = gR[q];
      }
    }
  } else if (c.xface16 || c.yface16) {
    // one pass for both halo faces: a y face in the x-normal frame with
    // rotated states and cotangents (the y-normal solver's arithmetic)
    const bool yf = c.yface16;
    const int lx = yf ? cx : cx - 1, ly = yf ? cy - 1 : cy;
    const T* Sb = yf ? &sm.S[1][0][sidx(lx, ly)] : &sm.S[0][0][sidx(lx, ly)];
    T L[5], gF[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      L[q] = Sb[q * kSW * kSW];
      gF[q] = gas.dtdx * (gout(go, q, cx, cy, k) - gout(go, q, lx, ly, k));
    }
    auto rot = [&](const T a[5], T r[5]) {
      r[0] = a[0];
      r[1] = yf ? a[2] : a[1];
      r[2] = yf ? a[3] : a[2];
      r[3] = yf ? a[1] : a[3];
      r[4] = a[4];
    };
    auto unrot = [&](const T r[5], T a[5]) {
      a[0] = r[0];
      a[1] = yf ? r[3] : r[1];
      a[2] = yf ? r[1] : r[2];
      a[3] = yf ? r[2] : r[3];
      a[4] = r[4];
    };
    T Lr[5], Rr[5], gFr[5];
    rot(L, Lr);
    rot(c.Ux, Rr);
    rot(gF, gFr);
    T gLr[5] = {T(0), T(0), T(0), T(0), T(0)}, gRr[5] = {T(0), T(0), T(0), T(0), T(0)};
    hllc_flux_vjp<0>(Lr, Rr, gas, wsp, gFr, gLr, gRr);
    T gL[5], gR[5];
    unrot(gLr, gL);
    unrot(gRr, gR);
    const int d = yf ? 1 : 0;
    const int f = yf ? yface_id(cx, cy, k) : xface_id(cx, cy, k);
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      ws[ws_at(d, 0, q, f)] = gL[q];
      ws[ws_at(d, 1, q, f)] = gR[q];
    }
  }
}

template <typename T, class Src>
__device__ __forceinline__ void adjoint_faces_pass(const Src& src, const T* __restrict__ go, T* __restrict__ ws,
                                                   const Gas<T>& gas, int first_order, int wsp, SmemFaces<T>& sm) {
  const int tid = threadIdx.x;
  const bool halo = tid < 64;
  const bool fo = first_order != 0;
  const int side = tid >> 4, kk = tid & 15;
  const int hx = side == 0 ? -1 : side == 1 ? 16 : kk, hy = side == 2 ? -1 : side == 3 ? 16 : kk;
  const int ox = side == 0 ? -2 : side == 1 ? 17 : kk, oy = side == 2 ? -2 : side == 3 ? 17 : kk;
  const int ex = (tid & 1) ? 16 : -1, ey = (tid & 2) ? 16 : -1;
  const bool has_edge = halo && tid < 4;
  const int64_t col_out = halo ? src.col(ox, oy) : 0;
  const int64_t col_edge = has_edge ? src.col(ex, ey) : 0;
  SplitCol<T, true> ci;
  SplitCol<T, false> ch;
  split_col_init(ci, src, tid & 15, tid >> 4, gas);
  if (halo) split_col_init(ch, src, hx, hy, gas);
  for (int k = -1; k <= 16; ++k) {
    split_col_publish(ci, src, k, gas, sm.P);
    if (halo) {
      split_col_publish(ch, src, k, gas, sm.P);
      if (k >= 0 && k <= 15) publish_outer(src, k, col_out, ox, oy, has_edge, col_edge, ex, ey, gas, sm.P);
    }
    __syncthreads();
    faces_col_states(ci, k, go, ws, gas, fo, wsp, sm);
    if (halo) faces_col_states(ch, k, go, ws, gas, fo, wsp, sm);
    __syncthreads();
    faces_col_faces(ci, k, go, ws, gas, wsp, sm);
    if (halo) faces_col_faces(ch, k, go, ws, gas, wsp, sm);
    split_col_shift(ci);
    if (halo) split_col_shift(ch);
  }
}

// cells kernel, states phase: reverse the Hancock predictor of the column's
// state cell at plane k from its six face cotangents.
template <typename T, bool kI>
__device__ __forceinline__ void cells_col_vjp(SplitCol<T, kI>& c, int k, const T* __restrict__ ws,
                                              const Gas<T>& gas, bool fo, SmemCells<T>& sm) {
  const int cx = c.cx, cy = c.cy;
  if (k > 16 || !in_state_plane(cx, cy, k)) return;
  const bool u0 = face_used(cx, cy, k, 0), u1 = face_used(cx, cy, k, 1), u2 = face_used(cx, cy, k, 2);
  const bool u3 = face_used(cx, cy, k, 3), u4 = face_used(cx, cy, k, 4), u5 = face_used(cx, cy, k, 5);
  T gWc[5];
  hancock_states_vjp_stream(
      c.Wc, gas, fo,
      [&](int d, int s, T W[5]) {
        if (d == 2) {
#pragma unroll
          for (int q = 0; q < 5; ++q) W[q] = s == 0 ? c.Wm[q] : c.Wp[q];
        } else {
          const int x = d == 0 ? cx + (s ? 1 : -1) : cx, y = d == 1 ? cy + (s ? 1 : -1) : cy;
#pragma unroll
          for (int q = 0; q < 5; ++q) W[q] = sm.P[q][pidx(x, y)];
        }
      },
      [&](int d, int s, T G[5]) {
        const int f = 2 * d + s;
        const bool used = f == 0 ? u0 : f == 1 ? u1 : f == 2 ? u2 : f == 3 ? u3 : f == 4 ? u4 : u5;
        // the low face of the cell holds the cell's state as the high side (1);
        // the high face as the low side (0)
        const int id = !used ? 0 : d == 0 ? xface_id(cx + s, cy, k) : d == 1 ? yface_id(cx, cy + s, k)
                                                          : zface_id(cx, cy, k + s);
#pragma unroll
        for (int q = 0; q < 5; ++q) G[q] = used ? ws[ws_at(d, 1 - s, q, id)] : T(0);
      },
      [&](int d, int s, const T G[5]) {
        if (d == 2) {
#pragma unroll
          for (int q = 0; q < 5; ++q) {
            if (s == 0) c.A0[q] = c.A0[q] + G[q];
            else c.A2[q] = c.A2[q] + G[q];
          }
        } else {
#pragma unroll
          for (int q = 0; q < 5; ++q) sm.O[2 * d + s][q][sidx(cx, cy)] = G[q];
        }
      },
      gWc);
#pragma unroll
  for (int q = 0; q < 5; ++q) c.A1[q] = c.A1[q] + gWc[q];
}

template <typename T>
__device__ __forceinline__ void cells_gather_plane(int x, int y, int j, const SmemCells<T>& sm, T g[5]) {
  const bool l = in_state_plane(x - 1, y, j), r = in_state_plane(x + 1, y, j);
  const bool d = in_state_plane(x, y - 1, j), u = in_state_plane(x, y + 1, j);
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    T s = g[q];
    if (l) s = s + sm.O[1][q][sidx(x - 1, y)];
    if (r) s = s + sm.O[0][q][sidx(x + 1, y)];
    if (d) s = s + sm.O[3][q][sidx(x, y - 1)];
    if (u) s = s + sm.O[2][q][sidx(x, y + 1)];
    g[q] = s;
  }
}

// cells kernel, finish phase: in-plane gather of plane k; plane k-1 is complete.
template <typename T, bool kI, class Src, class Sink>
__device__ __forceinline__ void cells_col_finish(SplitCol<T, kI>& c, const Src& src, int k, const T* __restrict__ go,
                                                 const Gas<T>& gas, const SmemCells<T>& sm, const Sink& sink) {
  if (k <= 16 && k >= c.zlo && k <= c.zhi) cells_gather_plane(c.cx, c.cy, k, sm, c.A1);
  if (k - 1 >= c.zlo && k - 1 <= c.zhi) finalize_cell(src, c.col, c.cx, c.cy, k - 1, c.A0, go, gas, sink);
  if (k == 17 && 17 <= c.zhi) finalize_cell(src, c.col, c.cx, c.cy, 17, c.A1, go, gas, sink);
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    c.A0[q] = c.A1[q];
    c.A1[q] = c.A2[q];
    c.A2[q] = T(0);
  }
}

template <typename T, class Src, class Sink>
__device__ __forceinline__ void adjoint_cells_pass(const Src& src, const T* __restrict__ go, const T* __restrict__ ws,
                                                   const Gas<T>& gas, int first_order, SmemCells<T>& sm,
                                                   const Sink& sink) {
  const int tid = threadIdx.x;
  const bool halo = tid < 64;
  const bool fo = first_order != 0;
  const int side = tid >> 4, kk = tid & 15;
  const int hx = side == 0 ? -1 : side == 1 ? 16 : kk, hy = side == 2 ? -1 : side == 3 ? 16 : kk;
  const int ox = side == 0 ? -2 : side == 1 ? 17 : kk, oy = side == 2 ? -2 : side == 3 ? 17 : kk;
  const int ex = (tid & 1) ? 16 : -1, ey = (tid & 2) ? 16 : -1;
  const bool has_edge = halo && tid < 4;
  const int64_t col_out = halo ? src.col(ox, oy) : 0;
  const int64_t col_edge = has_edge ? src.col(ex, ey) : 0;
  SplitCol<T, true> ci;
  SplitCol<T, false> ch;
  split_col_init(ci, src, tid & 15, tid >> 4, gas);
  if (halo) split_col_init(ch, src, hx, hy, gas);
  for (int k = -1; k <= 17; ++k) {
    if (k <= 16) {
      split_col_publish(ci, src, k, gas, sm.P);
      if (halo) {
        split_col_publish(ch, src, k, gas, sm.P);
        if (k >= 0 && k <= 15) publish_outer(src, k, col_out, ox, oy, has_edge, col_edge, ex, ey, gas, sm.P);
      }
    }
    __syncthreads();
    cells_col_vjp(ci, k, ws, gas, fo, sm);
    if (halo) cells_col_vjp(ch, k, ws, gas, fo, sm);
    __syncthreads();
    cells_col_finish(ci, src, k, go, gas, sm, sink);
    if (halo) {
      cells_col_finish(ch, src, k, go, gas, sm, sink);
      if (k >= 0 && k <= 15) {
        // the 2-deep and edge columns get only in-plane contributions
        T g[5] = {T(0), T(0), T(0), T(0), T(0)};
        cells_gather_plane(ox, oy, k, sm, g);
        finalize_cell(src, col_out, ox, oy, k, g, go, gas, sink);
        if (has_edge) {
          T e[5] = {T(0), T(0), T(0), T(0), T(0)};
          cells_gather_plane(ex, ey, k, sm, e);
          finalize_cell(src, col_edge, ex, ey, k, e, go, gas, sink);
        }
      }
    }
    split_col_shift(ci);
    if (halo) split_col_shift(ch);
  }
}

// ------------------------------------------------------------- kernels ----

template <typename T>
__device__ __forceinline__ void set_dt_adj(Gas<T>& gas, const double* dt_dev, double dx) {
  if (dt_dev != nullptr) {
    const double dt = *dt_dev;
    gas.dtdx = T(dt / dx);
    gas.half_dtdx = T(0.5 * (dt / dx));
  }
}

// Group of this workgroup in a level adjoint launch (grid rounded up to a
// multiple of 8): the XCD-blocked column-tile order of the level step, so
// that each XCD runs a contiguous range of neighbouring groups and finds
// their shared ghost cells in its L2; -1 for a padding workgroup.
__device__ __forceinline__ int64_t adj_level_group(const LevelGeom& geo) {
  const int64_t G = int64_t(geo.ngx) * geo.ngy * geo.ngz;
  const int64_t w = xcd_group(blockIdx.x, G);
  return w < G ? tile_group(w, geo) : -1;
}

template <typename T>
__global__ __launch_bounds__(kAdjThreads) __attribute__((amdgpu_waves_per_eu(AdjWaves<T>::value, AdjWaves<T>::value))) void adj_fused_padded(const T* __restrict__ Upad, const T* __restrict__ gout_,
                                                             T* __restrict__ gpad, int gh, Gas<T> gas, int first_order,
                                                             int ws) {
  __shared__ SmemF<T> sm;
  const int P = 16 + 2 * gh;
  const int64_t g = blockIdx.x;
  const int64_t P3 = int64_t(P) * P * P;
  PaddedSource<T> src{Upad + g * 5 * P3, P, gh};
  PadSink<T> sink{gpad + g * 5 * P3, P, gh};
  // the second-order scheme gets its own inlined copy (limiter unconditional)
  if (first_order == 0)
    adjoint_fused<T>(src, gout_ + g * 5 * 4096, gas, 0, ws, sm, sink);
  else
    adjoint_fused<T>(src, gout_ + g * 5 * 4096, gas, first_order, ws, sm, sink);
}

template <typename T>
__global__ __launch_bounds__(kAdjThreads) __attribute__((amdgpu_waves_per_eu(AdjWaves<T>::value, AdjWaves<T>::value))) void adj_fused_level(const T* __restrict__ level, const T* __restrict__ gout_,
                                                            T* __restrict__ gbox, LevelGeom geo, Gas<T> gas,
                                                            const double* __restrict__ dt_dev, double dx,
                                                            int first_order, int ws) {
  __shared__ SmemF<T> sm;
  set_dt_adj(gas, dt_dev, dx);
  const int64_t g = adj_level_group(geo);
  if (g < 0) return;  // uniform
  LevelSource<T> src{level, geo, int(g % geo.ngx), int((g / geo.ngx) % geo.ngy), int(g / (int64_t(geo.ngx) * geo.ngy))};
  BoxSink<T> sink{gbox + g * 5 * int64_t(kBox * kBox * kBox)};
  // the second-order scheme gets its own inlined copy (limiter unconditional)
  if (first_order == 0)
    adjoint_fused<T>(src, gout_ + g * 5 * 4096, gas, 0, ws, sm, sink);
  else
    adjoint_fused<T>(src, gout_ + g * 5 * 4096, gas, first_order, ws, sm, sink);
}

template <typename T>
__global__ __launch_bounds__(kAdjThreads) __attribute__((amdgpu_waves_per_eu(2, 2))) void adj_faces_padded(
    const T* __restrict__ Upad, const T* __restrict__ gout_, T* __restrict__ ws, int gh, Gas<T> gas,
    int first_order, int wsp) {
  __shared__ SmemFaces<T> sm;
  const int P = 16 + 2 * gh;
  const int64_t g = blockIdx.x;
  PaddedSource<T> src{Upad + g * 5 * int64_t(P) * P * P, P, gh};
  // the second-order scheme gets its own inlined copy (limiter unconditional)
  if (first_order == 0)
    adjoint_faces_pass<T>(src, gout_ + g * 5 * 4096, ws + g * kFaceWs, gas, 0, wsp, sm);
  else
    adjoint_faces_pass<T>(src, gout_ + g * 5 * 4096, ws + g * kFaceWs, gas, first_order, wsp, sm);
}

template <typename T>
__global__ __launch_bounds__(kAdjThreads) __attribute__((amdgpu_waves_per_eu(2, 2))) void adj_cells_padded(
    const T* __restrict__ Upad, const T* __restrict__ gout_, const T* __restrict__ ws, T* __restrict__ gpad, int gh,
    Gas<T> gas, int first_order) {
  __shared__ SmemCells<T> sm;
  const int P = 16 + 2 * gh;
  const int64_t g = blockIdx.x;
  const int64_t P3 = int64_t(P) * P * P;
  PaddedSource<T> src{Upad + g * 5 * P3, P, gh};
  PadSink<T> sink{gpad + g * 5 * P3, P, gh};
  // the second-order scheme gets its own inlined copy (limiter unconditional)
  if (first_order == 0)
    adjoint_cells_pass<T>(src, gout_ + g * 5 * 4096, ws + g * kFaceWs, gas, 0, sm, sink);
  else
    adjoint_cells_pass<T>(src, gout_ + g * 5 * 4096, ws + g * kFaceWs, gas, first_order, sm, sink);
}

template <typename T>
__global__ __launch_bounds__(kAdjThreads) __attribute__((amdgpu_waves_per_eu(2, 2))) void adj_faces_level(
    const T* __restrict__ level, const T* __restrict__ gout_, T* __restrict__ ws, LevelGeom geo, Gas<T> gas,
    const double* __restrict__ dt_dev, double dx, int first_order, int wsp) {
  __shared__ SmemFaces<T> sm;
  set_dt_adj(gas, dt_dev, dx);
  const int64_t g = adj_level_group(geo);
  if (g < 0) return;  // uniform
  LevelSource<T> src{level, geo, int(g % geo.ngx), int((g / geo.ngx) % geo.ngy), int(g / (int64_t(geo.ngx) * geo.ngy))};
  // the second-order scheme gets its own inlined copy (limiter unconditional)
  if (first_order == 0)
    adjoint_faces_pass<T>(src, gout_ + g * 5 * 4096, ws + g * kFaceWs, gas, 0, wsp, sm);
  else
    adjoint_faces_pass<T>(src, gout_ + g * 5 * 4096, ws + g * kFaceWs, gas, first_order, wsp, sm);
}

template <typename T>
__global__ __launch_bounds__(kAdjThreads) __attribute__((amdgpu_waves_per_eu(2, 2))) void adj_cells_level(
    const T* __restrict__ level, const T* __restrict__ gout_, const T* __restrict__ ws, T* __restrict__ gbox,
    LevelGeom geo, Gas<T> gas, const double* __restrict__ dt_dev, double dx, int first_order) {
  __shared__ SmemCells<T> sm;
  set_dt_adj(gas, dt_dev, dx);
  const int64_t g = adj_level_group(geo);
  if (g < 0) return;  // uniform
  LevelSource<T> src{level, geo, int(g % geo.ngx), int((g / geo.ngx) % geo.ngy), int(g / (int64_t(geo.ngx) * geo.ngy))};
  BoxSink<T> sink{gbox + g * 5 * int64_t(kBox * kBox * kBox)};
  // the second-order scheme gets its own inlined copy (limiter unconditional)
  if (first_order == 0)
    adjoint_cells_pass<T>(src, gout_ + g * 5 * 4096, ws + g * kFaceWs, gas, 0, sm, sink);
  else
    adjoint_cells_pass<T>(src, gout_ + g * 5 * 4096, ws + g * kFaceWs, gas, first_order, sm, sink);
}

// ------------------------------------------------------------ kernel C ----
// Is box position (x, y, z) (group-relative, [-2, 17]^3) a cell the step reads?
__device__ __forceinline__ bool reachable(int x, int y, int z) {
  const int dx = x < 0 ? -x : (x > 15 ? x - 15 : 0);
  const int dy = y < 0 ? -y : (y > 15 ? y - 15 : 0);
  const int dz = z < 0 ? -z : (z > 15 ? z - 15 : 0);
  const int o = (dx > 0) + (dy > 0) + (dz > 0);
  const int m = dx > dy ? (dx > dz ? dx : dz) : (dy > dz ? dy : dz);
  return o == 0 || (o == 1 && m <= 2) || (o == 2 && m <= 1);
}

// Positions that copy level index X along one axis under the ghost-fill index
// map with ghost width gh <= 16: position p in [-gh, 16 + gh) of group g
// stands for index i = 16 g + p, kept if 0 <= i < n, else mapped by the face
// it lies beyond (periodic: i -/+ n; outflow: the nearest interior index).
// Solving map(i) = X gives, as runs of consecutive positions in one group
// (at most five):
//   inside the domain  i = X, seen by the group holding X and, within gh of
//                      its faces, by the neighbouring group;
//   below the low face (group 0, p < 0): periodic p = X - n if that is
//                      >= -gh; outflow all gh positions when X = 0;
//   above the high face (group ng-1, p >= 16): periodic p = X + 16 if X < gh;
//                      outflow all gh positions when X = n - 1.
struct Run {
  int g, p, n;  // group along the axis, first position, number of positions
};

// The five run slots of one axis, each packed in one int (n: 5 bits, p + 64:
// 7 bits, g: the rest) and selected arithmetically, so that a run-time slot
// index keeps them in registers.
struct Runs {
  int v0, v1, v2, v3, v4;
  __device__ static int pack(int g, int p, int n) { return (g << 12) | ((p + 64) << 5) | n; }
  __device__ Run operator[](int k) const {
    int v = v0;
    v = k == 1 ? v1 : v;
    v = k == 2 ? v2 : v;
    v = k == 3 ? v3 : v;
    v = k == 4 ? v4 : v;
    return Run{v >> 12, ((v >> 5) & 127) - 64, v & 31};
  }
};

// Fixed slots (absent runs have n = 0): 0 the lower neighbour group, 1 the
// group holding X, 2 the upper neighbour group, 3 below the low face, 4 above
// the high face.
__device__ __forceinline__ Runs axis_runs(int X, int ng, int lo, int hi, int gh) {
  const int n = ng * 16, g0 = X >> 4, x = X & 15;
  Runs r;
  r.v0 = Runs::pack(g0 >= 1 ? g0 - 1 : 0, x + 16, (g0 >= 1 && x < gh) ? 1 : 0);
  r.v1 = Runs::pack(g0, x, 1);
  r.v2 = Runs::pack(g0 + 1, x - 16, (g0 + 1 < ng && x >= 16 - gh) ? 1 : 0);
  r.v3 = lo == 0 ? Runs::pack(0, X - n >= -gh ? X - n : 0, X - n >= -gh ? 1 : 0) : Runs::pack(0, -gh, X == 0 ? gh : 0);
  r.v4 = hi == 0 ? Runs::pack(ng - 1, X + 16, X < gh ? 1 : 0) : Runs::pack(ng - 1, 16, X == n - 1 ? gh : 0);
  return r;
}

// Up to 4 copies along one axis for ghost width 2 (the level path), compacted
// in slot order into packed (g, p) entries.  Four occur with an outflow face
// on one side and a periodic one on the other (the cell itself, two outflow
// ghost positions and the wrapped copy).
struct Copies4 {
  int v0, v1, v2, v3, n;
  __device__ void push(bool ok, int v) {
    v3 = ok ? v2 : v3;
    v2 = ok ? v1 : v2;
    v1 = ok ? v0 : v1;
    v0 = ok ? v : v0;
    n += ok ? 1 : 0;
  }
  // entry i in slot order (pushes shift older entries up)
  __device__ int at(int i) const {
    const int k = n - 1 - i;
    return k == 0 ? v0 : k == 1 ? v1 : k == 2 ? v2 : v3;
  }
};

__device__ __forceinline__ Copies4 axis_copies2(const Runs& r) {
  Copies4 c{0, 0, 0, 0, 0};
  const Run s0 = r[0], s1 = r[1], s2 = r[2], s3 = r[3], s4 = r[4];
  c.push(s0.n > 0, Runs::pack(s0.g, s0.p, 1));
  c.push(true, Runs::pack(s1.g, s1.p, 1));
  c.push(s2.n > 0, Runs::pack(s2.g, s2.p, 1));
  c.push(s3.n > 0, Runs::pack(s3.g, s3.p, 1));
  c.push(s3.n > 1, Runs::pack(s3.g, s3.p + 1, 1));
  c.push(s4.n > 0, Runs::pack(s4.g, s4.p, 1));
  c.push(s4.n > 1, Runs::pack(s4.g, s4.p + 1, 1));
  return c;
}

// Sum, per level cell, the cotangents of every copy of the cell: the adjoint
// of the ghost fill, written as a gather (fixed order, no atomics).  kBoxSrc:
// the source is the per-group [5][20^3] box of the level adjoint (positions
// [-2, 17], only stencil-reachable ones hold values); the x copies of each
// (z, y) pair are loaded together.  Otherwise a padded [5][P^3] block per
// group with ghost width gh (runs of up to gh positions per face).
// One workgroup of 256 threads per (group, z) plane of the level, so the
// group, its lattice position and the z runs are uniform (scalar) per
// workgroup and each thread maps only its (x, y).
template <typename T, bool kBoxSrc>
__global__ __launch_bounds__(256) void adj_gather(const T* __restrict__ src, T* __restrict__ glevel, LevelGeom geo,
                                                  int gh, int64_t ncells) {
  const unsigned int blk = blockIdx.x;
  const int z = int(blk & 15u);
  const int64_t g = int64_t(blk >> 4);
  const int x = int(threadIdx.x & 15u), y = int(threadIdx.x >> 4);
  // level cell (g, z, y, x) in group-major order
  const int64_t i = (g << 12) + (int64_t(z) << 8) + threadIdx.x;
  if (i >= ncells) return;
  const int gx = int(g % geo.ngx), gy = int((g / geo.ngx) % geo.ngy), gz = int(g / (int64_t(geo.ngx) * geo.ngy));
  const int w = kBoxSrc ? 2 : gh;        // position offset of the source block
  const int P = kBoxSrc ? kBox : 16 + 2 * gh;
  const int64_t P3 = int64_t(P) * P * P;
  const Runs rx = axis_runs(gx * 16 + x, geo.ngx, geo.bc[0], geo.bc[1], w);
  const Runs ry = axis_runs(gy * 16 + y, geo.ngy, geo.bc[2], geo.bc[3], w);
  const Runs rz = axis_runs(gz * 16 + z, geo.ngz, geo.bc[4], geo.bc[5], w);
  T s[5] = {T(0), T(0), T(0), T(0), T(0)};
  if (kBoxSrc) {
    const Copies4 cx = axis_copies2(rx), cy = axis_copies2(ry), cz = axis_copies2(rz);
#pragma unroll 1
    for (int a = 0; a < cz.n; ++a) {
      const int vz = cz.at(a);
      const int gzs = vz >> 12, pz = ((vz >> 5) & 127) - 64;
#pragma unroll 1
      for (int b = 0; b < cy.n; ++b) {
        const int vy = cy.at(b);
        const int gys = vy >> 12, py = ((vy >> 5) & 127) - 64;
        T v[4][5];
#pragma unroll
        for (int c = 0; c < 4; ++c) {
          const int vx = cx.at(c);
          const int gxs = vx >> 12, px = ((vx >> 5) & 127) - 64;
          const bool ok = c < cx.n && reachable(px, py, pz);
          const int64_t sg = (int64_t(gzs) * geo.ngy + gys) * geo.ngx + gxs;
          const T* base = src + sg * 5 * P3 + (int64_t(pz + w) * P + (py + w)) * P + (px + w);
#pragma unroll
          for (int q = 0; q < 5; ++q) v[c][q] = ok ? base[q * P3] : T(0);
        }
#pragma unroll
        for (int q = 0; q < 5; ++q) s[q] = s[q] + v[0][q] + v[1][q] + v[2][q] + v[3][q];
      }
    }
  } else {
#pragma unroll 1
    for (int a = 0; a < 5; ++a) {
      const Run ra = rz[a];
      for (int pz = ra.p; pz < ra.p + ra.n; ++pz)
#pragma unroll 1
        for (int b = 0; b < 5; ++b) {
          const Run rb = ry[b];
          for (int py = rb.p; py < rb.p + rb.n; ++py)
#pragma unroll 1
            for (int c = 0; c < 5; ++c) {
              const Run rc = rx[c];
              for (int px = rc.p; px < rc.p + rc.n; ++px) {
                const int64_t sg = (int64_t(ra.g) * geo.ngy + rb.g) * geo.ngx + rc.g;
                const T* base = src + sg * 5 * P3 + (int64_t(pz + w) * P + (py + w)) * P + (px + w);
#pragma unroll
                for (int q = 0; q < 5; ++q) s[q] = s[q] + base[q * P3];
              }
            }
        }
    }
  }
#pragma unroll
  for (int q = 0; q < 5; ++q) glevel[(g * 5 + q) * 4096 + (i & 4095)] = s[q];
}

template <typename T>
__global__ __launch_bounds__(256) void zero_kernel(T* __restrict__ p, int64_t n) {
  for (int64_t i = int64_t(blockIdx.x) * blockDim.x + threadIdx.x; i < n; i += int64_t(gridDim.x) * blockDim.x)
    p[i] = T(0);
}

}  // namespace

size_t adjoint_workspace_elems(int64_t n_groups, bool level) {
  // the face workspace of the split form, plus the reachable-cell box of the level path
  return size_t(n_groups) * (size_t(kFaceWs) + (level ? 5 * size_t(kBox * kBox * kBox) : 0));
}

template <typename T>
hipError_t launch_mhm_adjoint_padded(const T* U_pad, const T* g_out, T* g_pad, int64_t G, int ghost, const Gas<T>& gas,
                                     int first_order, int ws, T* work, bool split, hipStream_t stream) {
  if (G == 0) return hipSuccess;
  if (G > (int64_t(1) << 30)) return hipErrorInvalidValue;
  const int P = 16 + 2 * ghost;
  const int64_t n = G * 5 * int64_t(P) * P * P;
  int64_t zb = (n + 255) / 256;
  if (zb > 65536) zb = 65536;
  // positions the step does not read receive zero
  hipLaunchKernelGGL(zero_kernel<T>, dim3(unsigned(zb)), dim3(256), 0, stream, g_pad, n);
  if (split) {
    hipLaunchKernelGGL(adj_faces_padded<T>, dim3(unsigned(G)), dim3(kAdjThreads), 0, stream, U_pad, g_out, work,
                       ghost, gas, first_order, ws);
    hipLaunchKernelGGL(adj_cells_padded<T>, dim3(unsigned(G)), dim3(kAdjThreads), 0, stream, U_pad, g_out, work,
                       g_pad, ghost, gas, first_order);
  } else {
    hipLaunchKernelGGL(adj_fused_padded<T>, dim3(unsigned(G)), dim3(kAdjThreads), 0, stream, U_pad, g_out, g_pad,
                       ghost, gas, first_order, ws);
  }
  return hipGetLastError();
}

template <typename T>
hipError_t launch_mhm_adjoint_level(const T* level, const T* g_out, T* g_in, const LevelGeom& geo, const Gas<T>& gas,
                                    const double* dt_dev, double dx, int first_order, int ws, T* work, bool split,
                                    hipStream_t stream) {
  const int64_t G = int64_t(geo.ngx) * geo.ngy * geo.ngz;
  if (G == 0) return hipSuccess;
  if (G > (int64_t(1) << 28) - 1) return hipErrorInvalidValue;  // the gather takes G * 16 workgroups
  if (geo.ngx >= (1 << 19) || geo.ngy >= (1 << 19) || geo.ngz >= (1 << 19)) return hipErrorInvalidValue;
  T* gbox = work;  // [G][5][20^3]; only reachable positions are written, and only those are read
  T* fws = work + G * 5 * int64_t(kBox * kBox * kBox);
  const unsigned blocks = unsigned((G + 7) / 8 * 8);  // adj_level_group's padded grid
  if (split) {
    hipLaunchKernelGGL(adj_faces_level<T>, dim3(blocks), dim3(kAdjThreads), 0, stream, level, g_out, fws, geo,
                       gas, dt_dev, dx, first_order, ws);
    hipLaunchKernelGGL(adj_cells_level<T>, dim3(blocks), dim3(kAdjThreads), 0, stream, level, g_out, fws, gbox,
                       geo, gas, dt_dev, dx, first_order);
  } else {
    hipLaunchKernelGGL(adj_fused_level<T>, dim3(blocks), dim3(kAdjThreads), 0, stream, level, g_out, gbox, geo,
                       gas, dt_dev, dx, first_order, ws);
  }
  const int64_t ncells = G * 4096;
  hipLaunchKernelGGL((adj_gather<T, true>), dim3(unsigned(G * 16)), dim3(256), 0, stream, gbox, g_in, geo, 2, ncells);
  return hipGetLastError();
}

template <typename T>
hipError_t launch_gather_ghost_adjoint(const T* g_pad, T* g_level, const LevelGeom& geo, int ghost,
                                       hipStream_t stream) {
  const int64_t G = int64_t(geo.ngx) * geo.ngy * geo.ngz;
  if (G == 0) return hipSuccess;
  if (G > (int64_t(1) << 28) - 1) return hipErrorInvalidValue;  // one workgroup per (group, z) plane
  if (geo.ngx >= (1 << 19) || geo.ngy >= (1 << 19) || geo.ngz >= (1 << 19)) return hipErrorInvalidValue;
  const int64_t ncells = G * 4096;
  hipLaunchKernelGGL((adj_gather<T, false>), dim3(unsigned(G * 16)), dim3(256), 0, stream, g_pad, g_level, geo, ghost,
                     ncells);
  return hipGetLastError();
}

template hipError_t launch_mhm_adjoint_padded<double>(const double*, const double*, double*, int64_t, int,
                                                      const Gas<double>&, int, int, double*, bool, hipStream_t);
template hipError_t launch_mhm_adjoint_padded<float>(const float*, const float*, float*, int64_t, int,
                                                     const Gas<float>&, int, int, float*, bool, hipStream_t);
template hipError_t launch_mhm_adjoint_level<double>(const double*, const double*, double*, const LevelGeom&,
                                                     const Gas<double>&, const double*, double, int, int, double*,
                                                     bool, hipStream_t);
template hipError_t launch_mhm_adjoint_level<float>(const float*, const float*, float*, const LevelGeom&,
                                                    const Gas<float>&, const double*, double, int, int, float*, bool,
                                                    hipStream_t);
template hipError_t launch_gather_ghost_adjoint<double>(const double*, double*, const LevelGeom&, int, hipStream_t);
template hipError_t launch_gather_ghost_adjoint<float>(const float*, float*, const LevelGeom&, int, hipStream_t);

}  // namespace gh
