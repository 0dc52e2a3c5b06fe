// Plain FP64 CPU oracle for the per-patch-group MUSCL-Hancock (MHM) Euler step.
//
// TEST INFRASTRUCTURE ONLY.  Nothing on the product path may link, load or
// call this file: it exists so that tests, the smoke check and the benchmark's
// CPU baseline can compare the HIP kernels against an independent, obviously
// correct implementation.  It shares no source, header, table or helper with
// the HIP library.
//
// What it computes (Schive et al. 2018, "GAMER-2", Sec. 2.2 Hydrodynamics;
// the MHM scheme, PLM reconstruction, generalized minmod limiter and HLLC
// solver it names; Sec. 2.6 Eq. 2 for the CFL time-step of MHM):
//   a1  conserved -> primitive variables                  (cons_to_prim)
//   a2  PLM slopes with the generalized minmod limiter    (limited_slope)
//   a3  face states and physical fluxes                   (face_state_flux)
//   a4  conservative Hancock half step, unsplit           (hancock_cell)
//   a5  HLLC flux at every face                           (hllc_flux)
//   a6  conservative flux-difference update               (mhm_step_block)
//   a7  count of unphysical face states / updated cells   (mhm_step_block)
//   a8  per-patch CFL time-step, Eq. 2                    (patch_dt)
//   a0  ghost-zone fill, periodic or outflow              (fill_ghosts)
//   exact Riemann solver (Toro's pressure-function Newton method) for the
//   Sod-tube pin.
// The other options Sec. 2.2 lists, in the same plain style (step_block_any):
//   van Leer, van Albada and hybrid limiters          (limit_diffs)
//   PLM on characteristic variables                   (limited_slopes)
//   PPM reconstruction                                (face_values)
//   HLLE and Roe solvers, Roe switching to HLLC on an
//   unphysical intermediate state                     (hlle_flux, roe_flux)
//   CTU with 6 Riemann solves per cell                (step_block_any)
//   the procedure for unphysical results: first-order
//   unsplit, then split recompute of failed cells, then
//   level retries at dt * 0.8                         (level_step_repaired,
//                                                      oracle_level_step_fallback)
//   coarse-fine coupling in a W-cycle: ghost zones
//   interpolated from the coarse level, flux registers,
//   restriction, flux fix-up                          (amr_advance)
//
// Readings where the paper is silent (each stated in the function it governs):
//   * MHM predictor is the conservative unsplit Hancock step, no Riemann solve
//     in the predictor (MHM needs 3 Riemann solves per cell, Sec. 4.4 Table).
//   * PLM acts on primitive variables (rho, u, v, w, p).
//   * limiter: slope = sgn(dc) * min(theta*|dm|, |dc|, theta*|dp|) when dm and
//     dp are strictly of one sign, else 0; dc = (q[+1]-q[-1])/2; theta run-time.
//   * HLLC wave speeds: Einfeldt/Roe-averaged by default, Davis as an option.
//   * no positivity floors; unphysical states are only counted.
//
// Scalar types: the step is a template over the scalar so that the same code
// runs in plain double, in forward-mode dual numbers (exact Jacobian-vector
// products for the adjoint tests) and in an operation-counting type (the
// algorithmic flop count per cell update).  Branch decisions always use the
// value part.  Built with -ffp-contract=off: every operation rounds once.

#include <omp.h>

#include <cmath>
#include <cstdint>
#include <cstring>
#include <vector>

namespace {

// ---------------------------------------------------------------- scalars --

// Forward-mode dual number: value v and one tangent component d.
struct Dual {
  double v, d;
  Dual() : v(0), d(0) {}
  Dual(double x) : v(x), d(0) {}
  Dual(double x, double t) : v(x), d(t) {}
};
inline Dual operator+(Dual a, Dual b) { return Dual(a.v + b.v, a.d + b.d); }
inline Dual operator-(Dual a, Dual b) { return Dual(a.v - b.v, a.d - b.d); }
inline Dual operator-(Dual a) { return Dual(-a.v, -a.d); }
inline Dual operator*(Dual a, Dual b) { return Dual(a.v * b.v, a.d * b.v + a.v * b.d); }
inline Dual operator/(Dual a, Dual b) {
  double q = a.v / b.v;
  return Dual(q, (a.d - q * b.d) / b.v);
}
inline Dual tsqrt(Dual a) {
  double s = std::sqrt(a.v);
  return Dual(s, a.d / (2.0 * s));
}
inline double val(Dual a) { return a.v; }

// Operation-counting scalar: carries a double and counts what it does.
struct OpCount { int64_t add, mul, div, sqrt; };
thread_local OpCount g_ops = {0, 0, 0, 0};
struct Cnt {
  double v;
  Cnt() : v(0) {}
  Cnt(double x) : v(x) {}
};
inline Cnt operator+(Cnt a, Cnt b) { g_ops.add++; return Cnt(a.v + b.v); }
inline Cnt operator-(Cnt a, Cnt b) { g_ops.add++; return Cnt(a.v - b.v); }
inline Cnt operator-(Cnt a) { return Cnt(-a.v); }
inline Cnt operator*(Cnt a, Cnt b) { g_ops.mul++; return Cnt(a.v * b.v); }
inline Cnt operator/(Cnt a, Cnt b) { g_ops.div++; return Cnt(a.v / b.v); }
inline Cnt tsqrt(Cnt a) { g_ops.sqrt++; return Cnt(std::sqrt(a.v)); }
inline double val(Cnt a) { return a.v; }

inline double tsqrt(double a) { return std::sqrt(a); }
inline double tpow(double a, double e) { return std::pow(a, e); }
inline Dual tpow(Dual a, double e) {
  const double p = std::pow(a.v, e);
  return Dual(p, e * std::pow(a.v, e - 1.0) * a.d);
}
inline double val(double a) { return a; }

// ------------------------------------------------------ branch record ----
// When switched on for the calling thread, every branch decision of the step
// (the limiter's one-sign test, the sign of each |.|, which argument a
// min / max keeps, the HLLC branch) is folded, in evaluation order, into a
// 64-bit FNV-1a hash.  Two evaluations of the same cells take the same
// branches everywhere iff (up to hash collisions) their hashes agree; this is
// what a central difference needs to know (both sides on one smooth piece).
// Recording reads the decision only: the arithmetic is the same on or off.
thread_local bool g_sig_on = false;
thread_local uint64_t g_sig = 0;
inline void sig_mix(uint64_t code) {
  if (!g_sig_on) return;
  g_sig = (g_sig ^ code) * 0x100000001b3ull;
}

// |x| with derivative sign(x) * dx (never evaluated at x == 0 on a path whose
// derivative matters: the limiter only takes |.| of strictly signed values).
template <class T> inline T tabs(T x) {
  const bool neg = val(x) < 0.0;
  sig_mix(neg ? 3 : 4);
  return neg ? -x : x;
}

// min / max that keep the FIRST argument on ties (value and derivative).
template <class T> inline T tmin(T a, T b) {
  const bool second = val(b) < val(a);
  sig_mix(second ? 5 : 6);
  return second ? b : a;
}
template <class T> inline T tmax(T a, T b) {
  const bool second = val(b) > val(a);
  sig_mix(second ? 7 : 8);
  return second ? b : a;
}

// ------------------------------------------------------------ scheme word --
constexpr int SCHEME_ID_MASK = 0xff;
constexpr int SCHEME_MHM_PLM_HLLC = 1;
constexpr int WAVESPEED_SHIFT = 8;   // bits 8-9: 0 Einfeldt/Roe, 1 Davis
constexpr int FIRST_ORDER_BIT = 1 << 10;

// ------------------------------------------------------------ layouts ----
// One padded block: 5 fields, each (nz+2g) x (ny+2g) x (nx+2g), x fastest.
struct Block {
  int nx, ny, nz, g;
  int64_t px, py, pz;
  Block(int nx_, int ny_, int nz_, int g_)
      : nx(nx_), ny(ny_), nz(nz_), g(g_), px(nx_ + 2 * g_), py(ny_ + 2 * g_), pz(nz_ + 2 * g_) {}
  // (x, y, z) are interior-relative: 0..n-1 interior, negative / >= n ghosts.
  int64_t at(int f, int x, int y, int z) const {
    return ((int64_t(f) * pz + (z + g)) * py + (y + g)) * px + (x + g);
  }
  int64_t cells() const { return px * py * pz; }
};

// ------------------------------------------------ a1: primitive variables --
// rho, u = m_x/rho, v = m_y/rho, w = m_z/rho,
// p = (gamma-1) * (E - (m_x u + m_y v + m_z w)/2)   (Sec. 2.2, ideal gas EoS)
template <class T>
void cons_to_prim(const T U[5], double gamma, T W[5]) {
  const T rho = U[0];
  const T u = U[1] / rho, v = U[2] / rho, w = U[3] / rho;
  const T ke2 = U[1] * u + U[2] * v + U[3] * w;  // twice the kinetic energy
  W[0] = rho;
  W[1] = u;
  W[2] = v;
  W[3] = w;
  W[4] = T(gamma - 1.0) * (U[4] - T(0.5) * ke2);
}

// E = p/(gamma-1) + rho (u^2+v^2+w^2)/2
template <class T>
void prim_to_cons(const T W[5], double gamma, T U[5]) {
  const T rho = W[0];
  U[0] = rho;
  U[1] = rho * W[1];
  U[2] = rho * W[2];
  U[3] = rho * W[3];
  const T v2 = W[1] * W[1] + W[2] * W[2] + W[3] * W[3];
  U[4] = W[4] / T(gamma - 1.0) + T(0.5) * rho * v2;
}

// Physical Euler flux along direction d (0 = x, 1 = y, 2 = z) of a state
// given in both primitive (W) and conserved (U) form:
//   F_d = (rho u_d, m_x u_d + p delta_xd, m_y u_d + p delta_yd,
//          m_z u_d + p delta_zd, (E + p) u_d)
template <class T>
void euler_flux(const T W[5], const T U[5], int d, T F[5]) {
  const T ud = W[1 + d];
  F[0] = U[0] * ud;
  F[1] = U[1] * ud;
  F[2] = U[2] * ud;
  F[3] = U[3] * ud;
  F[1 + d] = F[1 + d] + W[4];
  F[4] = (U[4] + W[4]) * ud;
}

// ---------------------------------- a2: generalized minmod limited slope --
// Sec. 2.2 names the generalized minmod limiter; its form (theta in [1, 2]):
//   dm = q0 - qm, dp = qp - q0, dc = (qp - qm)/2
//   slope = sgn(dc) min(theta |dm|, |dc|, theta |dp|)  if dm, dp strictly same sign
//         = 0                                          otherwise
// theta = 1 gives minmod(dm, dp); theta = 2 gives the MC limiter.  The min keeps
// the first argument on ties (this fixes which argument carries the derivative).
template <class T>
T limited_slope(T qm, T q0, T qp, double theta) {
  const T dm = q0 - qm, dp = qp - q0;
  const bool same_sign = (val(dm) > 0.0 && val(dp) > 0.0) || (val(dm) < 0.0 && val(dp) < 0.0);
  sig_mix(same_sign ? 1 : 2);
  if (!same_sign) return T(0.0);
  const T dc = T(0.5) * (qp - qm);
  T m = T(theta) * tabs(dm);
  m = tmin(m, tabs(dc));
  m = tmin(m, T(theta) * tabs(dp));
  sig_mix(val(dc) > 0.0 ? 9 : 10);
  return val(dc) > 0.0 ? m : -m;
}

// ------------------------------------------------ a3 + a4: Hancock state --
// For one cell with primitive state Wc and axis neighbours Wm[d] (at -e_d) and
// Wp[d] (at +e_d), produce the six half-step-evolved face states in conserved
// form: Ut[d][0] at the cell's low face in d, Ut[d][1] at its high face.
//   W_{d,-} = Wc - dW_d/2,  W_{d,+} = Wc + dW_d/2,  U_{d,+-} = cons(W_{d,+-})
//   dU = (dt/(2 dx)) * sum_d [F_d(U_{d,-}) - F_d(U_{d,+})]     (summed x, y, z)
//   Ut_{d,+-} = U_{d,+-} + dU
template <class T>
void hancock_cell(const T Wc[5], const T Wm[3][5], const T Wp[3][5], double gamma, double theta,
                  T half_dtdx, bool first_order, T Ut[3][2][5]) {
  T Ff[3][2][5];
  for (int d = 0; d < 3; ++d) {
    T Wf[2][5];
    for (int q = 0; q < 5; ++q) {
      const T s = first_order ? T(0.0) : limited_slope(Wm[d][q], Wc[q], Wp[d][q], theta);
      Wf[0][q] = Wc[q] - T(0.5) * s;
      Wf[1][q] = Wc[q] + T(0.5) * s;
    }
    for (int side = 0; side < 2; ++side) {
      prim_to_cons(Wf[side], gamma, Ut[d][side]);
      euler_flux(Wf[side], Ut[d][side], d, Ff[d][side]);
    }
  }
  for (int q = 0; q < 5; ++q) {
    T s = Ff[0][0][q] - Ff[0][1][q];
    s = s + (Ff[1][0][q] - Ff[1][1][q]);
    s = s + (Ff[2][0][q] - Ff[2][1][q]);
    const T dU = half_dtdx * s;
    for (int d = 0; d < 3; ++d) {
      Ut[d][0][q] = Ut[d][0][q] + dU;
      Ut[d][1][q] = Ut[d][1][q] + dU;
    }
  }
}

// ------------------------------------------------------------- a5: HLLC ---
// HLLC flux (the HLLC solver Sec. 2.2 names) between left state UL and right
// state UR across a face normal to axis d.  Work in the normal frame
// (u_n, u_t1, u_t2) with (n, t1, t2) = (d, d+1, d+2) mod 3.
//   c_K   = sqrt(gamma p_K / rho_K)
//   wave speeds, Einfeldt/Roe (default): Roe averages with weights sqrt(rho_K)
//           of u_n, u_t1, u_t2 and H = (E+p)/rho, c~^2 = (gamma-1)(H~ - |u~|^2/2),
//           S_L = min(u_L - c_L, u~ - c~),  S_R = max(u_R + c_R, u~ + c~)
//   wave speeds, Davis: S_L = min(u_L - c_L, u_R - c_R), S_R = max(u_L + c_L, u_R + c_R)
//   S*    = [p_R - p_L + rho_L u_L (S_L - u_L) - rho_R u_R (S_R - u_R)]
//           / [rho_L (S_L - u_L) - rho_R (S_R - u_R)]
//   U*_K  = r_K (rho_K, rho_K S*, m_t1K, m_t2K,
//                E_K + (S* - u_K)(rho_K S* + p_K/(S_K - u_K))),
//           r_K = (S_K - u_K)/(S_K - S*)
//   F = F_L                     if S_L >= 0
//       F_L + S_L (U*_L - U_L)  else if S* >= 0
//       F_R + S_R (U*_R - U_R)  else if S_R > 0
//       F_R                     otherwise
// Returns true if either input state is unphysical (rho <= 0 or p <= 0, NaN
// included), in which case the flux is still evaluated as written.
template <class T>
bool hllc_flux(const T UL[5], const T UR[5], int d, double gamma, int wavespeed, T F[5]) {
  const int n = 1 + d, t1 = 1 + (d + 1) % 3, t2 = 1 + (d + 2) % 3;
  const T gm1 = T(gamma - 1.0);
  const T g = T(gamma);
  // normal-frame conserved states
  const T L[5] = {UL[0], UL[n], UL[t1], UL[t2], UL[4]};
  const T R[5] = {UR[0], UR[n], UR[t1], UR[t2], UR[4]};
  const T rL = L[0], rR = R[0];
  const T uL = L[1] / rL, vL = L[2] / rL, wL = L[3] / rL;
  const T uR = R[1] / rR, vR = R[2] / rR, wR = R[3] / rR;
  const T pL = gm1 * (L[4] - T(0.5) * rL * (uL * uL + vL * vL + wL * wL));
  const T pR = gm1 * (R[4] - T(0.5) * rR * (uR * uR + vR * vR + wR * wR));
  const bool bad = !(val(rL) > 0.0 && val(pL) > 0.0 && val(rR) > 0.0 && val(pR) > 0.0);
  const T cL = tsqrt(g * pL / rL), cR = tsqrt(g * pR / rR);

  T SL, SR;
  if (wavespeed == 1) {  // Davis
    SL = tmin(uL - cL, uR - cR);
    SR = tmax(uL + cL, uR + cR);
  } else {  // Einfeldt / Roe averages
    const T sL = tsqrt(rL), sR = tsqrt(rR);
    const T inv = T(1.0) / (sL + sR);
    const T ut = (sL * uL + sR * uR) * inv;
    const T vt = (sL * vL + sR * vR) * inv;
    const T wt = (sL * wL + sR * wR) * inv;
    const T HL = (L[4] + pL) / rL, HR = (R[4] + pR) / rR;
    const T Ht = (sL * HL + sR * HR) * inv;
    const T ct = tsqrt(gm1 * (Ht - T(0.5) * (ut * ut + vt * vt + wt * wt)));
    SL = tmin(uL - cL, ut - ct);
    SR = tmax(uR + cR, ut + ct);
  }

  const T Sst = (pR - pL + rL * uL * (SL - uL) - rR * uR * (SR - uR)) /
                (rL * (SL - uL) - rR * (SR - uR));

  // physical fluxes in the normal frame
  const T FL[5] = {L[1], L[1] * uL + pL, L[2] * uL, L[3] * uL, (L[4] + pL) * uL};
  const T FR[5] = {R[1], R[1] * uR + pR, R[2] * uR, R[3] * uR, (R[4] + pR) * uR};

  T Fn[5];
  sig_mix(val(SL) >= 0.0 ? 11 : val(Sst) >= 0.0 ? 12 : val(SR) > 0.0 ? 13 : 14);
  if (val(SL) >= 0.0) {
    for (int q = 0; q < 5; ++q) Fn[q] = FL[q];
  } else if (val(Sst) >= 0.0) {
    const T r = (SL - uL) / (SL - Sst);
    const T Us[5] = {r * rL, r * (rL * Sst), r * L[2], r * L[3],
                     r * (L[4] + (Sst - uL) * (rL * Sst + pL / (SL - uL)))};
    for (int q = 0; q < 5; ++q) Fn[q] = FL[q] + SL * (Us[q] - L[q]);
  } else if (val(SR) > 0.0) {
    const T r = (SR - uR) / (SR - Sst);
    const T Us[5] = {r * rR, r * (rR * Sst), r * R[2], r * R[3],
                     r * (R[4] + (Sst - uR) * (rR * Sst + pR / (SR - uR)))};
    for (int q = 0; q < 5; ++q) Fn[q] = FR[q] + SR * (Us[q] - R[q]);
  } else {
    for (int q = 0; q < 5; ++q) Fn[q] = FR[q];
  }
  F[0] = Fn[0];
  F[n] = Fn[1];
  F[t1] = Fn[2];
  F[t2] = Fn[3];
  F[4] = Fn[4];
  return bad;
}

// ------------------------------------------------- a1..a7: one MHM step ---
// Advance the interior of one padded block by one MHM step.
// Upad: [5][pz][py][px]; Uout: [5][nz][ny][nx].  Needs g >= 2.
// Returns the unphysical count: faces whose two HLLC input states are not both
// physical, plus interior cells whose updated state has rho <= 0 or p <= 0.
template <class T>
int64_t mhm_step_block(const T* Upad, T* Uout, const Block& b, double dt, double dx, double gamma,
                       double theta, int scheme) {
  const bool first_order = (scheme & FIRST_ORDER_BIT) != 0;
  const int wavespeed = (scheme >> WAVESPEED_SHIFT) & 3;
  const T dtdx = T(dt) / T(dx);
  const T half_dtdx = T(0.5) * dtdx;
  int64_t n_bad = 0;

  // a1: primitive variables on the box [-2, n+1]^3 (covers every cell the
  // stencil can reach; the extra box corners are computed but never used).
  const int wx = b.nx + 4, wy = b.ny + 4, wz = b.nz + 4;
  auto wi = [&](int x, int y, int z) { return ((int64_t(z + 2) * wy + (y + 2)) * wx + (x + 2)); };
  std::vector<T> W(size_t(wx) * wy * wz * 5);
  for (int z = -2; z < b.nz + 2; ++z)
    for (int y = -2; y < b.ny + 2; ++y)
      for (int x = -2; x < b.nx + 2; ++x) {
        T U[5];
        for (int f = 0; f < 5; ++f) U[f] = Upad[b.at(f, x, y, z)];
        cons_to_prim(U, gamma, &W[wi(x, y, z) * 5]);
      }

  // a2..a4: half-step-evolved face states on every cell of [-1, n]^3.
  const int sx = b.nx + 2, sy = b.ny + 2, sz = b.nz + 2;
  auto si = [&](int x, int y, int z) { return ((int64_t(z + 1) * sy + (y + 1)) * sx + (x + 1)); };
  std::vector<T> S(size_t(sx) * sy * sz * 30);
  for (int z = -1; z < b.nz + 1; ++z)
    for (int y = -1; y < b.ny + 1; ++y)
      for (int x = -1; x < b.nx + 1; ++x) {
        T Wm[3][5], Wp[3][5];
        const int ex[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
        for (int d = 0; d < 3; ++d)
          for (int q = 0; q < 5; ++q) {
            Wm[d][q] = W[wi(x - ex[d][0], y - ex[d][1], z - ex[d][2]) * 5 + q];
            Wp[d][q] = W[wi(x + ex[d][0], y + ex[d][1], z + ex[d][2]) * 5 + q];
          }
        T Ut[3][2][5];
        hancock_cell(&W[wi(x, y, z) * 5], Wm, Wp, gamma, theta, half_dtdx, first_order, Ut);
        T* dst = &S[si(x, y, z) * 30];
        for (int d = 0; d < 3; ++d)
          for (int s = 0; s < 2; ++s)
            for (int q = 0; q < 5; ++q) dst[(d * 2 + s) * 5 + q] = Ut[d][s][q];
      }
  auto state = [&](int x, int y, int z, int d, int s) -> const T* {
    return &S[si(x, y, z) * 30 + (d * 2 + s) * 5];
  };

  // a5: HLLC at the faces the update needs.  Fx[x] is the face between x-1
  // and x (x = 0..nx), likewise Fy and Fz.
  auto fxi = [&](int x, int y, int z) { return ((int64_t(z) * b.ny + y) * (b.nx + 1) + x) * 5; };
  auto fyi = [&](int x, int y, int z) { return ((int64_t(z) * (b.ny + 1) + y) * b.nx + x) * 5; };
  auto fzi = [&](int x, int y, int z) { return ((int64_t(z) * b.ny + y) * b.nx + x) * 5; };
  std::vector<T> Fx(size_t(b.nz) * b.ny * (b.nx + 1) * 5), Fy(size_t(b.nz) * (b.ny + 1) * b.nx * 5),
      Fz(size_t(b.nz + 1) * b.ny * b.nx * 5);
  for (int z = 0; z < b.nz; ++z)
    for (int y = 0; y < b.ny; ++y)
      for (int x = 0; x <= b.nx; ++x)
        n_bad += hllc_flux(state(x - 1, y, z, 0, 1), state(x, y, z, 0, 0), 0, gamma, wavespeed,
                           &Fx[fxi(x, y, z)]);
  for (int z = 0; z < b.nz; ++z)
    for (int y = 0; y <= b.ny; ++y)
      for (int x = 0; x < b.nx; ++x)
        n_bad += hllc_flux(state(x, y - 1, z, 1, 1), state(x, y, z, 1, 0), 1, gamma, wavespeed,
                           &Fy[fyi(x, y, z)]);
  for (int z = 0; z <= b.nz; ++z)
    for (int y = 0; y < b.ny; ++y)
      for (int x = 0; x < b.nx; ++x)
        n_bad += hllc_flux(state(x, y, z - 1, 2, 1), state(x, y, z, 2, 0), 2, gamma, wavespeed,
                           &Fz[fzi(x, y, z)]);

  // a6: U^{n+1} = U^n - (dt/dx) [(Fx+ - Fx-) + (Fy+ - Fy-) + (Fz+ - Fz-)],
  // summed in that order.  a7: count unphysical updated cells.
  const T gm1 = T(gamma - 1.0);
  for (int z = 0; z < b.nz; ++z)
    for (int y = 0; y < b.ny; ++y)
      for (int x = 0; x < b.nx; ++x) {
        T Un[5];
        for (int q = 0; q < 5; ++q) {
          T acc = Fx[fxi(x + 1, y, z) + q] - Fx[fxi(x, y, z) + q];
          acc = acc + (Fy[fyi(x, y + 1, z) + q] - Fy[fyi(x, y, z) + q]);
          acc = acc + (Fz[fzi(x, y, z + 1) + q] - Fz[fzi(x, y, z) + q]);
          Un[q] = Upad[b.at(q, x, y, z)] - dtdx * acc;
          Uout[((int64_t(q) * b.nz + z) * b.ny + y) * b.nx + x] = Un[q];
        }
        const T p = gm1 * (Un[4] - T(0.5) * (Un[1] * Un[1] + Un[2] * Un[2] + Un[3] * Un[3]) / Un[0]);
        if (!(val(Un[0]) > 0.0 && val(p) > 0.0)) ++n_bad;
      }
  return n_bad;
}

// ------------------------------------------------------- a8: CFL, Eq. 2 ---
// For one 8^3 patch: s_max = max over cells of |u|+|v|+|w|+3 c_s, c_s =
// sqrt(gamma p / rho), and dt_patch = (C_CFL * dx) / s_max.  Sums are taken
// left to right: ((|u|+|v|)+|w|)+3c.
double patch_dt(const double* Upad, const Block& b, int x0, int y0, int z0, double dx, double gamma,
                double c_cfl) {
  double smax = 0.0;
  for (int z = z0; z < z0 + 8; ++z)
    for (int y = y0; y < y0 + 8; ++y)
      for (int x = x0; x < x0 + 8; ++x) {
        const double rho = Upad[b.at(0, x, y, z)];
        const double mx = Upad[b.at(1, x, y, z)], my = Upad[b.at(2, x, y, z)],
                     mz = Upad[b.at(3, x, y, z)], E = Upad[b.at(4, x, y, z)];
        const double u = mx / rho, v = my / rho, w = mz / rho;
        const double p = (gamma - 1.0) * (E - 0.5 * ((mx * u + my * v) + mz * w));
        const double c = std::sqrt((gamma * p) / rho);
        const double s = ((std::fabs(u) + std::fabs(v)) + std::fabs(w)) + 3.0 * c;
        if (s > smax) smax = s;
      }
  return (c_cfl * dx) / smax;
}

// ------------------------------------------------------ a0: ghost fill ----
// Source index along one axis of n cells for a (possibly ghost) index i:
// periodic wraps, outflow copies the nearest interior cell.
inline int bc_index(int i, int n, int bc_lo, int bc_hi) {
  if (i < 0) return bc_lo == 0 ? i + n : 0;
  if (i >= n) return bc_hi == 0 ? i - n : n - 1;
  return i;
}

// level: interiors of all groups, group-major [G][5][16][16][16] with groups
// ordered g = (gz*NGy + gy)*NGx + gx.  Upad: [G][5][P][P][P], P = 16 + 2*ghost.
template <class T>
void fill_ghosts(const T* level, T* Upad, int ngx, int ngy, int ngz, int ghost, const int bc[6]) {
  const int N = 16, P = N + 2 * ghost;
  const int Nx = ngx * N, Ny = ngy * N, Nz = ngz * N;
  const int64_t G = int64_t(ngx) * ngy * ngz;
  auto src = [&](int f, int X, int Y, int Z) {
    const int gx = X / N, gy = Y / N, gz = Z / N;
    const int64_t g = (int64_t(gz) * ngy + gy) * ngx + gx;
    return level[(((g * 5 + f) * N + Z % N) * N + Y % N) * N + X % N];
  };
  for (int64_t g = 0; g < G; ++g) {
    const int gx = int(g % ngx), gy = int((g / ngx) % ngy), gz = int(g / (int64_t(ngx) * ngy));
    for (int f = 0; f < 5; ++f)
      for (int z = 0; z < P; ++z)
        for (int y = 0; y < P; ++y)
          for (int x = 0; x < P; ++x) {
            const int X = bc_index(gx * N + x - ghost, Nx, bc[0], bc[1]);
            const int Y = bc_index(gy * N + y - ghost, Ny, bc[2], bc[3]);
            const int Z = bc_index(gz * N + z - ghost, Nz, bc[4], bc[5]);
            Upad[(((g * 5 + f) * P + z) * P + y) * P + x] = src(f, X, Y, Z);
          }
  }
}

// Advance every group of a level: fill ghosts, then one MHM step per group.
template <class T>
int64_t level_step(const T* level, T* level_out, int ngx, int ngy, int ngz, int ghost, const int bc[6],
                   double dt, double dx, double gamma, double theta, int scheme) {
  const int P = 16 + 2 * ghost;
  const int64_t G = int64_t(ngx) * ngy * ngz;
  std::vector<T> pad(size_t(G) * 5 * P * P * P);
  fill_ghosts(level, pad.data(), ngx, ngy, ngz, ghost, bc);
  const Block b(16, 16, 16, ghost);
  int64_t n_bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : n_bad)
  for (int64_t g = 0; g < G; ++g)
    n_bad += mhm_step_block(pad.data() + g * b.cells() * 5, level_out + g * 5 * 4096, b, dt, dx, gamma,
                            theta, scheme);
  return n_bad;
}

// --------------------------------------------- exact Riemann solver (Sod) --
// Toro's method for the ideal-gas Riemann problem, written from the jump and
// rarefaction relations: find p* with f_L(p*) + f_R(p*) + (u_R - u_L) = 0 where
//   f_K(p) = (p - p_K) sqrt(A_K / (p + B_K)),  A_K = 2/((g+1) rho_K),
//            B_K = (g-1)/(g+1) p_K                      (shock, p > p_K)
//   f_K(p) = 2 c_K/(g-1) ((p/p_K)^((g-1)/(2g)) - 1)     (rarefaction, p <= p_K)
// then u* = (u_L + u_R)/2 + (f_R(p*) - f_L(p*))/2.
struct RP {
  double rL, uL, pL, rR, uR, pR, g;
};
void pressure_fn(double p, double rK, double pK, double g, double* f, double* df) {
  const double cK = std::sqrt(g * pK / rK);
  if (p > pK) {
    const double A = 2.0 / ((g + 1.0) * rK), B = (g - 1.0) / (g + 1.0) * pK;
    const double q = std::sqrt(A / (p + B));
    *f = (p - pK) * q;
    *df = q * (1.0 - 0.5 * (p - pK) / (B + p));
  } else {
    const double z = (g - 1.0) / (2.0 * g);
    *f = 2.0 * cK / (g - 1.0) * (std::pow(p / pK, z) - 1.0);
    *df = 1.0 / (rK * cK) * std::pow(p / pK, -(g + 1.0) / (2.0 * g));
  }
}
int star_state(const RP& s, double* pstar, double* ustar, int* iters) {
  const double g = s.g;
  const double cL = std::sqrt(g * s.pL / s.rL), cR = std::sqrt(g * s.pR / s.rR);
  if (2.0 / (g - 1.0) * (cL + cR) <= s.uR - s.uL) return -1;  // vacuum: not handled
  // start from the two-rarefaction closed form
  const double z = (g - 1.0) / (2.0 * g);
  double p = std::pow((cL + cR - 0.5 * (g - 1.0) * (s.uR - s.uL)) /
                          (cL / std::pow(s.pL, z) + cR / std::pow(s.pR, z)),
                      1.0 / z);
  if (!(p > 1e-14)) p = 1e-14;
  int it = 0;
  for (; it < 100; ++it) {
    double fL, dfL, fR, dfR;
    pressure_fn(p, s.rL, s.pL, g, &fL, &dfL);
    pressure_fn(p, s.rR, s.pR, g, &fR, &dfR);
    double pn = p - (fL + fR + (s.uR - s.uL)) / (dfL + dfR);
    if (pn < 1e-14) pn = 1e-14;
    const double change = std::fabs(pn - p) / (0.5 * (pn + p));
    p = pn;
    if (change < 1e-15) break;
  }
  double fL, dfL, fR, dfR;
  pressure_fn(p, s.rL, s.pL, g, &fL, &dfL);
  pressure_fn(p, s.rR, s.pR, g, &fR, &dfR);
  *pstar = p;
  *ustar = 0.5 * (s.uL + s.uR) + 0.5 * (fR - fL);
  if (iters) *iters = it;
  return 0;
}
// Density on the two sides of the contact.
void star_densities(const RP& s, double ps, double* rsL, double* rsR) {
  const double g = s.g, gr = (g - 1.0) / (g + 1.0);
  auto side = [&](double rK, double pK) {
    if (ps > pK) return rK * (ps / pK + gr) / (gr * ps / pK + 1.0);  // shock
    return rK * std::pow(ps / pK, 1.0 / g);                           // rarefaction
  };
  *rsL = side(s.rL, s.pL);
  *rsR = side(s.rR, s.pR);
}
// Self-similar solution at xi = x/t.
void sample(const RP& s, double ps, double us, double xi, double* r, double* u, double* p) {
  const double g = s.g;
  double rsL, rsR;
  star_densities(s, ps, &rsL, &rsR);
  if (xi <= us) {  // left of the contact
    const double cL = std::sqrt(g * s.pL / s.rL);
    if (ps > s.pL) {  // left shock
      const double SL = s.uL - cL * std::sqrt((g + 1.0) / (2.0 * g) * ps / s.pL + (g - 1.0) / (2.0 * g));
      if (xi <= SL) { *r = s.rL; *u = s.uL; *p = s.pL; }
      else { *r = rsL; *u = us; *p = ps; }
    } else {  // left rarefaction
      const double csL = cL * std::pow(ps / s.pL, (g - 1.0) / (2.0 * g));
      const double head = s.uL - cL, tail = us - csL;
      if (xi <= head) { *r = s.rL; *u = s.uL; *p = s.pL; }
      else if (xi >= tail) { *r = rsL; *u = us; *p = ps; }
      else {
        const double k = 2.0 / (g + 1.0) + (g - 1.0) / ((g + 1.0) * cL) * (s.uL - xi);
        *r = s.rL * std::pow(k, 2.0 / (g - 1.0));
        *u = 2.0 / (g + 1.0) * (cL + 0.5 * (g - 1.0) * s.uL + xi);
        *p = s.pL * std::pow(k, 2.0 * g / (g - 1.0));
      }
    }
  } else {  // right of the contact
    const double cR = std::sqrt(g * s.pR / s.rR);
    if (ps > s.pR) {  // right shock
      const double SR = s.uR + cR * std::sqrt((g + 1.0) / (2.0 * g) * ps / s.pR + (g - 1.0) / (2.0 * g));
      if (xi >= SR) { *r = s.rR; *u = s.uR; *p = s.pR; }
      else { *r = rsR; *u = us; *p = ps; }
    } else {  // right rarefaction
      const double csR = cR * std::pow(ps / s.pR, (g - 1.0) / (2.0 * g));
      const double head = s.uR + cR, tail = us + csR;
      if (xi >= head) { *r = s.rR; *u = s.uR; *p = s.pR; }
      else if (xi <= tail) { *r = rsR; *u = us; *p = ps; }
      else {
        const double k = 2.0 / (g + 1.0) - (g - 1.0) / ((g + 1.0) * cR) * (s.uR - xi);
        *r = s.rR * std::pow(k, 2.0 / (g - 1.0));
        *u = 2.0 / (g + 1.0) * (-cR + 0.5 * (g - 1.0) * s.uR + xi);
        *p = s.pR * std::pow(k, 2.0 * g / (g - 1.0));
      }
    }
  }
}

// n_steps MHM steps of one block without ghost refills: a step advances the
// box's interior and drops its 2-cell margin, so the box shrinks by 4 cells
// per axis and step, and after n steps it holds exactly the cells whose
// values the n steps determine from the box alone.  This gives a rollout's
// result on a sub-box of a level (a periodic level's box taken with wrapped
// indices), with the branch record of every decision made on the way.
// box [5][nz][ny][nx] (double), tbox (optional) its tangent (dual numbers);
// out / tout [5][nz-4n][ny-4n][nx-4n]; *sig_out (optional) the branch hash.
template <class T>
int64_t rollout_box(std::vector<T> cur, int nx, int ny, int nz, int n_steps, double dt, double dx, double gamma,
                    double theta, int scheme, std::vector<T>& result) {
  int64_t n_bad = 0;
  for (int s = 0; s < n_steps; ++s) {
    const Block b(nx - 4, ny - 4, nz - 4, 2);
    std::vector<T> nxt(size_t(5) * b.nx * b.ny * b.nz);
    n_bad += mhm_step_block(cur.data(), nxt.data(), b, dt, dx, gamma, theta, scheme);
    cur.swap(nxt);
    nx -= 4;
    ny -= 4;
    nz -= 4;
  }
  result.swap(cur);
  return n_bad;
}

// ================================================= other schemes (Sec. 2.2) ==
// Sec. 2.2 lists, beside MHM + PLM + generalized minmod + HLLC: the CTU scheme
// with 6 Riemann solves per cell, Roe's and the HLLE solver, PPM
// reconstruction, reconstruction of primitive or characteristic variables,
// van Leer-type, van Albada-type and hybrid (generalized minmod + van Leer)
// limiters, and a procedure for cells with unphysical results.  The paper
// defers the formulas to the literature; each function below states the
// textbook form it takes.  Scheme word bits beyond the default:
//   bits 0-7    scheme id: 1 MHM, 2 CTU
//   bits 11-12  limiter: 0 generalized minmod, 1 van Leer, 2 van Albada, 3 hybrid
//   bit 13      limit characteristic instead of primitive variables
//   bit 14      PPM instead of PLM
//   bits 16-17  Riemann solver: 0 HLLC, 1 Roe, 2 HLLE
//   bit 18      dual energy: a sixth field, the entropy per unit volume
constexpr int SCHEME_CTU = 2;
constexpr int LIMITER_SHIFT = 11;
constexpr int CHARACTERISTIC_BIT = 1 << 13;
constexpr int PPM_BIT = 1 << 14;
constexpr int RIEMANN_SHIFT = 16;
constexpr int DUAL_ENERGY_BIT = 1 << 18;  // 6 fields: the entropy s = p / rho^(gamma-1) as field 5

// Limited slope from the one-sided differences dm = q0 - q[-1], dp = q[+1] - q0
// and the central difference dc (zero unless dm and dp have one strict sign):
//   0 generalized minmod  sgn(dc) min(theta|dm|, |dc|, theta|dp|)
//   1 van Leer            2 dm dp / (dm + dp)            (harmonic mean)
//   2 van Albada          dm dp (dm + dp) / (dm^2 + dp^2)
//   3 hybrid              sgn(dc) min(generalized minmod, |van Leer|)  (the
//                         more restrictive of the two)
template <class T>
T limit_diffs(T dm, T dp, T dc, double theta, int limiter) {
  const bool same_sign = (val(dm) > 0.0 && val(dp) > 0.0) || (val(dm) < 0.0 && val(dp) < 0.0);
  sig_mix(same_sign ? 1 : 2);
  if (!same_sign) return T(0.0);
  if (limiter == 1) return T(2.0) * dm * dp / (dm + dp);
  if (limiter == 2) return dm * dp * (dm + dp) / (dm * dm + dp * dp);
  T m = T(theta) * tabs(dm);
  m = tmin(m, tabs(dc));
  m = tmin(m, T(theta) * tabs(dp));
  if (limiter == 3) m = tmin(m, tabs(T(2.0) * dm * dp / (dm + dp)));
  sig_mix(val(dc) > 0.0 ? 9 : 10);
  return val(dc) > 0.0 ? m : -m;
}

// Characteristic variables of the primitive Euler system along axis d
// (normal velocity n, transverse t1, t2; sound speed c of the cell):
//   a0 = (dp/c^2 - (rho/c) du_n)/2   (wave u - c)
//   a1 = drho - dp/c^2               (entropy wave, u)
//   a2 = du_t1, a3 = du_t2           (shear waves, u)
//   a4 = (dp/c^2 + (rho/c) du_n)/2   (wave u + c)
// and back: drho = a0 + a1 + a4, du_n = (c/rho)(a4 - a0), du_t1 = a2,
// du_t2 = a3, dp = c^2 (a0 + a4).
template <class T>
void to_characteristic(const T dW[5], int d, T rho, T c, T a[5]) {
  const int n = 1 + d, t1 = 1 + (d + 1) % 3, t2 = 1 + (d + 2) % 3;
  const T pc2 = dW[4] / (c * c);
  const T run = (rho / c) * dW[n];
  a[0] = T(0.5) * (pc2 - run);
  a[1] = dW[0] - pc2;
  a[2] = dW[t1];
  a[3] = dW[t2];
  a[4] = T(0.5) * (pc2 + run);
}
template <class T>
void from_characteristic(const T a[5], int d, T rho, T c, T dW[5]) {
  const int n = 1 + d, t1 = 1 + (d + 1) % 3, t2 = 1 + (d + 2) % 3;
  dW[0] = (a[0] + a[1]) + a[4];
  dW[n] = (c / rho) * (a[4] - a[0]);
  dW[t1] = a[2];
  dW[t2] = a[3];
  dW[4] = (c * c) * (a[0] + a[4]);
}

// Limited slopes of the five primitive variables of cell Wc along axis d.
// Primitive: each variable limited on its own (the generalized minmod with dc
// = (q[+1] - q[-1])/2, exactly as limited_slope).  Characteristic: the one-
// sided differences are projected with the cell's left eigenvectors, each
// component is limited (dc = the mean of its two one-sided differences) and
// the result is projected back with the right eigenvectors.
template <class T>
void limited_slopes(const T Wm[5], const T Wc[5], const T Wp[5], int d, double gamma, double theta, int scheme,
                    T s[5]) {
  const int lim = (scheme >> LIMITER_SHIFT) & 3;
  if (!(scheme & CHARACTERISTIC_BIT)) {
    for (int q = 0; q < 5; ++q)
      s[q] = limit_diffs(Wc[q] - Wm[q], Wp[q] - Wc[q], T(0.5) * (Wp[q] - Wm[q]), theta, lim);
    return;
  }
  const T c = tsqrt(T(gamma) * Wc[4] / Wc[0]);
  T dm[5], dp[5], am[5], ap[5], as[5];
  for (int q = 0; q < 5; ++q) {
    dm[q] = Wc[q] - Wm[q];
    dp[q] = Wp[q] - Wc[q];
  }
  to_characteristic(dm, d, Wc[0], c, am);
  to_characteristic(dp, d, Wc[0], c, ap);
  for (int k = 0; k < 5; ++k) as[k] = limit_diffs(am[k], ap[k], T(0.5) * (am[k] + ap[k]), theta, lim);
  from_characteristic(as, d, Wc[0], c, s);
}

// PPM interface values of one variable from its cells -1, 0, +1 (qm, q0, qp)
// and their limited slopes, with the monotonicity constraints.
template <class T>
void ppm_scalar(T qm, T q0, T qp, T sm, T s0, T sp, T& qL, T& qR) {
  qL = T(0.5) * (qm + q0) - (s0 - sm) / T(6.0);
  qR = T(0.5) * (q0 + qp) - (sp - s0) / T(6.0);
  const bool extremum = !(val((qR - q0) * (q0 - qL)) > 0.0);
  sig_mix(extremum ? 15 : 16);
  if (extremum) {
    qL = q0;
    qR = q0;
  } else {
    const T dq = qR - qL;
    const T q6 = T(6.0) * (q0 - T(0.5) * (qL + qR));
    const bool over_l = val(dq * q6) > val(dq * dq);
    const bool over_r = !over_l && val(-(dq * dq)) > val(dq * q6);
    sig_mix(over_l ? 17 : over_r ? 18 : 19);
    if (over_l) qL = T(3.0) * q0 - T(2.0) * qR;
    if (over_r) qR = T(3.0) * q0 - T(2.0) * qL;
  }
}

// Face values (primitive) of a cell along axis d from the stencil Ws[0..4] =
// cells at -2..+2 (PLM reads -1..+1 only):
//   PLM: W_{-,+} = W0 -+ s0/2
//   PPM (Colella & Woodward 1984, with limited slopes s_j of cells j = -1, 0, +1):
//     qL = (q[-1] + q0)/2 - (s0 - s[-1])/6,  qR = (q0 + q[+1])/2 - (s[+1] - s0)/6,
//     then the monotonicity constraints: qL = qR = q0 if q0 is a local extremum
//     ((qR - q0)(q0 - qL) <= 0); else with dq = qR - qL, q6 = 6(q0 - (qL+qR)/2):
//     qL = 3 q0 - 2 qR if dq q6 > dq^2, qR = 3 q0 - 2 qL if -dq^2 > dq q6.
// First order: both faces take the cell value.
template <class T>
void face_values(const T* const Ws[5], int d, double gamma, double theta, int scheme, T Wf[2][5]) {
  const T* Wc = Ws[2];
  if (scheme & FIRST_ORDER_BIT) {
    for (int q = 0; q < 5; ++q) Wf[0][q] = Wf[1][q] = Wc[q];
    return;
  }
  if (!(scheme & PPM_BIT)) {
    T s[5];
    limited_slopes(Ws[1], Wc, Ws[3], d, gamma, theta, scheme, s);
    for (int q = 0; q < 5; ++q) {
      Wf[0][q] = Wc[q] - T(0.5) * s[q];
      Wf[1][q] = Wc[q] + T(0.5) * s[q];
    }
    return;
  }
  T sm[5], s0[5], sp[5];
  limited_slopes(Ws[0], Ws[1], Ws[2], d, gamma, theta, scheme, sm);
  limited_slopes(Ws[1], Ws[2], Ws[3], d, gamma, theta, scheme, s0);
  limited_slopes(Ws[2], Ws[3], Ws[4], d, gamma, theta, scheme, sp);
  for (int q = 0; q < 5; ++q) ppm_scalar(Ws[1][q], Wc[q], Ws[3][q], sm[q], s0[q], sp[q], Wf[0][q], Wf[1][q]);
}

// Face values of a passively advected scalar q (the stencil q[0..4] at cells
// -2..+2), reconstructed as a primitive variable whatever the characteristic
// option (it is a wave of its own, moving with the flow).
template <class T>
void passive_face_values(const T q[5], double theta, int scheme, T out[2]) {
  if (scheme & FIRST_ORDER_BIT) {
    out[0] = out[1] = q[2];
    return;
  }
  const int lim = (scheme >> LIMITER_SHIFT) & 3;
  auto slope = [&](int j) { return limit_diffs(q[j] - q[j - 1], q[j + 1] - q[j], T(0.5) * (q[j + 1] - q[j - 1]), theta, lim); };
  if (!(scheme & PPM_BIT)) {
    const T sl = slope(2);
    out[0] = q[2] - T(0.5) * sl;
    out[1] = q[2] + T(0.5) * sl;
    return;
  }
  ppm_scalar(q[1], q[2], q[3], slope(1), slope(2), slope(3), out[0], out[1]);
}

// Normal-frame quantities of a face's two conserved states (shared by the
// HLLE and Roe solvers below; the HLLC solver above keeps its own copy).
template <class T>
struct FacePair {
  int n, t1, t2;
  T L[5], R[5];  // (rho, m_n, m_t1, m_t2, E)
  T rL, rR, uL, vL, wL, uR, vR, wR, pL, pR, cL, cR;
  bool bad;
  FacePair(const T UL[5], const T UR[5], int d, double gamma)
      : n(1 + d), t1(1 + (d + 1) % 3), t2(1 + (d + 2) % 3) {
    const T gm1 = T(gamma - 1.0), g = T(gamma);
    L[0] = UL[0]; L[1] = UL[n]; L[2] = UL[t1]; L[3] = UL[t2]; L[4] = UL[4];
    R[0] = UR[0]; R[1] = UR[n]; R[2] = UR[t1]; R[3] = UR[t2]; R[4] = UR[4];
    rL = L[0];
    rR = R[0];
    uL = L[1] / rL; vL = L[2] / rL; wL = L[3] / rL;
    uR = R[1] / rR; vR = R[2] / rR; wR = R[3] / rR;
    pL = gm1 * (L[4] - T(0.5) * rL * (uL * uL + vL * vL + wL * wL));
    pR = gm1 * (R[4] - T(0.5) * rR * (uR * uR + vR * vR + wR * wR));
    bad = !(val(rL) > 0.0 && val(pL) > 0.0 && val(rR) > 0.0 && val(pR) > 0.0);
    cL = tsqrt(g * pL / rL);
    cR = tsqrt(g * pR / rR);
  }
  void fluxes(T FL[5], T FR[5]) const {
    FL[0] = L[1]; FL[1] = L[1] * uL + pL; FL[2] = L[2] * uL; FL[3] = L[3] * uL; FL[4] = (L[4] + pL) * uL;
    FR[0] = R[1]; FR[1] = R[1] * uR + pR; FR[2] = R[2] * uR; FR[3] = R[3] * uR; FR[4] = (R[4] + pR) * uR;
  }
  void store(const T Fn[5], T F[5]) const {
    F[0] = Fn[0];
    F[n] = Fn[1];
    F[t1] = Fn[2];
    F[t2] = Fn[3];
    F[4] = Fn[4];
  }
};

// HLLE flux (Einfeldt 1988): wave speeds as in the HLLC solver (Einfeldt/Roe
// by default, Davis as an option), then
//   F = F_L if S_L >= 0;  F_R if S_R <= 0;
//   else (S_R F_L - S_L F_R + S_L S_R (U_R - U_L)) / (S_R - S_L).
template <class T>
bool hlle_flux(const T UL[5], const T UR[5], int d, double gamma, int wavespeed, T F[5]) {
  const FacePair<T> f(UL, UR, d, gamma);
  const T gm1 = T(gamma - 1.0);
  T SL, SR;
  if (wavespeed == 1) {
    SL = tmin(f.uL - f.cL, f.uR - f.cR);
    SR = tmax(f.uL + f.cL, f.uR + f.cR);
  } else {
    const T sL = tsqrt(f.rL), sR = tsqrt(f.rR);
    const T inv = T(1.0) / (sL + sR);
    const T ut = (sL * f.uL + sR * f.uR) * inv;
    const T vt = (sL * f.vL + sR * f.vR) * inv;
    const T wt = (sL * f.wL + sR * f.wR) * inv;
    const T HL = (f.L[4] + f.pL) / f.rL, HR = (f.R[4] + f.pR) / f.rR;
    const T Ht = (sL * HL + sR * HR) * inv;
    const T ct = tsqrt(gm1 * (Ht - T(0.5) * (ut * ut + vt * vt + wt * wt)));
    SL = tmin(f.uL - f.cL, ut - ct);
    SR = tmax(f.uR + f.cR, ut + ct);
  }
  T FL[5], FR[5], Fn[5];
  f.fluxes(FL, FR);
  sig_mix(val(SL) >= 0.0 ? 20 : val(SR) <= 0.0 ? 21 : 22);
  if (val(SL) >= 0.0) {
    for (int q = 0; q < 5; ++q) Fn[q] = FL[q];
  } else if (val(SR) <= 0.0) {
    for (int q = 0; q < 5; ++q) Fn[q] = FR[q];
  } else {
    const T inv = T(1.0) / (SR - SL);
    for (int q = 0; q < 5; ++q) Fn[q] = (SR * FL[q] - SL * FR[q] + SL * SR * (f.R[q] - f.L[q])) * inv;
  }
  f.store(Fn, F);
  return f.bad;
}

// Roe's flux (Roe 1981; wave strengths in the form of Toro 2009, Sec. 11.3):
// Roe averages u~, v~, w~, H~ (weights sqrt(rho)), a~^2 = (gamma-1)(H~ - q~^2/2);
// eigenvalues u~ - a~, u~ (x3), u~ + a~ with right eigenvectors
//   K1 = (1, u~-a~, v~, w~, H~ - u~ a~),  K2 = (1, u~, v~, w~, q~^2/2),
//   K3 = (0, 0, 1, 0, v~),  K4 = (0, 0, 0, 1, w~),  K5 = (1, u~+a~, v~, w~, H~ + u~ a~);
// strengths from dU = U_R - U_L:
//   al3 = dU2 - v~ dU0,  al4 = dU3 - w~ dU0,
//   al2 = (gamma-1)/a~^2 [dU0 (H~ - u~^2) + u~ dU1 - (dU4 - al3 v~ - al4 w~)],
//   al1 = [dU0 (u~ + a~) - dU1 - a~ al2] / (2 a~),  al5 = dU0 - (al1 + al2);
//   F = (F_L + F_R)/2 - (|l1| al1 K1 + |u~| (al2 K2 + al3 K3 + al4 K4) + |l5| al5 K5)/2.
// No entropy fix.  The states between the waves, U_L + al1 K1 and
// U_L + al1 K1 + al2 K2 + al3 K3 + al4 K4, are checked: if a~^2 <= 0 or either
// has rho <= 0 or p <= 0, the face's flux is recomputed with the HLLC solver
// (the first step of the paper's procedure for unphysical results).
template <class T>
bool roe_flux(const T UL[5], const T UR[5], int d, double gamma, int wavespeed, T F[5]) {
  const FacePair<T> f(UL, UR, d, gamma);
  const T gm1 = T(gamma - 1.0);
  const T sL = tsqrt(f.rL), sR = tsqrt(f.rR);
  const T inv = T(1.0) / (sL + sR);
  const T ut = (sL * f.uL + sR * f.uR) * inv;
  const T vt = (sL * f.vL + sR * f.vR) * inv;
  const T wt = (sL * f.wL + sR * f.wR) * inv;
  const T HL = (f.L[4] + f.pL) / f.rL, HR = (f.R[4] + f.pR) / f.rR;
  const T Ht = (sL * HL + sR * HR) * inv;
  const T q2 = ut * ut + vt * vt + wt * wt;
  const T a2 = gm1 * (Ht - T(0.5) * q2);
  bool ok = val(a2) > 0.0;
  T Fn[5];
  if (ok) {
    const T a = tsqrt(a2);
    T dU[5];
    for (int q = 0; q < 5; ++q) dU[q] = f.R[q] - f.L[q];
    const T al3 = dU[2] - vt * dU[0];
    const T al4 = dU[3] - wt * dU[0];
    const T al2 = gm1 / a2 * (dU[0] * (Ht - ut * ut) + ut * dU[1] - (dU[4] - al3 * vt - al4 * wt));
    const T al1 = (dU[0] * (ut + a) - dU[1] - a * al2) / (T(2.0) * a);
    const T al5 = dU[0] - (al1 + al2);
    const T K1[5] = {T(1.0), ut - a, vt, wt, Ht - ut * a};
    const T K2[5] = {T(1.0), ut, vt, wt, T(0.5) * q2};
    const T K3[5] = {T(0.0), T(0.0), T(1.0), T(0.0), vt};
    const T K4[5] = {T(0.0), T(0.0), T(0.0), T(1.0), wt};
    const T K5[5] = {T(1.0), ut + a, vt, wt, Ht + ut * a};
    // states between the waves
    T S1[5], S2[5];
    for (int q = 0; q < 5; ++q) {
      S1[q] = f.L[q] + al1 * K1[q];
      S2[q] = S1[q] + ((al2 * K2[q] + al3 * K3[q]) + al4 * K4[q]);
    }
    for (const T* S : {S1, S2}) {
      const T p = gm1 * (S[4] - T(0.5) * (S[1] * S[1] + S[2] * S[2] + S[3] * S[3]) / S[0]);
      if (!(val(S[0]) > 0.0 && val(p) > 0.0)) ok = false;
    }
    if (ok) {
      const T l1 = tabs(ut - a), l2 = tabs(ut), l5 = tabs(ut + a);
      T FL[5], FR[5];
      f.fluxes(FL, FR);
      for (int q = 0; q < 5; ++q) {
        const T diss = (l1 * al1 * K1[q] + l2 * ((al2 * K2[q] + al3 * K3[q]) + al4 * K4[q])) + l5 * al5 * K5[q];
        Fn[q] = T(0.5) * (FL[q] + FR[q]) - T(0.5) * diss;
      }
    }
  }
  sig_mix(ok ? 23 : 24);
  if (!ok) return hllc_flux(UL, UR, d, gamma, wavespeed, F);
  f.store(Fn, F);
  return f.bad;
}

template <class T>
bool riemann_flux(const T UL[5], const T UR[5], int d, double gamma, int scheme, T F[5]) {
  const int ws = (scheme >> WAVESPEED_SHIFT) & 3;
  switch ((scheme >> RIEMANN_SHIFT) & 3) {
    case 1: return roe_flux(UL, UR, d, gamma, ws, F);
    case 2: return hlle_flux(UL, UR, d, gamma, ws, F);
    default: return hllc_flux(UL, UR, d, gamma, ws, F);
  }
}

// Riemann flux of the nf = 5 Euler fields, plus, for nf = 6, the flux of a
// passive scalar carried by mass: F_5 = F_rho * (s/rho of the upwind side,
// by the sign of the mass flux).
template <class T>
bool riemann_nf(const T UL[], const T UR[], int d, double gamma, int scheme, int nf, T F[]) {
  const bool bad = riemann_flux(UL, UR, d, gamma, scheme, F);
  if (nf == 6) {
    const bool left = val(F[0]) >= 0.0;
    sig_mix(left ? 25 : 26);
    F[5] = F[0] * (left ? UL[5] / UL[0] : UR[5] / UR[0]);
  }
  return bad;
}

// Cons and flux of a primitive face state.
template <class T>
void face_cons_flux(const T W[5], int d, double gamma, T U[5], T F[5]) {
  prim_to_cons(W, gamma, U);
  euler_flux(W, U, d, F);
}

inline int recon_radius(int scheme) {
  if (scheme & FIRST_ORDER_BIT) return 0;
  return (scheme & PPM_BIT) ? 2 : 1;
}

// One step of a padded block with any of the schemes above.
//   MHM: face values (PLM/PPM, primitive/characteristic) -> conservative
//        Hancock half step with the face values' fluxes summed over x, y, z
//        (as hancock_cell) -> Riemann solve at every face -> update.
//   CTU (Colella 1990, the variant with 6 Riemann solves per cell):
//     1. along each axis d, face values and a half step with that axis' flux
//        difference only: U1_{d,-+} = U_{d,-+} + dt/(2dx) (F_d(U_{d,-}) - F_d(U_{d,+}));
//     2. first Riemann solves on every face between two such cells (3 per cell);
//     3. transverse correction of each axis' states with the other axes'
//        first-solve fluxes:
//          U2_{d,-+} = U1_{d,-+} - dt/(2dx) sum_{e != d} (F1_e(+1/2) - F1_e(-1/2))
//        (e ascending);
//     4. second Riemann solves with the corrected states (3 per cell);
//     5. conservative update with the second-solve fluxes.
// Needs ghost >= 2 (PLM) or 3 (PPM); the update order and unphysical count
// are those of mhm_step_block.
// Dual energy (the scheme word's bit 18; Sec. 2.2): a sixth field, the
// entropy per unit volume s = p / rho^(gamma-1), is advected as a passive
// scalar -- its specific value s/rho reconstructed like the primitive
// variables, its face values s = rho * (s/rho), its flux s u_n in the half
// steps and the mass flux times s/rho of the upwind side in the Riemann
// solves -- and after the update E is taken from s where E_th < xi E_kin,
// while s is reset from E elsewhere.
// face_flux (optional, 16^3 blocks only): the fluxes of the faces on the
// patch boundaries, [9][5][16][16]: plane p = 3 * axis + k holds the faces of
// that axis at normal coordinate 8 k (the face between 8k - 1 and 8k), entry
// [p][q][b][a] with (a, b) the transverse coordinates in the cyclic order
// (axis + 1, axis + 2).
template <class T>
int64_t step_block_any(const T* Upad, T* Uout, const Block& b, double dt, double dx, double gamma, double theta,
                       int scheme, T* face_flux = nullptr, double xi = 0.01) {
  const bool ctu = (scheme & SCHEME_ID_MASK) == SCHEME_CTU;
  const bool de = (scheme & DUAL_ENERGY_BIT) != 0;
  const int nf = de ? 6 : 5;
  const int R = recon_radius(scheme);
  const T dtdx = T(dt) / T(dx);
  const T half_dtdx = T(0.5) * dtdx;
  int64_t n_bad = 0;
  const int ex[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};

  // primitive variables on [-1-R, n+R]^3
  const int m = R + 1;
  const int wx = b.nx + 2 * m, wy = b.ny + 2 * m, wz = b.nz + 2 * m;
  auto wi = [&](int x, int y, int z) { return ((int64_t(z + m) * wy + (y + m)) * wx + (x + m)); };
  std::vector<T> W(size_t(wx) * wy * wz * nf);
  for (int z = -m; z < b.nz + m; ++z)
    for (int y = -m; y < b.ny + m; ++y)
      for (int x = -m; x < b.nx + m; ++x) {
        T U[5];
        for (int f = 0; f < 5; ++f) U[f] = Upad[b.at(f, x, y, z)];
        cons_to_prim(U, gamma, &W[wi(x, y, z) * nf]);
        if (de) W[wi(x, y, z) * nf + 5] = Upad[b.at(5, x, y, z)] / U[0];  // entropy per unit mass
      }

  // face states of every cell of [-1, n]^3: MHM's Hancock states, or CTU's
  // one-axis predicted states
  const int sx = b.nx + 2, sy = b.ny + 2, sz = b.nz + 2;
  auto si = [&](int x, int y, int z) { return ((int64_t(z + 1) * sy + (y + 1)) * sx + (x + 1)); };
  std::vector<T> S(size_t(sx) * sy * sz * 6 * nf);
  for (int z = -1; z < b.nz + 1; ++z)
    for (int y = -1; y < b.ny + 1; ++y)
      for (int x = -1; x < b.nx + 1; ++x) {
        T Wf[3][2][5], Pf[3][2];
        for (int d = 0; d < 3; ++d) {
          const T* Ws[5];
          T ph[5];
          for (int j = -2; j <= 2; ++j) {
            const int o = (j < -R || j > R) ? 0 : j;  // cells beyond the radius are not read
            Ws[j + 2] = &W[wi(x + o * ex[d][0], y + o * ex[d][1], z + o * ex[d][2]) * nf];
            if (de) ph[j + 2] = Ws[j + 2][5];
          }
          face_values(Ws, d, gamma, theta, scheme, Wf[d]);
          if (de) passive_face_values(ph, theta, scheme, Pf[d]);
        }
        T Ut[3][2][6], Ff[3][2][6];
        for (int d = 0; d < 3; ++d)
          for (int s = 0; s < 2; ++s) {
            face_cons_flux(Wf[d][s], d, gamma, Ut[d][s], Ff[d][s]);
            if (de) {
              Ut[d][s][5] = Wf[d][s][0] * Pf[d][s];
              Ff[d][s][5] = Ut[d][s][5] * Wf[d][s][1 + d];
            }
          }
        if (ctu) {
          for (int d = 0; d < 3; ++d)
            for (int q = 0; q < nf; ++q) {
              const T dU = half_dtdx * (Ff[d][0][q] - Ff[d][1][q]);
              Ut[d][0][q] = Ut[d][0][q] + dU;
              Ut[d][1][q] = Ut[d][1][q] + dU;
            }
        } else {
          for (int q = 0; q < nf; ++q) {
            T s = Ff[0][0][q] - Ff[0][1][q];
            s = s + (Ff[1][0][q] - Ff[1][1][q]);
            s = s + (Ff[2][0][q] - Ff[2][1][q]);
            const T dU = half_dtdx * s;
            for (int d = 0; d < 3; ++d) {
              Ut[d][0][q] = Ut[d][0][q] + dU;
              Ut[d][1][q] = Ut[d][1][q] + dU;
            }
          }
        }
        T* dst = &S[si(x, y, z) * 6 * nf];
        for (int d = 0; d < 3; ++d)
          for (int s = 0; s < 2; ++s)
            for (int q = 0; q < nf; ++q) dst[(d * 2 + s) * nf + q] = Ut[d][s][q];
      }
  auto state = [&](int x, int y, int z, int d, int s) -> T* { return &S[si(x, y, z) * 6 * nf + (d * 2 + s) * nf]; };

  if (ctu) {
    // first solves on faces between two cells of [-1, n]^3: face (d, x, y, z)
    // lies between the cell at (x, y, z) - e_d and (x, y, z), for the normal
    // coordinate 0..n and the transverse ones -1..n
    auto f1i = [&](int d, int x, int y, int z) {
      return (((int64_t(d) * (b.nz + 2) + (z + 1)) * (b.ny + 2) + (y + 1)) * (b.nx + 2) + (x + 1)) * nf;
    };
    std::vector<T> F1(size_t(3) * (b.nx + 2) * (b.ny + 2) * (b.nz + 2) * nf);
    for (int d = 0; d < 3; ++d)
      for (int z = -1; z <= b.nz; ++z)
        for (int y = -1; y <= b.ny; ++y)
          for (int x = -1; x <= b.nx; ++x) {
            const int c[3] = {x, y, z};
            if (c[d] < 0) continue;
            const int lx = x - ex[d][0], ly = y - ex[d][1], lz = z - ex[d][2];
            riemann_nf(state(lx, ly, lz, d, 1), state(x, y, z, d, 0), d, gamma, scheme, nf, &F1[f1i(d, x, y, z)]);
          }
    // transverse corrections of the states the second solves need: axis d's
    // states of cells with the normal coordinate in -1..n and the transverse
    // ones in 0..n-1
    for (int d = 0; d < 3; ++d)
      for (int z = -1; z <= b.nz; ++z)
        for (int y = -1; y <= b.ny; ++y)
          for (int x = -1; x <= b.nx; ++x) {
            const int c[3] = {x, y, z}, nn[3] = {b.nx, b.ny, b.nz};
            bool inside = true;
            for (int e = 0; e < 3; ++e)
              if (e != d && (c[e] < 0 || c[e] >= nn[e])) inside = false;
            if (!inside) continue;
            T corr[6];
            bool first = true;
            for (int e = 0; e < 3; ++e) {
              if (e == d) continue;
              const T* Fp = &F1[f1i(e, x + ex[e][0], y + ex[e][1], z + ex[e][2])];
              const T* Fm = &F1[f1i(e, x, y, z)];
              for (int q = 0; q < nf; ++q) corr[q] = first ? (Fp[q] - Fm[q]) : corr[q] + (Fp[q] - Fm[q]);
              first = false;
            }
            for (int s = 0; s < 2; ++s) {
              T* st = state(x, y, z, d, s);
              for (int q = 0; q < nf; ++q) st[q] = st[q] - half_dtdx * corr[q];
            }
          }
  }

  // (second) Riemann solves at the faces of the interior cells, update
  auto fxi = [&](int x, int y, int z) { return ((int64_t(z) * b.ny + y) * (b.nx + 1) + x) * nf; };
  auto fyi = [&](int x, int y, int z) { return ((int64_t(z) * (b.ny + 1) + y) * b.nx + x) * nf; };
  auto fzi = [&](int x, int y, int z) { return ((int64_t(z) * b.ny + y) * b.nx + x) * nf; };
  std::vector<T> Fx(size_t(b.nz) * b.ny * (b.nx + 1) * nf), Fy(size_t(b.nz) * (b.ny + 1) * b.nx * nf),
      Fz(size_t(b.nz + 1) * b.ny * b.nx * nf);
  for (int z = 0; z < b.nz; ++z)
    for (int y = 0; y < b.ny; ++y)
      for (int x = 0; x <= b.nx; ++x)
        n_bad += riemann_nf(state(x - 1, y, z, 0, 1), state(x, y, z, 0, 0), 0, gamma, scheme, nf, &Fx[fxi(x, y, z)]);
  for (int z = 0; z < b.nz; ++z)
    for (int y = 0; y <= b.ny; ++y)
      for (int x = 0; x < b.nx; ++x)
        n_bad += riemann_nf(state(x, y - 1, z, 1, 1), state(x, y, z, 1, 0), 1, gamma, scheme, nf, &Fy[fyi(x, y, z)]);
  for (int z = 0; z <= b.nz; ++z)
    for (int y = 0; y < b.ny; ++y)
      for (int x = 0; x < b.nx; ++x)
        n_bad += riemann_nf(state(x, y, z - 1, 2, 1), state(x, y, z, 2, 0), 2, gamma, scheme, nf, &Fz[fzi(x, y, z)]);
  if (face_flux != nullptr) {
    for (int k = 0; k < 3; ++k)
      for (int q = 0; q < 5; ++q)
        for (int bb = 0; bb < 16; ++bb)
          for (int a = 0; a < 16; ++a) {
            const int n = 8 * k;
            face_flux[((0 * 3 + k) * 5 + q) * 256 + bb * 16 + a] = Fx[fxi(n, a, bb) + q];   // a = y, b = z
            face_flux[((1 * 3 + k) * 5 + q) * 256 + bb * 16 + a] = Fy[fyi(bb, n, a) + q];   // a = z, b = x
            face_flux[((2 * 3 + k) * 5 + q) * 256 + bb * 16 + a] = Fz[fzi(a, bb, n) + q];   // a = x, b = y
          }
  }
  const T gm1 = T(gamma - 1.0);
  for (int z = 0; z < b.nz; ++z)
    for (int y = 0; y < b.ny; ++y)
      for (int x = 0; x < b.nx; ++x) {
        T Un[6];
        for (int q = 0; q < nf; ++q) {
          T acc = Fx[fxi(x + 1, y, z) + q] - Fx[fxi(x, y, z) + q];
          acc = acc + (Fy[fyi(x, y + 1, z) + q] - Fy[fyi(x, y, z) + q]);
          acc = acc + (Fz[fzi(x, y, z + 1) + q] - Fz[fzi(x, y, z) + q]);
          Un[q] = Upad[b.at(q, x, y, z)] - dtdx * acc;
        }
        if (de) {
          // dual energy (Sec. 2.2): where the thermal energy from the total
          // energy is below xi times the kinetic energy, take it from the
          // entropy, p = s rho^(gamma-1); elsewhere the entropy is set from
          // the total energy
          const T ekin = T(0.5) * (Un[1] * Un[1] + Un[2] * Un[2] + Un[3] * Un[3]) / Un[0];
          const T eth = Un[4] - ekin;
          const T rg = tpow(Un[0], gamma - 1.0);
          const bool use_s = val(eth) < xi * val(ekin);
          sig_mix(use_s ? 27 : 28);
          if (use_s) Un[4] = Un[5] * rg / gm1 + ekin;
          else Un[5] = gm1 * eth / rg;
        }
        for (int q = 0; q < nf; ++q) Uout[((int64_t(q) * b.nz + z) * b.ny + y) * b.nx + x] = Un[q];
        const T p = gm1 * (Un[4] - T(0.5) * (Un[1] * Un[1] + Un[2] * Un[2] + Un[3] * Un[3]) / Un[0]);
        if (!(val(Un[0]) > 0.0 && val(p) > 0.0)) ++n_bad;
      }
  return n_bad;
}

// ------------------------------------- procedure for unphysical results ---
// Sec. 2.2: (ii) a cell whose update gives rho <= 0 or p <= 0 is recomputed
// first-order in space and time, dimensionally unsplit; (iii) if that still
// fails, first-order and dimensionally split; (iv)-(v) if that fails too, the
// whole level is recomputed with the time-step reduced by a fixed ratio (0.8)
// until nothing fails or the step falls below a minimum.  Steps (ii)-(iii)
// touch only the failed cells.
//   first-order unsplit: U = U^n - dt/dx sum_d (F_d(+1/2) - F_d(-1/2)), F the
//     scheme's Riemann solver on the neighbouring cell averages of U^n;
//   first-order split: x sweep of U^n, then y sweep of the result, then z
//     sweep, each U' = U - dt/dx (F(+1/2) - F(-1/2)) of the sweep's axis; the
//     split update of a cell reads the 3x3x3 block of U^n around it.
template <class T>
bool cons_unphysical(const T U[5], double gamma) {
  const T p = T(gamma - 1.0) * (U[4] - T(0.5) * (U[1] * U[1] + U[2] * U[2] + U[3] * U[3]) / U[0]);
  return !(val(U[0]) > 0.0 && val(p) > 0.0);
}

// Level accessor: cell (X, Y, Z) of the level (global cell indices, mapped
// through the boundary conditions) into U[5].
struct LevelView {
  const double* level;
  int ngx, ngy, ngz;
  const int* bc;
  void get(int X, int Y, int Z, double U[5]) const {
    X = bc_index(X, ngx * 16, bc[0], bc[1]);
    Y = bc_index(Y, ngy * 16, bc[2], bc[3]);
    Z = bc_index(Z, ngz * 16, bc[4], bc[5]);
    const int64_t g = (int64_t(Z / 16) * ngy + Y / 16) * ngx + X / 16;
    for (int f = 0; f < 5; ++f) U[f] = level[((g * 5 + f) * 16 + Z % 16) * 256 + (Y % 16) * 16 + X % 16];
  }
};

void first_order_unsplit(const LevelView& lv, int X, int Y, int Z, double dtdx, double gamma, int scheme,
                         double out[5]) {
  const int ex[3][3] = {{1, 0, 0}, {0, 1, 0}, {0, 0, 1}};
  double U0[5];
  lv.get(X, Y, Z, U0);
  double acc[5];
  for (int d = 0; d < 3; ++d) {
    double Um[5], Up[5], Fm[5], Fp[5];
    lv.get(X - ex[d][0], Y - ex[d][1], Z - ex[d][2], Um);
    lv.get(X + ex[d][0], Y + ex[d][1], Z + ex[d][2], Up);
    riemann_flux(Um, U0, d, gamma, scheme, Fm);
    riemann_flux(U0, Up, d, gamma, scheme, Fp);
    for (int q = 0; q < 5; ++q) acc[q] = d == 0 ? (Fp[q] - Fm[q]) : acc[q] + (Fp[q] - Fm[q]);
  }
  for (int q = 0; q < 5; ++q) out[q] = U0[q] - dtdx * acc[q];
}

void first_order_split(const LevelView& lv, int X, int Y, int Z, double dtdx, double gamma, int scheme,
                       double out[5]) {
  // B[k][j][i][q]: the 3x3x3 block around the cell, offsets -1..1
  double B[3][3][3][5], C[3][3][3][5];
  for (int k = 0; k < 3; ++k)
    for (int j = 0; j < 3; ++j)
      for (int i = 0; i < 3; ++i) lv.get(X + i - 1, Y + j - 1, Z + k - 1, B[k][j][i]);
  auto sweep1 = [&](const double* Um, const double* U0, const double* Up, int d, double* res) {
    double Fm[5], Fp[5];
    riemann_flux(Um, U0, d, gamma, scheme, Fm);
    riemann_flux(U0, Up, d, gamma, scheme, Fp);
    for (int q = 0; q < 5; ++q) res[q] = U0[q] - dtdx * (Fp[q] - Fm[q]);
  };
  // x sweep on the 9 centre-x cells of every (y, z) line of the block (only
  // the x = 0 column is needed: its y and z neighbours feed the next sweeps)
  for (int k = 0; k < 3; ++k)
    for (int j = 0; j < 3; ++j) sweep1(B[k][j][0], B[k][j][1], B[k][j][2], 0, C[k][j][1]);
  // y sweep at y = 0 for z = -1..1
  double D[3][5];
  for (int k = 0; k < 3; ++k) sweep1(C[k][0][1], C[k][1][1], C[k][2][1], 1, D[k]);
  // z sweep at the cell
  sweep1(D[0], D[1], D[2], 2, out);
}

// One step of a level with the procedure for unphysical results applied to
// its output (steps ii-iii).  Returns the number of cells still unphysical;
// *n_unsplit / *n_split receive how many cells each step repaired.
int64_t level_step_repaired(const double* level, double* level_out, int ngx, int ngy, int ngz, int ghost,
                            const int bc[6], double dt, double dx, double gamma, double theta, int scheme,
                            int64_t* n_unsplit, int64_t* n_split) {
  const int P = 16 + 2 * ghost;
  const int64_t G = int64_t(ngx) * ngy * ngz;
  std::vector<double> pad(size_t(G) * 5 * P * P * P);
  fill_ghosts(level, pad.data(), ngx, ngy, ngz, ghost, bc);
  const Block b(16, 16, 16, ghost);
#pragma omp parallel for schedule(static)
  for (int64_t g = 0; g < G; ++g)
    step_block_any(pad.data() + g * b.cells() * 5, level_out + g * 5 * 4096, b, dt, dx, gamma, theta, scheme);
  const LevelView lv{level, ngx, ngy, ngz, bc};
  const double dtdx = dt / dx;
  int64_t left = 0, nu = 0, ns = 0;
  // first-order procedure: Riemann solver of the scheme, zero slopes
  const int fo = scheme | FIRST_ORDER_BIT;
  for (int64_t g = 0; g < G; ++g)
    for (int c = 0; c < 4096; ++c) {
      double U[5];
      for (int f = 0; f < 5; ++f) U[f] = level_out[(g * 5 + f) * 4096 + c];
      if (!cons_unphysical(U, gamma)) continue;
      const int gx = int(g % ngx), gy = int((g / ngx) % ngy), gz = int(g / (int64_t(ngx) * ngy));
      const int X = gx * 16 + c % 16, Y = gy * 16 + (c / 16) % 16, Z = gz * 16 + c / 256;
      double R[5];
      first_order_unsplit(lv, X, Y, Z, dtdx, gamma, fo, R);
      if (!cons_unphysical(R, gamma)) {
        ++nu;
      } else {
        first_order_split(lv, X, Y, Z, dtdx, gamma, fo, R);
        if (!cons_unphysical(R, gamma)) ++ns;
        else ++left;
      }
      for (int f = 0; f < 5; ++f) level_out[(g * 5 + f) * 4096 + c] = R[f];
    }
  if (n_unsplit) *n_unsplit = nu;
  if (n_split) *n_split = ns;
  return left;
}

// ===================================================== coarse-fine coupling ==
// Sec. 2.1 (AMR: patches of 8^3 cells, refinement ratio 2, groups of 2x2x2
// sibling patches, levels advanced in a W-cycle with dt_l = dt_0 / 2^l) and
// Sec. 2.2 (fix-up operations): the children of one coarse patch form one
// fine patch group (16^3 fine cells over 8^3 coarse cells).  A level is a set
// of groups at positions of its group lattice (level l: n_0 * 2^l groups per
// axis over the domain); level 0 covers the domain.
//   ghost zones of a fine group: copied from the sibling group that holds the
//     cell, else interpolated from the coarse level (conservative linear
//     interpolation: coarse value plus the minmod-limited slopes of the
//     conserved variables times the child's offset of +-1/4 coarse cell,
//     summed x, y, z), with the coarse state taken linearly in time between
//     the coarse step's input and output: (1 - a) U_old + a U_new;
//   flux registers: the time- and area-average of the fine fluxes over each
//     coarse face of the fine level's boundary, accumulated over the fine
//     substeps as sum_s (dt_f / dt_c) (1/4) (sum of the 2x2 fine faces);
//   restriction: a coarse cell covered by a fine group becomes the mean of
//     its 8 children;
//   fix-up: an uncovered coarse cell next to the fine region replaces the
//     coarse flux of that face by the register's, U += dt_c/dx_c (R - F_c)
//     on its low face, -= on its high face, faces taken x-, x+, y-, y+, z-, z+.
// Readings (the paper states the operations, not their formulas): the
// interpolation above, and refinement by whole coarse patches with at least
// one coarse patch of buffer (proper nesting), so that every coarse cell an
// interpolation reads exists.
struct AmrLevel {
  int n[3];            // group lattice of the level over the domain
  int64_t G;
  const int* pos;      // [G][3] group positions (x, y, z)
  std::vector<int> map;  // dense lattice -> group index or -1
  double* U;           // [G][5][16^3]
  void build_map() {
    map.assign(size_t(n[0]) * n[1] * n[2], -1);
    for (int64_t g = 0; g < G; ++g)
      map[(size_t(pos[3 * g + 2]) * n[1] + pos[3 * g + 1]) * n[0] + pos[3 * g]] = int(g);
  }
  int group_at(int gx, int gy, int gz) const { return map[(size_t(gz) * n[1] + gy) * n[0] + gx]; }
};

// Cell index along an axis of N cells through the boundary condition; -1 if
// it leaves the domain on an outflow face (clamped instead) is not needed:
// outflow clamps.
inline int amr_wrap(int i, int N, int lo, int hi) { return bc_index(i, N, lo, hi); }

// Value of cell (X, Y, Z) (global, already mapped) of a level: the group must exist.
inline const double* amr_cell(const AmrLevel& L, const double* U, int X, int Y, int Z, int64_t* g_out = nullptr) {
  const int g = L.group_at(X >> 4, Y >> 4, Z >> 4);
  if (g_out) *g_out = g;
  if (g < 0) return nullptr;
  return U + (int64_t(g) * 5) * 4096 + ((Z & 15) * 16 + (Y & 15)) * 16 + (X & 15);
}

inline double minmod2(double a, double b) {
  if (!(a * b > 0.0)) return 0.0;
  return std::fabs(a) < std::fabs(b) ? a : b;
}

// Interpolated value of fine cell (X, Y, Z) (global fine indices, mapped)
// from the coarse level at time weight a.
void amr_interp(const AmrLevel& C, const double* Uold, const double* Unew, double a, const int bc[6], int X, int Y,
                int Z, double out[5]) {
  const int N[3] = {16 * C.n[0], 16 * C.n[1], 16 * C.n[2]};
  const int c[3] = {X >> 1, Y >> 1, Z >> 1};
  const double off[3] = {(X & 1) ? 0.25 : -0.25, (Y & 1) ? 0.25 : -0.25, (Z & 1) ? 0.25 : -0.25};
  auto at = [&](int dx, int dy, int dz, double v[5]) {
    const int x = amr_wrap(c[0] + dx, N[0], bc[0], bc[1]);
    const int y = amr_wrap(c[1] + dy, N[1], bc[2], bc[3]);
    const int z = amr_wrap(c[2] + dz, N[2], bc[4], bc[5]);
    const double* o = amr_cell(C, Uold, x, y, z);
    const double* w = amr_cell(C, Unew, x, y, z);
    for (int q = 0; q < 5; ++q) v[q] = (1.0 - a) * o[q * 4096] + a * w[q * 4096];
  };
  double U0[5];
  at(0, 0, 0, U0);
  double s[3][5];
  for (int d = 0; d < 3; ++d) {
    double Um[5], Up[5];
    at(-(d == 0), -(d == 1), -(d == 2), Um);
    at(d == 0, d == 1, d == 2, Up);
    for (int q = 0; q < 5; ++q) s[d][q] = minmod2(U0[q] - Um[q], Up[q] - U0[q]);
  }
  for (int q = 0; q < 5; ++q) out[q] = ((U0[q] + s[0][q] * off[0]) + s[1][q] * off[1]) + s[2][q] * off[2];
}

// Padded blocks [G][5][P^3] of a level: cells from the level's own groups,
// else interpolated from the coarse level (level 0: own groups only).
void amr_fill(const AmrLevel& F, const AmrLevel* C, const double* Cold, const double* Cnew, double a, const int bc[6],
              int ghost, double* pad) {
  const int P = 16 + 2 * ghost;
  const int N[3] = {16 * F.n[0], 16 * F.n[1], 16 * F.n[2]};
#pragma omp parallel for schedule(static)
  for (int64_t g = 0; g < F.G; ++g)
    for (int z = 0; z < P; ++z)
      for (int y = 0; y < P; ++y)
        for (int x = 0; x < P; ++x) {
          const int X = amr_wrap(16 * F.pos[3 * g] + x - ghost, N[0], bc[0], bc[1]);
          const int Y = amr_wrap(16 * F.pos[3 * g + 1] + y - ghost, N[1], bc[2], bc[3]);
          const int Z = amr_wrap(16 * F.pos[3 * g + 2] + z - ghost, N[2], bc[4], bc[5]);
          const double* src = amr_cell(F, F.U, X, Y, Z);
          double v[5];
          if (src != nullptr) {
            for (int q = 0; q < 5; ++q) v[q] = src[q * 4096];
          } else {
            amr_interp(*C, Cold, Cnew, a, bc, X, Y, Z, v);
          }
          for (int q = 0; q < 5; ++q) pad[((g * 5 + q) * P + z) * int64_t(P) * P + int64_t(y) * P + x] = v[q];
        }
}

// Side s = 2 * axis + (0 low, 1 high) of a fine group has a coarse-fine
// interface if the group across it does not exist (a face on an outflow
// domain boundary has none).
bool amr_interface(const AmrLevel& F, int64_t g, int s, const int bc[6]) {
  const int d = s >> 1, hi = s & 1;
  int p[3] = {F.pos[3 * g], F.pos[3 * g + 1], F.pos[3 * g + 2]};
  p[d] += hi ? 1 : -1;
  if (p[d] < 0 || p[d] >= F.n[d]) {
    if (bc[2 * d + hi] != 0) return false;
    p[d] = (p[d] + F.n[d]) % F.n[d];
  }
  return F.group_at(p[0], p[1], p[2]) < 0;
}

// R[g][6][5][8][8] += w * (1/4) * (sum of the 2x2 fine faces) on interface sides.
void amr_accumulate(const AmrLevel& F, const double* face_flux, double w, const int bc[6], double* R) {
  for (int64_t g = 0; g < F.G; ++g)
    for (int s = 0; s < 6; ++s) {
      if (!amr_interface(F, g, s, bc)) continue;
      const int d = s >> 1, k = (s & 1) ? 2 : 0;
      const double* Fp = face_flux + (g * 9 + d * 3 + k) * 5 * 256;
      double* r = R + (g * 6 + s) * 5 * 64;
      for (int q = 0; q < 5; ++q)
        for (int j = 0; j < 8; ++j)
          for (int i = 0; i < 8; ++i) {
            const double* f = Fp + q * 256;
            const double sum = (f[(2 * j) * 16 + 2 * i] + f[(2 * j) * 16 + 2 * i + 1]) +
                               (f[(2 * j + 1) * 16 + 2 * i] + f[(2 * j + 1) * 16 + 2 * i + 1]);
            r[q * 64 + j * 8 + i] = r[q * 64 + j * 8 + i] + w * (0.25 * sum);
          }
    }
}

// Coarse cells covered by fine group g become the mean of their children.
void amr_restrict(const AmrLevel& F, AmrLevel& C) {
#pragma omp parallel for schedule(static)
  for (int64_t g = 0; g < F.G; ++g) {
    const int px = F.pos[3 * g], py = F.pos[3 * g + 1], pz = F.pos[3 * g + 2];  // = coarse patch
    const int gc = C.group_at(px >> 1, py >> 1, pz >> 1);
    for (int z = 0; z < 8; ++z)
      for (int y = 0; y < 8; ++y)
        for (int x = 0; x < 8; ++x) {
          const int cx = (px & 1) * 8 + x, cy = (py & 1) * 8 + y, cz = (pz & 1) * 8 + z;
          for (int q = 0; q < 5; ++q) {
            // pairwise: x pairs, then y, then z (a uniform state restricts exactly)
            auto ch = [&](int dx, int dy, int dz) {
              return F.U[(g * 5 + q) * 4096 + ((2 * z + dz) * 16 + (2 * y + dy)) * 16 + (2 * x + dx)];
            };
            const double s0 = (ch(0, 0, 0) + ch(1, 0, 0)) + (ch(0, 1, 0) + ch(1, 1, 0));
            const double s1 = (ch(0, 0, 1) + ch(1, 0, 1)) + (ch(0, 1, 1) + ch(1, 1, 1));
            C.U[(int64_t(gc) * 5 + q) * 4096 + (cz * 16 + cy) * 16 + cx] = 0.125 * (s0 + s1);
          }
        }
  }
}

// Fix-up of the uncovered coarse cells next to the fine level.
void amr_fixup(AmrLevel& C, const AmrLevel& F, const double* cface_flux, const double* R, double dtdx,
               const int bc[6]) {
  const int N[3] = {16 * C.n[0], 16 * C.n[1], 16 * C.n[2]};
  auto refined = [&](int X, int Y, int Z, int64_t* gf) {  // coarse cell's patch has children
    const int g = F.group_at(X >> 3, Y >> 3, Z >> 3);
    if (gf) *gf = g;
    return g >= 0;
  };
#pragma omp parallel for schedule(static)
  for (int64_t g = 0; g < C.G; ++g)
    for (int c = 0; c < 4096; ++c) {
      const int X = 16 * C.pos[3 * g] + (c & 15), Y = 16 * C.pos[3 * g + 1] + ((c >> 4) & 15),
                Z = 16 * C.pos[3 * g + 2] + (c >> 8);
      if (refined(X, Y, Z, nullptr)) continue;
      const int xyz[3] = {X, Y, Z};
      for (int s = 0; s < 6; ++s) {
        const int d = s >> 1, hi = s & 1;
        int nb[3] = {X, Y, Z};
        nb[d] += hi ? 1 : -1;
        if (nb[d] < 0 || nb[d] >= N[d]) {
          if (bc[2 * d + hi] != 0) continue;
          nb[d] = (nb[d] + N[d]) % N[d];
        }
        int64_t gf;
        if (!refined(nb[0], nb[1], nb[2], &gf)) continue;
        // coarse flux of the face: plane k of this cell's group (local normal
        // coordinate 0, 8 or 16)
        const int local = (xyz[d] & 15) + hi;
        const int k = local >> 3;
        const int a = xyz[(d + 1) % 3] & 15, b = xyz[(d + 2) % 3] & 15;
        const double* Fc = cface_flux + (g * 9 + d * 3 + k) * 5 * 256 + b * 16 + a;
        // the fine group's register on its side facing this cell
        const int fs = 2 * d + (hi ? 0 : 1);
        const int i = xyz[(d + 1) % 3] & 7, j = xyz[(d + 2) % 3] & 7;
        const double* r = R + (gf * 6 + fs) * 5 * 64 + j * 8 + i;
        for (int q = 0; q < 5; ++q) {
          const double corr = dtdx * (r[q * 64] - Fc[q * 256]);
          double& u = C.U[(g * 5 + q) * 4096 + c];
          u = hi ? u - corr : u + corr;
        }
      }
    }
}

// One step of a level from its padded blocks; face fluxes captured.
int64_t amr_step_level(AmrLevel& L, const double* pad, int ghost, double dt, double dx, double gamma, double theta,
                       int scheme, double* face_flux) {
  const Block b(16, 16, 16, ghost);
  int64_t n_bad = 0;
  std::vector<double> out(size_t(L.G) * 5 * 4096);
#pragma omp parallel for schedule(static) reduction(+ : n_bad)
  for (int64_t g = 0; g < L.G; ++g)
    n_bad += step_block_any(pad + g * b.cells() * 5, out.data() + g * 5 * 4096, b, dt, dx, gamma, theta, scheme,
                            face_flux + g * 9 * 5 * 256);
  std::memcpy(L.U, out.data(), sizeof(double) * out.size());
  return n_bad;
}

// Advance level l by dt (and, recursively, the finer levels by two steps of
// dt/2 each), given the coarse state before and after its current step
// (a0, a1: the time weights of this step's start and end within it).
int64_t amr_advance(std::vector<AmrLevel>& Ls, int l, double dt, double dx0, double gamma, double theta, int scheme,
                    int ghost, const int bc[6], const double* Cold, const double* Cnew, double a, double* R_parent) {
  AmrLevel& L = Ls[l];
  const double dx = dx0 / double(1 << l);
  const int P = 16 + 2 * ghost;
  std::vector<double> pad(size_t(L.G) * 5 * P * P * P), flux(size_t(L.G) * 9 * 5 * 256);
  std::vector<double> old(L.U, L.U + L.G * 5 * 4096);
  amr_fill(L, l > 0 ? &Ls[l - 1] : nullptr, Cold, Cnew, a, bc, ghost, pad.data());
  int64_t n_bad = amr_step_level(L, pad.data(), ghost, dt, dx, gamma, theta, scheme, flux.data());
  if (R_parent != nullptr) amr_accumulate(L, flux.data(), 0.5, bc, R_parent);
  if (l + 1 < int(Ls.size())) {
    std::vector<double> R(size_t(Ls[l + 1].G) * 6 * 5 * 64, 0.0);
    std::vector<double> nw(L.U, L.U + L.G * 5 * 4096);
    n_bad += amr_advance(Ls, l + 1, 0.5 * dt, dx0, gamma, theta, scheme, ghost, bc, old.data(), nw.data(), 0.0,
                         R.data());
    n_bad += amr_advance(Ls, l + 1, 0.5 * dt, dx0, gamma, theta, scheme, ghost, bc, old.data(), nw.data(), 0.5,
                         R.data());
    amr_restrict(Ls[l + 1], L);
    amr_fixup(L, Ls[l + 1], flux.data(), R.data(), dt / dx, bc);
  }
  return n_bad;
}

// Proper nesting: the 27 coarse patches around every fine group's parent
// patch exist on the coarse level (so every coarse cell a fine ghost zone or
// its interpolation slopes read exists).
bool amr_nested(const AmrLevel& F, const AmrLevel& C, const int bc[6]) {
  const int np[3] = {2 * C.n[0], 2 * C.n[1], 2 * C.n[2]};  // coarse patches per axis
  for (int64_t g = 0; g < F.G; ++g)
    for (int dz = -1; dz <= 1; ++dz)
      for (int dy = -1; dy <= 1; ++dy)
        for (int dx = -1; dx <= 1; ++dx) {
          int p[3] = {F.pos[3 * g] + dx, F.pos[3 * g + 1] + dy, F.pos[3 * g + 2] + dz};
          bool skip = false;
          for (int d = 0; d < 3; ++d)
            if (p[d] < 0 || p[d] >= np[d]) {
              if (bc[2 * d + (p[d] >= np[d])] != 0) skip = true;  // beyond an outflow face: clamped inside
              p[d] = (p[d] + np[d]) % np[d];
            }
          if (!skip && C.group_at(p[0] >> 1, p[1] >> 1, p[2] >> 1) < 0) return false;
        }
  return true;
}

}  // namespace

// =================================================================== C ABI ==
// Plain pointers to host memory, sizes as integers.  Return values: counts
// (>= 0) or -1 on bad arguments.
extern "C" {

// One MHM step of G padded 16^3 groups: Upad [G][5][P^3] -> Uout [G][5][16^3].
int64_t oracle_mhm_step(const double* Upad, double* Uout, int64_t G, int ghost, double dt, double dx,
                        double gamma, double theta, int scheme) {
  if (ghost < 2 || G < 0 || (scheme & SCHEME_ID_MASK) != SCHEME_MHM_PLM_HLLC) return -1;
  const Block b(16, 16, 16, ghost);
  int64_t n_bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : n_bad)
  for (int64_t g = 0; g < G; ++g)
    n_bad += mhm_step_block(Upad + g * b.cells() * 5, Uout + g * 5 * 4096, b, dt, dx, gamma, theta, scheme);
  return n_bad;
}

// One MHM step of a single padded block of arbitrary interior size.
int64_t oracle_mhm_step_block(const double* Upad, double* Uout, int nx, int ny, int nz, int ghost,
                              double dt, double dx, double gamma, double theta, int scheme) {
  if (ghost < 2 || nx < 1 || ny < 1 || nz < 1 || (scheme & SCHEME_ID_MASK) != SCHEME_MHM_PLM_HLLC)
    return -1;
  return mhm_step_block(Upad, Uout, Block(nx, ny, nz, ghost), dt, dx, gamma, theta, scheme);
}

// Per-patch CFL time-step of G padded groups: dt_patch[G*8], patch index
// p = (pz*2 + py)*2 + px inside each group.
int oracle_dt(const double* Upad, int64_t G, int ghost, double dx, double gamma, double c_cfl,
              double* dt_patch) {
  if (ghost < 0 || G < 0) return -1;
  const Block b(16, 16, 16, ghost);
#pragma omp parallel for schedule(static)
  for (int64_t g = 0; g < G; ++g)
    for (int p = 0; p < 8; ++p)
      dt_patch[g * 8 + p] = patch_dt(Upad + g * b.cells() * 5, b, 8 * (p & 1), 8 * ((p >> 1) & 1),
                                     8 * (p >> 2), dx, gamma, c_cfl);
  return 0;
}

int oracle_fill_ghosts(const double* level, double* Upad, int ngx, int ngy, int ngz, int ghost,
                       const int* bc) {
  if (ghost < 0 || ghost > 16 || ngx < 1 || ngy < 1 || ngz < 1) return -1;
  fill_ghosts(level, Upad, ngx, ngy, ngz, ghost, bc);
  return 0;
}

// n_steps steps of a level (group-major interiors), ghost fill every step.
// If dt_fixed > 0 every step uses it; otherwise each step takes the CFL
// time-step (min over patches of Eq. 2 with c_cfl).  dts[n_steps] receives
// the steps taken (may be null).  Returns the total unphysical count.
int64_t oracle_rollout(const double* level0, double* level_out, int ngx, int ngy, int ngz, int ghost,
                       const int* bc, int n_steps, double dt_fixed, double c_cfl, double dx, double gamma,
                       double theta, int scheme, double* dts) {
  if (ghost < 2 || n_steps < 0) return -1;
  const int64_t G = int64_t(ngx) * ngy * ngz;
  const int P = 16 + 2 * ghost;
  std::vector<double> cur(level0, level0 + G * 5 * 4096), nxt(G * 5 * 4096), pad(G * 5 * P * P * P),
      dtp(G * 8);
  int64_t n_bad = 0;
  for (int s = 0; s < n_steps; ++s) {
    double dt = dt_fixed;
    if (!(dt_fixed > 0.0)) {
      fill_ghosts(cur.data(), pad.data(), ngx, ngy, ngz, ghost, bc);
      oracle_dt(pad.data(), G, ghost, dx, gamma, c_cfl, dtp.data());
      dt = dtp[0];
      for (int64_t i = 1; i < G * 8; ++i)
        if (dtp[i] < dt) dt = dtp[i];
    }
    if (dts) dts[s] = dt;
    n_bad += level_step(cur.data(), nxt.data(), ngx, ngy, ngz, ghost, bc, dt, dx, gamma, theta, scheme);
    cur.swap(nxt);
  }
  std::memcpy(level_out, cur.data(), sizeof(double) * G * 5 * 4096);
  return n_bad;
}

// Forward-mode derivative of oracle_rollout at fixed dt: given level0 and a
// tangent t0 (same layout), return level_out and its tangent t_out.
int64_t oracle_rollout_jvp(const double* level0, const double* t0, double* level_out, double* t_out,
                           int ngx, int ngy, int ngz, int ghost, const int* bc, int n_steps, double dt,
                           double dx, double gamma, double theta, int scheme) {
  if (ghost < 2 || n_steps < 0 || !(dt > 0.0)) return -1;
  const int64_t G = int64_t(ngx) * ngy * ngz, n = G * 5 * 4096;
  std::vector<Dual> cur(n), nxt(n);
  for (int64_t i = 0; i < n; ++i) cur[i] = Dual(level0[i], t0[i]);
  int64_t n_bad = 0;
  for (int s = 0; s < n_steps; ++s) {
    n_bad += level_step(cur.data(), nxt.data(), ngx, ngy, ngz, ghost, bc, dt, dx, gamma, theta, scheme);
    cur.swap(nxt);
  }
  for (int64_t i = 0; i < n; ++i) {
    level_out[i] = cur[i].v;
    t_out[i] = cur[i].d;
  }
  return n_bad;
}

// Dual-number JVP of one step of padded groups (tangent given on Upad).
int64_t oracle_mhm_step_jvp(const double* Upad, const double* Tpad, double* Uout, double* Tout, int64_t G,
                            int ghost, double dt, double dx, double gamma, double theta, int scheme) {
  if (ghost < 2 || G < 0) return -1;
  const Block b(16, 16, 16, ghost);
  const int64_t np = b.cells() * 5;
  int64_t n_bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : n_bad)
  for (int64_t g = 0; g < G; ++g) {
    std::vector<Dual> in(np), out(5 * 4096);
    for (int64_t i = 0; i < np; ++i) in[i] = Dual(Upad[g * np + i], Tpad[g * np + i]);
    n_bad += mhm_step_block(in.data(), out.data(), b, dt, dx, gamma, theta, scheme);
    for (int64_t i = 0; i < 5 * 4096; ++i) {
      Uout[g * 5 * 4096 + i] = out[i].v;
      Tout[g * 5 * 4096 + i] = out[i].d;
    }
  }
  return n_bad;
}

// Number of OpenMP threads the oracle's parallel loops use, and a way to set
// it (n >= 1) for timing the oracle on fewer threads.
int oracle_num_threads(void) { return omp_get_max_threads(); }
void oracle_set_num_threads(int n) {
  if (n >= 1) omp_set_num_threads(n);
}

// Single HLLC flux (tests): UL, UR conserved, d = normal axis.  Returns 1 if an
// input state is unphysical.
int oracle_hllc(const double* UL, const double* UR, int d, double gamma, int wavespeed, double* F) {
  return hllc_flux(UL, UR, d, gamma, wavespeed, F) ? 1 : 0;
}

double oracle_limited_slope(double qm, double q0, double qp, double theta) {
  return limited_slope(qm, q0, qp, theta);
}

// Hancock face states of one cell (tests): Wc[5], Wm[3*5], Wp[3*5] -> Ut[3*2*5].
void oracle_hancock_cell(const double* Wc, const double* Wm, const double* Wp, double gamma, double theta,
                         double half_dtdx, int first_order, double* Ut) {
  double m[3][5], p[3][5], o[3][2][5];
  std::memcpy(m, Wm, sizeof m);
  std::memcpy(p, Wp, sizeof p);
  hancock_cell(Wc, m, p, gamma, theta, half_dtdx, first_order != 0, o);
  std::memcpy(Ut, o, sizeof o);
}

void oracle_cons_to_prim(const double* U, double gamma, double* W) { cons_to_prim(U, gamma, W); }
void oracle_prim_to_cons(const double* W, double gamma, double* U) { prim_to_cons(W, gamma, U); }

// Exact Riemann problem: star state out[0..4] = p*, u*, rho*_L, rho*_R, iterations.
int oracle_exact_star(double rL, double uL, double pL, double rR, double uR, double pR, double gamma,
                      double* out) {
  const RP s{rL, uL, pL, rR, uR, pR, gamma};
  double ps, us;
  int it;
  if (star_state(s, &ps, &us, &it) != 0) return -1;
  double a, b;
  star_densities(s, ps, &a, &b);
  out[0] = ps;
  out[1] = us;
  out[2] = a;
  out[3] = b;
  out[4] = it;
  return 0;
}

// Exact solution sampled at n points xi = x/t.
int oracle_exact_sample(double rL, double uL, double pL, double rR, double uR, double pR, double gamma,
                        const double* xi, int64_t n, double* r, double* u, double* p) {
  const RP s{rL, uL, pL, rR, uR, pR, gamma};
  double ps, us;
  if (star_state(s, &ps, &us, nullptr) != 0) return -1;
  for (int64_t i = 0; i < n; ++i) sample(s, ps, us, xi[i], &r[i], &u[i], &p[i]);
  return 0;
}

// Pressure-function residual f_L(p) + f_R(p) + (u_R - u_L) (tests).
double oracle_exact_residual(double rL, double uL, double pL, double rR, double uR, double pR, double gamma,
                             double p) {
  double fL, dfL, fR, dfR;
  pressure_fn(p, rL, pL, gamma, &fL, &dfL);
  pressure_fn(p, rR, pR, gamma, &fR, &dfR);
  return fL + fR + (uR - uL);
}

// Box rollout (see rollout_box above); returns the unphysical count or -1.
int64_t oracle_rollout_box(const double* box, const double* tbox, double* out, double* tout, int nx, int ny, int nz,
                           int n_steps, double dt, double dx, double gamma, double theta, int scheme,
                           uint64_t* sig_out) {
  if (n_steps < 0 || nx - 4 * n_steps < 1 || ny - 4 * n_steps < 1 || nz - 4 * n_steps < 1 ||
      (scheme & SCHEME_ID_MASK) != SCHEME_MHM_PLM_HLLC)
    return -1;
  const size_t n = size_t(5) * nx * ny * nz;
  const size_t m = size_t(5) * (nx - 4 * n_steps) * (ny - 4 * n_steps) * (nz - 4 * n_steps);
  g_sig_on = sig_out != nullptr;
  g_sig = 0xcbf29ce484222325ull;
  int64_t n_bad;
  if (tbox == nullptr) {
    std::vector<double> res;
    n_bad = rollout_box(std::vector<double>(box, box + n), nx, ny, nz, n_steps, dt, dx, gamma, theta, scheme, res);
    std::memcpy(out, res.data(), sizeof(double) * m);
  } else {
    std::vector<Dual> in(n), res;
    for (size_t i = 0; i < n; ++i) in[i] = Dual(box[i], tbox[i]);
    n_bad = rollout_box(std::move(in), nx, ny, nz, n_steps, dt, dx, gamma, theta, scheme, res);
    for (size_t i = 0; i < m; ++i) {
      out[i] = res[i].v;
      if (tout != nullptr) tout[i] = res[i].d;
    }
  }
  if (sig_out != nullptr) *sig_out = g_sig;
  g_sig_on = false;
  return n_bad;
}

// Algorithmic operation counts of the four per-item stages, each evaluated on
// the given sample data (ops[4*4]: {add, mul, div, sqrt} for cons_to_prim,
// hancock_cell, hllc_flux, one cell's update incl. its unphysical check).
void oracle_count_ops(const double* U, const double* Wc, const double* Wm, const double* Wp,
                      const double* UL, const double* UR, double gamma, double theta, double half_dtdx,
                      int64_t* ops) {
  auto take = [&](int k) {
    ops[k * 4 + 0] = g_ops.add;
    ops[k * 4 + 1] = g_ops.mul;
    ops[k * 4 + 2] = g_ops.div;
    ops[k * 4 + 3] = g_ops.sqrt;
    g_ops = {0, 0, 0, 0};
  };
  g_ops = {0, 0, 0, 0};
  {
    Cnt u[5], w[5];
    for (int q = 0; q < 5; ++q) u[q] = Cnt(U[q]);
    cons_to_prim(u, gamma, w);
  }
  take(0);
  {
    Cnt c[5], m[3][5], p[3][5], o[3][2][5];
    for (int q = 0; q < 5; ++q) c[q] = Cnt(Wc[q]);
    for (int d = 0; d < 3; ++d)
      for (int q = 0; q < 5; ++q) {
        m[d][q] = Cnt(Wm[d * 5 + q]);
        p[d][q] = Cnt(Wp[d * 5 + q]);
      }
    g_ops = {0, 0, 0, 0};
    hancock_cell(c, m, p, gamma, theta, Cnt(half_dtdx), false, o);
  }
  take(1);
  {
    Cnt l[5], r[5], f[5];
    for (int q = 0; q < 5; ++q) {
      l[q] = Cnt(UL[q]);
      r[q] = Cnt(UR[q]);
    }
    g_ops = {0, 0, 0, 0};
    hllc_flux(l, r, 0, gamma, 0, f);
  }
  take(2);
  {
    // one interior cell: 5 x (3 flux differences, 2 adds, 1 mul, 1 sub) and
    // the pressure of the new state for the unphysical check
    Cnt fx[2][5], un[5], dtdx(half_dtdx * 2.0), gm1(gamma - 1.0);
    for (int q = 0; q < 5; ++q) {
      fx[0][q] = Cnt(UL[q]);
      fx[1][q] = Cnt(UR[q]);
    }
    g_ops = {0, 0, 0, 0};
    for (int q = 0; q < 5; ++q) {
      Cnt acc = fx[1][q] - fx[0][q];
      acc = acc + (fx[1][q] - fx[0][q]);
      acc = acc + (fx[1][q] - fx[0][q]);
      un[q] = Cnt(U[q]) - dtdx * acc;
    }
    Cnt p = gm1 * (un[4] - Cnt(0.5) * (un[1] * un[1] + un[2] * un[2] + un[3] * un[3]) / un[0]);
    (void)p;
  }
  take(3);
}

// ------------------------------------------------- other schemes (C ABI) ---
static bool valid_any_scheme(int scheme, int ghost) {
  const int id = scheme & SCHEME_ID_MASK;
  if (scheme & ~(0xff | (3 << 8) | FIRST_ORDER_BIT | (3 << LIMITER_SHIFT) | CHARACTERISTIC_BIT | PPM_BIT |
                 (3 << RIEMANN_SHIFT) | DUAL_ENERGY_BIT))
    return false;
  if (id != SCHEME_MHM_PLM_HLLC && id != SCHEME_CTU) return false;
  if (((scheme >> RIEMANN_SHIFT) & 3) == 3) return false;
  return ghost >= recon_radius(scheme) + 1 && ghost >= 2;
}

// One step of G padded 16^3 groups with any scheme of the scheme word.
int64_t oracle_step_any(const double* Upad, double* Uout, int64_t G, int ghost, double dt, double dx, double gamma,
                        double theta, int scheme) {
  if (G < 0 || !valid_any_scheme(scheme, ghost) || (scheme & DUAL_ENERGY_BIT)) return -1;
  const Block b(16, 16, 16, ghost);
  int64_t n_bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : n_bad)
  for (int64_t g = 0; g < G; ++g)
    n_bad += step_block_any(Upad + g * b.cells() * 5, Uout + g * 5 * 4096, b, dt, dx, gamma, theta, scheme);
  return n_bad;
}

// oracle_step_any that also returns the fluxes of the patch-boundary faces of
// every group, [G][9][5][256] (step_block_any's face_flux layout).
int64_t oracle_step_any_flux(const double* Upad, double* Uout, double* face_flux, int64_t G, int ghost, double dt,
                             double dx, double gamma, double theta, int scheme) {
  if (G < 0 || !valid_any_scheme(scheme, ghost) || (scheme & DUAL_ENERGY_BIT)) return -1;
  const Block b(16, 16, 16, ghost);
  int64_t n_bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : n_bad)
  for (int64_t g = 0; g < G; ++g)
    n_bad += step_block_any(Upad + g * b.cells() * 5, Uout + g * 5 * 4096, b, dt, dx, gamma, theta, scheme,
                            face_flux + g * 9 * 5 * 256);
  return n_bad;
}

int64_t oracle_step_block_any(const double* Upad, double* Uout, int nx, int ny, int nz, int ghost, double dt,
                              double dx, double gamma, double theta, int scheme) {
  if (nx < 1 || ny < 1 || nz < 1 || !valid_any_scheme(scheme, ghost) || (scheme & DUAL_ENERGY_BIT)) return -1;
  return step_block_any(Upad, Uout, Block(nx, ny, nz, ghost), dt, dx, gamma, theta, scheme);
}

// Dual-number JVP of oracle_step_any.
int64_t oracle_step_any_jvp(const double* Upad, const double* Tpad, double* Uout, double* Tout, int64_t G, int ghost,
                            double dt, double dx, double gamma, double theta, int scheme) {
  if (G < 0 || !valid_any_scheme(scheme, ghost) || (scheme & DUAL_ENERGY_BIT)) return -1;
  const Block b(16, 16, 16, ghost);
  const int64_t np = b.cells() * 5;
  int64_t n_bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : n_bad)
  for (int64_t g = 0; g < G; ++g) {
    std::vector<Dual> in(np), out(5 * 4096);
    for (int64_t i = 0; i < np; ++i) in[i] = Dual(Upad[g * np + i], Tpad[g * np + i]);
    n_bad += step_block_any(in.data(), out.data(), b, dt, dx, gamma, theta, scheme);
    for (int64_t i = 0; i < 5 * 4096; ++i) {
      Uout[g * 5 * 4096 + i] = out[i].v;
      Tout[g * 5 * 4096 + i] = out[i].d;
    }
  }
  return n_bad;
}

// Dual-energy steps (scheme bit 18): 6 fields per cell, [G][6][P^3] ->
// [G][6][16^3], and one block [6][nz+2g][ny+2g][nx+2g] -> [6][nz][ny][nx].
int64_t oracle_step_any_de(const double* Upad, double* Uout, int64_t G, int ghost, double dt, double dx,
                           double gamma, double theta, int scheme, double xi) {
  if (G < 0 || !valid_any_scheme(scheme, ghost) || !(scheme & DUAL_ENERGY_BIT) || !(xi >= 0.0)) return -1;
  const Block b(16, 16, 16, ghost);
  int64_t n_bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : n_bad)
  for (int64_t g = 0; g < G; ++g)
    n_bad += step_block_any(Upad + g * b.cells() * 6, Uout + g * 6 * 4096, b, dt, dx, gamma, theta, scheme,
                            (double*)nullptr, xi);
  return n_bad;
}

int64_t oracle_step_block_any_de(const double* Upad, double* Uout, int nx, int ny, int nz, int ghost, double dt,
                                 double dx, double gamma, double theta, int scheme, double xi) {
  if (nx < 1 || ny < 1 || nz < 1 || !valid_any_scheme(scheme, ghost) || !(scheme & DUAL_ENERGY_BIT) || !(xi >= 0.0))
    return -1;
  return step_block_any(Upad, Uout, Block(nx, ny, nz, ghost), dt, dx, gamma, theta, scheme, (double*)nullptr, xi);
}

// Riemann flux of the scheme word's solver (tests).  Returns 1 if an input
// state is unphysical, -1 on a bad solver id.
int oracle_riemann(const double* UL, const double* UR, int d, double gamma, int scheme, double* F) {
  if (((scheme >> RIEMANN_SHIFT) & 3) == 3) return -1;
  return riemann_flux(UL, UR, d, gamma, scheme, F) ? 1 : 0;
}

double oracle_limit_diffs(double dm, double dp, double dc, double theta, int limiter) {
  return limit_diffs(dm, dp, dc, theta, limiter & 3);
}

void oracle_limited_slopes(const double* Wm, const double* Wc, const double* Wp, int d, double gamma, double theta,
                           int scheme, double* s) {
  limited_slopes(Wm, Wc, Wp, d, gamma, theta, scheme, s);
}

// Face values of one cell along axis d from the 5-cell stencil Ws[5*5]
// (cells -2..2) -> Wf[2*5] (low face, high face).
void oracle_face_values(const double* Ws, int d, double gamma, double theta, int scheme, double* Wf) {
  const double* st[5] = {Ws, Ws + 5, Ws + 10, Ws + 15, Ws + 20};
  double o[2][5];
  face_values(st, d, gamma, theta, scheme, o);
  std::memcpy(Wf, o, sizeof o);
}

void oracle_to_characteristic(const double* dW, int d, double rho, double c, double* a) {
  to_characteristic(dW, d, rho, c, a);
}
void oracle_from_characteristic(const double* a, int d, double rho, double c, double* dW) {
  from_characteristic(a, d, rho, c, dW);
}

// One step of a level (ghost fill + any scheme) without the procedure for
// unphysical results.  Returns the unphysical count.
int64_t oracle_level_step_any(const double* level, double* level_out, int ngx, int ngy, int ngz, int ghost,
                              const int* bc, double dt, double dx, double gamma, double theta, int scheme) {
  if (ngx < 1 || ngy < 1 || ngz < 1 || ghost > 16 || !valid_any_scheme(scheme, ghost) || (scheme & DUAL_ENERGY_BIT))
    return -1;
  const int P = 16 + 2 * ghost;
  const int64_t G = int64_t(ngx) * ngy * ngz;
  std::vector<double> pad(size_t(G) * 5 * P * P * P);
  fill_ghosts(level, pad.data(), ngx, ngy, ngz, ghost, bc);
  const Block b(16, 16, 16, ghost);
  int64_t n_bad = 0;
#pragma omp parallel for schedule(static) reduction(+ : n_bad)
  for (int64_t g = 0; g < G; ++g)
    n_bad += step_block_any(pad.data() + g * b.cells() * 5, level_out + g * 5 * 4096, b, dt, dx, gamma, theta,
                            scheme);
  return n_bad;
}

// One step of a level with the procedure for unphysical results: steps
// (ii)-(iii) on the failed cells, then (iv)-(v): while cells still fail and
// the reduced step dt*ratio is at least dt_min, recompute the level from its
// input with dt *= ratio.  out_info[4] receives: the dt of the accepted (or
// last) attempt, the number of retries, and the cells repaired unsplit and
// split in that attempt.  Returns the number of cells still unphysical (0 on
// success), or -1 on bad arguments.
int64_t oracle_level_step_fallback(const double* level, double* level_out, int ngx, int ngy, int ngz, int ghost,
                                   const int* bc, double dt, double dt_min, double ratio, double dx, double gamma,
                                   double theta, int scheme, double* out_info) {
  if (ngx < 1 || ngy < 1 || ngz < 1 || ghost > 16 || !valid_any_scheme(scheme, ghost) || (scheme & DUAL_ENERGY_BIT) ||
      !(dt > 0.0) ||
      !(ratio > 0.0 && ratio < 1.0) || !(dt_min >= 0.0))
    return -1;
  int retries = 0;
  for (;;) {
    int64_t nu = 0, ns = 0;
    const int64_t left =
        level_step_repaired(level, level_out, ngx, ngy, ngz, ghost, bc, dt, dx, gamma, theta, scheme, &nu, &ns);
    const double next = dt * ratio;
    if (left == 0 || next < dt_min) {
      out_info[0] = dt;
      out_info[1] = retries;
      out_info[2] = double(nu);
      out_info[3] = double(ns);
      return left;
    }
    dt = next;
    ++retries;
  }
}

// First-order recomputations of one cell of a level (tests): mode 0 unsplit,
// 1 split.  X, Y, Z are global cell indices.
void oracle_first_order_cell(const double* level, int ngx, int ngy, int ngz, const int* bc, int X, int Y, int Z,
                             double dtdx, double gamma, int scheme, int mode, double* out) {
  const LevelView lv{level, ngx, ngy, ngz, bc};
  if (mode == 0) first_order_unsplit(lv, X, Y, Z, dtdx, gamma, scheme | FIRST_ORDER_BIT, out);
  else first_order_split(lv, X, Y, Z, dtdx, gamma, scheme | FIRST_ORDER_BIT, out);
}

// ------------------------------------------------ coarse-fine coupling ABI ---
// Levels concatenated: G[l] groups of level l, positions pos [sum G][3]
// (x, y, z in the level's group lattice, n0 * 2^l per axis), states U
// [sum G][5][16^3] (in/out).  One coarse step of dt0 (W-cycle: level l takes
// 2^l steps of dt0 / 2^l).  Returns the unphysical count, or -1 on bad
// arguments (a position off the lattice or repeated, a level not properly
// nested, level 0 not covering the domain).
static bool amr_setup(int n_levels, const int* n0, const int64_t* G, const int* pos, double* U,
                      std::vector<AmrLevel>& Ls, const int* bc) {
  if (n_levels < 1 || n_levels > 8 || n0[0] < 1 || n0[1] < 1 || n0[2] < 1) return false;
  Ls.resize(n_levels);
  int64_t off = 0;
  for (int l = 0; l < n_levels; ++l) {
    AmrLevel& L = Ls[l];
    for (int d = 0; d < 3; ++d) L.n[d] = n0[d] << l;
    L.G = G[l];
    L.pos = pos + 3 * off;
    L.U = U + off * 5 * 4096;
    for (int64_t g = 0; g < L.G; ++g)
      for (int d = 0; d < 3; ++d)
        if (L.pos[3 * g + d] < 0 || L.pos[3 * g + d] >= L.n[d]) return false;
    L.build_map();
    int64_t filled = 0;
    for (int v : L.map) filled += v >= 0;
    if (filled != L.G) return false;                                 // repeated positions
    if (l == 0 && L.G != int64_t(L.n[0]) * L.n[1] * L.n[2]) return false;  // level 0 covers the domain
    if (l > 0 && !amr_nested(L, Ls[l - 1], bc)) return false;
    off += G[l];
  }
  return true;
}

int64_t oracle_amr_step(int n_levels, const int* n0, const int64_t* G, const int* pos, double* U, const int* bc,
                        int ghost, double dt0, double dx0, double gamma, double theta, int scheme) {
  if (ghost > 16 || !valid_any_scheme(scheme, ghost) || (scheme & DUAL_ENERGY_BIT)) return -1;
  std::vector<AmrLevel> Ls;
  if (!amr_setup(n_levels, n0, G, pos, U, Ls, bc)) return -1;
  return amr_advance(Ls, 0, dt0, dx0, gamma, theta, scheme, ghost, bc, nullptr, nullptr, 0.0, nullptr);
}

// Padded blocks of level `lev` of a hierarchy (ghosts from siblings, else
// interpolated from level lev-1 between Cold and Cnew at weight a; level
// lev-1's states are taken from Cold / Cnew, U supplies the positions and
// level lev's own states).  pad: [G[lev]][5][P^3].
int oracle_amr_fill(int n_levels, const int* n0, const int64_t* G, const int* pos, double* U, const int* bc,
                    int lev, const double* Cold, const double* Cnew, double a, int ghost, double* pad) {
  std::vector<AmrLevel> Ls;
  if (ghost < 0 || ghost > 16 || lev < 0 || lev >= n_levels || !amr_setup(n_levels, n0, G, pos, U, Ls, bc)) return -1;
  amr_fill(Ls[lev], lev > 0 ? &Ls[lev - 1] : nullptr, Cold, Cnew, a, bc, ghost, pad);
  return 0;
}

}  // extern "C"
