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

}  // extern "C"
