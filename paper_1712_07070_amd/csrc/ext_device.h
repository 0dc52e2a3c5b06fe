// Device arithmetic of the other options of GAMER-2's fluid solver (Sec. 2.2):
// van Leer, van Albada and hybrid slope limiters, PLM on characteristic
// variables, PPM reconstruction, the HLLE and Roe Riemann solvers (Roe
// switching to HLLC when a state between its waves is unphysical), and the
// first-order recomputations of the procedure for unphysical results.  Used
// by the multi-pass kernels of scheme_ext.hip; the default scheme's fused
// kernels keep hydro_device.h only.
#pragma once

#include "hydro_device.h"

namespace gh {

// Options of a scheme word (include/hydro.h: bits 0-7 id, 8-9 wave speeds,
// 10 first order, 11-12 limiter, 13 characteristic, 14 PPM, 16-17 solver).
struct ExtOpts {
  int ctu;          // 1: CTU (6 Riemann solves per cell), 0: MHM
  int ws;           // HLLC / HLLE wave speeds: 0 Einfeldt/Roe, 1 Davis
  int first_order;  // zero slopes
  int lim;          // 0 generalized minmod, 1 van Leer, 2 van Albada, 3 hybrid
  int chr;          // limit characteristic variables
  int ppm;          // PPM face values
  int solver;       // 0 HLLC, 1 Roe, 2 HLLE
  int de;           // dual energy: a sixth field, the entropy s = p / rho^(gamma-1)
  double xi;        // dual energy: E is taken from s where E_th < xi E_kin
  // cells of reconstruction reach on each side of a cell along an axis
  __host__ __device__ int radius() const { return first_order ? 0 : (ppm ? 2 : 1); }
};

// Full limited slope from the one-sided differences dm, dp and the central
// difference dc; zero unless dm and dp are of one strict sign.
//   0 generalized minmod  sgn(dc) min(theta|dm|, |dc|, theta|dp|)
//   1 van Leer            2 dm dp / (dm + dp)
//   2 van Albada          dm dp (dm + dp) / (dm^2 + dp^2)
//   3 hybrid              sgn(dc) min(generalized minmod, |van Leer|)
template <typename T>
__device__ __forceinline__ T ext_limit(T dm, T dp, T dc, T theta, int lim) {
  if (!(dm * dp > T(0))) return T(0);
  if (lim == 1) return Fp<T>::div(T(2) * dm * dp, dm + dp);
  if (lim == 2) return Fp<T>::div(dm * dp * (dm + dp), dm * dm + dp * dp);
  T m = fmin_(theta * fabs_(dm), fabs_(dc));
  m = fmin_(m, theta * fabs_(dp));
  if (lim == 3) m = fmin_(m, fabs_(Fp<T>::div(T(2) * dm * dp, dm + dp)));
  return copysign_(m, dc);
}

// Limited slopes of the primitive state Wc along axis D.  With `chr` the
// one-sided differences are projected on the characteristic fields of Wc
// (left eigenvectors of the primitive Euler system, sound speed c):
//   a0 = (dp/c^2 - (rho/c) du_n)/2, a1 = drho - dp/c^2, a2 = du_t1,
//   a3 = du_t2, a4 = (dp/c^2 + (rho/c) du_n)/2,
// limited component by component (dc the mean of the two differences) and
// projected back: drho = a0 + a1 + a4, du_n = (c/rho)(a4 - a0), dp = c^2 (a0 + a4).
template <int D, typename T>
__device__ __forceinline__ void ext_slopes(const T Wm[5], const T Wc[5], const T Wp[5], const Gas<T>& g,
                                           const ExtOpts& o, T s[5]) {
  if (!o.chr) {
#pragma unroll
    for (int q = 0; q < 5; ++q) s[q] = ext_limit(Wc[q] - Wm[q], Wp[q] - Wc[q], T(0.5) * (Wp[q] - Wm[q]), g.theta, o.lim);
    return;
  }
  constexpr int n = 1 + D, t1 = 1 + (D + 1) % 3, t2 = 1 + (D + 2) % 3;
  const T ir = Fp<T>::rcp(Wc[0]);
  const T c = Fp<T>::sqrt(g.gamma * Wc[4] * ir);
  const T ic = Fp<T>::rcp(c);
  const T ic2 = ic * ic;
  const T rc = Wc[0] * ic;
  T am[5], ap[5], a[5];
  {
    const T dm[5] = {Wc[0] - Wm[0], Wc[1] - Wm[1], Wc[2] - Wm[2], Wc[3] - Wm[3], Wc[4] - Wm[4]};
    const T dp[5] = {Wp[0] - Wc[0], Wp[1] - Wc[1], Wp[2] - Wc[2], Wp[3] - Wc[3], Wp[4] - Wc[4]};
    const T pm = dm[4] * ic2, pp = dp[4] * ic2, um = rc * dm[n], up = rc * dp[n];
    am[0] = T(0.5) * (pm - um);
    am[1] = dm[0] - pm;
    am[2] = dm[t1];
    am[3] = dm[t2];
    am[4] = T(0.5) * (pm + um);
    ap[0] = T(0.5) * (pp - up);
    ap[1] = dp[0] - pp;
    ap[2] = dp[t1];
    ap[3] = dp[t2];
    ap[4] = T(0.5) * (pp + up);
  }
#pragma unroll
  for (int k = 0; k < 5; ++k) a[k] = ext_limit(am[k], ap[k], T(0.5) * (am[k] + ap[k]), g.theta, o.lim);
  s[0] = (a[0] + a[1]) + a[4];
  s[n] = (c * ir) * (a[4] - a[0]);
  s[t1] = a[2];
  s[t2] = a[3];
  s[4] = (c * c) * (a[0] + a[4]);
}

// PPM interface values of one variable from cells -1, 0, +1 and their
// limited slopes, then the monotonicity constraints.
template <typename T>
__device__ __forceinline__ void ppm_scalar(T qm, T q0, T qp, T sm, T s0, T sp, T& qL, T& qR) {
  const T sixth = T(1) / T(6);
  qL = T(0.5) * (qm + q0) - (s0 - sm) * sixth;
  qR = T(0.5) * (q0 + qp) - (sp - s0) * sixth;
  if (!((qR - q0) * (q0 - qL) > T(0))) {
    qL = q0;
    qR = q0;
  } else {
    const T dq = qR - qL;
    const T q6 = T(6) * (q0 - T(0.5) * (qL + qR));
    if (dq * q6 > dq * dq) qL = T(3) * q0 - T(2) * qR;
    else if (-(dq * dq) > dq * q6) qR = T(3) * q0 - T(2) * qL;
  }
}

// Face values (low Wf[0], high Wf[1]) of the cell W[2] along axis D from the
// stencil W[0..4] = cells -2..+2 (PLM reads W[1..3]).  PPM (Colella &
// Woodward 1984): qL = (q-1 + q0)/2 - (s0 - s-1)/6, qR = (q0 + q+1)/2 -
// (s+1 - s0)/6 from the limited slopes of the three middle cells, then flat
// at an extremum ((qR - q0)(q0 - qL) <= 0), else with dq = qR - qL and
// q6 = 6 (q0 - (qL + qR)/2): qL = 3 q0 - 2 qR if dq q6 > dq^2, qR = 3 q0 - 2 qL
// if -dq^2 > dq q6.
template <int D, typename T>
__device__ __forceinline__ void ext_face_values(const T W[5][5], const Gas<T>& g, const ExtOpts& o, T Wf[2][5]) {
  if (o.first_order) {
#pragma unroll
    for (int q = 0; q < 5; ++q) Wf[0][q] = Wf[1][q] = W[2][q];
    return;
  }
  if (!o.ppm) {
    T s[5];
    ext_slopes<D>(W[1], W[2], W[3], g, o, s);
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      Wf[0][q] = W[2][q] - T(0.5) * s[q];
      Wf[1][q] = W[2][q] + T(0.5) * s[q];
    }
    return;
  }
  T sm[5], s0[5], sp[5];
  ext_slopes<D>(W[0], W[1], W[2], g, o, sm);
  ext_slopes<D>(W[1], W[2], W[3], g, o, s0);
  ext_slopes<D>(W[2], W[3], W[4], g, o, sp);
#pragma unroll
  for (int q = 0; q < 5; ++q) ppm_scalar(W[1][q], W[2][q], W[3][q], sm[q], s0[q], sp[q], Wf[0][q], Wf[1][q]);
}

// Face values of a passively advected scalar from its stencil q[0..4]
// (cells -2..+2): limited like a primitive variable (no characteristic
// projection: it is a wave of its own), PLM or PPM.
template <typename T>
__device__ __forceinline__ void passive_face_values(const T q[5], const Gas<T>& g, const ExtOpts& o, T out[2]) {
  if (o.first_order) {
    out[0] = out[1] = q[2];
    return;
  }
  auto slope = [&](int j) { return ext_limit(q[j] - q[j - 1], q[j + 1] - q[j], T(0.5) * (q[j + 1] - q[j - 1]), g.theta, o.lim); };
  if (!o.ppm) {
    const T sl = slope(2);
    out[0] = q[2] - T(0.5) * sl;
    out[1] = q[2] + T(0.5) * sl;
    return;
  }
  ppm_scalar(q[1], q[2], q[3], slope(1), slope(2), slope(3), out[0], out[1]);
}

// Conserved form and physical flux along D of a primitive face state.
template <int D, typename T>
__device__ __forceinline__ void ext_cons_flux(const T W[5], const Gas<T>& g, T U[5], T F[5]) {
  U[0] = W[0];
  U[1] = W[0] * W[1];
  U[2] = W[0] * W[2];
  U[3] = W[0] * W[3];
  U[4] = W[4] * g.inv_gm1 + T(0.5) * W[0] * (W[1] * W[1] + W[2] * W[2] + W[3] * W[3]);
  const T un = W[1 + D];
  F[0] = U[0] * un;
  F[1] = U[1] * un;
  F[2] = U[2] * un;
  F[3] = U[3] * un;
  F[1 + D] = F[1 + D] + W[4];
  F[4] = (U[4] + W[4]) * un;
}

// Normal-frame view of a face's two conserved states.
template <int D, typename T>
struct ExtPair {
  static constexpr int n = 1 + D, t1 = 1 + (D + 1) % 3, t2 = 1 + (D + 2) % 3;
  T L[5], R[5];  // (rho, m_n, m_t1, m_t2, E)
  T iL, iR, uL, vL, wL, uR, vR, wR, pL, pR, cL, cR;
  bool bad;
  __device__ __forceinline__ ExtPair(const T UL[5], const T UR[5], const Gas<T>& g) {
    L[0] = UL[0]; L[1] = UL[n]; L[2] = UL[t1]; L[3] = UL[t2]; L[4] = UL[4];
    R[0] = UR[0]; R[1] = UR[n]; R[2] = UR[t1]; R[3] = UR[t2]; R[4] = UR[4];
    iL = Fp<T>::rcp(L[0]);
    iR = Fp<T>::rcp(R[0]);
    uL = L[1] * iL; vL = L[2] * iL; wL = L[3] * iL;
    uR = R[1] * iR; vR = R[2] * iR; wR = R[3] * iR;
    pL = g.gm1 * (L[4] - T(0.5) * (L[1] * uL + L[2] * vL + L[3] * wL));
    pR = g.gm1 * (R[4] - T(0.5) * (R[1] * uR + R[2] * vR + R[3] * wR));
    bad = !(L[0] > T(0) && pL > T(0) && R[0] > T(0) && pR > T(0));
    cL = Fp<T>::sqrt(g.gamma * pL * iL);
    cR = Fp<T>::sqrt(g.gamma * pR * iR);
  }
  __device__ __forceinline__ void fluxes(T FL[5], T FR[5]) const {
    FL[0] = L[1]; FL[1] = L[1] * uL + pL; FL[2] = L[2] * uL; FL[3] = L[3] * uL; FL[4] = (L[4] + pL) * uL;
    FR[0] = R[1]; FR[1] = R[1] * uR + pR; FR[2] = R[2] * uR; FR[3] = R[3] * uR; FR[4] = (R[4] + pR) * uR;
  }
  __device__ __forceinline__ void store(const T Fn[5], T F[5]) const {
    F[0] = Fn[0];
    F[n] = Fn[1];
    F[t1] = Fn[2];
    F[t2] = Fn[3];
    F[4] = Fn[4];
  }
  // Roe averages (weights sqrt(rho)) of u, v, w and H = (E + p)/rho
  __device__ __forceinline__ void roe_avg(T& ua, T& va, T& wa, T& Ha) const {
    const T sL = Fp<T>::sqrt(L[0]), sR = Fp<T>::sqrt(R[0]);
    const T iw = Fp<T>::rcp(sL + sR);
    ua = (sL * uL + sR * uR) * iw;
    va = (sL * vL + sR * vR) * iw;
    wa = (sL * wL + sR * wR) * iw;
    Ha = (sL * ((L[4] + pL) * iL) + sR * ((R[4] + pR) * iR)) * iw;
  }
};

// HLLE (Einfeldt 1988) with the HLLC solver's wave speeds:
//   F = F_L if S_L >= 0, F_R if S_R <= 0, else
//   (S_R F_L - S_L F_R + S_L S_R (U_R - U_L)) / (S_R - S_L).
template <int D, typename T>
__device__ __forceinline__ bool hlle_flux(const T UL[5], const T UR[5], const Gas<T>& g, int ws, T F[5]) {
  const ExtPair<D, T> f(UL, UR, g);
  T SL, SR;
  if (ws == 1) {
    SL = min_first(f.uL - f.cL, f.uR - f.cR);
    SR = max_first(f.uL + f.cL, f.uR + f.cR);
  } else {
    T ua, va, wa, Ha;
    f.roe_avg(ua, va, wa, Ha);
    const T ca = Fp<T>::sqrt(g.gm1 * (Ha - T(0.5) * (ua * ua + va * va + wa * wa)));
    SL = min_first(f.uL - f.cL, ua - ca);
    SR = max_first(f.uR + f.cR, ua + ca);
  }
  T FL[5], FR[5], Fn[5];
  f.fluxes(FL, FR);
  if (SL >= T(0)) {
#pragma unroll
    for (int q = 0; q < 5; ++q) Fn[q] = FL[q];
  } else if (SR <= T(0)) {
#pragma unroll
    for (int q = 0; q < 5; ++q) Fn[q] = FR[q];
  } else {
    const T iw = Fp<T>::rcp(SR - SL);
#pragma unroll
    for (int q = 0; q < 5; ++q) Fn[q] = (SR * FL[q] - SL * FR[q] + SL * SR * (f.R[q] - f.L[q])) * iw;
  }
  f.store(Fn, F);
  return f.bad;
}

// Roe's flux with the wave strengths of the 3D Euler system (Toro 2009,
// Sec. 11.3), no entropy fix:
//   al3 = dU2 - v~ dU0, al4 = dU3 - w~ dU0,
//   al2 = (gamma-1)/a~^2 [dU0 (H~ - u~^2) + u~ dU1 - (dU4 - al3 v~ - al4 w~)],
//   al1 = [dU0 (u~ + a~) - dU1 - a~ al2] / (2 a~), al5 = dU0 - (al1 + al2),
//   F = (F_L + F_R)/2 - (|u~-a~| al1 K1 + |u~| (al2 K2 + al3 K3 + al4 K4)
//                        + |u~+a~| al5 K5)/2.
// If a~^2 <= 0 or a state between the waves (U_L + al1 K1, then + al2 K2 +
// al3 K3 + al4 K4) has rho <= 0 or p <= 0, the face takes the HLLC flux.
template <int D, typename T>
__device__ __forceinline__ bool roe_flux(const T UL[5], const T UR[5], const Gas<T>& g, int ws, T F[5]) {
  const ExtPair<D, T> f(UL, UR, g);
  T ua, va, wa, Ha;
  f.roe_avg(ua, va, wa, Ha);
  const T q2 = ua * ua + va * va + wa * wa;
  const T a2 = g.gm1 * (Ha - T(0.5) * q2);
  bool ok = a2 > T(0);
  T Fn[5];
  if (ok) {
    const T a = Fp<T>::sqrt(a2);
    T dU[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) dU[q] = f.R[q] - f.L[q];
    const T al3 = dU[2] - va * dU[0];
    const T al4 = dU[3] - wa * dU[0];
    const T al2 = Fp<T>::div(g.gm1, a2) * (dU[0] * (Ha - ua * ua) + ua * dU[1] - (dU[4] - al3 * va - al4 * wa));
    const T al1 = Fp<T>::div(dU[0] * (ua + a) - dU[1] - a * al2, T(2) * a);
    const T al5 = dU[0] - (al1 + al2);
    const T K1[5] = {T(1), ua - a, va, wa, Ha - ua * a};
    const T K2[5] = {T(1), ua, va, wa, T(0.5) * q2};
    const T K5[5] = {T(1), ua + a, va, wa, Ha + ua * a};
    // K3 = (0, 0, 1, 0, v~), K4 = (0, 0, 0, 1, w~)
    T S1[5], S2[5], mid[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) {
      const T k3 = q == 2 ? T(1) : (q == 4 ? va : T(0));
      const T k4 = q == 3 ? T(1) : (q == 4 ? wa : T(0));
      mid[q] = (al2 * K2[q] + al3 * k3) + al4 * k4;
      S1[q] = f.L[q] + al1 * K1[q];
      S2[q] = S1[q] + mid[q];
    }
    ok = !unphysical(S1, g) && !unphysical(S2, g);
    if (ok) {
      const T l1 = fabs_(ua - a), l2 = fabs_(ua), l5 = fabs_(ua + a);
      T FL[5], FR[5];
      f.fluxes(FL, FR);
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        const T diss = (l1 * al1 * K1[q] + l2 * mid[q]) + l5 * al5 * K5[q];
        Fn[q] = T(0.5) * (FL[q] + FR[q]) - T(0.5) * diss;
      }
    }
  }
  if (!ok) return hllc_flux<D>(UL, UR, g, ws, F);
  f.store(Fn, F);
  return f.bad;
}

template <int D, typename T>
__device__ __forceinline__ bool riemann_any(const T UL[5], const T UR[5], const Gas<T>& g, const ExtOpts& o, T F[5]) {
  if (o.solver == 1) return roe_flux<D>(UL, UR, g, o.ws, F);
  if (o.solver == 2) return hlle_flux<D>(UL, UR, g, o.ws, F);
  return hllc_flux<D>(UL, UR, g, o.ws, F);
}

// The Riemann flux of the Euler fields plus, with NF = 6, the flux of the
// passive entropy field: the mass flux times s/rho of the upwind side.
template <int D, int NF, typename T>
__device__ __forceinline__ bool riemann_nf(const T UL[NF], const T UR[NF], const Gas<T>& g, const ExtOpts& o,
                                           T F[NF]) {
  const bool bad = riemann_any<D>(UL, UR, g, o, F);
  if constexpr (NF == 6) F[5] = F[0] * (F[0] >= T(0) ? Fp<T>::div(UL[5], UL[0]) : Fp<T>::div(UR[5], UR[0]));
  return bad;
}

}  // namespace gh
