// Device-side arithmetic of the MHM + PLM + HLLC step (GAMER-2, Sec. 2.2).
//
// Everything here is __device__ __forceinline__ and templated on the floating
// type T (double or float).  Values are carried in registers; the kernels in
// mhm_fwd.hip decide what is staged in LDS.  Every expression has a single
// source form, and the library is built with -ffp-contract=on, so each
// inlined copy of a function rounds identically: a face computed by two
// workgroups (the shared face of neighbouring groups) gets bitwise-identical
// flux, which keeps the update conservative to round-off.
#pragma once

#include <hip/hip_runtime.h>
#include <stdint.h>

namespace gh {

// ------------------------------------------------------------ numerics ----
// Type-exact elementary helpers (the __builtin_f* forms without suffix are
// the double versions and would silently widen float arguments).
__device__ __forceinline__ double fabs_(double x) { return __builtin_fabs(x); }
__device__ __forceinline__ float fabs_(float x) { return __builtin_fabsf(x); }
__device__ __forceinline__ double fmin_(double a, double b) { return __builtin_fmin(a, b); }
__device__ __forceinline__ float fmin_(float a, float b) { return __builtin_fminf(a, b); }
__device__ __forceinline__ double copysign_(double a, double b) { return __builtin_copysign(a, b); }
__device__ __forceinline__ float copysign_(float a, float b) { return __builtin_copysignf(a, b); }
__device__ __forceinline__ double fma_(double a, double b, double c) { return __builtin_fma(a, b, c); }
__device__ __forceinline__ float fma_(float a, float b, float c) { return __builtin_fmaf(a, b, c); }

template <typename T> struct Fp;

// FP64: hardware reciprocal / reciprocal square root refined by one Newton /
// Goldschmidt step (relative error about 2^-47, far inside the 1e-12 parity
// bound; a division corrects its quotient once more) instead of the
// correctly rounded IEEE sequences, which cost two to three times as many
// instructions.
template <> struct Fp<double> {
  // the hardware reciprocal is good to about 2^-24; one Newton step gives
  // about 2^-48 relative
  static __device__ __forceinline__ double rcp(double x) {
    const double r = __builtin_amdgcn_rcp(x);
    const double e = __builtin_fma(-x, r, 1.0);
    return __builtin_fma(r, e, r);
  }
  // a times the refined reciprocal of b, corrected once with the exact
  // residual a - b q: nearly always the correctly rounded quotient, and a / a
  // is exactly 1 (which keeps a stationary contact exactly invariant)
  static __device__ __forceinline__ double div(double a, double b) {
    const double r = rcp(b);
    const double q = a * r;
    return __builtin_fma(__builtin_fma(-b, q, a), r, q);
  }
  // a / b as div, and the refined reciprocal of b it used
  static __device__ __forceinline__ double div(double a, double b, double& rb) {
    rb = rcp(b);
    const double q = a * rb;
    return __builtin_fma(__builtin_fma(-b, q, a), rb, q);
  }
  // One Goldschmidt step from the hardware reciprocal square root y ~ 1/sqrt(x):
  // g = x y, h = y/2, r = 1/2 - g h, sqrt(x) ~ g + g r (about 2^-47 relative).
  // The estimate is taken at x + 2^-1074, which equals x for every x >=
  // 2^-1020 and keeps it finite at x = 0, where the step then yields 0 (x
  // itself enters, so sqrt(+-0) = +-0; negative or NaN x give NaN).
  // Subnormal x (never a density or pressure here) get a coarser estimate.
  static __device__ __forceinline__ double sqrt(double x) {
    const double y = __builtin_amdgcn_rsq(x + 0x1p-1074);
    const double g = x * y, h = 0.5 * y;
    const double r = __builtin_fma(-g, h, 0.5);
    return __builtin_fma(g, r, g);
  }
};

// FP32: single hardware reciprocal and square root (about 1 ulp); the FP32
// path is held to 1e-5 relative.
template <> struct Fp<float> {
  static __device__ __forceinline__ float rcp(float x) { return __builtin_amdgcn_rcpf(x); }
  static __device__ __forceinline__ float div(float a, float b) { return a * __builtin_amdgcn_rcpf(b); }
  static __device__ __forceinline__ float div(float a, float b, float& rb) {
    rb = __builtin_amdgcn_rcpf(b);
    return a * rb;
  }
  static __device__ __forceinline__ float sqrt(float x) { return __builtin_amdgcn_sqrtf(x); }
};

// Constants of one launch, already converted to T.
template <typename T> struct Gas {
  T gamma;      // adiabatic index
  T gm1;        // gamma - 1
  T inv_gm1;    // 1 / (gamma - 1)
  T theta;      // generalized minmod parameter
  T half_theta; // theta / 2
  T dtdx;       // dt / dx
  T half_dtdx;  // dt / (2 dx)
};

// ------------------------------------------------------- branch record ----
// Diagnostic: a thread folds the code of every decision its arithmetic takes
// (limiter case and argument, wave-speed argument, HLLC region) into a
// 32-bit hash (FNV-1a steps), so that two evaluations with equal records took
// the same branches (up to a hash collision).  A null pointer records
// nothing and compiles to nothing.
__device__ __forceinline__ void record(unsigned* rec, unsigned code) {
  if (rec != nullptr) *rec = (*rec ^ code) * 16777619u;
}

// ------------------------------------------------- a1: cons -> primitive --
// W = (rho, u, v, w, p), p = (gamma-1) (E - (m.u)/2).
template <typename T>
__device__ __forceinline__ void cons_to_prim(const T U[5], const Gas<T>& g, T W[5]) {
  const T inv = Fp<T>::rcp(U[0]);
  W[0] = U[0];
  W[1] = U[1] * inv;
  W[2] = U[2] * inv;
  W[3] = U[3] * inv;
  W[4] = g.gm1 * (U[4] - T(0.5) * (U[1] * W[1] + U[2] * W[2] + U[3] * W[3]));
}

// ------------------------------------------- a2: generalized minmod slope --
// Half of the limited slope, h = slope/2, so that the face values are q0 -+ h:
//   dm = q0 - qm, dp = qp - q0, slope = sgn(dc) min(theta|dm|, |dc|, theta|dp|)
//   with dc = (qp - qm)/2 if dm and dp have one strict sign, else 0.
// Scaling by 1/2 and 1/4 is exact, so h is bit-identical to slope/2.  The
// one-sign test is dm*dp > 0: it differs from testing the signs separately
// only when the product underflows (|dm|, |dp| < 1e-154 in FP64), where the
// slope itself is below any resolvable level.
// Recorded decision: 0 when the slope is zero, else 1 + the argument that
// attains the minimum (theta|dm|, |dc|, theta|dp|; the first on ties).
template <typename T>
__device__ __forceinline__ T half_slope(T qm, T q0, T qp, T half_theta, unsigned* rec = nullptr) {
  const T dm = q0 - qm;
  const T dp = qp - q0;
  const T a = half_theta * fabs_(dm), b = T(0.25) * fabs_(qp - qm), c = half_theta * fabs_(dp);
  T h = fmin_(a, b);
  h = fmin_(h, c);
  if (rec != nullptr) {
    unsigned code = 0;
    if (dm * dp > T(0)) {
      const T m = b < a ? b : a;
      code = c < m ? 3u : (b < a ? 2u : 1u);
    }
    record(rec, code);
  }
  return dm * dp > T(0) ? copysign_(h, dp) : T(0);
}

// ----------------------------------------- a3 + a4: Hancock face states ---
// Given the primitive state of a cell (Wc) and of its six axis neighbours
// (Wn[d][0] at -e_d, Wn[d][1] at +e_d), return the six face states advanced
// by half a step in conserved form, Ut[d][0] on the low face and Ut[d][1] on
// the high face of axis d:
//   W_{d,-+} = Wc -+ dW_d / 2;   U_{d,-+} = cons(W_{d,-+})
//   dU = dt/(2dx) sum_d [F_d(U_{d,-}) - F_d(U_{d,+})];   Ut = U + dU
template <typename T>
__device__ __forceinline__ void hancock_states(const T Wc[5], const T Wn[3][2][5], const Gas<T>& g,
                                               bool first_order, T Ut[3][2][5], unsigned* rec = nullptr) {
  T s[5];
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    T dF[5], h[5];
#pragma unroll
    for (int q = 0; q < 5; ++q)
      h[q] = first_order ? T(0) : half_slope(Wn[d][0][q], Wc[q], Wn[d][1][q], g.half_theta, rec);
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      T W[5];
#pragma unroll
      for (int q = 0; q < 5; ++q) W[q] = side == 0 ? Wc[q] - h[q] : Wc[q] + h[q];
      T* U = Ut[d][side];
      U[0] = W[0];
      U[1] = W[0] * W[1];
      U[2] = W[0] * W[2];
      U[3] = W[0] * W[3];
      U[4] = W[4] * g.inv_gm1 + T(0.5) * W[0] * (W[1] * W[1] + W[2] * W[2] + W[3] * W[3]);
      // physical flux along d of this face state
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
    for (int q = 0; q < 5; ++q) s[q] = d == 0 ? dF[q] : s[q] + dF[q];
  }
#pragma unroll
  for (int q = 0; q < 5; ++q) {
#pragma unroll
    for (int d = 0; d < 3; ++d) {
      Ut[d][0][q] = fma_(g.half_dtdx, s[q], Ut[d][0][q]);
      Ut[d][1][q] = fma_(g.half_dtdx, s[q], Ut[d][1][q]);
    }
  }
}

// Minimum / maximum that keep the first argument unless the second is
// strictly smaller / larger.  Unlike fmin/fmax (where a NaN operand loses),
// a NaN first argument propagates, so unphysical states give the same wave
// speeds, fluxes and unphysical counts as an evaluation written this way.
template <typename T>
__device__ __forceinline__ T min_first(T a, T b) { return b < a ? b : a; }
template <typename T>
__device__ __forceinline__ T max_first(T a, T b) { return b > a ? b : a; }

// ------------------------------------------------------------- a5: HLLC ---
// HLLC flux between left state L and right state R (conserved) for K
// independent faces, each given in its normal frame (index 1 the normal
// momentum, 2 and 3 the transverse ones in cyclic order).
// Wave speeds: Einfeldt / Roe-averaged (ws == 0) or Davis (ws == 1).
// Star state U*_K = r_K (rho_K, rho_K S*, m_t1, m_t2,
//                        E_K + (S* - u_K)(rho_K S* + p_K / (S_K - u_K))),
// r_K = (S_K - u_K) / (S_K - S*).  bad[k] is set when an input state of face
// k has rho <= 0 or p <= 0 (or is NaN); the flux is evaluated regardless.
// Every statement is taken for each face in turn: the K dependency chains
// share instruction blocks, so one face's latencies can be filled with
// another's work (a face solved alone leaves the wave waiting on each FP64
// result in turn).  The arithmetic of each face is that of one solve.
// Recorded decision per face: bit 0 S_L from its first argument, bit 1 S_R
// from its first argument, bits 2-3 the region (0 F_L, 1 F_R, 2 F*_L, 3 F*_R).
template <int K, typename T>
__device__ __forceinline__ void hllc_normal_k(const T L[K][5], const T R[K][5], const Gas<T>& g, int ws, T Fn[K][5],
                                              bool bad[K], unsigned* rec) {
  T rL[K], rR[K], iL[K], iR[K], uL[K], vL[K], wL[K], uR[K], vR[K], wR[K], pL[K], pR[K], cL[K], cR[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    rL[k] = L[k][0];
    rR[k] = R[k][0];
    iL[k] = Fp<T>::rcp(rL[k]);
    iR[k] = Fp<T>::rcp(rR[k]);
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    uL[k] = L[k][1] * iL[k], vL[k] = L[k][2] * iL[k], wL[k] = L[k][3] * iL[k];
    uR[k] = R[k][1] * iR[k], vR[k] = R[k][2] * iR[k], wR[k] = R[k][3] * iR[k];
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    pL[k] = g.gm1 * (L[k][4] - T(0.5) * (L[k][1] * uL[k] + L[k][2] * vL[k] + L[k][3] * wL[k]));
    pR[k] = g.gm1 * (R[k][4] - T(0.5) * (R[k][1] * uR[k] + R[k][2] * vR[k] + R[k][3] * wR[k]));
  }
#pragma unroll
  for (int k = 0; k < K; ++k) {
    bad[k] = !(rL[k] > T(0) && pL[k] > T(0) && rR[k] > T(0) && pR[k] > T(0));
    cL[k] = Fp<T>::sqrt(g.gamma * pL[k] * iL[k]);
    cR[k] = Fp<T>::sqrt(g.gamma * pR[k] * iR[k]);
  }

  T SL[K], SR[K];
  bool sl_first[K], sr_first[K];
  if (ws == 1) {
#pragma unroll
    for (int k = 0; k < K; ++k) {
      SL[k] = min_first(uL[k] - cL[k], uR[k] - cR[k]);
      SR[k] = max_first(uL[k] + cL[k], uR[k] + cR[k]);
      sl_first[k] = !(uR[k] - cR[k] < uL[k] - cL[k]);
      sr_first[k] = !(uR[k] + cR[k] > uL[k] + cL[k]);
    }
  } else {
    T sL[K], sR[K], iw[K], ua[K], va[K], wa[K], Ha[K], ca[K];
#pragma unroll
    for (int k = 0; k < K; ++k) {
      sL[k] = Fp<T>::sqrt(rL[k]);
      sR[k] = Fp<T>::sqrt(rR[k]);
    }
#pragma unroll
    for (int k = 0; k < K; ++k) iw[k] = Fp<T>::rcp(sL[k] + sR[k]);
#pragma unroll
    for (int k = 0; k < K; ++k) {
      ua[k] = (sL[k] * uL[k] + sR[k] * uR[k]) * iw[k];
      va[k] = (sL[k] * vL[k] + sR[k] * vR[k]) * iw[k];
      wa[k] = (sL[k] * wL[k] + sR[k] * wR[k]) * iw[k];
      Ha[k] = (sL[k] * ((L[k][4] + pL[k]) * iL[k]) + sR[k] * ((R[k][4] + pR[k]) * iR[k])) * iw[k];  // H = (E + p)/rho
    }
#pragma unroll
    for (int k = 0; k < K; ++k)
      ca[k] = Fp<T>::sqrt(g.gm1 * (Ha[k] - T(0.5) * (ua[k] * ua[k] + va[k] * va[k] + wa[k] * wa[k])));
#pragma unroll
    for (int k = 0; k < K; ++k) {
      SL[k] = min_first(uL[k] - cL[k], ua[k] - ca[k]);
      SR[k] = max_first(uR[k] + cR[k], ua[k] + ca[k]);
      sl_first[k] = !(ua[k] - ca[k] < uL[k] - cL[k]);
      sr_first[k] = !(ua[k] + ca[k] > uR[k] + cR[k]);
    }
  }
  T aL[K], aR[K], Ss[K];
#pragma unroll
  for (int k = 0; k < K; ++k) {
    aL[k] = SL[k] - uL[k];
    aR[k] = SR[k] - uR[k];
  }
#pragma unroll
  for (int k = 0; k < K; ++k)
    Ss[k] = Fp<T>::div(pR[k] - pL[k] + rL[k] * uL[k] * aL[k] - rR[k] * uR[k] * aR[k],
                       rL[k] * aL[k] - rR[k] * aR[k]);

  // Regions in the order S_L >= 0 -> F_L; else S* >= 0 -> F*_L; else
  // S_R > 0 -> F*_R; else F_R.  Only one side K enters (left when S_L >= 0 or
  // S* >= 0): the flux is F_K + Sc (U*_K - U_K) with Sc = S_K in the two star
  // regions and Sc = 0 in the two supersonic ones, where it is F_K exactly:
  // there U*_K is formed from S_K - u_K = 0, S* = 0 and the divisor 1, so it
  // stays finite whenever F_K is (also for an unphysical state whose S* or
  // S_K is NaN).  One set of selects of the side's inputs replaces three
  // candidate fluxes.
#pragma unroll
  for (int k = 0; k < K; ++k) {
    const bool left = SL[k] >= T(0) || Ss[k] >= T(0);
    const bool star = left ? !(SL[k] >= T(0)) : SR[k] > T(0);
    const T r = left ? rL[k] : rR[k], u = left ? uL[k] : uR[k], p = left ? pL[k] : pR[k];
    const T mn = left ? L[k][1] : R[k][1], m1 = left ? L[k][2] : R[k][2], m2 = left ? L[k][3] : R[k][3];
    const T E = left ? L[k][4] : R[k][4];
    const T S = left ? SL[k] : SR[k], a = left ? aL[k] : aR[k];
    if (rec != nullptr)
      record(rec, unsigned(sl_first[k]) | unsigned(sr_first[k]) << 1 |
                      (left ? (star ? 2u : 0u) : (star ? 3u : 1u)) << 2);
    const T Sc = star ? S : T(0);
    const T den = star ? S - Ss[k] : T(1);
    const T Sx = star ? Ss[k] : T(0), ax = star ? a : T(0);
    // r_K p_K / (S_K - u_K) = p_K / (S_K - S*): the energy term takes the
    // reciprocal of S_K - S* that r_K's division already formed
    T t;
    const T rr = Fp<T>::div(ax, den, t);
    const T Us0 = rr * r;
    const T Us1 = rr * (r * Sx);
    const T Us2 = rr * m1;
    const T Us3 = rr * m2;
    const T Us4 = rr * E + (Sx - u) * (Us1 + p * t);
    Fn[k][0] = mn + Sc * (Us0 - r);
    Fn[k][1] = (mn * u + p) + Sc * (Us1 - mn);
    Fn[k][2] = m1 * u + Sc * (Us2 - m1);
    Fn[k][3] = m2 * u + Sc * (Us3 - m2);
    Fn[k][4] = (E + p) * u + Sc * (Us4 - E);
  }
}

// HLLC flux across a face normal to axis D: the states taken into the normal
// frame (n, t1, t2) = (D, D+1, D+2) mod 3, the flux returned in the axis
// frame.  Returns true when an input state has rho <= 0 or p <= 0 (or NaN).
template <int D, typename T>
__device__ __forceinline__ bool hllc_flux(const T L[5], const T R[5], const Gas<T>& g, int ws, T F[5],
                                          unsigned* rec = nullptr) {
  constexpr int n = 1 + D, t1 = 1 + (D + 1) % 3, t2 = 1 + (D + 2) % 3;
  const T Ln[1][5] = {{L[0], L[n], L[t1], L[t2], L[4]}};
  const T Rn[1][5] = {{R[0], R[n], R[t1], R[t2], R[4]}};
  T Fn[1][5];
  bool bad[1];
  hllc_normal_k<1>(Ln, Rn, g, ws, Fn, bad, rec);
  F[0] = Fn[0][0];
  F[n] = Fn[0][1];
  F[t1] = Fn[0][2];
  F[t2] = Fn[0][3];
  F[4] = Fn[0][4];
  return bad[0];
}

// Two faces at once (normal axes D0 and D1), interleaved as in hllc_normal_k.
template <int D0, int D1, typename T>
__device__ __forceinline__ int hllc_flux2(const T L0[5], const T R0[5], const T L1[5], const T R1[5],
                                          const Gas<T>& g, int ws, T F0[5], T F1[5], unsigned* rec = nullptr) {
  constexpr int n0 = 1 + D0, a0 = 1 + (D0 + 1) % 3, b0 = 1 + (D0 + 2) % 3;
  constexpr int n1 = 1 + D1, a1 = 1 + (D1 + 1) % 3, b1 = 1 + (D1 + 2) % 3;
  const T Ln[2][5] = {{L0[0], L0[n0], L0[a0], L0[b0], L0[4]}, {L1[0], L1[n1], L1[a1], L1[b1], L1[4]}};
  const T Rn[2][5] = {{R0[0], R0[n0], R0[a0], R0[b0], R0[4]}, {R1[0], R1[n1], R1[a1], R1[b1], R1[4]}};
  T Fn[2][5];
  bool bad[2];
  hllc_normal_k<2>(Ln, Rn, g, ws, Fn, bad, rec);
  F0[0] = Fn[0][0];
  F0[n0] = Fn[0][1];
  F0[a0] = Fn[0][2];
  F0[b0] = Fn[0][3];
  F0[4] = Fn[0][4];
  F1[0] = Fn[1][0];
  F1[n1] = Fn[1][1];
  F1[a1] = Fn[1][2];
  F1[b1] = Fn[1][3];
  F1[4] = Fn[1][4];
  return int(bad[0]) + int(bad[1]);
}

// True when a conserved state has rho <= 0 or p <= 0 (or NaN).
template <typename T>
__device__ __forceinline__ bool unphysical(const T U[5], const Gas<T>& g) {
  const T inv = Fp<T>::rcp(U[0]);
  const T p = g.gm1 * (U[4] - T(0.5) * (U[1] * U[1] + U[2] * U[2] + U[3] * U[3]) * inv);
  return !(U[0] > T(0) && p > T(0));
}

// ------------------------------------------------ a8: CFL signal speed ----
// |u| + |v| + |w| + 3 c_s of one cell (Sec. 2.6 Eq. 2), in double, every
// operation IEEE-rounded and uncontracted, summed ((|u|+|v|)+|w|)+3c.  Both
// the standalone CFL kernel and the CFL epilogue of the fused step call this.
__device__ __forceinline__ double cfl_signal_speed(double rho, double mx, double my, double mz, double E,
                                                   double gamma) {
#pragma clang fp contract(off)
  const double u = mx / rho, v = my / rho, w = mz / rho;
  const double p = (gamma - 1.0) * (E - 0.5 * ((mx * u + my * v) + mz * w));
  const double c = __builtin_sqrt((gamma * p) / rho);
  return ((__builtin_fabs(u) + __builtin_fabs(v)) + __builtin_fabs(w)) + 3.0 * c;
}

}  // namespace gh
