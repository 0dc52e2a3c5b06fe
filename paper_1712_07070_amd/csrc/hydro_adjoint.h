// Reverse-mode (vector-Jacobian) counterparts of the MHM step's device
// arithmetic in hydro_device.h.  Each *_vjp routine recomputes the forward
// intermediates it needs from the same inputs (so branch decisions -- limiter
// case, HLLC branch, min/max of wave speeds -- are taken exactly as in the
// forward pass) and returns the cotangents of its inputs given the cotangents
// of its outputs.
//
// Derivative conventions at non-smooth points (shared with the oracle's
// dual-number instantiation):
//   * limiter: zero when the one-sided differences are not strictly of one
//     sign; otherwise through the argument attaining the minimum, the first of
//     (theta|dm|, |dc|, theta|dp|) on ties; the sign factor has zero derivative;
//   * min/max of wave speeds: through the first argument unless the second is
//     strictly smaller/larger;
//   * HLLC: the derivative of the branch the forward pass took.
#pragma once

#include "hydro_device.h"

namespace gh {

// ----------------------------------------------- a1: cons -> primitive VJP --
// W = (rho, m/rho, p) with p = gm1 (E - (m.u)/2).  Given gW, add gU.
template <typename T>
__device__ __forceinline__ void cons_to_prim_vjp(const T U[5], const Gas<T>& g, const T gW[5], T gU[5]) {
  const T inv = Fp<T>::rcp(U[0]);
  const T u = U[1] * inv, v = U[2] * inv, w = U[3] * inv;
  const T gp = gW[4] * g.gm1;
  // p = gm1 (E - (m_x u + m_y v + m_z w)/2): dp/dm_i = -gm1 u_i, dp/drho = gm1 |u|^2 / 2
  gU[0] = gU[0] + gW[0] - (gW[1] * u + gW[2] * v + gW[3] * w) * inv + T(0.5) * gp * (u * u + v * v + w * w);
  gU[1] = gU[1] + gW[1] * inv - gp * u;
  gU[2] = gU[2] + gW[2] * inv - gp * v;
  gU[3] = gU[3] + gW[3] * inv - gp * w;
  gU[4] = gU[4] + gp;
}

// -------------------------------------------------- a2: limiter VJP -------
// h = half_slope(qm, q0, qp); given gh, add to gqm, gq0, gqp.
template <typename T>
__device__ __forceinline__ void half_slope_vjp(T qm, T q0, T qp, T half_theta, T gh, T& gqm, T& gq0, T& gqp) {
  const T dm = q0 - qm;
  const T dp = qp - q0;
  if (!(dm * dp > T(0))) return;
  const T a = half_theta * fabs_(dm);
  const T b = T(0.25) * fabs_(qp - qm);
  const T c = half_theta * fabs_(dp);
  // h = sgn * min(...) with sgn the common sign: h = half_theta*dm, (qp-qm)/4 or half_theta*dp
  int sel = 0;
  T m = a;
  if (b < m) {
    sel = 1;
    m = b;
  }
  if (c < m) sel = 2;
  if (sel == 0) {
    gq0 = gq0 + half_theta * gh;
    gqm = gqm - half_theta * gh;
  } else if (sel == 1) {
    gqp = gqp + T(0.25) * gh;
    gqm = gqm - T(0.25) * gh;
  } else {
    gqp = gqp + half_theta * gh;
    gq0 = gq0 - half_theta * gh;
  }
}

// ------------------------------------------- a3 + a4: Hancock states VJP ---
// Forward: hancock_states(Wc, Wn, g, first_order, Ut).  Streaming form: the
// neighbour states, the face-state cotangents and the neighbour outputs are
// reached through callbacks, one direction at a time, so that a caller can
// keep them in LDS and only one direction's values are live at once.
//   getW(d, side, T W[5])   primitive state of neighbour (d, side)
//   getG(d, side, T g[5])   cotangent gUt[d][side] (zero for unused faces)
//   putN(d, side, T g[5])   receives the cotangent of neighbour (d, side)
//   gWc                     receives the cotangent of the cell's own state
template <typename T, class GetW, class GetG, class PutN>
__device__ __forceinline__ void hancock_states_vjp_stream(const T Wc[5], const Gas<T>& g, bool first_order,
                                                          GetW&& getW, GetG&& getG, PutN&& putN, T gWc[5]) {
  // dU = half_dtdx * sum_d (F_d(-) - F_d(+)); every face state receives dU
  T gdU[5] = {T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    T a[5], b[5];
    getG(d, 0, a);
    getG(d, 1, b);
#pragma unroll
    for (int q = 0; q < 5; ++q) gdU[q] = gdU[q] + (a[q] + b[q]);
  }
#pragma unroll
  for (int q = 0; q < 5; ++q) {
    gdU[q] = g.half_dtdx * gdU[q];
    gWc[q] = T(0);
  }
  // the face cotangents are fetched again per direction below: keep the
  // compiler from holding all six vectors live across the loop
  asm volatile("" ::: "memory");
#pragma unroll
  for (int d = 0; d < 3; ++d) {
    T Wl[5], Wr[5];
    getW(d, 0, Wl);
    getW(d, 1, Wr);
    T h[5];
#pragma unroll
    for (int q = 0; q < 5; ++q) h[q] = first_order ? T(0) : half_slope(Wl[q], Wc[q], Wr[q], g.half_theta);
    T gh[5] = {T(0), T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int side = 0; side < 2; ++side) {
      const T sgn = side == 0 ? T(1) : T(-1);  // face flux enters dU with this sign
      T W[5];
#pragma unroll
      for (int q = 0; q < 5; ++q) W[q] = side == 0 ? Wc[q] - h[q] : Wc[q] + h[q];
      const T rho = W[0], u = W[1], v = W[2], w = W[3], p = W[4];
      const T U1 = rho * u, U2 = rho * v, U3 = rho * w;
      const T U4 = p * g.inv_gm1 + T(0.5) * rho * (u * u + v * v + w * w);
      const T un = W[1 + d];
      T gUt[5];
      getG(d, side, gUt);
      // cotangent of this face state's conserved variables: direct + via its flux
      T gF[5];
#pragma unroll
      for (int q = 0; q < 5; ++q) gF[q] = sgn * gdU[q];
      T gU[5];
#pragma unroll
      for (int q = 0; q < 5; ++q) gU[q] = gUt[q] + gF[q] * un;
      // flux: F = U * un (+ p on the normal momentum), F4 = (U4 + p) un
      T gW[5] = {T(0), T(0), T(0), T(0), T(0)};
      gW[1 + d] = gF[0] * rho + gF[1] * U1 + gF[2] * U2 + gF[3] * U3 + gF[4] * (U4 + p);
      gW[4] = gF[1 + d] + gF[4] * un;
      // cons: U = (rho, rho u, rho v, rho w, p/gm1 + rho |u|^2 / 2)
      gW[0] = gW[0] + gU[0] + gU[1] * u + gU[2] * v + gU[3] * w + gU[4] * (T(0.5) * (u * u + v * v + w * w));
      gW[1] = gW[1] + gU[1] * rho + gU[4] * (rho * u);
      gW[2] = gW[2] + gU[2] * rho + gU[4] * (rho * v);
      gW[3] = gW[3] + gU[3] * rho + gU[4] * (rho * w);
      gW[4] = gW[4] + gU[4] * g.inv_gm1;
      // W_{d,-} = Wc - h, W_{d,+} = Wc + h
#pragma unroll
      for (int q = 0; q < 5; ++q) {
        gWc[q] = gWc[q] + gW[q];
        gh[q] = side == 0 ? gh[q] - gW[q] : gh[q] + gW[q];
      }
    }
    T gl[5] = {T(0), T(0), T(0), T(0), T(0)}, gr[5] = {T(0), T(0), T(0), T(0), T(0)};
    if (!first_order) {
#pragma unroll
      for (int q = 0; q < 5; ++q) half_slope_vjp(Wl[q], Wc[q], Wr[q], g.half_theta, gh[q], gl[q], gWc[q], gr[q]);
    }
    putN(d, 0, gl);
    putN(d, 1, gr);
  }
}

// Array form: gWc (the cell's own primitive state) and gWn[3][2][5] (its six
// neighbours), overwriting both.
template <typename T>
__device__ __forceinline__ void hancock_states_vjp(const T Wc[5], const T Wn[3][2][5], const Gas<T>& g,
                                                   bool first_order, const T gUt[3][2][5], T gWc[5],
                                                   T gWn[3][2][5]) {
  hancock_states_vjp_stream(
      Wc, g, first_order,
      [&](int d, int side, T W[5]) {
#pragma unroll
        for (int q = 0; q < 5; ++q) W[q] = Wn[d][side][q];
      },
      [&](int d, int side, T G[5]) {
#pragma unroll
        for (int q = 0; q < 5; ++q) G[q] = gUt[d][side][q];
      },
      [&](int d, int side, const T G[5]) {
#pragma unroll
        for (int q = 0; q < 5; ++q) gWn[d][side][q] = G[q];
      },
      gWc);
}

// ---------------------------------------------------------- a5: HLLC VJP ---
// Forward: hllc_flux<D>(L, R, g, ws, F).  Given gF (axis frame), add the
// cotangents of the two conserved input states to gL and gR.
template <int D, typename T>
__device__ __forceinline__ void hllc_flux_vjp(const T Lx[5], const T Rx[5], const Gas<T>& g, int ws, const T gFx[5],
                                              T gLx[5], T gRx[5]) {
  constexpr int n = 1 + D, t1 = 1 + (D + 1) % 3, t2 = 1 + (D + 2) % 3;
  // normal frame
  const T rL = Lx[0], mnL = Lx[n], m1L = Lx[t1], m2L = Lx[t2], EL = Lx[4];
  const T rR = Rx[0], mnR = Rx[n], m1R = Rx[t1], m2R = Rx[t2], ER = Rx[4];
  const T gF[5] = {gFx[0], gFx[n], gFx[t1], gFx[t2], gFx[4]};
  // ---- forward recomputation
  const T iL = Fp<T>::rcp(rL), iR = Fp<T>::rcp(rR);
  const T uL = mnL * iL, vL = m1L * iL, wL = m2L * iL;
  const T uR = mnR * iR, vR = m1R * iR, wR = m2R * iR;
  const T pL = g.gm1 * (EL - T(0.5) * (mnL * uL + m1L * vL + m2L * wL));
  const T pR = g.gm1 * (ER - T(0.5) * (mnR * uR + m1R * vR + m2R * wR));
  const T cL = Fp<T>::sqrt(g.gamma * pL * iL);
  const T cR = Fp<T>::sqrt(g.gamma * pR * iR);
  T sL = T(0), sR = T(0), iw = T(0), ua = T(0), va = T(0), wa = T(0), HL = T(0), HR = T(0), Ha = T(0), ca = T(0);
  T SL, SR;
  bool sl_first, sr_first;
  if (ws == 1) {
    const T a1 = uL - cL, b1 = uR - cR, a2 = uL + cL, b2 = uR + cR;
    sl_first = !(b1 < a1);
    sr_first = !(b2 > a2);
    SL = sl_first ? a1 : b1;
    SR = sr_first ? a2 : b2;
  } else {
    sL = Fp<T>::sqrt(rL);
    sR = Fp<T>::sqrt(rR);
    iw = Fp<T>::rcp(sL + sR);
    ua = (sL * uL + sR * uR) * iw;
    va = (sL * vL + sR * vR) * iw;
    wa = (sL * wL + sR * wR) * iw;
    HL = (EL + pL) * iL;
    HR = (ER + pR) * iR;
    Ha = (sL * HL + sR * HR) * iw;
    ca = Fp<T>::sqrt(g.gm1 * (Ha - T(0.5) * (ua * ua + va * va + wa * wa)));
    const T a1 = uL - cL, b1 = ua - ca, a2 = uR + cR, b2 = ua + ca;
    sl_first = !(b1 < a1);
    sr_first = !(b2 > a2);
    SL = sl_first ? a1 : b1;
    SR = sr_first ? a2 : b2;
  }
  const T aL = SL - uL, aR = SR - uR;
  const T num = pR - pL + rL * uL * aL - rR * uR * aR;
  const T den = rL * aL - rR * aR;
  const T Ss = Fp<T>::div(num, den);

  // ---- reverse
  T grL = T(0), gmnL = T(0), gm1L = T(0), gm2L = T(0), gEL = T(0);
  T grR = T(0), gmnR = T(0), gm1R = T(0), gm2R = T(0), gER = T(0);
  T guL = T(0), gpL = T(0), guR = T(0), gpR = T(0);
  T gSL = T(0), gSR = T(0), gSs = T(0), gaL = T(0), gaR = T(0);

  if (SL >= T(0)) {
    // F = (mn, mn u + p, m1 u, m2 u, (E + p) u) of L
    gmnL = gF[0] + gF[1] * uL;
    guL = gF[1] * mnL + gF[2] * m1L + gF[3] * m2L + gF[4] * (EL + pL);
    gpL = gF[1] + gF[4] * uL;
    gm1L = gF[2] * uL;
    gm2L = gF[3] * uL;
    gEL = gF[4] * uL;
  } else if (!(Ss >= T(0)) && !(SR > T(0))) {
    gmnR = gF[0] + gF[1] * uR;
    guR = gF[1] * mnR + gF[2] * m1R + gF[3] * m2R + gF[4] * (ER + pR);
    gpR = gF[1] + gF[4] * uR;
    gm1R = gF[2] * uR;
    gm2R = gF[3] * uR;
    gER = gF[4] * uR;
  } else {
    const bool left = Ss >= T(0);
    const T r = left ? rL : rR, u = left ? uL : uR, p = left ? pL : pR;
    const T mn = left ? mnL : mnR, m1 = left ? m1L : m1R, m2 = left ? m2L : m2R, E = left ? EL : ER;
    const T S = left ? SL : SR, a = left ? aL : aR;
    const T Dn = S - Ss;
    const T iD = Fp<T>::rcp(Dn);
    const T rr = Fp<T>::div(a, Dn);
    const T ia = Fp<T>::rcp(a);
    const T Q = r * Ss + p * ia;
    const T G = E + (Ss - u) * Q;
    const T Us4 = rr * G;
    // F0 = mn + S (rr r - r), F1 = mn u + p + S (rr r Ss - mn), F2 = m1 u + S (rr m1 - m1),
    // F3 = m2 u + S (rr m2 - m2), F4 = (E + p) u + S (rr G - E)
    const T gS = gF[0] * (rr * r - r) + gF[1] * (rr * r * Ss - mn) + gF[2] * (rr * m1 - m1) +
                 gF[3] * (rr * m2 - m2) + gF[4] * (Us4 - E);
    const T grr = S * (gF[0] * r + gF[1] * r * Ss + gF[2] * m1 + gF[3] * m2 + gF[4] * G);
    const T gG = S * rr * gF[4];
    T gr = gF[0] * S * (rr - T(1)) + gF[1] * S * rr * Ss + gG * (Ss - u) * Ss;
    T gSs_s = gF[1] * S * rr * r + gG * (Q + (Ss - u) * r);
    const T gmn = gF[0] + gF[1] * (u - S);
    T gu = gF[1] * mn + gF[2] * m1 + gF[3] * m2 + gF[4] * (E + p) - gG * Q;
    const T gp = gF[1] + gF[4] * u + gG * (Ss - u) * ia;
    T ga = -gG * (Ss - u) * p * ia * ia;
    const T gm1 = gF[2] * (u + S * (rr - T(1)));
    const T gm2 = gF[3] * (u + S * (rr - T(1)));
    const T gE = gF[4] * (u - S) + gG;
    // rr = a / (S - Ss)
    ga = ga + grr * iD;
    const T gDn = -grr * rr * iD;
    T gSk = gS + gDn;
    gSs_s = gSs_s - gDn;
    // a = S - u
    gSk = gSk + ga;
    gu = gu - ga;
    gSs = gSs + gSs_s;
    if (left) {
      grL = grL + gr; guL = guL + gu; gpL = gpL + gp; gmnL = gmnL + gmn; gm1L = gm1L + gm1; gm2L = gm2L + gm2;
      gEL = gEL + gE; gSL = gSL + gSk;
    } else {
      grR = grR + gr; guR = guR + gu; gpR = gpR + gp; gmnR = gmnR + gmn; gm1R = gm1R + gm1; gm2R = gm2R + gm2;
      gER = gER + gE; gSR = gSR + gSk;
    }
  }

  // S* = num / den (its cotangent is nonzero only in the star branches)
  {
    const T iden = Fp<T>::rcp(den);
    const T gnum = gSs * iden;
    const T gden = -gSs * Ss * iden;
    gpR = gpR + gnum;
    gpL = gpL - gnum;
    grL = grL + gnum * uL * aL + gden * aL;
    guL = guL + gnum * rL * aL;
    gaL = gaL + gnum * rL * uL + gden * rL;
    grR = grR - gnum * uR * aR - gden * aR;
    guR = guR - gnum * rR * aR;
    gaR = gaR - gnum * rR * uR - gden * rR;
  }
  // aL = SL - uL, aR = SR - uR
  gSL = gSL + gaL;
  guL = guL - gaL;
  gSR = gSR + gaR;
  guR = guR - gaR;

  // wave speeds
  T gcL = T(0), gcR = T(0), gua = T(0), gca = T(0);
  if (ws == 1) {
    if (sl_first) { guL = guL + gSL; gcL = gcL - gSL; } else { guR = guR + gSL; gcR = gcR - gSL; }
    if (sr_first) { guL = guL + gSR; gcL = gcL + gSR; } else { guR = guR + gSR; gcR = gcR + gSR; }
  } else {
    if (sl_first) { guL = guL + gSL; gcL = gcL - gSL; } else { gua = gua + gSL; gca = gca - gSL; }
    if (sr_first) { guR = guR + gSR; gcR = gcR + gSR; } else { gua = gua + gSR; gca = gca + gSR; }
    // ca = sqrt(gm1 (Ha - |ua|^2/2))
    const T gca2 = gca * T(0.5) * Fp<T>::rcp(ca);
    const T gHa = g.gm1 * gca2;
    gua = gua - g.gm1 * gca2 * ua;
    const T gva = -g.gm1 * gca2 * va;
    const T gwa = -g.gm1 * gca2 * wa;
    // Roe averages: X = (sL xL + sR xR) iw for x in u, v, w, H
    T gsL = (gua * uL + gva * vL + gwa * wL + gHa * HL) * iw;
    T gsR = (gua * uR + gva * vR + gwa * wR + gHa * HR) * iw;
    guL = guL + gua * sL * iw;
    guR = guR + gua * sR * iw;
    const T gvL = gva * sL * iw, gvR = gva * sR * iw;
    const T gwL = gwa * sL * iw, gwR = gwa * sR * iw;
    const T gHL = gHa * sL * iw, gHR = gHa * sR * iw;
    const T giw = gua * (sL * uL + sR * uR) + gva * (sL * vL + sR * vR) + gwa * (sL * wL + sR * wR) +
                  gHa * (sL * HL + sR * HR);
    const T gsum = -giw * iw * iw;
    gsL = gsL + gsum;
    gsR = gsR + gsum;
    // H = (E + p) / rho
    gEL = gEL + gHL * iL;
    gpL = gpL + gHL * iL;
    grL = grL - gHL * HL * iL;
    gER = gER + gHR * iR;
    gpR = gpR + gHR * iR;
    grR = grR - gHR * HR * iR;
    // v, w of each side through m_t / rho
    gm1L = gm1L + gvL * iL;
    gm2L = gm2L + gwL * iL;
    grL = grL - (gvL * vL + gwL * wL) * iL;
    gm1R = gm1R + gvR * iR;
    gm2R = gm2R + gwR * iR;
    grR = grR - (gvR * vR + gwR * wR) * iR;
    // sqrt(rho)
    grL = grL + gsL * T(0.5) * Fp<T>::rcp(sL);
    grR = grR + gsR * T(0.5) * Fp<T>::rcp(sR);
  }
  // c = sqrt(gamma p / rho)
  {
    const T gxL = gcL * T(0.5) * Fp<T>::rcp(cL);
    gpL = gpL + gxL * g.gamma * iL;
    grL = grL - gxL * g.gamma * pL * iL * iL;
    const T gxR = gcR * T(0.5) * Fp<T>::rcp(cR);
    gpR = gpR + gxR * g.gamma * iR;
    grR = grR - gxR * g.gamma * pR * iR * iR;
  }
  // p = gm1 (E - (mn u + m1 v + m2 w)/2) written on conserved variables:
  // dp/dE = gm1, dp/dm_i = -gm1 u_i, dp/drho = gm1 |u|^2 / 2
  gEL = gEL + g.gm1 * gpL;
  gmnL = gmnL - g.gm1 * gpL * uL;
  gm1L = gm1L - g.gm1 * gpL * vL;
  gm2L = gm2L - g.gm1 * gpL * wL;
  grL = grL + T(0.5) * g.gm1 * gpL * (uL * uL + vL * vL + wL * wL);
  gER = gER + g.gm1 * gpR;
  gmnR = gmnR - g.gm1 * gpR * uR;
  gm1R = gm1R - g.gm1 * gpR * vR;
  gm2R = gm2R - g.gm1 * gpR * wR;
  grR = grR + T(0.5) * g.gm1 * gpR * (uR * uR + vR * vR + wR * wR);
  // u = mn / rho
  gmnL = gmnL + guL * iL;
  grL = grL - guL * uL * iL;
  gmnR = gmnR + guR * iR;
  grR = grR - guR * uR * iR;
  // back to the axis frame
  gLx[0] = gLx[0] + grL;
  gLx[n] = gLx[n] + gmnL;
  gLx[t1] = gLx[t1] + gm1L;
  gLx[t2] = gLx[t2] + gm2L;
  gLx[4] = gLx[4] + gEL;
  gRx[0] = gRx[0] + grR;
  gRx[n] = gRx[n] + gmnR;
  gRx[t1] = gRx[t1] + gm1R;
  gRx[t2] = gRx[t2] + gm2R;
  gRx[4] = gRx[4] + gER;
}

}  // namespace gh
