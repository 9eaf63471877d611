// HLLD Riemann solver (Miyoshi & Kusano 2005), the MHD flux of Sec. 2.3, for a
// face normal to coordinate axis D, shared by the 2D and 3D MHD kernels.
#pragma once

#include <hip/hip_runtime.h>

#include "dg_math.h"

namespace dg {

// ----------------------------------------------------------------- HLLD --
// States in the lab frame, conserved order rho, mx, my, mz, E, Bx, By, Bz;
// both carry the same normal field B[D].  Returns the lab-frame flux along
// +e_D (its B[D] component is zero).
//
// Miyoshi & Kusano's fan has outer waves S_L < S_R, Alfven waves S*_L, S*_R
// and the contact S_M.  The interface lies on the left of the contact exactly
// when S_M >= 0 (S_L >= 0 implies S_M > 0, S_R <= 0 implies S_M < 0), so the
// flux is built from one side a only:
//   F = F_a                                         (outside the fan)
//     = F_a + S_a (U*_a - U_a)                      (between S_a and S*_a)
//     = F_a + S_a (U*_a - U_a) + S*_a (U**_a - U*_a)  (between S*_a and S_M)
// with S_M, p*_T and the double-star states taken from both sides.
template <typename T, int D>
__device__ __forceinline__ void hlld_axis(const T* uL, const T* uR, T gamma, T eps, T* F,
                                          bool& bad) {
  constexpr int n = D, t1 = (D + 1) % 3, t2 = (D + 2) % 3;
  const T g = gamma, gm1 = gamma - T(1);
  const T Bn = uL[5 + n];
  const T Bn2 = Bn * Bn;
  // face-frame primitive variables: normal velocity u, tangential v, w,
  // tangential field b1, b2, total pressure pT, fast speed cf
  T u[2], v[2], w[2], pT[2], cf[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const T* q = s == 0 ? uL : uR;
    T ir = rcp(q[0]);
    u[s] = q[1 + n] * ir;
    v[s] = q[1 + t1] * ir;
    w[s] = q[1 + t2] * ir;
    T pm = T(0.5) * (Bn2 + q[5 + t1] * q[5 + t1] + q[5 + t2] * q[5 + t2]);
    T pg = gm1 * (q[4] - T(0.5) * (q[1 + n] * u[s] + q[1 + t1] * v[s] + q[1 + t2] * w[s]) - pm);
    bad |= !(q[0] > T(0)) || !(pg > T(0));
    pT[s] = pg + pm;
    T a2 = g * pg * ir;
    T sb = a2 + T(2) * pm * ir;
    T disc = fmax(sb * sb - T(4) * a2 * Bn2 * ir, T(0));
    cf[s] = sqrt_pos(T(0.5) * (sb + sqrt_nn(disc)));
  }
  const T cmax = fmax(cf[0], cf[1]);
  const T SL = fmin(u[0], u[1]) - cmax;
  const T SR = fmax(u[0], u[1]) + cmax;
  const T dL = (SL - u[0]) * uL[0], dR = (SR - u[1]) * uR[0];  // rho (S - u)
  const T idn = rcp(dR - dL);
  const T SM = (dR * u[1] - dL * u[0] - pT[1] + pT[0]) * idn;
  const T pTs = (dR * pT[0] - dL * pT[1] + dL * dR * (u[1] - u[0])) * idn;
  // single-star tangential states of both sides (needed by the double star)
  T rs[2], vs[2], ws[2], b1s[2], b2s[2], sq[2];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    const T* q = s == 0 ? uL : uR;
    const T S = s == 0 ? SL : SR;
    const T dS = s == 0 ? dL : dR;
    const T Su = S - u[s];
    rs[s] = dS * rcp(S - SM);
    const T den = dS * (S - SM) - Bn2;
    const T scale = dS * Su + Bn2;
    const bool deg = fabs(den) <= eps * scale;
    const T iden = deg ? T(0) : rcp(den);
    const T fv = deg ? T(0) : Bn * (SM - u[s]) * iden;
    const T fb = deg ? T(1) : (dS * Su - Bn2) * iden;
    vs[s] = v[s] - q[5 + t1] * fv;
    ws[s] = w[s] - q[5 + t2] * fv;
    b1s[s] = q[5 + t1] * fb;
    b2s[s] = q[5 + t2] * fb;
    sq[s] = sqrt_pos(rs[s]);
  }
  const T sgn = Bn < T(0) ? T(-1) : T(1);
  const T isum = rcp(sq[0] + sq[1]);
  const T vss = (sq[0] * vs[0] + sq[1] * vs[1] + (b1s[1] - b1s[0]) * sgn) * isum;
  const T wss = (sq[0] * ws[0] + sq[1] * ws[1] + (b2s[1] - b2s[0]) * sgn) * isum;
  const T b1ss = (sq[0] * b1s[1] + sq[1] * b1s[0] + sq[0] * sq[1] * (vs[1] - vs[0]) * sgn) * isum;
  const T b2ss = (sq[0] * b2s[1] + sq[1] * b2s[0] + sq[0] * sq[1] * (ws[1] - ws[0]) * sgn) * isum;
  // side a
  const bool lft = SM >= T(0);
  const T* q = lft ? uL : uR;
  const T S = lft ? SL : SR;
  const T ua = lft ? u[0] : u[1], va = lft ? v[0] : v[1], wa = lft ? w[0] : w[1];
  const T pTa = lft ? pT[0] : pT[1];
  const T rsa = lft ? rs[0] : rs[1], vsa = lft ? vs[0] : vs[1], wsa = lft ? ws[0] : ws[1];
  const T b1sa = lft ? b1s[0] : b1s[1], b2sa = lft ? b2s[0] : b2s[1];
  const T sqa = lft ? sq[0] : sq[1];
  const T Ss = lft ? SM - fabs(Bn) * rcp(sqa) : SM + fabs(Bn) * rcp(sqa);
  const bool outer = lft ? (SL >= T(0)) : (SR <= T(0));
  const bool single = lft ? (Ss >= T(0)) : (Ss <= T(0));
  const T b1 = q[5 + t1], b2 = q[5 + t2];
  const T vB = ua * Bn + va * b1 + wa * b2;
  const T vBs = SM * Bn + vsa * b1sa + wsa * b2sa;
  const T Es = ((S - ua) * q[4] - pTa * ua + pTs * SM + Bn * (vB - vBs)) * rcp(S - SM);
  const T vBss = SM * Bn + vss * b1ss + wss * b2ss;
  const T Ess = lft ? Es - sqa * (vBs - vBss) * sgn : Es + sqa * (vBs - vBss) * sgn;
  // outer flux and states of side a, components (rho, m_n, m_t1, m_t2, E, B_t1, B_t2)
  const T mu = q[1 + n];
  const T Fa[7] = {mu, mu * ua + pTa - Bn2, mu * va - Bn * b1, mu * wa - Bn * b2,
                   (q[4] + pTa) * ua - Bn * vB, b1 * ua - va * Bn, b2 * ua - wa * Bn};
  const T Ua[7] = {q[0], q[1 + n], q[1 + t1], q[1 + t2], q[4], b1, b2};
  const T Us[7] = {rsa, rsa * SM, rsa * vsa, rsa * wsa, Es, b1sa, b2sa};
  const T Uss[7] = {rsa, rsa * SM, rsa * vss, rsa * wss, Ess, b1ss, b2ss};
  T Fo[7];
#pragma unroll
  for (int k = 0; k < 7; ++k) {
    const T fs = fma(S, Us[k] - Ua[k], Fa[k]);
    const T fss = fma(Ss, Uss[k] - Us[k], fs);
    Fo[k] = outer ? Fa[k] : (single ? fs : fss);
  }
  F[0] = Fo[0];
  F[1 + n] = Fo[1];
  F[1 + t1] = Fo[2];
  F[1 + t2] = Fo[3];
  F[4] = Fo[4];
  F[5 + n] = T(0);
  F[5 + t1] = Fo[5];
  F[5 + t2] = Fo[6];
}

}  // namespace dg
