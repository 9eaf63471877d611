// Exact Riemann solver for the 2D Euler equations (the Euler face flux of
// Sec. 2.3), for a face normal to coordinate axis AX, on gfx950.
//
// In the face frame the solution of the Riemann problem between uL and uR is
// self-similar: a left wave, a contact moving with u*, a right wave; each outer
// wave is a shock (p* > p_K, Rankine-Hugoniot conditions) or a rarefaction
// (p* <= p_K, isentropic with a Riemann invariant).  Across the wave of side K
// the normal velocity changes by f_K(p*), so p* is the root of
//   f_L(p) + f_R(p) + u_R - u_L = 0,
// solved by Newton's method; u* = (u_L + u_R)/2 + (f_R(p*) - f_L(p*))/2.
// The flux is the physical flux of the solution on the face (x/t = 0), with
// the tangential velocity of the side upwind of the contact.  A lane that
// meets vacuum generation or a non-physical input raises `bad` (its flux is
// then not meaningful); every lane leaves the Newton loop after at most
// kExactMaxIter iterations.
//
// FP64 powers are software routines on gfx950, so the solver avoids them
// where an algebraically equal form exists:
// * the Newton start is the linearised (primitive-variable) estimate
//   p = (p_L + p_R)/2 - (u_R - u_L)(rho_L + rho_R)(c_L + c_R)/8 when the two
//   pressures are within a factor 2 and the estimate lies between them (weak
//   waves, where it is accurate to second order in the jump); otherwise the
//   two-rarefaction value, exact when both waves are rarefactions;
// * when the Newton step falls below the tolerance, f_L and f_R are carried
//   to the new p* along their tangents (the neglected term is of the order of
//   the squared step) instead of being evaluated again;
// * behind a rarefaction of side K the sound speed follows from the Riemann
//   invariant, c* = c_K + (gamma - 1) f_K(p*)/2, and the density from the
//   isentrope, rho* = gamma p*/c*^2; in the fan p = rho c^2/gamma.
#pragma once

#include <hip/hip_runtime.h>

#include "dg_math.h"

namespace dg {

constexpr int kExactMaxIter = 40;

// x^e for x > 0.
__device__ __forceinline__ double pow_pos(double x, double e) { return exp2(e * log2(x)); }
__device__ __forceinline__ float pow_pos(float x, float e) { return exp2f(e * log2f(x)); }

template <typename T>
struct ESide {
  T r, u, p, c;
};

// Velocity change f across the wave of one side at pressure ps, and df/dp.
template <typename T>
__device__ __forceinline__ void wave_relation(T ps, const ESide<T>& s, T gamma, T& f, T& df) {
  if (ps > s.p) {
    const T A = T(2) * rcp((gamma + T(1)) * s.r);
    const T B = (gamma - T(1)) * rcp(gamma + T(1)) * s.p;
    const T ipb = rcp(ps + B);
    const T q = sqrt_pos(A * ipb);
    f = (ps - s.p) * q;
    df = q * (T(1) - T(0.5) * (ps - s.p) * ipb);
  } else {
    const T z = (gamma - T(1)) * rcp(T(2) * gamma);
    const T rr = pow_pos(ps * rcp(s.p), z);
    f = T(2) * rcp(gamma - T(1)) * s.c * (rr - T(1));
    df = rr * s.p * rcp(ps * s.r * s.c);
  }
}

// Flux along +e_AX between conserved states (rho, m_x, m_y, E).
template <typename T, int AX>
__device__ __forceinline__ void exact_flux(const T* uL, const T* uR, T gamma, T* F, bool& bad) {
  constexpr int TX = 1 - AX;
  const T gm1 = gamma - T(1);
  const T tol = sizeof(T) == 8 ? T(1e-15) : T(1e-6);
  ESide<T> s[2];
  T ut[2];
#pragma unroll
  for (int a = 0; a < 2; ++a) {
    const T* q = a == 0 ? uL : uR;
    const T ir = rcp(q[0]);
    const T un = q[1 + AX] * ir, vt = q[1 + TX] * ir;
    const T p = gm1 * (q[3] - T(0.5) * (q[1 + AX] * un + q[1 + TX] * vt));
    bad |= !(q[0] > T(0)) || !(p > T(0));
    s[a].r = q[0];
    s[a].u = un;
    s[a].p = p;
    s[a].c = sqrt_pos(gamma * p * ir);
    ut[a] = vt;
  }
  const T du = s[1].u - s[0].u;
  bad |= !(T(2) * rcp(gm1) * (s[0].c + s[1].c) > du);
  const T z = gm1 * rcp(T(2) * gamma);
  const T pmin = fmin(s[0].p, s[1].p), pmax = fmax(s[0].p, s[1].p);
  T ps = T(0.5) * (s[0].p + s[1].p) - T(0.125) * du * (s[0].r + s[1].r) * (s[0].c + s[1].c);
  if (!(pmax <= T(2) * pmin && ps >= pmin && ps <= pmax))
    ps = pow_pos((s[0].c + s[1].c - T(0.5) * gm1 * du) *
                     rcp(s[0].c * pow_pos(s[0].p, -z) + s[1].c * pow_pos(s[1].p, -z)),
                 rcp(z));
  T fL, dfL, fR, dfR;
  bool conv = false;
  for (int it = 0; it < kExactMaxIter; ++it) {
    wave_relation(ps, s[0], gamma, fL, dfL);
    wave_relation(ps, s[1], gamma, fR, dfR);
    T pn = ps - (fL + fR + du) * rcp(dfL + dfR);
    if (!(pn > T(0))) pn = T(0.5) * ps;
    const T step = pn - ps;
    ps = pn;
    if (fabs(step) <= tol * (pn + pn - step)) {
      fL += dfL * step;
      fR += dfR * step;
      conv = true;
      break;
    }
  }
  if (!conv) {
    wave_relation(ps, s[0], gamma, fL, dfL);
    wave_relation(ps, s[1], gamma, fR, dfR);
  }
  const T us = T(0.5) * (s[0].u + s[1].u) + T(0.5) * (fR - fL);
  // The side of the contact the face lies on; the right side is mirrored
  // (velocities negated) onto the left-side formulas.
  const bool left = us >= T(0);
  const T sg = left ? T(1) : T(-1);
  const ESide<T> a = left ? s[0] : s[1];
  const T fa = left ? fL : fR;
  const T ua = sg * a.u, usa = sg * us, vt = left ? ut[0] : ut[1];
  T rho, u, pr;
  if (ps > a.p) {
    const T pr_ratio = ps * rcp(a.p);
    const T S = ua - a.c * sqrt_pos((gamma + T(1)) * rcp(T(2) * gamma) * pr_ratio + z);
    const T g6 = gm1 * rcp(gamma + T(1));
    if (S >= T(0)) {
      rho = a.r;
      u = ua;
      pr = a.p;
    } else {
      rho = a.r * (pr_ratio + g6) * rcp(g6 * pr_ratio + T(1));
      u = usa;
      pr = ps;
    }
  } else {
    const T cs = a.c + T(0.5) * gm1 * fa;
    const T head = ua - a.c;
    const T tail = usa - cs;
    if (head >= T(0)) {
      rho = a.r;
      u = ua;
      pr = a.p;
    } else if (tail < T(0)) {
      rho = gamma * ps * rcp(cs * cs);
      u = usa;
      pr = ps;
    } else {  // inside the rarefaction fan, where u = c
      const T cf = T(2) * rcp(gamma + T(1)) * (a.c + T(0.5) * gm1 * ua);
      u = cf;
      rho = a.r * pow_pos(cf * rcp(a.c), T(2) * rcp(gm1));
      pr = rho * cf * cf * rcp(gamma);
    }
  }
  u = sg * u;
  const T E = pr * rcp(gm1) + T(0.5) * rho * (u * u + vt * vt);
  F[0] = rho * u;
  F[1 + AX] = rho * u * u + pr;
  F[1 + TX] = rho * u * vt;
  F[3] = (E + pr) * u;
}

}  // namespace dg
