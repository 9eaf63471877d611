// Fused DG stage for 2D Euler on a periodic Cartesian mesh (gfx950, wave64).
//
// What one launch computes (Sec. 2.2, eqn:fv and eqn:dgderiv; limiter of
// Sec. 2.5; HLL face flux): for every cell, limit the P1 coefficients on read,
// evaluate both neighbours at the two Gauss points of each face, solve the
// Riemann problem, accumulate the surface terms of the mean and gradient
// equations, add the 2x2 Gauss volume term of F . grad(x_d), apply the inverse
// mass matrix diag(1/V, 12/(V hx^2), 12/(V hy^2)) and combine into an SSP-RK2
// stage.
//
// Work decomposition.  One wave (64 lanes) owns a tile of 60 columns and
// `rows_per_tile` rows.  Lane l holds column x0 + l - 2: lanes 0,1 and 62,63
// are halo columns whose results are discarded.  The wave marches up its rows
// keeping a two-row register window, so every coefficient is read from HBM
// once per tile (plus two halo rows).  x-neighbours come from lane shuffles,
// y-neighbours from the window: no LDS, no barriers, no atomics.  Each face is
// solved once: a lane solves its -x face and hands the flux to the lane on its
// left; the y-face between the window rows is solved by the lane of that
// column.
//
// MUSCL-Hancock mode (Sec. 2.4): the same faces and volume points, with every
// state taken from the cell's half-step primitive prediction (centroid
// primitive values and gradients from the limited conserved coefficients,
// advanced dt/2 with the quasi-linear Euler time derivatives, extrapolated
// linearly, converted back to conserved variables); one pass per step.
//
// Per-cell algebra (weights and the inverse mass matrix folded together).
// With S = F(g0) + F(g1) and D = F(g1) - F(g0) for the two Gauss points of a
// face (g0 at the lower tangential offset), and sum_q F_d(q) the volume
// flux sum over the four 2x2 Gauss points:
//   d mean/dt = (Sx- - Sx+)/(2 hx) + (Sy- - Sy+)/(2 hy)
//   d gx /dt  = 3 (sum_q Fx(q) - Sx- - Sx+)/hx^2 + sqrt(3) (Dy- - Dy+)/(hx hy)
//   d gy /dt  = 3 (sum_q Fy(q) - Sy- - Sy+)/hy^2 + sqrt(3) (Dx- - Dx+)/(hx hy)
#include <hip/hip_runtime.h>

#include <mutex>

#include "dg_internal.h"
#include "dg_math.h"
#include "euler_exact.h"

namespace dg {
namespace {

constexpr int kLanes = 64;
constexpr int kCols = 60;  // interior columns per wave

template <typename T>
struct P2 {
  const T* __restrict__ in;
  const T* __restrict__ u0;
  T* __restrict__ out;
  const double* dt_dev;
  double dt_host;
  int* status;
  double* dtpart;       // per-wave CFL minima (stage 2 with dt_next)
  double* dt_next;
  double cfl;
  int nx, ny, rows, tiles_x, ntiles, nc;
  T gamma, igm1;              // gamma, 1/(gamma - 1)
  T cmx, cmy, cgx, cgy, ccr;  // 1/(2hx), 1/(2hy), 3/hx^2, 3/hy^2, sqrt3/(hx hy)
  T hx2, hy2, qx, qy;         // hx/2, hy/2, hx/(2 sqrt3), hy/(2 sqrt3)
  double ihx, ihy;            // 1/hx, 1/hy
};

// One cell: 4 variables x (mean, gx, gy).
template <typename T>
struct Cell {
  T m[4], gx[4], gy[4];
};

// Coefficient arrays are addressed as (uniform array base, 32-bit byte offset
// of the cell): the base k*nc is scalar, so each load or store is one memory
// instruction with a scalar base and the row's vector offset, and no per-array
// 64-bit address arithmetic in the vector unit.
template <typename T>
__device__ __forceinline__ const T& at(const T* __restrict__ U, int nc, int k, unsigned off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(U + (size_t)k * nc) + off);
}
template <typename T>
__device__ __forceinline__ T& at(T* __restrict__ U, int nc, int k, unsigned off) {
  return *reinterpret_cast<T*>(reinterpret_cast<char*>(U + (size_t)k * nc) + off);
}

template <typename T>
__device__ __forceinline__ void load_cell(const T* __restrict__ U, int nc, int e, Cell<T>& c) {
  const unsigned off = (unsigned)e * sizeof(T);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    c.m[v] = at(U, nc, 3 * v, off);
    c.gx[v] = at(U, nc, 3 * v + 1, off);
    c.gy[v] = at(U, nc, 3 * v + 2, off);
  }
}

template <typename T>
__device__ __forceinline__ void load_means(const T* __restrict__ U, int nc, int e, T* m) {
  const unsigned off = (unsigned)e * sizeof(T);
#pragma unroll
  for (int v = 0; v < 4; ++v) m[v] = at(U, nc, 3 * v, off);
}

template <typename T>
__device__ __forceinline__ void store_cell(T* __restrict__ U, int nc, int e, const Cell<T>& c) {
  const unsigned off = (unsigned)e * sizeof(T);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    at(U, nc, 3 * v, off) = c.m[v];
    at(U, nc, 3 * v + 1, off) = c.gx[v];
    at(U, nc, 3 * v + 2, off) = c.gy[v];
  }
}

// Limiter of one cell from its x-neighbour means (lane exchange) and y-neighbour
// means.  On a Cartesian cell the +d and -d face centroids sit at -+ h_d/2,
// so the two psi of an axis reduce to min(max-phi, phi-min)/|g_d h_d/2| and
// alpha = min(1, D / max_d |g_d h_d / 2|).
template <typename T>
__device__ __forceinline__ void limit_cell(Cell<T>& c, const T* mS, const T* mN, const P2<T>& p) {
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    T mW = lane_up(c.m[v]);
    T mE = lane_down(c.m[v]);
    T phi = c.m[v];
    T hi = fmax(fmax(fmax(phi, mW), fmax(mE, mS[v])), mN[v]);
    T lo = fmin(fmin(fmin(phi, mW), fmin(mE, mS[v])), mN[v]);
    T D = fmin(hi - phi, phi - lo);
    T dm = fmax(fabs(c.gx[v]) * p.hx2, fabs(c.gy[v]) * p.hy2);
    T a = (dm > D) ? div_small(D, dm) : T(1);
    c.gx[v] *= a;
    c.gy[v] *= a;
  }
}

// Primitive (rho, v_x, v_y, p) of a cell's conserved means.
template <typename T>
__device__ __forceinline__ void prim_of(const T* m, T gm1, T* w) {
  const T ir = rcp(m[0]);
  w[0] = m[0];
  w[1] = m[1] * ir;
  w[2] = m[2] * ir;
  w[3] = gm1 * (m[3] - T(0.5) * (m[1] * w[1] + m[2] * w[2]));
}

// The WENO-type limiter of Sec. 2.5 on one cell.  Per primitive variable two
// candidate slopes: the stencil slope (on a box the least-squares fit to the
// four face neighbours' primitive means is the central difference), limited
// as in limit_cell; and the cell's unlimited DG slope (chain rule at the
// centroid).  Each gets the oscillation factor
//   o = sum over the four faces of |dphi| + |phi_nb - (phi + dphi)|,
// dphi = slope . (edge midpoint - centroid); the slopes are averaged with
// weights (eps + o)^(-1/2), eps the working precision's machine epsilon, and
// the conserved gradients are recomputed from the primitive ones.
template <typename T>
__device__ __forceinline__ void limit_cell_weno(Cell<T>& c, const T* mS, const T* mN,
                                                const P2<T>& p) {
  const T gm1 = p.gamma - T(1);
  const T eps = sizeof(T) == 8 ? T(2.220446049250313e-16) : T(1.1920929e-7);
  T mW[4], mE[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    mW[v] = lane_up(c.m[v]);
    mE[v] = lane_down(c.m[v]);
  }
  T wi[4], wW[4], wE[4], wS[4], wN[4];
  prim_of(c.m, gm1, wi);
  prim_of(mW, gm1, wW);
  prim_of(mE, gm1, wE);
  prim_of(mS, gm1, wS);
  prim_of(mN, gm1, wN);
  const T rho = wi[0], ir = rcp(rho), vx = wi[1], vy = wi[2];
  const T v2 = vx * vx + vy * vy;
  // DG primitive slopes
  T dx[4], dy[4];
  dx[0] = c.gx[0];
  dy[0] = c.gy[0];
  dx[1] = (c.gx[1] - vx * dx[0]) * ir;
  dy[1] = (c.gy[1] - vx * dy[0]) * ir;
  dx[2] = (c.gx[2] - vy * dx[0]) * ir;
  dy[2] = (c.gy[2] - vy * dy[0]) * ir;
  dx[3] = gm1 * (c.gx[3] - T(0.5) * v2 * dx[0] - rho * (vx * dx[1] + vy * dx[2]));
  dy[3] = gm1 * (c.gy[3] - T(0.5) * v2 * dy[0] - rho * (vx * dy[1] + vy * dy[2]));
  T nx_[4], ny_[4];
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    // stencil slope, limited
    T sx = (wE[k] - wW[k]) * p.cmx;
    T sy = (wN[k] - wS[k]) * p.cmy;
    const T hi = fmax(fmax(fmax(wi[k], wW[k]), fmax(wE[k], wS[k])), wN[k]);
    const T lo = fmin(fmin(fmin(wi[k], wW[k]), fmin(wE[k], wS[k])), wN[k]);
    // D >= 0 by definition; the clamp absorbs the rounding of a primitive
    // value that the compiler fuses into hi - w (w = m * (1/rho) is a product),
    // which could otherwise make D slightly negative and D/dm infinite
    const T D = fmax(fmin(hi - wi[k], wi[k] - lo), T(0));
    const T dm = fmax(fabs(sx) * p.hx2, fabs(sy) * p.hy2);
    const T a = (dm > D) ? div_small(D, dm) : T(1);
    sx *= a;
    sy *= a;
    // oscillation factors
    auto osc = [&](T gx, T gy) {
      const T ex = gx * p.hx2, ey = gy * p.hy2;
      return T(2) * (fabs(ex) + fabs(ey)) + fabs(wE[k] - (wi[k] + ex)) +
             fabs(wW[k] - (wi[k] - ex)) + fabs(wN[k] - (wi[k] + ey)) + fabs(wS[k] - (wi[k] - ey));
    };
    const T ws = rcp(sqrt_pos(eps + osc(sx, sy)));
    const T wd = rcp(sqrt_pos(eps + osc(dx[k], dy[k])));
    const T iw = rcp(ws + wd);
    nx_[k] = (ws * sx + wd * dx[k]) * iw;
    ny_[k] = (ws * sy + wd * dy[k]) * iw;
  }
  // conserved gradients from the primitive ones at the centroid
  c.gx[0] = nx_[0];
  c.gy[0] = ny_[0];
  c.gx[1] = vx * nx_[0] + rho * nx_[1];
  c.gy[1] = vx * ny_[0] + rho * ny_[1];
  c.gx[2] = vy * nx_[0] + rho * nx_[2];
  c.gy[2] = vy * ny_[0] + rho * ny_[2];
  const T igm1 = rcp(gm1);
  c.gx[3] = nx_[3] * igm1 + T(0.5) * v2 * nx_[0] + rho * (vx * nx_[1] + vy * nx_[2]);
  c.gy[3] = ny_[3] * igm1 + T(0.5) * v2 * ny_[0] + rho * (vx * ny_[1] + vy * ny_[2]);
}

// The limiter selected by LIM: 1 the Arepo limiter, 2 the WENO-type limiter.
template <typename T, int LIM>
__device__ __forceinline__ void limit_any(Cell<T>& c, const T* mS, const T* mN, const P2<T>& p) {
  if (LIM == 2)
    limit_cell_weno(c, mS, mN, p);
  else
    limit_cell(c, mS, mN, p);
}

// HLL flux (Davis wave speeds) along axis AX between states uL, uR, written
// as F = a F_L + b F_R + c (u_R - u_L) with (a, b, c) = (1, 0, 0) left of the
// fan, (0, 1, 0) right of it and (S_R, -S_L, S_L S_R)/(S_R - S_L) inside.
template <typename T, int AX>
__device__ __forceinline__ void hll(const T* uL, const T* uR, T gamma, T* F, bool& bad) {
  const T gm1 = gamma - T(1);
  T irL = rcp(uL[0]), irR = rcp(uR[0]);
  T vxL = uL[1] * irL, vyL = uL[2] * irL;
  T vxR = uR[1] * irR, vyR = uR[2] * irR;
  T pL = gm1 * (uL[3] - T(0.5) * (uL[1] * vxL + uL[2] * vyL));
  T pR = gm1 * (uR[3] - T(0.5) * (uR[1] * vxR + uR[2] * vyR));
  bad |= !(uL[0] > T(0)) || !(uR[0] > T(0)) || !(pL > T(0)) || !(pR > T(0));
  T cL = sqrt_pos(gamma * pL * irL), cR = sqrt_pos(gamma * pR * irR);
  T vnL = AX == 0 ? vxL : vyL;
  T vnR = AX == 0 ? vxR : vyR;
  T SL = fmin(vnL - cL, vnR - cR);
  T SR = fmax(vnL + cL, vnR + cR);
  T FL[4] = {uL[0] * vnL, uL[1] * vnL, uL[2] * vnL, (uL[3] + pL) * vnL};
  T FR[4] = {uR[0] * vnR, uR[1] * vnR, uR[2] * vnR, (uR[3] + pR) * vnR};
  FL[1 + AX] += pL;
  FR[1 + AX] += pR;
  T inv = rcp(SR - SL);
  T a = SR * inv, b = -SL * inv, c = SL * SR * inv;
  const bool left = SL >= T(0), right = SR <= T(0);
  a = left ? T(1) : (right ? T(0) : a);
  b = left ? T(0) : (right ? T(1) : b);
  c = (left || right) ? T(0) : c;
#pragma unroll
  for (int k = 0; k < 4; ++k) F[k] = fma(a, FL[k], fma(b, FR[k], c * (uR[k] - uL[k])));
}

// Face flux along axis AX: HLL (RS = 0) or the exact Riemann solver (RS = 1).
template <typename T, int AX, int RS>
__device__ __forceinline__ void riemann(const T* uL, const T* uR, T gamma, T* F, bool& bad) {
  if (RS == 1)
    exact_flux<T, AX>(uL, uR, gamma, F, bad);
  else
    hll<T, AX>(uL, uR, gamma, F, bad);
}

// Both Cartesian flux rows F_x, F_y at one state (volume term).
template <typename T>
__device__ __forceinline__ void flux_xy(const T* u, T gamma, T* Fx, T* Fy, bool& bad) {
  T ir = rcp(u[0]);
  T vx = u[1] * ir, vy = u[2] * ir;
  T p = (gamma - T(1)) * (u[3] - T(0.5) * (u[1] * vx + u[2] * vy));
  bad |= !(u[0] > T(0)) || !(p > T(0));
  Fx[0] = u[1];
  Fx[1] = u[1] * vx + p;
  Fx[2] = u[2] * vx;
  Fx[3] = (u[3] + p) * vx;
  Fy[0] = u[2];
  Fy[1] = u[1] * vy;
  Fy[2] = u[2] * vy + p;
  Fy[3] = (u[3] + p) * vy;
}

// Half-step primitive prediction of a limited cell: the returned Cell holds
// primitive values (rho, v_x, v_y, p) at the centroid advanced by h = dt/2 in
// m and the primitive gradients in gx, gy.
template <typename T>
__device__ __forceinline__ Cell<T> predict(const Cell<T>& c, T gamma, T h) {
  const T gm1 = gamma - T(1);
  const T rho = c.m[0], ir = rcp(rho);
  const T vx = c.m[1] * ir, vy = c.m[2] * ir;
  const T v2 = vx * vx + vy * vy;
  const T p = gm1 * (c.m[3] - T(0.5) * rho * v2);
  Cell<T> w;
  w.gx[0] = c.gx[0];
  w.gy[0] = c.gy[0];
  w.gx[1] = (c.gx[1] - vx * c.gx[0]) * ir;
  w.gy[1] = (c.gy[1] - vx * c.gy[0]) * ir;
  w.gx[2] = (c.gx[2] - vy * c.gx[0]) * ir;
  w.gy[2] = (c.gy[2] - vy * c.gy[0]) * ir;
  // E = p/(gamma-1) + rho |v|^2/2
  w.gx[3] = gm1 * (c.gx[3] - T(0.5) * v2 * c.gx[0] - rho * (vx * w.gx[1] + vy * w.gx[2]));
  w.gy[3] = gm1 * (c.gy[3] - T(0.5) * v2 * c.gy[0] - rho * (vx * w.gy[1] + vy * w.gy[2]));
  const T div = w.gx[1] + w.gy[2];
  const T rho_t = -(vx * w.gx[0] + vy * w.gy[0] + rho * div);
  const T vx_t = -(vx * w.gx[1] + vy * w.gy[1] + w.gx[3] * ir);
  const T vy_t = -(vx * w.gx[2] + vy * w.gy[2] + w.gy[3] * ir);
  const T p_t = -(gamma * p * div + vx * w.gx[3] + vy * w.gy[3]);
  w.m[0] = fma(h, rho_t, rho);
  w.m[1] = fma(h, vx_t, vx);
  w.m[2] = fma(h, vy_t, vy);
  w.m[3] = fma(h, p_t, p);
  return w;
}

// Conserved variables of a primitive state (in place).
template <typename T>
__device__ __forceinline__ void to_cons(T* u, T igm1) {
  const T rho = u[0], vx = u[1], vy = u[2];
  u[1] = rho * vx;
  u[2] = rho * vy;
  u[3] = fma(u[3], igm1, T(0.5) * rho * (vx * vx + vy * vy));
}

// x-face between the left neighbour L (lane - 1) and this cell R.  Returns
// S = F(g0) + F(g1), D = F(g1) - F(g0) per variable (g0 at y offset -qy).
template <typename T, bool PRIM = false, int RS = 0>
__device__ __forceinline__ void xface(const Cell<T>& L, const Cell<T>& R, const P2<T>& p, T* S,
                                      T* D, bool& bad) {
  T bl[4], br[4], tl[4], tr[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    bl[v] = fma(L.gx[v], p.hx2, L.m[v]);
    br[v] = fma(-R.gx[v], p.hx2, R.m[v]);
    tl[v] = L.gy[v] * p.qy;
    tr[v] = R.gy[v] * p.qy;
  }
  T uL[4], uR[4], F0[4], F1[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    uL[v] = bl[v] - tl[v];
    uR[v] = br[v] - tr[v];
  }
  if (PRIM) {
    to_cons(uL, p.igm1);
    to_cons(uR, p.igm1);
  }
  riemann<T, 0, RS>(uL, uR, p.gamma, F0, bad);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    uL[v] = bl[v] + tl[v];
    uR[v] = br[v] + tr[v];
  }
  if (PRIM) {
    to_cons(uL, p.igm1);
    to_cons(uR, p.igm1);
  }
  riemann<T, 0, RS>(uL, uR, p.gamma, F1, bad);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    S[v] = F0[v] + F1[v];
    D[v] = F1[v] - F0[v];
  }
}

// y-face between the lower cell L (previous row) and the upper cell R.
template <typename T, bool PRIM = false, int RS = 0>
__device__ __forceinline__ void yface(const Cell<T>& L, const Cell<T>& R, const P2<T>& p, T* S,
                                      T* D, bool& bad) {
  T bl[4], br[4], tl[4], tr[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    bl[v] = fma(L.gy[v], p.hy2, L.m[v]);
    br[v] = fma(-R.gy[v], p.hy2, R.m[v]);
    tl[v] = L.gx[v] * p.qx;
    tr[v] = R.gx[v] * p.qx;
  }
  T uL[4], uR[4], F0[4], F1[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    uL[v] = bl[v] - tl[v];
    uR[v] = br[v] - tr[v];
  }
  if (PRIM) {
    to_cons(uL, p.igm1);
    to_cons(uR, p.igm1);
  }
  riemann<T, 1, RS>(uL, uR, p.gamma, F0, bad);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    uL[v] = bl[v] + tl[v];
    uR[v] = br[v] + tr[v];
  }
  if (PRIM) {
    to_cons(uL, p.igm1);
    to_cons(uR, p.igm1);
  }
  riemann<T, 1, RS>(uL, uR, p.gamma, F1, bad);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    S[v] = F0[v] + F1[v];
    D[v] = F1[v] - F0[v];
  }
}

// Volume term: sums of F_x and F_y over the 2x2 Gauss points.
template <typename T, bool PRIM = false>
__device__ __forceinline__ void volume(const Cell<T>& c, const P2<T>& p, T* sx, T* sy,
                                       bool& bad) {
#pragma unroll
  for (int v = 0; v < 4; ++v) sx[v] = sy[v] = T(0);
#pragma unroll
  for (int q = 0; q < 4; ++q) {
    const T ox = (q & 2) ? p.qx : -p.qx;
    const T oy = (q & 1) ? p.qy : -p.qy;
    T u[4], Fx[4], Fy[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) u[v] = fma(c.gx[v], ox, fma(c.gy[v], oy, c.m[v]));
    if (PRIM) to_cons(u, p.igm1);
    flux_xy(u, p.gamma, Fx, Fy, bad);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      sx[v] += Fx[v];
      sy[v] += Fy[v];
    }
  }
}

// CFL bound of one cell from its means: 1 / sum_d (|v_d| + c)/h_d.
template <typename T>
__device__ __forceinline__ double cell_dt(const T* m, const P2<T>& p) {
  double r = m[0], ir = 1.0 / r;
  double vx = m[1] * ir, vy = m[2] * ir;
  double pr = ((double)p.gamma - 1.0) * (m[3] - 0.5 * r * (vx * vx + vy * vy));
  double c = sqrt((double)p.gamma * pr * ir);
  double s = (fabs(vx) + c) * p.ihx + (fabs(vy) + c) * p.ihy;
  return 1.0 / s;
}

// One wave's tile (tile index `wave` of the mesh described by p).  RS selects
// the face flux (0 HLL, 1 exact Riemann solver).
template <typename T, int MODE, int LIM, int RS = 0>
__device__ __forceinline__ void cart2d_tile(const P2<T>& p, int wave, int lane) {
  const int tx = wave % p.tiles_x, ty = wave / p.tiles_x;
  const int colu = tx * kCols + lane - 2;
  const bool own = lane >= 2 && lane < 2 + kCols && colu < p.nx;
  int col = colu % p.nx;
  if (col < 0) col += p.nx;
  const int nx = p.nx, ny = p.ny, nc = p.nc;
  const int y0 = ty * p.rows;
  const int y1 = min(y0 + p.rows, ny);
  auto wrap = [ny](int r) {
    r %= ny;
    return r < 0 ? r + ny : r;
  };
  auto next = [ny](int r) { return r + 1 == ny ? 0 : r + 1; };
  bool bad = false;
  double dtmin = 1e300;

  // Row window of the input: prev = row j-1 (limited; only its means before
  // the first iteration), cur = row j, nx1 = row j+1, nx2 = row j+2 (loads in
  // flight while row j is processed).
  Cell<T> prev, cur, nx1;
  load_means(p.in, nc, wrap(y0 - 2) * nx + col, prev.m);
  int r = wrap(y0 - 1);
  load_cell(p.in, nc, r * nx + col, cur);
  r = next(r);
  load_cell(p.in, nc, r * nx + col, nx1);
  int r2 = next(r);  // row index of j+2

  // Stage 2: window over u0 for the row being finalised (f = j-1):
  // u0m = means of f-1, u0c = row f, u0n = row f+1 (means only beyond y1-1).
  T u0m[4];
  Cell<T> u0c, u0n;
  int ru = 0;
  if (MODE == kStage2) {
    load_means(p.u0, nc, wrap(y0 - 1) * nx + col, u0m);
    ru = wrap(y0);
    load_cell(p.u0, nc, ru * nx + col, u0c);
    ru = next(ru);
    if (y0 + 1 <= y1 - 1)
      load_cell(p.u0, nc, ru * nx + col, u0n);
    else
      load_means(p.u0, nc, ru * nx + col, u0n.m);
    ru = next(ru);  // row f+2 for the first finalised row
  }
  T ySm[4], yDm[4];
  // the step size is first needed when row y0 is finalised
  T dt = T(0);
  if (MODE == kStage1 || MODE == kStage2 || MODE == kMH)
    dt = (T)(p.dt_dev ? *p.dt_dev : p.dt_host);
  // MUSCL-Hancock: predicted primitive cells of the window rows j-1 and j
  Cell<T> prevP, curP;

  for (int j = y0 - 1; j <= y1; ++j) {
    Cell<T> nx2;
    if (j + 2 <= y1)
      load_cell(p.in, nc, r2 * nx + col, nx2);
    else if (j + 2 == y1 + 1)
      load_means(p.in, nc, r2 * nx + col, nx2.m);
    r2 = next(r2);

    if (LIM != 0 || MODE == kLimit) limit_any<T, (LIM == 2 ? 2 : 1)>(cur, prev.m, nx1.m, p);
    if (MODE == kMH) curP = predict(cur, p.gamma, T(0.5) * dt);

    if (MODE == kLimit) {
      if (own && j >= y0 && j < y1) store_cell(p.out, nc, wrap(j) * nx + col, cur);
    } else {
      T Sy[4], Dy[4];
      if (j >= y0) {
        if (MODE == kMH)
          yface<T, true, RS>(prevP, curP, p, Sy, Dy, bad);
        else
          yface<T, false, RS>(prev, cur, p, Sy, Dy, bad);
      }
      if (j >= y0 + 1) {
        // Finalise row f = j - 1 (held in prev).
        Cell<T> u0nn;
        if (MODE == kStage2) {
          if (j + 1 <= y1 - 1)
            load_cell(p.u0, nc, ru * nx + col, u0nn);
          else if (j + 1 == y1)
            load_means(p.u0, nc, ru * nx + col, u0nn.m);
          ru = next(ru);
        }
        const Cell<T>& ev = MODE == kMH ? prevP : prev;  // the row's evaluated polynomial
        Cell<T> left;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          left.m[v] = lane_up(ev.m[v]);
          left.gx[v] = lane_up(ev.gx[v]);
          left.gy[v] = lane_up(ev.gy[v]);
        }
        T Sm[4], Dm[4], sx[4], sy[4];
        xface<T, MODE == kMH, RS>(left, ev, p, Sm, Dm, bad);
        volume<T, MODE == kMH>(ev, p, sx, sy, bad);
        Cell<T> o;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          T Sp = lane_down(Sm[v]);
          T Dp = lane_down(Dm[v]);
          T dm = (Sm[v] - Sp) * p.cmx + (ySm[v] - Sy[v]) * p.cmy;
          T dgx = (sx[v] - Sm[v] - Sp) * p.cgx + (yDm[v] - Dy[v]) * p.ccr;
          T dgy = (sy[v] - ySm[v] - Sy[v]) * p.cgy + (Dm[v] - Dp) * p.ccr;
          if (MODE == kRhs) {
            o.m[v] = dm;
            o.gx[v] = dgx;
            o.gy[v] = dgy;
          } else {
            o.m[v] = fma(dt, dm, prev.m[v]);
            o.gx[v] = fma(dt, dgx, prev.gx[v]);
            o.gy[v] = fma(dt, dgy, prev.gy[v]);
          }
        }
        if (MODE == kStage2) {
          Cell<T> ua = u0c;
          if (LIM != 0) limit_any<T, LIM>(ua, u0m, u0n.m, p);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            o.m[v] = T(0.5) * (ua.m[v] + o.m[v]);
            o.gx[v] = T(0.5) * (ua.gx[v] + o.gx[v]);
            o.gy[v] = T(0.5) * (ua.gy[v] + o.gy[v]);
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) u0m[v] = u0c.m[v];
          u0c = u0n;
          u0n = u0nn;
        }
        if (own) {
          store_cell(p.out, nc, wrap(j - 1) * nx + col, o);
          if ((MODE == kStage2 || MODE == kMH) && p.dt_next) dtmin = fmin(dtmin, cell_dt(o.m, p));
        }
      }
      if (j >= y0) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          ySm[v] = Sy[v];
          yDm[v] = Dy[v];
        }
      }
    }
    prev = cur;
    cur = nx1;
    nx1 = nx2;
    if (MODE == kMH) prevP = curP;
  }
  if (bad && own) atomicOr(p.status, 1);
  if ((MODE == kStage2 || MODE == kMH) && p.dt_next) {
    // per-wave CFL minimum; a one-workgroup kernel reduces them afterwards
    dtmin = wave_min(dtmin);
    if (lane == 0) p.dtpart[wave] = dtmin;
  }
}

template <typename T, int MODE, int LIM, int RS = 0>
__global__ __launch_bounds__(256) void k_cart2d(P2<T> p) {
  const int lane = threadIdx.x & (kLanes - 1);
  const int wave = xcd_remap(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
  if (wave >= p.ntiles) return;
  cart2d_tile<T, MODE, LIM, RS>(p, wave, lane);
}

// The same tile with the register budget of two waves per SIMD.  Used for
// stage 1 with the exact Riemann solver in FP64, where the second wave hides
// the latency of the divergent Newton loops and pays for the ~160 B per lane
// the cap spills (0.99 -> 0.88 ms at 2048^2); the other stage kernels spill
// far more under the cap (stage 2: 350-770 B) and run one wave per SIMD.
template <typename T, int MODE, int LIM, int RS = 0>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8)))
void k_cart2d_w2(P2<T> p) {
  const int lane = threadIdx.x & (kLanes - 1);
  const int wave = xcd_remap(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
  if (wave >= p.ntiles) return;
  cart2d_tile<T, MODE, LIM, RS>(p, wave, lane);
}

// ------------------------------------------------------------- fused step --
// Both SSP-RK2 stages of a step (Sec. 2.2 with the limiter of Sec. 2.5 at the
// start of each stage) in one pass.  A wave marches the rows of its strip
// twice over, the second march trailing the first: the stage-1 march turns
// the U^n window into V1 = Pi(U) + dt L(Pi(U)) one row at a time, and each V1
// row goes straight (in registers) into the window of the stage-2 march, which
// finalises U^{n+1} = (Pi(U) + Pi(V1) + dt L(Pi(V1)))/2 two rows behind.  The
// limited U^n rows wait for that combination in a per-wave LDS ring of three
// rows.  HBM traffic per step is one read of U^n and one write of U^{n+1} (24
// values per cell instead of 60 for the two stage launches); the price is a
// halo of two lanes on each side per stage (56 output columns per 64-lane
// wave) and four extra stage-1 rows per strip.  Results equal the two stage
// launches: the same row arithmetic, in the same order.

// Time derivative (Sec. 2.2) of the row a wave finalises, from the row's
// limited polynomial ev: its -x face (left neighbour by lane exchange) and +x
// face (the -x face of lane+1), the volume term, and the sums and differences
// of the fluxes at the Gauss points of the y-face below (ySm, yDm) and above
// (Sy, Dy), through the folded inverse mass matrix.  The row update of
// cart2d_tile, written out again so the tuned stage kernels keep their code.
template <typename T>
__device__ __forceinline__ void row_rates(const Cell<T>& ev, const T* ySm, const T* yDm,
                                          const T* Sy, const T* Dy, const P2<T>& p, bool& bad,
                                          Cell<T>& d) {
  Cell<T> left;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    left.m[v] = lane_up(ev.m[v]);
    left.gx[v] = lane_up(ev.gx[v]);
    left.gy[v] = lane_up(ev.gy[v]);
  }
  T Sm[4], Dm[4], sx[4], sy[4];
  xface<T>(left, ev, p, Sm, Dm, bad);
  volume<T>(ev, p, sx, sy, bad);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    T Sp = lane_down(Sm[v]);
    T Dp = lane_down(Dm[v]);
    d.m[v] = (Sm[v] - Sp) * p.cmx + (ySm[v] - Sy[v]) * p.cmy;
    d.gx[v] = (sx[v] - Sm[v] - Sp) * p.cgx + (yDm[v] - Dy[v]) * p.ccr;
    d.gy[v] = (sy[v] - ySm[v] - Sy[v]) * p.cgy + (Dm[v] - Dp) * p.ccr;
  }
}

constexpr int kStepCols = 56;
constexpr int kStepRing = 3;

template <typename T, int LIM>
__device__ __forceinline__ void cart2d_step_tile(const P2<T>& p, int wave, int lane,
                                                 T (*ring)[12][kLanes]) {
  const int tx = wave % p.tiles_x, ty = wave / p.tiles_x;
  const int colu = tx * kStepCols + lane - 4;
  // stage 1 is exact on lanes 2..61 (its limiter needs lane -+1, its faces the
  // limited lane -+1), stage 2 on lanes 4..59
  const bool liveA = lane >= 2 && lane < 62;
  const bool liveB = lane >= 4 && lane < 4 + kStepCols;
  const bool own = liveB && colu < p.nx;
  int col = colu % p.nx;
  if (col < 0) col += p.nx;
  const int nx = p.nx, ny = p.ny, nc = p.nc;
  const int y0 = ty * p.rows;
  const int y1 = min(y0 + p.rows, ny);
  // stage 2 outputs rows [y0, y1) and reads V1 rows [y0 - 2, y1 + 2), which
  // stage 1 computes from U^n rows [y0 - 4, y1 + 4)
  const int a0 = y0 - 2, a1 = y1 + 2;
  auto wrap = [ny](int r) {
    r %= ny;
    return r < 0 ? r + ny : r;
  };
  auto next = [ny](int r) { return r + 1 == ny ? 0 : r + 1; };
  bool badA = false, badB = false;
  double dtmin = 1e300;
  const T dt = (T)(p.dt_dev ? *p.dt_dev : p.dt_host);

  // stage-1 window over U^n: prev = row j-1 (limited), cur = row j, nx1 = j+1
  Cell<T> prev, cur, nx1;
  load_means(p.in, nc, wrap(a0 - 2) * nx + col, prev.m);
  int r = wrap(a0 - 1);
  load_cell(p.in, nc, r * nx + col, cur);
  r = next(r);
  load_cell(p.in, nc, r * nx + col, nx1);
  int r2 = next(r);
  T ySm[4], yDm[4];
  // stage-2 window over V1: pB = row f-2 (limited), cB = row f-1, nB = row f
  Cell<T> pB, cB, nB;
  T ySmB[4], yDmB[4];

  for (int j = a0 - 1; j <= a1; ++j) {
    Cell<T> nx2;
    if (j + 2 <= a1)
      load_cell(p.in, nc, r2 * nx + col, nx2);
    else if (j + 2 == a1 + 1)
      load_means(p.in, nc, r2 * nx + col, nx2.m);
    r2 = next(r2);

    if (LIM != 0) limit_any<T, 1>(cur, prev.m, nx1.m, p);
    T Sy[4], Dy[4];
    if (j >= a0) yface<T>(prev, cur, p, Sy, Dy, badA);
    if (j >= a0 + 1) {
      // stage 1 of row f = j - 1
      const int f = j - 1;
      Cell<T> o;
      row_rates<T>(prev, ySm, yDm, Sy, Dy, p, badA, o);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        o.m[v] = fma(dt, o.m[v], prev.m[v]);
        o.gx[v] = fma(dt, o.gx[v], prev.gx[v]);
        o.gy[v] = fma(dt, o.gy[v], prev.gy[v]);
      }
      // stage 2 takes V1 row f
      pB = cB;
      cB = nB;
      nB = o;
      if (LIM != 0 && f >= y0) limit_any<T, 1>(cB, pB.m, nB.m, p);
      T SyB[4], DyB[4];
      if (f - 1 >= y0) yface<T>(pB, cB, p, SyB, DyB, badB);
      if (f - 2 >= y0) {
        // finalise row g = f - 2 (held in pB); Pi(U^n) of row g from the ring
        const int g = f - 2;
        Cell<T> o2;
        row_rates<T>(pB, ySmB, yDmB, SyB, DyB, p, badB, o2);
        const int slot = (g - y0) % kStepRing;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          o2.m[v] = T(0.5) * (ring[slot][3 * v][lane] + fma(dt, o2.m[v], pB.m[v]));
          o2.gx[v] = T(0.5) * (ring[slot][3 * v + 1][lane] + fma(dt, o2.gx[v], pB.gx[v]));
          o2.gy[v] = T(0.5) * (ring[slot][3 * v + 2][lane] + fma(dt, o2.gy[v], pB.gy[v]));
        }
        if (own) {
          store_cell(p.out, nc, wrap(g) * nx + col, o2);
          if (p.dt_next) dtmin = fmin(dtmin, cell_dt(o2.m, p));
        }
      }
      if (f - 1 >= y0) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          ySmB[v] = SyB[v];
          yDmB[v] = DyB[v];
        }
      }
    }
    // Pi(U^n) of row j for the combination three rows later (its slot held
    // row j - 3, which stage 2 read above; LDS operations of a wave run in
    // order)
    if (j >= y0 && j < y1) {
      const int slot = (j - y0) % kStepRing;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        ring[slot][3 * v][lane] = cur.m[v];
        ring[slot][3 * v + 1][lane] = cur.gx[v];
        ring[slot][3 * v + 2][lane] = cur.gy[v];
      }
    }
    if (j >= a0) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        ySm[v] = Sy[v];
        yDm[v] = Dy[v];
      }
    }
    prev = cur;
    cur = nx1;
    nx1 = nx2;
  }
  if ((badA && liveA) || (badB && liveB)) atomicOr(p.status, 1);
  if (p.dt_next) {
    dtmin = wave_min(dtmin);
    if (lane == 0) p.dtpart[wave] = dtmin;
  }
}

template <typename T, int LIM>
__global__ __launch_bounds__(256) void k_cart2d_step(P2<T> p) {
  __shared__ T ring[4][kStepRing][12][kLanes];
  const int lane = threadIdx.x & (kLanes - 1);
  const int w = threadIdx.x >> 6;
  const int wave = xcd_remap(blockIdx.x, gridDim.x) * 4 + w;
  if (wave >= p.ntiles) return;
  cart2d_step_tile<T, LIM>(p, wave, lane, ring[w]);
}

// ---------------------------------------------------------------- batches --
// A batch of independent meshes stored one after another in the same
// coefficient-major arrays (stride nc = total cells of the batch).  Tile t
// belongs to instance tile_inst[t]; the instance record gives its geometry
// constants (precomputed on the host, in T), its first cell and first tile.
// The kernel is persistent when launched with fewer waves than tiles: each
// wave then walks the tile list with a stride of the launched wave count.
template <typename T>
struct BInst {
  int nx, ny, tiles_x, rows;
  int off, tile0, ntiles, pad;
  T cmx, cmy, cgx, cgy, ccr, hx2, hy2, qx, qy;
  double ihx, ihy;
};

template <typename T>
struct PB {
  P2<T> base;               // pointers, nc, gamma, status, dtpart, dt_next
  const BInst<T>* inst;
  const int* tile_inst;
  int ntiles;               // tiles of the whole batch
  int wpb;                  // waves per workgroup
};

template <typename T>
__device__ __forceinline__ P2<T> inst_params(const PB<T>& b, int i) {
  const BInst<T>& in = b.inst[i];
  P2<T> p = b.base;
  p.in = b.base.in + in.off;
  p.u0 = b.base.u0 ? b.base.u0 + in.off : nullptr;
  p.out = b.base.out + in.off;
  p.dt_dev = b.base.dt_dev ? b.base.dt_dev + i : nullptr;
  p.dtpart = b.base.dtpart + in.tile0;
  p.nx = in.nx;
  p.ny = in.ny;
  p.rows = in.rows;
  p.tiles_x = in.tiles_x;
  p.ntiles = in.ntiles;
  p.cmx = in.cmx;
  p.cmy = in.cmy;
  p.cgx = in.cgx;
  p.cgy = in.cgy;
  p.ccr = in.ccr;
  p.hx2 = in.hx2;
  p.hy2 = in.hy2;
  p.qx = in.qx;
  p.qy = in.qy;
  p.ihx = in.ihx;
  p.ihy = in.ihy;
  return p;
}

template <typename T, int MODE, int LIM>
__global__ __launch_bounds__(256) void k_cart2d_batch(PB<T> b) {
  const int lane = threadIdx.x & (kLanes - 1);
  const int nw = gridDim.x * b.wpb;
  int w = __builtin_amdgcn_readfirstlane(xcd_remap(blockIdx.x, gridDim.x) * b.wpb +
                                         (threadIdx.x >> 6));
  for (int t = w; t < b.ntiles; t += nw) {
    const int i = __builtin_amdgcn_readfirstlane(b.tile_inst[t]);
    const P2<T> p = inst_params(b, i);
    cart2d_tile<T, MODE, LIM>(p, t - b.inst[i].tile0, lane);
  }
}

// Per-tile CFL minima of a batch state (the tile decomposition of the stage
// kernels; each lane walks its column).
template <typename T>
__global__ __launch_bounds__(256) void k_cart2d_batch_cfl(PB<T> b) {
  const int lane = threadIdx.x & (kLanes - 1);
  const int nw = gridDim.x * b.wpb;
  int w = __builtin_amdgcn_readfirstlane(blockIdx.x * b.wpb + (threadIdx.x >> 6));
  for (int t = w; t < b.ntiles; t += nw) {
    const int i = __builtin_amdgcn_readfirstlane(b.tile_inst[t]);
    const P2<T> p = inst_params(b, i);
    const int lt = t - b.inst[i].tile0;
    const int tx = lt % p.tiles_x, ty = lt / p.tiles_x;
    const int col = tx * kCols + lane - 2;
    double d = 1e300;
    if (lane >= 2 && lane < 2 + kCols && col < p.nx) {
      const int y1 = min(ty * p.rows + p.rows, p.ny);
      for (int y = ty * p.rows; y < y1; ++y) {
        T m[4];
        load_means(p.in, p.nc, y * p.nx + col, m);
        d = fmin(d, cell_dt(m, p));
      }
    }
    d = wave_min(d);
    if (lane == 0) b.base.dtpart[t] = d;
  }
}

// dt[i] = cfl * min over instance i's tiles [first[i], first[i+1]).
__global__ __launch_bounds__(256) void k_min_finalize_batch(const double* part,
                                                            const int* first, double cfl,
                                                            double* dt) {
  __shared__ double s[4];
  const int i = blockIdx.x;
  double d = 1e300;
  for (int t = first[i] + threadIdx.x; t < first[i + 1]; t += 256) d = fmin(d, part[t]);
  d = wave_min(d);
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = d;
  __syncthreads();
  if (threadIdx.x == 0) dt[i] = cfl * fmin(fmin(s[0], s[1]), fmin(s[2], s[3]));
}

// Per-wave CFL minima of a state's cell means (stand-alone dg_cfl_dt).
template <typename T>
__global__ __launch_bounds__(256) void k_cart2d_cfl(P2<T> p) {
  const int e = blockIdx.x * blockDim.x + threadIdx.x;
  double d = 1e300;
  if (e < p.nc) {
    T m[4];
    load_means(p.in, p.nc, e, m);
    d = cell_dt(m, p);
  }
  for (int o = 32; o > 0; o >>= 1) d = fmin(d, __shfl_xor(d, o));
  if ((threadIdx.x & 63) == 0) p.dtpart[e >> 6] = d;
}

// Final minimum over the partials: *dt = cfl * min.  One workgroup of 1024
// threads; min is exact in any order, so the result is deterministic.
__global__ __launch_bounds__(1024) void k_min_finalize(const double* part, int n, double cfl,
                                                       double* dt) {
  __shared__ double s[16];
  double d = 1e300;
  for (int i = threadIdx.x; i < n; i += 1024) d = fmin(d, part[i]);
  d = wave_min(d);
  if ((threadIdx.x & 63) == 0) s[threadIdx.x >> 6] = d;
  __syncthreads();
  if (threadIdx.x < 64) {
    d = threadIdx.x < 16 ? s[threadIdx.x] : 1e300;
    d = wave_min(d);
    if (threadIdx.x == 0) *dt = cfl * d;
  }
}

template <typename T>
P2<T> make_params(const dg_mesh* m, const void* in, const void* u0, void* out,
                  const double* dt_dev, double dt_host) {
  P2<T> p;
  p.in = static_cast<const T*>(in);
  p.u0 = static_cast<const T*>(u0);
  p.out = static_cast<T*>(out);
  p.dt_dev = dt_dev;
  p.dt_host = dt_host;
  p.status = m->status;
  p.dtpart = m->dtpart;
  p.dt_next = nullptr;
  p.cfl = 0.0;
  p.nx = m->c2.nx;
  p.ny = m->c2.ny;
  p.rows = m->c2.rows_per_tile;
  p.tiles_x = m->c2.tiles_x;
  p.ntiles = m->c2.tiles_x * m->c2.tiles_y;
  p.nc = (int)m->ncells;
  const double hx = m->c2.hx, hy = m->c2.hy, s3 = 1.7320508075688772;
  p.gamma = (T)m->cfg.gamma;
  p.igm1 = (T)(1.0 / (m->cfg.gamma - 1.0));
  p.cmx = (T)(0.5 / hx);
  p.cmy = (T)(0.5 / hy);
  p.cgx = (T)(3.0 / (hx * hx));
  p.cgy = (T)(3.0 / (hy * hy));
  p.ccr = (T)(s3 / (hx * hy));
  p.hx2 = (T)(0.5 * hx);
  p.hy2 = (T)(0.5 * hy);
  p.qx = (T)(0.5 * hx / s3);
  p.qy = (T)(0.5 * hy / s3);
  p.ihx = 1.0 / hx;
  p.ihy = 1.0 / hy;
  return p;
}

// One stage kernel launch for limiter LIM (0 none, 1 Arepo, 2 WENO).
template <typename T, int MODE, int RS>
void launch_lim(int lim, int nblocks, const P2<T>& p, hipStream_t s) {
  if constexpr (MODE == kStage1 && RS == 1 && sizeof(T) == 8) {
    if (lim == 2)
      hipLaunchKernelGGL((k_cart2d_w2<T, MODE, 2, RS>), dim3(nblocks), dim3(256), 0, s, p);
    else if (lim == 1)
      hipLaunchKernelGGL((k_cart2d_w2<T, MODE, 1, RS>), dim3(nblocks), dim3(256), 0, s, p);
    else
      hipLaunchKernelGGL((k_cart2d_w2<T, MODE, 0, RS>), dim3(nblocks), dim3(256), 0, s, p);
    return;
  }
  if (lim == 2)
    hipLaunchKernelGGL((k_cart2d<T, MODE, 2, RS>), dim3(nblocks), dim3(256), 0, s, p);
  else if (lim == 1)
    hipLaunchKernelGGL((k_cart2d<T, MODE, 1, RS>), dim3(nblocks), dim3(256), 0, s, p);
  else
    hipLaunchKernelGGL((k_cart2d<T, MODE, 0, RS>), dim3(nblocks), dim3(256), 0, s, p);
}

template <typename T, int RS>
hipError_t launch_t(const dg_mesh* m, int mode, const void* in, const void* u0, void* out,
                    const double* dt_dev, double dt_host, double cfl, double* dt_next,
                    hipStream_t s) {
  P2<T> p = make_params<T>(m, in, u0, out, dt_dev, dt_host);
  const int nblocks = (p.ntiles + 3) / 4;
  const int lim = m->cfg.limiter;  // 0 none, 1 Arepo, 2 WENO
  if (mode == kStage2 || mode == kMH || mode == kStep) {
    p.dt_next = dt_next;
    p.cfl = cfl;
  }
  switch (mode) {
    case kRhs:
      hipLaunchKernelGGL((k_cart2d<T, kRhs, 0, RS>), dim3(nblocks), dim3(256), 0, s, p);
      break;
    case kLimit:
      if (lim == 2)
        hipLaunchKernelGGL((k_cart2d<T, kLimit, 2, 0>), dim3(nblocks), dim3(256), 0, s, p);
      else
        hipLaunchKernelGGL((k_cart2d<T, kLimit, 1, 0>), dim3(nblocks), dim3(256), 0, s, p);
      break;
    case kStage1:
      launch_lim<T, kStage1, RS>(lim, nblocks, p, s);
      break;
    case kStage2:
      launch_lim<T, kStage2, RS>(lim, nblocks, p, s);
      if (dt_next)
        hipLaunchKernelGGL(k_min_finalize, dim3(1), dim3(1024), 0, s, m->dtpart, p.ntiles, cfl,
                           dt_next);
      break;
    case kMH:
      launch_lim<T, kMH, RS>(lim, nblocks, p, s);
      if (dt_next)
        hipLaunchKernelGGL(k_min_finalize, dim3(1), dim3(1024), 0, s, m->dtpart, p.ntiles, cfl,
                           dt_next);
      break;
    case kStep: {
      // HLL and the limiter off or of Sec. 2.5 (the caller checks)
      if (RS != 0 || lim == 2 || m->cfg.physics != DG_EULER) return hipErrorInvalidValue;
      p.rows = m->c2.step_rows;
      p.tiles_x = m->c2.step_tiles_x;
      p.ntiles = m->c2.step_tiles_x * m->c2.step_tiles_y;
      const int nb = (p.ntiles + 3) / 4;
      if (lim == 1)
        hipLaunchKernelGGL((k_cart2d_step<T, 1>), dim3(nb), dim3(256), 0, s, p);
      else
        hipLaunchKernelGGL((k_cart2d_step<T, 0>), dim3(nb), dim3(256), 0, s, p);
      if (dt_next)
        hipLaunchKernelGGL(k_min_finalize, dim3(1), dim3(1024), 0, s, m->dtpart, p.ntiles, cfl,
                           dt_next);
      break;
    }
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t cfl_t(const dg_mesh* m, const void* U, double cfl, double* dt_dev, hipStream_t s) {
  P2<T> p = make_params<T>(m, U, nullptr, nullptr, nullptr, 0.0);
  p.dtpart = m->dtpart;
  const int64_t nblk = (m->ncells + 255) / 256;
  hipLaunchKernelGGL((k_cart2d_cfl<T>), dim3((unsigned)nblk), dim3(256), 0, s, p);
  const int nparts = (int)((m->ncells + 63) / 64);
  hipLaunchKernelGGL(k_min_finalize, dim3(1), dim3(1024), 0, s, m->dtpart, nparts, cfl, dt_dev);
  return hipGetLastError();
}

template <typename T>
PB<T> make_batch_params(const dg_mesh* m, const void* in, const void* u0, void* out,
                        const double* dt_dev, double dt_host) {
  PB<T> b;
  b.base = P2<T>{};
  b.base.in = static_cast<const T*>(in);
  b.base.u0 = static_cast<const T*>(u0);
  b.base.out = static_cast<T*>(out);
  b.base.dt_dev = dt_dev;
  b.base.dt_host = dt_host;
  b.base.status = m->status;
  b.base.dtpart = m->dtpart;
  b.base.dt_next = nullptr;
  b.base.nc = (int)m->ncells;
  b.base.gamma = (T)m->cfg.gamma;
  b.base.igm1 = (T)(1.0 / (m->cfg.gamma - 1.0));
  b.inst = static_cast<const BInst<T>*>(m->bt.inst);
  b.tile_inst = m->bt.tile_inst;
  b.ntiles = m->bt.ntiles;
  b.wpb = m->bt.wpb;
  return b;
}

template <typename T>
hipError_t launch_batch_t(const dg_mesh* m, int mode, const void* in, const void* u0, void* out,
                          const double* dt_dev, double dt_host, double cfl, double* dt_next,
                          hipStream_t s) {
  PB<T> b = make_batch_params<T>(m, in, u0, out, dt_dev, dt_host);
  const int wpb = b.wpb;
  int waves = b.ntiles;
  if (m->bt.grid_waves > 0 && m->bt.grid_waves < waves) waves = m->bt.grid_waves;
  const int nblocks = (waves + wpb - 1) / wpb;
  const dim3 grid(nblocks), block(64 * wpb);
  const bool lim = m->cfg.limiter == DG_LIMITER_MINMOD;
  if (mode == kStage2 || mode == kMH) {
    b.base.dt_next = dt_next;
    b.base.cfl = cfl;
  }
  switch (mode) {
    case kRhs:
      hipLaunchKernelGGL((k_cart2d_batch<T, kRhs, false>), grid, block, 0, s, b);
      break;
    case kLimit:
      hipLaunchKernelGGL((k_cart2d_batch<T, kLimit, true>), grid, block, 0, s, b);
      break;
    case kStage1:
      if (lim)
        hipLaunchKernelGGL((k_cart2d_batch<T, kStage1, true>), grid, block, 0, s, b);
      else
        hipLaunchKernelGGL((k_cart2d_batch<T, kStage1, false>), grid, block, 0, s, b);
      break;
    case kStage2:
      if (lim)
        hipLaunchKernelGGL((k_cart2d_batch<T, kStage2, true>), grid, block, 0, s, b);
      else
        hipLaunchKernelGGL((k_cart2d_batch<T, kStage2, false>), grid, block, 0, s, b);
      if (dt_next)
        hipLaunchKernelGGL(k_min_finalize_batch, dim3(m->bt.ninst), dim3(256), 0, s, m->dtpart,
                           m->bt.inst_tile0, cfl, dt_next);
      break;
    case kMH:
      if (lim)
        hipLaunchKernelGGL((k_cart2d_batch<T, kMH, true>), grid, block, 0, s, b);
      else
        hipLaunchKernelGGL((k_cart2d_batch<T, kMH, false>), grid, block, 0, s, b);
      if (dt_next)
        hipLaunchKernelGGL(k_min_finalize_batch, dim3(m->bt.ninst), dim3(256), 0, s, m->dtpart,
                           m->bt.inst_tile0, cfl, dt_next);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t batch_cfl_t(const dg_mesh* m, const void* U, double cfl, double* dt_dev,
                       hipStream_t s) {
  PB<T> b = make_batch_params<T>(m, U, nullptr, nullptr, nullptr, 0.0);
  b.wpb = 4;
  const int nblocks = (b.ntiles + 3) / 4;
  hipLaunchKernelGGL((k_cart2d_batch_cfl<T>), dim3(nblocks), dim3(256), 0, s, b);
  hipLaunchKernelGGL(k_min_finalize_batch, dim3(m->bt.ninst), dim3(256), 0, s, m->dtpart,
                     m->bt.inst_tile0, cfl, dt_dev);
  return hipGetLastError();
}

template <typename T>
void fill_inst(const BatchDesc& d, int rows, void* out_records) {
  BInst<T>* r = static_cast<BInst<T>*>(out_records);
  const double s3 = 1.7320508075688772;
  int off = 0, tile0 = 0;
  for (int i = 0; i < d.ninst; ++i) {
    const int nx = d.nx[i], ny = d.ny[i];
    const double hx = d.hx[i], hy = d.hy[i];
    BInst<T> b{};
    b.nx = nx;
    b.ny = ny;
    b.tiles_x = (nx + kCols - 1) / kCols;
    b.rows = rows < ny ? rows : ny;
    b.off = off;
    b.tile0 = tile0;
    b.ntiles = b.tiles_x * ((ny + b.rows - 1) / b.rows);
    b.cmx = (T)(0.5 / hx);
    b.cmy = (T)(0.5 / hy);
    b.cgx = (T)(3.0 / (hx * hx));
    b.cgy = (T)(3.0 / (hy * hy));
    b.ccr = (T)(s3 / (hx * hy));
    b.hx2 = (T)(0.5 * hx);
    b.hy2 = (T)(0.5 * hy);
    b.qx = (T)(0.5 * hx / s3);
    b.qy = (T)(0.5 * hy / s3);
    b.ihx = 1.0 / hx;
    b.ihy = 1.0 / hy;
    r[i] = b;
    off += nx * ny;
    tile0 += b.ntiles;
  }
}

}  // namespace

// Host-side instance records and tile tables of a batch for `rows` rows per
// tile.  records: ninst records of the precision's layout (batch_record_size
// bytes each); tile_inst[ntiles]; tile0[ninst + 1].  Returns the tile count.
size_t batch_record_size(bool f64) { return f64 ? sizeof(BInst<double>) : sizeof(BInst<float>); }

int batch_tables(const BatchDesc& d, bool f64, int rows, void* records,
                 std::vector<int>& tile_inst, std::vector<int>& tile0) {
  if (f64)
    fill_inst<double>(d, rows, records);
  else
    fill_inst<float>(d, rows, records);
  tile_inst.clear();
  tile0.assign(1, 0);
  for (int i = 0; i < d.ninst; ++i) {
    const int tx = (d.nx[i] + kCols - 1) / kCols;
    const int r = rows < d.ny[i] ? rows : d.ny[i];
    const int nt = tx * ((d.ny[i] + r - 1) / r);
    for (int t = 0; t < nt; ++t) tile_inst.push_back(i);
    tile0.push_back(tile0.back() + nt);
  }
  return (int)tile_inst.size();
}

hipError_t launch_cart2d_batch(const dg_mesh* m, int mode, const void* in, const void* u0,
                               void* out, const double* dt_dev, double dt_host, double cfl,
                               double* dt_next, hipStream_t s) {
  if (m->cfg.precision == DG_FP64)
    return launch_batch_t<double>(m, mode, in, u0, out, dt_dev, dt_host, cfl, dt_next, s);
  return launch_batch_t<float>(m, mode, in, u0, out, dt_dev, dt_host, cfl, dt_next, s);
}

hipError_t launch_cart2d_batch_cfl(const dg_mesh* m, const void* U, double cfl, double* dt_dev,
                                   hipStream_t s) {
  if (m->cfg.precision == DG_FP64) return batch_cfl_t<double>(m, U, cfl, dt_dev, s);
  return batch_cfl_t<float>(m, U, cfl, dt_dev, s);
}

hipError_t launch_cart2d(const dg_mesh* m, int mode, const void* in, const void* u0, void* out,
                         const double* dt_dev, double dt_host, double cfl, double* dt_next,
                         hipStream_t s) {
  const bool ex = m->cfg.flux == DG_FLUX_EXACT;
  if (m->cfg.precision == DG_FP64)
    return ex ? launch_t<double, 1>(m, mode, in, u0, out, dt_dev, dt_host, cfl, dt_next, s)
              : launch_t<double, 0>(m, mode, in, u0, out, dt_dev, dt_host, cfl, dt_next, s);
  return ex ? launch_t<float, 1>(m, mode, in, u0, out, dt_dev, dt_host, cfl, dt_next, s)
            : launch_t<float, 0>(m, mode, in, u0, out, dt_dev, dt_host, cfl, dt_next, s);
}

hipError_t launch_cart2d_cfl(const dg_mesh* m, const void* U, double cfl, double* dt_dev,
                             hipStream_t s) {
  if (m->cfg.precision == DG_FP64) return cfl_t<double>(m, U, cfl, dt_dev, s);
  return cfl_t<float>(m, U, cfl, dt_dev, s);
}

hipError_t launch_min_finalize(const double* part, int n, double cfl, double* dt,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_min_finalize, dim3(1), dim3(1024), 0, s, part, n, cfl, dt);
  return hipGetLastError();
}

}  // namespace dg

// ------------------------------------------- CFL step without allocation --
// dg_cfl_dt_static keeps the per-wave partial minima in this file-scope
// device array instead of the handle's workspace (each GPU holds its own copy
// until the process ends).  In host code its name is not a device address:
// the address comes from hipGetSymbolAddress, taken once per device at mesh
// creation with that device current, and only that pointer reaches kernels.
static __device__ __align__(256) double scratch[dg::kCflScratchParts];

namespace dg {
namespace {
constexpr int kMaxScratchDevices = 64;
std::mutex g_scratch_mu;
double* g_scratch[kMaxScratchDevices] = {};
}  // namespace

hipError_t cart2d_scratch_init() {
  int dev = 0;
  hipError_t e = hipGetDevice(&dev);
  if (e != hipSuccess) return e;
  if (dev < 0 || dev >= kMaxScratchDevices) return hipErrorInvalidDevice;
  std::lock_guard<std::mutex> lock(g_scratch_mu);
  if (g_scratch[dev]) return hipSuccess;
  void* ptr = nullptr;
  e = hipGetSymbolAddress(&ptr, HIP_SYMBOL(scratch));
  if (e != hipSuccess) return e;
  g_scratch[dev] = static_cast<double*>(ptr);
  return hipSuccess;
}

template <typename T>
hipError_t cfl_static_t(const dg_mesh* m, double* part, const void* U, double cfl,
                        double* dt_dev, hipStream_t s) {
  P2<T> p = make_params<T>(m, U, nullptr, nullptr, nullptr, 0.0);
  p.dtpart = part;
  const int64_t nblk = (m->ncells + 255) / 256;
  hipLaunchKernelGGL((k_cart2d_cfl<T>), dim3((unsigned)nblk), dim3(256), 0, s, p);
  const int nparts = (int)((m->ncells + 63) / 64);
  hipLaunchKernelGGL(k_min_finalize, dim3(1), dim3(1024), 0, s, part, nparts, cfl, dt_dev);
  return hipGetLastError();
}

// Same kernels as launch_cart2d_cfl; every partial the finalisation reads is
// written first by the CFL kernel of the same call, so nothing is cleared.
hipError_t launch_cart2d_cfl_static(const dg_mesh* m, const void* U, double cfl, double* dt_dev,
                                    hipStream_t s) {
  if (4 * ((m->ncells + 255) / 256) > kCflScratchParts) return hipErrorInvalidValue;
  double* part = nullptr;
  {
    std::lock_guard<std::mutex> lock(g_scratch_mu);
    if (m->device >= 0 && m->device < kMaxScratchDevices) part = g_scratch[m->device];
  }
  if (!part) return hipErrorInvalidSymbol;
  if (m->cfg.precision == DG_FP64) return cfl_static_t<double>(m, part, U, cfl, dt_dev, s);
  return cfl_static_t<float>(m, part, U, cfl, dt_dev, s);
}

}  // namespace dg
