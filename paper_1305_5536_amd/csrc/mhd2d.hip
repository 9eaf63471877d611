// DG stage kernels for 2D ideal MHD on a periodic Cartesian mesh (gfx950).
//
// Method (Sec. 2.2, two-dimensional case): P1 Taylor basis for rho, the three
// momenta and E (mean + in-plane gradient, 15 coefficients); the in-plane field
// (Bx, By) in the 2D locally divergence-free basis, V1, V2 for the means and
// V3 = (y, 0), V4 = (0, x), V5 = (x, -y) for the linear part (coefficients
// a1..a3); the out-of-plane Bz in the Taylor basis (mean + two gradient
// coefficients).  23 coefficients per cell, stored coefficient-major:
//   3v, 3v+1, 3v+2   mean, d/dx, d/dy of rho, mx, my, mz, E (v = 0..4)
//   15, 16, 17       means of Bx, By, Bz
//   18, 19, 20       a1, a2, a3
//   21, 22           d/dx, d/dy of Bz
// Surface terms at the two Gauss points of every edge with the HLLD flux
// (Sec. 2.3) on the face-averaged normal field (Sec. 2.6); volume terms at
// 2x2 Gauss points; the inverse mass matrices of a box are diagonal (the
// 3x3 Gram block of V3..V5 is diag(m_yy, m_xx, m_xx + m_yy)); slope limiter of
// Sec. 2.5 with one alpha for Bx, By and Bz.
//
// Kernels.
//   k_mhd2d : one SSP-RK2 stage (or L alone), limiting its input on read.  One
//             wave owns up to 60 x-columns (lanes 0, 1 and 62, 63 are halo
//             columns: a limited cell needs its x-neighbours' means, an owned
//             cell its x-neighbours limited) and marches up a range of rows.
//             The current limited row sits in wave-private LDS (each lane only
//             touches its own slot), the row above is loaded and limited while
//             the current row's x-faces and volume term are computed (its
//             y-neighbours' means are the current row and one row further up).
//             x-faces: each lane solves its -x face per Gauss point and hands
//             the flux to its left neighbour through DPP.  y-faces: solved once
//             per row pair, the lower row's sums carried to the next row; a
//             tile's first -y face is solved by both tiles that share it with
//             the same operands and arithmetic, so every face flux is
//             bit-identical on its two sides.  Stage 1 also writes Pi(U^n) of
//             its cells, which stage 2 reads for its combination.
//   k_lim2m : Pi(U) -> out, one thread per cell (dg_limit, and Pi(U^n) for a
//             stage 2 not preceded by the stage 1 of the same U).
//   k_cfl2m : per-wave minima of the CFL bound (fast magnetosonic speeds).
// The stage kernel is VALU-bound: four HLLD solves per cell and stage.
//
// Residual algebra per face of axis D (tangential axis t), Gauss points at
// tangential signs s, S = sum F, T = sum s F, cell on side sigma (+1 when it is
// the R cell, -1 when the L cell), all divided by the cell area:
//   mean_k    += sigma S_k / (2 h_D)
//   grad_v[D] -= 3 S_v / h_D^2
//   grad_v[t] += sigma sqrt3 T_v / (h_D h_t)
//   P[c][D]   -= S_Bc / 4,     P[c][t] += sigma h_t T_Bc / (4 sqrt3 h_D)
// volume (4 points): grad_v[e] += 3 F^e_v / h_e^2, P[c][e] += F^e(B_c) / 4.
// The field coefficients follow from P:
//   a1 = P[x][y] / mu_y, a2 = P[y][x] / mu_x, a3 = (P[x][x] - P[y][y]) / (mu_x + mu_y),
//   dBz/dx = P[z][x] / mu_x, dBz/dy = P[z][y] / mu_y,   mu_d = h_d^2 / 12.
#include <hip/hip_runtime.h>

#include "dg_internal.h"
#include "dg_math.h"
#include "mhd_hlld.h"

namespace dg {
namespace {

template <typename T>
struct P2M {
  const T* __restrict__ in;  // limited state (stage kernel) or raw state (limiter, CFL)
  const T* __restrict__ ua;  // stage 2: Pi(U^n)
  T* __restrict__ out;
  T* __restrict__ lim_out;   // stage 1 with the limiter: Pi(in) of the owned cells (or NULL)
  const double* dt_dev;
  double dt_host;
  int* status;
  double* dtpart;
  int nx, ny, nc;
  int width, tiles_x, rows, tiles_y, ntiles;
  T gamma, eps;
  T c2h[2];   // 1/(2 h_d)
  T c3[2];    // 3/h_d^2
  T cs;       // sqrt3/(h_x h_y)
  T pt[2];    // face of axis d: h_t/(4 sqrt3 h_d)
  T half[2];  // h_d/2
  T q[2];     // Gauss offset h_d/(2 sqrt3)
  T imu[3];   // 1/mu_x, 1/mu_y, 1/(mu_x + mu_y)
  double ih[2];
};

// Coefficients of one cell: hydro v = rho, mx, my, mz, E with mean m[v] and
// gradient g[v][d]; field means b[c]; a[0..4] = a1, a2, a3, dBz/dx, dBz/dy.
template <typename T>
struct Q2 {
  T m[5], g[5][2], b[3], a[5];
};

template <typename T>
__device__ __forceinline__ void load_q(const T* __restrict__ U, int nc, int e, Q2<T>& q) {
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    q.m[v] = U[(3 * v) * nc + e];
    q.g[v][0] = U[(3 * v + 1) * nc + e];
    q.g[v][1] = U[(3 * v + 2) * nc + e];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) q.b[c] = U[(15 + c) * nc + e];
#pragma unroll
  for (int j = 0; j < 5; ++j) q.a[j] = U[(18 + j) * nc + e];
}

template <typename T>
__device__ __forceinline__ void store_q(T* __restrict__ U, int nc, int e, const Q2<T>& q) {
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    U[(3 * v) * nc + e] = q.m[v];
    U[(3 * v + 1) * nc + e] = q.g[v][0];
    U[(3 * v + 2) * nc + e] = q.g[v][1];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) U[(15 + c) * nc + e] = q.b[c];
#pragma unroll
  for (int j = 0; j < 5; ++j) U[(18 + j) * nc + e] = q.a[j];
}

// Conserved means in the order rho, mx, my, mz, E, Bx, By, Bz.
template <typename T>
__device__ __forceinline__ void load_means(const T* __restrict__ U, int nc, int e, T* m) {
#pragma unroll
  for (int v = 0; v < 5; ++v) m[v] = U[(3 * v) * nc + e];
#pragma unroll
  for (int c = 0; c < 3; ++c) m[5 + c] = U[(15 + c) * nc + e];
}

// Gradient of B_c: grad Bx = (a3, a1), grad By = (a2, -a3), grad Bz = (a4, a5).
template <typename T>
__device__ __forceinline__ T dB(const T* a, int c, int d) {
  if (c == 0) return d == 0 ? a[2] : a[0];
  if (c == 1) return d == 0 ? a[1] : -a[2];
  return d == 0 ? a[3] : a[4];
}

// Limiter factor of one variable on a box: the linear extrapolation to the
// four edge midpoints stays within the neighbourhood's extreme means.
template <typename T>
__device__ __forceinline__ T alpha_of(T phi, T hi, T lo, T gx, T gy, const P2M<T>& p) {
  const T D = fmin(hi - phi, phi - lo);
  const T dm = fmax(fabs(gx) * p.half[0], fabs(gy) * p.half[1]);
  return (dm > D) ? div_small(D, dm) : T(1);
}

// The limiter of Sec. 2.5 applied to a cell held by this lane, inside a row
// held by the wave: the x-neighbours' means come from lanes -1 and +1 by DPP
// (the end lanes get wrong values; they are halo lanes whose results are not
// used), the y-neighbours' means are mS and mN (order rho, mx, my, mz, E, Bx,
// By, Bz).
template <typename T>
__device__ __forceinline__ void limit_in_row(Q2<T>& q, const T* mS, const T* mN,
                                             const P2M<T>& p) {
  T hi[8], lo[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    const T own = k < 5 ? q.m[k] : q.b[k - 5];
    const T l = lane_up(own), r = lane_down(own);
    hi[k] = fmax(fmax(fmax(own, l), fmax(r, mS[k])), mN[k]);
    lo[k] = fmin(fmin(fmin(own, l), fmin(r, mS[k])), mN[k]);
  }
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const T a = alpha_of(q.m[v], hi[v], lo[v], q.g[v][0], q.g[v][1], p);
    q.g[v][0] *= a;
    q.g[v][1] *= a;
  }
  T aB = T(1);
#pragma unroll
  for (int c = 0; c < 3; ++c)
    aB = fmin(aB, alpha_of(q.b[c], hi[5 + c], lo[5 + c], dB(q.a, c, 0), dB(q.a, c, 1), p));
#pragma unroll
  for (int jj = 0; jj < 5; ++jj) q.a[jj] *= aB;
}

template <typename T>
__device__ __forceinline__ void means_of(const Q2<T>& q, T* m) {
#pragma unroll
  for (int v = 0; v < 5; ++v) m[v] = q.m[v];
#pragma unroll
  for (int c = 0; c < 3; ++c) m[5 + c] = q.b[c];
}

// ------------------------------------------------------------- limiter --
template <typename T>
__global__ __launch_bounds__(256) void k_lim2m(P2M<T> p) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= p.nc) return;
  const int nx = p.nx, ny = p.ny;
  const int i = e % nx, j = e / nx;
  const int nb[4] = {e - i + (i == 0 ? nx - 1 : i - 1), e - i + (i == nx - 1 ? 0 : i + 1),
                     e + ((j == 0 ? ny - 1 : j - 1) - j) * nx,
                     e + ((j == ny - 1 ? 0 : j + 1) - j) * nx};
  Q2<T> q;
  load_q(p.in, p.nc, e, q);
  T hi[8], lo[8];
#pragma unroll
  for (int v = 0; v < 5; ++v) hi[v] = lo[v] = q.m[v];
#pragma unroll
  for (int c = 0; c < 3; ++c) hi[5 + c] = lo[5 + c] = q.b[c];
#pragma unroll
  for (int f = 0; f < 4; ++f) {
    T mn[8];
    load_means(p.in, p.nc, nb[f], mn);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      hi[k] = fmax(hi[k], mn[k]);
      lo[k] = fmin(lo[k], mn[k]);
    }
  }
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const T a = alpha_of(q.m[v], hi[v], lo[v], q.g[v][0], q.g[v][1], p);
    q.g[v][0] *= a;
    q.g[v][1] *= a;
  }
  T aB = T(1);
#pragma unroll
  for (int c = 0; c < 3; ++c)
    aB = fmin(aB, alpha_of(q.b[c], hi[5 + c], lo[5 + c], dB(q.a, c, 0), dB(q.a, c, 1), p));
#pragma unroll
  for (int jj = 0; jj < 5; ++jj) q.a[jj] *= aB;
  store_q(p.out, p.nc, e, q);
}

// Per-side values of the cell polynomial on a face of axis D: the state at
// the edge midpoint (normal offset +-h_D/2) and its increment to the Gauss
// point at tangential sign +1.
template <typename T, int D>
__device__ __forceinline__ void face_trace(const Q2<T>& q, T sgn_n, const P2M<T>& p, T* base,
                                           T* inc) {
  constexpr int t = 1 - D;
  const T hn = sgn_n * p.half[D];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    base[v] = fma(q.g[v][D], hn, q.m[v]);
    inc[v] = q.g[v][t] * p.q[t];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    base[5 + c] = fma(dB(q.a, c, D), hn, q.b[c]);
    inc[5 + c] = dB(q.a, c, t) * p.q[t];
  }
}

template <typename T>
struct Sums {
  T S[8], T1[8];
};

// Flux sums over the two Gauss points of a face of axis D between L and R.
template <typename T, int D>
__device__ __forceinline__ void face(const Q2<T>& L, const Q2<T>& R, const P2M<T>& p, Sums<T>& fs,
                                     bool& bad) {
  T bL[8], iL[8], bR[8], iR[8];
  face_trace<T, D>(L, T(1), p, bL, iL);
  face_trace<T, D>(R, T(-1), p, bR, iR);
#pragma unroll
  for (int k = 0; k < 8; ++k) fs.S[k] = fs.T1[k] = T(0);
#pragma unroll 1
  for (int g = 0; g < 2; ++g) {
    const T s = g ? T(1) : T(-1);
    T uL[8], uR[8], F[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      uL[k] = fma(s, iL[k], bL[k]);
      uR[k] = fma(s, iR[k], bR[k]);
    }
    // one normal field for the Riemann problem: the average of both sides
    const T bn = T(0.5) * (uL[5 + D] + uR[5 + D]);
    uL[5 + D] = bn;
    uR[5 + D] = bn;
    hlld_axis<T, D>(uL, uR, p.gamma, p.eps, F, bad);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      fs.S[k] += F[k];
      fs.T1[k] = fma(s, F[k], fs.T1[k]);
    }
  }
}

template <typename T>
struct Acc {
  T m[8], g[5][2], P[3][2];
};

template <typename T>
__device__ __forceinline__ void zero(Acc<T>& a) {
#pragma unroll
  for (int k = 0; k < 8; ++k) a.m[k] = T(0);
#pragma unroll
  for (int v = 0; v < 5; ++v) a.g[v][0] = a.g[v][1] = T(0);
#pragma unroll
  for (int c = 0; c < 3; ++c) a.P[c][0] = a.P[c][1] = T(0);
}

// Add one face's sums to a cell (sigma = +1: the cell's -D face, -1: its +D
// face).  The normal-field flux of a face of axis D is zero and is skipped.
template <typename T, int D>
__device__ __forceinline__ void add_face(Acc<T>& a, const Sums<T>& f, T sigma, const P2M<T>& p) {
  constexpr int t = 1 - D;
  const T cm = sigma * p.c2h[D], ct = sigma * p.cs, cp = sigma * p.pt[D];
#pragma unroll
  for (int k = 0; k < 8; ++k)
    if (k != 5 + D) a.m[k] = fma(cm, f.S[k], a.m[k]);
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    a.g[v][D] = fma(-p.c3[D], f.S[v], a.g[v][D]);
    a.g[v][t] = fma(ct, f.T1[v], a.g[v][t]);
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (c == D) continue;
    a.P[c][D] = fma(T(-0.25), f.S[5 + c], a.P[c][D]);
    a.P[c][t] = fma(cp, f.T1[5 + c], a.P[c][t]);
  }
}

// Volume term over the 2x2 Gauss points.
template <typename T>
__device__ __forceinline__ void add_volume(Acc<T>& a, const Q2<T>& q, const P2M<T>& p, bool& bad) {
  const T gm1 = p.gamma - T(1);
#pragma unroll 1
  for (int g = 0; g < 4; ++g) {
    const T o0 = (g & 2) ? p.q[0] : -p.q[0];
    const T o1 = (g & 1) ? p.q[1] : -p.q[1];
    T u[5], B[3];
#pragma unroll
    for (int v = 0; v < 5; ++v) u[v] = fma(q.g[v][0], o0, fma(q.g[v][1], o1, q.m[v]));
#pragma unroll
    for (int c = 0; c < 3; ++c) B[c] = fma(dB(q.a, c, 0), o0, fma(dB(q.a, c, 1), o1, q.b[c]));
    const T ir = rcp(u[0]);
    const T vel[3] = {u[1] * ir, u[2] * ir, u[3] * ir};
    const T pm = T(0.5) * (B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
    const T pg = gm1 * (u[4] - T(0.5) * (u[1] * vel[0] + u[2] * vel[1] + u[3] * vel[2]) - pm);
    bad |= !(u[0] > T(0)) || !(pg > T(0));
    const T pT = pg + pm;
    const T vB = vel[0] * B[0] + vel[1] * B[1] + vel[2] * B[2];
#pragma unroll
    for (int e = 0; e < 2; ++e) {
      T fe[5];
      fe[0] = u[1 + e];
#pragma unroll
      for (int k = 0; k < 3; ++k) fe[1 + k] = u[1 + k] * vel[e] - B[k] * B[e] + (k == e ? pT : T(0));
      fe[4] = (u[4] + pT) * vel[e] - B[e] * vB;
#pragma unroll
      for (int v = 0; v < 5; ++v) a.g[v][e] = fma(p.c3[e], fe[v], a.g[v][e]);
    }
    // induction fluxes F_e(B_c) = B_c v_e - v_c B_e
    const T fyx = B[0] * vel[1] - vel[0] * B[1];  // F_y(Bx) = -F_x(By)
    const T fxz = B[2] * vel[0] - vel[2] * B[0];  // F_x(Bz)
    const T fyz = B[2] * vel[1] - vel[2] * B[1];  // F_y(Bz)
    a.P[0][1] = fma(T(0.25), fyx, a.P[0][1]);
    a.P[1][0] = fma(T(-0.25), fyx, a.P[1][0]);
    a.P[2][0] = fma(T(0.25), fxz, a.P[2][0]);
    a.P[2][1] = fma(T(0.25), fyz, a.P[2][1]);
  }
}

// Time derivative of the coefficients from the accumulated residuals.
template <typename T>
__device__ __forceinline__ void finish(const Acc<T>& a, const P2M<T>& p, Q2<T>& d) {
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    d.m[v] = a.m[v];
    d.g[v][0] = a.g[v][0];
    d.g[v][1] = a.g[v][1];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) d.b[c] = a.m[5 + c];
  d.a[0] = a.P[0][1] * p.imu[1];
  d.a[1] = a.P[1][0] * p.imu[0];
  d.a[2] = (a.P[0][0] - a.P[1][1]) * p.imu[2];
  d.a[3] = a.P[2][0] * p.imu[0];
  d.a[4] = a.P[2][1] * p.imu[1];
}

// Accumulate one Gauss point of a face of axis D (tangential sign s) into a
// cell's residual, as add_face does for the sums of a face.
template <typename T, int D>
__device__ __forceinline__ void add_point(Acc<T>& a, const T* F, T s, T sigma, const P2M<T>& p) {
  constexpr int t = 1 - D;
  const T cm = sigma * p.c2h[D], ct = s * sigma * p.cs, cp = s * sigma * p.pt[D];
#pragma unroll
  for (int k = 0; k < 8; ++k)
    if (k != 5 + D) a.m[k] = fma(cm, F[k], a.m[k]);
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    a.g[v][D] = fma(-p.c3[D], F[v], a.g[v][D]);
    a.g[v][t] = fma(ct, F[v], a.g[v][t]);
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (c == D) continue;
    a.P[c][D] = fma(T(-0.25), F[5 + c], a.P[c][D]);
    a.P[c][t] = fma(cp, F[5 + c], a.P[c][t]);
  }
}

// Wave-private LDS copy of the current row's polynomials (one slot per lane),
// which keeps 23 values per lane out of the register file while the Riemann
// solves run.  Each lane touches only its own slot; the compiler barriers stop
// the compiler from forwarding the stores to the loads (which would put the
// row back into registers).
template <typename T>
struct Row {
  T v[23][64];
};

__device__ __forceinline__ void compiler_fence() { asm volatile("" ::: "memory"); }

template <typename T>
__device__ __forceinline__ void lds_put(Row<T>& r, int lane, const Q2<T>& q) {
  compiler_fence();
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    r.v[3 * v][lane] = q.m[v];
    r.v[3 * v + 1][lane] = q.g[v][0];
    r.v[3 * v + 2][lane] = q.g[v][1];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) r.v[15 + c][lane] = q.b[c];
#pragma unroll
  for (int j = 0; j < 5; ++j) r.v[18 + j][lane] = q.a[j];
  compiler_fence();
}

template <typename T>
__device__ __forceinline__ void lds_get(const Row<T>& r, int lane, Q2<T>& q) {
  compiler_fence();
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    q.m[v] = r.v[3 * v][lane];
    q.g[v][0] = r.v[3 * v + 1][lane];
    q.g[v][1] = r.v[3 * v + 2][lane];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) q.b[c] = r.v[15 + c][lane];
#pragma unroll
  for (int j = 0; j < 5; ++j) q.a[j] = r.v[18 + j][lane];
}

// CFL bound of a cell from its means: 1 / sum_d (|v_d| + c_f,d)/h_d over the
// two in-plane axes.
template <typename T>
__device__ __forceinline__ double cell_dt(const T* m, const P2M<T>& p) {
  const double r = m[0], ir = 1.0 / r;
  const double v[3] = {m[1] * ir, m[2] * ir, m[3] * ir};
  const double B[3] = {m[5], m[6], m[7]};
  const double B2 = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
  const double pg = ((double)p.gamma - 1.0) *
                    (m[4] - 0.5 * r * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) - 0.5 * B2);
  const double a2 = (double)p.gamma * pg * ir;
  const double sb = a2 + B2 * ir;
  double s = 0.0;
  for (int d = 0; d < 2; ++d) {
    const double disc = fmax(sb * sb - 4.0 * a2 * B[d] * B[d] * ir, 0.0);
    const double cf = sqrt(0.5 * (sb + sqrt(disc)));
    s += (fabs(v[d]) + cf) * p.ih[d];
  }
  return 1.0 / s;
}

// State at a point of a face of axis D: normal offset hn, tangential offset ht
// from the cell centroid.
template <typename T, int D>
__device__ __forceinline__ void point(const Q2<T>& q, T hn, T ht, T* u) {
  constexpr int t = 1 - D;
#pragma unroll
  for (int v = 0; v < 5; ++v) u[v] = fma(q.g[v][t], ht, fma(q.g[v][D], hn, q.m[v]));
#pragma unroll
  for (int c = 0; c < 3; ++c) u[5 + c] = fma(dB(q.a, c, t), ht, fma(dB(q.a, c, D), hn, q.b[c]));
}

// HLLD flux at the Gauss point of tangential sign s of the y-face between the
// cells lo (below) and hi (above).
template <typename T>
__device__ __forceinline__ void yface_point(const Q2<T>& lo, const Q2<T>& hi, T s,
                                            const P2M<T>& p, T* F, bool& bad) {
  T uL[8], uR[8];
  point<T, 1>(lo, p.half[1], s * p.q[0], uL);
  point<T, 1>(hi, -p.half[1], s * p.q[0], uR);
  // one normal field for the Riemann problem: the average of both sides
  const T bn = T(0.5) * (uL[6] + uR[6]);
  uL[6] = bn;
  uR[6] = bn;
  hlld_axis<T, 1>(uL, uR, p.gamma, p.eps, F, bad);
}

// Sums of a y-face from its two Gauss-point fluxes (s = -1, then +1).
template <typename T>
__device__ __forceinline__ void ysums(const T* Fm, const T* Fp, Sums<T>& f) {
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    f.S[k] = Fm[k] + Fp[k];
    f.T1[k] = Fp[k] - Fm[k];
  }
}

// Occupancy target (measured): one wave per SIMD in FP64, where the stage
// kernels then keep everything in registers (capping them at 256 for two waves
// spills and runs slower), three in FP32 (168 registers, no spills).
template <typename T>
struct Waves {
  static constexpr int n = sizeof(T) == 8 ? 1 : 3;
};

template <typename T, int MODE, bool LIM>
__global__ __launch_bounds__(64) __attribute__((amdgpu_waves_per_eu(Waves<T>::n, Waves<T>::n)))
void k_mhd2d(P2M<T> p) {
  __shared__ Row<T> row;  // the current (limited) row; each lane reads only its own slot
  const int lane = threadIdx.x;
  const int wave = xcd_remap(blockIdx.x, gridDim.x);
  if (wave >= p.ntiles) return;
  const int tx = wave % p.tiles_x, ty = wave / p.tiles_x;
  const int nx = p.nx, ny = p.ny, nc = p.nc;
  // lanes 0, 1 and 62, 63 are halo columns: a limited cell needs the means of
  // its x-neighbours, and an owned cell needs its x-neighbours limited
  const int colu = tx * p.width + lane - 2;
  const bool own = lane >= 2 && lane < 2 + p.width && colu < nx;
  int col = colu % nx;
  if (col < 0) col += nx;
  const int y0 = ty * p.rows;
  const int y1 = min(y0 + p.rows, ny);
  auto yw = [ny](int y) {
    y %= ny;
    return y < 0 ? y + ny : y;
  };
  bool bad = false;
  double dtmin = 1e300;

  Sums<T> carry;  // sums of the current row's -y face
  {
    Q2<T> prv, cur;
    load_q(p.in, nc, yw(y0 - 1) * nx + col, prv);
    load_q(p.in, nc, y0 * nx + col, cur);
    if (LIM) {
      T mA[8], mB[8], mP[8], mC[8];
      load_means(p.in, nc, yw(y0 - 2) * nx + col, mA);
      load_means(p.in, nc, yw(y0 + 1) * nx + col, mB);
      means_of(prv, mP);
      means_of(cur, mC);
      limit_in_row(prv, mA, mC, p);
      limit_in_row(cur, mP, mB, p);
    }
    T Fm[8], Fp[8];
    yface_point(prv, cur, T(-1), p, Fm, bad);
    yface_point(prv, cur, T(1), p, Fp, bad);
    ysums(Fm, Fp, carry);
    lds_put(row, lane, cur);
  }
  T dt = T(0);
  if (MODE != kRhs) dt = (T)(p.dt_dev ? *p.dt_dev : p.dt_host);

  for (int y = y0; y < y1; ++y) {
    Acc<T> acc;
    zero(acc);
    add_face<T, 1>(acc, carry, T(1), p);
    // x-faces: this lane solves its -x face at each Gauss point; the left
    // cell's +x point value comes from lane - 1 and the flux goes back to it
    // by DPP.  The row polynomial is re-read from LDS per point, so no face
    // trace stays live across a Riemann solve.
#pragma unroll 1
    for (int g = 0; g < 2; ++g) {
      const T s = g ? T(1) : T(-1);
      Q2<T> c;
      lds_get(row, lane, c);
      T uL[8], uR[8], F[8];
      point<T, 0>(c, p.half[0], s * p.q[1], uL);
      point<T, 0>(c, -p.half[0], s * p.q[1], uR);
#pragma unroll
      for (int k = 0; k < 8; ++k) uL[k] = lane_up(uL[k]);
      const T bn = T(0.5) * (uL[5] + uR[5]);
      uL[5] = bn;
      uR[5] = bn;
      hlld_axis<T, 0>(uL, uR, p.gamma, p.eps, F, bad);
      add_point<T, 0>(acc, F, s, T(1), p);
#pragma unroll
      for (int k = 0; k < 8; ++k) F[k] = lane_down(F[k]);
      add_point<T, 0>(acc, F, s, T(-1), p);
    }
    // the row above (limited on read: its y-neighbours are this row and the
    // row above it); the loads are in flight during the volume term.  In FP64
    // stage 2 issues its Pi(U^n) row here too: loaded right before the
    // combination, nothing would hide its latency at one wave per SIMD (FP32
    // runs three waves per SIMD within 168 registers, so it loads it late)
    constexpr bool kEarlyUa = sizeof(T) == 8;
    const int e = y * nx + col;
    Q2<T> nb;
    load_q(p.in, nc, yw(y + 1) * nx + col, nb);
    T mN2[8];
    if (LIM) load_means(p.in, nc, yw(y + 2) * nx + col, mN2);
    Q2<T> ua;
    if (MODE == kStage2 && kEarlyUa) load_q(p.ua, nc, e, ua);
    {
      Q2<T> c;
      lds_get(row, lane, c);
      add_volume(acc, c, p, bad);
    }
    if (LIM) {
      Q2<T> c;
      lds_get(row, lane, c);
      T mC[8];
      means_of(c, mC);
      limit_in_row(nb, mC, mN2, p);
    }
    {
      T Fm[8], Fp[8];
      {
        Q2<T> c;
        lds_get(row, lane, c);
        yface_point(c, nb, T(-1), p, Fm, bad);
      }
      add_point<T, 1>(acc, Fm, T(-1), T(-1), p);
      {
        Q2<T> c;
        lds_get(row, lane, c);
        yface_point(c, nb, T(1), p, Fp, bad);
      }
      add_point<T, 1>(acc, Fp, T(1), T(-1), p);
      ysums(Fm, Fp, carry);
    }
    Q2<T> d;
    finish(acc, p, d);
    if (MODE != kRhs) {
      Q2<T> c;
      lds_get(row, lane, c);
      if (MODE == kStage1 && LIM && p.lim_out && own) store_q(p.lim_out, nc, e, c);
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        d.m[v] = fma(dt, d.m[v], c.m[v]);
        d.g[v][0] = fma(dt, d.g[v][0], c.g[v][0]);
        d.g[v][1] = fma(dt, d.g[v][1], c.g[v][1]);
      }
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) d.b[cc] = fma(dt, d.b[cc], c.b[cc]);
#pragma unroll
      for (int j = 0; j < 5; ++j) d.a[j] = fma(dt, d.a[j], c.a[j]);
    }
    if (MODE == kStage2) {
      if (!kEarlyUa) load_q(p.ua, nc, e, ua);
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        d.m[v] = T(0.5) * (ua.m[v] + d.m[v]);
        d.g[v][0] = T(0.5) * (ua.g[v][0] + d.g[v][0]);
        d.g[v][1] = T(0.5) * (ua.g[v][1] + d.g[v][1]);
      }
#pragma unroll
      for (int c = 0; c < 3; ++c) d.b[c] = T(0.5) * (ua.b[c] + d.b[c]);
#pragma unroll
      for (int j = 0; j < 5; ++j) d.a[j] = T(0.5) * (ua.a[j] + d.a[j]);
    }
    if (own) {
      store_q(p.out, nc, e, d);
      if (MODE == kStage2 && p.dtpart) {
        const T mm[8] = {d.m[0], d.m[1], d.m[2], d.m[3], d.m[4], d.b[0], d.b[1], d.b[2]};
        dtmin = fmin(dtmin, cell_dt(mm, p));
      }
    }
    lds_put(row, lane, nb);
  }
  // every face is the -x or -y face of a cell owned by some wave, so the
  // owners' flags cover all quadrature points
  if (bad && own) atomicOr(p.status, 1);
  if (MODE == kStage2 && p.dtpart) {
    dtmin = wave_min(dtmin);
    if (lane == 0) p.dtpart[wave] = dtmin;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_cfl2m(P2M<T> p) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  double d = 1e300;
  if (e < p.nc) {
    T m[8];
    load_means(p.in, p.nc, e, m);
    d = cell_dt(m, p);
  }
  d = wave_min(d);
  if ((threadIdx.x & 63) == 0) p.dtpart[e >> 6] = d;
}

template <typename T>
P2M<T> make_params(const dg_mesh* m, const void* in, const void* ua, void* out,
                   const double* dt_dev, double dt_host) {
  P2M<T> p;
  p.in = static_cast<const T*>(in);
  p.ua = static_cast<const T*>(ua);
  p.out = static_cast<T*>(out);
  p.lim_out = nullptr;
  p.dt_dev = dt_dev;
  p.dt_host = dt_host;
  p.status = m->status;
  p.dtpart = nullptr;
  p.nx = m->c2.nx;
  p.ny = m->c2.ny;
  p.nc = (int)m->ncells;
  p.tiles_x = m->c2.tiles_x;
  p.width = (p.nx + p.tiles_x - 1) / p.tiles_x;
  p.rows = m->c2.rows_per_tile;
  p.tiles_y = m->c2.tiles_y;
  p.ntiles = p.tiles_x * p.tiles_y;
  p.gamma = (T)m->cfg.gamma;
  p.eps = (T)(m->cfg.precision == DG_FP64 ? 1e-12 : 1e-6);
  const double h[2] = {m->c2.hx, m->c2.hy};
  const double s3 = 1.7320508075688772;
  for (int d = 0; d < 2; ++d) {
    p.c2h[d] = (T)(0.5 / h[d]);
    p.c3[d] = (T)(3.0 / (h[d] * h[d]));
    p.pt[d] = (T)(h[1 - d] / (4.0 * s3 * h[d]));
    p.half[d] = (T)(0.5 * h[d]);
    p.q[d] = (T)(0.5 * h[d] / s3);
    p.ih[d] = 1.0 / h[d];
  }
  p.cs = (T)(s3 / (h[0] * h[1]));
  const double mx = h[0] * h[0] / 12.0, my = h[1] * h[1] / 12.0;
  p.imu[0] = (T)(1.0 / mx);
  p.imu[1] = (T)(1.0 / my);
  p.imu[2] = (T)(1.0 / (mx + my));
  return p;
}

template <typename T>
hipError_t lim_t(const dg_mesh* m, const void* in, void* out, hipStream_t s) {
  P2M<T> p = make_params<T>(m, in, nullptr, out, nullptr, 0.0);
  const unsigned nb = (unsigned)((m->ncells + 255) / 256);
  hipLaunchKernelGGL((k_lim2m<T>), dim3(nb), dim3(256), 0, s, p);
  return hipGetLastError();
}

// Stage kernel launch.  lim: limit `in` on read; lim_out: stage 1 also
// writes Pi(in) there.
template <typename T>
hipError_t rhs_t(const dg_mesh* m, int mode, bool lim, const void* in, const void* ua, void* out,
                 void* lim_out, const double* dt_dev, double dt_host, bool want_dt, hipStream_t s) {
  P2M<T> p = make_params<T>(m, in, ua, out, dt_dev, dt_host);
  if (want_dt) p.dtpart = m->dtpart;
  p.lim_out = static_cast<T*>(lim_out);
  const unsigned nb = (unsigned)p.ntiles;
  const dim3 g(nb), b(64);
  if (mode == kRhs && !lim)
    hipLaunchKernelGGL((k_mhd2d<T, kRhs, false>), g, b, 0, s, p);
  else if (mode == kStage1 && !lim)
    hipLaunchKernelGGL((k_mhd2d<T, kStage1, false>), g, b, 0, s, p);
  else if (mode == kStage1)
    hipLaunchKernelGGL((k_mhd2d<T, kStage1, true>), g, b, 0, s, p);
  else if (mode == kStage2 && !lim)
    hipLaunchKernelGGL((k_mhd2d<T, kStage2, false>), g, b, 0, s, p);
  else if (mode == kStage2)
    hipLaunchKernelGGL((k_mhd2d<T, kStage2, true>), g, b, 0, s, p);
  else
    return hipErrorInvalidValue;
  return hipGetLastError();
}

template <typename T>
hipError_t cfl_t(const dg_mesh* m, const void* U, hipStream_t s) {
  P2M<T> p = make_params<T>(m, U, nullptr, nullptr, nullptr, 0.0);
  p.dtpart = m->dtpart;
  const unsigned nb = (unsigned)((m->ncells + 255) / 256);
  hipLaunchKernelGGL((k_cfl2m<T>), dim3(nb), dim3(256), 0, s, p);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_min_finalize(const double* part, int n, double cfl, double* dt, hipStream_t s);

// Stage dispatch for 2D MHD.  The stage kernels limit their input on read;
// stage 1 also writes Pi(U) to ws_a, which a stage 2 on the same U reuses as
// its Pi(U^n) (any other stage 2 limits U^n into ws_a with a separate pass).
hipError_t launch_mhd2d(const dg_mesh* m, int mode, const void* in, const void* u0, void* out,
                        const double* dt_dev, double dt_host, double cfl, double* dt_next,
                        hipStream_t s) {
  const bool f64 = m->cfg.precision == DG_FP64;
  const bool lim = m->cfg.limiter == DG_LIMITER_MINMOD;
  auto limit = [&](const void* a, void* b) {
    return f64 ? lim_t<double>(m, a, b, s) : lim_t<float>(m, a, b, s);
  };
  auto rhs = [&](int md, bool l, const void* a, const void* ua, void* o, void* lo, bool want_dt) {
    return f64 ? rhs_t<double>(m, md, l, a, ua, o, lo, dt_dev, dt_host, want_dt, s)
               : rhs_t<float>(m, md, l, a, ua, o, lo, dt_dev, dt_host, want_dt, s);
  };
  hipError_t e = hipSuccess;
  switch (mode) {
    case kLimit:
      return limit(in, out);
    case kRhs:
      return rhs(kRhs, false, in, nullptr, out, nullptr, false);
    case kStage1:
      return rhs(kStage1, lim, in, nullptr, out, lim ? m->ws_a : nullptr, false);
    case kStage2: {
      // in = V1, u0 = U^n
      const void* ua = u0;
      if (lim) {
        if (!(m->ws_a_fresh && m->ws_a_src == u0)) e = limit(u0, m->ws_a);
        ua = m->ws_a;
      }
      if (e == hipSuccess) e = rhs(kStage2, lim, in, ua, out, nullptr, dt_next != nullptr);
      if (e == hipSuccess && dt_next)
        e = launch_min_finalize(m->dtpart, m->c2.tiles_x * m->c2.tiles_y, cfl, dt_next, s);
      return e;
    }
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_mhd2d_cfl(const dg_mesh* m, const void* U, double cfl, double* dt_dev,
                            hipStream_t s) {
  hipError_t e = m->cfg.precision == DG_FP64 ? cfl_t<double>(m, U, s) : cfl_t<float>(m, U, s);
  if (e != hipSuccess) return e;
  return launch_min_finalize(m->dtpart, (int)((m->ncells + 63) / 64), cfl, dt_dev, s);
}

}  // namespace dg
