// DG stage kernels for 3D ideal MHD on a periodic Cartesian mesh (gfx950).
//
// Method (Sec. 2.2): P1 Taylor basis for rho, rho v, E (mean + gradient, 20
// coefficients) and the locally divergence-free basis V1..V11 for B (3 means +
// a4..a11); weak-form surface terms at 2x2 Gauss points per face with the HLLD
// flux of Miyoshi & Kusano (2005) (Sec. 2.3) and the face-averaged normal B of
// Sec. 2.6; volume terms at 2x2x2 Gauss points; inverse mass matrices (the
// box second moments for the Taylor gradients, the Gram matrix of V4..V11 for
// B); slope limiter of Sec. 2.5 with one alpha for the three B components.
//
// Kernels.
//   k_lim3d  : Pi(U) -> out, one thread per cell (memory bound).
//   k_rhs3d  : L(Ulim) combined into an SSP-RK2 stage.  One wave owns a pencil
//              of up to 62 x-columns (lanes 0 and 63 are halo columns) of one
//              y-row and marches through a range of z-planes.  x-faces: each
//              lane solves its -x face and passes it left by shuffle.
//              z-faces: solved once per plane pair; the upper plane's share is
//              carried in registers.  y-faces: solved by both adjacent rows
//              (bitwise-identical arithmetic), which keeps waves independent.
//   k_cfl3d  : per-block minima of the CFL bound (fast magnetosonic speeds).
// The kernel is FP64/FP32 VALU-bound: 12 HLLD solves per cell and stage.
//
// Residual algebra per face of axis D (tangential axes t1, t2), Gauss points
// at tangential signs (s1, s2), S = sum F, T1 = sum s1 F, T2 = sum s2 F, cell on
// side sigma (+1 when it is the R cell, -1 when L), all divided by the volume:
//   mean_k        += sigma S_k / (4 h_D)
//   grad_v[D]     -= 1.5 S_v / h_D^2
//   grad_v[t]     += sigma (sqrt3/2) T_v / (h_D h_t)
//   P[c][D]       -= S_Bc / 8,     P[c][t] += sigma h_t T_Bc / (8 sqrt3 h_D)
// volume (8 points): grad_v[e] += 1.5 F^e_v / h_e^2 (summed), P[c][e] += F^e(B_c)/8.
// The divergence-free coefficients follow from P: ra4 = P[x][y], ra5 = P[x][z],
// ra6 = P[y][x], ra7 = P[y][z], ra8 = P[z][x], ra9 = P[z][y],
// ra10 = P[x][x] - P[y][y], ra11 = P[x][x] - P[z][z], and a = (M_B/V)^-1 ra
// with M_B the Gram matrix of V4..V11 (diagonal plus a 2x2 block on a box).
#include <hip/hip_runtime.h>

#include "dg_internal.h"
#include "dg_math.h"
#include "mhd_hlld.h"

namespace dg {
namespace {

constexpr int kNC = 31;

template <typename T>
struct P3 {
  const T* __restrict__ in;   // limited state (RHS) or raw state (limiter)
  const T* __restrict__ ua;   // stage 2: Pi(U^n)
  T* __restrict__ out;
  const double* dt_dev;
  double dt_host;
  int* status;
  double* dtpart;
  int nx, ny, nz, nc;
  int width, tiles_x, planes, tiles_z, ntiles;
  T gamma, eps;
  T h[3];
  T c4h[3];    // 1/(4 h_d)
  T c15[3];    // 1.5/h_d^2
  T cs[3][3];  // (sqrt3/2)/(h_d h_t)
  T pt[3][3];  // h_t/(8 sqrt3 h_d)
  T half[3];   // h_d/2
  T q[3];      // h_d/(2 sqrt3)
  T mu[3];     // h_d^2/12
  T ib[4];     // inverse of [[mx+my, mx], [mx, mx+mz]] (row-major)
  double ih[3];
};

// Coefficients of one cell.  Hydro variable v = rho, mx, my, mz, E: mean m[v],
// gradient g[v][d]; B means b[c]; divergence-free coefficients a[0..7] = a4..a11.
template <typename T>
struct Poly {
  T m[5], g[5][3], b[3], a[8];
};

template <typename T>
__device__ __forceinline__ void load_poly(const T* __restrict__ U, int nc, int e, Poly<T>& q) {
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    q.m[v] = U[(4 * v) * nc + e];
#pragma unroll
    for (int d = 0; d < 3; ++d) q.g[v][d] = U[(4 * v + 1 + d) * nc + e];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) q.b[c] = U[(20 + c) * nc + e];
#pragma unroll
  for (int j = 0; j < 8; ++j) q.a[j] = U[(23 + j) * nc + e];
}

template <typename T>
__device__ __forceinline__ void store_poly(T* __restrict__ U, int nc, int e, const Poly<T>& q) {
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    U[(4 * v) * nc + e] = q.m[v];
#pragma unroll
    for (int d = 0; d < 3; ++d) U[(4 * v + 1 + d) * nc + e] = q.g[v][d];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) U[(20 + c) * nc + e] = q.b[c];
#pragma unroll
  for (int j = 0; j < 8; ++j) U[(23 + j) * nc + e] = q.a[j];
}

// Conserved means in the order rho, mx, my, mz, E, Bx, By, Bz.
template <typename T>
__device__ __forceinline__ void load_means(const T* __restrict__ U, int nc, int e, T* m) {
#pragma unroll
  for (int v = 0; v < 5; ++v) m[v] = U[(4 * v) * nc + e];
#pragma unroll
  for (int c = 0; c < 3; ++c) m[5 + c] = U[(20 + c) * nc + e];
}

// Gradient of B_c from the divergence-free coefficients:
//   grad Bx = (a10+a11, a4, a5), grad By = (a6, -a10, a7), grad Bz = (a8, a9, -a11).
template <typename T>
__device__ __forceinline__ T dB(const T* a, int c, int d) {
  if (c == 0) return d == 0 ? a[6] + a[7] : (d == 1 ? a[0] : a[1]);
  if (c == 1) return d == 0 ? a[2] : (d == 1 ? -a[6] : a[3]);
  return d == 0 ? a[4] : (d == 1 ? a[5] : -a[7]);
}

template <typename T>
__device__ __forceinline__ T alpha_of(T phi, T hi, T lo, const T* g, const P3<T>& p) {
  T D = fmin(hi - phi, phi - lo);
  T dm = fmax(fmax(fabs(g[0]) * p.half[0], fabs(g[1]) * p.half[1]), fabs(g[2]) * p.half[2]);
  return (dm > D) ? div_small(D, dm) : T(1);
}

// ------------------------------------------------------------- limiter --
template <typename T>
__global__ __launch_bounds__(256) void k_lim3d(P3<T> p) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= p.nc) return;
  const int nx = p.nx, ny = p.ny, nz = p.nz;
  const int i = e % nx, j = (e / nx) % ny, k = e / (nx * ny);
  const int nb[6] = {
      e - i + (i == 0 ? nx - 1 : i - 1), e - i + (i == nx - 1 ? 0 : i + 1),
      e + ((j == 0 ? ny - 1 : j - 1) - j) * nx, e + ((j == ny - 1 ? 0 : j + 1) - j) * nx,
      e + ((k == 0 ? nz - 1 : k - 1) - k) * nx * ny, e + ((k == nz - 1 ? 0 : k + 1) - k) * nx * ny};
  Poly<T> q;
  load_poly(p.in, p.nc, e, q);
  T hi[8], lo[8];
  hi[0] = lo[0] = q.m[0];
#pragma unroll
  for (int v = 0; v < 5; ++v) hi[v] = lo[v] = q.m[v];
#pragma unroll
  for (int c = 0; c < 3; ++c) hi[5 + c] = lo[5 + c] = q.b[c];
#pragma unroll
  for (int f = 0; f < 6; ++f) {
    T mn[8];
    load_means(p.in, p.nc, nb[f], mn);
#pragma unroll
    for (int k2 = 0; k2 < 8; ++k2) {
      hi[k2] = fmax(hi[k2], mn[k2]);
      lo[k2] = fmin(lo[k2], mn[k2]);
    }
  }
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    T a = alpha_of(q.m[v], hi[v], lo[v], q.g[v], p);
#pragma unroll
    for (int d = 0; d < 3; ++d) q.g[v][d] *= a;
  }
  T aB = T(1);
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    T gb[3] = {dB(q.a, c, 0), dB(q.a, c, 1), dB(q.a, c, 2)};
    aB = fmin(aB, alpha_of(q.b[c], hi[5 + c], lo[5 + c], gb, p));
  }
#pragma unroll
  for (int jj = 0; jj < 8; ++jj) q.a[jj] *= aB;
  store_poly(p.out, p.nc, e, q);
}

template <typename T, int D>
__device__ __forceinline__ void hlld(const T* uL, const T* uR, const P3<T>& p, T* F, bool& bad) {
  hlld_axis<T, D>(uL, uR, p.gamma, p.eps, F, bad);
}

// Per-side values of the cell polynomial on a face of axis D: the state at
// the face centre (normal offset +-h_D/2) and its increments along the two
// tangential Gauss offsets.
template <typename T, int D>
__device__ __forceinline__ void face_trace(const Poly<T>& q, T sgn_n, const P3<T>& p, T* base,
                                           T* inc1, T* inc2) {
  constexpr int t1 = (D + 1) % 3, t2 = (D + 2) % 3;
  const T hn = sgn_n * p.half[D];
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    base[v] = fma(q.g[v][D], hn, q.m[v]);
    inc1[v] = q.g[v][t1] * p.q[t1];
    inc2[v] = q.g[v][t2] * p.q[t2];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    base[5 + c] = fma(dB(q.a, c, D), hn, q.b[c]);
    inc1[5 + c] = dB(q.a, c, t1) * p.q[t1];
    inc2[5 + c] = dB(q.a, c, t2) * p.q[t2];
  }
}

// Sums over the 2x2 Gauss points of a face of axis D between L and R.
template <typename T>
struct FaceSums {
  T S[8], T1[8], T2[8];
};

template <typename T, int D>
__device__ __forceinline__ void face(const Poly<T>& L, const Poly<T>& R, const P3<T>& p,
                                     FaceSums<T>& fs, bool& bad) {
  T bL[8], iL1[8], iL2[8], bR[8], iR1[8], iR2[8];
  face_trace<T, D>(L, T(1), p, bL, iL1, iL2);
  face_trace<T, D>(R, T(-1), p, bR, iR1, iR2);
#pragma unroll
  for (int k = 0; k < 8; ++k) fs.S[k] = fs.T1[k] = fs.T2[k] = T(0);
#pragma unroll 1
  for (int g = 0; g < 4; ++g) {
    const T s1 = (g & 2) ? T(1) : T(-1);
    const T s2 = (g & 1) ? T(1) : T(-1);
    T uL[8], uR[8], F[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      uL[k] = fma(s2, iL2[k], fma(s1, iL1[k], bL[k]));
      uR[k] = fma(s2, iR2[k], fma(s1, iR1[k], bR[k]));
    }
    // one normal field for the Riemann problem: the average of both sides
    const T bn = T(0.5) * (uL[5 + D] + uR[5 + D]);
    uL[5 + D] = bn;
    uR[5 + D] = bn;
    hlld<T, D>(uL, uR, p, F, bad);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      fs.S[k] += F[k];
      fs.T1[k] = fma(s1, F[k], fs.T1[k]);
      fs.T2[k] = fma(s2, F[k], fs.T2[k]);
    }
  }
}

template <typename T>
struct Acc {
  T m[8], g[5][3], P[3][3];
};

template <typename T>
__device__ __forceinline__ void zero(Acc<T>& a) {
#pragma unroll
  for (int k = 0; k < 8; ++k) a.m[k] = T(0);
#pragma unroll
  for (int v = 0; v < 5; ++v)
#pragma unroll
    for (int d = 0; d < 3; ++d) a.g[v][d] = T(0);
#pragma unroll
  for (int c = 0; c < 3; ++c)
#pragma unroll
    for (int d = 0; d < 3; ++d) a.P[c][d] = T(0);
}

// Add one face's sums to a cell: sigma = +1 if the cell is the R cell of the
// face (its -D face), -1 if it is the L cell (its +D face).
template <typename T, int D>
__device__ __forceinline__ void add_face(Acc<T>& a, const FaceSums<T>& f, T sigma,
                                         const P3<T>& p) {
  constexpr int t1 = (D + 1) % 3, t2 = (D + 2) % 3;
#pragma unroll
  for (int k = 0; k < 8; ++k)
    if (k != 5 + D) a.m[k] = fma(sigma * p.c4h[D], f.S[k], a.m[k]);
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    a.g[v][D] = fma(-p.c15[D], f.S[v], a.g[v][D]);
    a.g[v][t1] = fma(sigma * p.cs[D][t1], f.T1[v], a.g[v][t1]);
    a.g[v][t2] = fma(sigma * p.cs[D][t2], f.T2[v], a.g[v][t2]);
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (c != D) a.P[c][D] = fma(T(-0.125), f.S[5 + c], a.P[c][D]);
    a.P[c][t1] = fma(sigma * p.pt[D][t1], f.T1[5 + c], a.P[c][t1]);
    a.P[c][t2] = fma(sigma * p.pt[D][t2], f.T2[5 + c], a.P[c][t2]);
  }
}

// Volume term over the 2x2x2 Gauss points.
template <typename T>
__device__ __forceinline__ void add_volume(Acc<T>& a, const Poly<T>& q, const P3<T>& p,
                                           bool& bad) {
  const T gm1 = p.gamma - T(1);
#pragma unroll 1
  for (int g = 0; g < 8; ++g) {
    const T o[3] = {(g & 4) ? p.q[0] : -p.q[0], (g & 2) ? p.q[1] : -p.q[1],
                    (g & 1) ? p.q[2] : -p.q[2]};
    T u[5], B[3];
#pragma unroll
    for (int v = 0; v < 5; ++v)
      u[v] = fma(q.g[v][0], o[0], fma(q.g[v][1], o[1], fma(q.g[v][2], o[2], q.m[v])));
#pragma unroll
    for (int c = 0; c < 3; ++c)
      B[c] = fma(dB(q.a, c, 0), o[0], fma(dB(q.a, c, 1), o[1], fma(dB(q.a, c, 2), o[2], q.b[c])));
    const T ir = rcp(u[0]);
    const T vel[3] = {u[1] * ir, u[2] * ir, u[3] * ir};
    const T pm = T(0.5) * (B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
    const T pg = gm1 * (u[4] - T(0.5) * (u[1] * vel[0] + u[2] * vel[1] + u[3] * vel[2]) - pm);
    bad |= !(u[0] > T(0)) || !(pg > T(0));
    const T pT = pg + pm;
    const T vB = vel[0] * B[0] + vel[1] * B[1] + vel[2] * B[2];
#pragma unroll
    for (int e = 0; e < 3; ++e) {
      // flux along e of rho, m, E
      T fe[5];
      fe[0] = u[1 + e];
#pragma unroll
      for (int k = 0; k < 3; ++k) fe[1 + k] = u[1 + k] * vel[e] - B[k] * B[e] + (k == e ? pT : T(0));
      fe[4] = (u[4] + pT) * vel[e] - B[e] * vB;
#pragma unroll
      for (int v = 0; v < 5; ++v) a.g[v][e] = fma(p.c15[e], fe[v], a.g[v][e]);
    }
    // induction fluxes F_e(B_c) = B_c v_e - v_c B_e (antisymmetric in c, e)
    const T fyx = B[0] * vel[1] - vel[0] * B[1];  // F_y(Bx)
    const T fzx = B[0] * vel[2] - vel[0] * B[2];  // F_z(Bx)
    const T fzy = B[1] * vel[2] - vel[1] * B[2];  // F_z(By)
    a.P[0][1] = fma(T(0.125), fyx, a.P[0][1]);
    a.P[1][0] = fma(T(-0.125), fyx, a.P[1][0]);
    a.P[0][2] = fma(T(0.125), fzx, a.P[0][2]);
    a.P[2][0] = fma(T(-0.125), fzx, a.P[2][0]);
    a.P[1][2] = fma(T(0.125), fzy, a.P[1][2]);
    a.P[2][1] = fma(T(-0.125), fzy, a.P[2][1]);
  }
}

// Time derivative of the coefficients from the accumulated residuals.
template <typename T>
__device__ __forceinline__ void finish(const Acc<T>& a, const P3<T>& p, Poly<T>& d) {
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    d.m[v] = a.m[v];
#pragma unroll
    for (int e = 0; e < 3; ++e) d.g[v][e] = a.g[v][e];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) d.b[c] = a.m[5 + c];
  d.a[0] = a.P[0][1] / p.mu[1];
  d.a[1] = a.P[0][2] / p.mu[2];
  d.a[2] = a.P[1][0] / p.mu[0];
  d.a[3] = a.P[1][2] / p.mu[2];
  d.a[4] = a.P[2][0] / p.mu[0];
  d.a[5] = a.P[2][1] / p.mu[1];
  const T r10 = a.P[0][0] - a.P[1][1], r11 = a.P[0][0] - a.P[2][2];
  d.a[6] = p.ib[0] * r10 + p.ib[1] * r11;
  d.a[7] = p.ib[2] * r10 + p.ib[3] * r11;
}

template <typename T>
__device__ __forceinline__ void shfl_up_poly(const Poly<T>& q, Poly<T>& o) {
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    o.m[v] = lane_up(q.m[v]);
#pragma unroll
    for (int d = 0; d < 3; ++d) o.g[v][d] = lane_up(q.g[v][d]);
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) o.b[c] = lane_up(q.b[c]);
#pragma unroll
  for (int j = 0; j < 8; ++j) o.a[j] = lane_up(q.a[j]);
}

template <typename T>
__device__ __forceinline__ void shfl_down_sums(FaceSums<T>& f) {
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    f.S[k] = lane_down(f.S[k]);
    f.T1[k] = lane_down(f.T1[k]);
    f.T2[k] = lane_down(f.T2[k]);
  }
}

// CFL bound of a cell from its means: 1 / sum_d (|v_d| + c_f,d)/h_d.
template <typename T>
__device__ __forceinline__ double cell_dt3(const T* m, const P3<T>& p) {
  const double r = m[0], ir = 1.0 / r;
  const double v[3] = {m[1] * ir, m[2] * ir, m[3] * ir};
  const double B[3] = {m[5], m[6], m[7]};
  const double B2 = B[0] * B[0] + B[1] * B[1] + B[2] * B[2];
  const double pg = ((double)p.gamma - 1.0) *
                    (m[4] - 0.5 * r * (v[0] * v[0] + v[1] * v[1] + v[2] * v[2]) - 0.5 * B2);
  const double a2 = (double)p.gamma * pg * ir;
  const double sb = a2 + B2 * ir;
  double s = 0.0;
  for (int d = 0; d < 3; ++d) {
    double disc = fmax(sb * sb - 4.0 * a2 * B[d] * B[d] * ir, 0.0);
    double cf = sqrt(0.5 * (sb + sqrt(disc)));
    s += (fabs(v[d]) + cf) * p.ih[d];
  }
  return 1.0 / s;
}

// Per-wave LDS: the current plane's polynomial of every lane and the -z face
// sums carried from the previous plane.
template <typename T>
struct Lds3 {
  T cur[kNC][64];
  T carry[24][64];
};

template <typename T>
__device__ __forceinline__ void lds_put_poly(T (*dst)[64], int lane, const Poly<T>& q) {
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    dst[4 * v][lane] = q.m[v];
#pragma unroll
    for (int d = 0; d < 3; ++d) dst[4 * v + 1 + d][lane] = q.g[v][d];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) dst[20 + c][lane] = q.b[c];
#pragma unroll
  for (int j = 0; j < 8; ++j) dst[23 + j][lane] = q.a[j];
}

template <typename T>
__device__ __forceinline__ void lds_get_poly(const T (*src)[64], int lane, Poly<T>& q) {
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    q.m[v] = src[4 * v][lane];
#pragma unroll
    for (int d = 0; d < 3; ++d) q.g[v][d] = src[4 * v + 1 + d][lane];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) q.b[c] = src[20 + c][lane];
#pragma unroll
  for (int j = 0; j < 8; ++j) q.a[j] = src[23 + j][lane];
}

// Face of axis D whose contributions go only to one cell (sigma as in
// add_face): each Gauss point is accumulated straight into the cell's
// residual, so no per-face sums stay live.
template <typename T, int D>
__device__ __forceinline__ void face_into(const Poly<T>& L, const Poly<T>& R, T sigma,
                                          const P3<T>& p, Acc<T>& acc, bool& bad) {
  constexpr int t1 = (D + 1) % 3, t2 = (D + 2) % 3;
  T bL[8], iL1[8], iL2[8], bR[8], iR1[8], iR2[8];
  face_trace<T, D>(L, T(1), p, bL, iL1, iL2);
  face_trace<T, D>(R, T(-1), p, bR, iR1, iR2);
  const T cm = sigma * p.c4h[D];
  const T c1 = sigma * p.cs[D][t1], c2 = sigma * p.cs[D][t2];
  const T p1 = sigma * p.pt[D][t1], p2 = sigma * p.pt[D][t2];
#pragma unroll 1
  for (int g = 0; g < 4; ++g) {
    const T s1 = (g & 2) ? T(1) : T(-1);
    const T s2 = (g & 1) ? T(1) : T(-1);
    T uL[8], uR[8], F[8];
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      uL[k] = fma(s2, iL2[k], fma(s1, iL1[k], bL[k]));
      uR[k] = fma(s2, iR2[k], fma(s1, iR1[k], bR[k]));
    }
    const T bn = T(0.5) * (uL[5 + D] + uR[5 + D]);
    uL[5 + D] = bn;
    uR[5 + D] = bn;
    hlld<T, D>(uL, uR, p, F, bad);
#pragma unroll
    for (int k = 0; k < 8; ++k)
      if (k != 5 + D) acc.m[k] = fma(cm, F[k], acc.m[k]);
#pragma unroll
    for (int v = 0; v < 5; ++v) {
      acc.g[v][D] = fma(-p.c15[D], F[v], acc.g[v][D]);
      acc.g[v][t1] = fma(s1 * c1, F[v], acc.g[v][t1]);
      acc.g[v][t2] = fma(s2 * c2, F[v], acc.g[v][t2]);
    }
#pragma unroll
    for (int c = 0; c < 3; ++c) {
      if (c != D) acc.P[c][D] = fma(T(-0.125), F[5 + c], acc.P[c][D]);
      acc.P[c][t1] = fma(s1 * p1, F[5 + c], acc.P[c][t1]);
      acc.P[c][t2] = fma(s2 * p2, F[5 + c], acc.P[c][t2]);
    }
  }
}

template <typename T, int MODE>
__global__ __launch_bounds__(64) void k_rhs3d(P3<T> p) {
  __shared__ Lds3<T> sm;
  const int lane = threadIdx.x;
  const int wave = xcd_remap(blockIdx.x, gridDim.x);
  if (wave >= p.ntiles) return;
  const int tx = wave % p.tiles_x;
  const int rest = wave / p.tiles_x;
  const int y = rest % p.ny;
  const int tz = rest / p.ny;
  const int nx = p.nx, ny = p.ny, nz = p.nz, nc = p.nc;
  const int colu = tx * p.width + lane - 1;
  const bool own = lane >= 1 && lane <= p.width && colu < nx;
  int col = colu % nx;
  if (col < 0) col += nx;
  const int yS = y == 0 ? ny - 1 : y - 1;
  const int yN = y == ny - 1 ? 0 : y + 1;
  const int z0 = tz * p.planes;
  const int z1 = min(z0 + p.planes, nz);
  auto idx = [&](int yy, int zz) { return (zz * ny + yy) * nx + col; };
  auto zw = [nz](int z) { return z < 0 ? z + nz : (z >= nz ? z - nz : z); };
  bool bad = false;
  double dtmin = 1e300;
  const int left = lane == 0 ? 0 : lane - 1;

  {
    Poly<T> prv, cur;
    load_poly(p.in, nc, idx(y, zw(z0 - 1)), prv);
    load_poly(p.in, nc, idx(y, z0), cur);
    FaceSums<T> fz;
    face<T, 2>(prv, cur, p, fz, bad);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      sm.carry[k][lane] = fz.S[k];
      sm.carry[8 + k][lane] = fz.T1[k];
      sm.carry[16 + k][lane] = fz.T2[k];
    }
    lds_put_poly(sm.cur, lane, cur);
  }
  T dt = T(0);
  if (MODE != kRhs) dt = (T)(p.dt_dev ? *p.dt_dev : p.dt_host);

  for (int z = z0; z < z1; ++z) {
    Poly<T> nb;  // neighbour polynomial in flight: y-1, then y+1, then z+1
    Acc<T> acc;
    zero(acc);
    {
      FaceSums<T> fz;
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        fz.S[k] = sm.carry[k][lane];
        fz.T1[k] = sm.carry[8 + k][lane];
        fz.T2[k] = sm.carry[16 + k][lane];
      }
      add_face<T, 2>(acc, fz, T(1), p);
    }
    {
      // x-faces: this lane solves its -x face (left neighbour from LDS), the
      // +x face comes from lane+1 by shuffle
      Poly<T> l, c;
      lds_get_poly(sm.cur, left, l);
      lds_get_poly(sm.cur, lane, c);
      FaceSums<T> fx;
      face<T, 0>(l, c, p, fx, bad);
      add_face<T, 0>(acc, fx, T(1), p);
      shfl_down_sums(fx);
      add_face<T, 0>(acc, fx, T(-1), p);
    }
    load_poly(p.in, nc, idx(yS, z), nb);
    {
      Poly<T> c;
      lds_get_poly(sm.cur, lane, c);
      add_volume(acc, c, p, bad);
    }
    {
      Poly<T> c;
      lds_get_poly(sm.cur, lane, c);
      face_into<T, 1>(nb, c, T(1), p, acc, bad);
    }
    load_poly(p.in, nc, idx(yN, z), nb);
    {
      Poly<T> c;
      lds_get_poly(sm.cur, lane, c);
      face_into<T, 1>(c, nb, T(-1), p, acc, bad);
    }
    load_poly(p.in, nc, idx(y, zw(z + 1)), nb);
    {
      Poly<T> c;
      lds_get_poly(sm.cur, lane, c);
      FaceSums<T> fz;
      face<T, 2>(c, nb, p, fz, bad);
      add_face<T, 2>(acc, fz, T(-1), p);
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        sm.carry[k][lane] = fz.S[k];
        sm.carry[8 + k][lane] = fz.T1[k];
        sm.carry[16 + k][lane] = fz.T2[k];
      }
    }
    Poly<T> d;
    finish(acc, p, d);
    {
      Poly<T> c;
      lds_get_poly(sm.cur, lane, c);
      if (MODE != kRhs) {
#pragma unroll
        for (int v = 0; v < 5; ++v) {
          d.m[v] = fma(dt, d.m[v], c.m[v]);
#pragma unroll
          for (int e = 0; e < 3; ++e) d.g[v][e] = fma(dt, d.g[v][e], c.g[v][e]);
        }
#pragma unroll
        for (int cc = 0; cc < 3; ++cc) d.b[cc] = fma(dt, d.b[cc], c.b[cc]);
#pragma unroll
        for (int j = 0; j < 8; ++j) d.a[j] = fma(dt, d.a[j], c.a[j]);
      }
    }
    if (MODE == kStage2) {
      Poly<T> ua;
      load_poly(p.ua, nc, idx(y, z), ua);
#pragma unroll
      for (int v = 0; v < 5; ++v) {
        d.m[v] = T(0.5) * (ua.m[v] + d.m[v]);
#pragma unroll
        for (int e = 0; e < 3; ++e) d.g[v][e] = T(0.5) * (ua.g[v][e] + d.g[v][e]);
      }
#pragma unroll
      for (int cc = 0; cc < 3; ++cc) d.b[cc] = T(0.5) * (ua.b[cc] + d.b[cc]);
#pragma unroll
      for (int j = 0; j < 8; ++j) d.a[j] = T(0.5) * (ua.a[j] + d.a[j]);
    }
    if (own) {
      store_poly(p.out, nc, idx(y, z), d);
      if (MODE == kStage2 && p.dtpart) {
        T mm[8] = {d.m[0], d.m[1], d.m[2], d.m[3], d.m[4], d.b[0], d.b[1], d.b[2]};
        dtmin = fmin(dtmin, cell_dt3(mm, p));
      }
    }
    // the next plane becomes current (all lanes of the wave finished reading
    // their neighbours' slots above: LDS operations of one wave run in order)
    lds_put_poly(sm.cur, lane, nb);
  }
  if (bad && own) atomicOr(p.status, 1);
  if (MODE == kStage2 && p.dtpart) {
    dtmin = wave_min(dtmin);
    if (lane == 0) p.dtpart[wave] = dtmin;
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_cfl3d(P3<T> p) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  double d = 1e300;
  if (e < p.nc) {
    T m[8];
    load_means(p.in, p.nc, e, m);
    d = cell_dt3(m, p);
  }
  d = wave_min(d);
  if ((threadIdx.x & 63) == 0) p.dtpart[e >> 6] = d;
}

template <typename T>
P3<T> make_params(const dg_mesh* m, const void* in, const void* ua, void* out,
                  const double* dt_dev, double dt_host) {
  P3<T> p;
  p.in = static_cast<const T*>(in);
  p.ua = static_cast<const T*>(ua);
  p.out = static_cast<T*>(out);
  p.dt_dev = dt_dev;
  p.dt_host = dt_host;
  p.status = m->status;
  p.dtpart = nullptr;
  p.nx = m->c3.nx;
  p.ny = m->c3.ny;
  p.nz = m->c3.nz;
  p.nc = (int)m->ncells;
  p.tiles_x = m->c3.tiles_x;
  p.width = (p.nx + p.tiles_x - 1) / p.tiles_x;
  p.planes = m->c3.planes_per_tile;
  p.tiles_z = m->c3.tiles_z;
  p.ntiles = p.tiles_x * p.ny * p.tiles_z;
  p.gamma = (T)m->cfg.gamma;
  p.eps = (T)(m->cfg.precision == DG_FP64 ? 1e-12 : 1e-6);
  const double h[3] = {m->c3.hx, m->c3.hy, m->c3.hz};
  const double s3 = 1.7320508075688772;
  for (int d = 0; d < 3; ++d) {
    p.h[d] = (T)h[d];
    p.c4h[d] = (T)(0.25 / h[d]);
    p.c15[d] = (T)(1.5 / (h[d] * h[d]));
    p.half[d] = (T)(0.5 * h[d]);
    p.q[d] = (T)(0.5 * h[d] / s3);
    p.mu[d] = (T)(h[d] * h[d] / 12.0);
    p.ih[d] = 1.0 / h[d];
    for (int t = 0; t < 3; ++t) {
      p.cs[d][t] = (T)(0.5 * s3 / (h[d] * h[t]));
      p.pt[d][t] = (T)(h[t] / (8.0 * s3 * h[d]));
    }
  }
  const double mx = h[0] * h[0] / 12.0, my = h[1] * h[1] / 12.0, mz = h[2] * h[2] / 12.0;
  const double det = (mx + my) * (mx + mz) - mx * mx;
  p.ib[0] = (T)((mx + mz) / det);
  p.ib[1] = (T)(-mx / det);
  p.ib[2] = (T)(-mx / det);
  p.ib[3] = (T)((mx + my) / det);
  return p;
}

template <typename T>
hipError_t lim_t(const dg_mesh* m, const void* in, void* out, hipStream_t s) {
  P3<T> p = make_params<T>(m, in, nullptr, out, nullptr, 0.0);
  const unsigned nb = (unsigned)((m->ncells + 255) / 256);
  hipLaunchKernelGGL((k_lim3d<T>), dim3(nb), dim3(256), 0, s, p);
  return hipGetLastError();
}

template <typename T>
hipError_t rhs_t(const dg_mesh* m, int mode, const void* in, const void* ua, void* out,
                 const double* dt_dev, double dt_host, bool want_dt, hipStream_t s) {
  P3<T> p = make_params<T>(m, in, ua, out, dt_dev, dt_host);
  if (want_dt) p.dtpart = m->dtpart;
  const unsigned nb = (unsigned)p.ntiles;
  switch (mode) {
    case kRhs:
      hipLaunchKernelGGL((k_rhs3d<T, kRhs>), dim3(nb), dim3(64), 0, s, p);
      break;
    case kStage1:
      hipLaunchKernelGGL((k_rhs3d<T, kStage1>), dim3(nb), dim3(64), 0, s, p);
      break;
    case kStage2:
      hipLaunchKernelGGL((k_rhs3d<T, kStage2>), dim3(nb), dim3(64), 0, s, p);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t cfl_t(const dg_mesh* m, const void* U, hipStream_t s) {
  P3<T> p = make_params<T>(m, U, nullptr, nullptr, nullptr, 0.0);
  p.dtpart = m->dtpart;
  const unsigned nb = (unsigned)((m->ncells + 255) / 256);
  hipLaunchKernelGGL((k_cfl3d<T>), dim3(nb), dim3(256), 0, s, p);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_min_finalize(const double* part, int n, double cfl, double* dt, hipStream_t s);

// Stage dispatch for 3D MHD.  The limiter runs as its own pass into the
// workspace (ws_a holds Pi(U) of stage 1 for the stage-2 combination, ws_b
// holds Pi(V1)).
hipError_t launch_cart3d(const dg_mesh* m, int mode, const void* in, const void* u0, void* out,
                         const double* dt_dev, double dt_host, double cfl, double* dt_next,
                         hipStream_t s) {
  const bool f64 = m->cfg.precision == DG_FP64;
  const bool lim = m->cfg.limiter == DG_LIMITER_MINMOD;
  auto limit = [&](const void* a, void* b) {
    return f64 ? lim_t<double>(m, a, b, s) : lim_t<float>(m, a, b, s);
  };
  auto rhs = [&](int md, const void* a, const void* ua, void* o, bool want_dt) {
    return f64 ? rhs_t<double>(m, md, a, ua, o, dt_dev, dt_host, want_dt, s)
               : rhs_t<float>(m, md, a, ua, o, dt_dev, dt_host, want_dt, s);
  };
  hipError_t e = hipSuccess;
  switch (mode) {
    case kLimit:
      return limit(in, out);
    case kRhs:
      return rhs(kRhs, in, nullptr, out, false);
    case kStage1: {
      const void* a = in;
      if (lim) {
        e = limit(in, m->ws_a);
        a = m->ws_a;
      }
      if (e == hipSuccess) e = rhs(kStage1, a, nullptr, out, false);
      return e;
    }
    case kStage2: {
      // in = V1, u0 = U^n
      const void* ua = u0;
      const void* b = in;
      if (lim) {
        if (!(m->ws_a_fresh && m->ws_a_src == u0)) e = limit(u0, m->ws_a);
        ua = m->ws_a;
        if (e == hipSuccess) e = limit(in, m->ws_b);
        b = m->ws_b;
      }
      if (e == hipSuccess) e = rhs(kStage2, b, ua, out, dt_next != nullptr);
      if (e == hipSuccess && dt_next) {
        const int nt = m->c3.tiles_x * m->c3.ny * m->c3.tiles_z;
        e = launch_min_finalize(m->dtpart, nt, cfl, dt_next, s);
      }
      return e;
    }
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_cart3d_cfl(const dg_mesh* m, const void* U, double cfl, double* dt_dev,
                             hipStream_t s) {
  hipError_t e = m->cfg.precision == DG_FP64 ? cfl_t<double>(m, U, s) : cfl_t<float>(m, U, s);
  if (e != hipSuccess) return e;
  return launch_min_finalize(m->dtpart, (int)((m->ncells + 63) / 64), cfl, dt_dev, s);
}

}  // namespace dg
