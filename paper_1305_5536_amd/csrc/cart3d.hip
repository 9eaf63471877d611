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
//   k_lim3d  : Pi(U) -> out, four row-waves per workgroup marching in z, each
//              cell read once (memory bound).
//   k_rhs3d  : L(Ulim) combined into an SSP-RK2 stage.  A workgroup of four
//              row-waves owns a pencil of up to 62 x-columns (lanes 0 and 63
//              are halo columns) of four consecutive y-rows and marches
//              through a range of z-planes.  x-faces: each lane solves its -x
//              face and passes it left by shuffle.  z-faces: solved once per
//              plane pair, the upper plane's share carried in LDS.  y-faces:
//              solved once, by the upper row's wave, and handed to the wave
//              below through LDS; the group's top face is split by Gauss point
//              over the four waves.
//   k_cfl3d  : per-block minima of the CFL bound (fast magnetosonic speeds).
// The kernel is FP64/FP32 VALU-bound: 12 HLLD solves per cell and stage, 13
// per cell as executed (the top face of each group of rows is solved twice).
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

#include <algorithm>
#include <cstdint>

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
  int width, tiles_x, tiles_y, planes, tiles_z, ntiles;  // tiles_y: groups of kGW rows
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

// Element e of coefficient row k: the row's base is uniform across the wave
// and e enters as a 32-bit byte offset (ncells * 31 < 2^31 is checked at mesh
// creation, so 8 e < 2^32).
template <typename T>
__device__ __forceinline__ T ld_row(const T* __restrict__ U, int nc, int k, int e) {
  const char* row = reinterpret_cast<const char*>(U + (size_t)k * (size_t)nc);
  return *reinterpret_cast<const T*>(row + (uint32_t)e * (uint32_t)sizeof(T));
}
template <typename T>
__device__ __forceinline__ void st_row(T* __restrict__ U, int nc, int k, int e, T v) {
  char* row = reinterpret_cast<char*>(U + (size_t)k * (size_t)nc);
  *reinterpret_cast<T*>(row + (uint32_t)e * (uint32_t)sizeof(T)) = v;
}

template <typename T>
__device__ __forceinline__ void load_poly(const T* __restrict__ U, int nc, int e, Poly<T>& q) {
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    q.m[v] = ld_row(U, nc, 4 * v, e);
#pragma unroll
    for (int d = 0; d < 3; ++d) q.g[v][d] = ld_row(U, nc, 4 * v + 1 + d, e);
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) q.b[c] = ld_row(U, nc, 20 + c, e);
#pragma unroll
  for (int j = 0; j < 8; ++j) q.a[j] = ld_row(U, nc, 23 + j, e);
}

template <typename T>
__device__ __forceinline__ void store_poly(T* __restrict__ U, int nc, int e, const Poly<T>& q) {
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    st_row(U, nc, 4 * v, e, q.m[v]);
#pragma unroll
    for (int d = 0; d < 3; ++d) st_row(U, nc, 4 * v + 1 + d, e, q.g[v][d]);
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) st_row(U, nc, 20 + c, e, q.b[c]);
#pragma unroll
  for (int j = 0; j < 8; ++j) st_row(U, nc, 23 + j, e, q.a[j]);
}

// Conserved means in the order rho, mx, my, mz, E, Bx, By, Bz.
template <typename T>
__device__ __forceinline__ void load_means(const T* __restrict__ U, int nc, int e, T* m) {
#pragma unroll
  for (int v = 0; v < 5; ++v) m[v] = ld_row(U, nc, 4 * v, e);
#pragma unroll
  for (int c = 0; c < 3; ++c) m[5 + c] = ld_row(U, nc, 20 + c, e);
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
// Row-waves per workgroup of the stage kernel and of the limiter: kGW
// consecutive y-rows of one x-strip march through the same z-planes together.
constexpr int kGW = 4;

// Limits one cell (Sec. 2.5) from its bounds hi/lo over itself and its six
// face neighbours, in the order self, -x, +x, -y, +y, -z, +z.
template <typename T>
__device__ __forceinline__ void limit_cell3(Poly<T>& q, const T* hi, const T* lo,
                                            const P3<T>& p) {
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
}

template <typename T>
__device__ __forceinline__ void bound8(T* hi, T* lo, const T* mn) {
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    hi[k] = fmax(hi[k], mn[k]);
    lo[k] = fmin(lo[k], mn[k]);
  }
}

// Pi(U) -> out.  A workgroup of kGW row-waves owns a 64-column x-strip of kGW
// consecutive y-rows and marches through p.planes z-planes, so each cell's
// polynomial is read once: the x-neighbours' means come from the adjacent
// lane, the y-neighbours' from the adjacent row-wave through LDS, the
// z-neighbours' from the previous and the prefetched next plane in registers.
// Only strip and group edges (and periodic wraps) read neighbour means from
// memory.  Row-waves past the last row keep to the barriers only.
template <typename T>
__global__ __launch_bounds__(256) void k_lim3d(P3<T> p) {
  __shared__ T ml[kGW][8][64];
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int grp = xcd_remap(blockIdx.x, gridDim.x);
  if (grp >= p.ntiles) return;  // whole workgroup
  const int tx = grp % p.tiles_x;
  const int rest = grp / p.tiles_x;
  const int gy = rest % p.tiles_y;
  const int tz = rest / p.tiles_y;
  const int nx = p.nx, ny = p.ny, nz = p.nz, nc = p.nc;
  const int y0 = gy * kGW;
  const int top = min(kGW - 1, ny - 1 - y0);
  const bool real = w <= top;
  const int y = y0 + (real ? w : top);
  const int colu = tx * 64 + lane;
  const bool own = colu < nx;
  const int col = own ? colu : nx - 1;
  const int xm = col == 0 ? nx - 1 : col - 1;
  const int xp = col == nx - 1 ? 0 : col + 1;
  // neighbour in the adjacent lane of this wave (not across a periodic wrap)
  const bool xm_lane = lane > 0 && col > 0;
  const bool xp_lane = lane < 63 && col + 1 < nx;
  const int ym = y == 0 ? ny - 1 : y - 1;
  const int yp = y == ny - 1 ? 0 : y + 1;
  // neighbour row held by a row-wave of this group (its LDS slot)
  const int sm_ = ym >= y0 && ym <= y0 + top ? ym - y0 : -1;
  const int sp_ = yp >= y0 && yp <= y0 + top ? yp - y0 : -1;
  const int z0 = tz * p.planes;
  const int z1 = min(z0 + p.planes, nz);
  auto idx = [&](int xx, int yy, int zz) { return (zz * ny + yy) * nx + xx; };
  auto zw = [nz](int z) { return z < 0 ? z + nz : (z >= nz ? z - nz : z); };
  auto load_rest = [&](int e, Poly<T>& q) {
#pragma unroll
    for (int v = 0; v < 5; ++v)
#pragma unroll
      for (int d = 0; d < 3; ++d) q.g[v][d] = ld_row(p.in, nc, 4 * v + 1 + d, e);
#pragma unroll
    for (int j = 0; j < 8; ++j) q.a[j] = ld_row(p.in, nc, 23 + j, e);
  };

  // means of the planes below, at and above the current one (rho, m, E, B)
  T mprev[8], mc[8];
  if (real) {
    load_means(p.in, nc, idx(col, y, zw(z0 - 1)), mprev);
    load_means(p.in, nc, idx(col, y, z0), mc);
  }
  for (int z = z0; z < z1; ++z) {
    T mnx[8];
    Poly<T> q;
    if (real) {
      // the next plane's means and this cell's slopes, in flight across the
      // barriers
      load_means(p.in, nc, idx(col, y, zw(z + 1)), mnx);
      load_rest(idx(col, y, z), q);
    }
    __syncthreads();  // the previous plane's reads of ml are done
    if (real) {
#pragma unroll
      for (int k = 0; k < 8; ++k) ml[w][k][lane] = mc[k];
    }
    __syncthreads();
    if (real) {
      T hi[8], lo[8], mn[8];
#pragma unroll
      for (int k = 0; k < 8; ++k) hi[k] = lo[k] = mc[k];
#pragma unroll
      for (int k = 0; k < 8; ++k) mn[k] = lane_up(mc[k]);
      if (!xm_lane) load_means(p.in, nc, idx(xm, y, z), mn);
      bound8(hi, lo, mn);
#pragma unroll
      for (int k = 0; k < 8; ++k) mn[k] = lane_down(mc[k]);
      if (!xp_lane) load_means(p.in, nc, idx(xp, y, z), mn);
      bound8(hi, lo, mn);
      if (sm_ >= 0) {
#pragma unroll
        for (int k = 0; k < 8; ++k) mn[k] = ml[sm_][k][lane];
      } else {
        load_means(p.in, nc, idx(col, ym, z), mn);
      }
      bound8(hi, lo, mn);
      if (sp_ >= 0) {
#pragma unroll
        for (int k = 0; k < 8; ++k) mn[k] = ml[sp_][k][lane];
      } else {
        load_means(p.in, nc, idx(col, yp, z), mn);
      }
      bound8(hi, lo, mn);
      bound8(hi, lo, mprev);
      bound8(hi, lo, mnx);
#pragma unroll
      for (int v = 0; v < 5; ++v) q.m[v] = mc[v];
#pragma unroll
      for (int c = 0; c < 3; ++c) q.b[c] = mc[5 + c];
      limit_cell3(q, hi, lo, p);
      if (own) store_poly(p.out, nc, idx(col, y, z), q);
#pragma unroll
      for (int k = 0; k < 8; ++k) {
        mprev[k] = mc[k];
        mc[k] = mnx[k];
      }
    }
  }
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

// Volume term over the 2x2x2 Gauss points g0 .. g1-1 (of 8).
template <typename T>
__device__ __forceinline__ void add_volume(Acc<T>& a, const Poly<T>& q, const P3<T>& p,
                                           bool& bad, int g0 = 0, int g1 = 8) {
  const T gm1 = p.gamma - T(1);
#pragma unroll 1
  for (int g = g0; g < g1; ++g) {
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

// Face sums of axis D in 23 LDS rows: S without its normal-field entry (the
// normal flux of B_D, which no residual uses), then T1 and T2.
template <typename T, int D>
__device__ __forceinline__ void put_sums(T (*dst)[64], int lane, const FaceSums<T>& f) {
#pragma unroll
  for (int k = 0; k < 8; ++k)
    if (k != 5 + D) dst[k < 5 + D ? k : k - 1][lane] = f.S[k];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    dst[7 + k][lane] = f.T1[k];
    dst[15 + k][lane] = f.T2[k];
  }
}

template <typename T, int D>
__device__ __forceinline__ void get_sums(const T (*src)[64], int lane, FaceSums<T>& f) {
#pragma unroll
  for (int k = 0; k < 8; ++k) f.S[k] = k == 5 + D ? T(0) : src[k < 5 + D ? k : k - 1][lane];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    f.T1[k] = src[7 + k][lane];
    f.T2[k] = src[15 + k][lane];
  }
}

// HLLD flux at one Gauss point (tangential signs s1, s2) of a face of axis D,
// with the arithmetic of face() at that point.
template <typename T, int D>
__device__ __forceinline__ void face_point(const Poly<T>& L, const Poly<T>& R, T s1, T s2,
                                           const P3<T>& p, T* F, bool& bad) {
  T bL[8], iL1[8], iL2[8], bR[8], iR1[8], iR2[8];
  face_trace<T, D>(L, T(1), p, bL, iL1, iL2);
  face_trace<T, D>(R, T(-1), p, bR, iR1, iR2);
  T uL[8], uR[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) {
    uL[k] = fma(s2, iL2[k], fma(s1, iL1[k], bL[k]));
    uR[k] = fma(s2, iR2[k], fma(s1, iR1[k], bR[k]));
  }
  const T bn = T(0.5) * (uL[5 + D] + uR[5 + D]);
  uL[5 + D] = bn;
  uR[5 + D] = bn;
  hlld<T, D>(uL, uR, p, F, bad);
}

// LDS of one workgroup (FP64 162,304 B, FP32 81,152 B).
template <typename T>
struct Lds3 {
  T cur[kGW][kNC][64];      // each row-wave's current plane
  T carry[kGW][23][64];     // each row-wave's -z face sums, carried to the next plane
  T ysum[kGW - 1][23][64];  // -y face sums of row-waves 1.. for the row-wave below
  T xtra[kGW][8][64];       // row-wave w: flux at Gauss point w of the group's top +y face
};

// Stage kernel: a workgroup of kGW row-waves, row-wave w owning row y0 + w of
// an x-strip (62 interior lanes), all marching through the same z-planes.
// Per plane: x-faces by shuffle, the -z face carried from the previous plane,
// the -y face solved by the row-wave itself (the row below read from the
// neighbouring row-wave's LDS slot, from memory for w = 0) and handed to the
// row-wave below as its +y face; the group's top +y face is split by Gauss
// point over the kGW row-waves, so that each solves 13 HLLD problems per cell.
// Two barriers per plane; row-waves past the last row (ny not a multiple of
// kGW) keep to the barriers and their share of the top face only.  With one
// wave per SIMD nothing hides a load's latency but the wave's own work, so each
// load is issued well ahead of its use (stage 2 issues its Pi(U^n) row before
// the second barrier, which took the stage from 12.6 to 10.4 ms at 256^3).
template <typename T, int MODE>
__global__ __launch_bounds__(256) void k_rhs3d(P3<T> p) {
  __shared__ Lds3<T> sm;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane((int)(threadIdx.x >> 6));
  const int grp = xcd_remap(blockIdx.x, gridDim.x);
  if (grp >= p.ntiles) return;  // whole workgroup
  const int tx = grp % p.tiles_x;
  const int rest = grp / p.tiles_x;
  const int gy = rest % p.tiles_y;
  const int tz = rest / p.tiles_y;
  const int nx = p.nx, ny = p.ny, nz = p.nz, nc = p.nc;
  const int y0 = gy * kGW;
  const int top = min(kGW - 1, ny - 1 - y0);
  const bool real = w <= top;
  const int y = y0 + (real ? w : top);
  const int yS = y == 0 ? ny - 1 : y - 1;
  const int yT1 = y0 + top == ny - 1 ? 0 : y0 + top + 1;
  const int colu = tx * p.width + lane - 1;
  const bool own = lane >= 1 && lane <= p.width && colu < nx;
  int col = colu % nx;
  if (col < 0) col += nx;
  const int z0 = tz * p.planes;
  const int z1 = min(z0 + p.planes, nz);
  auto idx = [&](int yy, int zz) { return (zz * ny + yy) * nx + col; };
  auto zw = [nz](int z) { return z < 0 ? z + nz : (z >= nz ? z - nz : z); };
  bool bad = false;
  double dtmin = 1e300;
  const int left = lane == 0 ? 0 : lane - 1;
  // this row-wave's Gauss point of the top face (the order of face())
  const T gs1 = (w & 2) ? T(1) : T(-1);
  const T gs2 = (w & 1) ? T(1) : T(-1);

  if (real) {
    Poly<T> prv, cur;
    load_poly(p.in, nc, idx(y, zw(z0 - 1)), prv);
    load_poly(p.in, nc, idx(y, z0), cur);
    FaceSums<T> fz;
    face<T, 2>(prv, cur, p, fz, bad);
    put_sums<T, 2>(sm.carry[w], lane, fz);
    lds_put_poly(sm.cur[w], lane, cur);
  }
  T dt = T(0);
  if (MODE != kRhs) dt = (T)(p.dt_dev ? *p.dt_dev : p.dt_host);

  for (int z = z0; z < z1; ++z) {
    // every row-wave's plane z is in LDS; last plane's exchanges are consumed
    __syncthreads();
    Poly<T> nb;  // in flight: the row above the group, the row below (w = 0), plane z+1
    load_poly(p.in, nc, idx(yT1, z), nb);
    Acc<T> acc;
    zero(acc);
    Poly<T> ua;  // stage 2: Pi(U^n) of this row, loaded before the second barrier
    if (real) {
      FaceSums<T> fz;
      get_sums<T, 2>(sm.carry[w], lane, fz);
      add_face<T, 2>(acc, fz, T(1), p);
      // x-faces: this lane solves its -x face (left neighbour from LDS), the
      // +x face comes from lane+1 by shuffle
      Poly<T> l, c;
      lds_get_poly(sm.cur[w], left, l);
      lds_get_poly(sm.cur[w], lane, c);
      FaceSums<T> fx;
      face<T, 0>(l, c, p, fx, bad);
      add_face<T, 0>(acc, fx, T(1), p);
      shfl_down_sums(fx);
      add_face<T, 0>(acc, fx, T(-1), p);
    }
    {
      Poly<T> l;
      lds_get_poly(sm.cur[top], lane, l);
      T F[8];
      face_point<T, 1>(l, nb, gs1, gs2, p, F, bad);
#pragma unroll
      for (int k = 0; k < 8; ++k) sm.xtra[w][k][lane] = F[k];
    }
    if (real) {
      if (w == 0) load_poly(p.in, nc, idx(yS, z), nb);
      {
        // half the volume points cover the load of the row below (w = 0),
        // the other half, after the barrier, the load of plane z+1
        Poly<T> c;
        lds_get_poly(sm.cur[w], lane, c);
        add_volume(acc, c, p, bad, 0, 4);
      }
      if (w > 0) lds_get_poly(sm.cur[w - 1], lane, nb);
      Poly<T> c;
      lds_get_poly(sm.cur[w], lane, c);
      FaceSums<T> fy;
      face<T, 1>(nb, c, p, fy, bad);
      add_face<T, 1>(acc, fy, T(1), p);
      if (w > 0) put_sums<T, 1>(sm.ysum[w - 1], lane, fy);
      load_poly(p.in, nc, idx(y, zw(z + 1)), nb);
      if (MODE == kStage2) load_poly(p.ua, nc, idx(y, z), ua);
    }
    // the -y sums and the top face's Gauss-point fluxes are in LDS
    __syncthreads();
    if (!real) continue;
    {
      FaceSums<T> fy;
      if (w < top) {
        get_sums<T, 1>(sm.ysum[w], lane, fy);
      } else {
        // sum the four Gauss points in the order of face(), so that this face
        // matches bitwise the -y face the group above solves
#pragma unroll
        for (int k = 0; k < 8; ++k) fy.S[k] = fy.T1[k] = fy.T2[k] = T(0);
#pragma unroll
        for (int g = 0; g < 4; ++g) {
          const T s1 = (g & 2) ? T(1) : T(-1);
          const T s2 = (g & 1) ? T(1) : T(-1);
#pragma unroll
          for (int k = 0; k < 8; ++k) {
            const T F = sm.xtra[g][k][lane];
            fy.S[k] += F;
            fy.T1[k] = fma(s1, F, fy.T1[k]);
            fy.T2[k] = fma(s2, F, fy.T2[k]);
          }
        }
      }
      add_face<T, 1>(acc, fy, T(-1), p);
    }
    {
      Poly<T> c;
      lds_get_poly(sm.cur[w], lane, c);
      add_volume(acc, c, p, bad, 4, 8);
    }
    {
      Poly<T> c;
      lds_get_poly(sm.cur[w], lane, c);
      FaceSums<T> fz;
      face<T, 2>(c, nb, p, fz, bad);
      add_face<T, 2>(acc, fz, T(-1), p);
      put_sums<T, 2>(sm.carry[w], lane, fz);
    }
    Poly<T> d;
    finish(acc, p, d);
    {
      Poly<T> c;
      lds_get_poly(sm.cur[w], lane, c);
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
    // the next plane becomes current (the other row-waves read this slot only
    // before the barrier above)
    lds_put_poly(sm.cur[w], lane, nb);
  }
  if (bad && own) atomicOr(p.status, 1);
  if (MODE == kStage2 && p.dtpart) {
    dtmin = wave_min(dtmin);
    if (lane == 0) p.dtpart[grp * kGW + w] = dtmin;
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
  p.tiles_y = (p.ny + kGW - 1) / kGW;
  p.ntiles = p.tiles_x * p.tiles_y * p.tiles_z;
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
  // 64-column strips, groups of kGW rows, and a quarter of the stage kernel's
  // planes per workgroup (16 at 256^3: 16k row-waves, several rounds of
  // resident waves per SIMD for this memory-bound pass)
  p.width = 64;
  p.tiles_x = (p.nx + 63) / 64;
  p.planes = std::max(1, (m->c3.planes_per_tile + 3) / 4);
  p.tiles_z = (p.nz + p.planes - 1) / p.planes;
  p.ntiles = p.tiles_x * p.tiles_y * p.tiles_z;
  hipLaunchKernelGGL((k_lim3d<T>), dim3(p.ntiles), dim3(64 * kGW), 0, s, p);
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
      hipLaunchKernelGGL((k_rhs3d<T, kRhs>), dim3(nb), dim3(64 * kGW), 0, s, p);
      break;
    case kStage1:
      hipLaunchKernelGGL((k_rhs3d<T, kStage1>), dim3(nb), dim3(64 * kGW), 0, s, p);
      break;
    case kStage2:
      hipLaunchKernelGGL((k_rhs3d<T, kStage2>), dim3(nb), dim3(64 * kGW), 0, s, p);
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

// Row-waves of one stage launch (one partial CFL minimum each), for the
// mesh's tiling and for the finest one (one plane per row-wave).
int stage_waves3(const dg_mesh* m) {
  return m->c3.tiles_x * ((m->c3.ny + kGW - 1) / kGW) * kGW * m->c3.tiles_z;
}
// Workgroups of one z-range of the stage kernel (x-strips times groups of kGW
// rows), for a mesh of tiles_x strips and ny rows.
int64_t stage_groups3(int tiles_x, int ny) { return (int64_t)tiles_x * ((ny + kGW - 1) / kGW); }
int64_t max_stage_waves3(const dg_mesh* m) {
  return (int64_t)m->c3.tiles_x * ((m->c3.ny + kGW - 1) / kGW) * kGW * m->c3.nz;
}

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
        const int nt = stage_waves3(m);
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
