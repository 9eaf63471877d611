// Discrete adjoint of the 3D ideal-MHD Cartesian SSP-RK2 step: the HLLD flux of
// Sec. 2.3 at 2x2 Gauss points per face on the face-averaged normal field, the
// locally divergence-free field basis V1..V11 of Sec. 2.2 and the limiter of
// Sec. 2.5 with one alpha for B; dt frozen, the branch the forward step takes,
// ties to the first argument of min and max in the order self, -x, +x, -y,
// +y, -z, +z (the CPU oracle's dual-number conventions).
//
// The same two adjoint stages as in two dimensions (stage 2: P = V1,
// lam = lam', c_id = 1/2, c_L = dt/2; stage 1: P = U, lam = lam_V1, c_id = 1,
// c_L = dt, extra = lam' with weight 1/2), each the forward limiter (k_lim3d)
// into a workspace and two gathers, one thread per cell, no atomics:
//   k_adj3m_L    lamW of a cell from its six faces (four Gauss points each)
//                and its eight volume points; flux cotangents from the
//                transposed residual weights of both adjacent cells, the HLLD
//                Jacobian on this cell's side by forward-mode dual numbers
//                (eight directions), the Gauss-point extrapolation and the map
//                from residual moments to a4..a11 transposed by hand;
//   k_adj3m_lim  the limiter transpose: the cell's own limiter in its 31
//                coefficients and the part each neighbour's limiter takes from
//                this cell's means, by dual numbers.
// Correct first, not tuned: 192 dual HLLD solves per cell and adjoint stage
// (each face from both sides) against 12 HLLD solves per cell in a forward
// stage.
#include <hip/hip_runtime.h>

#include "dg_internal.h"
#include "dg_math.h"
#include "dual.h"
#include "mhd_hlld.h"

namespace dg {

hipError_t launch_cart3d(const dg_mesh* m, int mode, const void* in, const void* u0, void* out,
                         const double* dt_dev, double dt_host, double cfl, double* dt_next,
                         hipStream_t s);

namespace {

constexpr int kNC3 = 31;

// Coefficient layout (31 values): 4v the mean and 4v+1+d the gradient along d
// of rho, mx, my, mz, E (v = 0..4); 20..22 the means of Bx, By, Bz; 23..30
// a4..a11.  Mean index of conserved variable k (rho .. E, Bx, By, Bz).
__device__ __forceinline__ int mean3(int k) { return k < 5 ? 4 * k : 15 + k; }

// The gradient of B_c along d in a4..a11 (offsets 0..7):
//   grad Bx = (a10 + a11, a4, a5), grad By = (a6, -a10, a7), grad Bz = (a8, a9, -a11).
template <typename S>
__device__ __forceinline__ S dB3(const S* a, int c, int d) {
  if (c == 0) return d == 0 ? a[6] + a[7] : (d == 1 ? a[0] : a[1]);
  if (c == 1) return d == 0 ? a[2] : (d == 1 ? -a[6] : a[3]);
  return d == 0 ? a[4] : (d == 1 ? a[5] : -a[7]);
}

// Transpose of dB3: adds w times d(dB3(a, c, d))/da to abar.
template <typename T>
__device__ __forceinline__ void dB3_bar(int c, int d, T w, T* abar) {
  if (c == 0) {
    if (d == 0) {
      abar[6] += w;
      abar[7] += w;
    } else {
      abar[d == 1 ? 0 : 1] += w;
    }
  } else if (c == 1) {
    if (d == 1)
      abar[6] -= w;
    else
      abar[d == 0 ? 2 : 3] += w;
  } else {
    if (d == 2)
      abar[7] -= w;
    else
      abar[d == 0 ? 4 : 5] += w;
  }
}

template <typename T>
struct PJ3 {
  const T* W;
  const T* P;
  const T* lam;
  const T* extra;
  const T* lamW;
  T* out;
  const double* dt_dev;
  double dt_host;
  double c_id, c_L_over_dt, c_extra;
  int nx, ny, nz, nc;
  T gamma, eps;
  T c4h[3], c15[3], cs[3][3], pt[3][3], half[3], q[3], imu[3], ib[4];
};

template <typename T>
__device__ __forceinline__ void load31(const T* __restrict__ U, int nc, int e, T* c) {
#pragma unroll
  for (int k = 0; k < kNC3; ++k) c[k] = U[(size_t)k * nc + e];
}

// Face neighbours -x, +x, -y, +y, -z, +z of cell e (periodic).
__device__ __forceinline__ void neighbours3(int e, int nx, int ny, int nz, int* nb) {
  const int i = e % nx, j = (e / nx) % ny, k = e / (nx * ny);
  nb[0] = e - i + (i == 0 ? nx - 1 : i - 1);
  nb[1] = e - i + (i == nx - 1 ? 0 : i + 1);
  nb[2] = e + ((j == 0 ? ny - 1 : j - 1) - j) * nx;
  nb[3] = e + ((j == ny - 1 ? 0 : j + 1) - j) * nx;
  nb[4] = e + ((k == 0 ? nz - 1 : k - 1) - k) * nx * ny;
  nb[5] = e + ((k == nz - 1 ? 0 : k + 1) - k) * nx * ny;
}

// Adjoint of the residual accumulators from the adjoint of the time derivative
// (transpose of: identity for means and hydro gradients; a4 = P[x][y]/mu_y,
// a5 = P[x][z]/mu_z, a6 = P[y][x]/mu_x, a7 = P[y][z]/mu_z, a8 = P[z][x]/mu_x,
// a9 = P[z][y]/mu_y, (a10, a11) = ib (P[x][x] - P[y][y], P[x][x] - P[z][z])).
template <typename T>
struct AccBar3 {
  T m[8], g[5][3], P[3][3];
};

template <typename T>
__device__ __forceinline__ void acc_bar3(const T* lam, const PJ3<T>& p, AccBar3<T>& a) {
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    a.m[v] = lam[4 * v];
#pragma unroll
    for (int d = 0; d < 3; ++d) a.g[v][d] = lam[4 * v + 1 + d];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) a.m[5 + c] = lam[20 + c];
  a.P[0][1] = lam[23] * p.imu[1];
  a.P[0][2] = lam[24] * p.imu[2];
  a.P[1][0] = lam[25] * p.imu[0];
  a.P[1][2] = lam[26] * p.imu[2];
  a.P[2][0] = lam[27] * p.imu[0];
  a.P[2][1] = lam[28] * p.imu[1];
  const T r10 = p.ib[0] * lam[29] + p.ib[2] * lam[30];
  const T r11 = p.ib[1] * lam[29] + p.ib[3] * lam[30];
  a.P[0][0] = r10 + r11;
  a.P[1][1] = -r10;
  a.P[2][2] = -r11;
}

// Cotangent of a Gauss-point flux of a face of axis D (tangential signs s1,
// s2) from one adjacent cell (sigma +1 as R, -1 as L): the transpose of
//   mean_k += sigma F_k/(4 h_D)  (k not the normal field),
//   grad_v[D] -= 1.5 F_v/h_D^2,  grad_v[t_i] += sigma s_i (sqrt3/2) F_v/(h_D h_ti),
//   P[c][D] -= F_Bc/8 (c != D),  P[c][t_i] += sigma s_i h_ti F_Bc/(8 sqrt3 h_D).
template <typename T, int D>
__device__ __forceinline__ void flux_bar3(const AccBar3<T>& a, T s1, T s2, T sigma,
                                          const PJ3<T>& p, T* Fb) {
  constexpr int t1 = (D + 1) % 3, t2 = (D + 2) % 3;
  const T cm = sigma * p.c4h[D];
  const T g1 = sigma * s1 * p.cs[D][t1], g2 = sigma * s2 * p.cs[D][t2];
  const T b1 = sigma * s1 * p.pt[D][t1], b2 = sigma * s2 * p.pt[D][t2];
#pragma unroll
  for (int k = 0; k < 8; ++k)
    if (k != 5 + D) Fb[k] = fma(cm, a.m[k], Fb[k]);
#pragma unroll
  for (int v = 0; v < 5; ++v)
    Fb[v] = fma(-p.c15[D], a.g[v][D], fma(g1, a.g[v][t1], fma(g2, a.g[v][t2], Fb[v])));
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (c == D) continue;
    Fb[5 + c] = fma(T(-0.125), a.P[c][D], fma(b1, a.P[c][t1], fma(b2, a.P[c][t2], Fb[5 + c])));
  }
}

// State of a cell's polynomial at offset o from its centroid, and the
// transpose (the cotangent ub of the state added to the coefficient adjoint g).
template <typename T>
__device__ __forceinline__ void point3(const T* c, const T* o, T* u) {
#pragma unroll
  for (int v = 0; v < 5; ++v)
    u[v] = fma(c[4 * v + 3], o[2], fma(c[4 * v + 2], o[1], fma(c[4 * v + 1], o[0], c[4 * v])));
#pragma unroll
  for (int k = 0; k < 3; ++k)
    u[5 + k] = fma(dB3(c + 23, k, 2), o[2],
                   fma(dB3(c + 23, k, 1), o[1], fma(dB3(c + 23, k, 0), o[0], c[20 + k])));
}

template <typename T>
__device__ __forceinline__ void point3_bar(const T* ub, const T* o, T* g) {
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    g[4 * v] += ub[v];
#pragma unroll
    for (int d = 0; d < 3; ++d) g[4 * v + 1 + d] = fma(o[d], ub[v], g[4 * v + 1 + d]);
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    g[20 + k] += ub[5 + k];
#pragma unroll
    for (int d = 0; d < 3; ++d) dB3_bar(k, d, o[d] * ub[5 + k], g + 23);
  }
}

// Face of axis D of cell e (side 0: e is L, its +D face; side 1: e is R):
// adds the face's contribution to (dL/dW_e)^T lam to g.
template <typename T, int D>
__device__ void face_adjoint3(const T* ce, const AccBar3<T>& ae, const T* cn,
                              const AccBar3<T>& an, int side, const PJ3<T>& p, T* g) {
  constexpr int t1 = (D + 1) % 3, t2 = (D + 2) % 3;
  const T he = side == 0 ? p.half[D] : -p.half[D];
  const T sge = side == 0 ? T(-1) : T(1);
#pragma unroll 1
  for (int gp = 0; gp < 4; ++gp) {
    const T s1 = (gp & 2) ? T(1) : T(-1);
    const T s2 = (gp & 1) ? T(1) : T(-1);
    T oe[3], on[3];
    oe[D] = he;
    on[D] = -he;
    oe[t1] = on[t1] = s1 * p.q[t1];
    oe[t2] = on[t2] = s2 * p.q[t2];
    T ue[8], un[8], uL[8], uR[8], Fb[8];
    point3(ce, oe, ue);
    point3(cn, on, un);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      uL[k] = side == 0 ? ue[k] : un[k];
      uR[k] = side == 0 ? un[k] : ue[k];
      Fb[k] = T(0);
    }
    flux_bar3<T, D>(ae, s1, s2, sge, p, Fb);
    flux_bar3<T, D>(an, s1, s2, -sge, p, Fb);
    T ub[8];
#pragma unroll 1
    for (int k = 0; k < 8; ++k) {
      Dual<T> dL[8], dR[8], F[8];
#pragma unroll
      for (int j = 0; j < 8; ++j) {
        dL[j] = Dual<T>(uL[j], T(side == 0 && j == k ? 1 : 0));
        dR[j] = Dual<T>(uR[j], T(side == 1 && j == k ? 1 : 0));
      }
      const Dual<T> bn = Dual<T>(0.5) * (dL[5 + D] + dR[5 + D]);
      dL[5 + D] = bn;
      dR[5 + D] = bn;
      bool bad = false;
      hlld_axis<Dual<T>, D>(dL, dR, Dual<T>(p.gamma, T(0)), Dual<T>(p.eps, T(0)), F, bad);
      T acc = T(0);
#pragma unroll
      for (int j = 0; j < 8; ++j) acc = fma(Fb[j], F[j].d, acc);
      ub[k] = acc;
    }
    point3_bar(ub, oe, g);
  }
}

// Volume fluxes at one point: fe[e][v] the hydro flux along e, and the
// induction fluxes F_y(Bx), F_z(Bx), F_z(By) (the others follow by
// antisymmetry).
template <typename S>
__device__ __forceinline__ void volume_flux3(const S* u, const S* B, S gamma, S (*fe)[5],
                                             S* ind) {
  const S ir = rcp(u[0]);
  const S vel[3] = {u[1] * ir, u[2] * ir, u[3] * ir};
  const S pm = S(0.5) * (B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
  const S pg =
      (gamma - S(1)) * (u[4] - S(0.5) * (u[1] * vel[0] + u[2] * vel[1] + u[3] * vel[2]) - pm);
  const S pT = pg + pm;
  const S vB = vel[0] * B[0] + vel[1] * B[1] + vel[2] * B[2];
#pragma unroll
  for (int e = 0; e < 3; ++e) {
    fe[e][0] = u[1 + e];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      fe[e][1 + k] = u[1 + k] * vel[e] - B[k] * B[e];
      if (k == e) fe[e][1 + k] = fe[e][1 + k] + pT;
    }
    fe[e][4] = (u[4] + pT) * vel[e] - B[e] * vB;
  }
  ind[0] = B[0] * vel[1] - vel[0] * B[1];
  ind[1] = B[0] * vel[2] - vel[0] * B[2];
  ind[2] = B[1] * vel[2] - vel[1] * B[2];
}

// Volume term over the 2x2x2 Gauss points (forward: grad_v[e] += 1.5 fe/h_e^2,
// P[x][y] += F_y(Bx)/8, P[y][x] -= F_y(Bx)/8, P[x][z] += F_z(Bx)/8,
// P[z][x] -= F_z(Bx)/8, P[y][z] += F_z(By)/8, P[z][y] -= F_z(By)/8).
template <typename T>
__device__ void volume_adjoint3(const T* ce, const AccBar3<T>& ae, const PJ3<T>& p, T* g) {
  T feb[3][5], indb[3];
#pragma unroll
  for (int e = 0; e < 3; ++e)
#pragma unroll
    for (int v = 0; v < 5; ++v) feb[e][v] = p.c15[e] * ae.g[v][e];
  indb[0] = T(0.125) * (ae.P[0][1] - ae.P[1][0]);
  indb[1] = T(0.125) * (ae.P[0][2] - ae.P[2][0]);
  indb[2] = T(0.125) * (ae.P[1][2] - ae.P[2][1]);
#pragma unroll 1
  for (int gp = 0; gp < 8; ++gp) {
    const T o[3] = {(gp & 4) ? p.q[0] : -p.q[0], (gp & 2) ? p.q[1] : -p.q[1],
                    (gp & 1) ? p.q[2] : -p.q[2]};
    T u[8], ub[8];
    point3(ce, o, u);
#pragma unroll 1
    for (int k = 0; k < 8; ++k) {
      Dual<T> du[5], dB[3], fe[3][5], ind[3];
#pragma unroll
      for (int j = 0; j < 5; ++j) du[j] = Dual<T>(u[j], T(j == k ? 1 : 0));
#pragma unroll
      for (int j = 0; j < 3; ++j) dB[j] = Dual<T>(u[5 + j], T(5 + j == k ? 1 : 0));
      volume_flux3(du, dB, Dual<T>(p.gamma, T(0)), fe, ind);
      T acc = T(0);
#pragma unroll
      for (int e = 0; e < 3; ++e)
#pragma unroll
        for (int v = 0; v < 5; ++v) acc = fma(feb[e][v], fe[e][v].d, acc);
#pragma unroll
      for (int j = 0; j < 3; ++j) acc = fma(indb[j], ind[j].d, acc);
      ub[k] = acc;
    }
    point3_bar(ub, o, g);
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_adj3m_L(PJ3<T> p) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= p.nc) return;
  int nb[6];
  neighbours3(e, p.nx, p.ny, p.nz, nb);
  T ce[kNC3], le[kNC3], g[kNC3];
  load31(p.W, p.nc, e, ce);
  load31(p.lam, p.nc, e, le);
#pragma unroll
  for (int k = 0; k < kNC3; ++k) g[k] = T(0);
  AccBar3<T> ae;
  acc_bar3(le, p, ae);
#pragma unroll 1
  for (int f = 0; f < 6; ++f) {
    T cn[kNC3], ln[kNC3];
    load31(p.W, p.nc, nb[f], cn);
    load31(p.lam, p.nc, nb[f], ln);
    AccBar3<T> an;
    acc_bar3(ln, p, an);
    // the -D face: e is R (side 1); the +D face: e is L (side 0)
    const int side = (f & 1) ? 0 : 1;
    if (f < 2)
      face_adjoint3<T, 0>(ce, ae, cn, an, side, p, g);
    else if (f < 4)
      face_adjoint3<T, 1>(ce, ae, cn, an, side, p, g);
    else
      face_adjoint3<T, 2>(ce, ae, cn, an, side, p, g);
  }
  volume_adjoint3(ce, ae, p, g);
  const double dt = p.dt_dev ? *p.dt_dev : p.dt_host;
  const T cid = (T)p.c_id, cL = (T)(p.c_L_over_dt * dt), cx = (T)p.c_extra;
#pragma unroll
  for (int k = 0; k < kNC3; ++k) {
    T o = fma(cL, g[k], cid * le[k]);
    if (p.extra) o = fma(cx, p.extra[(size_t)k * p.nc + e], o);
    p.out[(size_t)k * p.nc + e] = o;
  }
}

// The limiter of k_lim3d on one cell (bounds over the cell and its six
// neighbours' means in the order -x, +x, -y, +y, -z, +z).
template <typename S, typename T>
__device__ __forceinline__ S alpha3(S phi, S hi, S lo, const S* g, const T* half) {
  const S D = fmin(hi - phi, phi - lo);
  const S dm = fmax(fmax(fabs(g[0]) * S(half[0]), fabs(g[1]) * S(half[1])),
                    fabs(g[2]) * S(half[2]));
  return (dm > D) ? div_small(D, dm) : S(1);
}

template <typename S, typename T>
__device__ __forceinline__ void limit_cell3(S* c, const S (*nbm)[8], const T* half) {
  S hi[8], lo[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) hi[k] = lo[k] = c[mean3(k)];
#pragma unroll
  for (int f = 0; f < 6; ++f)
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      hi[k] = fmax(hi[k], nbm[f][k]);
      lo[k] = fmin(lo[k], nbm[f][k]);
    }
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const S a = alpha3(c[4 * v], hi[v], lo[v], c + 4 * v + 1, half);
#pragma unroll
    for (int d = 0; d < 3; ++d) c[4 * v + 1 + d] = c[4 * v + 1 + d] * a;
  }
  S aB = S(1);
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    const S gb[3] = {dB3(c + 23, k, 0), dB3(c + 23, k, 1), dB3(c + 23, k, 2)};
    aB = fmin(aB, alpha3(c[20 + k], hi[5 + k], lo[5 + k], gb, half));
  }
#pragma unroll
  for (int j = 0; j < 8; ++j) c[23 + j] = c[23 + j] * aB;
}

template <typename T>
__global__ __launch_bounds__(256) void k_adj3m_lim(PJ3<T> p) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= p.nc) return;
  int cand[7];
  cand[0] = e;
  neighbours3(e, p.nx, p.ny, p.nz, cand + 1);
  T out[kNC3];
#pragma unroll
  for (int k = 0; k < kNC3; ++k) out[k] = T(0);
#pragma unroll 1
  for (int ci = 0; ci < 7; ++ci) {
    const int n = cand[ci];
    bool seen = false;
    for (int cj = 0; cj < ci; ++cj) seen |= cand[cj] == n;
    if (seen) continue;
    int nn[6];
    neighbours3(n, p.nx, p.ny, p.nz, nn);
    T cn[kNC3], lw[kNC3], nbm[6][8];
    load31(p.P, p.nc, n, cn);
    load31(p.lamW, p.nc, n, lw);
#pragma unroll
    for (int f = 0; f < 6; ++f)
#pragma unroll
      for (int k = 0; k < 8; ++k) nbm[f][k] = p.P[(size_t)mean3(k) * p.nc + nn[f]];
#pragma unroll 1
    for (int k = 0; k < kNC3; ++k) {
      // the mean slot of coefficient k (-1: read by the cell's own limiter only)
      const int ks = k < 20 ? (k % 4 == 0 ? k / 4 : -1) : (k < 23 ? k - 15 : -1);
      bool any = n == e;
      for (int f = 0; f < 6; ++f) any |= ks >= 0 && nn[f] == e;
      if (!any) continue;
      Dual<T> c[kNC3], m[6][8];
#pragma unroll
      for (int j = 0; j < kNC3; ++j) c[j] = Dual<T>(cn[j], T(n == e && j == k ? 1 : 0));
#pragma unroll
      for (int f = 0; f < 6; ++f)
#pragma unroll
        for (int j = 0; j < 8; ++j)
          m[f][j] = Dual<T>(nbm[f][j], T(nn[f] == e && j == ks ? 1 : 0));
      limit_cell3(c, m, p.half);
      T acc = T(0);
#pragma unroll
      for (int j = 0; j < kNC3; ++j) acc = fma(lw[j], c[j].d, acc);
      out[k] += acc;
    }
  }
#pragma unroll
  for (int k = 0; k < kNC3; ++k) p.out[(size_t)k * p.nc + e] = out[k];
}

template <typename T>
PJ3<T> make_adj3_params(const dg_mesh* m, const double* dt_dev, double dt) {
  PJ3<T> p{};
  p.dt_dev = dt_dev;
  p.dt_host = dt;
  p.nx = m->c3.nx;
  p.ny = m->c3.ny;
  p.nz = m->c3.nz;
  p.nc = (int)m->ncells;
  p.gamma = (T)m->cfg.gamma;
  p.eps = (T)(m->cfg.precision == DG_FP64 ? 1e-12 : 1e-6);  // as the forward HLLD
  const double h[3] = {m->c3.hx, m->c3.hy, m->c3.hz};
  const double s3 = 1.7320508075688772;
  for (int d = 0; d < 3; ++d) {
    p.c4h[d] = (T)(0.25 / h[d]);
    p.c15[d] = (T)(1.5 / (h[d] * h[d]));
    p.half[d] = (T)(0.5 * h[d]);
    p.q[d] = (T)(0.5 * h[d] / s3);
    p.imu[d] = (T)(12.0 / (h[d] * h[d]));
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
hipError_t adjoint3_t(const dg_mesh* m, const void* U, const void* V1, const double* dt_dev,
                      double dt, const void* lam_np1, void* lam_n, void* ws1, void* ws2,
                      hipStream_t s) {
  const bool lim = m->cfg.limiter == DG_LIMITER_MINMOD;
  const dim3 grid((unsigned)((m->ncells + 255) / 256)), block(256);
  const PJ3<T> p = make_adj3_params<T>(m, dt_dev, dt);
  auto adj_stage = [&](const void* P, const void* lam, const void* extra, double c_id,
                       double c_L_over_dt, double c_extra, void* out) -> hipError_t {
    const void* W = P;
    if (lim) {
      hipError_t r = launch_cart3d(m, kLimit, P, nullptr, ws1, nullptr, 0.0, 0.0, nullptr, s);
      if (r != hipSuccess) return r;
      W = ws1;
    }
    PJ3<T> a = p;
    a.W = static_cast<const T*>(W);
    a.lam = static_cast<const T*>(lam);
    a.extra = static_cast<const T*>(extra);
    a.c_id = c_id;
    a.c_L_over_dt = c_L_over_dt;
    a.c_extra = c_extra;
    a.out = static_cast<T*>(lim ? ws2 : out);
    hipLaunchKernelGGL((k_adj3m_L<T>), grid, block, 0, s, a);
    if (!lim) return hipGetLastError();
    PJ3<T> b = p;
    b.P = static_cast<const T*>(P);
    b.lamW = static_cast<const T*>(ws2);
    b.out = static_cast<T*>(out);
    hipLaunchKernelGGL((k_adj3m_lim<T>), grid, block, 0, s, b);
    return hipGetLastError();
  };
  // stage 2 into lam_n (limiter) or ws2, then stage 1 into lam_n
  void* lam_v1 = lim ? lam_n : ws2;
  hipError_t e = adj_stage(V1, lam_np1, nullptr, 0.5, 0.5, 0.0, lam_v1);
  if (e != hipSuccess) return e;
  return adj_stage(U, lam_v1, lam_np1, 1.0, 1.0, 0.5, lam_n);
}

}  // namespace

hipError_t launch_adjoint_mhd3d(const dg_mesh* m, const void* U, const void* V1,
                                const double* dt_dev, double dt, const void* lam_np1,
                                void* lam_n, void* ws1, void* ws2, hipStream_t s) {
  if (m->cfg.precision == DG_FP64)
    return adjoint3_t<double>(m, U, V1, dt_dev, dt, lam_np1, lam_n, ws1, ws2, s);
  return adjoint3_t<float>(m, U, V1, dt_dev, dt, lam_np1, lam_n, ws1, ws2, s);
}

}  // namespace dg
