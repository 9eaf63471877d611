// Discrete adjoint of the 2D ideal-MHD Cartesian SSP-RK2 step: the HLLD flux of
// Sec. 2.3 on the face-averaged normal field, the 2D divergence-free field
// basis of Sec. 2.2 and the limiter of Sec. 2.5 with one alpha for B; dt is
// frozen and every branch (limiter, HLLD wave region) is the one the forward
// step takes.  Ties follow the first argument of min and max, in the order
// self, -x, +x, -y, +y, and |x| takes +x at 0, as the CPU oracle's dual
// numbers do.
//
// As for 2D Euler, the two stages are two "adjoint stages"
//   out = Pi_P^T lamW,   lamW = c_id lam + c_L (dL/dW)^T lam + c_extra extra,
//   W = Pi(P),
// stage 2: P = V1, lam = lam', c_id = 1/2, c_L = dt/2; stage 1: P = U,
// lam = lam_V1, c_id = 1, c_L = dt, extra = lam' with c_extra = 1/2.  Each
// runs the forward limiter (k_lim2m) into a workspace and two gather kernels,
// one thread per cell, no atomics:
//   k_adj2m_L    lamW of a cell from its four faces (two Gauss points each)
//                and its four volume points.  The cotangent of a face flux is
//                the transpose of the linear residual weights (the same
//                algebra as the forward accumulation) applied to the adjoints
//                of both adjacent cells; the Jacobian of the flux with respect
//                to this cell's Gauss-point state comes from forward-mode dual
//                numbers through the HLLD solver, one direction per state
//                component; the extrapolation to the Gauss point is
//                transposed by hand (it is linear).
//   k_adj2m_lim  the limiter transpose: the cell's own limiter differentiated
//                in each of its 23 coefficients, plus what each neighbour's
//                limiter takes from this cell's means (the bounds), by dual
//                numbers.
// Not tuned for speed: each face flux is differentiated from both sides (64
// dual HLLD solves per cell and adjoint stage, against 4 HLLD solves per cell
// in a forward stage).
#include <hip/hip_runtime.h>

#include "dg_internal.h"
#include "dg_math.h"
#include "dual.h"
#include "mhd_hlld.h"

namespace dg {

hipError_t launch_mhd2d(const dg_mesh* m, int mode, const void* in, const void* u0, void* out,
                        const double* dt_dev, double dt_host, double cfl, double* dt_next,
                        hipStream_t s);

namespace {

// Coefficient layout of a cell (23 values): 3v, 3v+1, 3v+2 the mean and x, y
// gradient of rho, mx, my, mz, E (v = 0..4); 15..17 the means of Bx, By, Bz;
// 18..22 a1, a2, a3, dBz/dx, dBz/dy.  The gradient of B_c along axis d is
// sgn(c, d) a[j(c, d)]: grad Bx = (a3, a1), grad By = (a2, -a3), grad Bz =
// (dBz/dx, dBz/dy).
__device__ __forceinline__ int bj(int c, int d) {
  return c == 0 ? (d == 0 ? 2 : 0) : (c == 1 ? (d == 0 ? 1 : 2) : (d == 0 ? 3 : 4));
}
__device__ __forceinline__ int bs(int c, int d) { return (c == 1 && d == 1) ? -1 : 1; }

// Coefficient index of conserved mean k (rho, mx, my, mz, E, Bx, By, Bz).
__device__ __forceinline__ int mean_index(int k) { return k < 5 ? 3 * k : 10 + k; }

template <typename T>
struct PJ {
  const T* W;      // Pi(P), the state the stage's operator sees
  const T* P;      // the stage input (limiter transpose)
  const T* lam;    // adjoint of the stage output (k_adj2m_L)
  const T* extra;  // added to lamW with weight c_extra (may be NULL)
  const T* lamW;   // k_adj2m_lim input
  T* out;
  const double* dt_dev;
  double dt_host;
  double c_id, c_L_over_dt, c_extra;
  int nx, ny, nc;
  T gamma, eps;
  T c2h[2], c3[2], cs, pt[2], half[2], q[2], imu[3];
};

template <typename T>
__device__ __forceinline__ void load23(const T* __restrict__ U, int nc, int e, T* c) {
#pragma unroll
  for (int k = 0; k < 23; ++k) c[k] = U[(size_t)k * nc + e];
}

// The four face neighbours -x, +x, -y, +y of cell e (periodic).
__device__ __forceinline__ void neighbours(int e, int nx, int ny, int* nb) {
  const int i = e % nx, j = e / nx;
  nb[0] = j * nx + (i == 0 ? nx - 1 : i - 1);
  nb[1] = j * nx + (i == nx - 1 ? 0 : i + 1);
  nb[2] = (j == 0 ? ny - 1 : j - 1) * nx + i;
  nb[3] = (j == ny - 1 ? 0 : j + 1) * nx + i;
}

// Adjoint of the residual accumulators of a cell (means of the 8 conserved
// variables, hydro gradients, the field moments P[c][d]) from the adjoint of
// its time derivative: the transpose of the map from accumulators to
// coefficients (identity, and a1 = P[x][y]/mu_y, a2 = P[y][x]/mu_x,
// a3 = (P[x][x] - P[y][y])/(mu_x + mu_y), dBz/dx = P[z][x]/mu_x,
// dBz/dy = P[z][y]/mu_y).
template <typename T>
struct AccBar {
  T m[8], g[5][2], P[3][2];
};

template <typename T>
__device__ __forceinline__ void acc_bar(const T* lam, const PJ<T>& p, AccBar<T>& a) {
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    a.m[v] = lam[3 * v];
    a.g[v][0] = lam[3 * v + 1];
    a.g[v][1] = lam[3 * v + 2];
  }
#pragma unroll
  for (int c = 0; c < 3; ++c) a.m[5 + c] = lam[15 + c];
  a.P[0][1] = lam[18] * p.imu[1];
  a.P[1][0] = lam[19] * p.imu[0];
  a.P[0][0] = lam[20] * p.imu[2];
  a.P[1][1] = -lam[20] * p.imu[2];
  a.P[2][0] = lam[21] * p.imu[0];
  a.P[2][1] = lam[22] * p.imu[1];
}

// Cotangent of a Gauss-point flux F of a face of axis D (tangential sign s)
// from one adjacent cell (sigma = +1 when it is the R cell, -1 the L cell):
// the transpose of the forward accumulation
//   mean_k += sigma F_k/(2 h_D)           (k other than the normal field)
//   grad_v[D] -= 3 F_v / h_D^2,  grad_v[t] += s sigma sqrt3 F_v / (h_D h_t)
//   P[c][D] -= F_Bc / 4,  P[c][t] += s sigma h_t F_Bc / (4 sqrt3 h_D)  (c != D).
template <typename T, int D>
__device__ __forceinline__ void flux_bar(const AccBar<T>& a, T s, T sigma, const PJ<T>& p,
                                         T* Fb) {
  constexpr int t = 1 - D;
  const T cm = sigma * p.c2h[D], ct = s * sigma * p.cs, cp = s * sigma * p.pt[D];
#pragma unroll
  for (int k = 0; k < 8; ++k)
    if (k != 5 + D) Fb[k] = fma(cm, a.m[k], Fb[k]);
#pragma unroll
  for (int v = 0; v < 5; ++v) Fb[v] = fma(-p.c3[D], a.g[v][D], fma(ct, a.g[v][t], Fb[v]));
#pragma unroll
  for (int c = 0; c < 3; ++c) {
    if (c == D) continue;
    Fb[5 + c] = fma(T(-0.25), a.P[c][D], fma(cp, a.P[c][t], Fb[5 + c]));
  }
}

// State of a cell's polynomial at the point (hn along axis D, ht along the
// other axis) from its centroid: hydro Taylor terms and the field basis.
template <typename T, int D>
__device__ __forceinline__ void point_state(const T* c, T hn, T ht, T* u) {
  constexpr int t = 1 - D;
#pragma unroll
  for (int v = 0; v < 5; ++v) u[v] = fma(c[3 * v + 1 + t], ht, fma(c[3 * v + 1 + D], hn, c[3 * v]));
#pragma unroll
  for (int k = 0; k < 3; ++k)
    u[5 + k] = fma(T(bs(k, t)) * c[18 + bj(k, t)], ht,
                   fma(T(bs(k, D)) * c[18 + bj(k, D)], hn, c[15 + k]));
}

// Transpose of point_state: the cotangent ub of the point state added to the
// coefficient adjoint g.
template <typename T, int D>
__device__ __forceinline__ void point_state_bar(const T* ub, T hn, T ht, T* g) {
  constexpr int t = 1 - D;
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    g[3 * v] += ub[v];
    g[3 * v + 1 + D] = fma(hn, ub[v], g[3 * v + 1 + D]);
    g[3 * v + 1 + t] = fma(ht, ub[v], g[3 * v + 1 + t]);
  }
#pragma unroll
  for (int k = 0; k < 3; ++k) {
    g[15 + k] += ub[5 + k];
    g[18 + bj(k, D)] = fma(T(bs(k, D)) * hn, ub[5 + k], g[18 + bj(k, D)]);
    g[18 + bj(k, t)] = fma(T(bs(k, t)) * ht, ub[5 + k], g[18 + bj(k, t)]);
  }
}

// Face of axis D of cell e (side 0: e is L, i.e. the face is e's +D face;
// side 1: e is R) with neighbour coefficients cn and adjoint an: adds the
// face's contribution to (dL/dW_e)^T lam to g.
template <typename T, int D>
__device__ void face_adjoint(const T* ce, const AccBar<T>& ae, const T* cn, const AccBar<T>& an,
                             int side, const PJ<T>& p, T* g) {
  constexpr int t = 1 - D;
  // e's side of the face: normal offset +h_D/2 as L, -h_D/2 as R; the residual
  // sign sigma -1 as L, +1 as R (values are selected element by element: an
  // array picked through a pointer would leave the registers)
  const T he = side == 0 ? p.half[D] : -p.half[D];
  const T sge = side == 0 ? T(-1) : T(1);
#pragma unroll 1
  for (int gp = 0; gp < 2; ++gp) {
    const T s = gp ? T(1) : T(-1);
    const T ht = s * p.q[t];
    T ue[8], un[8], uL[8], uR[8], Fb[8];
    point_state<T, D>(ce, he, ht, ue);
    point_state<T, D>(cn, -he, ht, un);
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      uL[k] = side == 0 ? ue[k] : un[k];
      uR[k] = side == 0 ? un[k] : ue[k];
      Fb[k] = T(0);
    }
    flux_bar<T, D>(ae, s, sge, p, Fb);
    flux_bar<T, D>(an, s, -sge, p, Fb);
    // the Jacobian of the flux on this cell's side, one direction at a time;
    // the normal field enters through the average of both sides
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
    point_state_bar<T, D>(ub, he, ht, g);
  }
}

// Volume fluxes at one point: fe[e][v] the hydro flux along axis e, and the
// induction fluxes F_y(Bx) (= -F_x(By)), F_x(Bz), F_y(Bz).
template <typename S>
__device__ __forceinline__ void volume_flux(const S* u, const S* B, S gamma, S (*fe)[5],
                                            S* ind) {
  const S ir = rcp(u[0]);
  const S vel[3] = {u[1] * ir, u[2] * ir, u[3] * ir};
  const S pm = S(0.5) * (B[0] * B[0] + B[1] * B[1] + B[2] * B[2]);
  const S pg =
      (gamma - S(1)) * (u[4] - S(0.5) * (u[1] * vel[0] + u[2] * vel[1] + u[3] * vel[2]) - pm);
  const S pT = pg + pm;
  const S vB = vel[0] * B[0] + vel[1] * B[1] + vel[2] * B[2];
#pragma unroll
  for (int e = 0; e < 2; ++e) {
    fe[e][0] = u[1 + e];
#pragma unroll
    for (int k = 0; k < 3; ++k) {
      fe[e][1 + k] = u[1 + k] * vel[e] - B[k] * B[e];
      if (k == e) fe[e][1 + k] = fe[e][1 + k] + pT;
    }
    fe[e][4] = (u[4] + pT) * vel[e] - B[e] * vB;
  }
  ind[0] = B[0] * vel[1] - vel[0] * B[1];
  ind[1] = B[2] * vel[0] - vel[2] * B[0];
  ind[2] = B[2] * vel[1] - vel[2] * B[1];
}

// Volume term of cell e over the 2x2 Gauss points: adds its contribution to
// (dL/dW_e)^T lam to g.  Forward: grad_v[e] += 3 fe[e][v] / h_e^2,
// P[x][y] += F_y(Bx)/4, P[y][x] -= F_y(Bx)/4, P[z][x] += F_x(Bz)/4,
// P[z][y] += F_y(Bz)/4.
template <typename T>
__device__ void volume_adjoint(const T* ce, const AccBar<T>& ae, const PJ<T>& p, T* g) {
  T feb[2][5], indb[3];
#pragma unroll
  for (int e = 0; e < 2; ++e)
#pragma unroll
    for (int v = 0; v < 5; ++v) feb[e][v] = p.c3[e] * ae.g[v][e];
  indb[0] = T(0.25) * (ae.P[0][1] - ae.P[1][0]);
  indb[1] = T(0.25) * ae.P[2][0];
  indb[2] = T(0.25) * ae.P[2][1];
#pragma unroll 1
  for (int gp = 0; gp < 4; ++gp) {
    const T o0 = (gp & 2) ? p.q[0] : -p.q[0];
    const T o1 = (gp & 1) ? p.q[1] : -p.q[1];
    T u[8];
    point_state<T, 0>(ce, o0, o1, u);
    T ub[8];
#pragma unroll 1
    for (int k = 0; k < 8; ++k) {
      Dual<T> du[5], dB[3], fe[2][5], ind[3];
#pragma unroll
      for (int j = 0; j < 5; ++j) du[j] = Dual<T>(u[j], T(j == k ? 1 : 0));
#pragma unroll
      for (int j = 0; j < 3; ++j) dB[j] = Dual<T>(u[5 + j], T(5 + j == k ? 1 : 0));
      volume_flux(du, dB, Dual<T>(p.gamma, T(0)), fe, ind);
      T acc = T(0);
#pragma unroll
      for (int e = 0; e < 2; ++e)
#pragma unroll
        for (int v = 0; v < 5; ++v) acc = fma(feb[e][v], fe[e][v].d, acc);
#pragma unroll
      for (int j = 0; j < 3; ++j) acc = fma(indb[j], ind[j].d, acc);
      ub[k] = acc;
    }
    point_state_bar<T, 0>(ub, o0, o1, g);
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_adj2m_L(PJ<T> p) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= p.nc) return;
  int nb[4];
  neighbours(e, p.nx, p.ny, nb);
  T ce[23], le[23], g[23];
  load23(p.W, p.nc, e, ce);
  load23(p.lam, p.nc, e, le);
#pragma unroll
  for (int k = 0; k < 23; ++k) g[k] = T(0);
  AccBar<T> ae;
  acc_bar(le, p, ae);
#pragma unroll 1
  for (int f = 0; f < 4; ++f) {
    T cn[23], ln[23];
    load23(p.W, p.nc, nb[f], cn);
    load23(p.lam, p.nc, nb[f], ln);
    AccBar<T> an;
    acc_bar(ln, p, an);
    // -x: e is R; +x: e is L; -y: e is R; +y: e is L
    const int side = (f & 1) ? 0 : 1;
    if (f < 2)
      face_adjoint<T, 0>(ce, ae, cn, an, side, p, g);
    else
      face_adjoint<T, 1>(ce, ae, cn, an, side, p, g);
  }
  volume_adjoint(ce, ae, p, g);
  const double dt = p.dt_dev ? *p.dt_dev : p.dt_host;
  const T cid = (T)p.c_id, cL = (T)(p.c_L_over_dt * dt), cx = (T)p.c_extra;
#pragma unroll
  for (int k = 0; k < 23; ++k) {
    T o = fma(cL, g[k], cid * le[k]);
    if (p.extra) o = fma(cx, p.extra[(size_t)k * p.nc + e], o);
    p.out[(size_t)k * p.nc + e] = o;
  }
}

// The limiter of Sec. 2.5 on one cell from its 23 coefficients c and the
// means of its neighbours nbm (order -x, +x, -y, +y; rho, mx, my, mz, E, Bx,
// By, Bz), in the forward kernels' arithmetic.
template <typename S, typename T>
__device__ __forceinline__ S alpha_of(S phi, S hi, S lo, S gx, S gy, T hx2, T hy2) {
  const S D = fmin(hi - phi, phi - lo);
  const S dm = fmax(fabs(gx) * S(hx2), fabs(gy) * S(hy2));
  return (dm > D) ? div_small(D, dm) : S(1);
}

template <typename S, typename T>
__device__ __forceinline__ void limit_cell(S* c, const S (*nbm)[8], T hx2, T hy2) {
  S hi[8], lo[8];
#pragma unroll
  for (int k = 0; k < 8; ++k) hi[k] = lo[k] = c[mean_index(k)];
#pragma unroll
  for (int f = 0; f < 4; ++f)
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      hi[k] = fmax(hi[k], nbm[f][k]);
      lo[k] = fmin(lo[k], nbm[f][k]);
    }
#pragma unroll
  for (int v = 0; v < 5; ++v) {
    const S a = alpha_of(c[3 * v], hi[v], lo[v], c[3 * v + 1], c[3 * v + 2], hx2, hy2);
    c[3 * v + 1] = c[3 * v + 1] * a;
    c[3 * v + 2] = c[3 * v + 2] * a;
  }
  S aB = S(1);
#pragma unroll
  for (int k = 0; k < 3; ++k)
    aB = fmin(aB, alpha_of(c[15 + k], hi[5 + k], lo[5 + k], S(T(bs(k, 0))) * c[18 + bj(k, 0)],
                           S(T(bs(k, 1))) * c[18 + bj(k, 1)], hx2, hy2));
#pragma unroll
  for (int j = 0; j < 5; ++j) c[18 + j] = c[18 + j] * aB;
}

// out_e = sum over the cells n whose limiter reads P_e (e itself and its face
// neighbours, each counted once) of (d Pi_n / d P_e)^T lamW_n.
template <typename T>
__global__ __launch_bounds__(256) void k_adj2m_lim(PJ<T> p) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= p.nc) return;
  int cand[5];
  cand[0] = e;
  neighbours(e, p.nx, p.ny, cand + 1);
  T out[23];
#pragma unroll
  for (int k = 0; k < 23; ++k) out[k] = T(0);
#pragma unroll 1
  for (int ci = 0; ci < 5; ++ci) {
    const int n = cand[ci];
    bool seen = false;
    for (int cj = 0; cj < ci; ++cj) seen |= cand[cj] == n;
    if (seen) continue;
    int nn[4];
    neighbours(n, p.nx, p.ny, nn);
    T cn[23], lw[23], nbm[4][8];
    load23(p.P, p.nc, n, cn);
    load23(p.lamW, p.nc, n, lw);
#pragma unroll
    for (int f = 0; f < 4; ++f)
#pragma unroll
      for (int k = 0; k < 8; ++k) nbm[f][k] = p.P[(size_t)mean_index(k) * p.nc + nn[f]];
#pragma unroll 1
    for (int k = 0; k < 23; ++k) {
      // the mean slot of coefficient k (-1: a gradient or field coefficient,
      // which only the cell's own limiter reads)
      const int ks = k < 15 ? (k % 3 == 0 ? k / 3 : -1) : (k < 18 ? k - 10 : -1);
      bool any = n == e;
      for (int f = 0; f < 4; ++f) any |= ks >= 0 && nn[f] == e;
      if (!any) continue;
      Dual<T> c[23], m[4][8];
#pragma unroll
      for (int j = 0; j < 23; ++j) c[j] = Dual<T>(cn[j], T(n == e && j == k ? 1 : 0));
#pragma unroll
      for (int f = 0; f < 4; ++f)
#pragma unroll
        for (int j = 0; j < 8; ++j)
          m[f][j] = Dual<T>(nbm[f][j], T(nn[f] == e && j == ks ? 1 : 0));
      limit_cell(c, m, p.half[0], p.half[1]);
      T acc = T(0);
#pragma unroll
      for (int j = 0; j < 23; ++j) acc = fma(lw[j], c[j].d, acc);
      out[k] += acc;
    }
  }
#pragma unroll
  for (int k = 0; k < 23; ++k) p.out[(size_t)k * p.nc + e] = out[k];
}

template <typename T>
PJ<T> make_adj_params(const dg_mesh* m, const double* dt_dev, double dt) {
  PJ<T> p{};
  p.dt_dev = dt_dev;
  p.dt_host = dt;
  p.nx = m->c2.nx;
  p.ny = m->c2.ny;
  p.nc = (int)m->ncells;
  p.gamma = (T)m->cfg.gamma;
  p.eps = (T)(m->cfg.precision == DG_FP64 ? 1e-12 : 1e-6);  // as the forward HLLD
  const double h[2] = {m->c2.hx, m->c2.hy};
  const double s3 = 1.7320508075688772;
  for (int d = 0; d < 2; ++d) {
    p.c2h[d] = (T)(0.5 / h[d]);
    p.c3[d] = (T)(3.0 / (h[d] * h[d]));
    p.pt[d] = (T)(h[1 - d] / (4.0 * s3 * h[d]));
    p.half[d] = (T)(0.5 * h[d]);
    p.q[d] = (T)(0.5 * h[d] / s3);
  }
  p.cs = (T)(s3 / (h[0] * h[1]));
  const double mx = h[0] * h[0] / 12.0, my = h[1] * h[1] / 12.0;
  p.imu[0] = (T)(1.0 / mx);
  p.imu[1] = (T)(1.0 / my);
  p.imu[2] = (T)(1.0 / (mx + my));
  return p;
}

template <typename T>
hipError_t adjoint_t(const dg_mesh* m, const void* U, const void* V1, const double* dt_dev,
                     double dt, const void* lam_np1, void* lam_n, void* ws1, void* ws2,
                     hipStream_t s) {
  const bool lim = m->cfg.limiter == DG_LIMITER_MINMOD;
  const dim3 grid((unsigned)((m->ncells + 255) / 256)), block(256);
  PJ<T> p = make_adj_params<T>(m, dt_dev, dt);
  hipError_t e = hipSuccess;
  auto adj_stage = [&](const void* P, const void* lam, const void* extra, double c_id,
                       double c_L_over_dt, double c_extra, void* out) -> hipError_t {
    // W = Pi(P) into ws1; lamW into ws2 (or straight into out without a
    // limiter); out = Pi_P^T lamW
    const void* W = P;
    if (lim) {
      hipError_t r = launch_mhd2d(m, kLimit, P, nullptr, ws1, nullptr, 0.0, 0.0, nullptr, s);
      if (r != hipSuccess) return r;
      W = ws1;
    }
    PJ<T> a = p;
    a.W = static_cast<const T*>(W);
    a.lam = static_cast<const T*>(lam);
    a.extra = static_cast<const T*>(extra);
    a.c_id = c_id;
    a.c_L_over_dt = c_L_over_dt;
    a.c_extra = c_extra;
    a.out = static_cast<T*>(lim ? ws2 : out);
    hipLaunchKernelGGL((k_adj2m_L<T>), grid, block, 0, s, a);
    if (!lim) return hipGetLastError();
    PJ<T> b = p;
    b.P = static_cast<const T*>(P);
    b.lamW = static_cast<const T*>(ws2);
    b.out = static_cast<T*>(out);
    hipLaunchKernelGGL((k_adj2m_lim<T>), grid, block, 0, s, b);
    return hipGetLastError();
  };
  // stage 2: lam_V1 = Pi_V1^T [lam'/2 + (dt/2) L^T lam'] (in lam_n with the
  // limiter, else in ws2)
  void* lam_v1 = lim ? lam_n : ws2;
  e = adj_stage(V1, lam_np1, nullptr, 0.5, 0.5, 0.0, lam_v1);
  if (e != hipSuccess) return e;
  // stage 1: lam_n = Pi_U^T [lam_V1 + dt L^T lam_V1 + lam'/2]
  return adj_stage(U, lam_v1, lam_np1, 1.0, 1.0, 0.5, lam_n);
}

}  // namespace

hipError_t launch_adjoint_mhd2d(const dg_mesh* m, const void* U, const void* V1,
                                const double* dt_dev, double dt, const void* lam_np1,
                                void* lam_n, void* ws1, void* ws2, hipStream_t s) {
  if (m->cfg.precision == DG_FP64)
    return adjoint_t<double>(m, U, V1, dt_dev, dt, lam_np1, lam_n, ws1, ws2, s);
  return adjoint_t<float>(m, U, V1, dt_dev, dt, lam_np1, lam_n, ws1, ws2, s);
}

}  // namespace dg
