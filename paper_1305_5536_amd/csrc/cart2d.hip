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
// Per-cell algebra (weights and the inverse mass matrix folded together).
// With S = F(g0) + F(g1) and D = F(g1) - F(g0) for the two Gauss points of a
// face (g0 at the lower tangential offset), and sum_q F_d(q) the volume
// flux sum over the four 2x2 Gauss points:
//   d mean/dt = (Sx- - Sx+)/(2 hx) + (Sy- - Sy+)/(2 hy)
//   d gx /dt  = 3 (sum_q Fx(q) - Sx- - Sx+)/hx^2 + sqrt(3) (Dy- - Dy+)/(hx hy)
//   d gy /dt  = 3 (sum_q Fy(q) - Sy- - Sy+)/hy^2 + sqrt(3) (Dx- - Dx+)/(hx hy)
#include <hip/hip_runtime.h>

#include "dg_internal.h"

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
  double* dtpart;
  int nx, ny, rows, tiles_x, ntiles;
  int64_t nc;
  T hx, hy, gamma;
  T cmx, cmy, cgx, cgy, ccr;  // 1/(2hx), 1/(2hy), 3/hx^2, 3/hy^2, sqrt3/(hx hy)
  T hx2, hy2, qx, qy;         // hx/2, hy/2, hx/(2 sqrt3), hy/(2 sqrt3)
};

// One row of a column: 4 variables x (mean, gx, gy).
template <typename T>
struct Cell {
  T m[4], gx[4], gy[4];
};

template <typename T>
__device__ __forceinline__ void load_cell(const T* __restrict__ U, int64_t nc, int64_t e,
                                          Cell<T>& c) {
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    c.m[v] = U[(3 * v) * nc + e];
    c.gx[v] = U[(3 * v + 1) * nc + e];
    c.gy[v] = U[(3 * v + 2) * nc + e];
  }
}

template <typename T>
__device__ __forceinline__ void load_means(const T* __restrict__ U, int64_t nc, int64_t e, T* m) {
#pragma unroll
  for (int v = 0; v < 4; ++v) m[v] = U[(3 * v) * nc + e];
}

// Limiter of one cell from its x-neighbour means (shuffled) and y-neighbour
// means (window).  On a Cartesian cell the +d and -d face centroids sit at
// -+ h_d/2, so the two psi of an axis reduce to min(max-phi, phi-min)/|g_d h_d/2|
// and alpha = min(1, D / max_d |g_d h_d / 2|).
template <typename T>
__device__ __forceinline__ void limit_cell(Cell<T>& c, const T* mS, const T* mN, const P2<T>& p) {
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    T mW = __shfl_up(c.m[v], 1);
    T mE = __shfl_down(c.m[v], 1);
    T phi = c.m[v];
    T hi = fmax(fmax(fmax(phi, mW), fmax(mE, mS[v])), mN[v]);
    T lo = fmin(fmin(fmin(phi, mW), fmin(mE, mS[v])), mN[v]);
    T D = fmin(hi - phi, phi - lo);
    T dm = fmax(fabs(c.gx[v]) * p.hx2, fabs(c.gy[v]) * p.hy2);
    T a = (dm > D) ? D / dm : T(1);
    c.gx[v] *= a;
    c.gy[v] *= a;
  }
}

// HLL flux (Davis wave speeds) along axis AX between states uL, uR.
template <typename T, int AX>
__device__ __forceinline__ void hll(const T* uL, const T* uR, T gamma, T* F, bool& bad) {
  const T gm1 = gamma - T(1);
  T irL = T(1) / uL[0], irR = T(1) / uR[0];
  T vxL = uL[1] * irL, vyL = uL[2] * irL;
  T vxR = uR[1] * irR, vyR = uR[2] * irR;
  T pL = gm1 * (uL[3] - T(0.5) * (uL[1] * vxL + uL[2] * vyL));
  T pR = gm1 * (uR[3] - T(0.5) * (uR[1] * vxR + uR[2] * vyR));
  bad |= !(uL[0] > T(0)) || !(uR[0] > T(0)) || !(pL > T(0)) || !(pR > T(0));
  T cL = sqrt(gamma * pL * irL), cR = sqrt(gamma * pR * irR);
  T vnL = AX == 0 ? vxL : vyL;
  T vnR = AX == 0 ? vxR : vyR;
  T SL = fmin(vnL - cL, vnR - cR);
  T SR = fmax(vnL + cL, vnR + cR);
  T FL[4] = {uL[0] * vnL, uL[1] * vnL, uL[2] * vnL, (uL[3] + pL) * vnL};
  T FR[4] = {uR[0] * vnR, uR[1] * vnR, uR[2] * vnR, (uR[3] + pR) * vnR};
  FL[1 + AX] += pL;
  FR[1 + AX] += pR;
  T inv = T(1) / (SR - SL);
  T SLSR = SL * SR;
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    T mid = (SR * FL[k] - SL * FR[k] + SLSR * (uR[k] - uL[k])) * inv;
    F[k] = SL >= T(0) ? FL[k] : (SR <= T(0) ? FR[k] : mid);
  }
}

// Both Cartesian flux rows F_x, F_y at one state (volume term).
template <typename T>
__device__ __forceinline__ void flux_xy(const T* u, T gamma, T* Fx, T* Fy, bool& bad) {
  T ir = T(1) / u[0];
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

template <typename T>
__device__ __forceinline__ void shfl_up_cell(const Cell<T>& c, Cell<T>& o) {
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    o.m[v] = __shfl_up(c.m[v], 1);
    o.gx[v] = __shfl_up(c.gx[v], 1);
    o.gy[v] = __shfl_up(c.gy[v], 1);
  }
}

// x-face between the left neighbour L (lane-1) and this cell R: returns S, D.
template <typename T>
__device__ __forceinline__ void xface(const Cell<T>& L, const Cell<T>& R, const P2<T>& p, T* S,
                                      T* D, bool& bad) {
  T F0[4], F1[4];
  {
    T uL[4], uR[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      T bl = L.m[v] + L.gx[v] * p.hx2, br = R.m[v] - R.gx[v] * p.hx2;
      uL[v] = bl - L.gy[v] * p.qy;
      uR[v] = br - R.gy[v] * p.qy;
    }
    hll<T, 0>(uL, uR, p.gamma, F0, bad);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      T bl = L.m[v] + L.gx[v] * p.hx2, br = R.m[v] - R.gx[v] * p.hx2;
      uL[v] = bl + L.gy[v] * p.qy;
      uR[v] = br + R.gy[v] * p.qy;
    }
    hll<T, 0>(uL, uR, p.gamma, F1, bad);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    S[v] = F0[v] + F1[v];
    D[v] = F1[v] - F0[v];
  }
}

// y-face between the lower cell L (previous row) and the upper cell R.
template <typename T>
__device__ __forceinline__ void yface(const Cell<T>& L, const Cell<T>& R, const P2<T>& p, T* S,
                                      T* D, bool& bad) {
  T F0[4], F1[4];
  T uL[4], uR[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    T bl = L.m[v] + L.gy[v] * p.hy2, br = R.m[v] - R.gy[v] * p.hy2;
    uL[v] = bl - L.gx[v] * p.qx;
    uR[v] = br - R.gx[v] * p.qx;
  }
  hll<T, 1>(uL, uR, p.gamma, F0, bad);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    T bl = L.m[v] + L.gy[v] * p.hy2, br = R.m[v] - R.gy[v] * p.hy2;
    uL[v] = bl + L.gx[v] * p.qx;
    uR[v] = br + R.gx[v] * p.qx;
  }
  hll<T, 1>(uL, uR, p.gamma, F1, bad);
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    S[v] = F0[v] + F1[v];
    D[v] = F1[v] - F0[v];
  }
}

// Volume term: sum of F_x and F_y over the 2x2 Gauss points.
template <typename T>
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
    for (int v = 0; v < 4; ++v) u[v] = c.m[v] + c.gx[v] * ox + c.gy[v] * oy;
    flux_xy(u, p.gamma, Fx, Fy, bad);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      sx[v] += Fx[v];
      sy[v] += Fy[v];
    }
  }
}

template <typename T>
struct Acc {
  T m[4], x[4], y[4];
};

template <typename T>
__device__ __forceinline__ void zero(Acc<T>& a) {
#pragma unroll
  for (int v = 0; v < 4; ++v) a.m[v] = a.x[v] = a.y[v] = T(0);
}

// CFL bound of one cell from its means: 1 / sum_d (|v_d| + c)/h_d.
template <typename T>
__device__ __forceinline__ double cell_dt(const T* m, const P2<T>& p) {
  double r = m[0], ir = 1.0 / r;
  double vx = m[1] * ir, vy = m[2] * ir;
  double pr = ((double)p.gamma - 1.0) * (m[3] - 0.5 * r * (vx * vx + vy * vy));
  double c = sqrt((double)p.gamma * pr * ir);
  double s = (fabs(vx) + c) / (double)p.hx + (fabs(vy) + c) / (double)p.hy;
  return 1.0 / s;
}

__device__ __forceinline__ int xcd_remap(int b, int nb) {
  // Workgroups are dispatched round-robin over the 8 XCDs; give each XCD a
  // contiguous range of tiles so vertically/horizontally adjacent tiles (and
  // their halo rows) share that XCD's L2.
  int per = nb >> 3;
  if (b < (per << 3)) return (b & 7) * per + (b >> 3);
  return b;
}

template <typename T, int MODE, bool LIM>
__global__ __launch_bounds__(256) void k_cart2d(P2<T> p) {
  const int lane = threadIdx.x & (kLanes - 1);
  const int wave = xcd_remap(blockIdx.x, gridDim.x) * 4 + (threadIdx.x >> 6);
  if (wave >= p.ntiles) return;
  const int tx = wave % p.tiles_x, ty = wave / p.tiles_x;
  const int colu = tx * kCols + lane - 2;
  const bool own = lane >= 2 && lane < 2 + kCols && colu < p.nx;
  int col = colu % p.nx;
  if (col < 0) col += p.nx;
  const int y0 = ty * p.rows;
  const int y1 = min(y0 + p.rows, p.ny);
  const int64_t nc = p.nc;
  auto rowi = [&](int r) -> int64_t {
    r %= p.ny;
    if (r < 0) r += p.ny;
    return (int64_t)r * p.nx + col;
  };
  T dt = T(0);
  if (MODE == kStage1 || MODE == kStage2) dt = (T)(p.dt_dev ? *p.dt_dev : p.dt_host);
  bool bad = false;
  double dtmin = 1e300;

  Cell<T> cur, prevlim;
  T mS[4];  // means of row j-1 (raw)
  load_means(p.in, nc, rowi(y0 - 2), mS);
  load_cell(p.in, nc, rowi(y0 - 1), cur);
  // stage 2: window over u0 (rows j-2 means, j-1 full)
  T u0S[4];
  Cell<T> u0C;
  if (MODE == kStage2) {
    load_means(p.u0, nc, rowi(y0 - 1), u0S);
    load_cell(p.u0, nc, rowi(y0), u0C);
  }
  Acc<T> accP, accC;
  zero(accP);
  zero(accC);

  for (int j = y0 - 1; j <= y1; ++j) {
    // next raw row (only means needed beyond the halo row)
    Cell<T> nxt;
    T mN[4];
    if (j + 1 <= y1) {
      load_cell(p.in, nc, rowi(j + 1), nxt);
#pragma unroll
      for (int v = 0; v < 4; ++v) mN[v] = nxt.m[v];
    } else {
      load_means(p.in, nc, rowi(j + 1), mN);
    }
    Cell<T> lim = cur;
    if (LIM || MODE == kLimit) limit_cell(lim, mS, mN, p);

    if (MODE == kLimit) {
      if (own && j >= y0 && j < y1) {
        const int64_t e = rowi(j);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          p.out[(3 * v) * nc + e] = lim.m[v];
          p.out[(3 * v + 1) * nc + e] = lim.gx[v];
          p.out[(3 * v + 2) * nc + e] = lim.gy[v];
        }
      }
    } else {
      if (j >= y0) {
        T S[4], D[4];
        yface(prevlim, lim, p, S, D, bad);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          accP.m[v] -= S[v] * p.cmy;
          accP.y[v] -= S[v] * p.cgy;
          accP.x[v] -= D[v] * p.ccr;
          accC.m[v] += S[v] * p.cmy;
          accC.y[v] -= S[v] * p.cgy;
          accC.x[v] += D[v] * p.ccr;
        }
      }
      if (j >= y0 && j < y1) {
        Cell<T> left;
        shfl_up_cell(lim, left);
        T Sm[4], Dm[4];
        xface(left, lim, p, Sm, Dm, bad);
        T sx[4], sy[4];
        volume(lim, p, sx, sy, bad);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          T Sp = __shfl_down(Sm[v], 1);
          T Dp = __shfl_down(Dm[v], 1);
          accC.m[v] += (Sm[v] - Sp) * p.cmx;
          accC.x[v] += (sx[v] - Sm[v] - Sp) * p.cgx;
          accC.y[v] += (sy[v]) * p.cgy + (Dm[v] - Dp) * p.ccr;
        }
      }
      if (j - 1 >= y0) {
        // finalize row j-1
        Cell<T> o;
        if (MODE == kRhs) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            o.m[v] = accP.m[v];
            o.gx[v] = accP.x[v];
            o.gy[v] = accP.y[v];
          }
        } else if (MODE == kStage1) {
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            o.m[v] = prevlim.m[v] + dt * accP.m[v];
            o.gx[v] = prevlim.gx[v] + dt * accP.x[v];
            o.gy[v] = prevlim.gy[v] + dt * accP.y[v];
          }
        } else {  // kStage2
          T u0N[4];
          Cell<T> u0nxt;
          if (j < y1) {
            load_cell(p.u0, nc, rowi(j), u0nxt);
#pragma unroll
            for (int v = 0; v < 4; ++v) u0N[v] = u0nxt.m[v];
          } else {
            load_means(p.u0, nc, rowi(j), u0N);
          }
          Cell<T> ua = u0C;
          if (LIM) limit_cell(ua, u0S, u0N, p);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            o.m[v] = T(0.5) * ua.m[v] + T(0.5) * (prevlim.m[v] + dt * accP.m[v]);
            o.gx[v] = T(0.5) * ua.gx[v] + T(0.5) * (prevlim.gx[v] + dt * accP.x[v]);
            o.gy[v] = T(0.5) * ua.gy[v] + T(0.5) * (prevlim.gy[v] + dt * accP.y[v]);
          }
#pragma unroll
          for (int v = 0; v < 4; ++v) u0S[v] = u0C.m[v];
          if (j < y1) u0C = u0nxt;
        }
        if (own) {
          const int64_t e = rowi(j - 1);
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            p.out[(3 * v) * nc + e] = o.m[v];
            p.out[(3 * v + 1) * nc + e] = o.gx[v];
            p.out[(3 * v + 2) * nc + e] = o.gy[v];
          }
          if (MODE == kStage2 && p.dtpart) dtmin = fmin(dtmin, cell_dt(o.m, p));
        }
      }
      accP = accC;
      zero(accC);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) mS[v] = cur.m[v];
    prevlim = lim;
    if (j + 1 <= y1) cur = nxt;
  }
  if (bad && own) atomicOr(p.status, 1);
  if (MODE == kStage2 && p.dtpart) {
    // wave minimum (lanes exchange via shuffles), one write per wave
    for (int o = 32; o > 0; o >>= 1) dtmin = fmin(dtmin, __shfl_xor(dtmin, o));
    if (lane == 0) p.dtpart[wave] = dtmin;
  }
}

// Per-wave CFL minima of a state's cell means (stand-alone dg_cfl_dt).
template <typename T>
__global__ __launch_bounds__(256) void k_cart2d_cfl(P2<T> p) {
  const int64_t e = (int64_t)blockIdx.x * blockDim.x + threadIdx.x;
  double d = 1e300;
  if (e < p.nc) {
    T m[4];
    load_means(p.in, p.nc, e, m);
    d = cell_dt(m, p);
  }
  for (int o = 32; o > 0; o >>= 1) d = fmin(d, __shfl_xor(d, o));
  if ((threadIdx.x & 63) == 0) p.dtpart[e >> 6] = d;
}

// Final minimum over the partials: *dt = cfl * min.  One workgroup, fixed
// order (deterministic).
__global__ __launch_bounds__(256) void k_min_finalize(const double* part, int n, double cfl,
                                                      double* dt) {
  __shared__ double s[256];
  double d = 1e300;
  for (int i = threadIdx.x; i < n; i += 256) d = fmin(d, part[i]);
  s[threadIdx.x] = d;
  __syncthreads();
  for (int w = 128; w > 0; w >>= 1) {
    if ((int)threadIdx.x < w) s[threadIdx.x] = fmin(s[threadIdx.x], s[threadIdx.x + w]);
    __syncthreads();
  }
  if (threadIdx.x == 0) *dt = cfl * s[0];
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
  p.dtpart = nullptr;
  p.nx = m->c2.nx;
  p.ny = m->c2.ny;
  p.rows = m->c2.rows_per_tile;
  p.tiles_x = m->c2.tiles_x;
  p.ntiles = m->c2.tiles_x * m->c2.tiles_y;
  p.nc = m->ncells;
  const double hx = m->c2.hx, hy = m->c2.hy, s3 = 1.7320508075688772;
  p.hx = (T)hx;
  p.hy = (T)hy;
  p.gamma = (T)m->cfg.gamma;
  p.cmx = (T)(0.5 / hx);
  p.cmy = (T)(0.5 / hy);
  p.cgx = (T)(3.0 / (hx * hx));
  p.cgy = (T)(3.0 / (hy * hy));
  p.ccr = (T)(s3 / (hx * hy));
  p.hx2 = (T)(0.5 * hx);
  p.hy2 = (T)(0.5 * hy);
  p.qx = (T)(0.5 * hx / s3);
  p.qy = (T)(0.5 * hy / s3);
  return p;
}

template <typename T>
hipError_t launch_t(const dg_mesh* m, int mode, const void* in, const void* u0, void* out,
                    const double* dt_dev, double dt_host, hipStream_t s) {
  P2<T> p = make_params<T>(m, in, u0, out, dt_dev, dt_host);
  const int nblocks = (p.ntiles + 3) / 4;
  const bool lim = m->cfg.limiter == DG_LIMITER_MINMOD;
  if (mode == kStage2) p.dtpart = m->dtpart;
  switch (mode) {
    case kRhs:
      hipLaunchKernelGGL((k_cart2d<T, kRhs, false>), dim3(nblocks), dim3(256), 0, s, p);
      break;
    case kLimit:
      hipLaunchKernelGGL((k_cart2d<T, kLimit, true>), dim3(nblocks), dim3(256), 0, s, p);
      break;
    case kStage1:
      if (lim)
        hipLaunchKernelGGL((k_cart2d<T, kStage1, true>), dim3(nblocks), dim3(256), 0, s, p);
      else
        hipLaunchKernelGGL((k_cart2d<T, kStage1, false>), dim3(nblocks), dim3(256), 0, s, p);
      break;
    case kStage2:
      if (lim)
        hipLaunchKernelGGL((k_cart2d<T, kStage2, true>), dim3(nblocks), dim3(256), 0, s, p);
      else
        hipLaunchKernelGGL((k_cart2d<T, kStage2, false>), dim3(nblocks), dim3(256), 0, s, p);
      break;
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
  hipLaunchKernelGGL(k_min_finalize, dim3(1), dim3(256), 0, s, m->dtpart, nparts, cfl, dt_dev);
  return hipGetLastError();
}

}  // namespace

hipError_t launch_cart2d(const dg_mesh* m, int mode, const void* in, const void* u0, void* out,
                         const double* dt_dev, double dt_host, hipStream_t s) {
  if (m->cfg.precision == DG_FP64)
    return launch_t<double>(m, mode, in, u0, out, dt_dev, dt_host, s);
  return launch_t<float>(m, mode, in, u0, out, dt_dev, dt_host, s);
}

hipError_t launch_cart2d_cfl(const dg_mesh* m, const void* U, double cfl, double* dt_dev,
                             hipStream_t s) {
  if (m->cfg.precision == DG_FP64) return cfl_t<double>(m, U, cfl, dt_dev, s);
  return cfl_t<float>(m, U, cfl, dt_dev, s);
}

hipError_t launch_min_finalize(const double* part, int n, double cfl, double* dt,
                               hipStream_t s) {
  hipLaunchKernelGGL(k_min_finalize, dim3(1), dim3(256), 0, s, part, n, cfl, dt);
  return hipGetLastError();
}

}  // namespace dg
