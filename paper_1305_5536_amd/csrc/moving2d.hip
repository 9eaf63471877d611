// 2D Euler DG on a moving periodic Voronoi mesh (Sec. 2.3) with the
// MUSCL-Hancock step (Sec. 2.4), on gfx950.
//
// The mesh is the Voronoi tessellation of generators that move with their
// cell's fluid velocity (mean momentum over mean density, constant over a
// step).  Every step rebuilds it on the GPU, one thread per cell, with no
// atomics and no global triangulation:
//   * the cell of generator i is the intersection of the half-planes closer to
//     i than to each candidate j; the candidates are i's neighbours and their
//     neighbours in the previous mesh (a cell's new neighbours over one CFL
//     step were among them).  Its faces are found by walking around it
//     counter-clockwise from the nearest candidate: the next face is the
//     candidate whose bisector first cuts the current face's bisector (no
//     polygon is stored, only the ring of neighbours);
//   * each Voronoi vertex is then recomputed as the circumcentre of its three
//     generators, in the frame of the smallest of the three indices, so that
//     every cell that shares a vertex or a face derives it from the same
//     operands (a face's flux is computed by both of its cells; the canonical
//     operands make the two results agree);
//   * faces shorter than 1e-10 times their generators' distance (four nearly
//     cocircular generators) are dropped by both cells;
//   * areas, centroids and second moments (the mass matrix of Sec. 2.2, which
//     a moving mesh recomputes every step) are the exact polygon moments.
// A cell whose candidates do not bound it, a polygon beyond the capacities
// below, or a neighbour that does not list the cell back, latches status bit 2
// (reported by dg_check).  Every kernel maps its blocks XCD by XCD
// (xcd_remap): with cells numbered along a space-filling curve each XCD's L2
// then holds the positions, rings and states of one compact region, which the
// neighbour gathers reuse.
//
// One step, n -> n+1 (sets: t^n, the half step, t^{n+1}):
//   k_mv_lim   limiter on the mesh of t^n (none, the Arepo limiter on the
//              conserved coefficients, or the WENO-type limiter on primitive
//              variables with a least-squares stencil slope), and the
//              generator positions at t^{n+1/2} and t^{n+1};
//   k_mv_walk, k_mv_geom  the mesh of the half-step generators;
//   k_mv_upd   per cell of the half-step mesh: for each face and Gauss point,
//              both cells' half-step primitive predictions (centred at the
//              t^n centroids) at the point, boosted into the frame of the face
//              there (the bisector's velocity), the Riemann flux (HLL or
//              exact) in that frame carried back to the lab frame
//              (F_m = F - U w^T); the volume flux F - U w_e^T on the half-step
//              cell's 4-point rule; out: the conserved totals V^n ubar +
//              dt (...) and the first moments about the cell's origin carried
//              along with w_e (c^n + t w_e);
//   k_mv_walk, k_mv_geom  the mesh of t^{n+1}, then the new state: means = totals /
//              V^{n+1}, gradients = (M^{n+1})^-1 (moments - (c^{n+1} - c^n -
//              dt w_e) totals), and the cell's CFL bound.
// Geometry is FP64 (absolute positions in a box); the state is T.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cstdlib>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "dg_internal.h"
#include "dg_math.h"
#include "euler_exact.h"

namespace dg {

constexpr int kRing = 16;  // neighbours a cell may have
constexpr int kPoly = kRing + 1;  // ring entries during the walk
constexpr int kGeo = 6;    // V, centroid - generator (2), Mxx, Mxy, Myy
constexpr int kChunk = 4;  // candidates gathered together in the walk
constexpr int kCand = 40;  // distinct candidates of one cell's walk kept in LDS
constexpr int kWalkThreads = 128;  // threads per block of the walk (LDS: kCand ints each)

struct MVDev {
  int n = 0;
  double box[2] = {1.0, 1.0};
  int motion = 1;
  int cur = 0, nxt = 2;  // sets holding t^n and t^{n+1}; set 1 is the half step
  // [4][n]: x block, y block, then the same positions interleaved (x, y) per
  // generator, which the walk gathers with one 16-byte load per candidate
  double* pos[3] = {nullptr, nullptr, nullptr};
  int* ring[3] = {nullptr, nullptr, nullptr};    // [n][kRing], counter-clockwise
  int* deg[3] = {nullptr, nullptr, nullptr};     // [n]
  double* geo[3] = {nullptr, nullptr, nullptr};  // [kGeo][n]
  void* ua = nullptr;                            // limited state
  int cand_cap = kCand;                          // LDS list length of the walk (<= kCand)
  bool timing = false;                           // record events around each kernel
  std::vector<hipEvent_t> ev;                    // 5 per timed step
};

namespace {

// One set of mesh arrays as kernels see it.
struct MSet {
  const double* x;  // x block of the positions (y = x + n, interleaved pairs from x + 2n)
  const int* ring;
  const int* deg;
  const double* geo;
};
struct MOut {
  double* x;
  int* ring;
  int* deg;
  double* geo;
};

template <typename T>
struct PM {
  const T* __restrict__ in;
  const T* __restrict__ ua;
  T* __restrict__ ua_out;
  T* __restrict__ out;
  const double* dt_dev;
  double dt_host;
  int* status;
  double* dtpart;
  int n;
  double Lx, Ly;
  T gamma;
  int motion;
  int cand_cap;   // k_mv_walk: candidates kept in LDS before streaming them
  int write_pos;  // k_mv_lim: write the half-step and next positions
  MSet s0;        // t^n
  MSet sh;        // half step
  double* xh;     // positions written by k_mv_lim
  double* x1;
};

__device__ __forceinline__ double mimg(double d, double L) { return d - L * rint(d / L); }

// x + s w wrapped into [0, L), rounded as (s w) then the sum.
__device__ __forceinline__ double advance(double x, double s, double w, double L) {
#pragma clang fp contract(off)
  const double y = x + s * w;
  if (y < 0.0) return y + L;
  if (y >= L) return y - L;
  return y;
}

// Circumcentre of generators a, b, c as an offset from generator f.  Worked
// in the frame of the smallest of the three indices from minimum-image
// offsets, without contraction, so that every cell sharing the vertex gets the
// same bits before the final shift.
__device__ __forceinline__ void circumcentre(const double* __restrict__ X, int n, double Lx,
                                          double Ly, int a, int b, int c, int f, double& ox,
                                          double& oy) {
#pragma clang fp contract(off)
  int t;
  if (a > b) { t = a; a = b; b = t; }
  if (b > c) { t = b; b = c; c = t; }
  if (a > b) { t = a; a = b; b = t; }
  // the interleaved copy of the positions: one 16-byte load per generator
  const double2* P = reinterpret_cast<const double2*>(X + 2 * (size_t)n);
  const double2 pa = P[a], pb = P[b], pc = P[c];
  const double px = mimg(pb.x - pa.x, Lx), py = mimg(pb.y - pa.y, Ly);
  const double qx = mimg(pc.x - pa.x, Lx), qy = mimg(pc.y - pa.y, Ly);
  const double D = 2.0 * (px * qy - py * qx);
  const double pp = px * px + py * py, qq = qx * qx + qy * qy;
  double ux = (qy * pp - py * qq) / D;
  double uy = (px * qq - qx * pp) / D;
  if (a != f) {
    const double2 pf = P[f];
    ux += mimg(pa.x - pf.x, Lx);
    uy += mimg(pa.y - pf.y, Ly);
  }
  ox = ux;
  oy = uy;
}

// Face between cells L < R whose Voronoi edge ends at the circumcentres of
// (L, R, ka) and (L, R, kb): endpoints (from L's generator) ordered so that
// the normal (e_y, -e_x)/|e| points from L towards R, the generator offset
// dLR, and the length.  Every argument order gives the same bits.
struct FaceG {
  double ax, ay, bx, by;  // endpoints
  double dx, dy;          // R's generator - L's generator
  double A, nx, ny;
};

__device__ __forceinline__ void face_geometry(const double* __restrict__ X, int n, double Lx,
                                              double Ly, int L, int R, int ka, int kb,
                                              FaceG& g) {
#pragma clang fp contract(off)
  double ax, ay, bx, by;
  circumcentre(X, n, Lx, Ly, L, R, ka, L, ax, ay);
  circumcentre(X, n, Lx, Ly, L, R, kb, L, bx, by);
  const double2* P = reinterpret_cast<const double2*>(X + 2 * (size_t)n);
  const double2 pL = P[L], pR = P[R];
  const double dx = mimg(pR.x - pL.x, Lx), dy = mimg(pR.y - pL.y, Ly);
  double ex = bx - ax, ey = by - ay;
  if (ey * dx - ex * dy < 0.0) {
    double t = ax; ax = bx; bx = t;
    t = ay; ay = by; by = t;
    ex = -ex;
    ey = -ey;
  }
  g.ax = ax;
  g.ay = ay;
  g.bx = bx;
  g.by = by;
  g.dx = dx;
  g.dy = dy;
  g.A = sqrt(ex * ex + ey * ey);
  g.nx = ey / g.A;
  g.ny = -ex / g.A;
}

// Polygon moments about the generator from vertex offsets v[0..m): area,
// first and second moments (fan triangles from the generator).
__device__ __forceinline__ void polygon_moments(const double* vx, const double* vy, int m,
                                                double* geo) {
  double V = 0, m1x = 0, m1y = 0, mxx = 0, mxy = 0, myy = 0;
  for (int k = 0; k < m; ++k) {
    const int k1 = k + 1 == m ? 0 : k + 1;
    const double e0x = vx[k], e0y = vy[k], e1x = vx[k1], e1y = vy[k1];
    const double ar = 0.5 * (e0x * e1y - e0y * e1x);
    const double sx = e0x + e1x, sy = e0y + e1y;
    V += ar;
    m1x += ar * sx / 3.0;
    m1y += ar * sy / 3.0;
    const double w = ar / 12.0;
    mxx += w * (e0x * e0x + e1x * e1x + sx * sx);
    mxy += w * (e0x * e0y + e1x * e1y + sx * sy);
    myy += w * (e0y * e0y + e1y * e1y + sy * sy);
  }
  const double cx = m1x / V, cy = m1y / V;
  geo[0] = V;
  geo[1] = cx;
  geo[2] = cy;
  geo[3] = mxx - V * cx * cx;
  geo[4] = mxy - V * cx * cy;
  geo[5] = myy - V * cy * cy;
}

// Vertices of cell e of a mesh set (offsets from its generator): vertex k is
// the circumcentre of (e, ring[k-1], ring[k]).
__device__ __forceinline__ int cell_polygon(const MSet& s, int n, double Lx, double Ly, int e,
                                            double* vx, double* vy, int* nb) {
  const int d = min(s.deg[e], kRing);
  for (int k = 0; k < d; ++k) nb[k] = s.ring[e * kRing + k];
  for (int k = 0; k < d; ++k)
    circumcentre(s.x, n, Lx, Ly, e, nb[k == 0 ? d - 1 : k - 1], nb[k], e, vx[k], vy[k]);
  return d;
}

template <typename T>
__device__ __forceinline__ void load12(const T* __restrict__ U, int n, int e, T* q) {
#pragma unroll
  for (int k = 0; k < 12; ++k) q[k] = U[(size_t)k * n + e];
}

template <typename T>
__device__ __forceinline__ double step_size(const PM<T>& p) {
  return p.dt_dev ? *p.dt_dev : p.dt_host;
}

// Primitive (rho, v_x, v_y, p) of conserved means.
template <typename T>
__device__ __forceinline__ void prim4(const T* m, T gm1, T* w) {
  const T ir = rcp(m[0]);
  w[0] = m[0];
  w[1] = m[1] * ir;
  w[2] = m[2] * ir;
  w[3] = gm1 * (m[3] - T(0.5) * (m[1] * w[1] + m[2] * w[2]));
}

// ------------------------------------------------------------- limiter --
// Per cell of the mesh of t^n.  LIM 0 copies, 1 the Arepo limiter on the
// conserved coefficients, 2 the WENO-type limiter on (rho, v, p) with the
// least-squares stencil slope over the face neighbours.  Also moves the
// generators (when write_pos) and checks that every neighbour lists the
// cell back.
template <typename T, int LIM>
__global__ __launch_bounds__(256) void k_mv_lim(PM<T> p) {
  const int e = xcd_remap(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
  if (e >= p.n) return;
  const int n = p.n;
  T q[12];
  load12(p.in, n, e, q);
  const MSet& s = p.s0;
  const int* re = s.ring + e * kRing;
  const int d = min(s.deg[e], kRing);
  bool meshbad = s.deg[e] > kRing || s.deg[e] < 3;
  for (int k = 0; k < d; ++k) {
    const int j = re[k];
    bool back = false;
    const int dj = min(s.deg[j], kRing);
    for (int a = 0; a < dj; ++a) back |= s.ring[j * kRing + a] == e;
    meshbad |= !back;
  }
  if (meshbad) atomicOr(p.status, 2);
  const double dcx = s.geo[1 * n + e], dcy = s.geo[2 * n + e];
  // The faces are visited in passes that recompute what they need (the face
  // centroid from the two circumcentres that end the face, the neighbour's
  // centroid offset and means) instead of keeping per-face arrays, which
  // would live in per-lane scratch memory.
  // Face centroids, in order: vertex k is the circumcentre of (e, ring[k-1],
  // ring[k]); face k runs from vertex k to vertex k+1.
  auto faces = [&](auto&& f) {
    if (d < 3) return;
    double ax, ay;
    circumcentre(s.x, n, p.Lx, p.Ly, e, re[d - 1], re[0], e, ax, ay);
    const double a0x = ax, a0y = ay;
    for (int k = 0; k < d; ++k) {
      double bx = a0x, by = a0y;
      if (k + 1 < d) circumcentre(s.x, n, p.Lx, p.Ly, e, re[k], re[k + 1], e, bx, by);
      f(k, re[k], (T)(0.5 * (ax + bx) - dcx), (T)(0.5 * (ay + by) - dcy));
      ax = bx;
      ay = by;
    }
  };
  if (LIM != 0) {
    const T gm1 = p.gamma - T(1);
    if (LIM == 1) {
      T hi[4], lo[4], alpha[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        hi[v] = lo[v] = q[3 * v];
        alpha[v] = T(1);
      }
      for (int k = 0; k < d; ++k) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const T m = p.in[(size_t)(3 * v) * n + re[k]];
          hi[v] = fmax(hi[v], m);
          lo[v] = fmin(lo[v], m);
        }
      }
      faces([&](int, int, T rx, T ry) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const T dd = q[3 * v + 1] * rx + q[3 * v + 2] * ry;
          const T num = dd > T(0) ? hi[v] - q[3 * v] : lo[v] - q[3 * v];
          const T psi = dd > T(0) ? div_small(num, dd) : (dd < T(0) ? div_small(-num, -dd) : T(1));
          alpha[v] = fmin(alpha[v], psi);
        }
      });
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        q[3 * v + 1] *= alpha[v];
        q[3 * v + 2] *= alpha[v];
      }
    } else {
      const T eps = sizeof(T) == 8 ? T(2.220446049250313e-16) : T(1.1920929e-7);
      T mi[4] = {q[0], q[3], q[6], q[9]};
      T wi[4];
      prim4(mi, gm1, wi);
      auto nbr_prim = [&](int j, T* w) {
        T mj[4];
#pragma unroll
        for (int v = 0; v < 4; ++v) mj[v] = p.in[(size_t)(3 * v) * n + j];
        prim4(mj, gm1, w);
      };
      const T rho = wi[0], ir = rcp(rho), ux = wi[1], uy = wi[2];
      const T v2 = ux * ux + uy * uy;
      // DG primitive slopes (chain rule at the centroid)
      T gx[4], gy[4];
      gx[0] = q[1];
      gy[0] = q[2];
      gx[1] = (q[4] - ux * gx[0]) * ir;
      gy[1] = (q[5] - ux * gy[0]) * ir;
      gx[2] = (q[7] - uy * gx[0]) * ir;
      gy[2] = (q[8] - uy * gy[0]) * ir;
      gx[3] = gm1 * (q[10] - T(0.5) * v2 * gx[0] - rho * (ux * gx[1] + uy * gx[2]));
      gy[3] = gm1 * (q[11] - T(0.5) * v2 * gy[0] - rho * (ux * gy[1] + uy * gy[2]));
      // pass 1: least-squares normal equations of the stencil, bounds
      T a00 = T(0), a01 = T(0), a11 = T(0), b0[4], b1[4], hi[4], lo[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        b0[v] = b1[v] = T(0);
        hi[v] = lo[v] = wi[v];
      }
      const double2* P = reinterpret_cast<const double2*>(s.x + 2 * (size_t)n);
      const double2 pe = P[e];
      for (int k = 0; k < d; ++k) {
        const int j = re[k];
        const double2 pj = P[j];
        const T dnx = (T)(mimg(pj.x - pe.x, p.Lx) + s.geo[1 * n + j] - dcx);
        const T dny = (T)(mimg(pj.y - pe.y, p.Ly) + s.geo[2 * n + j] - dcy);
        a00 += dnx * dnx;
        a01 += dnx * dny;
        a11 += dny * dny;
        T wj[4];
        nbr_prim(j, wj);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const T dw = wj[v] - wi[v];
          b0[v] += dnx * dw;
          b1[v] += dny * dw;
          hi[v] = fmax(hi[v], wj[v]);
          lo[v] = fmin(lo[v], wj[v]);
        }
      }
      const T idet = rcp(a00 * a11 - a01 * a01);
      T sx[4], sy[4], alpha[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        sx[v] = (a11 * b0[v] - a01 * b1[v]) * idet;
        sy[v] = (a00 * b1[v] - a01 * b0[v]) * idet;
        alpha[v] = T(1);
      }
      // pass 2: the stencil slope limited as in the Arepo limiter
      faces([&](int, int, T rx, T ry) {
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const T dd = sx[v] * rx + sy[v] * ry;
          // the clamp absorbs rounding of hi - w (w a product): D >= 0
          const T num = dd > T(0) ? fmax(hi[v] - wi[v], T(0)) : fmin(lo[v] - wi[v], T(0));
          const T psi = dd > T(0) ? div_small(num, dd) : (dd < T(0) ? div_small(-num, -dd) : T(1));
          alpha[v] = fmin(alpha[v], psi);
        }
      });
      // pass 3: oscillation factors of the two candidates
      T os[4], od[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        sx[v] *= alpha[v];
        sy[v] *= alpha[v];
        os[v] = od[v] = T(0);
      }
      faces([&](int, int j, T rx, T ry) {
        T wj[4];
        nbr_prim(j, wj);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const T ds = sx[v] * rx + sy[v] * ry;
          const T dg = gx[v] * rx + gy[v] * ry;
          os[v] += fabs(ds) + fabs(wj[v] - (wi[v] + ds));
          od[v] += fabs(dg) + fabs(wj[v] - (wi[v] + dg));
        }
      });
      T ngx[4], ngy[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const T ws = rcp(sqrt_pos(eps + os[v])), wd = rcp(sqrt_pos(eps + od[v]));
        const T iw = rcp(ws + wd);
        ngx[v] = (ws * sx[v] + wd * gx[v]) * iw;
        ngy[v] = (ws * sy[v] + wd * gy[v]) * iw;
      }
      q[1] = ngx[0];
      q[2] = ngy[0];
      q[4] = ux * ngx[0] + rho * ngx[1];
      q[5] = ux * ngy[0] + rho * ngy[1];
      q[7] = uy * ngx[0] + rho * ngx[2];
      q[8] = uy * ngy[0] + rho * ngy[2];
      const T igm1 = rcp(gm1);
      q[10] = ngx[3] * igm1 + T(0.5) * v2 * ngx[0] + rho * (ux * ngx[1] + uy * ngx[2]);
      q[11] = ngy[3] * igm1 + T(0.5) * v2 * ngy[0] + rho * (ux * ngy[1] + uy * ngy[2]);
    }
  }
#pragma unroll
  for (int k = 0; k < 12; ++k) p.ua_out[(size_t)k * n + e] = q[k];
  if (p.write_pos) {
    const double dt = step_size(p);
    double wx = 0.0, wy = 0.0;
    if (p.motion) {
      wx = (double)q[3] / (double)q[0];
      wy = (double)q[6] / (double)q[0];
    }
    const double x = s.x[e], y = s.x[n + e];
    const double hx = advance(x, 0.5 * dt, wx, p.Lx), hy = advance(y, 0.5 * dt, wy, p.Ly);
    const double nx1 = advance(x, dt, wx, p.Lx), ny1 = advance(y, dt, wy, p.Ly);
    p.xh[e] = hx;
    p.xh[n + e] = hy;
    reinterpret_cast<double2*>(p.xh + 2 * (size_t)n)[e] = make_double2(hx, hy);
    p.x1[e] = nx1;
    p.x1[n + e] = ny1;
    reinterpret_cast<double2*>(p.x1 + 2 * (size_t)n)[e] = make_double2(nx1, ny1);
  }
}

// ----------------------------------------------------------------- mesh --
// The mesh of the positions dst.x in two launches.  k_mv_walk: the ring of
// every cell from the 2-ring of the mesh `src` (written to dst.ring, dst.deg).
// k_mv_geom: the cell geometry from the ring (canonical vertices, polygon
// moments); with FINISH also the new state from the totals and moments in
// p.out (the mesh of t^n in p.s0, the limited state p.ua for w_e) and the
// cell's CFL bound in the per-wave minima when p.dtpart is set.  Split in two
// so that the walk, a chain of dependent gathers, runs at a higher occupancy
// than the register-heavy geometry and update.
template <typename T>
__global__ __launch_bounds__(kWalkThreads) void k_mv_walk(PM<T> p, MSet src, MOut dst) {
  // each thread's distinct candidates, in a column of its own (no barrier)
  __shared__ int cl[kCand * kWalkThreads];
  const int tl = threadIdx.x;
  const int e = xcd_remap(blockIdx.x, gridDim.x) * kWalkThreads + tl;
  if (e < p.n) {
    const int n = p.n;
    const double2* XY = reinterpret_cast<const double2*>(dst.x + 2 * (size_t)n);
    const double2 pe = XY[e];
    const double xe = pe.x, ye = pe.y;
    bool bad = false;
    const int d0 = min(src.deg[e], kRing);
    const double iLx = 1.0 / p.Lx, iLy = 1.0 / p.Ly;
    // The candidates (the previous neighbours and the entries of their
    // rings) are listed once, without repeats, in LDS; a cell with more than
    // kCand of them streams them from the rings instead (repeats included:
    // they give equal values and the index tie-break makes them harmless).
    int nc = 0;
    bool stream = false;
    for (int a = 0; a < d0 && !stream; ++a) {
      const int j = src.ring[e * kRing + a];
      const int dj = min(src.deg[j], kRing);
      for (int b = -1; b < dj; ++b) {
        const int k = b < 0 ? j : src.ring[j * kRing + b];
        if (k == e) continue;
        bool seen = false;
        for (int c = 0; c < nc; ++c) seen |= cl[c * kWalkThreads + tl] == k;
        if (seen) continue;
        if (nc == p.cand_cap) {
          stream = true;
          break;
        }
        cl[nc++ * kWalkThreads + tl] = k;
      }
    }
    auto offset = [&](int k, double& dx, double& dy) {
      const double2 pk = XY[k];
      dx = pk.x - xe;
      dy = pk.y - ye;
      dx -= p.Lx * rint(dx * iLx);
      dy -= p.Ly * rint(dy * iLy);
    };
    // f(k, dx, dy) for every candidate: its offset from this generator; the
    // positions of kChunk candidates are loaded together so that the gathers
    // overlap.
    auto visit = [&](auto&& f) {
      if (stream) {
        for (int a = 0; a < d0; ++a) {
          const int j = src.ring[e * kRing + a];
          const int dj = min(src.deg[j], kRing);
          for (int b = -1; b < dj; ++b) {
            const int k = b < 0 ? j : src.ring[j * kRing + b];
            if (k == e) continue;
            double dx, dy;
            offset(k, dx, dy);
            f(k, dx, dy);
          }
        }
        return;
      }
      for (int c0 = 0; c0 < nc; c0 += kChunk) {
        int kk[kChunk];
        double kx[kChunk], ky[kChunk];
#pragma unroll
        for (int q = 0; q < kChunk; ++q) kk[q] = c0 + q < nc ? cl[(c0 + q) * kWalkThreads + tl] : e;
#pragma unroll
        for (int q = 0; q < kChunk; ++q) {
          const double2 pk = XY[kk[q]];
          kx[q] = pk.x;
          ky[q] = pk.y;
        }
#pragma unroll
        for (int q = 0; q < kChunk; ++q) {
          if (c0 + q >= nc) continue;
          double dx = kx[q] - xe, dy = ky[q] - ye;
          dx -= p.Lx * rint(dx * iLx);
          dy -= p.Ly * rint(dy * iLy);
          f(kk[q], dx, dy);
        }
      }
    };
    // The cell is walked counter-clockwise, one face at a time.  The nearest
    // candidate is a neighbour (the midpoint of the two generators lies on
    // their common face).  The face of neighbour j lies on the bisector
    // x(t) = d_j/2 + t perp(d_j), perp(d) = (-d_y, d_x); candidate k bounds it
    // from the counter-clockwise side at t_k = (|d_k|^2 - d_j . d_k) / (2
    // perp(d_j) . d_k) when perp(d_j) . d_k > 0, and the next neighbour is the
    // candidate with the smallest t_k.  The walk ends back at the first
    // neighbour; nothing but the ring is stored.
    int j0 = -1;
    double best = 1e300;
    visit([&](int k, double dx, double dy) {
      const double dd = dx * dx + dy * dy;
      if (dd < best || (dd == best && k < j0)) {
        best = dd;
        j0 = k;
      }
    });
    bad |= j0 < 0;
    int ring[kPoly];
    int d = 0;
    int cur = j0;
    while (!bad) {
      if (d > kRing) {
        bad = true;
        break;
      }
      ring[d++] = cur;
      const double2 pc = XY[cur];
      double cx = pc.x - xe, cy = pc.y - ye;
      cx -= p.Lx * rint(cx * iLx);
      cy -= p.Ly * rint(cy * iLy);
      // smallest t_k = num_k / (2 den_k), compared as num_k den_b < num_b den_k
      int nxt = -1;
      double nb_ = 1.0, db_ = 0.0;
      visit([&](int k, double kx, double ky) {
        if (k == cur) return;
        const double den = cx * ky - cy * kx;  // perp(d_cur) . d_k
        if (!(den > 0.0)) return;
        const double num = kx * kx + ky * ky - (cx * kx + cy * ky);
        const double l = num * db_, r = nb_ * den;
        if (nxt < 0 || l < r || (l == r && k < nxt)) {
          nb_ = num;
          db_ = den;
          nxt = k;
        }
      });
      if (nxt < 0) {
        bad = true;
        break;
      }
      if (nxt == j0) break;
      cur = nxt;
    }
    bad |= d > kRing;
    if (!bad) {
      for (int k = 0; k < d; ++k) dst.ring[e * kRing + k] = ring[k];
      for (int k = d; k < kRing; ++k) dst.ring[e * kRing + k] = -1;
      dst.deg[e] = d;
    } else {
      dst.deg[e] = 0;
      for (int k = 0; k < kRing; ++k) dst.ring[e * kRing + k] = -1;
      atomicOr(p.status, 2);
    }
  }
}

template <typename T, bool FINISH>
__global__ __launch_bounds__(256) void k_mv_geom(PM<T> p, MOut dst) {
  const int e = xcd_remap(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
  double dtb = 1e300;
  if (e < p.n) {
    const int n = p.n;
    const double* X = dst.x;
    const double xe = X[e], ye = X[n + e];
    int d = dst.deg[e];
    bool bad = d < 3 || d > kRing;
    int ring[kRing];
    for (int k = 0; k < kRing; ++k) ring[k] = dst.ring[e * kRing + k];
    if (!bad) {
      // drop the faces shorter than 1e-10 of their generators' distance (their
      // existence is decided by rounding); both cells of such a face decide it
      // from the same canonical operands
      int keep[kRing];
      int dk = 0;
      for (int k = 0; k < d; ++k) {
        const int j = ring[k];
        const int L = min(e, j), Rr = max(e, j);
        FaceG g;
        face_geometry(X, n, p.Lx, p.Ly, L, Rr, ring[k == 0 ? d - 1 : k - 1],
                      ring[k + 1 == d ? 0 : k + 1], g);
        if (g.A >= 1e-10 * sqrt(g.dx * g.dx + g.dy * g.dy)) keep[dk++] = j;
      }
      for (int k = 0; k < dk; ++k)
        for (int k2 = k + 1; k2 < dk; ++k2) bad |= keep[k] == keep[k2];
      bad |= dk < 3;
      if (dk != d && !bad) {
        for (int k = 0; k < dk; ++k) dst.ring[e * kRing + k] = keep[k];
        for (int k = dk; k < kRing; ++k) dst.ring[e * kRing + k] = -1;
        dst.deg[e] = dk;
      }
      d = dk;
      for (int k = 0; k < d; ++k) ring[k] = keep[k];
      if (bad) {
        dst.deg[e] = 0;
        atomicOr(p.status, 2);
      }
    }
    double geo[kGeo] = {0, 0, 0, 0, 0, 0};
    double vx[kRing], vy[kRing];
    if (!bad) {
      for (int k = 0; k < d; ++k)
        circumcentre(X, n, p.Lx, p.Ly, e, ring[k == 0 ? d - 1 : k - 1], ring[k], e, vx[k], vy[k]);
      polygon_moments(vx, vy, d, geo);
      bad |= !(geo[0] > 0.0) || !(geo[3] * geo[5] - geo[4] * geo[4] > 0.0);
      if (bad) atomicOr(p.status, 2);
    }
    if (bad) {
      d = 0;
      geo[0] = 1.0;
      geo[1] = geo[2] = geo[4] = 0.0;
      geo[3] = geo[5] = 1.0;
    }
    for (int k = 0; k < kGeo; ++k) dst.geo[(size_t)k * n + e] = geo[k];
    (void)xe;
    (void)ye;
    if (FINISH) {
      const double dt = step_size(p);
      T Q[12];
      load12(p.out, n, e, Q);
      const T r0 = p.ua[e], wxT = p.ua[(size_t)3 * n + e], wyT = p.ua[(size_t)6 * n + e];
      double wx = 0.0, wy = 0.0;
      if (p.motion) {
        wx = (double)wxT / (double)r0;
        wy = (double)wyT / (double)r0;
      }
      const MSet& s0 = p.s0;
      const double delx = mimg(xe - s0.x[e], p.Lx) + geo[1] - s0.geo[1 * n + e] - dt * wx;
      const double dely = mimg(ye - s0.x[n + e], p.Ly) + geo[2] - s0.geo[2 * n + e] - dt * wy;
      const double V = geo[0], Mxx = geo[3], Mxy = geo[4], Myy = geo[5];
      const double idet = 1.0 / (Mxx * Myy - Mxy * Mxy);
      T u[12];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const double q0 = (double)Q[3 * v];
        const double qx = (double)Q[3 * v + 1] - delx * q0;
        const double qy = (double)Q[3 * v + 2] - dely * q0;
        u[3 * v] = (T)(q0 / V);
        u[3 * v + 1] = (T)((Myy * qx - Mxy * qy) * idet);
        u[3 * v + 2] = (T)((Mxx * qy - Mxy * qx) * idet);
      }
#pragma unroll
      for (int k = 0; k < 12; ++k) p.out[(size_t)k * n + e] = u[k];
      if (p.dtpart && !bad) {
        // CFL bound 2 V / sum_f A_f (|(v - w) . n_f| + c): w = v when the
        // generators move with the flow, w = 0 when they are held still
        const double rho = (double)u[0], ir = 1.0 / rho;
        const double ux = (double)u[3] * ir, uy = (double)u[6] * ir;
        const double pr =
            ((double)p.gamma - 1.0) * ((double)u[9] - 0.5 * rho * (ux * ux + uy * uy));
        const double cs = sqrt((double)p.gamma * pr * ir);
        double s = 0.0;
        for (int k = 0; k < d; ++k) {
          const int k1 = k + 1 == d ? 0 : k + 1;
          const double ex = vx[k1] - vx[k], ey = vy[k1] - vy[k];
          s += cs * sqrt(ex * ex + ey * ey);
          if (!p.motion) s += fabs(ux * ey - uy * ex);  // A |v . n|, n = (e_y, -e_x) / A
        }
        dtb = 2.0 * V / s;
      }
    }
  }
  if (FINISH && p.dtpart) {
    dtb = wave_min(dtb);
    if ((threadIdx.x & 63) == 0) p.dtpart[e >> 6] = dtb;
  }
}

// ------------------------------------------------------------- update --
// Half-step primitive prediction of a limited cell (Sec. 2.4): values at
// the centroid advanced by h in w[0..3], primitive gradients in gx, gy.
template <typename T>
struct Pred {
  T w[4], gx[4], gy[4];
};

template <typename T>
__device__ __forceinline__ Pred<T> predict(const T* q, T gamma, T h) {
  const T gm1 = gamma - T(1);
  const T rho = q[0], ir = rcp(rho);
  const T vx = q[3] * ir, vy = q[6] * ir;
  const T v2 = vx * vx + vy * vy;
  const T pr = gm1 * (q[9] - T(0.5) * rho * v2);
  Pred<T> o;
  o.gx[0] = q[1];
  o.gy[0] = q[2];
  o.gx[1] = (q[4] - vx * q[1]) * ir;
  o.gy[1] = (q[5] - vx * q[2]) * ir;
  o.gx[2] = (q[7] - vy * q[1]) * ir;
  o.gy[2] = (q[8] - vy * q[2]) * ir;
  o.gx[3] = gm1 * (q[10] - T(0.5) * v2 * q[1] - rho * (vx * o.gx[1] + vy * o.gx[2]));
  o.gy[3] = gm1 * (q[11] - T(0.5) * v2 * q[2] - rho * (vx * o.gy[1] + vy * o.gy[2]));
  const T div = o.gx[1] + o.gy[2];
  const T rho_t = -(vx * o.gx[0] + vy * o.gy[0] + rho * div);
  const T vx_t = -(vx * o.gx[1] + vy * o.gy[1] + o.gx[3] * ir);
  const T vy_t = -(vx * o.gx[2] + vy * o.gy[2] + o.gy[3] * ir);
  const T p_t = -(gamma * pr * div + vx * o.gx[3] + vy * o.gy[3]);
  o.w[0] = rho + h * rho_t;
  o.w[1] = vx + h * vx_t;
  o.w[2] = vy + h * vy_t;
  o.w[3] = pr + h * p_t;
  return o;
}

// Conserved state, boosted into the frame moving with (wx, wy), of the
// predicted primitive polynomial at offset (rx, ry) from the centroid.
template <typename T>
__device__ __forceinline__ void boosted_state(const Pred<T>& c, T rx, T ry, T wx, T wy, T igm1,
                                              T* u) {
  const T rho = c.w[0] + c.gx[0] * rx + c.gy[0] * ry;
  const T vx = c.w[1] + c.gx[1] * rx + c.gy[1] * ry - wx;
  const T vy = c.w[2] + c.gx[2] * rx + c.gy[2] * ry - wy;
  const T pr = c.w[3] + c.gx[3] * rx + c.gy[3] * ry;
  u[0] = rho;
  u[1] = rho * vx;
  u[2] = rho * vy;
  u[3] = pr * igm1 + T(0.5) * rho * (vx * vx + vy * vy);
}

// Lab-frame flux F - U w^T from the flux Fb of the same state in the frame
// moving with w.
template <typename T>
__device__ __forceinline__ void unboost(T* F, T wx, T wy) {
  const T f0 = F[0], f1 = F[1], f2 = F[2];
  F[1] = f1 + f0 * wx;
  F[2] = f2 + f0 * wy;
  F[3] = F[3] + wx * f1 + wy * f2 + T(0.5) * (wx * wx + wy * wy) * f0;
}

// HLL flux along x (Davis speeds).
template <typename T>
__device__ __forceinline__ void hll_x(const T* uL, const T* uR, T gamma, T* F, bool& bad) {
  const T gm1 = gamma - T(1);
  const T irL = rcp(uL[0]), irR = rcp(uR[0]);
  const T vL = uL[1] * irL, vR = uR[1] * irR;
  const T pL = gm1 * (uL[3] - T(0.5) * (uL[1] * vL + uL[2] * uL[2] * irL));
  const T pR = gm1 * (uR[3] - T(0.5) * (uR[1] * vR + uR[2] * uR[2] * irR));
  bad |= !(uL[0] > T(0)) || !(uR[0] > T(0)) || !(pL > T(0)) || !(pR > T(0));
  const T cL = sqrt_pos(gamma * pL * irL), cR = sqrt_pos(gamma * pR * irR);
  const T SL = fmin(vL - cL, vR - cR), SR = fmax(vL + cL, vR + cR);
  T FL[4] = {uL[1], uL[1] * vL + pL, uL[2] * vL, (uL[3] + pL) * vL};
  T FR[4] = {uR[1], uR[1] * vR + pR, uR[2] * vR, (uR[3] + pR) * vR};
  const T inv = rcp(SR - SL);
  T a = SR * inv, b = -SL * inv, c = SL * SR * inv;
  const bool left = SL >= T(0), right = SR <= T(0);
  a = left ? T(1) : (right ? T(0) : a);
  b = left ? T(0) : (right ? T(1) : b);
  c = (left || right) ? T(0) : c;
#pragma unroll
  for (int k = 0; k < 4; ++k) F[k] = fma(a, FL[k], fma(b, FR[k], c * (uR[k] - uL[k])));
}

// Riemann flux along the unit normal (nx, ny): rotate into (normal,
// tangential) components, solve along x, rotate back.
template <typename T, int RS>
__device__ __forceinline__ void riemann_n(const T* uL, const T* uR, T nx, T ny, T gamma, T* F,
                                          bool& bad) {
  T a[4] = {uL[0], uL[1] * nx + uL[2] * ny, uL[2] * nx - uL[1] * ny, uL[3]};
  T b[4] = {uR[0], uR[1] * nx + uR[2] * ny, uR[2] * nx - uR[1] * ny, uR[3]};
  T G[4];
  if (RS == 1)
    exact_flux<T, 0>(a, b, gamma, G, bad);
  else
    hll_x(a, b, gamma, G, bad);
  F[0] = G[0];
  F[1] = G[1] * nx - G[2] * ny;
  F[2] = G[1] * ny + G[2] * nx;
  F[3] = G[3];
}

// The register budget of two waves per SIMD: with the exact solver in FP64
// the kernel needs ~280 registers, and one wave per SIMD cannot hide the
// neighbour gathers behind the divergent Newton loops; under the cap it spills
// ~110 B per lane and runs 20% faster (0.33 -> 0.27 ms at 512^2).  The other
// instantiations fit two or more waves without it.
template <typename T, int RS>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 8)))
void k_mv_upd(PM<T> p) {
  const int e = xcd_remap(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
  if (e >= p.n) return;
  const int n = p.n;
  const double dt = step_size(p);
  const T half = T(0.5 * dt);
  const T gamma = p.gamma, igm1 = rcp(gamma - T(1));
  const MSet& s0 = p.s0;
  const MSet& sh = p.sh;
  const double* Xh = sh.x;
  // interleaved (x, y) positions of the half step and of t^n
  const double2* PH = reinterpret_cast<const double2*>(Xh + 2 * (size_t)n);
  const double2* P0 = reinterpret_cast<const double2*>(s0.x + 2 * (size_t)n);
  bool bad = false;
  T qe[12];
  load12(p.ua, n, e, qe);
  const T wex = p.motion ? qe[3] / qe[0] : T(0), wey = p.motion ? qe[6] / qe[0] : T(0);
  T S0[4] = {T(0), T(0), T(0), T(0)}, Sx[4] = {T(0), T(0), T(0), T(0)},
    Sy[4] = {T(0), T(0), T(0), T(0)};
  const int d = min(sh.deg[e], kRing);
  constexpr double kG = 0.28867513459481288225;  // 1/(2 sqrt 3)
  for (int k = 0; k < d; ++k) {
    const int j = sh.ring[e * kRing + k];
    const int jp = sh.ring[e * kRing + (k == 0 ? d - 1 : k - 1)];
    const int jn = sh.ring[e * kRing + (k + 1 == d ? 0 : k + 1)];
    const int L = min(e, j), R = max(e, j);
    FaceG g;
    face_geometry(Xh, n, p.Lx, p.Ly, L, R, jp, jn, g);
    // both cells' limited polynomials, predicted half a step
    T qL[12], qR[12];
    load12(p.ua, n, L, qL);
    load12(p.ua, n, R, qR);
    const Pred<T> pL = predict(qL, gamma, half), pR = predict(qR, gamma, half);
    const T wLx = p.motion ? qL[3] / qL[0] : T(0), wLy = p.motion ? qL[6] / qL[0] : T(0);
    const T wRx = p.motion ? qR[3] / qR[0] : T(0), wRy = p.motion ? qR[6] / qR[0] : T(0);
    // offsets of L's half-step generator from its t^n centroid, and R's
    const double2 hL = PH[L], hR = PH[R], zL = P0[L], zR = P0[R];
    const double oLx = mimg(hL.x - zL.x, p.Lx) - s0.geo[1 * n + L];
    const double oLy = mimg(hL.y - zL.y, p.Ly) - s0.geo[2 * n + L];
    const double oRx = mimg(hR.x - zR.x, p.Lx) - s0.geo[1 * n + R] - g.dx;
    const double oRy = mimg(hR.y - zR.y, p.Ly) - s0.geo[2 * n + R] - g.dy;
    const double dd = g.dx * g.dx + g.dy * g.dy;
    const T nx = (T)g.nx, ny = (T)g.ny, wq = (T)(0.5 * g.A);
    const double mx = 0.5 * (g.ax + g.bx), my = 0.5 * (g.ay + g.by);
    const double tx = kG * (g.bx - g.ax), ty = kG * (g.by - g.ay);
    const T sg = e == L ? -wq : wq;
#pragma unroll
    for (int q = 0; q < 2; ++q) {
      const double gx = q == 0 ? mx - tx : mx + tx, gy = q == 0 ? my - ty : my + ty;
      // face velocity at the Gauss point: the mean of the generator velocities
      // plus the bisector's normal motion there
      const double sw = ((double)(wLx - wRx) * (gx - 0.5 * g.dx) +
                         (double)(wLy - wRy) * (gy - 0.5 * g.dy)) / dd;
      const T fwx = (T)(0.5 * (double)(wLx + wRx) + sw * g.dx);
      const T fwy = (T)(0.5 * (double)(wLy + wRy) + sw * g.dy);
      const T rLx = (T)(gx + oLx), rLy = (T)(gy + oLy);
      const T rRx = (T)(gx + oRx), rRy = (T)(gy + oRy);
      T uL[4], uR[4], F[4];
      boosted_state(pL, rLx, rLy, fwx, fwy, igm1, uL);
      boosted_state(pR, rRx, rRy, fwx, fwy, igm1, uR);
      riemann_n<T, RS>(uL, uR, nx, ny, gamma, F, bad);
      unboost(F, fwx, fwy);
      const T rx = (e == L ? rLx : rRx) - half * wex;
      const T ry = (e == L ? rLy : rRy) - half * wey;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        S0[v] += sg * F[v];
        Sx[v] += sg * F[v] * rx;
        Sy[v] += sg * F[v] * ry;
      }
    }
  }
  // volume term on the half-step cell's principal-axis rule
  {
    const double Vh = sh.geo[e], a = sh.geo[3 * n + e], b = sh.geo[4 * n + e],
                 c = sh.geo[5 * n + e];
    const double2 he = PH[e], ze = P0[e];
    const double ox = mimg(he.x - ze.x, p.Lx) + sh.geo[1 * n + e] - s0.geo[1 * n + e];
    const double oy = mimg(he.y - ze.y, p.Ly) + sh.geo[2 * n + e] - s0.geo[2 * n + e];
    const double tr = 0.5 * (a + c), disc = sqrt(0.25 * (a - c) * (a - c) + b * b);
    const double lam[2] = {tr + disc, tr - disc};
    double ev[2][2];
    if (b == 0.0) {
      const bool xfirst = a >= c;
      ev[0][0] = xfirst ? 1.0 : 0.0;
      ev[0][1] = xfirst ? 0.0 : 1.0;
      ev[1][0] = xfirst ? 0.0 : 1.0;
      ev[1][1] = xfirst ? 1.0 : 0.0;
    } else {
      for (int k = 0; k < 2; ++k) {
        const double vx = b, vy = lam[k] - a, nn = sqrt(vx * vx + vy * vy);
        ev[k][0] = vx / nn;
        ev[k][1] = vy / nn;
      }
    }
    const Pred<T> pe = predict(qe, gamma, half);
    const T wv = (T)(0.25 * Vh);
    for (int k = 0; k < 2; ++k) {
      const double r = sqrt(2.0 * fmax(lam[k], 0.0) / Vh);
      for (int sgn = -1; sgn <= 1; sgn += 2) {
        const T rx = (T)(ox + sgn * r * ev[k][0]), ry = (T)(oy + sgn * r * ev[k][1]);
        T u[4];
        boosted_state(pe, rx, ry, wex, wey, igm1, u);
        const T ir = rcp(u[0]), vx = u[1] * ir, vy = u[2] * ir;
        const T pr = (gamma - T(1)) * (u[3] - T(0.5) * (u[1] * vx + u[2] * vy));
        bad |= !(u[0] > T(0)) || !(pr > T(0));
        T Fx[4] = {u[1], u[1] * vx + pr, u[2] * vx, (u[3] + pr) * vx};
        T Fy[4] = {u[2], u[1] * vy, u[2] * vy + pr, (u[3] + pr) * vy};
        unboost(Fx, wex, wey);
        unboost(Fy, wex, wey);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          Sx[v] += wv * Fx[v];
          Sy[v] += wv * Fy[v];
        }
      }
    }
  }
  // totals and moments about the carried origin
  const T V0 = (T)s0.geo[e], Mxx = (T)s0.geo[3 * n + e], Mxy = (T)s0.geo[4 * n + e],
          Myy = (T)s0.geo[5 * n + e];
  const T tdt = (T)dt;
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    p.out[(size_t)(3 * v) * n + e] = V0 * qe[3 * v] + tdt * S0[v];
    p.out[(size_t)(3 * v + 1) * n + e] = Mxx * qe[3 * v + 1] + Mxy * qe[3 * v + 2] + tdt * Sx[v];
    p.out[(size_t)(3 * v + 2) * n + e] = Mxy * qe[3 * v + 1] + Myy * qe[3 * v + 2] + tdt * Sy[v];
  }
  if (bad || !(qe[0] > T(0))) atomicOr(p.status, 1);
}

// CFL bound on the mesh of t^n (dg_cfl_dt).
template <typename T>
__global__ __launch_bounds__(256) void k_mv_cfl(PM<T> p) {
  const int e = xcd_remap(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
  double dtb = 1e300;
  if (e < p.n) {
    const int n = p.n;
    int nb[kRing];
    double vx[kRing], vy[kRing];
    const int d = cell_polygon(p.s0, n, p.Lx, p.Ly, e, vx, vy, nb);
    const double rho = (double)p.in[e], ir = 1.0 / rho;
    const double ux = (double)p.in[(size_t)3 * n + e] * ir, uy = (double)p.in[(size_t)6 * n + e] * ir;
    const double pr =
        ((double)p.gamma - 1.0) * ((double)p.in[(size_t)9 * n + e] - 0.5 * rho * (ux * ux + uy * uy));
    const double cs = sqrt((double)p.gamma * pr * ir);
    double s = 0.0;
    for (int k = 0; k < d; ++k) {
      const int k1 = k + 1 == d ? 0 : k + 1;
      const double ex = vx[k1] - vx[k], ey = vy[k1] - vy[k];
      s += cs * sqrt(ex * ex + ey * ey);
      if (!p.motion) s += fabs(ux * ey - uy * ex);
    }
    dtb = 2.0 * p.s0.geo[e] / s;
  }
  dtb = wave_min(dtb);
  if ((threadIdx.x & 63) == 0) p.dtpart[e >> 6] = dtb;
}

template <typename T>
PM<T> make_params(const dg_mesh* m, const void* in, void* out) {
  const MVDev& v = *m->mvd;
  PM<T> p;
  std::memset(&p, 0, sizeof(p));
  p.in = static_cast<const T*>(in);
  p.ua = static_cast<const T*>(v.ua);
  p.ua_out = static_cast<T*>(v.ua);
  p.out = static_cast<T*>(out);
  p.status = m->status;
  p.n = v.n;
  p.Lx = v.box[0];
  p.Ly = v.box[1];
  p.gamma = (T)m->cfg.gamma;
  p.motion = v.motion;
  p.cand_cap = v.cand_cap;
  p.s0 = MSet{v.pos[v.cur], v.ring[v.cur], v.deg[v.cur], v.geo[v.cur]};
  p.sh = MSet{v.pos[1], v.ring[1], v.deg[1], v.geo[1]};
  p.xh = v.pos[1];
  p.x1 = v.pos[v.nxt];
  return p;
}

template <typename T>
hipError_t lim_launch(const PM<T>& p, int lim, hipStream_t s) {
  const dim3 g((p.n + 255) / 256), b(256);
  if (lim == DG_LIMITER_WENO)
    hipLaunchKernelGGL((k_mv_lim<T, 2>), g, b, 0, s, p);
  else if (lim == DG_LIMITER_MINMOD)
    hipLaunchKernelGGL((k_mv_lim<T, 1>), g, b, 0, s, p);
  else
    hipLaunchKernelGGL((k_mv_lim<T, 0>), g, b, 0, s, p);
  return hipGetLastError();
}

template <typename T>
hipError_t step_t(dg_mesh* m, const void* in, void* out, const double* dt_dev, double dt_host,
                  bool want_dt, hipStream_t s) {
  MVDev& v = *m->mvd;
  PM<T> p = make_params<T>(m, in, out);
  p.dt_dev = dt_dev;
  p.dt_host = dt_host;
  p.write_pos = 1;
  const dim3 g((p.n + 255) / 256), b(256);
  // per-phase events go straight into the record (launch_moving drops the
  // ones of a step that fails)
  auto mark = [&]() {
    if (!v.timing) return hipSuccess;
    hipEvent_t ev;
    hipError_t r = hipEventCreate(&ev);
    if (r != hipSuccess) return r;
    v.ev.push_back(ev);
    return hipEventRecord(ev, s);
  };
  hipError_t e = mark();
  if (e == hipSuccess) e = lim_launch(p, m->cfg.limiter, s);
  if (e == hipSuccess) e = mark();
  if (e != hipSuccess) return e;
  // mesh of the half-step generators (candidates from t^n)
  const MOut half{v.pos[1], v.ring[1], v.deg[1], v.geo[1]};
  const dim3 gw((p.n + kWalkThreads - 1) / kWalkThreads), bw(kWalkThreads);
  hipLaunchKernelGGL((k_mv_walk<T>), gw, bw, 0, s, p, p.s0, half);
  hipLaunchKernelGGL((k_mv_geom<T, false>), g, b, 0, s, p, half);
  e = mark();
  if (e != hipSuccess) return e;
  if (m->cfg.flux == DG_FLUX_EXACT)
    hipLaunchKernelGGL((k_mv_upd<T, 1>), g, b, 0, s, p);
  else
    hipLaunchKernelGGL((k_mv_upd<T, 0>), g, b, 0, s, p);
  e = mark();
  if (e != hipSuccess) return e;
  // mesh of t^{n+1} (candidates from the half step) and the new state
  if (want_dt) p.dtpart = m->dtpart;
  const MOut next{v.pos[v.nxt], v.ring[v.nxt], v.deg[v.nxt], v.geo[v.nxt]};
  hipLaunchKernelGGL((k_mv_walk<T>), gw, bw, 0, s, p, p.sh, next);
  hipLaunchKernelGGL((k_mv_geom<T, true>), g, b, 0, s, p, next);
  e = hipGetLastError();
  if (e == hipSuccess) std::swap(v.cur, v.nxt);
  return e;
}

}  // namespace

hipError_t launch_min_finalize(const double* part, int n, double cfl, double* dt, hipStream_t s);

hipError_t launch_moving(dg_mesh* m, int mode, const void* in, void* out, const double* dt_dev,
                         double dt_host, double cfl, double* dt_next, hipStream_t s) {
  const bool f64 = m->cfg.precision == DG_FP64;
  if (mode == kLimit) {
    if (f64) {
      PM<double> p = make_params<double>(m, in, nullptr);
      p.ua_out = static_cast<double*>(out);
      return lim_launch(p, m->cfg.limiter, s);
    }
    PM<float> p = make_params<float>(m, in, nullptr);
    p.ua_out = static_cast<float*>(out);
    return lim_launch(p, m->cfg.limiter, s);
  }
  if (mode != kMH) return hipErrorInvalidValue;
  MVDev& v = *m->mvd;
  const size_t ev0 = v.ev.size();
  hipError_t e = f64 ? step_t<double>(m, in, out, dt_dev, dt_host, dt_next != nullptr, s)
                     : step_t<float>(m, in, out, dt_dev, dt_host, dt_next != nullptr, s);
  if (e == hipSuccess && dt_next)
    e = launch_min_finalize(m->dtpart, (int)((m->ncells + 63) / 64), cfl, dt_next, s);
  if (e == hipSuccess && v.timing) {
    // the fifth event closes the new-mesh kernel and the dt reduction
    hipEvent_t last;
    e = hipEventCreate(&last);
    if (e == hipSuccess) {
      v.ev.push_back(last);
      e = hipEventRecord(last, s);
    }
  }
  if (e != hipSuccess) {
    // a failed step leaves no partial record: the timings stay in groups of five
    for (size_t k = ev0; k < v.ev.size(); ++k) (void)hipEventDestroy(v.ev[k]);
    v.ev.resize(ev0);
  }
  return e;
}

hipError_t launch_moving_cfl(const dg_mesh* m, const void* U, double cfl, double* dt_dev,
                             hipStream_t s) {
  const dim3 g((m->ncells + 255) / 256), b(256);
  if (m->cfg.precision == DG_FP64) {
    PM<double> p = make_params<double>(m, U, nullptr);
    p.dtpart = m->dtpart;
    hipLaunchKernelGGL((k_mv_cfl<double>), g, b, 0, s, p);
  } else {
    PM<float> p = make_params<float>(m, U, nullptr);
    p.dtpart = m->dtpart;
    hipLaunchKernelGGL((k_mv_cfl<float>), g, b, 0, s, p);
  }
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return e;
  return launch_min_finalize(m->dtpart, (int)((m->ncells + 63) / 64), cfl, dt_dev, s);
}

// ------------------------------------------------------------ host setup --
void moving_destroy(dg_mesh* m) {
  if (!m->mvd) return;
  MVDev& v = *m->mvd;
  for (hipEvent_t e : v.ev) (void)hipEventDestroy(e);
  for (int k = 0; k < 3; ++k) {
    (void)hipFree(v.pos[k]);
    (void)hipFree(v.ring[k]);
    (void)hipFree(v.deg[k]);
    (void)hipFree(v.geo[k]);
  }
  (void)hipFree(v.ua);
  delete m->mvd;
  m->mvd = nullptr;
}

dg_status moving_create(dg_mesh* m, const dg_mesh_desc* d) {
  const int64_t n = d->ncells, nf = d->nfaces;
  if (n < 64 || n > (1 << 26) || nf < 1) {
    set_error("dg_mesh_create: a moving mesh needs 64 <= ncells <= 2^26 and its initial faces");
    return DG_EINVAL;
  }
  if (!d->generators || !d->face_cells || !d->face_shift) {
    set_error("dg_mesh_create: a moving mesh needs generators, face_cells and face_shift");
    return DG_EINVAL;
  }
  const double Lx = d->box[0], Ly = d->box[1];
  if (!(Lx > 0) || !(Ly > 0) || !std::isfinite(Lx) || !std::isfinite(Ly)) {
    set_error("dg_mesh_create: moving mesh box must be positive");
    return DG_EINVAL;
  }
  std::vector<double> pos(4 * n);
  for (int64_t i = 0; i < n; ++i) {
    const double x = d->generators[2 * i], y = d->generators[2 * i + 1];
    if (!std::isfinite(x) || !std::isfinite(y) || x < 0 || x >= Lx || y < 0 || y >= Ly) {
      set_error("dg_mesh_create: generator " + std::to_string(i) + " is not inside [0, box)");
      return DG_EINVAL;
    }
    pos[i] = x;
    pos[n + i] = y;
    pos[2 * n + 2 * i] = x;
    pos[2 * n + 2 * i + 1] = y;
  }
  // initial rings: each cell's face neighbours sorted by angle
  std::vector<std::vector<std::pair<double, int>>> nbr(n);
  for (int64_t f = 0; f < nf; ++f) {
    const int L = d->face_cells[2 * f], R = d->face_cells[2 * f + 1];
    if (L < 0 || L >= n || R < 0 || R >= n || L == R) {
      set_error("dg_mesh_create: initial face " + std::to_string(f) + " has bad cells");
      return DG_EINVAL;
    }
    const double dx = pos[R] + d->face_shift[2 * f] * Lx - pos[L];
    const double dy = pos[n + R] + d->face_shift[2 * f + 1] * Ly - pos[n + L];
    nbr[L].push_back({std::atan2(dy, dx), R});
    nbr[R].push_back({std::atan2(-dy, -dx), L});
  }
  std::vector<int> ring((size_t)n * kRing, -1), deg(n);
  for (int64_t i = 0; i < n; ++i) {
    auto& v = nbr[i];
    std::sort(v.begin(), v.end());
    if (v.size() < 3 || v.size() > (size_t)kRing) {
      set_error("dg_mesh_create: cell " + std::to_string(i) + " has " + std::to_string(v.size()) +
                " faces (3 to 16 supported)");
      return DG_EINVAL;
    }
    for (size_t k = 0; k < v.size(); ++k) {
      for (size_t k2 = 0; k2 < k; ++k2)
        if (v[k2].second == v[k].second) {
          set_error("dg_mesh_create: cells " + std::to_string(i) + " and " +
                    std::to_string(v[k].second) + " share two faces (mesh too coarse)");
          return DG_EINVAL;
        }
      ring[i * kRing + k] = v[k].second;
    }
    deg[i] = (int)v.size();
  }
  m->mvd = new (std::nothrow) MVDev();
  if (!m->mvd) {
    set_error("dg_mesh_create: out of host memory");
    return DG_ENOMEM;
  }
  MVDev& v = *m->mvd;
  v.n = (int)n;
  v.box[0] = Lx;
  v.box[1] = Ly;
  v.motion = 1;
  v.cur = 0;
  v.nxt = 2;
  // DG_MOVING_CANDIDATES caps the walk's LDS candidate list (tests use it to
  // drive every cell through the streaming path)
  if (const char* env = std::getenv("DG_MOVING_CANDIDATES"))
    v.cand_cap = std::max(0, std::min(kCand, std::atoi(env)));
  hipError_t e = hipSuccess;
  for (int k = 0; k < 3 && e == hipSuccess; ++k) {
    e = hipMalloc((void**)&v.pos[k], sizeof(double) * 4 * n);
    if (e == hipSuccess) e = hipMalloc((void**)&v.ring[k], sizeof(int) * kRing * n);
    if (e == hipSuccess) e = hipMalloc((void**)&v.deg[k], sizeof(int) * n);
    if (e == hipSuccess) e = hipMalloc((void**)&v.geo[k], sizeof(double) * kGeo * n);
  }
  if (e == hipSuccess) e = hipMalloc(&v.ua, m->elem * 12 * n);
  if (e == hipSuccess)
    e = hipMemcpy(v.pos[0], pos.data(), sizeof(double) * 4 * n, hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(v.ring[1], ring.data(), sizeof(int) * kRing * n, hipMemcpyHostToDevice);
  if (e == hipSuccess) e = hipMemcpy(v.deg[1], deg.data(), sizeof(int) * n, hipMemcpyHostToDevice);
  if (e != hipSuccess) {
    moving_destroy(m);
    return hip_fail(e, "dg_mesh_create: moving mesh upload");
  }
  return DG_OK;
}

// Build the mesh of t^0 from the uploaded rings (set 1) and positions (set 0);
// the caller checks the status word afterwards.
hipError_t moving_init(dg_mesh* m) {
  MVDev& v = *m->mvd;
  PM<double> p;
  std::memset(&p, 0, sizeof(p));
  p.status = m->status;
  p.cand_cap = v.cand_cap;
  p.n = v.n;
  p.Lx = v.box[0];
  p.Ly = v.box[1];
  p.gamma = m->cfg.gamma;
  const dim3 g((v.n + 255) / 256), b(256);
  const MOut first{v.pos[0], v.ring[0], v.deg[0], v.geo[0]};
  const dim3 gw((v.n + kWalkThreads - 1) / kWalkThreads), bw(kWalkThreads);
  hipLaunchKernelGGL((k_mv_walk<double>), gw, bw, 0, nullptr, p,
                     MSet{v.pos[0], v.ring[1], v.deg[1], v.geo[1]}, first);
  hipLaunchKernelGGL((k_mv_geom<double, false>), g, b, 0, nullptr, p, first);
  return hipGetLastError();
}

}  // namespace dg

namespace dg {

// Host copy of the current mesh (synchronous).  Any output may be NULL.
int moving_read(const dg_mesh* m, double* gen, double* vol, double* cen, int32_t* ring,
                int32_t* deg) {
  const MVDev& v = *m->mvd;
  const int n = v.n;
  std::vector<double> pos(2 * (size_t)n), geo((size_t)kGeo * n);
  hipError_t e = hipDeviceSynchronize();
  if (e == hipSuccess)
    e = hipMemcpy(pos.data(), v.pos[v.cur], sizeof(double) * 2 * n, hipMemcpyDeviceToHost);
  if (e == hipSuccess)
    e = hipMemcpy(geo.data(), v.geo[v.cur], sizeof(double) * kGeo * n, hipMemcpyDeviceToHost);
  if (e == hipSuccess && ring)
    e = hipMemcpy(ring, v.ring[v.cur], sizeof(int) * kRing * n, hipMemcpyDeviceToHost);
  if (e == hipSuccess && deg)
    e = hipMemcpy(deg, v.deg[v.cur], sizeof(int) * n, hipMemcpyDeviceToHost);
  if (e != hipSuccess) return (int)e;
  for (int i = 0; i < n; ++i) {
    if (gen) {
      gen[2 * i] = pos[i];
      gen[2 * i + 1] = pos[n + i];
    }
    if (vol) vol[i] = geo[i];
    if (cen) {
      cen[2 * i] = pos[i] + geo[(size_t)n + i];
      cen[2 * i + 1] = pos[n + i] + geo[2 * (size_t)n + i];
    }
  }
  return 0;
}

void moving_set_motion(dg_mesh* m, int motion) { m->mvd->motion = motion ? 1 : 0; }

static void drop_events(MVDev& v) {
  for (hipEvent_t e : v.ev) (void)hipEventDestroy(e);
  v.ev.clear();
}

void moving_set_timing(dg_mesh* m, int on) {
  drop_events(*m->mvd);
  m->mvd->timing = on != 0;
}

// Average durations (ms) of the four kernels of the timed steps since the
// last call, then a fresh record.
int moving_timing(dg_mesh* m, double* avg_ms, int* nsteps) {
  MVDev& v = *m->mvd;
  hipError_t e = hipDeviceSynchronize();
  const int ns = (int)(v.ev.size() / 5);
  double acc[4] = {0, 0, 0, 0};
  for (int k = 0; k < ns && e == hipSuccess; ++k)
    for (int j = 0; j < 4 && e == hipSuccess; ++j) {
      float ms = 0.0f;
      e = hipEventElapsedTime(&ms, v.ev[5 * k + j], v.ev[5 * k + j + 1]);
      acc[j] += ms;
    }
  drop_events(v);
  if (e != hipSuccess) return (int)e;
  for (int j = 0; j < 4; ++j) avg_ms[j] = ns ? acc[j] / ns : 0.0;
  if (nsteps) *nsteps = ns;
  return 0;
}

}  // namespace dg
