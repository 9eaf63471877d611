// Discrete adjoint of the 2D Euler Cartesian SSP-RK2 step (vector-Jacobian
// products of the exact discrete step, dt frozen, the limiter and the HLL wave
// speeds following the branch the forward computation takes).
//
// Forward step (Sec. 2.2 operator L, Sec. 2.5 limiter Pi):
//   Ua = Pi(U);  V1 = Ua + dt L(Ua);  Ub = Pi(V1);  U' = Ua/2 + (Ub + dt L(Ub))/2
// Backward, given lam' = dJ/dU':
//   lam_V1 = Pi_V1^T [ lam'/2 + (dt/2) L_Ub^T lam' ]                 (stage 2)
//   lam    = Pi_U^T  [ lam_V1 + dt L_Ua^T lam_V1 + lam'/2 ]            (stage 1)
// so both stages are one "adjoint stage"
//   out = Pi_P^T lamW,   lamW = c_id lam + c_L (dL/dW)^T lam + c_extra extra,
//   W = Pi(P),
// and each adjoint stage is one kernel (k_adj_row_*), laid out like the forward
// stage kernels: one wave owns 58 columns (lanes 3..60; three halo lanes on
// each side) and marches up `rows` rows with its rows in registers.  x
// neighbours come from DPP lane shifts, y neighbours from the row window; no
// LDS, no barriers, no atomics.  Per row the wave
//   S1  limits P (W and the limiter's branch data) one row behind the loads,
//   S2  solves the VJP of the row's -x faces (the left side's share goes to
//       the left lane by a lane shift), of the y face below it and of the
//       volume term, accumulating lamW of that row and of the row below,
//   S3  finishes lamW two rows behind, applies the cell's own part of the
//       limiter transpose (gradient scale, D and dm branches) and writes the
//       gradient adjoints,
//   S4  three rows behind, adds to each mean adjoint what the cell received as
//       its neighbours' arg-max / arg-min, and writes it.
// A tile of R output rows marches R + 4 rows.
//
// Ties (min/max arguments, the limiter's branch) take the first argument in
// the order self, -x, +x, -y, +y, as the CPU oracle's dual numbers do.
#include <hip/hip_runtime.h>

#include "dg_internal.h"
#include "dg_math.h"

namespace dg {
namespace {

constexpr int kLanesA = 64;
constexpr int kHaloA = 3;
static_assert(kLanesA - 2 * kHaloA == kAdjCols, "adjoint tile width");

template <typename T>
struct PA {
  const T* __restrict__ P;     // pre-limit state of the stage
  const T* __restrict__ lam;   // adjoint of the stage output
  const T* __restrict__ extra; // added to lamW with weight c_extra (may be NULL)
  T* __restrict__ out;
  const AdjInst* inst;
  const int* tile_inst;        // tile -> instance (batched); NULL: one instance
  const double* dt_dev;        // per instance (batched) or one value; NULL: dt_host
  double dt_host;
  double c_id, c_L_over_dt;    // c_L = c_L_over_dt * dt
  double c_extra;
  int nc;                      // global stride of the coefficient arrays
  int ntiles;
  T gamma;
};

__device__ __forceinline__ int wrapi(int a, int n) {
  a %= n;
  return a < 0 ? a + n : a;
}

// ------------------------------------------------------------ forward bits --
// Limiter coefficient of one variable on a Cartesian cell, with its branch
// data: the arg-max / arg-min neighbour codes (0 self, 1 -x, 2 +x, 3 -y, 4 +y),
// whether D came from the max side, and whether dm came from the x axis.
template <typename T>
struct LimInfo {
  T alpha, D, dm;
  int amax, amin;
  bool active, dplus, xaxis;
};

template <typename T>
__device__ __forceinline__ LimInfo<T> lim_info(const T* nb, T gx, T gy, T hx2, T hy2) {
  // nb: means of self, -x, +x, -y, +y
  LimInfo<T> r;
  T hi = nb[0], lo = nb[0];
  r.amax = 0;
  r.amin = 0;
#pragma unroll
  for (int k = 1; k < 5; ++k) {
    if (nb[k] > hi) {
      hi = nb[k];
      r.amax = k;
    }
    if (nb[k] < lo) {
      lo = nb[k];
      r.amin = k;
    }
  }
  const T dp = hi - nb[0], dmn = nb[0] - lo;
  r.dplus = dp < dmn;
  r.D = r.dplus ? dp : dmn;
  const T ax = fabs(gx) * hx2, ay = fabs(gy) * hy2;
  r.xaxis = ax >= ay;
  r.dm = r.xaxis ? ax : ay;
  r.active = r.dm > r.D;
  r.alpha = r.active ? div_small(r.D, r.dm) : T(1);
  return r;
}

// HLL along axis AX and its VJP: given lamF (4), accumulates lamL, lamR (4).
template <typename T, int AX>
__device__ __forceinline__ void hll_vjp(const T* uL, const T* uR, T gamma, const T* lamF, T* lamL,
                                        T* lamR) {
  const T gm1 = gamma - T(1);
  const T* u[2] = {uL, uR};
  T ir[2], vx[2], vy[2], p[2], c[2], vn[2], Fs[2][4];
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    ir[s] = rcp(u[s][0]);
    vx[s] = u[s][1] * ir[s];
    vy[s] = u[s][2] * ir[s];
    p[s] = gm1 * (u[s][3] - T(0.5) * (u[s][1] * vx[s] + u[s][2] * vy[s]));
    c[s] = sqrt_pos(gamma * p[s] * ir[s]);
    vn[s] = AX == 0 ? vx[s] : vy[s];
    Fs[s][0] = u[s][0] * vn[s];
    Fs[s][1] = u[s][1] * vn[s] + (AX == 0 ? p[s] : T(0));
    Fs[s][2] = u[s][2] * vn[s] + (AX == 1 ? p[s] : T(0));
    Fs[s][3] = (u[s][3] + p[s]) * vn[s];
  }
  const T a1 = vn[0] - c[0], a2 = vn[1] - c[1];
  const T b1 = vn[0] + c[0], b2 = vn[1] + c[1];
  const bool slR = a2 < a1;   // S_L from the right state (ties: left)
  const bool srR = b2 > b1;   // S_R from the right state (ties: left)
  const T SL = slR ? a2 : a1, SR = srR ? b2 : b1;
  T lFs[2][4];
  T lvn[2] = {T(0), T(0)}, lc[2] = {T(0), T(0)};
  T lu[2][4];
#pragma unroll
  for (int s = 0; s < 2; ++s)
#pragma unroll
    for (int k = 0; k < 4; ++k) lu[s][k] = T(0);
  if (SL >= T(0)) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      lFs[0][k] = lamF[k];
      lFs[1][k] = T(0);
    }
  } else if (SR <= T(0)) {
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      lFs[0][k] = T(0);
      lFs[1][k] = lamF[k];
    }
  } else {
    const T inv = rcp(SR - SL);
    T lSL = T(0), lSR = T(0);
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const T du = u[1][k] - u[0][k];
      const T F = (SR * Fs[0][k] - SL * Fs[1][k] + SL * SR * du) * inv;
      lFs[0][k] = SR * inv * lamF[k];
      lFs[1][k] = -SL * inv * lamF[k];
      const T ld = SL * SR * inv * lamF[k];
      lu[1][k] += ld;
      lu[0][k] -= ld;
      lSR += lamF[k] * (Fs[0][k] + SL * du - F) * inv;
      lSL += lamF[k] * (F - Fs[1][k] + SR * du) * inv;
    }
    if (slR) {
      lvn[1] += lSL;
      lc[1] -= lSL;
    } else {
      lvn[0] += lSL;
      lc[0] -= lSL;
    }
    if (srR) {
      lvn[1] += lSR;
      lc[1] += lSR;
    } else {
      lvn[0] += lSR;
      lc[0] += lSR;
    }
  }
#pragma unroll
  for (int s = 0; s < 2; ++s) {
    // F = [rho vn, mx vn + dx p, my vn + dy p, (E + p) vn]
    T lp = (AX == 0 ? lFs[s][1] : lFs[s][2]) + lFs[s][3] * vn[s];
    lvn[s] += lFs[s][0] * u[s][0] + lFs[s][1] * u[s][1] + lFs[s][2] * u[s][2] +
              lFs[s][3] * (u[s][3] + p[s]);
    lu[s][0] += lFs[s][0] * vn[s];
    lu[s][1] += lFs[s][1] * vn[s];
    lu[s][2] += lFs[s][2] * vn[s];
    lu[s][3] += lFs[s][3] * vn[s];
    // c = sqrt(gamma p ir)
    T lir = T(0);
    if (lc[s] != T(0)) {
      const T h = T(0.5) * gamma * rcp(c[s]);
      lp += lc[s] * h * ir[s];
      lir += lc[s] * h * p[s];
    }
    T lvx = AX == 0 ? lvn[s] : T(0), lvy = AX == 1 ? lvn[s] : T(0);
    // p = gm1 (E - (mx vx + my vy)/2)
    lu[s][3] += gm1 * lp;
    lu[s][1] -= T(0.5) * gm1 * lp * vx[s];
    lvx -= T(0.5) * gm1 * lp * u[s][1];
    lu[s][2] -= T(0.5) * gm1 * lp * vy[s];
    lvy -= T(0.5) * gm1 * lp * u[s][2];
    // vx = mx ir, vy = my ir
    lu[s][1] += lvx * ir[s];
    lu[s][2] += lvy * ir[s];
    lir += lvx * u[s][1] + lvy * u[s][2];
    lu[s][0] -= lir * ir[s] * ir[s];
  }
#pragma unroll
  for (int k = 0; k < 4; ++k) {
    lamL[k] += lu[0][k];
    lamR[k] += lu[1][k];
  }
}

// VJP of the two volume flux rows at one state: a = lam F_x, b = lam F_y.
template <typename T>
__device__ __forceinline__ void flux_xy_vjp(const T* u, T gamma, const T* a, const T* b, T* lu) {
  const T gm1 = gamma - T(1);
  const T ir = rcp(u[0]);
  const T vx = u[1] * ir, vy = u[2] * ir;
  const T p = gm1 * (u[3] - T(0.5) * (u[1] * vx + u[2] * vy));
  T lmx = a[0] + a[1] * vx + b[1] * vy;
  T lmy = a[2] * vx + b[0] + b[2] * vy;
  T lE = a[3] * vx + b[3] * vy;
  const T lp = a[1] + a[3] * vx + b[2] + b[3] * vy;
  T lvx = a[1] * u[1] + a[2] * u[2] + a[3] * (u[3] + p);
  T lvy = b[1] * u[1] + b[2] * u[2] + b[3] * (u[3] + p);
  lE += gm1 * lp;
  lmx -= T(0.5) * gm1 * lp * vx;
  lvx -= T(0.5) * gm1 * lp * u[1];
  lmy -= T(0.5) * gm1 * lp * vy;
  lvy -= T(0.5) * gm1 * lp * u[2];
  lmx += lvx * ir;
  lmy += lvy * ir;
  const T lir = lvx * u[1] + lvy * u[2];
  lu[0] += -lir * ir * ir;
  lu[1] += lmx;
  lu[2] += lmy;
  lu[3] += lE;
}

// ------------------------------------------------------------ row kernel --
// Limiter branch data of one row (per lane): alpha per variable, the
// arg-max / arg-min codes (6 bits per variable) and the active / D-from-max /
// dm-from-x flags (3 bits per variable).  dm is recomputed from the gradient
// and the axis flag when needed.
template <typename T>
struct LimRow {
  T alpha[4];
  unsigned code, flag;
};

// Limiter transpose data of one row: what the cell routes to its arg-max and
// arg-min means, and the codes naming them.
template <typename T>
struct PitRow {
  T lhi[4], llo[4];
  unsigned code;
};

// Array k of a state: a uniform array base (k * nc) plus the cell's 32-bit
// byte offset.
template <typename T>
__device__ __forceinline__ T ld(const T* __restrict__ U, int nc, int k, unsigned off) {
  return *reinterpret_cast<const T*>(reinterpret_cast<const char*>(U + (size_t)k * nc) + off);
}
template <typename T>
__device__ __forceinline__ void st(T* __restrict__ U, int nc, int k, unsigned off, T v) {
  *reinterpret_cast<T*>(reinterpret_cast<char*>(U + (size_t)k * nc) + off) = v;
}

__device__ __forceinline__ unsigned lane_up_u(unsigned v) { return (unsigned)dpp_shr1((int)v); }
__device__ __forceinline__ unsigned lane_down_u(unsigned v) { return (unsigned)dpp_shl1((int)v); }

template <typename T, bool LIM>
__device__ __forceinline__ void adj_row_body(const PA<T>& p) {
  const int lane = threadIdx.x & (kLanesA - 1);
  const int wave = __builtin_amdgcn_readfirstlane(xcd_remap(blockIdx.x, gridDim.x) * 4 +
                                                  (threadIdx.x >> 6));
  if (wave >= p.ntiles) return;
  const int ii = p.tile_inst ? __builtin_amdgcn_readfirstlane(p.tile_inst[wave]) : 0;
  const AdjInst& in = p.inst[ii];
  const int nx = in.nx, ny = in.ny, nc = p.nc, rows = in.rows;
  const int t = wave - in.tx0;
  const int tx = t % in.tiles_x, ty = t / in.tiles_x;
  const int colu = tx * kAdjCols + lane - kHaloA;
  const bool own = lane >= kHaloA && lane < kHaloA + kAdjCols && colu < nx;
  const int col = wrapi(colu, nx);
  const int y0 = ty * rows, y1 = min(y0 + rows, ny);
  const T* __restrict__ P = p.P + in.off;
  const T* __restrict__ L = p.lam + in.off;
  const T* __restrict__ X = p.extra ? p.extra + in.off : nullptr;
  T* __restrict__ O = p.out + in.off;
  const T hx = (T)in.hx, hy = (T)in.hy;
  const T hx2 = T(0.5) * hx, hy2 = T(0.5) * hy;
  const T s3 = T(1.7320508075688772);
  const T qx = hx2 / s3, qy = hy2 / s3;
  const T cmx = T(0.5) / hx, cmy = T(0.5) / hy, cgx = T(3) / (hx * hx), cgy = T(3) / (hy * hy),
          ccr = s3 / (hx * hy);
  const double dt = p.dt_dev ? p.dt_dev[ii] : p.dt_host;
  const T cI = (T)p.c_id, cL = (T)(p.c_L_over_dt * dt), cX = (T)p.c_extra;
  const T gam = p.gamma;
  auto roff = [&](int r) { return (unsigned)(wrapi(r, ny) * nx + col) * (unsigned)sizeof(T); };

  // Row window (rows relative to the iteration j): means m2 = j-2, m1 = j-1,
  // m0 = j (mn = j+1 in flight); gradients g2 = j-2, g1 = j-1 (gn = j in
  // flight); adjoint l2 = j-2, l1 = j-1 (ln = j in flight); extra x1 = j-1.
  T m2[4], m1[4], m0[4], mn[4];
  T g2[8], g1[8], gn[8];
  T l2[12], l1[12], ln[12], x1[12], xn[12];
  LimRow<T> lr2, lr1;
  T acc2[12], acc1[12];
  PitRow<T> pr4, pr3;
  T own3[4];
  const int jb = y0 - 1, je = y1 + 2;
  {
    const unsigned o3 = roff(jb - 2), o2 = roff(jb - 1), o1 = roff(jb);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      m1[v] = ld(P, nc, 3 * v, o3);  // rotated into m2 below (row jb-2)
      m0[v] = ld(P, nc, 3 * v, o2);  // row jb-1
      mn[v] = ld(P, nc, 3 * v, o1);  // row jb
      gn[2 * v] = ld(P, nc, 3 * v + 1, o2);
      gn[2 * v + 1] = ld(P, nc, 3 * v + 2, o2);
    }
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      ln[k] = ld(L, nc, k, o2);
      xn[k] = T(0);
      l1[k] = T(0);
      acc1[k] = T(0);
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      g1[2 * v] = g1[2 * v + 1] = T(0);
      lr1.alpha[v] = T(1);
      pr3.lhi[v] = pr3.llo[v] = T(0);
      own3[v] = T(0);
    }
    lr1.code = lr1.flag = 0;
    pr3.code = 0;
  }

  for (int j = jb; j <= je; ++j) {
    // rotate the window: arrivals of the previous iteration's loads
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      m2[v] = m1[v];
      m1[v] = m0[v];
      m0[v] = mn[v];
    }
#pragma unroll
    for (int k = 0; k < 8; ++k) {
      g2[k] = g1[k];
      g1[k] = gn[k];
    }
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      l2[k] = l1[k];
      l1[k] = ln[k];
      x1[k] = xn[k];
      acc2[k] = acc1[k];
    }
    lr2 = lr1;
    const int r1 = j - 1;
    const bool s2_cell = r1 >= y0 - 1 && r1 <= y1;
    if (s2_cell) {
#pragma unroll
      for (int k = 0; k < 12; ++k) acc1[k] = cI * l1[k] + cX * x1[k];
    }
    // issue this iteration's loads (used from the next iteration on)
    if (j < je) {
      const unsigned o = roff(j + 1);
#pragma unroll
      for (int v = 0; v < 4; ++v) mn[v] = ld(P, nc, 3 * v, o);
    }
    if (j <= y1 + 1) {
      const unsigned o = roff(j);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        gn[2 * v] = ld(P, nc, 3 * v + 1, o);
        gn[2 * v + 1] = ld(P, nc, 3 * v + 2, o);
      }
#pragma unroll
      for (int k = 0; k < 12; ++k) ln[k] = ld(L, nc, k, o);
      if (X && j <= y1) {
#pragma unroll
        for (int k = 0; k < 12; ++k) xn[k] = ld(X, nc, k, o);
      }
    }

    // S1: limit row j-1 (W = mean, alpha * gradient) and keep its branch data
    lr1.code = lr1.flag = 0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      if (LIM) {
        T nb[5] = {m1[v], lane_up(m1[v]), lane_down(m1[v]), m2[v], m0[v]};
        LimInfo<T> li = lim_info(nb, g1[2 * v], g1[2 * v + 1], hx2, hy2);
        lr1.alpha[v] = li.alpha;
        lr1.code |= (unsigned)(li.amax | (li.amin << 3)) << (6 * v);
        lr1.flag |= (unsigned)((li.active ? 1 : 0) | (li.dplus ? 2 : 0) | (li.xaxis ? 4 : 0))
                    << (3 * v);
      } else {
        lr1.alpha[v] = T(1);
      }
    }

    // S2: faces and volume of row j-1
    T W1[12];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      W1[3 * v] = m1[v];
      W1[3 * v + 1] = lr1.alpha[v] * g1[2 * v];
      W1[3 * v + 2] = lr1.alpha[v] * g1[2 * v + 1];
    }
    if (s2_cell) {
      // -x face of this lane: L = lane - 1, R = this lane
      T WL[12], lL[12];
#pragma unroll
      for (int k = 0; k < 12; ++k) {
        WL[k] = lane_up(W1[k]);
        lL[k] = lane_up(l1[k]);
      }
      T lamF[2][4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const T a = cmx * (l1[3 * v] - lL[3 * v]) - cgx * (l1[3 * v + 1] + lL[3 * v + 1]);
        const T b = ccr * (l1[3 * v + 2] - lL[3 * v + 2]);
        lamF[0][v] = a - b;
        lamF[1][v] = a + b;
      }
      T AL[4], BL[4], AR[4], BR[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) AL[v] = BL[v] = AR[v] = BR[v] = T(0);
#pragma unroll
      for (int gp = 0; gp < 2; ++gp) {
        const T sg = gp == 0 ? T(-1) : T(1);
        T uL[4], uR[4], luL[4] = {T(0), T(0), T(0), T(0)}, luR[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          uL[v] = WL[3 * v] + WL[3 * v + 1] * hx2 + sg * WL[3 * v + 2] * qy;
          uR[v] = W1[3 * v] - W1[3 * v + 1] * hx2 + sg * W1[3 * v + 2] * qy;
        }
        hll_vjp<T, 0>(uL, uR, gam, lamF[gp], luL, luR);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          AL[v] += luL[v];
          BL[v] += sg * luL[v];
          AR[v] += luR[v];
          BR[v] += sg * luR[v];
        }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        // this lane is the R side of its -x face; its +x face's L share comes
        // from the right lane
        const T aL = lane_down(AL[v]), bL = lane_down(BL[v]);
        acc1[3 * v] += cL * (AR[v] + aL);
        acc1[3 * v + 1] += cL * hx2 * (aL - AR[v]);
        acc1[3 * v + 2] += cL * qy * (BR[v] + bL);
      }
      // volume term
#pragma unroll 1
      for (int q = 0; q < 4; ++q) {
        const T ox = (q & 2) ? qx : -qx, oy = (q & 1) ? qy : -qy;
        T u[4], a[4], b[4], lu[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          u[v] = W1[3 * v] + W1[3 * v + 1] * ox + W1[3 * v + 2] * oy;
          a[v] = cgx * l1[3 * v + 1];
          b[v] = cgy * l1[3 * v + 2];
        }
        flux_xy_vjp(u, gam, a, b, lu);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          acc1[3 * v] += cL * lu[v];
          acc1[3 * v + 1] += cL * ox * lu[v];
          acc1[3 * v + 2] += cL * oy * lu[v];
        }
      }
    }
    if (r1 >= y0 - 1 && r1 <= y1 + 1) {
      // y face between rows j-2 (L) and j-1 (R)
      T W2[12];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        W2[3 * v] = m2[v];
        W2[3 * v + 1] = lr2.alpha[v] * g2[2 * v];
        W2[3 * v + 2] = lr2.alpha[v] * g2[2 * v + 1];
      }
      T lamF[2][4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const T a = cmy * (l1[3 * v] - l2[3 * v]) - cgy * (l1[3 * v + 2] + l2[3 * v + 2]);
        const T b = ccr * (l1[3 * v + 1] - l2[3 * v + 1]);
        lamF[0][v] = a - b;
        lamF[1][v] = a + b;
      }
      T AL[4], BL[4], AR[4], BR[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) AL[v] = BL[v] = AR[v] = BR[v] = T(0);
#pragma unroll
      for (int gp = 0; gp < 2; ++gp) {
        const T sg = gp == 0 ? T(-1) : T(1);
        T uL[4], uR[4], luL[4] = {T(0), T(0), T(0), T(0)}, luR[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          uL[v] = W2[3 * v] + W2[3 * v + 2] * hy2 + sg * W2[3 * v + 1] * qx;
          uR[v] = W1[3 * v] - W1[3 * v + 2] * hy2 + sg * W1[3 * v + 1] * qx;
        }
        hll_vjp<T, 1>(uL, uR, gam, lamF[gp], luL, luR);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          AL[v] += luL[v];
          BL[v] += sg * luL[v];
          AR[v] += luR[v];
          BR[v] += sg * luR[v];
        }
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        acc1[3 * v] += cL * AR[v];
        acc1[3 * v + 2] -= cL * hy2 * AR[v];
        acc1[3 * v + 1] += cL * qx * BR[v];
        acc2[3 * v] += cL * AL[v];
        acc2[3 * v + 2] += cL * hy2 * AL[v];
        acc2[3 * v + 1] += cL * qx * BL[v];
      }
    }

    // S3: row j-2 is complete: lamW = acc2
    const int r2 = j - 2;
    PitRow<T> pr2;
    T own2[4];
    pr2.code = 0;
#pragma unroll
    for (int v = 0; v < 4; ++v) pr2.lhi[v] = pr2.llo[v] = own2[v] = T(0);
    if (r2 >= y0 - 1 && r2 <= y1) {
      const bool wr = own && r2 >= y0 && r2 < y1;
      const unsigned o = roff(r2);
      if (!LIM) {
        if (wr) {
#pragma unroll
          for (int k = 0; k < 12; ++k) st(O, nc, k, o, acc2[k]);
        }
      } else {
        pr2.code = lr2.code;
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const T gx = g2[2 * v], gy = g2[2 * v + 1];
          const T lgx = acc2[3 * v + 1], lgy = acc2[3 * v + 2];
          const T al = lr2.alpha[v];
          const unsigned fl = (lr2.flag >> (3 * v)) & 7u;
          T om = acc2[3 * v], ogx = al * lgx, ogy = al * lgy;
          if (fl & 1u) {
            const T la = gx * lgx + gy * lgy;
            const T dm = (fl & 4u) ? fabs(gx) * hx2 : fabs(gy) * hy2;
            const T lD = div_small(la, dm);
            const T ldm = -div_small(la * al, dm);
            if (fl & 2u) {
              pr2.lhi[v] = lD;
              om -= lD;
            } else {
              pr2.llo[v] = -lD;
              om += lD;
            }
            if (fl & 4u)
              ogx += ldm * hx2 * (gx < T(0) ? T(-1) : T(1));
            else
              ogy += ldm * hy2 * (gy < T(0) ? T(-1) : T(1));
          }
          own2[v] = om;
          if (wr) {
            st(O, nc, 3 * v + 1, o, ogx);
            st(O, nc, 3 * v + 2, o, ogy);
          }
        }
      }
    }

    // S4: row j-3's mean adjoints (self, -x, +x, -y = row j-4, +y = row j-2)
    if (LIM) {
      const int r3 = j - 3;
      const bool wr = own && r3 >= y0 && r3 < y1;
      const unsigned o = roff(r3);
      const unsigned cla = lane_up_u(pr3.code), cra = lane_down_u(pr3.code);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        // lane shifts run on every lane; only the owning lanes use them
        const T lhl = lane_up(pr3.lhi[v]), lll = lane_up(pr3.llo[v]);
        const T lhr = lane_down(pr3.lhi[v]), llr = lane_down(pr3.llo[v]);
        const int sh = 6 * v;
        T om = own3[v];
        // the code a neighbour uses for this cell: self 0, from -x it is +x (2),
        // from +x it is -x (1), from -y (row below) +y (4), from +y -y (3)
        const unsigned cs = (pr3.code >> sh) & 63u, cl = (cla >> sh) & 63u,
                       cr = (cra >> sh) & 63u, cd = (pr4.code >> sh) & 63u,
                       cu = (pr2.code >> sh) & 63u;
        if ((cs & 7u) == 0u) om += pr3.lhi[v];
        if ((cs >> 3) == 0u) om += pr3.llo[v];
        if ((cl & 7u) == 2u) om += lhl;
        if ((cl >> 3) == 2u) om += lll;
        if ((cr & 7u) == 1u) om += lhr;
        if ((cr >> 3) == 1u) om += llr;
        if ((cd & 7u) == 4u) om += pr4.lhi[v];
        if ((cd >> 3) == 4u) om += pr4.llo[v];
        if ((cu & 7u) == 3u) om += pr2.lhi[v];
        if ((cu >> 3) == 3u) om += pr2.llo[v];
        if (wr) st(O, nc, 3 * v, o, om);
      }
      pr4 = pr3;
      pr3 = pr2;
#pragma unroll
      for (int v = 0; v < 4; ++v) own3[v] = own2[v];
    }
  }
}

template <bool LIM>
__global__ __launch_bounds__(256) void k_adj_row_f64(PA<double> p) {
  adj_row_body<double, LIM>(p);
}

// FP32: two waves per SIMD, at the price of a few values spilled (16 bytes per
// lane), measured faster than one wave per SIMD without spills.
template <bool LIM>
__global__ __launch_bounds__(256) __attribute__((amdgpu_waves_per_eu(2, 2))) void k_adj_row_f32(
    PA<float> p) {
  adj_row_body<float, LIM>(p);
}

template <typename T, bool LIM>
void launch_row(const dim3& grid, const dim3& block, hipStream_t s, const PA<T>& p);
template <>
void launch_row<double, true>(const dim3& g, const dim3& b, hipStream_t s, const PA<double>& p) {
  hipLaunchKernelGGL((k_adj_row_f64<true>), g, b, 0, s, p);
}
template <>
void launch_row<double, false>(const dim3& g, const dim3& b, hipStream_t s, const PA<double>& p) {
  hipLaunchKernelGGL((k_adj_row_f64<false>), g, b, 0, s, p);
}
template <>
void launch_row<float, true>(const dim3& g, const dim3& b, hipStream_t s, const PA<float>& p) {
  hipLaunchKernelGGL((k_adj_row_f32<true>), g, b, 0, s, p);
}
template <>
void launch_row<float, false>(const dim3& g, const dim3& b, hipStream_t s, const PA<float>& p) {
  hipLaunchKernelGGL((k_adj_row_f32<false>), g, b, 0, s, p);
}

template <typename T>
hipError_t adj_stage_t(const AdjInst* inst, const int* tile_inst, int ntiles, int nc, const T* P,
                       const T* lam, const T* extra, T* out, double c_id, double c_L_over_dt,
                       double c_extra, const double* dt_dev, double dt_host, double gamma,
                       bool lim, hipStream_t s) {
  PA<T> p;
  p.P = P;
  p.lam = lam;
  p.extra = extra;
  p.out = out;
  p.inst = inst;
  p.tile_inst = tile_inst;
  p.dt_dev = dt_dev;
  p.dt_host = dt_host;
  p.c_id = c_id;
  p.c_L_over_dt = c_L_over_dt;
  p.c_extra = c_extra;
  p.nc = nc;
  p.ntiles = ntiles;
  p.gamma = (T)gamma;
  const dim3 grid((ntiles + 3) / 4), block(256);
  if (lim)
    launch_row<T, true>(grid, block, s, p);
  else
    launch_row<T, false>(grid, block, s, p);
  return hipGetLastError();
}

}  // namespace

// One adjoint step of a set of 2D Euler Cartesian instances (a single mesh is
// one instance).  inst/tile_inst are device tables; V1 is the stage-1 output
// of the forward step from U.  lam_np1 -> lam_n.  ws: one state-sized
// workspace (lam_V1).
hipError_t launch_adjoint2d(const void* inst, const int* tile_inst, int ntiles, int nc,
                            int64_t total, bool f64, bool lim, double gamma, const void* U,
                            const void* V1, const double* dt_dev, double dt_host,
                            const void* lam_np1, void* lam_n, void* ws1, void* ws2,
                            hipStream_t s) {
  const AdjInst* in = static_cast<const AdjInst*>(inst);
  (void)total;
  (void)ws1;
  hipError_t e;
  // stage 2: ws2 = lam_V1 = Pi_V1^T [lam'/2 + (dt/2) L^T lam']
  // stage 1: lam_n = Pi_U^T [lam_V1 + dt L^T lam_V1 + lam'/2]
  if (f64) {
    using T = double;
    e = adj_stage_t<T>(in, tile_inst, ntiles, nc, (const T*)V1, (const T*)lam_np1, nullptr,
                       (T*)ws2, 0.5, 0.5, 0.0, dt_dev, dt_host, gamma, lim, s);
    if (e == hipSuccess)
      e = adj_stage_t<T>(in, tile_inst, ntiles, nc, (const T*)U, (const T*)ws2,
                         (const T*)lam_np1, (T*)lam_n, 1.0, 1.0, 0.5, dt_dev, dt_host, gamma,
                         lim, s);
  } else {
    using T = float;
    e = adj_stage_t<T>(in, tile_inst, ntiles, nc, (const T*)V1, (const T*)lam_np1, nullptr,
                       (T*)ws2, 0.5, 0.5, 0.0, dt_dev, dt_host, gamma, lim, s);
    if (e == hipSuccess)
      e = adj_stage_t<T>(in, tile_inst, ntiles, nc, (const T*)U, (const T*)ws2,
                         (const T*)lam_np1, (T*)lam_n, 1.0, 1.0, 0.5, dt_dev, dt_host, gamma,
                         lim, s);
  }
  return e;
}

}  // namespace dg
