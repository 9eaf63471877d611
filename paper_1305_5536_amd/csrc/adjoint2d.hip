// Discrete adjoint of the 2D Euler Cartesian SSP-RK2 step (vector-Jacobian
// products of the exact discrete step, dt frozen, the limiter and the HLL wave
// speeds following the branch the forward computation takes).
//
// Forward step (Sec. 2.2 operator L, Sec. 2.5 limiter Pi):
//   Ua = Pi(U);  V1 = Ua + dt L(Ua);  Ub = Pi(V1);  U' = Ua/2 + (Ub + dt L(Ub))/2
// Backward, given lam' = dJ/dU':
//   lam_V1 = Pi_V1^T [ lam'/2 + (dt/2) L_Ub^T lam' ]                 (stage 2)
//   lam    = Pi_U^T  [ lam_V1 + dt L_Ua^T lam_V1 + lam'/2 ]            (stage 1)
// so both stages are one "adjoint stage":  out = Pi_P^T [c_id lam + c_L
// L_W^T lam + extra],  W = Pi(P), run by two kernels:
//   k_adj_lt  : lam_W = c_id lam + c_L (dL/dW)^T lam + extra    (15x16 tiles)
//   k_adj_pit : out = (dPi/dP)^T lam_W                           (15x16 tiles)
// Each tile stages its halo in LDS (coefficient records padded to an odd
// stride, so lanes reading consecutive cells hit distinct banks).  k_adj_lt
// solves every face's VJP once per tile in two rounds, x faces (16 per row x
// 16 rows) then y faces (17 per column x 15 columns), so each round fills the
// 256 threads once; per face it keeps, for each side, the sum over the two
// Gauss points of the state adjoint and of its tangentially weighted sum,
// which the owning cells gather (no atomics).  Boundary faces of a tile are
// recomputed by the neighbouring tile.  k_adj_pit computes the limiter data of
// the tile and its halo, then gathers, for each cell, the contributions of the
// neighbours whose max/min it supplied.
//
// Ties (min/max arguments, the limiter's branch) take the first argument in
// the order self, -x, +x, -y, +y, as the CPU oracle's dual numbers do.
#include <hip/hip_runtime.h>

#include "dg_internal.h"
#include "dg_math.h"

namespace dg {
namespace {

constexpr int TX = kAdjTileX;         // interior columns of a tile
constexpr int TY = kAdjTileY;         // interior rows
constexpr int HX = TX + 2;            // with a halo of 1
constexpr int HY = TY + 2;
constexpr int NH = HX * HY;
constexpr int NCELL = TX * TY;        // 240 of the 256 threads own a cell
constexpr int CS = 13;                // LDS stride of a 12-coefficient record
constexpr int NFX = (TX + 1) * TY;    // x faces of a tile (256)
constexpr int NFY = (TY + 1) * TX;    // y faces of a tile (255)
constexpr int FS = 17;                // LDS stride of a face record (16 values)
static_assert(NFX <= 256 && NFY <= 256, "one face per thread and round");
constexpr int GX = TX + 4;            // with a halo of 2 (limiter stencils of the halo)
constexpr int GY = TY + 4;
constexpr int NG = GX * GY;
constexpr int MS = 5;                 // LDS stride of a 4-mean record

template <typename T>
struct PA {
  const T* __restrict__ P;     // pre-limit state
  const T* __restrict__ lam;   // adjoint of the stage output
  const T* __restrict__ extra; // added to lam_W (may be NULL)
  const T* __restrict__ lamW;  // k_adj_pit input
  T* __restrict__ out;
  const AdjInst* inst;
  const int* tile_inst;        // tile -> instance (batched); NULL: one instance
  const double* dt_dev;        // per instance (batched) or one value
  double dt_host;
  double c_id, c_L_over_dt;    // c_L = c_L_over_dt * dt
  double c_extra;
  int nc;                      // global stride of the coefficient arrays
  int ntiles;
  T gamma;
  int limiter;
};

struct Geo {
  int nx, ny, off, tx, ty;
  double hx, hy;
};

template <typename T>
__device__ __forceinline__ Geo tile_geo(const PA<T>& p, int tile) {
  const int i = p.tile_inst ? p.tile_inst[tile] : 0;
  const AdjInst in = p.inst[i];
  Geo g;
  g.nx = in.nx;
  g.ny = in.ny;
  g.off = in.off;
  const int t = tile - in.tx0;
  g.tx = t % in.tiles_x;
  g.ty = t / in.tiles_x;
  g.hx = in.hx;
  g.hy = in.hy;
  return g;
}

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
  r.alpha = r.active ? r.D * rcp(r.dm) : T(1);
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

// ------------------------------------------------------------ L^T kernel --
template <typename T>
struct LtSmem {
  T W[NH * CS];     // limited state, tile + halo 1
  T lam[NH * CS];   // adjoint of the stage output, tile + halo 1
  T f[256 * FS];    // per face of the current round: (A_L, B_L, A_R, B_R) x 4
};

template <typename T, bool LIM>
__global__ __launch_bounds__(256) void k_adj_lt(PA<T> p) {
  __shared__ LtSmem<T> sm;
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const Geo g = tile_geo(p, tile);
  const int nc = p.nc;
  const int x0 = g.tx * TX, y0 = g.ty * TY;
  const T hx = (T)g.hx, hy = (T)g.hy;
  const T hx2 = T(0.5) * hx, hy2 = T(0.5) * hy;
  const T s3 = T(1.7320508075688772);
  const T qx = hx2 / s3, qy = hy2 / s3;
  const T cmx = T(0.5) / hx, cmy = T(0.5) / hy, cgx = T(3) / (hx * hx), cgy = T(3) / (hy * hy),
          ccr = s3 / (hx * hy);
  const int tid = threadIdx.x;
  auto gidx = [&](int lx, int ly) {  // tile-local (may be negative) -> global
    return g.off + wrapi(y0 + ly, g.ny) * g.nx + wrapi(x0 + lx, g.nx);
  };
  // means of P on the tile + halo 2 (the limiter stencils of the halo cells),
  // staged in the face area, which is free until the face rounds
  T* mean = sm.f;
  if (LIM) {
    static_assert(NG * MS <= 256 * FS, "means fit in the face area");
    for (int i = tid; i < NG; i += 256) {
      const int e = gidx(i % GX - 2, i / GX - 2);
#pragma unroll
      for (int v = 0; v < 4; ++v) mean[i * MS + v] = p.P[3 * v * nc + e];
    }
    __syncthreads();
  }
  // W = Pi(P) and lam on the tile + halo 1
  for (int i = tid; i < NH; i += 256) {
    const int lx = i % HX - 1, ly = i / HX - 1;
    const int e = gidx(lx, ly);
    T q[12];
#pragma unroll
    for (int k = 0; k < 12; ++k) q[k] = p.P[k * nc + e];
    if (LIM) {
      const int gi = ((ly + 2) * GX + lx + 2) * MS;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        T nb[5] = {q[3 * v], mean[gi - MS + v], mean[gi + MS + v], mean[gi - GX * MS + v],
                   mean[gi + GX * MS + v]};
        LimInfo<T> li = lim_info(nb, q[3 * v + 1], q[3 * v + 2], hx2, hy2);
        q[3 * v + 1] *= li.alpha;
        q[3 * v + 2] *= li.alpha;
      }
    }
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      sm.W[i * CS + k] = q[k];
      sm.lam[i * CS + k] = p.lam[k * nc + e];
    }
  }
  __syncthreads();
  auto li1 = [](int lx, int ly) { return ((ly + 1) * HX + (lx + 1)) * CS; };
  T acc[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) acc[k] = T(0);
  const int cx = tid % TX, cy = tid / TX;  // this thread's interior cell (tid < NCELL)
  // two rounds: x faces (AX = 0) then y faces (AX = 1).  x face j of row r
  // joins tile-local cells (j-1, r) and (j, r); y face j of column c joins
  // (c, j-1) and (c, j).
#pragma unroll
  for (int ax = 0; ax < 2; ++ax) {
    const int nf = ax == 0 ? NFX : NFY;
    if (tid < nf) {
      const int f = tid;
      int iL, iR;
      if (ax == 0) {
        const int r = f / (TX + 1), j = f % (TX + 1);
        iL = li1(j - 1, r);
        iR = li1(j, r);
      } else {
        const int c = f / (TY + 1), j = f % (TY + 1);
        iL = li1(c, j - 1);
        iR = li1(c, j);
      }
      const T* WL = sm.W + iL;
      const T* WR = sm.W + iR;
      const T* lL = sm.lam + iL;
      const T* lR = sm.lam + iR;
      T lamF[2][4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        if (ax == 0) {
          const T a = cmx * (lR[3 * v] - lL[3 * v]) - cgx * (lR[3 * v + 1] + lL[3 * v + 1]);
          const T b = ccr * (lR[3 * v + 2] - lL[3 * v + 2]);
          lamF[0][v] = a - b;
          lamF[1][v] = a + b;
        } else {
          const T a = cmy * (lR[3 * v] - lL[3 * v]) - cgy * (lR[3 * v + 2] + lL[3 * v + 2]);
          const T b = ccr * (lR[3 * v + 1] - lL[3 * v + 1]);
          lamF[0][v] = a - b;
          lamF[1][v] = a + b;
        }
      }
      T AL[4], BL[4], AR[4], BR[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) AL[v] = BL[v] = AR[v] = BR[v] = T(0);
#pragma unroll
      for (int gp = 0; gp < 2; ++gp) {
        const T sg = gp == 0 ? T(-1) : T(1);
        T uL[4], uR[4], lu_L[4] = {T(0), T(0), T(0), T(0)}, lu_R[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          if (ax == 0) {
            uL[v] = WL[3 * v] + WL[3 * v + 1] * hx2 + sg * WL[3 * v + 2] * qy;
            uR[v] = WR[3 * v] - WR[3 * v + 1] * hx2 + sg * WR[3 * v + 2] * qy;
          } else {
            uL[v] = WL[3 * v] + WL[3 * v + 2] * hy2 + sg * WL[3 * v + 1] * qx;
            uR[v] = WR[3 * v] - WR[3 * v + 2] * hy2 + sg * WR[3 * v + 1] * qx;
          }
        }
        if (ax == 0)
          hll_vjp<T, 0>(uL, uR, p.gamma, lamF[gp], lu_L, lu_R);
        else
          hll_vjp<T, 1>(uL, uR, p.gamma, lamF[gp], lu_L, lu_R);
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          AL[v] += lu_L[v];
          AR[v] += lu_R[v];
          BL[v] += sg * lu_L[v];
          BR[v] += sg * lu_R[v];
        }
      }
      T* rec = sm.f + f * FS;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        rec[v] = AL[v];
        rec[4 + v] = BL[v];
        rec[8 + v] = AR[v];
        rec[12 + v] = BR[v];
      }
    }
    __syncthreads();
    // gather: the cell is the R side of its lower face and the L side of its
    // upper face along the axis
    if (tid < NCELL) {
      const int fm = ax == 0 ? cy * (TX + 1) + cx : cx * (TY + 1) + cy;
      const T* m = sm.f + fm * FS;        // cell on the R side
      const T* pl = sm.f + (fm + 1) * FS; // cell on the L side
      const T hn = ax == 0 ? hx2 : hy2, qt = ax == 0 ? qy : qx;
      const int kn = ax == 0 ? 1 : 2, kt = ax == 0 ? 2 : 1;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        acc[3 * v] += m[8 + v] + pl[v];
        acc[3 * v + kn] += hn * (pl[v] - m[8 + v]);
        acc[3 * v + kt] += qt * (m[12 + v] + pl[4 + v]);
      }
    }
    __syncthreads();
  }
  if (tid >= NCELL) return;
  // volume term
  {
    const T* Wc = sm.W + li1(cx, cy);
    const T* lc = sm.lam + li1(cx, cy);
#pragma unroll 1
    for (int q = 0; q < 4; ++q) {
      const T ox = (q & 2) ? qx : -qx, oy = (q & 1) ? qy : -qy;
      T u[4], a[4], b[4], lu[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        u[v] = Wc[3 * v] + Wc[3 * v + 1] * ox + Wc[3 * v + 2] * oy;
        a[v] = cgx * lc[3 * v + 1];
        b[v] = cgy * lc[3 * v + 2];
      }
      flux_xy_vjp(u, p.gamma, a, b, lu);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        acc[3 * v] += lu[v];
        acc[3 * v + 1] += ox * lu[v];
        acc[3 * v + 2] += oy * lu[v];
      }
    }
  }
  if (x0 + cx < g.nx && y0 + cy < g.ny) {
    const int i = p.tile_inst ? p.tile_inst[tile] : 0;
    const double dt = p.dt_dev ? p.dt_dev[i] : p.dt_host;
    const T cL = (T)(p.c_L_over_dt * dt), cI = (T)p.c_id;
    const int e = g.off + (y0 + cy) * g.nx + (x0 + cx);
    const T* lc = sm.lam + li1(cx, cy);
#pragma unroll
    for (int k = 0; k < 12; ++k) {
      T v = cI * lc[k] + cL * acc[k];
      if (p.extra) v += (T)p.c_extra * p.extra[k * nc + e];
      p.out[k * nc + e] = v;
    }
  }
}

// ----------------------------------------------- limiter transpose kernel --
template <typename T>
struct PitSmem {
  T mean[NG * MS];        // means of P, tile + halo 2
  T lhi[NH * MS];         // adjoint routed to the arg-max / arg-min means
  T llo[NH * MS];
  T own[NH * MS];         // interior cells: the mean adjoint from the cell's own alpha
  unsigned char code[NH][4];  // amax | amin << 3
};

template <typename T>
__global__ __launch_bounds__(256) void k_adj_pit(PA<T> p) {
  __shared__ PitSmem<T> sm;
  const int tile = xcd_remap(blockIdx.x, gridDim.x);
  const Geo g = tile_geo(p, tile);
  const int nc = p.nc;
  const int x0 = g.tx * TX, y0 = g.ty * TY;
  const T hx2 = T(0.5) * (T)g.hx, hy2 = T(0.5) * (T)g.hy;
  const int tid = threadIdx.x;
  auto gidx = [&](int lx, int ly) {
    return g.off + wrapi(y0 + ly, g.ny) * g.nx + wrapi(x0 + lx, g.nx);
  };
  for (int i = tid; i < NG; i += 256) {
    const int e = gidx(i % GX - 2, i / GX - 2);
#pragma unroll
    for (int v = 0; v < 4; ++v) sm.mean[i * MS + v] = p.P[3 * v * nc + e];
  }
  __syncthreads();
  // limiter data of the tile and its halo: what each cell routes to its
  // arg-max / arg-min neighbours; interior cells also finish their gradient
  // adjoints and the own part of their mean adjoint
  for (int i = tid; i < NH; i += 256) {
    const int lx = i % HX - 1, ly = i / HX - 1;
    const int e = gidx(lx, ly);
    const bool inner = lx >= 0 && ly >= 0 && lx < TX && ly < TY && x0 + lx < g.nx &&
                       y0 + ly < g.ny;
    const int gi = ((ly + 2) * GX + lx + 2) * MS;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const T gx = p.P[(3 * v + 1) * nc + e], gy = p.P[(3 * v + 2) * nc + e];
      T nb[5] = {sm.mean[gi + v], sm.mean[gi - MS + v], sm.mean[gi + MS + v],
                 sm.mean[gi - GX * MS + v], sm.mean[gi + GX * MS + v]};
      LimInfo<T> li = lim_info(nb, gx, gy, hx2, hy2);
      const T lgx = p.lamW[(3 * v + 1) * nc + e], lgy = p.lamW[(3 * v + 2) * nc + e];
      T lhi = T(0), llo = T(0), om = T(0), ogx = li.alpha * lgx, ogy = li.alpha * lgy;
      if (li.active) {
        const T la = gx * lgx + gy * lgy;
        const T idm = rcp(li.dm);
        const T lD = la * idm;
        const T ldm = -la * li.alpha * idm;
        if (li.dplus)
          lhi = lD;
        else
          llo = -lD;
        // D = hi - phi (dplus) or phi - lo: the phi part
        om = li.dplus ? -lD : lD;
        if (li.xaxis)
          ogx += ldm * hx2 * (gx < T(0) ? T(-1) : T(1));
        else
          ogy += ldm * hy2 * (gy < T(0) ? T(-1) : T(1));
      }
      sm.lhi[i * MS + v] = lhi;
      sm.llo[i * MS + v] = llo;
      sm.code[i][v] = (unsigned char)(li.amax | (li.amin << 3));
      if (inner) {
        sm.own[i * MS + v] = om + p.lamW[3 * v * nc + e];
        p.out[(3 * v + 1) * nc + e] = ogx;
        p.out[(3 * v + 2) * nc + e] = ogy;
      }
    }
  }
  __syncthreads();
  const int cx = tid % TX, cy = tid / TX;
  if (tid >= NCELL || x0 + cx >= g.nx || y0 + cy >= g.ny) return;
  const int e = g.off + (y0 + cy) * g.nx + (x0 + cx);
  auto li1 = [](int lx, int ly) { return (ly + 1) * HX + (lx + 1); };
  // neighbour slots in LDS and the code that names this cell from each of them
  const int sl[5] = {li1(cx, cy), li1(cx - 1, cy), li1(cx + 1, cy), li1(cx, cy - 1),
                     li1(cx, cy + 1)};
  const int back[5] = {0, 2, 1, 4, 3};  // from the -x neighbour, this cell is its +x
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    T om = sm.own[sl[0] * MS + v];
    // means that supplied a max or min (self included)
#pragma unroll
    for (int k = 0; k < 5; ++k) {
      const unsigned char cd = sm.code[sl[k]][v];
      if ((cd & 7) == back[k]) om += sm.lhi[sl[k] * MS + v];
      if ((cd >> 3) == back[k]) om += sm.llo[sl[k] * MS + v];
    }
    p.out[3 * v * nc + e] = om;
  }
}

template <typename T>
hipError_t adj_stage_t(const AdjInst* inst, const int* tile_inst, int ntiles, int nc,
                       int64_t total, const T* P, const T* lam, const T* extra, T* lamW, T* out,
                       double c_id, double c_L_over_dt, double c_extra, const double* dt_dev,
                       double dt_host, double gamma, bool lim, hipStream_t s) {
  PA<T> p;
  p.P = P;
  p.lam = lam;
  p.extra = extra;
  p.lamW = lamW;
  p.out = lim ? lamW : out;
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
  p.limiter = lim;
  if (lim)
    hipLaunchKernelGGL((k_adj_lt<T, true>), dim3(ntiles), dim3(256), 0, s, p);
  else
    hipLaunchKernelGGL((k_adj_lt<T, false>), dim3(ntiles), dim3(256), 0, s, p);
  if (!lim) return hipGetLastError();
  p.out = out;
  hipLaunchKernelGGL((k_adj_pit<T>), dim3(ntiles), dim3(256), 0, s, p);
  (void)total;
  return hipGetLastError();
}

}  // namespace

// One adjoint step of a set of 2D Euler Cartesian instances (a single mesh is
// one instance).  inst/tile_inst are device tables; V1 is the stage-1 output
// of the forward step from U.  lam_np1 -> lam_n.  ws1, ws2: state-sized
// workspaces.
hipError_t launch_adjoint2d(const void* inst, const int* tile_inst, int ntiles, int nc,
                            int64_t total, bool f64, bool lim, double gamma, const void* U,
                            const void* V1, const double* dt_dev, double dt_host,
                            const void* lam_np1, void* lam_n, void* ws1, void* ws2,
                            hipStream_t s) {
  const AdjInst* in = static_cast<const AdjInst*>(inst);
  hipError_t e;
  // stage 2: ws2 = lam_V1 = Pi_V1^T [lam'/2 + (dt/2) L^T lam']
  // stage 1: lam_n = Pi_U^T [lam_V1 + dt L^T lam_V1 + lam'/2]
  if (f64) {
    using T = double;
    e = adj_stage_t<T>(in, tile_inst, ntiles, nc, total, (const T*)V1, (const T*)lam_np1, nullptr,
                       (T*)ws1, (T*)ws2, 0.5, 0.5, 0.0, dt_dev, dt_host, gamma, lim, s);
    if (e == hipSuccess)
      e = adj_stage_t<T>(in, tile_inst, ntiles, nc, total, (const T*)U, (const T*)ws2,
                         (const T*)lam_np1, (T*)ws1, (T*)lam_n, 1.0, 1.0, 0.5, dt_dev, dt_host,
                         gamma, lim, s);
  } else {
    using T = float;
    e = adj_stage_t<T>(in, tile_inst, ntiles, nc, total, (const T*)V1, (const T*)lam_np1, nullptr,
                       (T*)ws1, (T*)ws2, 0.5, 0.5, 0.0, dt_dev, dt_host, gamma, lim, s);
    if (e == hipSuccess)
      e = adj_stage_t<T>(in, tile_inst, ntiles, nc, total, (const T*)U, (const T*)ws2,
                         (const T*)lam_np1, (T*)ws1, (T*)lam_n, 1.0, 1.0, 0.5, dt_dev, dt_host,
                         gamma, lim, s);
  }
  return e;
}

}  // namespace dg
