// DG stage kernels for 2D Euler on a periodic face-list mesh (static Voronoi).
//
// Same method as the Cartesian kernels (Sec. 2.2 weak form, HLL face flux,
// limiter of Sec. 2.5, SSP-RK2), on general polygons: two Gauss points per
// edge, the 4-point principal-axis volume rule (points c -+ sqrt(2 lambda_k/V)
// e_k of the second-moment matrix M, weights V/4: exact for quadratics), and
// the per-cell 2x2 inverse of M for the gradients.
//
// Work decomposition.  Cells are split into blocks of up to 256 consecutive
// indices (a space-filling-curve numbering makes a block compact).  The host
// lists, per block, every face incident to one of its cells ("slots": faces
// on the block boundary appear in both blocks) and a block-local CSR from each
// cell to its (slot, side) incidences.  One workgroup per block:
//   1. each thread solves the Riemann problems of some slots (HLL at both Gauss
//      points) and writes the 2 x 4 fluxes to LDS;
//   2. after one barrier each thread gathers its own cell's incidences from
//      LDS (a segmented reduction, no atomics; each incidence's weight and
//      Gauss-point offsets come from a record stored in incidence order), adds
//      the volume term, applies M^-1 and the RK combination.
// The limiter is a separate pass (k_fl_lim) into the workspace, as on 3D
// meshes; stage 2 reuses Pi(U^n) from stage 1.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "dg_internal.h"
#include "dg_math.h"

namespace dg {

// Device arrays of a face-list mesh (allocated at create, in the mesh's
// working precision for geometry).
struct FLDev {
  int ncells, nblocks, max_slots;
  int64_t ninc;       // incidences of the global CSR (2 x faces)
  int* blk_cell0;     // [nblocks+1] first cell of each block
  int* blk_slot0;     // [nblocks+1] first slot of each block
  int* slot_cells;    // [2*nslots] global L, R
  void* slot_geo;     // [nslots][10] nx, ny, w, rL0x, rL0y, rL1x, rL1y, rR0x, rR0y, (rR1 = rR0 + rL1 - rL0)
  int* cell_inc0;     // [ncells+1] block-local CSR start (global index into cell_inc)
  int* cell_inc;      // slot_local*2 + side
  void* inc_geo;      // [per cell_inc entry][5] signed weight (+-A/2), the two Gauss
                      // points' offsets from the cell's own centroid
  void* cell_geo;     // [ncells][8] 1/V, Minv00, Minv01, Minv11, a1x, a1y, a2x, a2y
  int* lim_inc0;      // [ncells+1] global CSR for the limiter and the CFL bound
  int* lim_nbr;       // neighbour cell of each incidence
  void* lim_geo;      // [ninc][2] face-centroid offsets, then [ninc][2] A n outward
  void* cell_perim;   // [ncells] sum of face lengths
};

namespace {

constexpr int kBlock = 256;
constexpr int kMaxSlots = 1024;  // LDS table: 64 KB of fluxes in FP64

template <typename T>
struct PF {
  const T* __restrict__ in;
  const T* __restrict__ ua;
  T* __restrict__ out;
  const double* dt_dev;
  double dt_host;
  int* status;
  double* dtpart;
  int ncells, nc;
  T gamma;
  const int* blk_cell0;
  const int* blk_slot0;
  const int* slot_cells;
  const T* slot_geo;
  const int* cell_inc0;
  const int* cell_inc;
  const T* inc_geo;
  const T* cell_geo;
  const int* lim_inc0;
  const int* lim_nbr;
  const T* lim_geo;  // face-centroid offsets (the limiter)
  const T* lim_an;   // A n outward (the CFL bound)
  const T* perim;
};

template <typename T>
__device__ __forceinline__ void load12(const T* __restrict__ U, int nc, int e, T* q) {
#pragma unroll
  for (int k = 0; k < 12; ++k) q[k] = U[k * nc + e];
}

// HLL flux along the unit normal n (Davis speeds), F = a F_L + b F_R + c dU.
template <typename T>
__device__ __forceinline__ void hll_n(const T* uL, const T* uR, T nx, T ny, T gamma, T* F,
                                      bool& bad) {
  const T gm1 = gamma - T(1);
  T irL = rcp(uL[0]), irR = rcp(uR[0]);
  T vxL = uL[1] * irL, vyL = uL[2] * irL, vxR = uR[1] * irR, vyR = uR[2] * irR;
  T pL = gm1 * (uL[3] - T(0.5) * (uL[1] * vxL + uL[2] * vyL));
  T pR = gm1 * (uR[3] - T(0.5) * (uR[1] * vxR + uR[2] * vyR));
  bad |= !(uL[0] > T(0)) || !(uR[0] > T(0)) || !(pL > T(0)) || !(pR > T(0));
  T cL = sqrt_pos(gamma * pL * irL), cR = sqrt_pos(gamma * pR * irR);
  T vnL = vxL * nx + vyL * ny, vnR = vxR * nx + vyR * ny;
  T SL = fmin(vnL - cL, vnR - cR), SR = fmax(vnL + cL, vnR + cR);
  T FL[4] = {uL[0] * vnL, uL[1] * vnL + pL * nx, uL[2] * vnL + pL * ny, (uL[3] + pL) * vnL};
  T FR[4] = {uR[0] * vnR, uR[1] * vnR + pR * nx, uR[2] * vnR + pR * ny, (uR[3] + pR) * vnR};
  T inv = rcp(SR - SL);
  T a = SR * inv, b = -SL * inv, c = SL * SR * inv;
  const bool left = SL >= T(0), right = SR <= T(0);
  a = left ? T(1) : (right ? T(0) : a);
  b = left ? T(0) : (right ? T(1) : b);
  c = (left || right) ? T(0) : c;
#pragma unroll
  for (int k = 0; k < 4; ++k) F[k] = fma(a, FL[k], fma(b, FR[k], c * (uR[k] - uL[k])));
}

// ------------------------------------------------------------- limiter --
template <typename T>
__global__ __launch_bounds__(256) void k_fl_lim(PF<T> p) {
  // blocks mapped XCD by XCD: neighbouring blocks (Morton-ordered cells) share
  // their neighbours' means in the same L2
  const int e = xcd_remap(blockIdx.x, gridDim.x) * 256 + threadIdx.x;
  if (e >= p.ncells) return;
  T q[12];
  load12(p.in, p.nc, e, q);
  T hi[4], lo[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) hi[v] = lo[v] = q[3 * v];
  // Incidences are taken kBatch at a time, every load of a batch issued before
  // any is used (a per-incidence loop waits out one gather chain per face);
  // padding slots repeat the cell itself, which changes no max, min or bound.
  constexpr int kBatch = 8;
  const int i0 = p.lim_inc0[e], i1 = p.lim_inc0[e + 1];
  for (int b0 = i0; b0 < i1; b0 += kBatch) {
    int nb[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) nb[u] = b0 + u < i1 ? p.lim_nbr[b0 + u] : e;
    T m[kBatch][4];
#pragma unroll
    for (int u = 0; u < kBatch; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) m[u][v] = p.in[(3 * v) * p.nc + nb[u]];
#pragma unroll
    for (int u = 0; u < kBatch; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        hi[v] = fmax(hi[v], m[u][v]);
        lo[v] = fmin(lo[v], m[u][v]);
      }
  }
  T alpha[4] = {T(1), T(1), T(1), T(1)};
  for (int b0 = i0; b0 < i1; b0 += kBatch) {
    T rx[kBatch], ry[kBatch];
#pragma unroll
    for (int u = 0; u < kBatch; ++u) {
      const int i = b0 + u < i1 ? b0 + u : b0;
      rx[u] = p.lim_geo[2 * i];
      ry[u] = p.lim_geo[2 * i + 1];
    }
#pragma unroll
    for (int u = 0; u < kBatch; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const T d = q[3 * v + 1] * rx[u] + q[3 * v + 2] * ry[u];
        // psi = (max - phi)/d for d > 0, (min - phi)/d for d < 0, 1 for d = 0
        const T num = d > T(0) ? hi[v] - q[3 * v] : lo[v] - q[3 * v];
        const T psi = d > T(0) ? div_small(num, d) : (d < T(0) ? div_small(-num, -d) : T(1));
        alpha[v] = fmin(alpha[v], psi);
      }
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    p.out[(3 * v) * p.nc + e] = q[3 * v];
    p.out[(3 * v + 1) * p.nc + e] = alpha[v] * q[3 * v + 1];
    p.out[(3 * v + 2) * p.nc + e] = alpha[v] * q[3 * v + 2];
  }
}

// ------------------------------------------------------------------ RHS --
template <typename T, int MODE>
__global__ __launch_bounds__(kBlock) void k_fl_rhs(PF<T> p) {
  __shared__ T sF[kMaxSlots][8];
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int c0 = p.blk_cell0[b], c1 = p.blk_cell0[b + 1];
  const int s0 = p.blk_slot0[b], s1 = p.blk_slot0[b + 1];
  const int nc = p.nc;
  bool bad = false;
  // 1. face fluxes into LDS
  for (int s = s0 + (int)threadIdx.x; s < s1; s += kBlock) {
    const int L = p.slot_cells[2 * s], R = p.slot_cells[2 * s + 1];
    const T* g = p.slot_geo + 10 * (size_t)s;
    const T nx = g[0], ny = g[1];
    const T rL0x = g[3], rL0y = g[4], rL1x = g[5], rL1y = g[6], rR0x = g[7], rR0y = g[8];
    const T rR1x = rR0x + (rL1x - rL0x), rR1y = rR0y + (rL1y - rL0y);
    T qL[12], qR[12];
    load12(p.in, nc, L, qL);
    load12(p.in, nc, R, qR);
    T uL[4], uR[4], F0[4], F1[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      uL[v] = fma(qL[3 * v + 1], rL0x, fma(qL[3 * v + 2], rL0y, qL[3 * v]));
      uR[v] = fma(qR[3 * v + 1], rR0x, fma(qR[3 * v + 2], rR0y, qR[3 * v]));
    }
    hll_n(uL, uR, nx, ny, p.gamma, F0, bad);
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      uL[v] = fma(qL[3 * v + 1], rL1x, fma(qL[3 * v + 2], rL1y, qL[3 * v]));
      uR[v] = fma(qR[3 * v + 1], rR1x, fma(qR[3 * v + 2], rR1y, qR[3 * v]));
    }
    hll_n(uL, uR, nx, ny, p.gamma, F1, bad);
    const int ls = s - s0;
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      sF[ls][v] = F0[v];
      sF[ls][4 + v] = F1[v];
    }
  }
  __syncthreads();
  // 2. per cell: gather incident faces, volume term, M^-1, RK combination
  const int e = c0 + (int)threadIdx.x;
  double dtmin = 1e300;
  if (e < c1) {
    T q[12];
    load12(p.in, nc, e, q);
    T rm[4] = {T(0), T(0), T(0), T(0)};
    T rx[4] = {T(0), T(0), T(0), T(0)};
    T ry[4] = {T(0), T(0), T(0), T(0)};
    // the cell's incidences: the slot's fluxes from LDS, this side's weight and
    // Gauss-point offsets from a record laid out in incidence order (the
    // block's cells read one contiguous run of them)
    const int i0 = p.cell_inc0[e], i1 = p.cell_inc0[e + 1];
    for (int i = i0; i < i1; ++i) {
      const int ls = p.cell_inc[i] >> 1;
      const T* g = p.inc_geo + 5 * (size_t)i;
      const T w = g[0], r0x = g[1], r0y = g[2], r1x = g[3], r1y = g[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const T f0 = sF[ls][v], f1 = sF[ls][4 + v];
        rm[v] = fma(w, f0 + f1, rm[v]);
        rx[v] = fma(w, fma(f0, r0x, f1 * r1x), rx[v]);
        ry[v] = fma(w, fma(f0, r0y, f1 * r1y), ry[v]);
      }
    }
    const T* cg = p.cell_geo + 8 * (size_t)e;
    const T iV = cg[0];
    const T m00 = cg[1], m01 = cg[2], m11 = cg[3];
    // volume term: 4 principal-axis points, weights V/4 (the 1/V of the
    // inverse mass matrix is folded in: rx, ry are per unit volume below)
    T vx[4] = {T(0), T(0), T(0), T(0)}, vy[4] = {T(0), T(0), T(0), T(0)};
#pragma unroll
    for (int k = 0; k < 4; ++k) {
      const T sgn = (k & 1) ? T(1) : T(-1);
      const T ox = sgn * ((k & 2) ? cg[6] : cg[4]);
      const T oy = sgn * ((k & 2) ? cg[7] : cg[5]);
      T u[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) u[v] = fma(q[3 * v + 1], ox, fma(q[3 * v + 2], oy, q[3 * v]));
      const T ir = rcp(u[0]);
      const T ux = u[1] * ir, uy = u[2] * ir;
      const T pr = (p.gamma - T(1)) * (u[3] - T(0.5) * (u[1] * ux + u[2] * uy));
      bad |= !(u[0] > T(0)) || !(pr > T(0));
      vx[0] += u[1];
      vx[1] += u[1] * ux + pr;
      vx[2] += u[2] * ux;
      vx[3] += (u[3] + pr) * ux;
      vy[0] += u[2];
      vy[1] += u[1] * uy;
      vy[2] += u[2] * uy + pr;
      vy[3] += (u[3] + pr) * uy;
    }
    T d[12];
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      // surface terms carry V implicitly through the face lengths; the volume
      // sums need the factor V/4
      const T gx = rx[v] * iV + T(0.25) * vx[v];
      const T gy = ry[v] * iV + T(0.25) * vy[v];
      d[3 * v] = rm[v] * iV;
      d[3 * v + 1] = m00 * gx + m01 * gy;
      d[3 * v + 2] = m01 * gx + m11 * gy;
    }
    T o[12];
    if (MODE == kRhs) {
#pragma unroll
      for (int k = 0; k < 12; ++k) o[k] = d[k];
    } else {
      const T dt = (T)(p.dt_dev ? *p.dt_dev : p.dt_host);
#pragma unroll
      for (int k = 0; k < 12; ++k) o[k] = fma(dt, d[k], q[k]);
      if (MODE == kStage2) {
        T a[12];
        load12(p.ua, nc, e, a);
#pragma unroll
        for (int k = 0; k < 12; ++k) o[k] = T(0.5) * (a[k] + o[k]);
      }
    }
#pragma unroll
    for (int k = 0; k < 12; ++k) p.out[k * nc + e] = o[k];
    if (MODE == kStage2 && p.dtpart) {
      // CFL bound 2V / sum_f A (|v.n| + c) from the new means
      const double r = o[0], ir = 1.0 / r, ux = o[3] * ir, uy = o[6] * ir;
      const double pr = ((double)p.gamma - 1.0) * (o[9] - 0.5 * r * (ux * ux + uy * uy));
      const double cs = sqrt((double)p.gamma * pr * ir);
      double s = cs * (double)p.perim[e];
      for (int i = p.lim_inc0[e]; i < p.lim_inc0[e + 1]; ++i)
        s += fabs(ux * (double)p.lim_an[2 * i] + uy * (double)p.lim_an[2 * i + 1]);
      dtmin = 2.0 / ((double)iV * s);
    }
  }
  if (bad) atomicOr(p.status, 1);
  if (MODE == kStage2 && p.dtpart) {
    dtmin = wave_min(dtmin);
    __shared__ double sd[kBlock / 64];
    if ((threadIdx.x & 63) == 0) sd[threadIdx.x >> 6] = dtmin;
    __syncthreads();
    if (threadIdx.x == 0) {
      double m = sd[0];
      for (int w = 1; w < kBlock / 64; ++w) m = fmin(m, sd[w]);
      p.dtpart[b] = m;
    }
  }
}

template <typename T>
__global__ __launch_bounds__(256) void k_fl_cfl(PF<T> p) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  double d = 1e300;
  if (e < p.ncells) {
    const double r = p.in[e], ir = 1.0 / r, ux = p.in[3 * p.nc + e] * ir,
                 uy = p.in[6 * p.nc + e] * ir;
    const double pr =
        ((double)p.gamma - 1.0) * (p.in[9 * p.nc + e] - 0.5 * r * (ux * ux + uy * uy));
    const double cs = sqrt((double)p.gamma * pr * ir);
    double s = cs * (double)p.perim[e];
    for (int i = p.lim_inc0[e]; i < p.lim_inc0[e + 1]; ++i)
      s += fabs(ux * (double)p.lim_an[2 * i] + uy * (double)p.lim_an[2 * i + 1]);
    d = 2.0 / ((double)p.cell_geo[8 * (size_t)e] * s);
  }
  d = wave_min(d);
  if ((threadIdx.x & 63) == 0) p.dtpart[e >> 6] = d;
}

template <typename T>
PF<T> make_params(const dg_mesh* m, const void* in, const void* ua, void* out,
                  const double* dt_dev, double dt_host) {
  const FLDev& f = *m->fld;
  PF<T> p;
  p.in = static_cast<const T*>(in);
  p.ua = static_cast<const T*>(ua);
  p.out = static_cast<T*>(out);
  p.dt_dev = dt_dev;
  p.dt_host = dt_host;
  p.status = m->status;
  p.dtpart = nullptr;
  p.ncells = f.ncells;
  p.nc = f.ncells;
  p.gamma = (T)m->cfg.gamma;
  p.blk_cell0 = f.blk_cell0;
  p.blk_slot0 = f.blk_slot0;
  p.slot_cells = f.slot_cells;
  p.slot_geo = static_cast<const T*>(f.slot_geo);
  p.cell_inc0 = f.cell_inc0;
  p.cell_inc = f.cell_inc;
  p.inc_geo = static_cast<const T*>(f.inc_geo);
  p.cell_geo = static_cast<const T*>(f.cell_geo);
  p.lim_inc0 = f.lim_inc0;
  p.lim_nbr = f.lim_nbr;
  p.lim_geo = static_cast<const T*>(f.lim_geo);
  p.lim_an = p.lim_geo + 2 * f.ninc;
  p.perim = static_cast<const T*>(f.cell_perim);
  return p;
}

template <typename T>
hipError_t lim_t(const dg_mesh* m, const void* in, void* out, hipStream_t s) {
  PF<T> p = make_params<T>(m, in, nullptr, out, nullptr, 0.0);
  hipLaunchKernelGGL((k_fl_lim<T>), dim3((p.ncells + 255) / 256), dim3(256), 0, s, p);
  return hipGetLastError();
}

template <typename T>
hipError_t rhs_t(const dg_mesh* m, int mode, const void* in, const void* ua, void* out,
                 const double* dt_dev, double dt_host, bool want_dt, hipStream_t s) {
  PF<T> p = make_params<T>(m, in, ua, out, dt_dev, dt_host);
  if (want_dt) p.dtpart = m->dtpart;
  const dim3 g(m->fld->nblocks), b(kBlock);
  switch (mode) {
    case kRhs:
      hipLaunchKernelGGL((k_fl_rhs<T, kRhs>), g, b, 0, s, p);
      break;
    case kStage1:
      hipLaunchKernelGGL((k_fl_rhs<T, kStage1>), g, b, 0, s, p);
      break;
    case kStage2:
      hipLaunchKernelGGL((k_fl_rhs<T, kStage2>), g, b, 0, s, p);
      break;
    default:
      return hipErrorInvalidValue;
  }
  return hipGetLastError();
}

template <typename T>
hipError_t cfl_t(const dg_mesh* m, const void* U, hipStream_t s) {
  PF<T> p = make_params<T>(m, U, nullptr, nullptr, nullptr, 0.0);
  p.dtpart = m->dtpart;
  hipLaunchKernelGGL((k_fl_cfl<T>), dim3((p.ncells + 255) / 256), dim3(256), 0, s, p);
  return hipGetLastError();
}

// ------------------------------------------------------------ host setup --
template <typename T>
hipError_t upload(const std::vector<double>& h, void** d) {
  std::vector<T> t(h.begin(), h.end());
  hipError_t e = hipMalloc(d, sizeof(T) * std::max<size_t>(t.size(), 1));
  if (e == hipSuccess && !t.empty())
    e = hipMemcpy(*d, t.data(), sizeof(T) * t.size(), hipMemcpyHostToDevice);
  return e;
}

hipError_t upload_i(const std::vector<int>& h, int** d) {
  hipError_t e = hipMalloc((void**)d, sizeof(int) * std::max<size_t>(h.size(), 1));
  if (e == hipSuccess && !h.empty())
    e = hipMemcpy(*d, h.data(), sizeof(int) * h.size(), hipMemcpyHostToDevice);
  return e;
}

}  // namespace

void facelist_destroy(dg_mesh* m);

dg_status facelist_create(dg_mesh* m, const dg_mesh_desc* d) {
  const int64_t nc = d->ncells, nf = d->nfaces;
  if (nc < 1 || nf < 1) {
    set_error("dg_mesh_create: face list needs ncells >= 1 and nfaces >= 1");
    return DG_EINVAL;
  }
  if (!d->cell_volume || !d->cell_centroid || !d->cell_moments || !d->face_cells ||
      !d->face_area || !d->face_normal || !d->face_centroid || !d->face_shift) {
    set_error("dg_mesh_create: face list with a NULL array");
    return DG_EINVAL;
  }
  if (!(d->box[0] > 0) || !(d->box[1] > 0)) {
    set_error("dg_mesh_create: face list box must be positive");
    return DG_EINVAL;
  }
  const double bx[2] = {d->box[0], d->box[1]};
  // validation: indices, positive sizes, unit normals, closure
  std::vector<double> closure(2 * nc, 0.0), perim(nc, 0.0);
  for (int64_t f = 0; f < nf; ++f) {
    const int L = d->face_cells[2 * f], R = d->face_cells[2 * f + 1];
    if (L < 0 || L >= nc || R < 0 || R >= nc) {
      set_error("dg_mesh_create: face " + std::to_string(f) + " has a cell index out of range");
      return DG_EINVAL;
    }
    const double A = d->face_area[f], nx = d->face_normal[2 * f], ny = d->face_normal[2 * f + 1];
    if (!(A > 0) || std::fabs(nx * nx + ny * ny - 1.0) > 1e-10) {
      set_error("dg_mesh_create: face " + std::to_string(f) + " needs A > 0 and a unit normal");
      return DG_EINVAL;
    }
    for (int k = 0; k < 2; ++k) {
      const int s = d->face_shift[2 * f + k];
      if (s < -1 || s > 1) {
        set_error("dg_mesh_create: face shifts must be -1, 0 or 1");
        return DG_EINVAL;
      }
    }
    closure[2 * L] += A * nx;
    closure[2 * L + 1] += A * ny;
    closure[2 * R] -= A * nx;
    closure[2 * R + 1] -= A * ny;
    perim[L] += A;
    perim[R] += A;
  }
  for (int64_t e = 0; e < nc; ++e) {
    const double V = d->cell_volume[e];
    const double a = d->cell_moments[3 * e], b = d->cell_moments[3 * e + 1],
                 c = d->cell_moments[3 * e + 2];
    if (!(V > 0) || !(a > 0) || !(c > 0) || !(a * c - b * b > 0)) {
      set_error("dg_mesh_create: cell " + std::to_string(e) +
                " needs V > 0 and positive-definite moments");
      return DG_EINVAL;
    }
    if (std::hypot(closure[2 * e], closure[2 * e + 1]) > 1e-9 * perim[e]) {
      set_error("dg_mesh_create: cell " + std::to_string(e) + " is not closed (sum A n != 0)");
      return DG_EINVAL;
    }
  }
  // per-cell geometry: 1/V, M^-1, scaled principal axes
  std::vector<double> cgeo(8 * nc);
  for (int64_t e = 0; e < nc; ++e) {
    const double V = d->cell_volume[e];
    const double a = d->cell_moments[3 * e], b = d->cell_moments[3 * e + 1],
                 c = d->cell_moments[3 * e + 2];
    const double det = a * c - b * b;
    // inverse mass matrix per unit volume: V * M^-1
    cgeo[8 * e] = 1.0 / V;
    cgeo[8 * e + 1] = V * c / det;
    cgeo[8 * e + 2] = -V * b / det;
    cgeo[8 * e + 3] = V * a / det;
    const double tr = 0.5 * (a + c), disc = std::sqrt(0.25 * (a - c) * (a - c) + b * b);
    const double lam[2] = {tr + disc, tr - disc};
    double ev[2][2];
    if (b == 0.0) {
      if (a >= c) {
        ev[0][0] = 1; ev[0][1] = 0; ev[1][0] = 0; ev[1][1] = 1;
      } else {
        ev[0][0] = 0; ev[0][1] = 1; ev[1][0] = 1; ev[1][1] = 0;
      }
    } else {
      for (int k = 0; k < 2; ++k) {
        const double vx = b, vy = lam[k] - a, nn = std::hypot(vx, vy);
        ev[k][0] = vx / nn;
        ev[k][1] = vy / nn;
      }
    }
    for (int k = 0; k < 2; ++k) {
      const double r = std::sqrt(2.0 * lam[k] / V);
      cgeo[8 * e + 4 + 2 * k] = r * ev[k][0];
      cgeo[8 * e + 5 + 2 * k] = r * ev[k][1];
    }
  }
  // global incidence CSR (limiter, CFL): per cell its faces as seen from it
  std::vector<int> inc0(nc + 1, 0);
  for (int64_t f = 0; f < nf; ++f) {
    inc0[d->face_cells[2 * f] + 1]++;
    inc0[d->face_cells[2 * f + 1] + 1]++;
  }
  for (int64_t e = 0; e < nc; ++e) inc0[e + 1] += inc0[e];
  std::vector<int> fill(inc0.begin(), inc0.end() - 1), nbr(inc0[nc]);
  // offsets of all incidences, then their A n (the limiter reads only the first block)
  const size_t ninc = (size_t)inc0[nc];
  std::vector<double> lgeo(4 * ninc);
  // face geometry offsets (from each side's centroid)
  auto offsets = [&](int64_t f, double* rc, double* dLR) {
    const int L = d->face_cells[2 * f], R = d->face_cells[2 * f + 1];
    for (int k = 0; k < 2; ++k) {
      rc[k] = d->face_centroid[2 * f + k] - d->cell_centroid[2 * L + k];
      dLR[k] = d->cell_centroid[2 * R + k] + d->face_shift[2 * f + k] * bx[k] -
               d->cell_centroid[2 * L + k];
    }
  };
  for (int64_t f = 0; f < nf; ++f) {
    const int L = d->face_cells[2 * f], R = d->face_cells[2 * f + 1];
    double rc[2], dLR[2];
    offsets(f, rc, dLR);
    const double A = d->face_area[f], nx = d->face_normal[2 * f], ny = d->face_normal[2 * f + 1];
    int i = fill[L]++;
    nbr[i] = R;
    lgeo[2 * i] = rc[0];
    lgeo[2 * i + 1] = rc[1];
    lgeo[2 * ninc + 2 * i] = A * nx;
    lgeo[2 * ninc + 2 * i + 1] = A * ny;
    i = fill[R]++;
    nbr[i] = L;
    lgeo[2 * i] = rc[0] - dLR[0];
    lgeo[2 * i + 1] = rc[1] - dLR[1];
    lgeo[2 * ninc + 2 * i] = -A * nx;
    lgeo[2 * ninc + 2 * i + 1] = -A * ny;
  }
  // face ids per cell (same order as the global CSR)
  std::vector<int> cface(inc0[nc]), cside(inc0[nc]);
  {
    std::vector<int> fl2(inc0.begin(), inc0.end() - 1);
    for (int64_t f = 0; f < nf; ++f) {
      const int L = d->face_cells[2 * f], R = d->face_cells[2 * f + 1];
      int i = fl2[L]++;
      cface[i] = (int)f;
      cside[i] = 0;
      i = fl2[R]++;
      cface[i] = (int)f;
      cside[i] = 1;
    }
  }
  // blocks of up to kBlock consecutive cells; a block is halved until its
  // distinct incident faces fit the LDS flux table
  std::vector<int> blk_cell0{0}, blk_slot0{0}, slot_cells, cell_inc0(nc + 1, 0), cell_inc;
  std::vector<double> sgeo, igeo;
  {
    std::vector<int64_t> mark(nf, -1);
    int64_t stamp = 0, e = 0;
    while (e < nc) {
      int64_t e1 = std::min<int64_t>(e + kBlock, nc);
      for (;;) {
        ++stamp;
        int ns = 0;
        for (int64_t c = e; c < e1; ++c)
          for (int i = inc0[c]; i < inc0[c + 1]; ++i)
            if (mark[cface[i]] != stamp) {
              mark[cface[i]] = stamp;
              ++ns;
            }
        if (ns <= kMaxSlots || e1 - e <= 1) break;
        e1 = e + (e1 - e) / 2;
      }
      blk_cell0.push_back((int)e1);
      e = e1;
    }
  }
  const int nblocks = (int)blk_cell0.size() - 1;
  std::vector<int> slot_of_face(nf, -1);
  int max_slots = 0;
  for (int b = 0; b < nblocks; ++b) {
    const int ca = blk_cell0[b], cb = blk_cell0[b + 1];
    const int first = (int)slot_cells.size() / 2;
    std::vector<int> touched;
    for (int c = ca; c < cb; ++c) {
      for (int i = inc0[c]; i < inc0[c + 1]; ++i) {
        const int f = cface[i];
        if (slot_of_face[f] < 0) {
          slot_of_face[f] = (int)slot_cells.size() / 2 - first;
          touched.push_back(f);
          const int L = d->face_cells[2 * f], R = d->face_cells[2 * f + 1];
          slot_cells.push_back(L);
          slot_cells.push_back(R);
          double rc[2], dLR[2];
          offsets(f, rc, dLR);
          const double A = d->face_area[f], nx = d->face_normal[2 * f],
                       ny = d->face_normal[2 * f + 1];
          const double o = A / (2.0 * std::sqrt(3.0));
          const double t[2] = {-ny, nx};
          const double rL0[2] = {rc[0] - o * t[0], rc[1] - o * t[1]};
          const double rL1[2] = {rc[0] + o * t[0], rc[1] + o * t[1]};
          const double g[10] = {nx, ny, 0.5 * A, rL0[0], rL0[1], rL1[0], rL1[1],
                                rL0[0] - dLR[0], rL0[1] - dLR[1], 0.0};
          sgeo.insert(sgeo.end(), g, g + 10);
        }
        cell_inc.push_back(slot_of_face[f] * 2 + cside[i]);
        {
          // this side's weight and Gauss-point offsets (R: rR1 = rR0 + (rL1 - rL0))
          double rc[2], dLR[2];
          offsets(f, rc, dLR);
          const double A = d->face_area[f], nx = d->face_normal[2 * f],
                       ny = d->face_normal[2 * f + 1];
          const double o = A / (2.0 * std::sqrt(3.0));
          const double t[2] = {-ny, nx};
          const double rL0[2] = {rc[0] - o * t[0], rc[1] - o * t[1]};
          const double rL1[2] = {rc[0] + o * t[0], rc[1] + o * t[1]};
          if (cside[i] == 0) {
            const double r[5] = {-0.5 * A, rL0[0], rL0[1], rL1[0], rL1[1]};
            igeo.insert(igeo.end(), r, r + 5);
          } else {
            const double rR0[2] = {rL0[0] - dLR[0], rL0[1] - dLR[1]};
            const double r[5] = {0.5 * A, rR0[0], rR0[1], rR0[0] + (rL1[0] - rL0[0]),
                                 rR0[1] + (rL1[1] - rL0[1])};
            igeo.insert(igeo.end(), r, r + 5);
          }
        }
      }
      cell_inc0[c + 1] = (int)cell_inc.size();
    }
    for (int f : touched) slot_of_face[f] = -1;
    const int ns = (int)slot_cells.size() / 2 - first;
    if (ns > kMaxSlots) {
      set_error("dg_mesh_create: a cell block has too many incident faces");
      return DG_EINVAL;
    }
    max_slots = std::max(max_slots, ns);
    blk_slot0.push_back((int)slot_cells.size() / 2);
  }
  FLDev* fd = new FLDev();
  std::memset(fd, 0, sizeof(FLDev));
  fd->ncells = (int)nc;
  fd->nblocks = nblocks;
  fd->max_slots = max_slots;
  fd->ninc = (int64_t)ninc;
  m->fld = fd;
  m->fl.nblocks = nblocks;
  m->ncells = nc;
  const bool f64 = m->cfg.precision == DG_FP64;
  hipError_t err = upload_i(blk_cell0, &fd->blk_cell0);
  if (err == hipSuccess) err = upload_i(blk_slot0, &fd->blk_slot0);
  if (err == hipSuccess) err = upload_i(slot_cells, &fd->slot_cells);
  if (err == hipSuccess) err = upload_i(cell_inc0, &fd->cell_inc0);
  if (err == hipSuccess) err = upload_i(cell_inc, &fd->cell_inc);
  if (err == hipSuccess) err = upload_i(inc0, &fd->lim_inc0);
  if (err == hipSuccess) err = upload_i(nbr, &fd->lim_nbr);
  auto up = [&](const std::vector<double>& h, void** dst) {
    return f64 ? upload<double>(h, dst) : upload<float>(h, dst);
  };
  if (err == hipSuccess) err = up(sgeo, &fd->slot_geo);
  if (err == hipSuccess) err = up(igeo, &fd->inc_geo);
  if (err == hipSuccess) err = up(cgeo, &fd->cell_geo);
  if (err == hipSuccess) err = up(lgeo, &fd->lim_geo);
  if (err == hipSuccess) err = up(perim, &fd->cell_perim);
  if (err != hipSuccess) {
    facelist_destroy(m);
    return hip_fail(err, "dg_mesh_create: face-list upload");
  }
  return DG_OK;
}

void facelist_destroy(dg_mesh* m) {
  FLDev* f = m->fld;
  if (!f) return;
  (void)hipFree(f->blk_cell0);
  (void)hipFree(f->blk_slot0);
  (void)hipFree(f->slot_cells);
  (void)hipFree(f->slot_geo);
  (void)hipFree(f->cell_inc0);
  (void)hipFree(f->cell_inc);
  (void)hipFree(f->inc_geo);
  (void)hipFree(f->cell_geo);
  (void)hipFree(f->lim_inc0);
  (void)hipFree(f->lim_nbr);
  (void)hipFree(f->lim_geo);
  (void)hipFree(f->cell_perim);
  delete f;
  m->fld = nullptr;
}

hipError_t launch_min_finalize(const double* part, int n, double cfl, double* dt, hipStream_t s);

hipError_t launch_facelist(const dg_mesh* m, int mode, const void* in, const void* u0, void* out,
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
      const void* ua = u0;
      const void* b = in;
      if (lim) {
        if (!(m->ws_a_fresh && m->ws_a_src == u0)) e = limit(u0, m->ws_a);
        ua = m->ws_a;
        if (e == hipSuccess) e = limit(in, m->ws_b);
        b = m->ws_b;
      }
      if (e == hipSuccess) e = rhs(kStage2, b, ua, out, dt_next != nullptr);
      if (e == hipSuccess && dt_next) e = launch_min_finalize(m->dtpart, m->fld->nblocks, cfl, dt_next, s);
      return e;
    }
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_facelist_cfl(const dg_mesh* m, const void* U, double cfl, double* dt_dev,
                               hipStream_t s) {
  hipError_t e = m->cfg.precision == DG_FP64 ? cfl_t<double>(m, U, s) : cfl_t<float>(m, U, s);
  if (e != hipSuccess) return e;
  return launch_min_finalize(m->dtpart, (m->fld->ncells + 63) / 64, cfl, dt_dev, s);
}

}  // namespace dg
