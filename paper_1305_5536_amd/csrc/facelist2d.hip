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
// lists, per block, its "halo" (the outside cells that share a face with it)
// and every face incident to one of its cells ("slots": faces on the block
// boundary appear in both blocks), each slot with its two cells' block-local
// indices and one geometry record (unit normal, length, face-centroid offset
// from L's centroid, offset from L's centroid to R's periodic image), and per
// cell its incidences (slot, side) with the face-centroid offset from the
// cell's own centroid.  One workgroup per block, limit on read:
//   0. the raw coefficients of the block's cells and of its halo go to LDS;
//   1. each cell of the block is limited from its neighbours' means in LDS and
//      its incidences' face-centroid offsets; each halo cell from the global
//      face lists (its neighbours' means gathered); the limited gradients
//      replace the raw ones in LDS;
//   2. the slots' Riemann problems (HLL at both Gauss points, which sit at the
//      face centroid -+ A/(2 sqrt 3) along the tangent) go to an LDS table as
//      the weighted sum and half-difference of the two fluxes and A n, half
//      the slots at a time;
//   3. each cell gathers its incidences from that table (a segmented
//      reduction, no atomics);
//   4. the volume term, M^-1 and the RK combination (stage 2 takes Pi(U^n),
//      which stage 1 wrote, for the combination).
// Loads of later phases that depend on nothing the block computes (incidence
// ranges and entries, geometry, Pi(U^n), the first pass's slots) are issued
// before the first barrier, so that their latency overlaps phase 0.
// A stand-alone limiter kernel (k_fl_lim) serves dg_limit.  The discrete
// adjoint of a step (k_adjfl_L, k_adjfl_lim) gathers over the global incidence
// lists, one thread per cell.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstring>
#include <string>
#include <vector>

#include "dg_internal.h"
#include "dg_math.h"
#include "dual.h"

namespace dg {

// Device arrays of a face-list mesh (allocated at create, in the mesh's
// working precision for geometry).
struct FLDev {
  int ncells, nblocks, max_slots;
  int64_t ninc;       // incidences of the global CSR (2 x faces)
  int* blk_cell0;     // [nblocks+1] first cell of each block
  int* blk_slot0;     // [nblocks+1] first slot of each block
  int* blk_halo0;     // [nblocks+1] first halo entry of each block
  int* halo_cell;     // global index of each halo cell
  int* slot_lr;       // [nslots] block-local L | R << 16 (own cell i: i; halo h: nown + h)
  void* slot_geo;     // [nslots][8] nx, ny, A, x_f - c_L (2), c_R' - c_L (2), 0
  int* cell_inc0;     // [ncells+1] block-local CSR start (global index into cell_inc)
  int* cell_inc;      // slot_local*2 + side | neighbour's block-local index << 16,
                      // each cell's incidences by slot
  void* inc_rf;       // [per cell_inc entry][2] face centroid - the cell's own centroid
  void* cell_geo;     // [ncells][8] 1/V, V Minv00, V Minv01, V Minv11, a1x, a1y, a2x, a2y
  int* lim_inc0;      // [ncells+1] global CSR for k_fl_lim, halo cells and the CFL bound
  int* lim_nbr;       // neighbour cell of each incidence
  void* lim_geo;      // [ninc][2] face-centroid offsets, then [ninc][2] A n outward
  void* cell_perim;   // [ncells] sum of face lengths
  // the discrete adjoint (gathers over the global CSR)
  int* inc_face;      // [ninc] face id << 1 | side (0: the cell is L) of each incidence
  int* face_lr;       // [nfaces][2] L, R
  void* face_geo;     // [nfaces][8] nx, ny, A, x_f - c_L (2), c_R' - c_L (2), 0
};

namespace {

constexpr int kBlock = 256;      // cells of a block at most (one thread each)
constexpr int kMaxSlots = 1024;  // distinct faces of a block
constexpr int kMaxHalo = 128;    // outside neighbours of a block
constexpr int kHalf = 512;       // slots per pass of the LDS flux table
constexpr int kLocal = kBlock + kMaxHalo;

template <typename T>
struct PF {
  const T* __restrict__ in;
  const T* __restrict__ ua;
  T* __restrict__ out;
  T* __restrict__ lim_out;  // stage 1: Pi(in) of each cell (NULL: not kept)
  const double* dt_dev;
  double dt_host;
  int* status;
  double* dtpart;
  int ncells, nc;
  T gamma;
  const int* blk_cell0;
  const int* blk_slot0;
  const int* blk_halo0;
  const int* halo_cell;
  const int* slot_lr;
  const T* slot_geo;
  const int* cell_inc0;
  const int* cell_inc;
  const T* inc_rf;
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

// ------------------------------------------------------------ stage --
// alpha = min(1, min_f psi_f) of one conserved variable (Sec. 2.5): psi from
// the face-centroid increment d = g . (x_f - c) and the bounds hi, lo of the
// means of the cell and its face neighbours.
template <typename T>
__device__ __forceinline__ T psi_of(T d, T phi, T hi, T lo) {
  const T num = d > T(0) ? hi - phi : lo - phi;
  return d > T(0) ? div_small(num, d) : (d < T(0) ? div_small(-num, -d) : T(1));
}

// Limit the gradients of q (12 coefficients, means untouched) of a block cell
// whose incidences are [i0, i1) of the block-local CSR, from the block-local
// means m[v][local] in LDS.  Incidences are taken kInc at a time with all
// their loads in flight; padding entries repeat the cell itself (no change to
// a bound, psi = 1).
constexpr int kInc = 4;
constexpr int kPre = 2 * kInc;  // incidences of a cell loaded ahead (two batches)

// Incidence i's entries of the block-local CSR for the batch starting at b0
// (padding repeats the batch's first entry, a batch past the end the cell's
// first, so every index stays inside the cell's list).  Only the entries are
// loaded ahead; the offsets of the alpha pass are loaded where they are used,
// with nothing they wait on.
__device__ __forceinline__ int batch_index(int b0, int u, int i0, int i1) {
  return b0 + u < i1 ? b0 + u : (b0 < i1 ? b0 : i0);
}

struct IncPre {  // a cell's first kPre incidences, loaded before the block's first barrier
  int inc[kPre];
};

template <typename T>
__device__ __forceinline__ void load_inc_pre(const PF<T>& p, int i0, int i1, IncPre& a) {
#pragma unroll
  for (int u = 0; u < kPre; ++u)
    a.inc[u] = p.cell_inc[batch_index(i0 + (u / kInc) * kInc, u % kInc, i0, i1)];
}

template <typename T>
__device__ __forceinline__ void limit_block_cell(const PF<T>& p, int i0, int i1, int self,
                                                 const T (*m)[kLocal], T* q,
                                                 const IncPre& pre) {
  T hi[4], lo[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) hi[v] = lo[v] = q[3 * v];
  T alpha[4] = {T(1), T(1), T(1), T(1)};
  auto bound = [&](int nbu) {
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      const T mm = m[3 * v][nbu];
      hi[v] = fmax(hi[v], mm);
      lo[v] = fmin(lo[v], mm);
    }
  };
  auto limit_by = [&](T rx, T ry) {
#pragma unroll
    for (int v = 0; v < 4; ++v)
      alpha[v] = fmin(alpha[v], psi_of(q[3 * v + 1] * rx + q[3 * v + 2] * ry, q[3 * v],
                                       hi[v], lo[v]));
  };
  // batches of kInc in incidence order, the first two from registers
#pragma unroll
  for (int u = 0; u < kPre; ++u) {
    const int b0 = i0 + (u / kInc) * kInc;
    if (b0 < i1) bound(b0 + u % kInc < i1 ? (pre.inc[u] >> 16) : self);
  }
  for (int b0 = i0 + kPre; b0 < i1; b0 += kInc) {
    int nb[kInc];
#pragma unroll
    for (int u = 0; u < kInc; ++u) nb[u] = b0 + u < i1 ? (p.cell_inc[b0 + u] >> 16) : self;
#pragma unroll
    for (int u = 0; u < kInc; ++u) bound(nb[u]);
  }
  for (int b0 = i0; b0 < i1; b0 += kInc) {
    T rx[kInc], ry[kInc];
#pragma unroll
    for (int u = 0; u < kInc; ++u) {
      const int i = b0 + u < i1 ? b0 + u : b0;
      rx[u] = p.inc_rf[2 * (size_t)i];
      ry[u] = p.inc_rf[2 * (size_t)i + 1];
    }
#pragma unroll
    for (int u = 0; u < kInc; ++u) limit_by(rx[u], ry[u]);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    q[3 * v + 1] *= alpha[v];
    q[3 * v + 2] *= alpha[v];
  }
}

// The same limiter for a cell outside the block (a halo cell) from the global
// face lists: neighbour means gathered from `U`, eight incidences at a time
// with all their loads in flight (padding repeats the cell itself).  The
// cell's incidence range and first eight neighbours come preloaded.
constexpr int kHB = 8;
struct HaloPre {
  int i0, i1;
  int nb[kHB];
};

template <typename T>
__device__ __forceinline__ void load_halo_pre(const PF<T>& p, int e, HaloPre& a) {
  a.i0 = p.lim_inc0[e];
  a.i1 = p.lim_inc0[e + 1];
#pragma unroll
  for (int u = 0; u < kHB; ++u) a.nb[u] = a.i0 + u < a.i1 ? p.lim_nbr[a.i0 + u] : e;
}

template <typename T>
__device__ __forceinline__ void limit_global_cell(const PF<T>& p, const T* __restrict__ U, int e,
                                                  T* q, const HaloPre& pre) {
  T hi[4], lo[4];
#pragma unroll
  for (int v = 0; v < 4; ++v) hi[v] = lo[v] = q[3 * v];
  const int i0 = pre.i0, i1 = pre.i1;
  auto bounds = [&](const int* nb) {
    T m[kHB][4];
#pragma unroll
    for (int u = 0; u < kHB; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) m[u][v] = U[(3 * v) * p.nc + nb[u]];
#pragma unroll
    for (int u = 0; u < kHB; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        hi[v] = fmax(hi[v], m[u][v]);
        lo[v] = fmin(lo[v], m[u][v]);
      }
  };
  T alpha[4] = {T(1), T(1), T(1), T(1)};
  auto limit_by = [&](const T* rx, const T* ry) {
#pragma unroll
    for (int u = 0; u < kHB; ++u)
#pragma unroll
      for (int v = 0; v < 4; ++v)
        alpha[v] = fmin(alpha[v], psi_of(q[3 * v + 1] * rx[u] + q[3 * v + 2] * ry[u], q[3 * v],
                                         hi[v], lo[v]));
  };
  if (i0 < i1) bounds(pre.nb);
  for (int b0 = i0 + kHB; b0 < i1; b0 += kHB) {
    int nb[kHB];
#pragma unroll
    for (int u = 0; u < kHB; ++u) nb[u] = b0 + u < i1 ? p.lim_nbr[b0 + u] : e;
    bounds(nb);
  }
  for (int b0 = i0; b0 < i1; b0 += kHB) {
    T rx[kHB], ry[kHB];
#pragma unroll
    for (int u = 0; u < kHB; ++u) {
      const int i = b0 + u < i1 ? b0 + u : b0;
      rx[u] = p.lim_geo[2 * i];
      ry[u] = p.lim_geo[2 * i + 1];
    }
    limit_by(rx, ry);
  }
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    q[3 * v + 1] *= alpha[v];
    q[3 * v + 2] *= alpha[v];
  }
}

// One stage (MODE kRhs, kStage1, kStage2) of a block of cells; LIM: limit on
// read (Pi of `in`, and in stage 2 Pi of `ua` for the combination).
template <typename T, int MODE, bool LIM>
__global__ __launch_bounds__(kBlock) void k_fl_step(PF<T> p) {
  __shared__ T cU[12][kLocal];  // coefficients of the block's and the halo's cells
  __shared__ T sF[10][kHalf];   // per slot: w (F0 + F1), w (F1 - F0)/2, A n
  const int b = xcd_remap(blockIdx.x, gridDim.x);
  const int tid = threadIdx.x;
  const int c0 = p.blk_cell0[b], nown = p.blk_cell0[b + 1] - c0;
  const int h0 = p.blk_halo0[b], nhalo = p.blk_halo0[b + 1] - h0;
  const int s0 = p.blk_slot0[b], nslot = p.blk_slot0[b + 1] - s0;
  const int nc = p.nc;
  bool bad = false;
  const int e = c0 + tid;
  // Loads that later phases need, issued before the first barrier so that
  // their latency overlaps phase 0 (the LDS sets the occupancy, two
  // workgroups per CU, so these registers cost none): the cell's incidence
  // range, first incidences, geometry and (stage 2) Pi(U^n) row; the halo
  // cell's first neighbours; this thread's slots of the first flux pass.
  int i0 = 0, i1 = 0;
  T cg[8], ua[12];
  IncPre ipre;
  HaloPre hpre;
  int f0 = 0, f1 = 0;  // stage 2's CFL bound: the cell's global incidence range
  if (tid < nown) {
    i0 = p.cell_inc0[e];
    i1 = p.cell_inc0[e + 1];
#pragma unroll
    for (int k = 0; k < 8; ++k) cg[k] = p.cell_geo[8 * (size_t)e + k];
    if (MODE == kStage2) {
      load12(p.ua, nc, e, ua);
      if (p.dtpart) {
        f0 = p.lim_inc0[e];
        f1 = p.lim_inc0[e + 1];
      }
    }
  }
  int hg = 0;
  if (LIM && tid < nhalo) {
    hg = p.halo_cell[h0 + tid];
    load_halo_pre(p, hg, hpre);
  }
  if (LIM && tid < nown) load_inc_pre(p, i0, i1, ipre);
  constexpr int kSP = kHalf / kBlock;  // slots per thread and flux pass
  int slr[kSP];
  T sgeo[kSP][7];
#pragma unroll
  for (int j = 0; j < kSP; ++j) {
    const int sl = tid + j * kBlock;
    if (sl < min(nslot, kHalf)) {
      slr[j] = p.slot_lr[s0 + sl];
#pragma unroll
      for (int k = 0; k < 7; ++k) sgeo[j][k] = p.slot_geo[8 * (size_t)(s0 + sl) + k];
    }
  }
  // 0. raw coefficients of the block's cells and its halo
  for (int i = tid; i < nown + nhalo; i += kBlock) {
    const int g = i < nown ? c0 + i : p.halo_cell[h0 + i - nown];
#pragma unroll
    for (int k = 0; k < 12; ++k) cU[k][i] = p.in[k * nc + g];
  }
  __syncthreads();
  // 1. limit on read (the limiter reads only means; only gradients change)
  T q[12];
  if (tid < nown) {
#pragma unroll
    for (int k = 0; k < 12; ++k) q[k] = cU[k][tid];
  }
  if (LIM) {
    T qh[12];
    if (tid < nhalo) {
#pragma unroll
      for (int k = 0; k < 12; ++k) qh[k] = cU[k][nown + tid];
      limit_global_cell(p, p.in, hg, qh, hpre);
    }
    if (tid < nown) {
      limit_block_cell(p, i0, i1, tid, cU, q, ipre);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        cU[3 * v + 1][tid] = q[3 * v + 1];
        cU[3 * v + 2][tid] = q[3 * v + 2];
      }
      // stage 1 hands Pi(U^n) of its cells to stage 2's combination
      if (MODE == kStage1 && p.lim_out) {
#pragma unroll
        for (int k = 0; k < 12; ++k) p.lim_out[k * nc + e] = q[k];
      }
    }
    if (tid < nhalo) {
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        cU[3 * v + 1][nown + tid] = qh[3 * v + 1];
        cU[3 * v + 2][nown + tid] = qh[3 * v + 2];
      }
    }
    __syncthreads();
  }
  // 2-3. slot fluxes into LDS, half the slots at a time; each cell gathers its
  // incidences of the half (they are sorted by slot)
  T rm[4] = {T(0), T(0), T(0), T(0)};
  T rx[4] = {T(0), T(0), T(0), T(0)};
  T ry[4] = {T(0), T(0), T(0), T(0)};
  const T is3 = T(0.57735026918962576451);  // 1/sqrt(3)
  int ii = i0;
  for (int sa = 0; sa < nslot; sa += kHalf) {
    const int sb = min(nslot, sa + kHalf);
#pragma unroll
    for (int j = 0; j < kSP; ++j) {
      const int sl = sa + tid + j * kBlock;
      if (sl >= sb) break;
      int lr;
      T g[7];
      if (sa == 0) {
        lr = slr[j];
#pragma unroll
        for (int k = 0; k < 7; ++k) g[k] = sgeo[j][k];
      } else {
        lr = p.slot_lr[s0 + sl];
#pragma unroll
        for (int k = 0; k < 7; ++k) g[k] = p.slot_geo[8 * (size_t)(s0 + sl) + k];
      }
      const int L = lr & 0xffff, R = lr >> 16;
      const T nx = g[0], ny = g[1], A = g[2], fx = g[3], fy = g[4], dx = g[5], dy = g[6];
      // Gauss points x_f -+ A/(2 sqrt 3) t, t = (-n_y, n_x), from L's centroid
      const T o = T(0.5) * A * is3;
      const T tx = -ny * o, ty = nx * o;
      T uL[4], uR[4], F0[4], F1[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const T gLx = cU[3 * v + 1][L], gLy = cU[3 * v + 2][L];
        const T gRx = cU[3 * v + 1][R], gRy = cU[3 * v + 2][R];
        uL[v] = cU[3 * v][L] + gLx * (fx - tx) + gLy * (fy - ty);
        uR[v] = cU[3 * v][R] + gRx * (fx - tx - dx) + gRy * (fy - ty - dy);
      }
      hll_n(uL, uR, nx, ny, p.gamma, F0, bad);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const T gLx = cU[3 * v + 1][L], gLy = cU[3 * v + 2][L];
        const T gRx = cU[3 * v + 1][R], gRy = cU[3 * v + 2][R];
        uL[v] = cU[3 * v][L] + gLx * (fx + tx) + gLy * (fy + ty);
        uR[v] = cU[3 * v][R] + gRx * (fx + tx - dx) + gRy * (fy + ty - dy);
      }
      hll_n(uL, uR, nx, ny, p.gamma, F1, bad);
      const T w = T(0.5) * A;
      const int ls = sl - sa;
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        sF[v][ls] = w * (F0[v] + F1[v]);
        sF[4 + v][ls] = T(0.5) * w * (F1[v] - F0[v]);
      }
      sF[8][ls] = A * nx;
      sF[9][ls] = A * ny;
    }
    __syncthreads();
    if (tid < nown) {
      // side 0 (L) takes -flux, side 1 (R) +flux; the Gauss-point offsets
      // from the cell's centroid are r_f -+ delta/2, delta = (A/sqrt3) t.
      // The half's incidences (sorted by slot) kInc at a time, loads first;
      // the first incidence of a later half ends the pass.
      bool stop = false;
      while (!stop && ii < i1) {
        int inc[kInc];
        T fx[kInc], fy[kInc];
#pragma unroll
        for (int u = 0; u < kInc; ++u) {
          const int i = ii + u < i1 ? ii + u : ii;
          inc[u] = p.cell_inc[i];
          fx[u] = p.inc_rf[2 * (size_t)i];
          fy[u] = p.inc_rf[2 * (size_t)i + 1];
        }
        int done = 0;
#pragma unroll
        for (int u = 0; u < kInc; ++u) {
          const int ls = ((inc[u] & 0xffff) >> 1) - sa;
          if (stop || ii + u >= i1 || ls >= kHalf) {
            stop = true;
            continue;
          }
          const T sg = (inc[u] & 1) ? T(1) : T(-1);
          const T Anx = sF[8][ls], Any = sF[9][ls];
          const T ddx = -Any * is3, ddy = Anx * is3;
#pragma unroll
          for (int v = 0; v < 4; ++v) {
            const T G = sg * sF[v][ls], K = sg * sF[4 + v][ls];
            rm[v] += G;
            rx[v] += fma(G, fx[u], K * ddx);
            ry[v] += fma(G, fy[u], K * ddy);
          }
          ++done;
        }
        ii += done;
      }
    }
    if (sb < nslot) __syncthreads();  // the next half overwrites the table
  }
  // 4. volume term, M^-1, RK combination
  double dtmin = 1e300;
  if (tid < nown) {
    const T iV = cg[0];
    const T m00 = cg[1], m01 = cg[2], m11 = cg[3];
    // volume term: 4 principal-axis points, weights V/4 (the 1/V of the
    // inverse mass matrix is folded in)
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
        // ua: Pi(U^n) (written by stage 1 of the same U^n, or by the
        // stand-alone limiter), U^n itself without a limiter
#pragma unroll
        for (int k = 0; k < 12; ++k) o[k] = T(0.5) * (ua[k] + o[k]);
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
      for (int i = f0; i < f1; ++i)
        s += fabs(ux * (double)p.lim_an[2 * i] + uy * (double)p.lim_an[2 * i + 1]);
      dtmin = 2.0 / ((double)iV * s);
    }
  }
  if (bad) atomicOr(p.status, 1);
  if (MODE == kStage2 && p.dtpart) {
    dtmin = wave_min(dtmin);
    __shared__ double sd[kBlock / 64];
    if ((tid & 63) == 0) sd[tid >> 6] = dtmin;
    __syncthreads();
    if (tid == 0) {
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
  p.lim_out = nullptr;
  p.dt_dev = dt_dev;
  p.dt_host = dt_host;
  p.status = m->status;
  p.dtpart = nullptr;
  p.ncells = f.ncells;
  p.nc = f.ncells;
  p.gamma = (T)m->cfg.gamma;
  p.blk_cell0 = f.blk_cell0;
  p.blk_slot0 = f.blk_slot0;
  p.blk_halo0 = f.blk_halo0;
  p.halo_cell = f.halo_cell;
  p.slot_lr = f.slot_lr;
  p.slot_geo = static_cast<const T*>(f.slot_geo);
  p.cell_inc0 = f.cell_inc0;
  p.cell_inc = f.cell_inc;
  p.inc_rf = static_cast<const T*>(f.inc_rf);
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
hipError_t step_t(const dg_mesh* m, int mode, const void* in, const void* ua, void* out,
                  void* lim_out, const double* dt_dev, double dt_host, bool want_dt,
                  hipStream_t s) {
  PF<T> p = make_params<T>(m, in, ua, out, dt_dev, dt_host);
  p.lim_out = static_cast<T*>(lim_out);
  if (want_dt) p.dtpart = m->dtpart;
  const dim3 g(m->fld->nblocks), b(kBlock);
  const bool lim = m->cfg.limiter == DG_LIMITER_MINMOD;
  switch (mode) {
    case kRhs:
      hipLaunchKernelGGL((k_fl_step<T, kRhs, false>), g, b, 0, s, p);
      break;
    case kStage1:
      if (lim)
        hipLaunchKernelGGL((k_fl_step<T, kStage1, true>), g, b, 0, s, p);
      else
        hipLaunchKernelGGL((k_fl_step<T, kStage1, false>), g, b, 0, s, p);
      break;
    case kStage2:
      if (lim)
        hipLaunchKernelGGL((k_fl_step<T, kStage2, true>), g, b, 0, s, p);
      else
        hipLaunchKernelGGL((k_fl_step<T, kStage2, false>), g, b, 0, s, p);
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

// ------------------------------------------------------- discrete adjoint --
// Adjoint of a stage (as for the Cartesian meshes):
//   out = Pi_P^T lamW,   lamW = c_id lam + c_L (dL/dW)^T lam + c_extra extra,
// W = Pi(P), the branch the forward step takes (dt frozen).  k_adjfl_L gathers
// lamW of a cell over its incidences and its volume points; k_adjfl_lim the
// limiter transpose.  One thread per cell, no atomics; the flux and limiter
// Jacobians come from forward-mode dual numbers through hll_n and the
// limiter arithmetic, the linear parts (Gauss-point extrapolation, the
// residual weights, M^-1) are transposed by hand.
template <typename T>
struct PFA {
  const T* W;      // Pi(P)
  const T* P;      // the stage input (k_adjfl_lim)
  const T* lam;    // adjoint of the stage output (k_adjfl_L)
  const T* extra;  // added to lamW with weight c_extra (may be NULL)
  const T* lamW;   // k_adjfl_lim input
  T* out;
  const double* dt_dev;
  double dt_host;
  double c_id, c_L_over_dt, c_extra;
  int nc;
  T gamma;
  const int* inc0;
  const int* nbr;
  const int* inc_face;
  const int* face_lr;
  const T* face_geo;
  const T* lim_geo;
  const T* cell_geo;
};

// Cotangents of a cell's residual sums from the adjoint of its time
// derivative: d mean = rm / V, d grad = (V M^-1) (r / V + vol / 4), with r the
// face moments sum_g w F_g (x_g - c) and vol the sums of the volume fluxes.
template <typename T>
struct Cot {
  T rm[4], rx[4], ry[4], vx[4], vy[4];
};

template <typename T>
__device__ __forceinline__ void cotangents(const T* lam, const T* cg, Cot<T>& c) {
  const T iV = cg[0], m00 = cg[1], m01 = cg[2], m11 = cg[3];
#pragma unroll
  for (int v = 0; v < 4; ++v) {
    const T gx = fma(m00, lam[3 * v + 1], m01 * lam[3 * v + 2]);
    const T gy = fma(m01, lam[3 * v + 1], m11 * lam[3 * v + 2]);
    c.rm[v] = iV * lam[3 * v];
    c.rx[v] = iV * gx;
    c.ry[v] = iV * gy;
    c.vx[v] = T(0.25) * gx;
    c.vy[v] = T(0.25) * gy;
  }
}

// Both Cartesian Euler fluxes at one state (the volume term's point flux).
template <typename S>
__device__ __forceinline__ void euler_xy(const S* u, S gamma, S* Fx, S* Fy) {
  const S ir = rcp(u[0]);
  const S ux = u[1] * ir, uy = u[2] * ir;
  const S pr = (gamma - S(1)) * (u[3] - S(0.5) * (u[1] * ux + u[2] * uy));
  Fx[0] = u[1];
  Fx[1] = u[1] * ux + pr;
  Fx[2] = u[2] * ux;
  Fx[3] = (u[3] + pr) * ux;
  Fy[0] = u[2];
  Fy[1] = u[1] * uy;
  Fy[2] = u[2] * uy + pr;
  Fy[3] = (u[3] + pr) * uy;
}

template <typename T>
__global__ __launch_bounds__(256) void k_adjfl_L(PFA<T> p) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= p.nc) return;
  const T is3 = T(0.57735026918962576451);  // 1/sqrt(3)
  T we[12], le[12], g[12];
  load12(p.W, p.nc, e, we);
  load12(p.lam, p.nc, e, le);
  const T* cge = p.cell_geo + 8 * (size_t)e;
  Cot<T> ce;
  cotangents(le, cge, ce);
#pragma unroll
  for (int k = 0; k < 12; ++k) g[k] = T(0);
  const Dual<T> dgam(p.gamma, T(0));
  for (int i = p.inc0[e]; i < p.inc0[e + 1]; ++i) {
    const int fs = p.inc_face[i], f = fs >> 1, side = fs & 1;
    const int nb = side ? p.face_lr[2 * f] : p.face_lr[2 * f + 1];
    const T* fg = p.face_geo + 8 * (size_t)f;
    const T nx = fg[0], ny = fg[1], A = fg[2], fx = fg[3], fy = fg[4], dx = fg[5], dy = fg[6];
    T wn[12], ln[12];
    load12(p.W, p.nc, nb, wn);
    load12(p.lam, p.nc, nb, ln);
    Cot<T> cn;
    cotangents(ln, p.cell_geo + 8 * (size_t)nb, cn);
    // Gauss points x_f -+ A/(2 sqrt 3) t, t = (-n_y, n_x); weights A/2; the L
    // cell takes -w F, the R cell +w F (mean and the moments about its
    // centroid).  Values of e and nb are selected element by element (an
    // array picked through a pointer would leave the registers).
    const T w = T(0.5) * A, o = T(0.5) * A * is3;
    const T tx = -ny * o, ty = nx * o;
    const T se = side ? T(1) : T(-1);
#pragma unroll 1
    for (int gp = 0; gp < 2; ++gp) {
      const T sg = gp ? T(1) : T(-1);
      const T rLx = fma(sg, tx, fx), rLy = fma(sg, ty, fy);
      const T rRx = rLx - dx, rRy = rLy - dy;
      const T rex = side ? rRx : rLx, rey = side ? rRy : rLy;
      const T rnx = side ? rLx : rRx, rny = side ? rLy : rRy;
      T uL[4], uR[4], Fb[4];
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        const T ue = we[3 * v] + we[3 * v + 1] * rex + we[3 * v + 2] * rey;
        const T un = wn[3 * v] + wn[3 * v + 1] * rnx + wn[3 * v + 2] * rny;
        uL[v] = side ? un : ue;
        uR[v] = side ? ue : un;
        Fb[v] = w * se * ((ce.rm[v] + ce.rx[v] * rex + ce.ry[v] * rey) -
                          (cn.rm[v] + cn.rx[v] * rnx + cn.ry[v] * rny));
      }
      T ub[4];
#pragma unroll 1
      for (int k = 0; k < 4; ++k) {
        Dual<T> dL[4], dR[4], F[4];
#pragma unroll
        for (int j = 0; j < 4; ++j) {
          dL[j] = Dual<T>(uL[j], T(side == 0 && j == k ? 1 : 0));
          dR[j] = Dual<T>(uR[j], T(side == 1 && j == k ? 1 : 0));
        }
        bool bad = false;
        hll_n(dL, dR, Dual<T>(nx, T(0)), Dual<T>(ny, T(0)), dgam, F, bad);
        T acc = T(0);
#pragma unroll
        for (int j = 0; j < 4; ++j) acc = fma(Fb[j], F[j].d, acc);
        ub[k] = acc;
      }
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        g[3 * v] += ub[v];
        g[3 * v + 1] = fma(rex, ub[v], g[3 * v + 1]);
        g[3 * v + 2] = fma(rey, ub[v], g[3 * v + 2]);
      }
    }
  }
  // volume term: the 4 principal-axis points c -+ a_k
#pragma unroll 1
  for (int q = 0; q < 4; ++q) {
    const T sgn = (q & 1) ? T(1) : T(-1);
    const T ox = sgn * ((q & 2) ? cge[6] : cge[4]);
    const T oy = sgn * ((q & 2) ? cge[7] : cge[5]);
    T u[4], ub[4];
#pragma unroll
    for (int v = 0; v < 4; ++v) u[v] = fma(we[3 * v + 1], ox, fma(we[3 * v + 2], oy, we[3 * v]));
#pragma unroll 1
    for (int k = 0; k < 4; ++k) {
      Dual<T> du[4], Fx[4], Fy[4];
#pragma unroll
      for (int j = 0; j < 4; ++j) du[j] = Dual<T>(u[j], T(j == k ? 1 : 0));
      euler_xy(du, dgam, Fx, Fy);
      T acc = T(0);
#pragma unroll
      for (int j = 0; j < 4; ++j) acc = fma(ce.vx[j], Fx[j].d, fma(ce.vy[j], Fy[j].d, acc));
      ub[k] = acc;
    }
#pragma unroll
    for (int v = 0; v < 4; ++v) {
      g[3 * v] += ub[v];
      g[3 * v + 1] = fma(ox, ub[v], g[3 * v + 1]);
      g[3 * v + 2] = fma(oy, ub[v], g[3 * v + 2]);
    }
  }
  const double dt = p.dt_dev ? *p.dt_dev : p.dt_host;
  const T cid = (T)p.c_id, cL = (T)(p.c_L_over_dt * dt), cx = (T)p.c_extra;
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    T o = fma(cL, g[k], cid * le[k]);
    if (p.extra) o = fma(cx, p.extra[(size_t)k * p.nc + e], o);
    p.out[(size_t)k * p.nc + e] = o;
  }
}

// out_e = sum over the cells n whose limiter reads P_e (e itself and its face
// neighbours, each counted once) of (d Pi_n / d P_e)^T lamW_n: the limiter of
// k_fl_lim (bounds over the cell and its neighbours in the incidence order,
// alpha = min over the incidences of psi at the face centroid) in dual numbers.
template <typename T>
__global__ __launch_bounds__(256) void k_adjfl_lim(PFA<T> p) {
  const int e = blockIdx.x * 256 + threadIdx.x;
  if (e >= p.nc) return;
  T out[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) out[k] = T(0);
  const int e0 = p.inc0[e], e1 = p.inc0[e + 1];
  for (int ci = e0 - 1; ci < e1; ++ci) {
    const int n = ci < e0 ? e : p.nbr[ci];
    bool seen = ci >= e0 && n == e;
    for (int cj = e0; cj < ci && !seen; ++cj) seen = p.nbr[cj] == n;
    if (seen) continue;
    const int n0 = p.inc0[n], n1 = p.inc0[n + 1];
    bool reads_e = n == e;
    for (int i = n0; i < n1; ++i) reads_e |= p.nbr[i] == e;
    if (!reads_e) continue;
    T pn[12], lw[12];
    load12(p.P, p.nc, n, pn);
    load12(p.lamW, p.nc, n, lw);
#pragma unroll 1
    for (int k = 0; k < 12; ++k) {
      // the mean slot of coefficient k (-1: a gradient, read by the own limiter only)
      const int ks = k % 3 == 0 ? k / 3 : -1;
      if (n != e && ks < 0) continue;
      Dual<T> q[12], hi[4], lo[4], al[4];
#pragma unroll
      for (int j = 0; j < 12; ++j) q[j] = Dual<T>(pn[j], T(n == e && j == k ? 1 : 0));
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        hi[v] = lo[v] = q[3 * v];
        al[v] = Dual<T>(1.0);
      }
      for (int i = n0; i < n1; ++i) {
        const int m = p.nbr[i];
#pragma unroll
        for (int v = 0; v < 4; ++v) {
          const Dual<T> mv(p.P[(size_t)(3 * v) * p.nc + m], T(m == e && v == ks ? 1 : 0));
          hi[v] = fmax(hi[v], mv);
          lo[v] = fmin(lo[v], mv);
        }
      }
      for (int i = n0; i < n1; ++i) {
        const Dual<T> rx(p.lim_geo[2 * (size_t)i], T(0)), ry(p.lim_geo[2 * (size_t)i + 1], T(0));
#pragma unroll
        for (int v = 0; v < 4; ++v)
          al[v] = fmin(al[v], psi_of(q[3 * v + 1] * rx + q[3 * v + 2] * ry, q[3 * v], hi[v], lo[v]));
      }
      T acc = T(0);
#pragma unroll
      for (int v = 0; v < 4; ++v) {
        acc = fma(lw[3 * v], q[3 * v].d, acc);
        acc = fma(lw[3 * v + 1], (al[v] * q[3 * v + 1]).d, acc);
        acc = fma(lw[3 * v + 2], (al[v] * q[3 * v + 2]).d, acc);
      }
      out[k] += acc;
    }
  }
#pragma unroll
  for (int k = 0; k < 12; ++k) p.out[(size_t)k * p.nc + e] = out[k];
}

template <typename T>
hipError_t adjoint_t(const dg_mesh* m, const void* U, const void* V1, const double* dt_dev,
                     double dt, const void* lam_np1, void* lam_n, void* ws1, void* ws2,
                     hipStream_t s) {
  const FLDev& f = *m->fld;
  const bool lim = m->cfg.limiter == DG_LIMITER_MINMOD;
  const dim3 grid((unsigned)((f.ncells + 255) / 256)), block(256);
  PFA<T> p{};
  p.dt_dev = dt_dev;
  p.dt_host = dt;
  p.nc = f.ncells;
  p.gamma = (T)m->cfg.gamma;
  p.inc0 = f.lim_inc0;
  p.nbr = f.lim_nbr;
  p.inc_face = f.inc_face;
  p.face_lr = f.face_lr;
  p.face_geo = static_cast<const T*>(f.face_geo);
  p.lim_geo = static_cast<const T*>(f.lim_geo);
  p.cell_geo = static_cast<const T*>(f.cell_geo);
  auto adj_stage = [&](const void* P, const void* lam, const void* extra, double c_id,
                       double c_L_over_dt, double c_extra, void* out) -> hipError_t {
    // W = Pi(P) into ws1; lamW into ws2 (or straight into out without a
    // limiter); out = Pi_P^T lamW
    const void* W = P;
    if (lim) {
      hipError_t r = lim_t<T>(m, P, ws1, s);
      if (r != hipSuccess) return r;
      W = ws1;
    }
    PFA<T> a = p;
    a.W = static_cast<const T*>(W);
    a.lam = static_cast<const T*>(lam);
    a.extra = static_cast<const T*>(extra);
    a.c_id = c_id;
    a.c_L_over_dt = c_L_over_dt;
    a.c_extra = c_extra;
    a.out = static_cast<T*>(lim ? ws2 : out);
    hipLaunchKernelGGL((k_adjfl_L<T>), grid, block, 0, s, a);
    if (!lim) return hipGetLastError();
    PFA<T> b = p;
    b.P = static_cast<const T*>(P);
    b.lamW = static_cast<const T*>(ws2);
    b.out = static_cast<T*>(out);
    hipLaunchKernelGGL((k_adjfl_lim<T>), grid, block, 0, s, b);
    return hipGetLastError();
  };
  // stage 2: lam_V1 = Pi_V1^T [lam'/2 + (dt/2) L^T lam'] (in lam_n with the
  // limiter, else in ws2); stage 1: lam_n = Pi_U^T [lam_V1 + dt L^T lam_V1 + lam'/2]
  void* lam_v1 = lim ? lam_n : ws2;
  hipError_t e = adj_stage(V1, lam_np1, nullptr, 0.5, 0.5, 0.0, lam_v1);
  if (e != hipSuccess) return e;
  return adj_stage(U, lam_v1, lam_np1, 1.0, 1.0, 0.5, lam_n);
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
    if (!(perim[e] > 0)) {
      set_error("dg_mesh_create: cell " + std::to_string(e) + " has no faces");
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
  // the adjoint's incidence codes and global face records
  std::vector<int> inc_face(inc0[nc]), face_lr(2 * nf);
  std::vector<double> fgeo(8 * nf, 0.0);
  for (int64_t i = 0; i < (int64_t)inc0[nc]; ++i) inc_face[i] = (cface[i] << 1) | cside[i];
  for (int64_t f = 0; f < nf; ++f) {
    double rc[2], dLR[2];
    offsets(f, rc, dLR);
    face_lr[2 * f] = d->face_cells[2 * f];
    face_lr[2 * f + 1] = d->face_cells[2 * f + 1];
    fgeo[8 * f] = d->face_normal[2 * f];
    fgeo[8 * f + 1] = d->face_normal[2 * f + 1];
    fgeo[8 * f + 2] = d->face_area[f];
    fgeo[8 * f + 3] = rc[0];
    fgeo[8 * f + 4] = rc[1];
    fgeo[8 * f + 5] = dLR[0];
    fgeo[8 * f + 6] = dLR[1];
  }
  // blocks of up to kBlock consecutive cells; a block is halved until its
  // distinct incident faces fit the slot table and its outside neighbours the
  // halo table
  std::vector<int> blk_cell0{0};
  {
    std::vector<int64_t> fmark(nf, -1), cmark(nc, -1);
    int64_t stamp = 0, e = 0;
    while (e < nc) {
      int64_t e1 = std::min<int64_t>(e + kBlock, nc);
      for (;;) {
        ++stamp;
        int ns = 0, nh = 0;
        for (int64_t c = e; c < e1; ++c)
          for (int i = inc0[c]; i < inc0[c + 1]; ++i) {
            const int f = cface[i];
            if (fmark[f] != stamp) {
              fmark[f] = stamp;
              ++ns;
            }
            const int o = cside[i] ? d->face_cells[2 * f] : d->face_cells[2 * f + 1];
            if ((o < e || o >= e1) && cmark[o] != stamp) {
              cmark[o] = stamp;
              ++nh;
            }
          }
        if ((ns <= kMaxSlots && nh <= kMaxHalo) || e1 - e <= 1) break;
        e1 = e + (e1 - e) / 2;
      }
      blk_cell0.push_back((int)e1);
      e = e1;
    }
  }
  const int nblocks = (int)blk_cell0.size() - 1;
  std::vector<int> blk_slot0{0}, blk_halo0{0}, halo_cell, slot_lr, cell_inc0(nc + 1, 0), cell_inc;
  std::vector<double> sgeo, irf;
  std::vector<int> slot_of_face(nf, -1), local_of(nc, -1);
  int max_slots = 0;
  for (int b = 0; b < nblocks; ++b) {
    const int ca = blk_cell0[b], cb = blk_cell0[b + 1], nown = cb - ca;
    // block-local indices: own cells first, then the halo in first-seen order
    std::vector<int> halo;
    for (int c = ca; c < cb; ++c) local_of[c] = c - ca;
    for (int c = ca; c < cb; ++c)
      for (int i = inc0[c]; i < inc0[c + 1]; ++i) {
        const int f = cface[i];
        const int o = cside[i] ? d->face_cells[2 * f] : d->face_cells[2 * f + 1];
        if (local_of[o] < 0) {
          local_of[o] = nown + (int)halo.size();
          halo.push_back(o);
        }
      }
    if ((int)halo.size() > kMaxHalo) {
      set_error("dg_mesh_create: a cell block has too many outside neighbours");
      return DG_EINVAL;
    }
    // slots in first-seen order; each cell's incidences sorted by slot
    std::vector<int> touched;
    int ns = 0;
    for (int c = ca; c < cb; ++c) {
      std::vector<std::pair<int, int>> mine;  // (slot, incidence index in the global CSR)
      for (int i = inc0[c]; i < inc0[c + 1]; ++i) {
        const int f = cface[i];
        if (slot_of_face[f] < 0) {
          slot_of_face[f] = ns++;
          touched.push_back(f);
          const int L = d->face_cells[2 * f], R = d->face_cells[2 * f + 1];
          slot_lr.push_back(local_of[L] | (local_of[R] << 16));
          double rc[2], dLR[2];
          offsets(f, rc, dLR);
          const double g[8] = {d->face_normal[2 * f], d->face_normal[2 * f + 1], d->face_area[f],
                               rc[0], rc[1], dLR[0], dLR[1], 0.0};
          sgeo.insert(sgeo.end(), g, g + 8);
        }
        mine.emplace_back(slot_of_face[f], i);
      }
      std::sort(mine.begin(), mine.end());
      for (const auto& si : mine) {
        const int i = si.second, f = cface[i];
        const int o = cside[i] ? d->face_cells[2 * f] : d->face_cells[2 * f + 1];
        cell_inc.push_back((si.first * 2 + cside[i]) | (local_of[o] << 16));
        double rc[2], dLR[2];
        offsets(f, rc, dLR);
        // face centroid from this side's centroid (R: its image next to L)
        irf.push_back(cside[i] ? rc[0] - dLR[0] : rc[0]);
        irf.push_back(cside[i] ? rc[1] - dLR[1] : rc[1]);
      }
      cell_inc0[c + 1] = (int)cell_inc.size();
    }
    for (int f : touched) slot_of_face[f] = -1;
    for (int c = ca; c < cb; ++c) local_of[c] = -1;
    for (int o : halo) local_of[o] = -1;
    if (ns > kMaxSlots) {
      set_error("dg_mesh_create: a cell block has too many incident faces");
      return DG_EINVAL;
    }
    max_slots = std::max(max_slots, ns);
    blk_slot0.push_back(blk_slot0.back() + ns);
    halo_cell.insert(halo_cell.end(), halo.begin(), halo.end());
    blk_halo0.push_back((int)halo_cell.size());
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
  if (err == hipSuccess) err = upload_i(blk_halo0, &fd->blk_halo0);
  if (err == hipSuccess) err = upload_i(halo_cell, &fd->halo_cell);
  if (err == hipSuccess) err = upload_i(slot_lr, &fd->slot_lr);
  if (err == hipSuccess) err = upload_i(cell_inc0, &fd->cell_inc0);
  if (err == hipSuccess) err = upload_i(cell_inc, &fd->cell_inc);
  if (err == hipSuccess) err = upload_i(inc0, &fd->lim_inc0);
  if (err == hipSuccess) err = upload_i(nbr, &fd->lim_nbr);
  auto up = [&](const std::vector<double>& h, void** dst) {
    return f64 ? upload<double>(h, dst) : upload<float>(h, dst);
  };
  if (err == hipSuccess) err = up(sgeo, &fd->slot_geo);
  if (err == hipSuccess) err = up(irf, &fd->inc_rf);
  if (err == hipSuccess) err = up(cgeo, &fd->cell_geo);
  if (err == hipSuccess) err = up(lgeo, &fd->lim_geo);
  if (err == hipSuccess) err = up(perim, &fd->cell_perim);
  if (err == hipSuccess) err = upload_i(inc_face, &fd->inc_face);
  if (err == hipSuccess) err = upload_i(face_lr, &fd->face_lr);
  if (err == hipSuccess) err = up(fgeo, &fd->face_geo);
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
  (void)hipFree(f->blk_halo0);
  (void)hipFree(f->halo_cell);
  (void)hipFree(f->slot_lr);
  (void)hipFree(f->slot_geo);
  (void)hipFree(f->cell_inc0);
  (void)hipFree(f->cell_inc);
  (void)hipFree(f->inc_rf);
  (void)hipFree(f->cell_geo);
  (void)hipFree(f->lim_inc0);
  (void)hipFree(f->lim_nbr);
  (void)hipFree(f->lim_geo);
  (void)hipFree(f->cell_perim);
  (void)hipFree(f->inc_face);
  (void)hipFree(f->face_lr);
  (void)hipFree(f->face_geo);
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
  auto step = [&](int md, const void* ua, void* lim_out, bool want_dt) {
    return f64 ? step_t<double>(m, md, in, ua, out, lim_out, dt_dev, dt_host, want_dt, s)
               : step_t<float>(m, md, in, ua, out, lim_out, dt_dev, dt_host, want_dt, s);
  };
  hipError_t e = hipSuccess;
  switch (mode) {
    case kLimit:
      return limit(in, out);
    case kRhs:
      return step(kRhs, nullptr, nullptr, false);
    case kStage1:
      // keeps Pi(U) of every cell in ws_a for the stage 2 of the same U
      return step(kStage1, nullptr, lim ? m->ws_a : nullptr, false);
    case kStage2: {
      const void* ua = u0;
      if (lim) {
        if (!(m->ws_a_fresh && m->ws_a_src == u0)) e = limit(u0, m->ws_a);
        ua = m->ws_a;
      }
      if (e == hipSuccess) e = step(kStage2, ua, nullptr, dt_next != nullptr);
      if (e == hipSuccess && dt_next)
        e = launch_min_finalize(m->dtpart, m->fld->nblocks, cfl, dt_next, s);
      return e;
    }
    default:
      return hipErrorInvalidValue;
  }
}

hipError_t launch_adjoint_facelist(const dg_mesh* m, const void* U, const void* V1,
                                   const double* dt_dev, double dt, const void* lam_np1,
                                   void* lam_n, void* ws1, void* ws2, hipStream_t s) {
  if (m->cfg.precision == DG_FP64)
    return adjoint_t<double>(m, U, V1, dt_dev, dt, lam_np1, lam_n, ws1, ws2, s);
  return adjoint_t<float>(m, U, V1, dt_dev, dt, lam_np1, lam_n, ws1, ws2, s);
}

hipError_t launch_facelist_cfl(const dg_mesh* m, const void* U, double cfl, double* dt_dev,
                               hipStream_t s) {
  hipError_t e = m->cfg.precision == DG_FP64 ? cfl_t<double>(m, U, s) : cfl_t<float>(m, U, s);
  if (e != hipSuccess) return e;
  return launch_min_finalize(m->dtpart, (m->fld->ncells + 63) / 64, cfl, dt_dev, s);
}

}  // namespace dg
