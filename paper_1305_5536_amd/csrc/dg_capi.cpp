// Host side of the C ABI declared in include/dg.h: validation, device
// allocation, kernel dispatch and error reporting.  No arithmetic of the DG
// update happens here; every step runs in the HIP kernels.
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdlib>
#include <cstdio>
#include <cstring>
#include <new>
#include <vector>
#include <string>

#include "dg.h"
#include "dg_internal.h"

namespace dg {

static thread_local std::string g_err;

void set_error(const std::string& msg) { g_err = msg; }

dg_status hip_fail(hipError_t e, const char* what) {
  set_error(std::string(what) + ": " + hipGetErrorName(e) + " (" + hipGetErrorString(e) + ")");
  return DG_EHIP;
}

static dg_status einval(const std::string& msg) {
  set_error(msg);
  return DG_EINVAL;
}

hipError_t launch_min_finalize(const double* part, int n, double cfl, double* dt, hipStream_t s);
hipError_t launch_moving(dg_mesh* m, int mode, const void* in, void* out, const double* dt_dev,
                         double dt_host, double cfl, double* dt_next, hipStream_t s);
hipError_t launch_moving_cfl(const dg_mesh* m, const void* U, double cfl, double* dt_dev,
                             hipStream_t s);
dg_status moving_create(dg_mesh* m, const dg_mesh_desc* d);
void moving_destroy(dg_mesh* m);
hipError_t moving_init(dg_mesh* m);
int moving_read(const dg_mesh* m, double* gen, double* vol, double* cen, int32_t* ring,
                int32_t* deg);
void moving_set_motion(dg_mesh* m, int motion);
void moving_set_timing(dg_mesh* m, int on);
int moving_timing(dg_mesh* m, double* avg_ms, int* nsteps);
dg_status facelist_create(dg_mesh* m, const dg_mesh_desc* d);
void facelist_destroy(dg_mesh* m);
hipError_t launch_facelist(const dg_mesh* m, int mode, const void* in, const void* u0, void* out,
                           const double* dt_dev, double dt_host, double cfl, double* dt_next,
                           hipStream_t s);
hipError_t launch_facelist_cfl(const dg_mesh* m, const void* U, double cfl, double* dt_dev,
                               hipStream_t s);
hipError_t launch_adjoint_mhd3d(const dg_mesh* m, const void* U, const void* V1,
                                const double* dt_dev, double dt, const void* lam_np1,
                                void* lam_n, void* ws1, void* ws2, hipStream_t s);
hipError_t launch_adjoint_facelist(const dg_mesh* m, const void* U, const void* V1,
                                   const double* dt_dev, double dt, const void* lam_np1,
                                   void* lam_n, void* ws1, void* ws2, hipStream_t s);
hipError_t launch_cart3d(const dg_mesh* m, int mode, const void* in, const void* u0, void* out,
                         const double* dt_dev, double dt_host, double cfl, double* dt_next,
                         hipStream_t s);
hipError_t launch_mhd2d(const dg_mesh* m, int mode, const void* in, const void* u0, void* out,
                        const double* dt_dev, double dt_host, double cfl, double* dt_next,
                        hipStream_t s);
hipError_t launch_adjoint_mhd2d(const dg_mesh* m, const void* U, const void* V1,
                                const double* dt_dev, double dt, const void* lam_np1,
                                void* lam_n, void* ws1, void* ws2, hipStream_t s);
hipError_t launch_mhd2d_cfl(const dg_mesh* m, const void* U, double cfl, double* dt_dev,
                            hipStream_t s);
hipError_t launch_cart3d_cfl(const dg_mesh* m, const void* U, double cfl, double* dt_dev,
                             hipStream_t s);
int64_t max_stage_waves3(const dg_mesh* m);
int64_t stage_groups3(int tiles_x, int ny);

// Rows (2D) or planes (3D) marched by one wave.  Chosen so a launch has
// several waves per SIMD on 256 CUs.  The DG_TILE_ROWS environment variable
// overrides this and every model-based default below for the whole process
// (launch-shape experiments; dg_set_tiling, which the autotuner uses, takes
// precedence over both).
static int default_rows(int64_t ntiles_x, int64_t nrows) {
  const char* env = std::getenv("DG_TILE_ROWS");
  if (env) {
    int r = std::atoi(env);
    if (r > 0) return r;
  }
  // target >= 4096 waves when the mesh allows, rows in [4, 64]
  int64_t want_tiles = 4096;
  int64_t rows = (ntiles_x * nrows + want_tiles - 1) / want_tiles;
  if (rows < 4) rows = 4;
  if (rows > 64) rows = 64;
  if (rows > nrows) rows = nrows;
  return (int)rows;
}

// Rows per tile of every instance of a batch: 16 (DG_TILE_ROWS overrides).
static int default_batch_rows() {
  const char* env = std::getenv("DG_TILE_ROWS");
  return env && std::atoi(env) > 0 ? std::atoi(env) : 16;
}

// Planes per workgroup of the 3D stage kernel (DG_TILE_ROWS overrides): one
// workgroup per CU in FP64 and two in FP32 (set by the LDS), so P in [4, 64]
// minimises rounds x (P + 1), a workgroup of P planes costing about P + 1
// plane times (its prologue solves one extra z-face) (256^3: FP64 64 planes,
// five rounds of 256; FP32 32 planes, five rounds of 512, 8.81 against 9.19 ms
// per step at 64).
static int default_planes3d(int tiles_x, int ny, int64_t nz, bool f64) {
  const char* env = std::getenv("DG_TILE_ROWS");
  if (env && std::atoi(env) > 0) return (int)std::min<int64_t>(std::atoi(env), nz);
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0) {
    (void)hipGetLastError();
    cus = 256;
  }
  const int64_t slots = (int64_t)cus * (f64 ? 1 : 2);
  const int64_t groups = stage_groups3(tiles_x, ny);
  double best = 1e300;
  int64_t planes = 4;
  for (int64_t r = 4; r <= 64; ++r) {
    const int64_t pp = std::min(r, nz);
    const int64_t wgs = groups * ((nz + pp - 1) / pp);
    const double cost = (double)((wgs + slots - 1) / slots) * ((double)pp + 1.0);
    if (cost < best - 1e-9) {
      best = cost;
      planes = pp;
    }
  }
  return (int)std::min<int64_t>(planes, nz);
}

// Rows per wave of the 2D Euler stage kernels and the MUSCL-Hancock step.
// FP64: stage 1 runs two waves per SIMD, stage 2 and the MUSCL-Hancock kernel
// one (registers); a wave of R rows costs about R + 2 row times, so R in
// [4, 128] minimises (rounds at two waves per SIMD + rounds at one) x (R + 2)
// (2048^2: 36 rows, 1995 waves, one round of stage 1 and two of stage 2).
// FP32 runs several waves per SIMD, which hide each other's latency: the
// generic rule (about 4096 waves).  DG_TILE_ROWS overrides both.
static int default_rows_euler2d(int64_t ntiles_x, int64_t nrows, bool f64) {
  if (!f64 || std::getenv("DG_TILE_ROWS")) return default_rows(ntiles_x, nrows);
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0) {
    (void)hipGetLastError();
    cus = 256;
  }
  const int64_t one = (int64_t)cus * 4;
  double best = 1e300;
  int64_t rows = 4;
  for (int64_t r = 4; r <= 128; ++r) {
    const int64_t rr = std::min(r, nrows);
    const int64_t waves = ntiles_x * ((nrows + rr - 1) / rr);
    const int64_t rounds = (waves + 2 * one - 1) / (2 * one) + (waves + one - 1) / one;
    const double cost = (double)rounds * ((double)rr + 2.0);
    if (cost < best - 1e-9) {
      best = cost;
      rows = rr;
    }
  }
  return (int)std::min<int64_t>(rows, nrows);
}

// Rows per wave of the fused 2D Euler step (DG_STEP_ROWS overrides).  A wave
// of R rows costs about R + 1.85 stage-2 row times (its four extra stage-1
// rows are a little cheaper than stage-2 rows), and the waves run in rounds of
// one per SIMD (FP64: one wave per SIMD by registers; FP32: two), so R in
// [8, 128] minimises rounds x (R + 1.85): the last round should be nearly full
// (2048^2: FP64 76 rows, one round of 999 waves; FP32 38 rows).
static int default_step_rows(int64_t ntiles_x, int64_t nrows, bool f64) {
  const char* env = std::getenv("DG_STEP_ROWS");
  int64_t rows = env ? std::atoi(env) : 0;
  if (rows <= 0) {
    int dev = 0, cus = 256;
    if (hipGetDevice(&dev) != hipSuccess ||
        hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
        cus <= 0) {
      (void)hipGetLastError();
      cus = 256;
    }
    const int64_t slots = (int64_t)cus * 4 * (f64 ? 1 : 2);
    double best = 1e300;
    for (int64_t r = 8; r <= 128; ++r) {
      const int64_t rr = std::min(r, nrows);
      const int64_t waves = ntiles_x * ((nrows + rr - 1) / rr);
      const double cost = (double)((waves + slots - 1) / slots) * ((double)rr + 1.85);
      if (cost < best - 1e-9) {
        best = cost;
        rows = rr;
      }
    }
  }
  return (int)std::min<int64_t>(rows, nrows);
}

// Rows per wave of the 2D MHD stage kernel.  FP64 runs one wave per SIMD (by
// registers): a wave of R rows costs about R + 3 row times (the prologue loads
// and limits two rows and solves one extra y-face row) and the waves run in
// rounds of one per SIMD, so R in [2, 32] minimises rounds x (R + 3) (512^2:
// 5 rows, one round of 927 waves, 0.117 ms per step against 0.152 at 2 rows
// in three rounds; 2048^2: 24 rows, 1.39 against 1.43 ms).  FP32 runs three
// waves per SIMD, which hide each other's latency: about 8192 waves over the
// mesh, 2 to 16 rows, measured best (2048^2: 9 rows, 0.760 ms against 0.773
// with the FP64 model's 24).
static int default_rows_mhd2d(int64_t ntiles_x, int64_t nrows, bool f64) {
  if (std::getenv("DG_TILE_ROWS")) return default_rows(ntiles_x, nrows);
  if (!f64) {
    int64_t rows = (ntiles_x * nrows + 8191) / 8192;
    rows = std::max<int64_t>(2, std::min<int64_t>(16, rows));
    return (int)std::min<int64_t>(rows, nrows);
  }
  int dev = 0, cus = 256;
  if (hipGetDevice(&dev) != hipSuccess ||
      hipDeviceGetAttribute(&cus, hipDeviceAttributeMultiprocessorCount, dev) != hipSuccess ||
      cus <= 0) {
    (void)hipGetLastError();
    cus = 256;
  }
  const int64_t slots = (int64_t)cus * 4;
  double best = 1e300;
  int64_t rows = 2;
  for (int64_t r = 2; r <= 32; ++r) {
    const int64_t rr = std::min(r, nrows);
    const int64_t waves = ntiles_x * ((nrows + rr - 1) / rr);
    const double cost = (double)((waves + slots - 1) / slots) * ((double)rr + 3.0);
    if (cost < best - 1e-9) {
      best = cost;
      rows = rr;
    }
  }
  return (int)std::min<int64_t>(rows, nrows);
}

// Meshes that keep Pi(U) of stage 1 in ws_a for stage 2 (3D MHD limits in
// passes of its own into ws_a / ws_b; 2D MHD and face lists limit on read and
// their stage 1 writes Pi(U) to ws_a); the 2D Euler Cartesian kernels limit
// inside the stage kernel and recompute Pi(U^n) in stage 2.
static bool limiter_pass(const dg_mesh* m) {
  return m->dim == 3 || m->kind == 1 || m->cfg.physics == DG_MHD;
}

static dg_status dispatch(const dg_mesh* m, int mode, const void* in, const void* u0, void* out,
                          const double* dt_dev, double dt_host, hipStream_t s,
                          double cfl = 0.0, double* dt_next = nullptr) {
  hipError_t e;
  if (m->kind == 3) {
    if (mode != kLimit && mode != kMH) {
      set_error("moving Voronoi meshes step with dg_step_mh only (the moving-mesh "
                "MUSCL-Hancock step); dg_limit is built too");
      return DG_EUNSUPPORTED;
    }
    e = launch_moving(const_cast<dg_mesh*>(m), mode, in, out, dt_dev, dt_host, cfl, dt_next, s);
    if (e != hipSuccess) return hip_fail(e, "kernel launch");
    return DG_OK;
  }
  if (m->kind == 1)
    e = launch_facelist(m, mode, in, u0, out, dt_dev, dt_host, cfl, dt_next, s);
  else if (m->kind == 2)
    e = launch_cart2d_batch(m, mode, in, u0, out, dt_dev, dt_host, cfl, dt_next, s);
  else if (m->dim == 2 && m->cfg.physics == DG_MHD)
    e = launch_mhd2d(m, mode, in, u0, out, dt_dev, dt_host, cfl, dt_next, s);
  else if (m->dim == 2)
    e = launch_cart2d(m, mode, in, u0, out, dt_dev, dt_host, cfl, dt_next, s);
  else
    e = launch_cart3d(m, mode, in, u0, out, dt_dev, dt_host, cfl, dt_next, s);
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return DG_OK;
}

// Forward tile tables of a batch at its current rows per tile.
static dg_status batch_upload(dg_mesh* m) {
  Batch& b = m->bt;
  const bool f64 = m->cfg.precision == DG_FP64;
  std::vector<char> rec(batch_record_size(f64) * b.ninst);
  std::vector<int> ti, t0;
  b.ntiles = batch_tables(b.d, f64, b.rows, rec.data(), ti, t0);
  hipError_t e = hipMemcpy(b.inst, rec.data(), rec.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(b.tile_inst, ti.data(), sizeof(int) * ti.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess)
    e = hipMemcpy(b.inst_tile0, t0.data(), sizeof(int) * t0.size(), hipMemcpyHostToDevice);
  if (e != hipSuccess) return hip_fail(e, "batch tables");
  return DG_OK;
}

// Adjoint tables (58-column strips of kAdjRows rows) of one or more 2D Cartesian instances.
static dg_status adjoint_tables(dg_mesh* m, const BatchDesc& d, bool batched) {
  std::vector<AdjInst> ai(d.ninst);
  std::vector<int> ti;
  int tile0 = 0;
  // rows per wave: about kAdjWaves waves over the whole set, within
  // [kAdjRowsMin, kAdjRowsMax] (each wave marches 4 rows beyond its own)
  int64_t strips = 0;
  for (int i = 0; i < d.ninst; ++i)
    strips += (int64_t)((d.nx[i] + kAdjCols - 1) / kAdjCols) * d.ny[i];
  const int rows = (int)std::min<int64_t>(
      kAdjRowsMax, std::max<int64_t>(kAdjRowsMin, (strips + kAdjWaves - 1) / kAdjWaves));
  for (int i = 0; i < d.ninst; ++i) {
    AdjInst a{};
    a.nx = d.nx[i];
    a.ny = d.ny[i];
    a.off = (int)d.off[i];
    a.tx0 = tile0;
    a.rows = std::min(rows, a.ny);
    a.tiles_x = (a.nx + kAdjCols - 1) / kAdjCols;
    a.tiles_y = (a.ny + a.rows - 1) / a.rows;
    a.hx = d.hx[i];
    a.hy = d.hy[i];
    ai[i] = a;
    for (int t = 0; t < a.tiles_x * a.tiles_y; ++t) ti.push_back(i);
    tile0 += a.tiles_x * a.tiles_y;
  }
  m->adj_tiles = tile0;
  hipError_t e = hipMalloc(&m->adj_inst, sizeof(AdjInst) * ai.size());
  if (e == hipSuccess)
    e = hipMemcpy(m->adj_inst, ai.data(), sizeof(AdjInst) * ai.size(), hipMemcpyHostToDevice);
  if (e == hipSuccess && batched) {
    e = hipMalloc(&m->bt.adj_tile_inst, sizeof(int) * ti.size());
    if (e == hipSuccess)
      e = hipMemcpy(m->bt.adj_tile_inst, ti.data(), sizeof(int) * ti.size(),
                    hipMemcpyHostToDevice);
  }
  if (e != hipSuccess) return hip_fail(e, "dg_mesh_create: adjoint tables");
  return DG_OK;
}

static void free_graph(RunGraph& g) {
  if (g.exec) (void)hipGraphExecDestroy(g.exec);
  if (g.graph) (void)hipGraphDestroy(g.graph);
  g.exec = nullptr;
  g.graph = nullptr;
}

static void drop_graph(dg_mesh* m) {
  for (RunGraph& g : m->runs) free_graph(g);
  m->runs.clear();
}

}  // namespace dg

using namespace dg;

extern "C" {

const char* dg_last_error(void) { return g_err.c_str(); }

dg_status dg_mesh_create(const dg_mesh_desc* d, const dg_config* cfg, dg_mesh_t* out) {
  if (!out) return einval("dg_mesh_create: out is NULL");
  *out = nullptr;
  if (!d || !cfg) return einval("dg_mesh_create: NULL descriptor or config");
  if (cfg->precision != DG_FP64 && cfg->precision != DG_FP32)
    return einval("dg_mesh_create: unknown precision");
  if (cfg->limiter != DG_LIMITER_NONE && cfg->limiter != DG_LIMITER_MINMOD &&
      cfg->limiter != DG_LIMITER_WENO)
    return einval("dg_mesh_create: unknown limiter");
  if (cfg->limiter == DG_LIMITER_WENO &&
      (cfg->physics != DG_EULER || (d->kind != 0 && d->kind != 3) || d->dim != 2)) {
    set_error("dg_mesh_create: the WENO-type limiter is built for 2D Euler on Cartesian and "
              "moving Voronoi meshes");
    return DG_EUNSUPPORTED;
  }
  if (!(cfg->gamma > 1.0) || !std::isfinite(cfg->gamma))
    return einval("dg_mesh_create: gamma must be finite and > 1");
  if (cfg->physics == DG_EULER) {
    if (cfg->flux != DG_FLUX_HLL && cfg->flux != DG_FLUX_EXACT) {
      set_error("dg_mesh_create: Euler takes the HLL or the exact Riemann flux");
      return DG_EUNSUPPORTED;
    }
    if (cfg->flux == DG_FLUX_EXACT && ((d->kind != 0 && d->kind != 3) || d->dim != 2)) {
      set_error("dg_mesh_create: the exact Riemann flux is built for 2D Cartesian and moving "
                "Voronoi meshes");
      return DG_EUNSUPPORTED;
    }
  } else if (cfg->physics == DG_MHD) {
    if (cfg->flux != DG_FLUX_HLLD) {
      set_error("dg_mesh_create: MHD supports the HLLD flux only");
      return DG_EUNSUPPORTED;
    }
    if (d->kind != 0) {
      set_error("dg_mesh_create: MHD is built for 2D and 3D Cartesian meshes only");
      return DG_EUNSUPPORTED;
    }
  } else {
    return einval("dg_mesh_create: unknown physics");
  }
  if (d->kind != 0 && d->kind != 1 && d->kind != 2 && d->kind != 3)
    return einval("dg_mesh_create: unknown mesh kind");
  if (d->kind == 3 && (cfg->physics != DG_EULER || d->dim != 2)) {
    set_error("dg_mesh_create: moving Voronoi meshes are built for 2D Euler");
    return DG_EUNSUPPORTED;
  }
  if (d->kind == 2) {
    if (cfg->physics != DG_EULER) {
      set_error("dg_mesh_create: batches are built for 2D Euler only");
      return DG_EUNSUPPORTED;
    }
    if (d->dim != 2) return einval("dg_mesh_create: batch instances are 2D (dim = 2)");
    if (d->ninst < 1 || d->ninst > (1 << 20) || !d->inst_n || !d->inst_box)
      return einval("dg_mesh_create: batch needs ninst >= 1, inst_n and inst_box");
    for (int i = 0; i < d->ninst; ++i) {
      if (d->inst_n[2 * i] < 1 || d->inst_n[2 * i + 1] < 1 || d->inst_n[2 * i] > (1 << 16) ||
          d->inst_n[2 * i + 1] > (1 << 16))
        return einval("dg_mesh_create: bad instance cell count");
      const double* bx = d->inst_box + 4 * i;
      if (!(bx[2] > bx[0]) || !(bx[3] > bx[1]))
        return einval("dg_mesh_create: instance box needs hi > lo");
    }
  }
  if (d->kind == 1 && d->dim != 2) {
    set_error("dg_mesh_create: face-list meshes are 2D only");
    return DG_EUNSUPPORTED;
  }
  // face lists address 12 state arrays of ncells and, per face, at most two
  // block slots of 10 geometry values (and two incidences of 5) in 32 bits
  if (d->kind == 1 && (d->ncells * 12 >= ((int64_t)1 << 31) || d->nfaces * 20 >= ((int64_t)1 << 31)))
    return einval("dg_mesh_create: face list too large for 32-bit indexing "
                  "(needs 12 ncells < 2^31 and 20 nfaces < 2^31)");
  if (d->kind == 0) {
    if (d->dim != 2 && d->dim != 3) return einval("dg_mesh_create: dim must be 2 or 3");
    if (d->dim == 3 && cfg->physics != DG_MHD) {
      set_error("dg_mesh_create: 3D Cartesian meshes are built for MHD only");
      return DG_EUNSUPPORTED;
    }
    int64_t cells = 1;
    for (int k = 0; k < d->dim; ++k) {
      if (d->n[k] < 1 || d->n[k] > (1 << 20)) return einval("dg_mesh_create: bad cell count");
      if (!(d->hi[k] > d->lo[k])) return einval("dg_mesh_create: hi must exceed lo");
      cells *= d->n[k];
    }
    // the kernels address coefficient k of cell e as k * ncells + e in 32 bits
    const int64_t ncoef = d->dim == 3 ? 31 : (cfg->physics == DG_MHD ? 23 : 12);
    if (cells * ncoef >= ((int64_t)1 << 31))
      return einval("dg_mesh_create: mesh too large for 32-bit indexing (ncells * ncoef >= 2^31)");
  }

  dg_mesh* m = new (std::nothrow) dg_mesh();
  if (!m) {
    set_error("dg_mesh_create: out of host memory");
    return DG_ENOMEM;
  }
  m->cfg = *cfg;
  m->dim = d->dim;
  m->kind = d->kind;
  m->elem = cfg->precision == DG_FP64 ? 8 : 4;
  (void)hipGetDevice(&m->device);
  int64_t nwaves = 0;
  if (d->kind == 0 && d->dim == 2) {
    const bool mhd = cfg->physics == DG_MHD;
    m->ncoef = mhd ? 23 : 12;
    m->ncells = d->n[0] * d->n[1];
    m->c2.nx = (int)d->n[0];
    m->c2.ny = (int)d->n[1];
    m->c2.hx = (d->hi[0] - d->lo[0]) / d->n[0];
    m->c2.hy = (d->hi[1] - d->lo[1]) / d->n[1];
    for (int k = 0; k < 2; ++k) {
      m->c2.lo[k] = d->lo[k];
      m->c2.hi[k] = d->hi[k];
    }
    m->c2.tiles_x = (int)((d->n[0] + 59) / 60);  // 60 interior columns per wave
    m->c2.rows_per_tile =
        mhd ? default_rows_mhd2d(m->c2.tiles_x, d->n[1], cfg->precision == DG_FP64)
            : default_rows_euler2d(m->c2.tiles_x, d->n[1], cfg->precision == DG_FP64);
    m->c2.tiles_y = (int)((d->n[1] + m->c2.rows_per_tile - 1) / m->c2.rows_per_tile);
    nwaves = (int64_t)m->c2.tiles_x * m->c2.tiles_y;
    m->c2.step_tiles_x = (int)((d->n[0] + 55) / 56);  // 56 output columns per wave
    m->c2.step_rows =
        default_step_rows(m->c2.step_tiles_x, d->n[1], cfg->precision == DG_FP64);
    m->c2.step_tiles_y = (int)((d->n[1] + m->c2.step_rows - 1) / m->c2.step_rows);
    if (cfg->physics == DG_EULER) {
      // the static scratch of dg_cfl_dt_static on this device (the device
      // that is current here is the mesh's); without its address only that
      // entry point is unavailable (it then returns DG_EHIP)
      if (cart2d_scratch_init() != hipSuccess) (void)hipGetLastError();
      BatchDesc one;
      one.ninst = 1;
      one.nx = {m->c2.nx};
      one.ny = {m->c2.ny};
      one.hx = {m->c2.hx};
      one.hy = {m->c2.hy};
      one.off = {0, m->ncells};
      dg_status st = adjoint_tables(m, one, false);
      if (st != DG_OK) {
        dg_mesh_destroy(m);
        return st;
      }
    }
  } else if (d->kind == 0 && d->dim == 3) {
    m->ncoef = 31;
    m->ncells = d->n[0] * d->n[1] * d->n[2];
    m->c3.nx = (int)d->n[0];
    m->c3.ny = (int)d->n[1];
    m->c3.nz = (int)d->n[2];
    m->c3.hx = (d->hi[0] - d->lo[0]) / d->n[0];
    m->c3.hy = (d->hi[1] - d->lo[1]) / d->n[1];
    m->c3.hz = (d->hi[2] - d->lo[2]) / d->n[2];
    m->c3.tiles_x = (int)((d->n[0] + 61) / 62);
    m->c3.tiles_y = (int)d->n[1];
    m->c3.planes_per_tile =
        default_planes3d(m->c3.tiles_x, m->c3.ny, d->n[2], cfg->precision == DG_FP64);
    m->c3.tiles_z = (int)((d->n[2] + m->c3.planes_per_tile - 1) / m->c3.planes_per_tile);
    nwaves = (int64_t)m->c3.tiles_x * m->c3.tiles_y * m->c3.tiles_z;
  } else if (d->kind == 2) {
    m->ncoef = 12;
    BatchDesc& bd = m->bt.d;
    bd.ninst = d->ninst;
    bd.off.assign(1, 0);
    int64_t maxtiles = 0;
    for (int i = 0; i < d->ninst; ++i) {
      const int nx = d->inst_n[2 * i], ny = d->inst_n[2 * i + 1];
      const double* bx = d->inst_box + 4 * i;
      bd.nx.push_back(nx);
      bd.ny.push_back(ny);
      bd.hx.push_back((bx[2] - bx[0]) / nx);
      bd.hy.push_back((bx[3] - bx[1]) / ny);
      bd.off.push_back(bd.off.back() + (int64_t)nx * ny);
      maxtiles += (int64_t)((nx + 59) / 60) * ny;  // one row per tile
    }
    m->ncells = bd.off.back();
    if (m->ncells * 12 >= ((int64_t)1 << 31)) {
      delete m;
      return einval("dg_mesh_create: batch too large for 32-bit indexing");
    }
    m->bt.ninst = d->ninst;
    m->bt.rows = default_batch_rows();
    const bool f64 = cfg->precision == DG_FP64;
    hipError_t e2 = hipMalloc(&m->bt.inst, batch_record_size(f64) * d->ninst);
    if (e2 == hipSuccess) e2 = hipMalloc(&m->bt.tile_inst, sizeof(int) * maxtiles);
    if (e2 == hipSuccess) e2 = hipMalloc(&m->bt.inst_tile0, sizeof(int) * (d->ninst + 1));
    if (e2 != hipSuccess) {
      dg_mesh_destroy(m);
      return hip_fail(e2, "dg_mesh_create: batch tables");
    }
    dg_status st = batch_upload(m);
    if (st == DG_OK) st = adjoint_tables(m, bd, true);
    if (st != DG_OK) {
      dg_mesh_destroy(m);
      return st;
    }
    nwaves = maxtiles;
  } else if (d->kind == 3) {
    m->ncoef = 12;
    m->ncells = d->ncells;
    dg_status st = moving_create(m, d);
    if (st != DG_OK) {
      delete m;
      return st;
    }
    nwaves = (m->ncells + 63) / 64;
  } else {
    m->ncoef = 12;
    dg_status st = facelist_create(m, d);
    if (st != DG_OK) {
      delete m;
      return st;
    }
    nwaves = m->fl.nblocks * 4;
  }
  const size_t bytes = (size_t)m->ncoef * (size_t)m->ncells * m->elem;
  hipError_t e = hipMalloc(&m->v1, bytes);
  const bool separate_limiter = limiter_pass(m);
  if (e == hipSuccess && separate_limiter) e = hipMalloc(&m->ws_a, bytes);
  // (2D MHD limits on read: its stage kernels need only ws_a, for Pi(U^n))
  if (e == hipSuccess && m->dim == 3) e = hipMalloc(&m->ws_b, bytes);
  if (e == hipSuccess) e = hipMalloc(&m->status, sizeof(int));
  if (e == hipSuccess) e = hipMemset(m->status, 0, sizeof(int));
  // partial minima: one per wave of the fused stage, or one per 64 cells of
  // the stand-alone CFL kernel (whole 256-thread blocks write)
  // (the finest 2D tiling, one row per wave, has at most ncells/60 + rows
  // waves, ncells/56 + rows for the fused step; 3D: one plane per row-wave)
  if (m->kind == 0)
    nwaves = std::max<int64_t>(nwaves, m->dim == 2 ? (m->ncells + 55) / 56 + m->c2.ny
                                                   : max_stage_waves3(m));
  m->ndtpart = (int)std::max<int64_t>(nwaves, 4 * ((m->ncells + 255) / 256));
  if (e == hipSuccess) e = hipMalloc(&m->dtpart, sizeof(double) * m->ndtpart);

  if (e != hipSuccess) {
    dg_status st = hip_fail(e, "dg_mesh_create: device allocation");
    dg_mesh_destroy(m);
    return e == hipErrorOutOfMemory ? DG_ENOMEM : st;
  }
  if (m->kind == 3) {
    // the mesh of the initial generators, built by the same walk as every step
    e = moving_init(m);
    if (e == hipSuccess) e = hipDeviceSynchronize();
    int flag = 0;
    if (e == hipSuccess) e = hipMemcpy(&flag, m->status, sizeof(int), hipMemcpyDeviceToHost);
    if (e != hipSuccess) {
      dg_status st = hip_fail(e, "dg_mesh_create: initial moving mesh");
      dg_mesh_destroy(m);
      return st;
    }
    if (flag) {
      dg_mesh_destroy(m);
      return einval("dg_mesh_create: the initial faces do not give a Voronoi mesh of the "
                    "generators");
    }
  }
  *out = m;
  return DG_OK;
}

void dg_mesh_destroy(dg_mesh_t m) {
  if (!m) return;
  (void)hipDeviceSynchronize();
  if (m->kind == 1) facelist_destroy(m);
  if (m->kind == 3) moving_destroy(m);
  drop_graph(m);
  if (m->cap_stream) (void)hipStreamDestroy(m->cap_stream);
  (void)hipFree(m->run_ws);
  (void)hipFree(m->bt.inst);
  (void)hipFree(m->bt.tile_inst);
  (void)hipFree(m->bt.inst_tile0);
  (void)hipFree(m->bt.adj_tile_inst);
  (void)hipFree(m->v1);
  (void)hipFree(m->tmp);
  (void)hipFree(m->ws_a);
  (void)hipFree(m->adj_inst);
  (void)hipFree(m->adj_ws1);
  (void)hipFree(m->adj_ws2);
  (void)hipFree(m->ws_b);
  (void)hipFree(m->status);
  (void)hipFree(m->dtpart);
  delete m;
}

int64_t dg_state_len(dg_mesh_t m) { return m ? (int64_t)m->ncoef * m->ncells : -1; }

int dg_ncoef(dg_mesh_t m) { return m ? m->ncoef : -1; }

dg_status dg_rhs(dg_mesh_t m, const void* U, void* dUdt, void* stream) {
  if (m) m->ws_a_fresh = false;
  if (!m || !U || !dUdt) return einval("dg_rhs: NULL argument");
  if (U == dUdt) return einval("dg_rhs: U and dUdt must not alias");
  return dispatch(m, kRhs, U, nullptr, dUdt, nullptr, 0.0, (hipStream_t)stream);
}

dg_status dg_limit(dg_mesh_t m, const void* U, void* Ul, void* stream) {
  if (m) m->ws_a_fresh = false;
  if (!m || !U || !Ul) return einval("dg_limit: NULL argument");
  if (U == Ul) return einval("dg_limit: U and U_lim must not alias");
  return dispatch(m, kLimit, U, nullptr, Ul, nullptr, 0.0, (hipStream_t)stream);
}

// Meshes whose SSP-RK2 step runs as one fused kernel (both stages in one pass
// over the rows): 2D Euler on a single Cartesian mesh with HLL and the limiter
// off or that of Sec. 2.5.
static bool fused_step(const dg_mesh* m) {
  return m->kind == 0 && m->dim == 2 && m->cfg.physics == DG_EULER &&
         m->cfg.flux == DG_FLUX_HLL && m->cfg.limiter != DG_LIMITER_WENO;
}

static dg_status step_impl(dg_mesh_t m, const void* U, void* Un, const double* dt_dev,
                           double dt_host, hipStream_t s, double cfl = 0.0,
                           double* dt_next = nullptr) {
  m->ws_a_fresh = false;
  void* target = Un;
  if (U == Un) {
    if (!m->tmp) {
      hipError_t e = hipMalloc(&m->tmp, (size_t)m->ncoef * m->ncells * m->elem);
      if (e != hipSuccess) return hip_fail(e, "dg_step: workspace allocation");
    }
    target = m->tmp;
  }
  dg_status st;
  if (fused_step(m)) {
    st = dispatch(m, kStep, U, nullptr, target, dt_dev, dt_host, s, cfl, dt_next);
  } else {
    st = dispatch(m, kStage1, U, nullptr, m->v1, dt_dev, dt_host, s);
    if (st != DG_OK) return st;
    // a separate limiter pass keeps Pi(U) of stage 1 for the stage-2 combination
    m->ws_a_fresh = true;
    m->ws_a_src = U;
    st = dispatch(m, kStage2, m->v1, U, target, dt_dev, dt_host, s, cfl, dt_next);
    m->ws_a_fresh = false;
  }
  if (st != DG_OK) return st;
  if (target != Un) {
    hipError_t e = hipMemcpyAsync(Un, target, (size_t)m->ncoef * m->ncells * m->elem,
                                  hipMemcpyDeviceToDevice, s);
    if (e != hipSuccess) return hip_fail(e, "dg_step: copy back");
  }
  return DG_OK;
}

dg_status dg_step(dg_mesh_t m, const void* U, void* Un, double dt, void* stream) {
  if (!m || !U || !Un) return einval("dg_step: NULL argument");
  if (!std::isfinite(dt) || dt < 0) return einval("dg_step: dt must be finite and >= 0");
  return step_impl(m, U, Un, nullptr, dt, (hipStream_t)stream);
}

dg_status dg_stage1(dg_mesh_t m, const void* U, void* V1, double dt, const double* dt_dev,
                    void* stream) {
  if (!m || !U || !V1) return einval("dg_stage1: NULL argument");
  if (U == V1) return einval("dg_stage1: U and V1 must not alias");
  if (!dt_dev && (!std::isfinite(dt) || dt < 0)) return einval("dg_stage1: dt must be finite and >= 0");
  dg_status st = dispatch(m, kStage1, U, nullptr, V1, dt_dev, dt, (hipStream_t)stream);
  // a separate limiter pass keeps Pi(U); an immediately following dg_stage2 on
  // the same U reuses it
  m->ws_a_fresh = st == DG_OK && limiter_pass(m);
  m->ws_a_src = U;
  return st;
}

dg_status dg_stage2(dg_mesh_t m, const void* U, const void* V1, void* Un, double dt,
                    const double* dt_dev, double cfl, double* dt_next_dev, void* stream) {
  if (!m || !U || !V1 || !Un) return einval("dg_stage2: NULL argument");
  if (Un == U || Un == V1) return einval("dg_stage2: U_next must not alias U or V1");
  if (!dt_dev && (!std::isfinite(dt) || dt < 0)) return einval("dg_stage2: dt must be finite and >= 0");
  if (dt_next_dev && !(cfl > 0 && std::isfinite(cfl))) return einval("dg_stage2: cfl must be > 0");
  dg_status st = dispatch(m, kStage2, V1, U, Un, dt_dev, dt, (hipStream_t)stream, cfl, dt_next_dev);
  m->ws_a_fresh = false;
  return st;
}

dg_status dg_step_devdt(dg_mesh_t m, const void* U, void* Un, const double* dt_dev,
                        void* stream) {
  if (!m || !U || !Un || !dt_dev) return einval("dg_step_devdt: NULL argument");
  return step_impl(m, U, Un, dt_dev, 0.0, (hipStream_t)stream);
}

dg_status dg_step_cfl(dg_mesh_t m, const void* U, void* Un, const double* dt_dev, double cfl,
                      double* dt_next_dev, void* stream) {
  if (!m || !U || !Un || !dt_dev) return einval("dg_step_cfl: NULL argument");
  if (dt_next_dev && !(cfl > 0 && std::isfinite(cfl))) return einval("dg_step_cfl: cfl must be > 0");
  if (m->kind == 3) {
    set_error("dg_step_cfl: moving Voronoi meshes step with dg_step_mh");
    return DG_EUNSUPPORTED;
  }
  return step_impl(m, U, Un, dt_dev, 0.0, (hipStream_t)stream, cfl, dt_next_dev);
}

dg_status dg_cfl_dt(dg_mesh_t m, const void* U, double cfl, double* dt_dev, void* stream) {
  if (m) m->ws_a_fresh = false;
  if (!m || !U || !dt_dev) return einval("dg_cfl_dt: NULL argument");
  if (!(cfl > 0) || !std::isfinite(cfl)) return einval("dg_cfl_dt: cfl must be > 0");
  hipError_t e;
  hipStream_t s = (hipStream_t)stream;
  if (m->kind == 3)
    e = launch_moving_cfl(m, U, cfl, dt_dev, s);
  else if (m->kind == 1)
    e = launch_facelist_cfl(m, U, cfl, dt_dev, s);
  else if (m->kind == 2)
    e = launch_cart2d_batch_cfl(m, U, cfl, dt_dev, s);
  else if (m->dim == 2 && m->cfg.physics == DG_MHD)
    e = launch_mhd2d_cfl(m, U, cfl, dt_dev, s);
  else if (m->dim == 2)
    e = launch_cart2d_cfl(m, U, cfl, dt_dev, s);
  else
    e = launch_cart3d_cfl(m, U, cfl, dt_dev, s);
  if (e != hipSuccess) return hip_fail(e, "dg_cfl_dt launch");
  return DG_OK;
}

dg_status dg_cfl_dt_static(dg_mesh_t m, const void* U, double cfl, double* dt_dev,
                           void* stream) {
  if (!m || !U || !dt_dev) return einval("dg_cfl_dt_static: NULL argument");
  if (!(cfl > 0) || !std::isfinite(cfl)) return einval("dg_cfl_dt_static: cfl must be > 0");
  if (m->kind != 0 || m->dim != 2 || m->cfg.physics != DG_EULER) {
    set_error("dg_cfl_dt_static: built for single 2D Cartesian Euler meshes");
    return DG_EUNSUPPORTED;
  }
  if (4 * ((m->ncells + 255) / 256) > kCflScratchParts)
    return einval("dg_cfl_dt_static: mesh above the static scratch limit of " +
                  std::to_string(kCflScratchParts * 64) + " cells");
  m->ws_a_fresh = false;
  hipError_t e = launch_cart2d_cfl_static(m, U, cfl, dt_dev, (hipStream_t)stream);
  if (e == hipErrorInvalidSymbol) {
    set_error("dg_cfl_dt_static: no static scratch address for this device");
    return DG_EHIP;
  }
  if (e != hipSuccess) return hip_fail(e, "dg_cfl_dt_static launch");
  return DG_OK;
}

dg_status dg_adjoint_step(dg_mesh_t m, const void* U, const void* V1, double dt,
                          const double* dt_dev, const void* lam_np1, void* lam_n, void* stream) {
  if (!m || !U || !lam_np1 || !lam_n) return einval("dg_adjoint_step: NULL argument");
  m->ws_a_fresh = false;
  // 2D ideal MHD on a single Cartesian mesh (HLLD, limiter of Sec. 2.5 or none)
  const bool mhd2 = m->kind == 0 && m->dim == 2 && m->cfg.physics == DG_MHD &&
                    m->cfg.limiter != DG_LIMITER_WENO;
  const bool mhd3 = m->kind == 0 && m->dim == 3 && m->cfg.limiter != DG_LIMITER_WENO;
  // 2D Euler on a static face-list mesh (HLL, limiter of Sec. 2.5 or none)
  const bool flist = m->kind == 1 && m->cfg.physics == DG_EULER &&
                     m->cfg.flux == DG_FLUX_HLL && m->cfg.limiter != DG_LIMITER_WENO;
  if (!mhd2 && !mhd3 && !flist &&
      (!m->adj_inst || m->cfg.flux != DG_FLUX_HLL || m->cfg.limiter == DG_LIMITER_WENO)) {
    set_error("dg_adjoint_step: built for 2D Euler Cartesian meshes, batches and static "
              "face-list meshes with HLL and the Arepo limiter, and 2D and 3D MHD Cartesian "
              "meshes with HLLD");
    return DG_EUNSUPPORTED;
  }
  if (!dt_dev && (!std::isfinite(dt) || dt < 0))
    return einval("dg_adjoint_step: dt must be finite and >= 0");
  if (lam_n == lam_np1 || lam_n == U || lam_n == V1)
    return einval("dg_adjoint_step: lam_n must not alias U, V1 or lam_np1");
  hipStream_t s = (hipStream_t)stream;
  const size_t bytes = (size_t)m->ncoef * m->ncells * m->elem;
  hipError_t e = hipSuccess;
  if (!m->adj_ws1) e = hipMalloc(&m->adj_ws1, bytes);
  if (e == hipSuccess && !m->adj_ws2) e = hipMalloc(&m->adj_ws2, bytes);
  if (e != hipSuccess) return hip_fail(e, "dg_adjoint_step: workspace allocation");
  if (!V1) {
    dg_status st = dispatch(m, kStage1, U, nullptr, m->v1, dt_dev, dt, s);
    if (st != DG_OK) return st;
    V1 = m->v1;
  }
  if (mhd2 || mhd3 || flist) {
    e = mhd2   ? launch_adjoint_mhd2d(m, U, V1, dt_dev, dt, lam_np1, lam_n, m->adj_ws1,
                                      m->adj_ws2, s)
        : mhd3 ? launch_adjoint_mhd3d(m, U, V1, dt_dev, dt, lam_np1, lam_n, m->adj_ws1,
                                      m->adj_ws2, s)
               : launch_adjoint_facelist(m, U, V1, dt_dev, dt, lam_np1, lam_n, m->adj_ws1,
                                         m->adj_ws2, s);
    if (e != hipSuccess) return hip_fail(e, "dg_adjoint_step launch");
    return DG_OK;
  }
  e = launch_adjoint2d(m->adj_inst, m->kind == 2 ? m->bt.adj_tile_inst : nullptr, m->adj_tiles,
                       (int)m->ncells, dg_state_len(m), m->cfg.precision == DG_FP64,
                       m->cfg.limiter == DG_LIMITER_MINMOD, m->cfg.gamma, U, V1, dt_dev, dt,
                       lam_np1, lam_n, m->adj_ws1, m->adj_ws2, s);
  if (e != hipSuccess) return hip_fail(e, "dg_adjoint_step launch");
  return DG_OK;
}

static bool mh_supported(const dg_mesh* m) {
  return m->cfg.physics == DG_EULER &&
         ((m->kind == 0 && m->dim == 2) || m->kind == 2 || m->kind == 3);
}

dg_status dg_step_mh(dg_mesh_t m, const void* U, void* Un, double dt, const double* dt_dev,
                     double cfl, double* dt_next_dev, void* stream) {
  if (!m || !U || !Un) return einval("dg_step_mh: NULL argument");
  m->ws_a_fresh = false;
  if (!mh_supported(m)) {
    set_error("dg_step_mh: built for 2D Euler Cartesian meshes, batches and moving meshes");
    return DG_EUNSUPPORTED;
  }
  if (U == Un) return einval("dg_step_mh: U_next must not alias U");
  if (!dt_dev && (!std::isfinite(dt) || dt < 0)) return einval("dg_step_mh: dt must be finite and >= 0");
  if (dt_next_dev && !(cfl > 0 && std::isfinite(cfl))) return einval("dg_step_mh: cfl must be > 0");
  return dispatch(m, kMH, U, nullptr, Un, dt_dev, dt, (hipStream_t)stream, cfl, dt_next_dev);
}

dg_status dg_run(dg_mesh_t m, const void* U_in, void* U_out, int nsteps, double cfl,
                 double* dt_hist, int ckpt_every, void* const* ckpt, void* const* v1_keep,
                 int flags, void* stream) {
  if (!m || !U_in || !U_out || !dt_hist) return einval("dg_run: NULL argument");
  if (nsteps < 1) return einval("dg_run: nsteps must be >= 1");
  if (!(cfl >= 0) || !std::isfinite(cfl)) return einval("dg_run: cfl must be finite and >= 0");
  if (ckpt_every < 0 || (ckpt_every > 0 && nsteps > ckpt_every && !ckpt))
    return einval("dg_run: checkpoints need ckpt_every >= 0 and a ckpt array");
  if (nsteps == 1 && U_out == U_in) return einval("dg_run: U_out may equal U_in only for >= 2 steps");
  if (flags & ~(DG_RUN_GRAPH | DG_RUN_MUSCL_HANCOCK | DG_RUN_TWO_STAGE))
    return einval("dg_run: unknown flag");
  const bool mh = (flags & DG_RUN_MUSCL_HANCOCK) != 0;
  const bool two_stage = (flags & DG_RUN_TWO_STAGE) != 0;
  if (mh && two_stage) return einval("dg_run: DG_RUN_TWO_STAGE is a flag of the SSP-RK2 step");
  if (m->kind == 3) {
    set_error("dg_run: not built for moving meshes (step them with dg_step_mh)");
    return DG_EUNSUPPORTED;
  }
  if (mh && !mh_supported(m)) {
    set_error("dg_run: MUSCL-Hancock is built for 2D Euler Cartesian meshes and batches");
    return DG_EUNSUPPORTED;
  }
  if (mh && v1_keep) return einval("dg_run: v1_keep needs the SSP-RK2 integrator");
  m->ws_a_fresh = false;
  hipStream_t s = (hipStream_t)stream;
  const size_t bytes = (size_t)m->ncoef * m->ncells * m->elem;
  hipError_t e = hipSuccess;
  if (!m->tmp) e = hipMalloc(&m->tmp, bytes);
  if (e == hipSuccess && !m->run_ws) e = hipMalloc(&m->run_ws, bytes);
  if (e != hipSuccess) return hip_fail(e, "dg_run: workspace allocation");
  const int nd = m->kind == 2 ? m->bt.ninst : 1;
  const int nck = ckpt_every > 0 ? (nsteps - 1) / ckpt_every : 0;

  auto enqueue = [&](hipStream_t q) -> dg_status {
    if (cfl > 0) {
      dg_status st = dg_cfl_dt(m, U_in, cfl, dt_hist, q);
      if (st != DG_OK) return st;
    }
    const void* cur = U_in;
    for (int n = 0; n < nsteps; ++n) {
      void* V1 = v1_keep ? v1_keep[n] : m->v1;
      void* out;
      if (n + 1 == nsteps)
        out = U_out;
      else if (ckpt_every > 0 && (n + 1) % ckpt_every == 0)
        out = ckpt[(n + 1) / ckpt_every - 1];
      else
        out = cur == m->tmp ? m->run_ws : m->tmp;
      const double* dtn = dt_hist + (int64_t)n * nd;
      if (mh) {
        dg_status st = dispatch(m, kMH, cur, nullptr, out, dtn, 0.0, q, cfl,
                                cfl > 0 ? dt_hist + (int64_t)(n + 1) * nd : nullptr);
        if (st != DG_OK) return st;
        cur = out;
        continue;
      }
      if (!v1_keep && !two_stage && fused_step(m)) {
        dg_status st = dispatch(m, kStep, cur, nullptr, out, dtn, 0.0, q, cfl,
                                cfl > 0 ? dt_hist + (int64_t)(n + 1) * nd : nullptr);
        if (st != DG_OK) return st;
        cur = out;
        continue;
      }
      dg_status st = dispatch(m, kStage1, cur, nullptr, V1, dtn, 0.0, q);
      if (st != DG_OK) return st;
      m->ws_a_fresh = true;
      m->ws_a_src = cur;
      st = dispatch(m, kStage2, V1, cur, out, dtn, 0.0, q, cfl,
                    cfl > 0 ? dt_hist + (int64_t)(n + 1) * nd : nullptr);
      m->ws_a_fresh = false;
      if (st != DG_OK) return st;
      cur = out;
    }
    return DG_OK;
  };

  if (!(flags & DG_RUN_GRAPH)) return enqueue(s);

  std::vector<const void*> key = {U_in, U_out, dt_hist, (const void*)(intptr_t)nsteps,
                                  (const void*)(intptr_t)ckpt_every, (const void*)(intptr_t)flags};
  int64_t cbits;
  std::memcpy(&cbits, &cfl, sizeof(cbits));
  key.push_back((const void*)(intptr_t)cbits);
  for (int j = 0; j < nck; ++j) key.push_back(ckpt[j]);
  if (v1_keep)
    for (int n = 0; n < nsteps; ++n) key.push_back(v1_keep[n]);
  else
    key.push_back(nullptr);
  RunGraph* hit = nullptr;
  for (RunGraph& g : m->runs)
    if (g.key == key) hit = &g;
  if (!hit) {
    if ((int)m->runs.size() >= kMaxRunGraphs) {
      auto old = std::min_element(m->runs.begin(), m->runs.end(),
                                  [](const RunGraph& a, const RunGraph& b) {
                                    return a.last_use < b.last_use;
                                  });
      free_graph(*old);
      m->runs.erase(old);
    }
    if (!m->cap_stream) {
      e = hipStreamCreateWithFlags(&m->cap_stream, hipStreamNonBlocking);
      if (e != hipSuccess) return hip_fail(e, "dg_run: capture stream");
    }
    e = hipStreamBeginCapture(m->cap_stream, hipStreamCaptureModeRelaxed);
    if (e != hipSuccess) return hip_fail(e, "dg_run: begin capture");
    dg_status st = enqueue(m->cap_stream);
    RunGraph g;
    e = hipStreamEndCapture(m->cap_stream, &g.graph);
    if (st != DG_OK) {
      free_graph(g);
      return st;
    }
    if (e != hipSuccess) return hip_fail(e, "dg_run: end capture");
    e = hipGraphInstantiate(&g.exec, g.graph, nullptr, nullptr, 0);
    if (e != hipSuccess) {
      free_graph(g);
      return hip_fail(e, "dg_run: instantiate graph");
    }
    g.key = key;
    m->runs.push_back(g);
    hit = &m->runs.back();
  }
  hit->last_use = ++m->run_clock;
  e = hipGraphLaunch(hit->exec, s);
  if (e != hipSuccess) return hip_fail(e, "dg_run: graph launch");
  return DG_OK;
}

int dg_ninst(dg_mesh_t m) { return m ? (m->kind == 2 ? m->bt.ninst : 1) : -1; }

dg_status dg_instance_offsets(dg_mesh_t m, int64_t* off) {
  if (!m || !off) return einval("dg_instance_offsets: NULL argument");
  if (m->kind != 2) {
    off[0] = 0;
    off[1] = m->ncells;
    return DG_OK;
  }
  for (int i = 0; i <= m->bt.ninst; ++i) off[i] = m->bt.d.off[i];
  return DG_OK;
}

dg_status dg_set_launch(dg_mesh_t m, int waves_per_group, int grid_waves) {
  if (!m) return einval("dg_set_launch: NULL handle");
  if (waves_per_group != 1 && waves_per_group != 2 && waves_per_group != 4)
    return einval("dg_set_launch: waves_per_group must be 1, 2 or 4");
  if (grid_waves < 0) return einval("dg_set_launch: grid_waves must be >= 0");
  if (m->kind != 2) return DG_OK;
  m->bt.wpb = waves_per_group;
  m->bt.grid_waves = grid_waves;
  drop_graph(m);
  return DG_OK;
}

dg_status dg_get_launch(dg_mesh_t m, int* waves_per_group, int* grid_waves) {
  if (!m || !waves_per_group || !grid_waves) return einval("dg_get_launch: NULL argument");
  *waves_per_group = m->kind == 2 ? m->bt.wpb : 4;
  *grid_waves = m->kind == 2 ? m->bt.grid_waves : 0;
  return DG_OK;
}

dg_status dg_set_tiling(dg_mesh_t m, int rows) {
  if (!m) return einval("dg_set_tiling: NULL handle");
  if (rows < 0) return einval("dg_set_tiling: rows must be >= 0");
  drop_graph(m);
  if (m->kind == 2) {
    hipError_t e = hipDeviceSynchronize();
    if (e != hipSuccess) return hip_fail(e, "dg_set_tiling: synchronise");
    m->bt.rows = rows ? rows : default_batch_rows();
    return batch_upload(m);
  }
  if (m->kind != 0) return DG_OK;
  if (m->dim == 2) {
    int r = rows ? std::min(rows, m->c2.ny)
                 : (m->cfg.physics == DG_MHD ? default_rows_mhd2d(m->c2.tiles_x, m->c2.ny,
                                                                  m->cfg.precision == DG_FP64)
                                             : default_rows_euler2d(m->c2.tiles_x, m->c2.ny,
                                                                    m->cfg.precision == DG_FP64));
    m->c2.rows_per_tile = r;
    m->c2.tiles_y = (m->c2.ny + r - 1) / r;
    const int rs = rows ? std::min(rows, m->c2.ny)
                        : default_step_rows(m->c2.step_tiles_x, m->c2.ny,
                                            m->cfg.precision == DG_FP64);
    m->c2.step_rows = rs;
    m->c2.step_tiles_y = (m->c2.ny + rs - 1) / rs;
  } else {
    int r = rows ? std::min(rows, m->c3.nz)
                 : default_planes3d(m->c3.tiles_x, m->c3.ny, m->c3.nz,
                                    m->cfg.precision == DG_FP64);
    m->c3.planes_per_tile = r;
    m->c3.tiles_z = (m->c3.nz + r - 1) / r;
  }
  return DG_OK;
}

int dg_get_tiling(dg_mesh_t m) {
  if (!m) return -1;
  if (m->kind == 2) return m->bt.rows;
  if (m->kind != 0) return 0;
  return m->dim == 2 ? m->c2.rows_per_tile : m->c3.planes_per_tile;
}

dg_status dg_check(dg_mesh_t m) {
  if (!m) return einval("dg_check: NULL handle");
  hipError_t e = hipDeviceSynchronize();
  if (e != hipSuccess) return hip_fail(e, "dg_check: synchronise");
  int flag = 0;
  e = hipMemcpy(&flag, m->status, sizeof(int), hipMemcpyDeviceToHost);
  if (e != hipSuccess) return hip_fail(e, "dg_check: read status");
  if (flag) {
    e = hipMemset(m->status, 0, sizeof(int));
    if (e != hipSuccess) return hip_fail(e, "dg_check: clear status");
    if (flag & 2) {
      set_error("moving mesh: a cell's Voronoi polygon could not be built from its previous "
                "neighbourhood, exceeded 16 faces, or its neighbours disagree");
      return DG_EMESH;
    }
    set_error("non-physical state (rho <= 0, p <= 0 or non-finite) at a quadrature point");
    return DG_ENONPHYSICAL;
  }
  return DG_OK;
}

dg_status dg_set_mesh_motion(dg_mesh_t m, int motion) {
  if (!m) return einval("dg_set_mesh_motion: NULL handle");
  if (m->kind != 3) {
    set_error("dg_set_mesh_motion: only moving meshes have generator motion");
    return DG_EUNSUPPORTED;
  }
  if (motion != 0 && motion != 1) return einval("dg_set_mesh_motion: motion must be 0 or 1");
  moving_set_motion(m, motion);
  return DG_OK;
}

dg_status dg_set_moving_timing(dg_mesh_t m, int on) {
  if (!m) return einval("dg_set_moving_timing: NULL handle");
  if (m->kind != 3) {
    set_error("dg_set_moving_timing: built for moving meshes");
    return DG_EUNSUPPORTED;
  }
  moving_set_timing(m, on);
  return DG_OK;
}

dg_status dg_moving_timing(dg_mesh_t m, double* avg_ms, int* nsteps) {
  if (!m || !avg_ms) return einval("dg_moving_timing: NULL argument");
  if (m->kind != 3) {
    set_error("dg_moving_timing: built for moving meshes");
    return DG_EUNSUPPORTED;
  }
  const int r = moving_timing(m, avg_ms, nsteps);
  if (r) return hip_fail((hipError_t)r, "dg_moving_timing");
  return DG_OK;
}

dg_status dg_mesh_geometry(dg_mesh_t m, double* generators, double* volume, double* centroid,
                           int32_t* ring, int32_t* degree) {
  if (!m) return einval("dg_mesh_geometry: NULL handle");
  if (m->kind != 3) {
    set_error("dg_mesh_geometry: built for moving meshes");
    return DG_EUNSUPPORTED;
  }
  const int r = moving_read(m, generators, volume, centroid, ring, degree);
  if (r) return hip_fail((hipError_t)r, "dg_mesh_geometry: copy");
  return DG_OK;
}

// ------------------------------------------------------------------ batches
// A dg_batch_t wraps one batch mesh (kind 2) built from single 2D Cartesian
// Euler meshes; every call forwards to the mesh-handle entry points.

dg_status dg_batch_create(const dg_mesh_t* meshes, int ninst, const char* autotune_cache,
                          dg_batch_t* out) {
  if (!out) return einval("dg_batch_create: out is NULL");
  *out = nullptr;
  if (!meshes || ninst < 1) return einval("dg_batch_create: needs ninst >= 1 meshes");
  const dg_mesh* m0 = meshes[0];
  if (!m0) return einval("dg_batch_create: NULL mesh");
  std::vector<int32_t> inst_n(2 * (size_t)ninst);
  std::vector<double> inst_box(4 * (size_t)ninst);
  for (int i = 0; i < ninst; ++i) {
    const dg_mesh* m = meshes[i];
    if (!m) return einval("dg_batch_create: NULL mesh");
    if (m->kind != 0 || m->dim != 2 || m->cfg.physics != DG_EULER) {
      set_error("dg_batch_create: instances must be single 2D Cartesian Euler meshes");
      return DG_EUNSUPPORTED;
    }
    if (m->cfg.precision != m0->cfg.precision || m->cfg.flux != m0->cfg.flux ||
        m->cfg.limiter != m0->cfg.limiter || m->cfg.gamma != m0->cfg.gamma)
      return einval("dg_batch_create: instances need identical dg_config");
    inst_n[2 * i] = m->c2.nx;
    inst_n[2 * i + 1] = m->c2.ny;
    inst_box[4 * i] = m->c2.lo[0];
    inst_box[4 * i + 1] = m->c2.lo[1];
    inst_box[4 * i + 2] = m->c2.hi[0];
    inst_box[4 * i + 3] = m->c2.hi[1];
  }
  int rows = 0, wpb = 0, grid = -1;
  if (autotune_cache) {
    FILE* f = std::fopen(autotune_cache, "r");
    if (!f) return einval(std::string("dg_batch_create: cannot read ") + autotune_cache);
    const int got = std::fscanf(f, "%d %d %d", &rows, &wpb, &grid);
    std::fclose(f);
    if (got != 3 || rows < 1 || grid < 0)
      return einval("dg_batch_create: launch file needs 'rows waves_per_group grid_waves'");
  }
  dg_mesh_desc d{};
  d.dim = 2;
  d.kind = 2;
  d.ninst = ninst;
  d.inst_n = inst_n.data();
  d.inst_box = inst_box.data();
  dg_mesh_t bm = nullptr;
  dg_status st = dg_mesh_create(&d, &m0->cfg, &bm);
  if (st != DG_OK) return st;
  if (autotune_cache) {
    st = dg_set_tiling(bm, rows);
    if (st == DG_OK) st = dg_set_launch(bm, wpb, grid);
    if (st != DG_OK) {
      dg_mesh_destroy(bm);
      return st;
    }
  }
  dg_batch* b = new (std::nothrow) dg_batch();
  if (!b) {
    dg_mesh_destroy(bm);
    set_error("dg_batch_create: out of host memory");
    return DG_ENOMEM;
  }
  b->mesh = bm;
  *out = b;
  return DG_OK;
}

dg_mesh_t dg_batch_mesh(dg_batch_t b) { return b ? b->mesh : nullptr; }

int64_t dg_batch_offset(dg_batch_t b, int inst) {
  if (!b || inst < 0 || inst > b->mesh->bt.ninst) return -1;
  return b->mesh->bt.d.off[inst];
}

dg_status dg_batch_run(dg_batch_t b, void* U, double cfl, double* dt_hist_dev, int nsteps,
                       void* stream) {
  if (!b || !U || !dt_hist_dev) return einval("dg_batch_run: NULL argument");
  if (nsteps < 1) return einval("dg_batch_run: nsteps must be >= 1");
  dg_mesh* m = b->mesh;
  if (nsteps >= 2)
    return dg_run(m, U, U, nsteps, cfl, dt_hist_dev, 0, nullptr, nullptr, DG_RUN_GRAPH, stream);
  // one step in place: through the handle's staging buffer
  const size_t bytes = (size_t)m->ncoef * m->ncells * m->elem;
  if (!m->tmp) {
    hipError_t e = hipMalloc(&m->tmp, bytes);
    if (e != hipSuccess) return hip_fail(e, "dg_batch_run: workspace allocation");
  }
  dg_status st = dg_run(m, U, m->tmp, 1, cfl, dt_hist_dev, 0, nullptr, nullptr, DG_RUN_GRAPH,
                        stream);
  if (st != DG_OK) return st;
  hipError_t e = hipMemcpyAsync(U, m->tmp, bytes, hipMemcpyDeviceToDevice, (hipStream_t)stream);
  if (e != hipSuccess) return hip_fail(e, "dg_batch_run: copy");
  return DG_OK;
}

dg_status dg_batch_adjoint_step(dg_batch_t b, const void* U_n, const double* dt_dev,
                                const void* lam_np1, void* lam_n, void* stream) {
  if (!b || !dt_dev) return einval("dg_batch_adjoint_step: NULL argument");
  return dg_adjoint_step(b->mesh, U_n, nullptr, 0.0, dt_dev, lam_np1, lam_n, stream);
}

void dg_batch_destroy(dg_batch_t b) {
  if (!b) return;
  dg_mesh_destroy(b->mesh);
  delete b;
}

}  // extern "C"
