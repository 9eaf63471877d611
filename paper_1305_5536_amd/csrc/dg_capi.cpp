// Host side of the C ABI declared in include/dg.h: validation, device
// allocation, kernel dispatch and error reporting.  No arithmetic of the DG
// update happens here; every step runs in the HIP kernels.
#include <hip/hip_runtime.h>

#include <cmath>
#include <cstdio>
#include <cstring>
#include <new>
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
dg_status facelist_create(dg_mesh* m, const dg_mesh_desc* d);
void facelist_destroy(dg_mesh* m);
hipError_t launch_facelist(const dg_mesh* m, int mode, const void* in, const void* u0, void* out,
                           const double* dt_dev, double dt_host, double cfl, double* dt_next,
                           hipStream_t s);
hipError_t launch_facelist_cfl(const dg_mesh* m, const void* U, double cfl, double* dt_dev,
                               hipStream_t s);
hipError_t launch_cart3d(const dg_mesh* m, int mode, const void* in, const void* u0, void* out,
                         const double* dt_dev, double dt_host, double cfl, double* dt_next,
                         hipStream_t s);
hipError_t launch_cart3d_cfl(const dg_mesh* m, const void* U, double cfl, double* dt_dev,
                             hipStream_t s);

// Rows (2D) or planes (3D) marched by one wave.  Chosen so a launch has
// several waves per SIMD on 256 CUs; an explicit override comes from the
// DG_TILE_ROWS environment variable (used by the autotuner).
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

static dg_status dispatch(const dg_mesh* m, int mode, const void* in, const void* u0, void* out,
                          const double* dt_dev, double dt_host, hipStream_t s,
                          double cfl = 0.0, double* dt_next = nullptr) {
  hipError_t e;
  if (m->kind == 1)
    e = launch_facelist(m, mode, in, u0, out, dt_dev, dt_host, cfl, dt_next, s);
  else if (m->dim == 2)
    e = launch_cart2d(m, mode, in, u0, out, dt_dev, dt_host, cfl, dt_next, s);
  else
    e = launch_cart3d(m, mode, in, u0, out, dt_dev, dt_host, cfl, dt_next, s);
  if (e != hipSuccess) return hip_fail(e, "kernel launch");
  return DG_OK;
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
  if (cfg->limiter != DG_LIMITER_NONE && cfg->limiter != DG_LIMITER_MINMOD)
    return einval("dg_mesh_create: unknown limiter");
  if (!(cfg->gamma > 1.0) || !std::isfinite(cfg->gamma))
    return einval("dg_mesh_create: gamma must be finite and > 1");
  if (cfg->physics == DG_EULER) {
    if (cfg->flux != DG_FLUX_HLL) {
      set_error("dg_mesh_create: Euler supports the HLL flux only");
      return DG_EUNSUPPORTED;
    }
  } else if (cfg->physics == DG_MHD) {
    if (cfg->flux != DG_FLUX_HLLD) {
      set_error("dg_mesh_create: MHD supports the HLLD flux only");
      return DG_EUNSUPPORTED;
    }
    if (d->dim != 3 || d->kind != 0) {
      set_error("dg_mesh_create: MHD is built for 3D Cartesian meshes only");
      return DG_EUNSUPPORTED;
    }
  } else {
    return einval("dg_mesh_create: unknown physics");
  }
  if (d->kind != 0 && d->kind != 1) return einval("dg_mesh_create: unknown mesh kind");
  if (d->kind == 1 && d->dim != 2) {
    set_error("dg_mesh_create: face-list meshes are 2D only");
    return DG_EUNSUPPORTED;
  }
  if (d->kind == 0) {
    if (d->dim != 2 && d->dim != 3) return einval("dg_mesh_create: dim must be 2 or 3");
    if (d->dim == 3 && cfg->physics != DG_MHD) {
      set_error("dg_mesh_create: 3D Cartesian meshes are built for MHD only");
      return DG_EUNSUPPORTED;
    }
    for (int k = 0; k < d->dim; ++k) {
      if (d->n[k] < 1 || d->n[k] > (1 << 20)) return einval("dg_mesh_create: bad cell count");
      if (!(d->hi[k] > d->lo[k])) return einval("dg_mesh_create: hi must exceed lo");
    }
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
    m->ncoef = 12;
    m->ncells = d->n[0] * d->n[1];
    m->c2.nx = (int)d->n[0];
    m->c2.ny = (int)d->n[1];
    m->c2.hx = (d->hi[0] - d->lo[0]) / d->n[0];
    m->c2.hy = (d->hi[1] - d->lo[1]) / d->n[1];
    m->c2.tiles_x = (int)((d->n[0] + 59) / 60);
    m->c2.rows_per_tile = default_rows(m->c2.tiles_x, d->n[1]);
    m->c2.tiles_y = (int)((d->n[1] + m->c2.rows_per_tile - 1) / m->c2.rows_per_tile);
    nwaves = (int64_t)m->c2.tiles_x * m->c2.tiles_y;
    if (cfg->physics == DG_EULER) {
      dg::AdjInst ai{};
      ai.nx = m->c2.nx;
      ai.ny = m->c2.ny;
      ai.off = 0;
      ai.tx0 = 0;
      ai.tiles_x = (ai.nx + dg::kAdjTile - 1) / dg::kAdjTile;
      ai.tiles_y = (ai.ny + dg::kAdjTile - 1) / dg::kAdjTile;
      ai.hx = m->c2.hx;
      ai.hy = m->c2.hy;
      m->adj_tiles = ai.tiles_x * ai.tiles_y;
      hipError_t e2 = hipMalloc(&m->adj_inst, sizeof(dg::AdjInst));
      if (e2 == hipSuccess)
        e2 = hipMemcpy(m->adj_inst, &ai, sizeof(dg::AdjInst), hipMemcpyHostToDevice);
      if (e2 != hipSuccess) {
        dg_mesh_destroy(m);
        return hip_fail(e2, "dg_mesh_create: adjoint table");
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
    m->c3.planes_per_tile = default_rows((int64_t)m->c3.tiles_x * d->n[1], d->n[2]);
    m->c3.tiles_z = (int)((d->n[2] + m->c3.planes_per_tile - 1) / m->c3.planes_per_tile);
    nwaves = (int64_t)m->c3.tiles_x * m->c3.tiles_y * m->c3.tiles_z;
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
  const bool separate_limiter = m->dim == 3 || m->kind == 1;
  if (e == hipSuccess && separate_limiter) e = hipMalloc(&m->ws_a, bytes);
  if (e == hipSuccess && separate_limiter) e = hipMalloc(&m->ws_b, bytes);
  if (e == hipSuccess) e = hipMalloc(&m->status, sizeof(int));
  if (e == hipSuccess) e = hipMemset(m->status, 0, sizeof(int));
  // partial minima: one per wave of the fused stage, or one per 64 cells of
  // the stand-alone CFL kernel (whole 256-thread blocks write)
  // (the finest tiling, one row per wave, has at most ncells/60 + rows waves)
  nwaves = std::max<int64_t>(nwaves, (m->ncells + 59) / 60 + (m->dim == 2 ? m->c2.ny : m->c3.ny * m->c3.nz));
  m->ndtpart = (int)std::max<int64_t>(nwaves, 4 * ((m->ncells + 255) / 256));
  if (e == hipSuccess) e = hipMalloc(&m->dtpart, sizeof(double) * m->ndtpart);

  if (e != hipSuccess) {
    dg_status st = hip_fail(e, "dg_mesh_create: device allocation");
    dg_mesh_destroy(m);
    return e == hipErrorOutOfMemory ? DG_ENOMEM : st;
  }
  *out = m;
  return DG_OK;
}

void dg_mesh_destroy(dg_mesh_t m) {
  if (!m) return;
  (void)hipDeviceSynchronize();
  if (m->kind == 1) facelist_destroy(m);
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

static dg_status step_impl(dg_mesh_t m, const void* U, void* Un, const double* dt_dev,
                           double dt_host, hipStream_t s) {
  void* target = Un;
  if (U == Un) {
    if (!m->tmp) {
      hipError_t e = hipMalloc(&m->tmp, (size_t)m->ncoef * m->ncells * m->elem);
      if (e != hipSuccess) return hip_fail(e, "dg_step: workspace allocation");
    }
    target = m->tmp;
  }
  dg_status st = dispatch(m, kStage1, U, nullptr, m->v1, dt_dev, dt_host, s);
  if (st != DG_OK) return st;
  // 3D keeps Pi(U) of stage 1 in its workspace for the stage-2 combination
  m->ws_a_fresh = true;
  m->ws_a_src = U;
  st = dispatch(m, kStage2, m->v1, U, target, dt_dev, dt_host, s);
  m->ws_a_fresh = false;
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
  // 3D keeps Pi(U) in its workspace; an immediately following dg_stage2 on
  // the same U reuses it
  m->ws_a_fresh = st == DG_OK && (m->dim == 3 || m->kind == 1);
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

dg_status dg_cfl_dt(dg_mesh_t m, const void* U, double cfl, double* dt_dev, void* stream) {
  if (m) m->ws_a_fresh = false;
  if (!m || !U || !dt_dev) return einval("dg_cfl_dt: NULL argument");
  if (!(cfl > 0) || !std::isfinite(cfl)) return einval("dg_cfl_dt: cfl must be > 0");
  hipError_t e;
  hipStream_t s = (hipStream_t)stream;
  if (m->kind == 1)
    e = launch_facelist_cfl(m, U, cfl, dt_dev, s);
  else if (m->dim == 2)
    e = launch_cart2d_cfl(m, U, cfl, dt_dev, s);
  else
    e = launch_cart3d_cfl(m, U, cfl, dt_dev, s);
  if (e != hipSuccess) return hip_fail(e, "dg_cfl_dt launch");
  return DG_OK;
}

dg_status dg_adjoint_step(dg_mesh_t m, const void* U, const void* V1, double dt,
                          const void* lam_np1, void* lam_n, void* stream) {
  if (!m || !U || !lam_np1 || !lam_n) return einval("dg_adjoint_step: NULL argument");
  m->ws_a_fresh = false;
  if (m->kind != 0 || m->dim != 2 || !m->adj_inst) {
    set_error("dg_adjoint_step: built for 2D Euler Cartesian meshes");
    return DG_EUNSUPPORTED;
  }
  if (!std::isfinite(dt) || dt < 0) return einval("dg_adjoint_step: dt must be finite and >= 0");
  if (lam_n == lam_np1 || lam_n == U || lam_n == V1)
    return einval("dg_adjoint_step: lam_n must not alias U, V1 or lam_np1");
  hipStream_t s = (hipStream_t)stream;
  const size_t bytes = (size_t)m->ncoef * m->ncells * m->elem;
  hipError_t e = hipSuccess;
  if (!m->adj_ws1) e = hipMalloc(&m->adj_ws1, bytes);
  if (e == hipSuccess && !m->adj_ws2) e = hipMalloc(&m->adj_ws2, bytes);
  if (e != hipSuccess) return hip_fail(e, "dg_adjoint_step: workspace allocation");
  if (!V1) {
    dg_status st = dispatch(m, kStage1, U, nullptr, m->v1, nullptr, dt, s);
    if (st != DG_OK) return st;
    V1 = m->v1;
  }
  e = launch_adjoint2d(m->adj_inst, nullptr, m->adj_tiles, (int)m->ncells, dg_state_len(m),
                       m->cfg.precision == DG_FP64, m->cfg.limiter == DG_LIMITER_MINMOD,
                       m->cfg.gamma, U, V1, nullptr, dt, lam_np1, lam_n, m->adj_ws1, m->adj_ws2,
                       s);
  if (e != hipSuccess) return hip_fail(e, "dg_adjoint_step launch");
  return DG_OK;
}

dg_status dg_set_tiling(dg_mesh_t m, int rows) {
  if (!m) return einval("dg_set_tiling: NULL handle");
  if (rows < 0) return einval("dg_set_tiling: rows must be >= 0");
  if (m->kind != 0) return DG_OK;
  if (m->dim == 2) {
    int r = rows ? std::min(rows, m->c2.ny) : default_rows(m->c2.tiles_x, m->c2.ny);
    m->c2.rows_per_tile = r;
    m->c2.tiles_y = (m->c2.ny + r - 1) / r;
  } else {
    int r = rows ? std::min(rows, m->c3.nz)
                 : default_rows((int64_t)m->c3.tiles_x * m->c3.tiles_y, m->c3.nz);
    m->c3.planes_per_tile = r;
    m->c3.tiles_z = (m->c3.nz + r - 1) / r;
  }
  return DG_OK;
}

int dg_get_tiling(dg_mesh_t m) {
  if (!m) return -1;
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
    set_error("non-physical state (rho <= 0, p <= 0 or non-finite) at a quadrature point");
    return DG_ENONPHYSICAL;
  }
  return DG_OK;
}

}  // extern "C"
