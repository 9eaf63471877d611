/*
 * dg.h - C ABI of the MI355X (gfx950) library for the second-order
 * centroidal-Taylor discontinuous Galerkin scheme of Mocz et al. (2013),
 * "A discontinuous Galerkin method for solving the fluid and MHD equations in
 * astrophysical simulations".
 *
 * The library computes, on the GPU, the per-stage DG right-hand side of the
 * weak form (Sec. 2.2, eqn:dg, eqn:fv, eqn:dgderiv, eqn:fv3d, eqn:dgderiv3d,
 * eqn:GalerkUpdate): P1 Taylor coefficients evaluated at face Gauss points,
 * the face Riemann problem (HLL for Euler, HLLD for ideal MHD; Sec. 2.3),
 * surface-flux accumulation, volume quadrature of F . grad(basis), the inverse
 * mass matrices, the slope limiter of Sec. 2.5, and SSP-RK2 stages.
 *
 * Conventions shared by every entry point
 * ---------------------------------------
 * State layout.  Coefficient-major structure of arrays: element
 *   U[k * ncells + cell]
 * Hydro variable v (rho, rho v_x, rho v_y[, rho v_z], E) owns coefficients
 * k = v*(1+dim) + c, c = 0 the cell mean, c = 1..dim the gradient along x, y(,
 * z) about the cell centroid (the Taylor basis of Sec. 2.2).  Ideal MHD (3D)
 * appends the three B means and the coefficients a4..a11 of the locally
 * divergence-free functions V4..V11 of Sec. 2.2 (31 arrays in all).  Ideal
 * MHD in 2D carries three momenta (rho v_z too) as Taylor variables
 * (k = 3v + c, v = 0..4), then the means of Bx, By, Bz (15..17), the
 * coefficients a1, a2, a3 of the 2D divergence-free functions (x-y field)
 * V3 = (y, 0), V4 = (0, x), V5 = (x, -y) (18..20) and the x and y gradients of
 * Bz (21, 22): 23 arrays in all.
 * Cartesian cells are numbered x fastest: cell = (k*ny + j)*nx + i.
 * Element type is double (DG_FP64) or float (DG_FP32), per dg_config.
 *
 * Batches (mesh kind 2).  A handle can hold many independent periodic 2D
 * Cartesian Euler instances of uneven sizes, stored one after another in the
 * same coefficient-major arrays: instance i owns cells [off_i, off_i+1) of
 *   U[k * ncells + cell],  ncells = sum_i nx_i ny_i
 * (dg_instance_offsets).  Every entry point works on a batch; each instance
 * has its own step size, so a device step-size argument (dt_dev, dt_next_dev)
 * points to ninst doubles, one per instance, and a host dt applies to all.
 *
 * Ownership.  State, derivative and adjoint buffers are DEVICE pointers owned
 * by the caller (at least 16-byte aligned, contiguous, dg_state_len elements).
 * The library owns the mesh handle, its device geometry and its workspace
 * (allocated in dg_mesh_create, freed in dg_mesh_destroy).  Host arrays passed
 * in a descriptor are copied during dg_mesh_create and not retained.
 *
 * Streams.  `stream` is a hipStream_t (NULL = the null stream).  Every compute
 * call only enqueues work and returns without synchronising.
 *
 * Errors.  Functions return dg_status; nothing is thrown across the ABI.  On a
 * non-OK status, dg_last_error() returns a thread-local message.  Device-side
 * detection of a non-physical state (rho <= 0, p <= 0 or a non-finite value at
 * any quadrature point) is latched in a per-mesh status word and reported (and
 * cleared) by dg_check().  A handle must not be used from two host threads at
 * once.
 */
#ifndef DG_H
#define DG_H

#include <stdint.h>

#ifdef __cplusplus
extern "C" {
#endif

typedef struct dg_mesh* dg_mesh_t;

typedef enum {
  DG_OK = 0,
  DG_EINVAL = 1,        /* invalid argument, descriptor or size */
  DG_ENOMEM = 2,        /* device or host allocation failed */
  DG_EHIP = 3,          /* a HIP runtime call failed (message in dg_last_error) */
  DG_EUNSUPPORTED = 4,  /* valid but not built: e.g. MHD on a face-list mesh */
  DG_ENONPHYSICAL = 5,  /* latched non-physical state (dg_check only) */
  DG_EMESH = 6          /* latched moving-mesh failure (dg_check only) */
} dg_status;

typedef enum { DG_EULER = 0, DG_MHD = 1 } dg_physics;
typedef enum { DG_FP64 = 0, DG_FP32 = 1 } dg_precision;
typedef enum { DG_FLUX_HLL = 0, DG_FLUX_HLLD = 1, DG_FLUX_EXACT = 2 } dg_flux;
typedef enum { DG_LIMITER_NONE = 0, DG_LIMITER_MINMOD = 1, DG_LIMITER_WENO = 2 } dg_limiter;

/* Physics and numerics of a mesh.  Euler takes DG_FLUX_HLL (HLL with Davis
 * wave speeds) on every mesh kind, or DG_FLUX_EXACT (the exact Riemann solver
 * of the Euler equations, the paper's Euler flux, Sec. 2.3) on a single 2D
 * Cartesian mesh (kind 0; not with dg_adjoint_step).  MHD needs DG_FLUX_HLLD
 * and a 2D or 3D Cartesian mesh (kind 0).  gamma is the adiabatic index of
 * p_gas = (gamma - 1) rho u (Sec. 2.1). */
typedef struct {
  int physics;    /* dg_physics */
  int precision;  /* dg_precision */
  int flux;       /* dg_flux */
  int limiter;    /* dg_limiter: the slope limiters of Sec. 2.5: DG_LIMITER_MINMOD is the
                   * Arepo limiter (alpha = min(1, min_j psi_ij)) on every mesh kind;
                   * DG_LIMITER_WENO, the WENO-type blend of the stencil and DG primitive
                   * slopes, on single 2D Cartesian Euler meshes (not with
                   * dg_adjoint_step) */
  double gamma;
} dg_config;

/* Mesh descriptor.
 * kind 0: periodic Cartesian box [lo, hi] of n[0] x n[1] (x n[2]) cells.
 * kind 1: periodic 2D face list (e.g. a static Voronoi mesh built on the
 *   host).  All arrays are HOST arrays, copied at create:
 *   cell_volume[ncells], cell_centroid[ncells][2],
 *   cell_moments[ncells][3] = (Mxx, Mxy, Myy), the second moments about the
 *     centroid (the mass matrix of Sec. 2.2),
 *   face_cells[nfaces][2] = (L, R) with the unit normal pointing from L to R,
 *   face_area[nfaces] (edge length), face_normal[nfaces][2],
 *   face_centroid[nfaces][2] (edge midpoint, in L's periodic frame),
 *   face_shift[nfaces][2] in {-1, 0, 1}: R's image next to L sits at
 *     centroid[R] + shift * box.
 *   Every cell must have at least one face and be closed: sum over its faces of
 *   A n = 0 (both checked).
 * kind 2: a batch of ninst periodic 2D Cartesian Euler instances (dim = 2):
 *   inst_n[ninst][2] = (nx, ny), inst_box[ninst][4] = (lo_x, lo_y, hi_x, hi_y),
 *   host arrays copied at create.
 * kind 3: a moving periodic 2D Voronoi mesh (Sec. 2.3), 2D Euler only, in the
 *   box [0, box[0]) x [0, box[1]) with ncells >= 64 generators
 *   generators[ncells][2] (inside the box) and their initial Voronoi faces
 *   face_cells[nfaces][2] with face_shift[nfaces][2] (R's generator image next
 *   to L is generators[R] + shift * box), host arrays copied at create; the
 *   other face-list arrays are ignored.  The library builds and owns the mesh:
 *   the generators move with their cell's velocity (mean momentum / mean
 *   density) and dg_step_mh rebuilds the Voronoi mesh every step on the GPU
 *   (geometry, areas, centroids and second moments: the mass matrix of Sec.
 *   2.2 recomputed per step).  At most 16 faces per cell; a cell's neighbours
 *   after a step must lie within two rings of its neighbours before it (any
 *   CFL-limited step); a failure latches DG_EMESH (dg_check).  The mesh must
 *   be fine enough that no two cells share two faces (ncells >= 64).  Every
 *   step reads and rewrites the mesh the handle holds, so the calls on one
 *   moving mesh must be issued in order on one stream (calls that overlap
 *   race). */
typedef struct {
  int dim;
  int kind;
  int64_t n[3];
  double lo[3], hi[3];
  int64_t ncells, nfaces;
  double box[2];
  const double* cell_volume;
  const double* cell_centroid;
  const double* cell_moments;
  const int32_t* face_cells;
  const double* face_area;
  const double* face_normal;
  const double* face_centroid;
  const int8_t* face_shift;
  int32_t ninst;
  const int32_t* inst_n;
  const double* inst_box;
  const double* generators;
} dg_mesh_desc;

/* Create a mesh handle: validates the descriptor and configuration, uploads
 * the geometry and allocates the workspace.  On failure *out is NULL.  The
 * kernels address coefficient k of cell e as k * ncells + e in 32 bits, so
 * meshes with ncells * ncoef >= 2^31 (e.g. a 3D MHD box above ~69M cells) and
 * face lists with 12 ncells >= 2^31 or 20 nfaces >= 2^31 return DG_EINVAL
 * before any allocation. */
dg_status dg_mesh_create(const dg_mesh_desc* desc, const dg_config* cfg, dg_mesh_t* out);

/* Release the handle and its device memory (synchronises the device).
 * NULL is ignored. */
void dg_mesh_destroy(dg_mesh_t mesh);

/* Number of state elements (ncoef * ncells), or -1 for a NULL handle. */
int64_t dg_state_len(dg_mesh_t mesh);

/* Number of coefficient arrays per cell (12 for 2D Euler, 23 for 2D MHD, 31
 * for 3D MHD). */
int dg_ncoef(dg_mesh_t mesh);

/* dUdt = L(U): the semi-discrete DG right-hand side (Sec. 2.2) without the
 * limiter: face Gauss-point states, Riemann fluxes, surface and volume
 * terms, inverse mass matrices.  U and dUdt must not alias. */
dg_status dg_rhs(dg_mesh_t mesh, const void* U, void* dUdt, void* stream);

/* U_lim = Pi(U): the slope limiter of Sec. 2.5, alpha = min(1, min_j psi_ij)
 * per conserved variable from the means of the cell and its face neighbours
 * and the linear extrapolation to each face centroid; means are unchanged;
 * the three B components share one alpha.  U and U_lim must not alias.
 * With DG_LIMITER_WENO (2D Euler) the WENO-type limiter of Sec. 2.5 instead
 * blends, per primitive variable, the stencil slope (limited as above) and the
 * cell's own DG slope with weights (eps + o)^(-1/2).  On a moving mesh the
 * limiter acts on the handle's current mesh; the stencil slope is the
 * least-squares fit to the face neighbours' primitive means. */
dg_status dg_limit(dg_mesh_t mesh, const void* U, void* U_lim, void* stream);

/* One SSP-RK2 step of size dt with the limiter (if configured) at the start of
 * each stage:
 *   Ua = Pi(U); V1 = Ua + dt L(Ua); Ub = Pi(V1); U_next = Ua/2 + (Ub + dt L(Ub))/2.
 * U_next is stored unlimited; the next step limits it first.  U_next may
 * equal U (the library then stages the result in its workspace and copies it
 * back: one extra state copy).  2D Euler on a Cartesian mesh with HLL and the
 * limiter off or DG_LIMITER_MINMOD runs both stages in one kernel (V1 never
 * reaches device memory; the result equals the two-stage sequence below);
 * other meshes run dg_stage1 and dg_stage2. */
dg_status dg_step(dg_mesh_t mesh, const void* U, void* U_next, double dt, void* stream);

/* The two stages of dg_step as separate launches:
 *   dg_stage1: V1 = Pi(U) + dt L(Pi(U))                          (one kernel)
 *   dg_stage2: U_next = Pi(U)/2 + (Pi(V1) + dt L(Pi(V1)))/2      (one kernel)
 * The step size is *dt_dev when dt_dev is not NULL (a device double), else dt.
 * When dt_next_dev is not NULL, dg_stage2 also writes
 *   *dt_next_dev = cfl * min_e (CFL bound of U_next's cell means)
 * (the formula of dg_cfl_dt), from per-wave minima taken inside the stage
 * kernel plus one single-workgroup reduction; it may equal dt_dev.
 * V1 must not alias U; U_next must alias neither U nor V1.
 * On MHD and face-list meshes the limiter runs as its own pass: dg_stage1
 * keeps Pi(U) in the handle's workspace, and a dg_stage2 that immediately
 * follows it on the same handle with the same U pointer reuses that copy (U
 * must not be modified in between); any other dg_stage2 limits U again. */
dg_status dg_stage1(dg_mesh_t mesh, const void* U, void* V1, double dt, const double* dt_dev,
                    void* stream);
dg_status dg_stage2(dg_mesh_t mesh, const void* U, const void* V1, void* U_next, double dt,
                    const double* dt_dev, double cfl, double* dt_next_dev, void* stream);

/* Same as dg_step with the step size read from device memory (*dt_dev, a
 * double), so a step can follow dg_cfl_dt without a host synchronisation. */
dg_status dg_step_devdt(dg_mesh_t mesh, const void* U, void* U_next, const double* dt_dev,
                        void* stream);

/* dg_step_devdt that also writes the CFL step of U_next, when dt_next_dev is
 * not NULL: *dt_next_dev = cfl * min_e (CFL bound of U_next's cell means), the
 * formula of dg_cfl_dt, from per-wave minima taken inside the step kernel plus
 * one single-workgroup reduction (it may equal dt_dev).  A stepping loop with
 * no host synchronisation: dg_cfl_dt once, then dg_step_cfl per step.
 * DG_EINVAL for NULL U, U_next or dt_dev, or cfl <= 0 with dt_next_dev;
 * DG_EUNSUPPORTED on moving meshes (dg_step_mh). */
dg_status dg_step_cfl(dg_mesh_t mesh, const void* U, void* U_next, const double* dt_dev,
                      double cfl, double* dt_next_dev, void* stream);

/* One MUSCL-Hancock step, the paper's own integrator (Sec. 2.4):
 *   Ua = Pi(U);  U_next = Ua + dt L_MH(Ua; dt/2),
 * where L_MH has the surface and volume terms of dg_rhs (eqn:GalerkUpdate)
 * but takes every face Gauss-point and volume-point state from the cell's
 * half-step prediction: primitive values (rho, v, p) and gradients at the
 * centroid from the conserved mean and gradients (chain rule), advanced by
 * dt/2 with the quasi-linear Euler time derivatives, extrapolated linearly
 * and converted back to conserved variables.  One kernel per step (half the
 * flux passes of the SSP-RK2 step).  Step size: *dt_dev (one per instance on
 * a batch) when dt_dev is not NULL, else dt.  When dt_next_dev is not NULL,
 * also writes the CFL step of U_next (as dg_stage2).  U_next must not alias
 * U.  Built for 2D Euler on Cartesian meshes, batches and moving meshes
 * (DG_EUNSUPPORTED otherwise).
 * On a moving mesh (kind 3) the step also moves the mesh held by the handle
 * from t^n to t^{n+1}, so U must be the state on the handle's current mesh and
 * U_next is the state on the new one.  The step (Sec. 2.3, Sec. 2.4): limit U
 * on the mesh of t^n; move the generators with constant velocity w_e (their
 * cell's mean velocity, or 0 after dg_set_mesh_motion(mesh, 0)); take every
 * flux on the Voronoi mesh of the half-step generators, with both cells'
 * half-step predictions (centred at the t^n centroids) at each face Gauss
 * point, the Riemann problem (HLL or exact, per dg_config.flux) solved in the
 * frame of the face at that point (the velocity of the bisector there) and
 * carried back to the lab frame, F_m = F - U w^T, and the volume flux
 * F - U w_e^T on the half-step cell; the conserved totals V ubar and the first
 * moments (about the cell's origin carried with w_e) are advanced by dt, and
 * the new state is read off the mesh of t^{n+1}: ubar = totals / V, gradients
 * from the new mass matrix after moving the moments to the new centroid.
 * CFL (dt_next_dev, dg_cfl_dt): cfl * min_e 2 V_e / sum_f A_f
 * (|(v_e - w_e) . n_f| + c_e). */
dg_status dg_step_mh(dg_mesh_t mesh, const void* U, void* U_next, double dt, const double* dt_dev,
                     double cfl, double* dt_next_dev, void* stream);

/* Discrete adjoint of dg_step (vector-Jacobian product), dt frozen:
 *   lam_n = (d step(U, dt) / d U)^T lam_np1
 * through both stages, both limiter applications (the branch the forward step
 * takes: alpha = 1, or alpha = D/dm with its arg-max/arg-min neighbour) and
 * the face flux (HLL: the active wave-speed estimates; HLLD: the active region
 * of the fan).  Ties follow the first
 * argument in the order self, -x, +x, -y, +y.  The step size is *dt_dev (one
 * per instance on a batch) when dt_dev is not NULL, else dt.  V1 is the
 * stage-1 output of the forward step from U (dg_stage1 with the same step
 * size), or NULL to recompute it.  Built for 2D Euler on Cartesian meshes,
 * batches and static face-list meshes (HLL; limiter off or DG_LIMITER_MINMOD;
 * on a face list the bounds and alpha run over the cell's faces in the mesh's
 * incidence order) and for 2D and 3D ideal MHD on Cartesian meshes (HLLD on
 * the face-averaged normal field, the divergence-free field bases of Sec. 2.2;
 * limiter off or DG_LIMITER_MINMOD with one alpha for B, ties in the same
 * order, then -z, +z); DG_EUNSUPPORTED otherwise (the exact Riemann solver,
 * the WENO-type limiter, moving meshes).  lam_n must
 * not alias U, V1 or lam_np1.  Allocates two state-sized workspaces on the
 * first call (kept by the handle). */
dg_status dg_adjoint_step(dg_mesh_t mesh, const void* U, const void* V1, double dt,
                          const double* dt_dev, const void* lam_np1, void* lam_n, void* stream);

/* Flags of dg_run: capture the launch sequence into a hipGraph; step with
 * dg_step_mh (MUSCL-Hancock, one kernel per step) instead of SSP-RK2; step
 * SSP-RK2 with the dg_stage1/dg_stage2 pair even where dg_step has a fused
 * one-kernel step (the results then equal those of the stage calls and of a
 * batch holding the mesh, bit for bit; on small meshes the pair is also the
 * faster path). */
#define DG_RUN_GRAPH 1
#define DG_RUN_MUSCL_HANCOCK 2
#define DG_RUN_TWO_STAGE 4

/* nsteps SSP-RK2 steps (dg_step's kernels: the fused step, or the
 * dg_stage1/dg_stage2 pair when v1_keep asks for the stage-1 outputs or
 * flags has DG_RUN_TWO_STAGE) from U_in
 * to U_out, with per-step (per-instance) step sizes in the device array
 * dt_hist, nd = dg_ninst doubles per step:
 *   cfl > 0: adaptive.  dt_hist[0..nd) = the CFL step of U_in (dg_cfl_dt) and
 *            step n's stage 2 writes step n+1's into dt_hist[(n+1) nd ...],
 *            so dt_hist holds (nsteps + 1) nd doubles, the history of the run.
 *   cfl = 0: dt_hist[n nd ...] is read as the step size of step n.
 * ckpt_every > 0: ckpt is a HOST array of floor((nsteps - 1) / ckpt_every)
 *   state-sized DEVICE buffers; ckpt[j] receives the state after step
 *   (j + 1) ckpt_every (written by that step's stage 2, no extra copy).
 * v1_keep: NULL, or a HOST array of nsteps DEVICE buffers that receive each
 *   step's stage-1 output (the V1 of dg_adjoint_step); SSP-RK2 only.
 * U_in is not modified (unless it is U_out); U_out may equal U_in only when
 * nsteps >= 2; U_out, the checkpoints and v1_keep buffers must be distinct.
 * Intermediate states ping-pong through two state-sized workspaces of the
 * handle (allocated on the first call).
 * flags & DG_RUN_GRAPH: the whole sequence is captured once into a hipGraph,
 * cached on the handle for these arguments (pointer values included; up to 32
 * argument sets, least recently used evicted), and replayed with one graph
 * launch; the capture uses no memset or allocation.  dg_set_tiling and
 * dg_set_launch drop the cache. */
dg_status dg_run(dg_mesh_t mesh, const void* U_in, void* U_out, int nsteps, double cfl,
                 double* dt_hist, int ckpt_every, void* const* ckpt, void* const* v1_keep,
                 int flags, void* stream);

/* Number of instances (1 for a single mesh), or -1 for a NULL handle. */
int dg_ninst(dg_mesh_t mesh);

/* off[0..ninst] = first cell of each instance and the total cell count
 * (host array of dg_ninst + 1 elements). */
dg_status dg_instance_offsets(dg_mesh_t mesh, int64_t* off);

/* Launch shape of the batched stage kernel: waves per workgroup (1, 2 or 4)
 * and, when grid_waves > 0, a persistent launch of that many waves, each
 * walking the tile list with a stride of grid_waves (0: one wave per tile).
 * Results do not depend on it.  Ignored (DG_OK) for single meshes. */
dg_status dg_set_launch(dg_mesh_t mesh, int waves_per_group, int grid_waves);
dg_status dg_get_launch(dg_mesh_t mesh, int* waves_per_group, int* grid_waves);

/* *dt_dev = cfl * min_e 2 V_e / sum_{f of e} A_f (|v_e . n_f| + c_e(n_f)) from
 * the cell means of U (c the sound speed, or the fast magnetosonic speed along
 * n_f for MHD).  dt_dev is a device pointer to one double. */
dg_status dg_cfl_dt(dg_mesh_t mesh, const void* U, double cfl, double* dt_dev, void* stream);

/* For callers that cannot allocate (code under HIP graph capture, tight
 * serving loops, harnesses that forbid hipMalloc): dg_cfl_dt with its
 * per-wave partial minima in a static device array of 4 MiB per GPU (held
 * until the process ends) instead of the handle's workspace; the call
 * allocates nothing (no hipMalloc, hipFree or allocating library routine).
 * Same result as dg_cfl_dt, bit for bit.  Built for single 2D Cartesian Euler
 * meshes (kind 0; DG_EUNSUPPORTED otherwise) of at most 2^25 cells (DG_EINVAL
 * above).  Every call on one GPU shares that GPU's array: calls that overlap
 * on one GPU (on different streams or from different host threads) race. */
dg_status dg_cfl_dt_static(dg_mesh_t mesh, const void* U, double cfl, double* dt_dev,
                           void* stream);

/* Launch shape of the Cartesian stage kernels: the number of rows (2D, and
 * every instance of a batch) one wave marches through, or of z-planes (3D)
 * one workgroup of four row-waves marches through.  0 restores the library
 * default, which a positive DG_TILE_ROWS (stage kernels, batches) or
 * DG_STEP_ROWS (fused 2D Euler step) environment variable replaces for the
 * whole process.
 * Results do not depend on it (every face and cell is computed with the same
 * arithmetic whatever the tiling); only speed does.  Face-list meshes ignore
 * it.  Returns DG_EINVAL for a negative value. */
dg_status dg_set_tiling(dg_mesh_t mesh, int rows_per_tile);

/* Current rows (or planes) per wave, or -1 for a NULL handle. */
int dg_get_tiling(dg_mesh_t mesh);

/* Synchronise the device, then return DG_EMESH if a moving mesh failed to
 * rebuild a cell (see kind 3), else DG_ENONPHYSICAL if any kernel of this mesh
 * met a non-physical state since the last call (and clear the flags), else
 * DG_OK (or DG_EHIP if synchronisation failed). */
dg_status dg_check(dg_mesh_t mesh);

/* Moving meshes (kind 3): 1 (the default) moves the generators with their
 * cell velocity in dg_step_mh, 0 holds them still (the step is then the static
 * MUSCL-Hancock step on the Voronoi mesh).  DG_EUNSUPPORTED on other kinds. */
dg_status dg_set_mesh_motion(dg_mesh_t mesh, int motion);

/* Moving meshes (kind 3): host copies of the current mesh (synchronises the
 * device).  generators[ncells][2] (in [0, box)), volume[ncells],
 * centroid[ncells][2] (generator + centroid offset, not wrapped),
 * ring[ncells][16] the neighbours in counter-clockwise order padded with -1,
 * degree[ncells].  Any output may be NULL.  DG_EUNSUPPORTED on other kinds. */
dg_status dg_mesh_geometry(dg_mesh_t mesh, double* generators, double* volume, double* centroid,
                           int32_t* ring, int32_t* degree);

/* Moving meshes (kind 3): on != 0 makes every following dg_step_mh record HIP
 * events on its stream around its four kernels (limiter; mesh of the half-step
 * generators; fluxes and update; mesh of t^{n+1} with the new state and the dt
 * reduction); 0 stops and drops the record.  dg_moving_timing synchronises the
 * device and writes the average duration of each of the four, in ms, over the
 * steps timed since the last call into avg_ms[4] (and their count into
 * *nsteps when not NULL), then starts a fresh record.  DG_EUNSUPPORTED on
 * other kinds. */
dg_status dg_set_moving_timing(dg_mesh_t mesh, int on);
dg_status dg_moving_timing(dg_mesh_t mesh, double* avg_ms, int* nsteps);

/* ------------------------------------------------------------ batch handles
 * Many independent periodic 2D Euler simulations of uneven sizes advanced
 * together (the batched stepper).  A dg_batch_t is built from single meshes
 * and owns one batch mesh (kind 2) whose state stores the instances one after
 * another in the coefficient-major arrays (see "Batches" above); every call
 * below forwards to the mesh-handle entry points on it, and dg_batch_mesh
 * exposes that handle for the others (dg_rhs, dg_stage1/2, dg_cfl_dt,
 * dg_check, ...).  Computes what the single meshes compute (Sec. 2.2-2.5),
 * instance by instance, bit for bit. */
typedef struct dg_batch* dg_batch_t;

/* Build a batch from ninst single meshes: each meshes[i] a 2D Cartesian Euler
 * mesh (kind 0), all with the same dg_config; instance i takes meshes[i]'s
 * cells and box.  The meshes are only read (they stay valid and independent).
 * autotune_cache: NULL for the library's default launch shape, or the path of
 * a text file holding three integers "rows waves_per_group grid_waves" (the
 * shape an autotuner chose for this batch: dg_set_tiling and dg_set_launch
 * values).  DG_EUNSUPPORTED for other mesh kinds or physics; DG_EINVAL for
 * mismatched configurations, an unreadable or malformed file, or a batch too
 * large for 32-bit indexing.  On failure *out is NULL. */
dg_status dg_batch_create(const dg_mesh_t* meshes, int ninst, const char* autotune_cache,
                          dg_batch_t* out);

/* The batch mesh handle (kind 2) of b, owned by b; NULL for a NULL batch. */
dg_mesh_t dg_batch_mesh(dg_batch_t b);

/* First cell of instance inst in the batch state (inst = ninst gives the total
 * cell count), or -1 for a NULL batch or an index outside [0, ninst]. */
int64_t dg_batch_offset(dg_batch_t b, int inst);

/* Advance every instance nsteps SSP-RK2 steps in place (U, device, the batch
 * state): the dg_run sequence with DG_RUN_GRAPH (captured once per argument
 * set into a hipGraph and replayed).  cfl > 0: adaptive per-instance steps,
 * dt_hist_dev receives (nsteps + 1) * ninst doubles (the step history, as in
 * dg_run); cfl = 0: dt_hist_dev holds nsteps * ninst given step sizes.  One
 * step (nsteps = 1) goes through the handle's staging buffer and a device
 * copy. */
dg_status dg_batch_run(dg_batch_t b, void* U, double cfl, double* dt_hist_dev, int nsteps,
                       void* stream);

/* Discrete adjoint of one batch step (dg_adjoint_step with V1 recomputed):
 * lam_n = (d step(U_n) / d U_n)^T lam_np1 with the per-instance step sizes
 * dt_dev[ninst] (device).  Same semantics, aliasing rules and workspaces as
 * dg_adjoint_step. */
dg_status dg_batch_adjoint_step(dg_batch_t b, const void* U_n, const double* dt_dev,
                                const void* lam_np1, void* lam_n, void* stream);

/* Release the batch and its batch mesh (synchronises the device).  NULL is
 * ignored. */
void dg_batch_destroy(dg_batch_t b);

/* Thread-local text for the last non-OK status returned on this thread. */
const char* dg_last_error(void);

#ifdef __cplusplus
}
#endif

#endif /* DG_H */
