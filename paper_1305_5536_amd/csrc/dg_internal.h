// Internal declarations shared by the host side of the library and its kernel
// launchers.  Not part of the public ABI (that is include/dg.h).
#pragma once

#include <hip/hip_runtime.h>

#include <cstdint>
#include <string>
#include <vector>

#include "dg.h"

namespace dg {

// Kernel modes of a fused stage.
enum StageMode : int {
  kRhs = 0,     // out = L(in)
  kStage1 = 1,  // out = Pi(in) + dt L(Pi(in))
  kStage2 = 2,  // out = Pi(u0)/2 + (Pi(in) + dt L(Pi(in)))/2
  kLimit = 3,   // out = Pi(in)
  kMH = 4,      // out = Pi(in) + dt L_MH(Pi(in); dt/2): one MUSCL-Hancock step
  kStep = 5     // out = one SSP-RK2 step of in (both stages in one pass)
};

// Geometry and launch shape of a periodic 2D Cartesian mesh.
struct Cart2D {
  int nx, ny;
  double hx, hy;
  double lo[2], hi[2];  // the box as given at create
  int rows_per_tile;  // rows marched by one wave
  int tiles_x, tiles_y;
  // the fused SSP-RK2 step (2D Euler): 56 output columns per wave
  int step_rows, step_tiles_x, step_tiles_y;
};

struct Cart3D {
  int nx, ny, nz;
  double hx, hy, hz;
  int planes_per_tile;  // z-planes marched by one wave
  int tiles_x, tiles_y, tiles_z;
};

// Face-list mesh bookkeeping kept on the host side of the handle; the device
// arrays live in FLDev (facelist2d.hip).
struct FaceList2D {
  int nblocks;
};
struct FLDev;
struct MVDev;  // moving Voronoi mesh (moving2d.hip)

// One 2D Cartesian instance of the adjoint kernel: a mesh of nx x ny cells
// starting at cell `off` of the global state arrays, whose adjoint tiles
// (kAdjCols columns x `rows` rows, one wave each) start at tile `tx0` of the
// tile list.
constexpr int kAdjCols = 58;
constexpr int kAdjRowsMin = 16;
constexpr int kAdjRowsMax = 64;
constexpr int kAdjWaves = 2048;
struct AdjInst {
  int nx, ny, off, tx0;
  int tiles_x, tiles_y, rows, pad;
  double hx, hy;
};

// Host copy of a batch of 2D Cartesian instances (mesh kind 2).
struct BatchDesc {
  int ninst = 0;
  std::vector<int> nx, ny;
  std::vector<double> hx, hy;
  std::vector<int64_t> off;  // first cell of each instance, plus the total
};

// Device tables and launch shape of a batch.
struct Batch {
  BatchDesc d;
  int ninst = 0;
  int rows = 16;          // rows per forward tile (all instances)
  int ntiles = 0;         // forward tiles at the current rows
  int wpb = 4;            // waves per workgroup of the batched stage kernel
  int grid_waves = 0;     // > 0: persistent launch of this many waves
  void* inst = nullptr;   // device instance records (BInst<T>[ninst])
  int* tile_inst = nullptr;   // device, forward tile -> instance
  int* inst_tile0 = nullptr;  // device, first forward tile of each instance (+ total)
  int* adj_tile_inst = nullptr;  // device, adjoint tile -> instance
};

// Cached hipGraph of a dg_run launch sequence and the arguments it was
// captured with.
struct RunGraph {
  hipGraph_t graph = nullptr;
  hipGraphExec_t exec = nullptr;
  std::vector<const void*> key;
  uint64_t last_use = 0;
};
constexpr int kMaxRunGraphs = 32;

}  // namespace dg

struct dg_batch {
  dg_mesh* mesh = nullptr;  // a batch mesh (kind 2) built from the instances
};

struct dg_mesh {
  dg_config cfg;
  int dim = 2;
  int kind = 0;
  int ncoef = 0;
  int64_t ncells = 0;
  dg::Cart2D c2{};
  dg::Cart3D c3{};
  dg::FaceList2D fl{};
  dg::FLDev* fld = nullptr;
  dg::MVDev* mvd = nullptr;   // kind 3
  size_t elem = 8;            // sizeof(element)
  void* v1 = nullptr;         // workspace: stage-1 output
  void* tmp = nullptr;        // workspace: staging for in-place steps (lazy)
  void* ws_a = nullptr;       // 3D: Pi(U) of stage 1 (reused by stage 2)
  void* ws_b = nullptr;       // 3D: Pi(V1)
  bool ws_a_fresh = false;    // ws_a holds Pi(ws_a_src) from the preceding stage 1
  const void* ws_a_src = nullptr;
  int* status = nullptr;      // device status word
  double* dtpart = nullptr;   // per-wave partial minima for dg_cfl_dt
  int ndtpart = 0;
  int device = 0;
  dg::AdjInst* adj_inst = nullptr;  // device copy (2D Cartesian meshes)
  int adj_tiles = 0;
  void* adj_ws1 = nullptr;          // adjoint workspaces (lazy)
  void* adj_ws2 = nullptr;
  dg::Batch bt;                     // kind 2
  void* run_ws = nullptr;           // dg_run: second ping-pong buffer (lazy)
  hipStream_t cap_stream = nullptr; // dg_run: capture stream (lazy)
  std::vector<dg::RunGraph> runs;  // dg_run graph cache (least recently used evicted)
  uint64_t run_clock = 0;
};

namespace dg {

void set_error(const std::string& msg);
dg_status hip_fail(hipError_t e, const char* what);

// Launchers (return hipSuccess or the launch error).
// Step size: *dt_dev when dt_dev is not NULL, else dt_host.  Stage 2 with
// dt_next != NULL also writes *dt_next = cfl * min CFL bound of its output.
hipError_t launch_cart2d(const dg_mesh* m, int mode, const void* in, const void* u0, void* out,
                         const double* dt_dev, double dt_host, double cfl, double* dt_next,
                         hipStream_t s);
// dg_cfl_dt_static: partial minima in a static device array of this many
// doubles per GPU (4 MiB); the stand-alone CFL kernel writes four per 256 cells.
constexpr int64_t kCflScratchParts = (int64_t)1 << 19;
hipError_t cart2d_scratch_init();  // once per device, with that device current
hipError_t launch_cart2d_cfl_static(const dg_mesh* m, const void* U, double cfl, double* dt_dev,
                                    hipStream_t s);
hipError_t launch_cart2d_cfl(const dg_mesh* m, const void* U, double cfl, double* dt_dev,
                             hipStream_t s);
hipError_t launch_cart2d_batch(const dg_mesh* m, int mode, const void* in, const void* u0,
                               void* out, const double* dt_dev, double dt_host, double cfl,
                               double* dt_next, hipStream_t s);
hipError_t launch_cart2d_batch_cfl(const dg_mesh* m, const void* U, double cfl, double* dt_dev,
                                   hipStream_t s);
size_t batch_record_size(bool f64);
int batch_tables(const BatchDesc& d, bool f64, int rows, void* records,
                 std::vector<int>& tile_inst, std::vector<int>& tile0);
hipError_t launch_adjoint2d(const void* inst, const int* tile_inst, int ntiles, int nc,
                            int64_t total, bool f64, bool lim, double gamma, const void* U,
                            const void* V1, const double* dt_dev, double dt_host,
                            const void* lam_np1, void* lam_n, void* ws1, void* ws2,
                            hipStream_t s);

}  // namespace dg
