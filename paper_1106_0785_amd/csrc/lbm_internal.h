// Library-internal helpers shared by the single-problem, batched and adjoint
// entry points (not part of the C ABI).
#pragma once

#include <hip/hip_runtime.h>

#include "../../include/lbm.h"
#include "lbm_kernels.h"
#include "lbm_multistep.h"
#include "lbm_fused2.h"

namespace lbm {

lbm_status fail(lbm_status s, const char* fmt, ...);
lbm_status hip_fail(hipError_t e, const char* what);
void clear_error();
long long row_pitch(int nx);
lbm_status validate(const lbm_params* p);
// Coefficients of one problem as stored in device memory.
struct Consts {
  Hot hot;
  Cold cold;
};

size_t consts_bytes();
void make_coef(const lbm_params* p, Hot* c, Cold* cold);
// Tile shape of the fused step kernel: rows per tile and wavefronts per
// workgroup (2 or 4; problems with NEQ walls always use 4).
struct TileShape {
  int rows;
  int waves;
  int nt = 1;  // 1: non-temporal stores; 0: ordinary stores
};
MarchGeom march_geom(int nx, int ny, TileShape t);
bool has_walls(const lbm_params* p);
hipError_t launch_step(const Field& F, const Hot* c, const Cold* cold, int version, bool walls, int scheme,
                       int variant, TileShape t, int* flag, hipStream_t s);
TileShape default_tile(int nx, int ny);
// Two steps per launch (lbm_fused2.h): scheme 0 without NEQ walls.
bool two_step_problem(const lbm_params* p);
March2Geom march2_geom(int nx, int ny, TileShape t);
hipError_t launch_step2(const Field& F, const Hot* c, const Cold* cold, int version, TileShape t, int* flag,
                        hipStream_t s);
TileShape default_tile2(int nx, int ny);
int default_variant(const lbm_params* p);
// Small-grid and windowed kernels (lbm_multistep.h) and their selection
// rules, as lbm_create applies them.
bool small_problem(const lbm_params* p);
bool narrow_problem(const lbm_params* p);
WinGeom default_window(const lbm_params* p);
hipError_t launch_small(const Field& F, const Hot* c, const Cold* cold, int version, bool walls, int nsteps,
                        int* flag, hipStream_t s);
hipError_t launch_window(const Field& F, const Hot* c, const Cold* cold, int version, bool walls,
                         const WinGeom& g, int nsteps, int* flag, hipStream_t s);

}  // namespace lbm
