// C ABI of the single-problem path (declarations and contracts in include/lbm.h).
#include <climits>
#include <hip/hip_runtime.h>

#include <algorithm>
#include <cmath>
#include <cstdarg>
#include <cstdio>
#include <cstring>
#include <string>

#include "../../include/lbm.h"
#include "lbm_internal.h"
#include "lbm_multistep.h"

using namespace lbm;

namespace {
thread_local std::string g_err;
}

namespace lbm {

lbm_status fail(lbm_status s, const char* fmt, ...) {
  char buf[512];
  va_list ap;
  va_start(ap, fmt);
  vsnprintf(buf, sizeof(buf), fmt, ap);
  va_end(ap);
  g_err = buf;
  return s;
}

lbm_status hip_fail(hipError_t e, const char* what) {
  (void)hipGetLastError();  // reset HIP's sticky last error so later launch checks do not see it
  return fail(LBM_EHIP, "%s: %s", what, hipGetErrorString(e));
}

void clear_error() { g_err.clear(); }

long long row_pitch(int nx) { return ((long long)nx + 63) / 64 * 64; }

bool has_walls(const lbm_params* p) {
  for (int k = 0; k < 4; ++k)
    if (p->bc[k] == LBM_BC_NEQ_WALL) return true;
  return false;
}

size_t consts_bytes() { return (sizeof(Consts) + 255) / 256 * 256; }

lbm_status validate(const lbm_params* p) {
  if (!p) return fail(LBM_EINVAL, "params is NULL");
  if (p->nx < 1 || p->ny < 1) return fail(LBM_EINVAL, "nx and ny must be >= 1 (got %d x %d)", p->nx, p->ny);
  if ((long long)p->nx * p->ny > (1LL << 31)) return fail(LBM_EINVAL, "grid too large");
  if (!(p->dx > 0) || !(p->dy > 0) || !(p->dt > 0)) return fail(LBM_EINVAL, "dx, dy, dt must be > 0");
  double smax = 0;
  for (int k = 4; k < 16; ++k) {
    if (!(p->s[k] > 0)) return fail(LBM_EINVAL, "s_%d must be > 0", k + 1);
    smax = std::max(smax, p->s[k]);
  }
  if (smax * p->dt > 2.0)
    return fail(LBM_EINVAL, "max_k s_k dt = %g > 2: the explicit relaxation is unstable", smax * p->dt);
  if (p->eq_version < 1 || p->eq_version > 3) return fail(LBM_EINVAL, "eq_version must be 1, 2 or 3");
  if (p->modified < 0 || p->modified > 2) return fail(LBM_EINVAL, "modified must be 0, 1 or 2");
  if (p->scheme < 0 || p->scheme > 1) return fail(LBM_EINVAL, "scheme must be 0 or 1");
  for (int k = 0; k < 4; ++k)
    if (p->bc[k] < 0 || p->bc[k] > 4) return fail(LBM_EINVAL, "bc[%d] = %d is not a boundary kind", k, p->bc[k]);
  for (int a = 0; a < 2; ++a)
    if ((p->bc[2 * a] == LBM_BC_PERIODIC) != (p->bc[2 * a + 1] == LBM_BC_PERIODIC))
      return fail(LBM_EINVAL, "periodic boundaries must be paired on an axis");
  const bool xw = p->bc[0] == LBM_BC_NEQ_WALL || p->bc[1] == LBM_BC_NEQ_WALL;
  const bool yw = p->bc[2] == LBM_BC_NEQ_WALL || p->bc[3] == LBM_BC_NEQ_WALL;
  if (xw && yw) return fail(LBM_EINVAL, "NEQ walls on both axes are not supported");
  if ((xw || yw) && p->scheme == 1) return fail(LBM_EINVAL, "NEQ walls are not supported with scheme 1");
  if (xw && p->nx < 3) return fail(LBM_EINVAL, "NEQ walls on x need nx >= 3");
  if (yw && p->ny < 3) return fail(LBM_EINVAL, "NEQ walls on y need ny >= 3");
  if (p->nx == 1 && p->bc[0] != LBM_BC_PERIODIC) return fail(LBM_EINVAL, "an axis of extent 1 must be periodic");
  if (p->ny == 1 && p->bc[2] != LBM_BC_PERIODIC) return fail(LBM_EINVAL, "an axis of extent 1 must be periodic");
  for (int sd = 0; sd < 4; ++sd) {
    if (p->bc[sd] == LBM_BC_DIRICHLET_EQ && (!(p->wall[sd][0] > 0) || !(p->wall[sd][3] > 0)))
      return fail(LBM_EINVAL, "fixed-state side %d needs rho > 0 and T > 0", sd);
    if (p->bc[sd] == LBM_BC_NEQ_WALL && !(p->wall[sd][3] > 0))
      return fail(LBM_EINVAL, "wall side %d needs T > 0", sd);
  }
  return LBM_OK;
}

void make_coef(const lbm_params* p, Hot* c, Cold* cold) {
  std::memset(c, 0, sizeof(*c));
  std::memset(cold, 0, sizeof(*cold));
  const double dt = p->dt;
  for (int k = 4; k < 16; ++k) c->cq[k - 4] = -dt * p->s[k];
  if (p->modified) {
    const double s5 = p->s[4], s6 = p->s[5], s7 = p->s[6], s8 = p->s[7];
    const double sgn = (p->modified == 2) ? 1.0 : -1.0;
    c->cmod[0] = -dt * (s7 / s5 - 1.0);
    c->cmod[1] = -dt * (s7 / s6 - 1.0);
    c->cmod[2] = -dt * (s8 / s6 - 1.0);
    c->cmod[3] = -dt * sgn * (s8 / s5 - 1.0);
  }
  c->inv2dx = 1.0 / (2.0 * p->dx);
  c->inv2dy = 1.0 / (2.0 * p->dy);
  const double rx = dt / p->dx, ry = dt / p->dy;
  for (int v = 1; v <= 2; ++v) {
    const double cx = v * rx, cy = v * ry;
    c->lx[2 * (v - 1)] = 0.5 * cx * cx - 0.5 * cx;
    c->lx[2 * (v - 1) + 1] = 0.5 * cx * cx + 0.5 * cx;
    c->ly[2 * (v - 1)] = 0.5 * cy * cy - 0.5 * cy;
    c->ly[2 * (v - 1) + 1] = 0.5 * cy * cy + 0.5 * cy;
    c->tx[2 * (v - 1)] = cx;
    c->tx[2 * (v - 1) + 1] = 0.5 * cx * (1.0 - cx);
    c->ty[2 * (v - 1)] = cy;
    c->ty[2 * (v - 1) + 1] = 0.5 * cy * (1.0 - cy);
  }
  for (int sd = 0; sd < 4; ++sd) {
    for (int j = 0; j < 4; ++j) cold->wall[sd][j] = p->wall[sd][j];
    if (p->bc[sd] == LBM_BC_DIRICHLET_EQ)
      equilibrium_f(p->eq_version, p->wall[sd][0], p->wall[sd][1], p->wall[sd][2], p->wall[sd][3], cold->ghost[sd]);
    c->bc[sd] = p->bc[sd];
  }
  c->version = p->eq_version;
  c->modified = p->modified;
  c->scheme = p->scheme;
}

MarchGeom march_geom(int nx, int ny, TileShape t) {
  MarchGeom g;
  const int w = t.waves;
  g.nstrips = (nx + STRIP - 1) / STRIP;
  int rows = std::max(w, std::min(t.rows, (ny + w - 1) / w * w));
  g.rows = (rows + w - 1) / w * w;
  g.nsegs = (ny + g.rows - 1) / g.rows;
  g.ntiles = g.nstrips * g.nsegs;
  g.per_xcd = (g.ntiles + 7) / 8;
  return g;
}

hipError_t launch_step(const Field& F, const Hot* c, const Cold* cold, int version, bool walls, int scheme,
                       int variant, TileShape t, int* flag, hipStream_t s) {
  if (variant == 1) {
    dim3 block(64, 4);
    dim3 grid((F.nx + 63) / 64, (F.ny + 3) / 4);
    auto k = version == 2 ? k_step_plain<2> : version == 3 ? k_step_plain<3> : k_step_plain<1>;
    hipLaunchKernelGGL(k, grid, block, 0, s, F, c, cold, flag);
    return hipGetLastError();
  }
  // NEQ walls and the flux-limited scheme use 4-wave tiles
  if (walls || scheme == 1 || t.waves != 2) t.waves = 4;
  const MarchGeom g = march_geom(F.nx, F.ny, t);
  decltype(&k_step_fused<1, false, 4, 1, true>) k;
#define LBM_FUSED(WALLS, W, HR)                                                                            \
  k = t.nt ? (version == 2 ? k_step_fused<2, WALLS, W, HR, true>                                          \
                           : version == 3 ? k_step_fused<3, WALLS, W, HR, true> : k_step_fused<1, WALLS, W, HR, true>) \
           : (version == 2 ? k_step_fused<2, WALLS, W, HR, false>                                         \
                           : version == 3 ? k_step_fused<3, WALLS, W, HR, false> : k_step_fused<1, WALLS, W, HR, false>)
  if (walls)
    LBM_FUSED(true, 4, 1);
  else if (scheme == 1)
    LBM_FUSED(false, 4, 2);
  else if (t.waves == 2)
    LBM_FUSED(false, 2, 1);
  else
    LBM_FUSED(false, 4, 1);
#undef LBM_FUSED
  hipLaunchKernelGGL(k, dim3(8 * g.per_xcd), dim3(64 * t.waves), 0, s, F, c, cold, g, flag);
  return hipGetLastError();
}

bool two_step_problem(const lbm_params* p) { return p->scheme == 0 && !has_walls(p); }

March2Geom march2_geom(int nx, int ny, TileShape t) {
  March2Geom g;
  const int w = t.waves;
  g.nstrips = (nx + OSTRIP - 1) / OSTRIP;
  int rows = std::max(w, std::min(t.rows, (ny + w - 1) / w * w));
  g.rows = (rows + w - 1) / w * w;
  g.nsegs = (ny + g.rows - 1) / g.rows;
  g.ntiles = g.nstrips * g.nsegs;
  g.per_xcd = (g.ntiles + 7) / 8;
  return g;
}

hipError_t launch_step2(const Field& F, const Hot* c, const Cold* cold, int version, TileShape t, int* flag,
                        hipStream_t s) {
  if (t.waves != 2) t.waves = 4;
  const March2Geom g = march2_geom(F.nx, F.ny, t);
  decltype(&k_step_fused2<1, 4, true>) k;
#define LBM_FUSED2(W)                                                                                    \
  k = t.nt ? (version == 2 ? k_step_fused2<2, W, true> : version == 3 ? k_step_fused2<3, W, true>        \
                                                                      : k_step_fused2<1, W, true>)        \
           : (version == 2 ? k_step_fused2<2, W, false> : version == 3 ? k_step_fused2<3, W, false>      \
                                                                       : k_step_fused2<1, W, false>)
  if (t.waves == 2)
    LBM_FUSED2(2);
  else
    LBM_FUSED2(4);
#undef LBM_FUSED2
  hipLaunchKernelGGL(k, dim3(8 * g.per_xcd), dim3(64 * t.waves), 0, s, F, c, cold, g, flag);
  return hipGetLastError();
}

TileShape default_tile2(int nx, int ny) {
  // two waves per workgroup (two workgroups per CU), and tiles tall enough
  // to leave just under two per workgroup slot (512 slots): the tuner's
  // pick at 4096 x 1024 (70-row tiles, 164 us per step against 178 for
  // 16-row tiles); heights rounded up to even
  const long long strips = (nx + OSTRIP - 1) / OSTRIP;
  const long long segs = std::max(1ll, 1024 / strips);
  int rows = (int)std::min<long long>(1024, (ny + segs - 1) / segs);
  rows = std::max(2, (rows + 1) / 2 * 2);
  const long long bytes = (long long)nx * ny * 256;
  const int nt = (bytes > (32ll << 20) && bytes <= (512ll << 20)) ? 0 : 1;
  return TileShape{rows, 2, nt};
}

// Default kernel of a problem: the whole grid in one workgroup when it fits,
// windows for narrow grids, two steps per launch where both distribution
// buffers exceed the 256 MB last-level cache (the step is then bound by HBM,
// and the two-step kernel halves its traffic), else the one-step kernel.
int default_variant(const lbm_params* p) {
  if (small_problem(p)) return 2;
  if (narrow_problem(p)) return 3;
  const long long bytes = (long long)p->nx * p->ny * 256;
  if (two_step_problem(p) && bytes > (512ll << 20)) return 4;
  return 0;
}

// True when the whole grid fits the one-workgroup multi-step kernel.
bool small_problem(const lbm_params* p) {
  return p->scheme == 0 && (long long)p->nx * p->ny <= SMALL_NODES;
}

hipError_t launch_small(const Field& F, const Hot* c, const Cold* cold, int version, bool walls, int nsteps,
                        int* flag, hipStream_t s) {
  decltype(&k_step_small<1, false>) k;
  if (walls)
    k = version == 2 ? k_step_small<2, true> : version == 3 ? k_step_small<3, true> : k_step_small<1, true>;
  else
    k = version == 2 ? k_step_small<2, false> : version == 3 ? k_step_small<3, false> : k_step_small<1, false>;
  const int threads = (F.nx * F.ny + 63) / 64 * 64;
  hipLaunchKernelGGL(k, dim3(1), dim3(threads), 0, s, F, c, cold, nsteps, flag);
  return hipGetLastError();
}

// True when the windowed kernel applies: scheme 0 and too big for the
// small-grid kernel.
bool window_problem(const lbm_params* p) { return p->scheme == 0 && !small_problem(p); }

// True when the windowed kernel is the default: narrow grids (<= 16 rows).
bool narrow_problem(const lbm_params* p) { return window_problem(p) && p->ny <= 16; }

// One axis of the window shape: the whole axis in one window when it fits,
// else windows of w nodes overlapping by `halo` nodes on each cut side and
// writing w - 2 halo each. halo = h, or h + 1 on an axis with NEQ walls (a
// wall node takes its neighbour's value of the same step).
WinAxis win_axis(int len, int w, int h, bool walls) {
  WinAxis a;
  a.halo = h + (walls ? 1 : 0);
  if (len <= w) {
    a.w = len;
    a.v = len;
    a.nwin = 1;
    a.whole = 1;
  } else {
    a.w = w;
    a.v = w - 2 * a.halo;
    a.nwin = a.v >= 1 ? (len + a.v - 1) / a.v : 0;  // v < 1: rejected by make_window
    a.whole = 0;
  }
  return a;
}

// Checks a window shape (wc columns, wr rows, h steps per launch) for
// problem p; fills g when it is valid.
bool make_window(const lbm_params* p, int wc, int wr, int h, WinGeom* g) {
  if (h < 1 || wc < 1 || wr < 1) return false;
  const bool xw = p->bc[0] == LBM_BC_NEQ_WALL || p->bc[1] == LBM_BC_NEQ_WALL;
  const bool yw = p->bc[2] == LBM_BC_NEQ_WALL || p->bc[3] == LBM_BC_NEQ_WALL;
  const WinAxis x = win_axis(p->nx, wc, h, xw), y = win_axis(p->ny, wr, h, yw);
  if (x.v < 1 || y.v < 1) return false;
  if ((long long)x.w * y.w > SMALL_NODES) return false;
  g->x = x;
  g->y = y;
  g->h = h;
  return true;
}

// Default window shape: narrow grids take every row and 64 columns (32 when
// ny > 8), h = columns / 8; other grids 32 x 16 nodes, h = 2.
WinGeom default_window(const lbm_params* p) {
  WinGeom g{};
  if (p->ny <= 16) {
    const int wc = p->ny <= 8 ? 64 : 32;
    make_window(p, wc, p->ny, wc / 8, &g);
  } else {
    make_window(p, 32, 16, 2, &g);
  }
  return g;
}

hipError_t launch_window(const Field& F, const Hot* c, const Cold* cold, int version, bool walls,
                         const WinGeom& g, int nsteps, int* flag, hipStream_t s) {
  decltype(&k_step_window<1, false, SMALL_NODES>) k;
  const int threads = (g.x.w * g.y.w + 63) / 64 * 64;
  if (threads <= SMALL_NODES / 2) {  // half the LDS: two workgroups per CU
    if (walls)
      k = version == 2 ? k_step_window<2, true, SMALL_NODES / 2>
                       : version == 3 ? k_step_window<3, true, SMALL_NODES / 2> : k_step_window<1, true, SMALL_NODES / 2>;
    else
      k = version == 2 ? k_step_window<2, false, SMALL_NODES / 2>
                       : version == 3 ? k_step_window<3, false, SMALL_NODES / 2>
                                      : k_step_window<1, false, SMALL_NODES / 2>;
  } else if (walls) {
    k = version == 2 ? k_step_window<2, true, SMALL_NODES>
                     : version == 3 ? k_step_window<3, true, SMALL_NODES> : k_step_window<1, true, SMALL_NODES>;
  } else {
    k = version == 2 ? k_step_window<2, false, SMALL_NODES>
                     : version == 3 ? k_step_window<3, false, SMALL_NODES> : k_step_window<1, false, SMALL_NODES>;
  }
  hipLaunchKernelGGL(k, dim3(g.x.nwin * g.y.nwin), dim3(threads), 0, s, F, c, cold, g, nsteps, flag);
  return hipGetLastError();
}

TileShape default_tile(int nx, int ny) {
  // tall tiles amortise the two halo rows; keep at least ~2 workgroups per CU
  const long long strips = (nx + STRIP - 1) / STRIP;
  int rows = 64;
  while (rows > WAVES && strips * ((ny + rows - 1) / rows) < 1024) rows /= 2;
  // ordinary stores while both buffers (256 bytes per node) take between 32
  // and 512 MB (measured per step: faster at 1024 x 256 and 2048 x 512,
  // slower at 512 x 128 and 4096 x 1024)
  const long long bytes = (long long)nx * ny * 256;
  const int nt = (bytes > (32ll << 20) && bytes <= (512ll << 20)) ? 0 : 1;
  return TileShape{rows, WAVES, nt};
}

}  // namespace lbm

struct lbm_handle {
  lbm_params p;
  Consts host;   // coefficients (host copy)
  Consts* dev;   // device copy (in the workspace)
  hipStream_t stream;
  int device;
  double* f[2];
  int cur;
  int* flag;
  long long pitch, plane;
  int variant;
  TileShape tile;
  TileShape tile2;  // tile shape of variant 4 (two steps per launch)
  WinGeom win;  // window shape of variant 3
};

static Field field_of(const lbm_handle* h, int from) {
  Field F;
  F.fin = h->f[from];
  F.fout = h->f[from ^ 1];
  F.nx = h->p.nx;
  F.ny = h->p.ny;
  F.pitch = h->pitch;
  F.plane = h->plane;
  return F;
}

extern "C" {

size_t lbm_workspace_bytes(const lbm_params* p) {
  if (validate(p) != LBM_OK) return 0;
  const long long plane = row_pitch(p->nx) * p->ny;
  return (size_t)(2 * 16 * plane * sizeof(double)) + 256 + consts_bytes();
}

lbm_status lbm_create(const lbm_params* p, void* d_workspace, size_t ws_bytes, void* hip_stream,
                      lbm_handle** out) {
  if (!out) return fail(LBM_EINVAL, "out is NULL");
  *out = nullptr;
  lbm_status st = validate(p);
  if (st != LBM_OK) return st;
  const size_t need = lbm_workspace_bytes(p);
  if (!d_workspace) return fail(LBM_EINVAL, "workspace is NULL");
  if (((uintptr_t)d_workspace) % 256) return fail(LBM_EINVAL, "workspace must be 256-byte aligned");
  if (ws_bytes < need) return fail(LBM_ENOMEM, "workspace has %zu bytes, needs %zu", ws_bytes, need);
  lbm_handle* h = new (std::nothrow) lbm_handle;
  if (!h) return fail(LBM_ENOMEM, "host allocation failed");
  h->p = *p;
  make_coef(p, &h->host.hot, &h->host.cold);
  h->stream = (hipStream_t)hip_stream;
  hipError_t e = hipGetDevice(&h->device);
  if (e != hipSuccess) {
    delete h;
    return hip_fail(e, "hipGetDevice");
  }
  h->pitch = row_pitch(p->nx);
  h->plane = h->pitch * p->ny;
  char* base = (char*)d_workspace;
  h->f[0] = (double*)base;
  h->f[1] = (double*)(base + 16 * h->plane * sizeof(double));
  h->flag = (int*)(base + 2 * 16 * h->plane * sizeof(double));
  h->dev = (Consts*)(base + 2 * 16 * h->plane * sizeof(double) + 256);
  h->cur = 0;
  h->variant = default_variant(p);
  h->win = default_window(p);
  h->tile = default_tile(p->nx, p->ny);
  h->tile2 = default_tile2(p->nx, p->ny);
  e = hipMemsetAsync(h->flag, 0, 256, h->stream);
  if (e == hipSuccess)
    e = hipMemcpyAsync(h->dev, &h->host, sizeof(Consts), hipMemcpyHostToDevice, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);  // the host copy source is the handle
  if (e != hipSuccess) {
    delete h;
    return hip_fail(e, "uploading the problem constants");
  }
  *out = h;
  clear_error();
  return LBM_OK;
}

lbm_status lbm_init(lbm_handle* h, const double* d_rho, const double* d_ux, const double* d_uy, const double* d_T) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  if (!d_rho || !d_ux || !d_uy || !d_T) return fail(LBM_EINVAL, "initial fields must not be NULL");
  Field F = field_of(h, h->cur ^ 1);  // write into the current buffer
  dim3 grid((h->p.nx + 63) / 64, h->p.ny);
  auto k = h->p.eq_version == 2 ? k_init<2> : h->p.eq_version == 3 ? k_init<3> : k_init<1>;
  hipLaunchKernelGGL(k, grid, dim3(64), 0, h->stream, F, d_rho, d_ux, d_uy, d_T);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "k_init launch");
  // the other buffer gets the same state so wall nodes are defined in both
  e = hipMemcpyAsync(h->f[h->cur ^ 1], h->f[h->cur], 16 * h->plane * sizeof(double), hipMemcpyDeviceToDevice,
                     h->stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpyAsync");
  return LBM_OK;
}

lbm_status lbm_step(lbm_handle* h, int64_t nsteps) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  if (nsteps < 0) return fail(LBM_EINVAL, "nsteps must be >= 0");
  if (h->variant == 2) {
    // whole grid in one workgroup: up to SMALL_CHUNK steps per launch
    constexpr int64_t SMALL_CHUNK = 1 << 16;
    for (int64_t n = 0; n < nsteps; n += SMALL_CHUNK) {
      const int k = (int)std::min<int64_t>(SMALL_CHUNK, nsteps - n);
      hipError_t e = launch_small(field_of(h, h->cur), &h->dev->hot, &h->dev->cold, h->p.eq_version,
                                  has_walls(&h->p), k, h->flag, h->stream);
      if (e != hipSuccess) return hip_fail(e, "small-problem kernel launch");
      h->cur ^= 1;
    }
    return LBM_OK;
  }
  if (h->variant == 3) {
    // up to win.h steps per launch in LDS windows
    const int64_t hmax = h->win.h;
    for (int64_t n = 0; n < nsteps; n += hmax) {
      const int k = (int)std::min<int64_t>(hmax, nsteps - n);
      hipError_t e = launch_window(field_of(h, h->cur), &h->dev->hot, &h->dev->cold, h->p.eq_version,
                                   has_walls(&h->p), h->win, k, h->flag, h->stream);
      if (e != hipSuccess) return hip_fail(e, "windowed kernel launch");
      h->cur ^= 1;
    }
    return LBM_OK;
  }
  int64_t n = 0;
  if (h->variant == 4) {
    // two steps per launch; an odd last step takes the one-step kernel
    for (; n + 2 <= nsteps; n += 2) {
      hipError_t e = launch_step2(field_of(h, h->cur), &h->dev->hot, &h->dev->cold, h->p.eq_version, h->tile2,
                                  h->flag, h->stream);
      if (e != hipSuccess) return hip_fail(e, "two-step kernel launch");
      h->cur ^= 1;
    }
  }
  for (; n < nsteps; ++n) {
    hipError_t e =
        launch_step(field_of(h, h->cur), &h->dev->hot, &h->dev->cold, h->p.eq_version, has_walls(&h->p),
                    h->p.scheme, h->variant == 4 ? 0 : h->variant, h->tile, h->flag, h->stream);
    if (e != hipSuccess) return hip_fail(e, "step kernel launch");
    h->cur ^= 1;
  }
  return LBM_OK;
}

lbm_status lbm_moments(lbm_handle* h, double* d_rho, double* d_ux, double* d_uy, double* d_T, double* d_p) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  Field F = field_of(h, h->cur);
  dim3 grid((h->p.nx + 63) / 64, h->p.ny);
  hipLaunchKernelGGL(k_moments<0>, grid, dim3(64), 0, h->stream, F, d_rho, d_ux, d_uy, d_T, d_p);
  hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "k_moments launch");
  return LBM_OK;
}

lbm_status lbm_get_f(lbm_handle* h, double* d_f) {
  if (!h || !d_f) return fail(LBM_EINVAL, "NULL argument");
  hipError_t e = hipMemcpy2DAsync(d_f, h->p.nx * sizeof(double), h->f[h->cur], h->pitch * sizeof(double),
                                  h->p.nx * sizeof(double), (size_t)16 * h->p.ny, hipMemcpyDeviceToDevice, h->stream);
  if (e != hipSuccess) return hip_fail(e, "hipMemcpy2DAsync");
  return LBM_OK;
}

lbm_status lbm_set_f(lbm_handle* h, const double* d_f) {
  if (!h || !d_f) return fail(LBM_EINVAL, "NULL argument");
  for (int b = 0; b < 2; ++b) {
    hipError_t e = hipMemcpy2DAsync(h->f[b], h->pitch * sizeof(double), d_f, h->p.nx * sizeof(double),
                                    h->p.nx * sizeof(double), (size_t)16 * h->p.ny, hipMemcpyDeviceToDevice,
                                    h->stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemcpy2DAsync");
  }
  return LBM_OK;
}

lbm_status lbm_check(lbm_handle* h) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  int flag = 0;
  hipError_t e = hipMemcpyAsync(&flag, h->flag, sizeof(int), hipMemcpyDeviceToHost, h->stream);
  if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
  if (e != hipSuccess) return hip_fail(e, "reading the health flag");
  if (flag) {
    e = hipMemsetAsync(h->flag, 0, sizeof(int), h->stream);
    if (e != hipSuccess) return hip_fail(e, "hipMemsetAsync");
    return fail(LBM_ENONFINITE, "a step produced rho <= 0, T <= 0 or NaN");
  }
  return LBM_OK;
}

lbm_status lbm_set_variant(lbm_handle* h, int32_t variant) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  if (variant < 0 || variant > 4) return fail(LBM_EINVAL, "variant must be 0, 1, 2, 3 or 4");
  if (variant == 4 && !two_step_problem(&h->p))
    return fail(LBM_EINVAL, "variant 4 needs scheme 0 and no NEQ walls");
  if (variant == 2 && !small_problem(&h->p))
    return fail(LBM_EINVAL, "variant 2 needs scheme 0 and nx ny <= %d nodes", SMALL_NODES);
  if (variant == 3 && !window_problem(&h->p))
    return fail(LBM_EINVAL, "variant 3 needs scheme 0 and nx ny > %d nodes", SMALL_NODES);
  h->variant = variant;
  return LBM_OK;
}

lbm_status lbm_set_tile(lbm_handle* h, int32_t rows, int32_t waves) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  if (rows < 1 || rows > 1024) return fail(LBM_EINVAL, "rows must be in 1..1024");
  if (waves != 2 && waves != 4) return fail(LBM_EINVAL, "waves must be 2 or 4");
  if (h->variant == 4) {
    h->tile2 = TileShape{rows, waves, h->tile2.nt};
    return LBM_OK;
  }
  // NEQ walls and the flux-limited scheme always run 4-wave tiles
  h->tile = TileShape{rows, (has_walls(&h->p) || h->p.scheme == 1) ? 4 : waves, h->tile.nt};
  return LBM_OK;
}

lbm_status lbm_set_store_mode(lbm_handle* h, int32_t nontemporal) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  if (nontemporal != 0 && nontemporal != 1) return fail(LBM_EINVAL, "nontemporal must be 0 or 1");
  h->tile.nt = nontemporal;
  h->tile2.nt = nontemporal;
  return LBM_OK;
}

lbm_status lbm_get_store_mode(const lbm_handle* h, int32_t* nontemporal) {
  if (!h || !nontemporal) return fail(LBM_EINVAL, "NULL argument");
  *nontemporal = h->tile.nt;
  return LBM_OK;
}

lbm_status lbm_set_window(lbm_handle* h, int32_t cols, int32_t rows, int32_t steps) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  WinGeom g;
  if (!make_window(&h->p, cols, rows, steps, &g))
    return fail(LBM_EINVAL,
                "window %d x %d with %d steps: need steps >= 1, a cut axis longer than 2 steps, "
                "and at most %d nodes held",
                cols, rows, steps, SMALL_NODES);
  h->win = g;
  return LBM_OK;
}

lbm_status lbm_get_window(const lbm_handle* h, int32_t* cols, int32_t* rows, int32_t* steps) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  if (cols) *cols = h->win.x.w;
  if (rows) *rows = h->win.y.w;
  if (steps) *steps = h->win.h;
  return LBM_OK;
}

lbm_status lbm_tune(lbm_handle* h, int64_t probe_steps, double* d_scratch, size_t scratch_bytes, int32_t* rows_out,
                    int32_t* waves_out, double* best_ms) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  if (probe_steps < 1) return fail(LBM_EINVAL, "probe_steps must be >= 1");
  const size_t state = 16 * (size_t)h->plane * sizeof(double);
  if (d_scratch && scratch_bytes < state) return fail(LBM_EINVAL, "scratch needs %zu bytes", state);
  hipError_t e = hipSuccess;
  if (d_scratch) e = hipMemcpyAsync(d_scratch, h->f[h->cur], state, hipMemcpyDeviceToDevice, h->stream);
  if (e != hipSuccess) return hip_fail(e, "saving the state");
  const int saved_cur = h->cur, saved_variant = h->variant;
  // the windowed and two-step kernels compete with the fused one unless
  // another variant was chosen
  const bool windows = window_problem(&h->p) && (saved_variant == 0 || saved_variant == 3 || saved_variant == 4);
  const bool two_step = two_step_problem(&h->p) && (saved_variant == 0 || saved_variant == 3 || saved_variant == 4);
  // the two-step kernel is timed over an even number of steps (an odd count
  // would end with a one-step launch)
  const int64_t probe2 = (probe_steps + 1) / 2 * 2;
  hipEvent_t t0 = nullptr, t1 = nullptr;
  e = hipEventCreate(&t0);
  if (e == hipSuccess) e = hipEventCreate(&t1);
  if (e != hipSuccess) {
    if (t0) (void)hipEventDestroy(t0);
    return hip_fail(e, "hipEventCreate");
  }
  lbm_status st = LBM_OK;
  // probe_steps steps of the current configuration after a 2-step warm-up
  auto time_it = [&](float& ms) -> bool {
    const int64_t n = h->variant == 4 ? probe2 : probe_steps;
    st = lbm_step(h, 2);
    if (st != LBM_OK) return false;
    e = hipEventRecord(t0, h->stream);
    if (e == hipSuccess) st = lbm_step(h, n);
    if (e == hipSuccess) e = hipEventRecord(t1, h->stream);
    if (e == hipSuccess) e = hipEventSynchronize(t1);
    if (e == hipSuccess && st == LBM_OK) e = hipEventElapsedTime(&ms, t0, t1);
    ms *= (float)probe_steps / (float)n;  // per probe_steps steps
    return e == hipSuccess && st == LBM_OK;
  };
  const int cand[] = {4, 8, 12, 16, 20, 24, 28, 32, 40, 48, 56, 64, 96, 128, 192, 256};
  const int wcand[] = {4, 2};
  TileShape best = h->tile;
  float best_t = 1e30f;
  WinGeom best_win = h->win;
  float best_win_t = 1e30f;
  bool good = true;
  h->variant = 0;
  for (int nt : {1, 0}) {
    for (int wv : wcand) {
      if (wv != 4 && (has_walls(&h->p) || h->p.scheme == 1)) continue;
      int last_rows = -1;
      for (int r : cand) {
        const MarchGeom g = march_geom(h->p.nx, h->p.ny, TileShape{r, wv, nt});
        if (g.rows == last_rows) continue;  // same tiling as a smaller candidate
        last_rows = g.rows;
        h->tile = TileShape{g.rows, wv, nt};
        float ms = 0;
        if (!(good = time_it(ms))) break;
        if (ms < best_t) {
          best_t = ms;
          best = h->tile;
        }
      }
      if (!good) break;
    }
    if (!good) break;
  }
  h->tile = best;
  TileShape best2 = h->tile2;
  float best2_t = 1e30f;
  if (good && two_step) {
    // two steps per launch: 2 or 4 waves, tile heights down from the
    // fastest of the fused kernel's list, plus heights that give just under
    // one, two or three tiles per workgroup slot (two per CU)
    h->variant = 4;
    int rc[32];
    int nrc = 0;
    for (int r : cand) rc[nrc++] = r;
    const long long strips = (h->p.nx + OSTRIP - 1) / OSTRIP;
    for (int k = 1; k <= 3; ++k) {
      const long long segs = std::max(1ll, (long long)k * 512 / strips);
      rc[nrc++] = (int)std::min<long long>(1024, (h->p.ny + segs - 1) / segs);
    }
    for (int nt : {1, 0}) {
      for (int wv : {2, 4}) {
        int seen[32];
        int nseen = 0;
        for (int j = 0; j < nrc && good; ++j) {
          const March2Geom g = march2_geom(h->p.nx, h->p.ny, TileShape{rc[j], wv, nt});
          if (std::find(seen, seen + nseen, g.rows) != seen + nseen) continue;
          seen[nseen++] = g.rows;
          h->tile2 = TileShape{g.rows, wv, nt};
          float ms = 0;
          if (!(good = time_it(ms))) break;
          if (ms < best2_t) {
            best2_t = ms;
            best2 = h->tile2;
          }
        }
      }
    }
    h->tile2 = best2;
  }
  if (good && windows) {
    // window shapes: narrow grids keep every row; others take 2-D windows
    int shapes[24][3];
    int ns = 0;
    if (h->p.ny <= 16) {
      for (int wc = 32; wc <= SMALL_NODES; wc *= 2)
        for (int div : {16, 8, 4})
          if (ns < 24) shapes[ns][0] = wc, shapes[ns][1] = h->p.ny, shapes[ns][2] = wc / div, ++ns;
    } else {
      const int two_d[][3] = {{32, 16, 2}, {32, 16, 3}, {16, 32, 2}, {16, 32, 3},
                              {32, 8, 2},  {64, 8, 2},  {16, 16, 2}, {16, 16, 3}};
      for (const auto& c3 : two_d) shapes[ns][0] = c3[0], shapes[ns][1] = c3[1], shapes[ns][2] = c3[2], ++ns;
    }
    h->variant = 3;
    for (int i = 0; i < ns && good; ++i) {
      WinGeom g;
      if (!make_window(&h->p, shapes[i][0], shapes[i][1], shapes[i][2], &g)) continue;
      h->win = g;
      float ms = 0;
      if (!(good = time_it(ms))) break;
      if (ms < best_win_t) {
        best_win_t = ms;
        best_win = g;
      }
    }
    h->win = best_win;
  }
  (void)hipEventDestroy(t0);
  (void)hipEventDestroy(t1);
  if (windows || two_step) {
    h->variant = 0;
    float bt = best_t;
    if (best_win_t < bt) h->variant = 3, bt = best_win_t;
    if (best2_t < bt) h->variant = 4, bt = best2_t;
  } else {
    h->variant = saved_variant;
  }
  if (e != hipSuccess) return hip_fail(e, "tuning run");
  if (st != LBM_OK) return st;
  if (d_scratch) {
    h->cur = saved_cur;
    e = hipMemcpyAsync(h->f[h->cur], d_scratch, state, hipMemcpyDeviceToDevice, h->stream);
    if (e == hipSuccess) e = hipStreamSynchronize(h->stream);
    if (e != hipSuccess) return hip_fail(e, "restoring the state");
  }
  const TileShape& kept = h->variant == 4 ? h->tile2 : best;
  if (rows_out) *rows_out = kept.rows;
  if (waves_out) *waves_out = kept.waves;
  if (best_ms) *best_ms = std::min(best_t, std::min(best_win_t, best2_t));
  return LBM_OK;
}

lbm_status lbm_get_variant(const lbm_handle* h, int32_t* variant) {
  if (!h || !variant) return fail(LBM_EINVAL, "NULL argument");
  *variant = h->variant;
  return LBM_OK;
}

lbm_status lbm_get_tile(const lbm_handle* h, int32_t* rows, int32_t* waves) {
  if (!h) return fail(LBM_EINVAL, "handle is NULL");
  const TileShape& t = h->variant == 4 ? h->tile2 : h->tile;
  if (rows) *rows = t.rows;
  if (waves) *waves = t.waves;
  return LBM_OK;
}

const char* lbm_last_error(void) { return g_err.c_str(); }

void lbm_destroy(lbm_handle* h) { delete h; }


lbm_status lbm_stream_copy(const double* d_src, double* d_dst, int32_t nx, int32_t ny, void* hip_stream) {
  if (!d_src || !d_dst) return fail(LBM_EINVAL, "NULL argument");
  if (nx < 1 || ny < 1) return fail(LBM_EINVAL, "nx and ny must be >= 1");
  const long long pitch = row_pitch(nx);
  const int rows = 32;
  const int nstrips = (int)(pitch / STRIP);
  const long long ntiles = (long long)nstrips * ((ny + rows - 1) / rows);
  if (ntiles > INT_MAX) return fail(LBM_EINVAL, "field too large");
  hipLaunchKernelGGL(k_stream_copy<0>, dim3((unsigned)ntiles), dim3(64 * WAVES), 0, (hipStream_t)hip_stream, d_src, d_dst,
                     ny, pitch, rows, nstrips, (int)ntiles);
  const hipError_t e = hipGetLastError();
  if (e != hipSuccess) return hip_fail(e, "k_stream_copy launch");
  return LBM_OK;
}

}  // extern "C"
