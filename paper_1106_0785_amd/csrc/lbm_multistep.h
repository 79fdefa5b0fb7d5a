// Multi-step kernels for grids that one launch per step leaves bound by
// launch cost or latency: the small-grid kernel (the whole grid in one
// workgroup's LDS) and the windowed kernel (overlapping LDS windows, several
// steps per launch). Both use the plain kernel's stencil, ghost rules and
// node arithmetic.
#pragma once

#include "lbm_kernels.h"

namespace lbm {

// ---------------------------------------------------------------------------
// Small problems (nx ny <= SMALL_NODES nodes): one workgroup holds the whole
// grid in LDS (two buffers of 16 planes) and advances it nsteps time steps in
// one launch, one thread per node, with the plain kernel's stencil, ghost
// rules and arithmetic. Such grids are bound by the cost of a launch, which
// this pays once for many steps.
// ---------------------------------------------------------------------------
constexpr int SMALL_NODES = 512;

template <int VER, bool WALLS>
__global__ __launch_bounds__(SMALL_NODES) void k_step_small(Field F, const Hot* __restrict__ hot,
                                                           const Cold* __restrict__ cold, int nsteps, int* flag) {
  __shared__ double buf[2][16][SMALL_NODES];
  __shared__ Hot hs;
  stage_hot(hot, &hs);
  const Hot& c = hs;
  const int N = F.nx * F.ny;
  const int t = threadIdx.x;
  const bool active = t < N;
  const int x = active ? t % F.nx : 0, y = active ? t / F.nx : 0;
  if (active) {
#pragma unroll
    for (int i = 0; i < 16; ++i) buf[0][i][t] = F.fin[i * F.plane + (long long)y * F.pitch + x];
  }
  __syncthreads();
  const Src cx = resolve(x, F.nx, c.bc[0], c.bc[1], 0), cy = resolve(y, F.ny, c.bc[2], c.bc[3], 2);
  const Src sxp = resolve(x + 1, F.nx, c.bc[0], c.bc[1], 0), sxm = resolve(x - 1, F.nx, c.bc[0], c.bc[1], 0);
  const Src syp = resolve(y + 1, F.ny, c.bc[2], c.bc[3], 2), sym = resolve(y - 1, F.ny, c.bc[2], c.bc[3], 2);
  // the stencil point (sx, sy) of buffer b with its ghost rule
  auto point = [&](int b, const Src& sx, const Src& sy, double* f) {
    const int k = sy.idx * F.nx + sx.idx;
#pragma unroll
    for (int i = 0; i < 16; ++i) f[i] = buf[b][i][k];
    fix_ghost(cold, sx, sy, f);
  };
  const bool wall = WALLS && active && is_wall_node(c, x, y, F.nx, F.ny);
  // a wall node's fluid neighbour and side (walls on one axis only)
  int wnb = 0, wside = 0;
  if (WALLS && wall) {
    if (c.bc[2] == BC_NEQ_WALL && y == 0) { wnb = 1 * F.nx + x; wside = 2; }
    else if (c.bc[3] == BC_NEQ_WALL && y == F.ny - 1) { wnb = (F.ny - 2) * F.nx + x; wside = 3; }
    else if (c.bc[0] == BC_NEQ_WALL && x == 0) { wnb = y * F.nx + 1; wside = 0; }
    else { wnb = y * F.nx + F.nx - 2; wside = 1; }
  }
  bool ok = true;
  int P = 0;
  for (int s = 0; s < nsteps; ++s) {
    const int Q = P ^ 1;
    if (active && !wall) {
      double f[16], fxp[16], fxm[16], fyp[16], fym[16];
      point(P, cx, cy, f);
      point(P, sxp, cy, fxp);
      point(P, sxm, cy, fxm);
      point(P, cx, syp, fyp);
      point(P, cx, sym, fym);
      NbrVel nv;
      velocity_of(fxp, nv.ux_xp, nv.uy_xp);
      velocity_of(fxm, nv.ux_xm, nv.uy_xm);
      velocity_of(fyp, nv.ux_yp, nv.uy_yp);
      velocity_of(fym, nv.ux_ym, nv.uy_ym);
      double out[16];
      ok &= node_update<VER>(c, f, fxp, fxm, fyp, fym, nv, out);
#pragma unroll
      for (int i = 0; i < 16; ++i) buf[Q][i][t] = out[i];
    }
    __syncthreads();
    if (WALLS) {
      if (wall) {
        double fn[16], fw[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) fn[i] = buf[Q][i][wnb];
        neq_wall<VER>(cold->wall[wside], fn, fw);
#pragma unroll
        for (int i = 0; i < 16; ++i) buf[Q][i][t] = fw[i];
      }
      __syncthreads();
    }
    P = Q;
  }
  if (active) {
#pragma unroll
    for (int i = 0; i < 16; ++i) F.fout[i * F.plane + (long long)y * F.pitch + x] = buf[P][i][t];
  }
  if (!ok) flag[0] = 1;
}

// ---------------------------------------------------------------------------
// Windowed multi-step kernel: each workgroup holds a window of wc columns by
// wr rows in LDS (one thread per node) and advances it up to h steps per
// launch (temporal blocking). Along an axis that one window covers whole,
// neighbours follow the ghost rules as in the other kernels. Along an axis
// cut into windows, windows overlap by h nodes on each side cut from a
// neighbouring window; after k steps a node is exact if it lies at least k
// nodes from every cut side, so the middle (w - 2 h) nodes are written back
// and those parts tile the axis. On a periodic cut axis the window holds the
// periodic images of the stored nodes (the update is translation invariant);
// on other cut axes windows are clipped to the domain and the ghost rules
// apply at the domain edge. Narrow grids (few rows) use one window row.
// Each node's arithmetic is the plain kernel's.
// ---------------------------------------------------------------------------
struct WinAxis {
  int w;      // window extent (nodes held); the whole axis when nwin == 1 and whole
  int v;      // nodes written per window (w - 2 halo on a cut axis)
  int nwin;   // windows along the axis
  int whole;  // 1: one window holds the whole axis (no cuts)
  int halo;   // overlap per cut side: h, or h + 1 on an axis with NEQ walls
              // (a wall node takes its fluid neighbour's value of the same
              // step, so it is exact one step less long than its distance
              // from a cut side)
};

struct WinGeom {
  WinAxis x, y;
  int h;  // most steps per launch
};

// One axis of one window: held nodes [s, e) (virtual on a periodic cut
// axis), the nodes it writes [o, o + v), and which sides are cuts.
struct WinSpan {
  int s, n, o, v;
  bool lo_cut, hi_cut;
};

__device__ __forceinline__ WinSpan win_span(const WinAxis& a, int win, int len, bool per) {
  WinSpan r;
  if (a.whole) {
    r.s = 0;
    r.n = len;
    r.o = 0;
    r.v = len;
    r.lo_cut = r.hi_cut = false;
    return r;
  }
  r.o = win * a.v;
  r.v = a.v;
  int s = r.o - a.halo, e = r.o + a.v + a.halo;
  if (!per) {
    s = max(s, 0);
    e = min(e, len);
  }
  r.s = s;
  r.n = e - s;
  r.lo_cut = per || s > 0;
  r.hi_cut = per || e < len;
  return r;
}

// Neighbour (offset d = +-1) of local node w along one axis of a window:
// local index and ghost treatment. At a cut side the node's own index is
// returned: the node is outside the exact region from the first step on.
__device__ __forceinline__ Src win_nbr(const WinSpan& sp, int w, int g, int d, int len, int bc_lo, int bc_hi,
                                       int side, int& local) {
  const int w2 = w + d;
  if (w2 >= 0 && w2 < sp.n) {
    local = w2;
    return Src{w2, 0, -1};
  }
  if ((d < 0 && sp.lo_cut) || (d > 0 && sp.hi_cut)) {
    local = w;
    return Src{w, 0, -1};
  }
  const Src sg = resolve(g + d, len, bc_lo, bc_hi, side);
  local = sg.idx - sp.s;
  return sg;
}

// NODES: most nodes a window holds (512, or 256 so that two workgroups
// share a CU's LDS).
template <int VER, bool WALLS, int NODES>
__global__ __launch_bounds__(NODES) void k_step_window(Field F, const Hot* __restrict__ hot,
                                                      const Cold* __restrict__ cold, WinGeom wg, int nsteps,
                                                      int* flag) {
  // 16 distributions and the velocity of every held node, two buffers
  __shared__ double buf[2][NV][NODES];
  __shared__ Hot hs;
  stage_hot(hot, &hs);
  const Hot& c = hs;
  const bool xper = c.bc[0] == BC_PERIODIC, yper = c.bc[2] == BC_PERIODIC;
  const WinSpan sx = win_span(wg.x, blockIdx.x % wg.x.nwin, F.nx, xper);
  const WinSpan sy = win_span(wg.y, blockIdx.x / wg.x.nwin, F.ny, yper);
  const int t = threadIdx.x;
  const bool active = t < sx.n * sy.n;
  const int xw = active ? t % sx.n : 0, yw = active ? t / sx.n : 0;
  const int xv = sx.s + xw, yv = sy.s + yw;  // virtual on a periodic cut axis
  const int xg = xper ? ((xv % F.nx) + F.nx) % F.nx : xv;
  const int yg = yper ? ((yv % F.ny) + F.ny) % F.ny : yv;
  // a node's distributions and velocity into buffer b
  auto put = [&](int b, const double* f) {
    double ux, uy;
    velocity_of(f, ux, uy);
#pragma unroll
    for (int i = 0; i < 16; ++i) buf[b][i][t] = f[i];
    buf[b][16][t] = ux;
    buf[b][17][t] = uy;
  };
  if (active) {
    double f[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) f[i] = F.fin[i * F.plane + (long long)yg * F.pitch + xg];
    put(0, f);
  }
  __syncthreads();
  int lxp, lxm, lyp, lym;
  const Src nxp = win_nbr(sx, xw, xg, 1, F.nx, c.bc[0], c.bc[1], 0, lxp);
  const Src nxm = win_nbr(sx, xw, xg, -1, F.nx, c.bc[0], c.bc[1], 0, lxm);
  const Src nyp = win_nbr(sy, yw, yg, 1, F.ny, c.bc[2], c.bc[3], 2, lyp);
  const Src nym = win_nbr(sy, yw, yg, -1, F.ny, c.bc[2], c.bc[3], 2, lym);
  const Src cx{xw, 0, -1}, cy{yw, 0, -1};
  // a neighbour's distributions and velocity: the stored velocity, or, for
  // a ghost point, the velocity of the ghost distributions
  auto point = [&](int b, int lx, int ly, const Src& gx, const Src& gy, double* f, double& ux, double& uy) {
    const int k = ly * sx.n + lx;
#pragma unroll
    for (int i = 0; i < 16; ++i) f[i] = buf[b][i][k];
    if ((gx.mode | gy.mode) != 0) {
      fix_ghost(cold, gx, gy, f);
      velocity_of(f, ux, uy);
    } else {
      ux = buf[b][16][k];
      uy = buf[b][17][k];
    }
  };
  const bool wall = WALLS && active && is_wall_node(c, xg, yg, F.nx, F.ny);
  int wnb = 0, wside = 0;
  if (WALLS && wall) {
    if (c.bc[2] == BC_NEQ_WALL && yg == 0) { wnb = (yw + 1) * sx.n + xw; wside = 2; }
    else if (c.bc[3] == BC_NEQ_WALL && yg == F.ny - 1) { wnb = (yw - 1) * sx.n + xw; wside = 3; }
    else if (c.bc[0] == BC_NEQ_WALL && xg == 0) { wnb = yw * sx.n + xw + 1; wside = 0; }
    else { wnb = yw * sx.n + xw - 1; wside = 1; }
  }
  bool ok = true;
  int P = 0;
  for (int s = 1; s <= nsteps; ++s) {
    const int Q = P ^ 1;
    if (active && !wall) {
      double f[16], fxp[16], fxm[16], fyp[16], fym[16];
      const int k0 = yw * sx.n + xw;
#pragma unroll
      for (int i = 0; i < 16; ++i) f[i] = buf[P][i][k0];
      NbrVel nv;
      point(P, lxp, yw, nxp, cy, fxp, nv.ux_xp, nv.uy_xp);
      point(P, lxm, yw, nxm, cy, fxm, nv.ux_xm, nv.uy_xm);
      point(P, xw, lyp, cx, nyp, fyp, nv.ux_yp, nv.uy_yp);
      point(P, xw, lym, cx, nym, fym, nv.ux_ym, nv.uy_ym);
      double out[16];
      const bool exact = (!sx.lo_cut || xw >= s) && (!sx.hi_cut || xw < sx.n - s) && (!sy.lo_cut || yw >= s) &&
                         (!sy.hi_cut || yw < sy.n - s);
      ok &= node_update<VER>(c, f, fxp, fxm, fyp, fym, nv, out) || !exact;
      put(Q, out);
    }
    __syncthreads();
    if (WALLS) {
      if (wall) {
        double fn[16], fw[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) fn[i] = buf[Q][i][wnb];
        neq_wall<VER>(cold->wall[wside], fn, fw);
        put(Q, fw);
      }
      __syncthreads();
    }
    P = Q;
  }
  if (active && xv >= sx.o && xv < sx.o + sx.v && xv >= 0 && xv < F.nx && yv >= sy.o && yv < sy.o + sy.v &&
      yv >= 0 && yv < F.ny) {
#pragma unroll
    for (int i = 0; i < 16; ++i) F.fout[i * F.plane + (long long)yg * F.pitch + xg] = buf[P][i][t];
  }
  if (!ok) flag[0] = 1;
}

}  // namespace lbm
