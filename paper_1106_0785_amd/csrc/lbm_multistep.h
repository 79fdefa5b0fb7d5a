// Multi-step kernels for grids that one launch per step leaves bound by
// launch cost: the small-grid kernel (the whole grid in one workgroup's LDS)
// and the narrow-grid kernel (overlapping LDS windows of all rows). Both use
// the plain kernel's stencil, ghost rules and node arithmetic.
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
// Narrow grids (few rows, many columns; more than SMALL_NODES nodes): each
// workgroup holds a window of wc columns by all ny rows in LDS and advances
// it up to h steps per launch (temporal blocking). Windows overlap by h
// columns on each side that is cut from a neighbouring window; after k steps
// a node is exact if it is at least k columns from every cut side, so the
// middle v = wc - 2 h columns are written back. On a periodic x axis the
// window columns are the periodic images of the stored ones (the update is
// translation invariant); on other x boundaries the window is clipped to the
// domain and the ghost rules apply at the domain edge, as in the other
// kernels. Each node's arithmetic is the plain kernel's.
// ---------------------------------------------------------------------------
struct BandGeom {
  int wc;    // window columns (wc ny <= SMALL_NODES)
  int h;     // most steps per launch
  int v;     // columns written per window: wc - 2 h
  int nwin;  // windows: ceil(nx / v)
};

template <int VER, bool WALLS>
__global__ __launch_bounds__(SMALL_NODES) void k_step_band(Field F, const Hot* __restrict__ hot,
                                                          const Cold* __restrict__ cold, BandGeom bg, int nsteps,
                                                          int* flag) {
  __shared__ double buf[2][16][SMALL_NODES];
  __shared__ Hot hs;
  stage_hot(hot, &hs);
  const Hot& c = hs;
  const bool xper = c.bc[0] == BC_PERIODIC;
  const int x0 = blockIdx.x * bg.v;  // first column this window writes
  int xs = x0 - bg.h, xe = x0 + bg.v + bg.h;
  if (!xper) {
    xs = max(xs, 0);
    xe = min(xe, F.nx);
  }
  const int ncols = xe - xs;
  const bool lo_cut = xper || xs > 0, hi_cut = xper || xe < F.nx;
  const int t = threadIdx.x;
  const bool active = t < ncols * F.ny;
  const int xw = active ? t % ncols : 0, y = active ? t / ncols : 0;
  const int xv = xs + xw;                                    // column (virtual on a periodic axis)
  const int xg = xper ? ((xv % F.nx) + F.nx) % F.nx : xv;  // stored column
  if (active) {
#pragma unroll
    for (int i = 0; i < 16; ++i) buf[0][i][t] = F.fin[i * F.plane + (long long)y * F.pitch + xg];
  }
  __syncthreads();
  // x neighbours: inside the window; the ghost rule at a domain edge; at a
  // cut side the node's own column (the node is outside the exact region
  // from the first step on, and is neither written back nor checked)
  auto xnbr = [&](int d, int& col) -> Src {
    const int w2 = xw + d;
    if (w2 >= 0 && w2 < ncols) {
      col = w2;
      return Src{w2, 0, -1};
    }
    if ((d < 0 && lo_cut) || (d > 0 && hi_cut)) {
      col = xw;
      return Src{xw, 0, -1};
    }
    const Src sg = resolve(xg + d, F.nx, c.bc[0], c.bc[1], 0);
    col = sg.idx - xs;
    return sg;
  };
  int cxp, cxm;
  const Src sxp = xnbr(1, cxp), sxm = xnbr(-1, cxm);
  const Src cx{xw, 0, -1}, cy = resolve(y, F.ny, c.bc[2], c.bc[3], 2);
  const Src syp = resolve(y + 1, F.ny, c.bc[2], c.bc[3], 2), sym = resolve(y - 1, F.ny, c.bc[2], c.bc[3], 2);
  auto point = [&](int b, int col, const Src& sx, const Src& sy, double* f) {
    const int k = sy.idx * ncols + col;
#pragma unroll
    for (int i = 0; i < 16; ++i) f[i] = buf[b][i][k];
    fix_ghost(cold, sx, sy, f);
  };
  const bool wall = WALLS && active && is_wall_node(c, xg, y, F.nx, F.ny);
  int wnb = 0, wside = 0;
  if (WALLS && wall) {
    if (c.bc[2] == BC_NEQ_WALL && y == 0) { wnb = 1 * ncols + xw; wside = 2; }
    else if (c.bc[3] == BC_NEQ_WALL && y == F.ny - 1) { wnb = (F.ny - 2) * ncols + xw; wside = 3; }
    else if (c.bc[0] == BC_NEQ_WALL && xg == 0) { wnb = y * ncols + xw + 1; wside = 0; }
    else { wnb = y * ncols + xw - 1; wside = 1; }
  }
  bool ok = true;
  int P = 0;
  for (int s = 1; s <= nsteps; ++s) {
    const int Q = P ^ 1;
    if (active && !wall) {
      double f[16], fxp[16], fxm[16], fyp[16], fym[16];
      point(P, xw, cx, cy, f);
      point(P, cxp, sxp, cy, fxp);
      point(P, cxm, sxm, cy, fxm);
      point(P, xw, cx, syp, fyp);
      point(P, xw, cx, sym, fym);
      NbrVel nv;
      velocity_of(fxp, nv.ux_xp, nv.uy_xp);
      velocity_of(fxm, nv.ux_xm, nv.uy_xm);
      velocity_of(fyp, nv.ux_yp, nv.uy_yp);
      velocity_of(fym, nv.ux_ym, nv.uy_ym);
      double out[16];
      const bool exact = (!lo_cut || xw >= s) && (!hi_cut || xw < ncols - s);
      ok &= node_update<VER>(c, f, fxp, fxm, fyp, fym, nv, out) || !exact;
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
  if (active && xv >= x0 && xv < x0 + bg.v && xv >= 0 && xv < F.nx) {
#pragma unroll
    for (int i = 0; i < 16; ++i) F.fout[i * F.plane + (long long)y * F.pitch + xg] = buf[P][i][t];
  }
  if (!ok) flag[0] = 1;
}

}  // namespace lbm
