// Two time steps per launch (temporal blocking of the fused step kernel).
//
// The step kernel moves 256 bytes per node-step through HBM and the chip
// writes more slowly than it reads, so the step is bound by memory while its
// arithmetic takes well under half the time. This kernel reads f^n once,
// computes f^{n+1} into a second LDS ring and f^{n+2} from it, and writes
// f^{n+2} once: 128 bytes per node-step. Each node update is the fused
// kernel's (same functions, same order), and the ghost values of the
// intermediate level are made from its own boundary values by the same rules
// the step kernel applies when it loads them, so two steps here are two
// launches of the step kernel up to rounding (the velocities of the columns
// beside a strip come from a lane sum, and the strips lie elsewhere).
//
// Geometry. A workgroup of W wavefronts owns an output strip of OSTRIP = 62
// columns [62k, 62k + 62) by `rows` rows. Lane l works on column
// X = 62k - 1 + l (l = 0..63) at the intermediate level, so the 62 output
// columns have both their intermediate neighbours in the wavefront; the level
// n values are needed at columns 62k - 2 .. 62k + 63 (ring 0: the lanes' own
// columns plus one neighbour column each side, loaded as the step kernel
// loads them). Rows march up as in the step kernel: in iteration i wave w
// computes level n+1 at row a = y0 - 1 + i W + w (ring 0 -> ring 1) and, after
// a barrier, level n+2 at row a - 1 (ring 1 -> HBM).
//
// Intermediate ghosts. On a periodic side the ghost column or row of level
// n+1 is computed like any node (its level n inputs wrap). On the other kinds
// it is not a node: the lane (or wavefront) that computes the boundary column
// (row) also writes the ghost entry next to it from its own new values
// (mirror: velocities mirrored across the side; zero gradient: a copy; fixed
// state: the side's equilibrium). A ghost row whose boundary row is computed
// by another wavefront of the same iteration is computed again by the ghost
// row's wavefront (same arithmetic, same values).
#pragma once

#include "lbm_kernels.h"

namespace lbm {

constexpr int OSTRIP = 62;

struct March2Geom {
  int nstrips;  // ceil(nx / OSTRIP)
  int rows;     // output rows per tile (multiple of the wavefront count)
  int nsegs;    // ceil(ny / rows)
  int ntiles;   // nstrips * nsegs
  int per_xcd;  // ceil(ntiles / 8)
};

__device__ __forceinline__ int xcd_tile2(int b, const March2Geom& g) { return (b % 8) * g.per_xcd + b / 8; }

// Copies one intermediate node's values (16 distributions + velocity) into a
// ring-1 entry after the ghost rule `mode` of the side it borders: 0 as is,
// 1 mirrored in x, 2 mirrored in y, 3 the fixed state of side `side`.
template <int RWT>
__device__ __forceinline__ void put_entry(double (*row)[RWT], int col, const double* v, double ux, double uy,
                                          int mode, const Cold* __restrict__ cold, int side) {
  if (mode == 3) {
    const double* gh = cold->ghost[side];
    double gx, gy;
    velocity_of(gh, gx, gy);
#pragma unroll
    for (int i = 0; i < 16; ++i) row[i][col] = gh[i];
    row[16][col] = gx;
    row[17][col] = gy;
  } else if (mode == 1) {
#pragma unroll
    for (int i = 0; i < 16; ++i) row[i][col] = v[MIRROR_X[i]];
    row[16][col] = -ux;
    row[17][col] = uy;
  } else if (mode == 2) {
#pragma unroll
    for (int i = 0; i < 16; ++i) row[i][col] = v[MIRROR_Y[i]];
    row[16][col] = ux;
    row[17][col] = -uy;
  } else {
#pragma unroll
    for (int i = 0; i < 16; ++i) row[i][col] = v[i];
    row[16][col] = ux;
    row[17][col] = uy;
  }
}

// Ghost rule of a non-periodic side for the intermediate level: 1/2 mirror in
// x/y, 0 zero gradient (copy), 3 fixed state; -1 periodic (computed as a node).
__device__ __forceinline__ int ghost_mode(int bc, bool x_axis) {
  switch (bc) {
    case BC_SPECULAR: return x_axis ? 1 : 2;
    case BC_DIRICHLET_EQ: return 3;
    case BC_PERIODIC: return -1;
    default: return 0;  // zero gradient (NEQ walls are not taken by this kernel)
  }
}

template <int VER, int W, bool NT>
__device__ __forceinline__ void fused2_tile(Field F, const Hot* __restrict__ hot, const Cold* __restrict__ cold,
                                            March2Geom g, int tile, int* flag) {
  constexpr int R = W + 2;   // rows held by each ring
  constexpr int C0 = 66;     // ring 0 columns: 62k-2 .. 62k+63
  constexpr int C1 = 64;     // ring 1 columns: 62k-1 .. 62k+62
  __shared__ double ring0[R][NV][C0];
  __shared__ double ring1[R][NV][C1];
  __shared__ Hot hs;
  stage_hot(hot, &hs);
  const Hot& c = hs;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int strip = tile % g.nstrips, seg = tile / g.nstrips;
  const int nx = F.nx, ny = F.ny;
  const int X = strip * OSTRIP - 1 + lane;  // this lane's column
  const int y0 = seg * g.rows;
  const int y1 = min(y0 + g.rows, ny);
  const int ylast = y1 + 1;  // last level-n row the tile reads
  const int base0 = y0 - 2, base1 = y0 - 3;
  // level-n column of this lane (lanes past nx + 1 are never needed: they
  // read column nx - 1 and their results are dropped)
  const Src sx = (X < nx + 2) ? resolve(X, nx, c.bc[0], c.bc[1], 0) : Src{nx - 1, 0, -1};
  const int bylo = __builtin_amdgcn_readfirstlane(hot->bc[2]);
  const int byhi = __builtin_amdgcn_readfirstlane(hot->bc[3]);
  // (rows are wave-uniform: the ghost rule is scalar code)
  auto ysrc = [&](int yr) -> Src {
    if (yr < 0 || yr >= ny) return resolve(yr, ny, bylo, byhi, 2);
    return Src{yr, 0, -1};
  };
  // ghost rules of the intermediate level
  const int gxl = ghost_mode(c.bc[0], true), gxh = ghost_mode(c.bc[1], true);
  const int gyl = ghost_mode(bylo, false), gyh = ghost_mode(byhi, false);

  // neighbour columns of ring 0: lane l holds plane l & 15 of column
  // 62k - 2 (l & 16 == 0) or 62k + 63, with the x ghost rule in the address
  const int ep = lane & 15, e = (lane >> 4) & 1;
  const int ecol = e ? C0 - 1 : 0;
  const double* eptr;
  long long estride;
  {
    const int ex = strip * OSTRIP - 2 + (e ? 65 : 0);
    const Src es = (ex < nx + 2) ? resolve(ex, nx, c.bc[0], c.bc[1], 0) : Src{nx - 1, 0, -1};
    if (es.mode == 2) {
      eptr = &cold->ghost[es.side][ep];
      estride = 0;
    } else {
      const int pl = (es.mode == 1) ? lane_table(MIRROR_X, ep) : ep;
      eptr = F.fin + (long long)pl * F.plane + es.idx;
      estride = F.pitch;
    }
  }
  const double evx = (double)lane_table(VX, ep), evy = (double)lane_table(VY, ep);

  auto to_ring0 = [&](int slot, const double* f, double ev) {
    double ux, uy;
    velocity_of(f, ux, uy);
#pragma unroll
    for (int i = 0; i < 16; ++i) ring0[slot][i][lane + 1] = f[i];
    ring0[slot][16][lane + 1] = ux;
    ring0[slot][17][lane + 1] = uy;
    ring0[slot][ep][ecol] = ev;
    const double er = row16_sum(ev), ejx = row16_sum(evx * ev), ejy = row16_sum(evy * ev);
    const double ir = 1.0 / er;
    ring0[slot][16][ecol] = ejx * ir;
    ring0[slot][17][ecol] = ejy * ir;
  };
  auto load_row = [&](int yr, double* f, double& ev) {
    const int yi = ysrc(min(yr, ylast)).idx;
    load_raw(F, sx.idx, yi, f);
    ev = eptr[yi * estride];
  };
  auto enter_row = [&](int yr, double* f, double ev) {
    fix_ghost(cold, sx, ysrc(yr), f);
    to_ring0((unsigned)(yr - base0) % R, f, ev);
  };

  // Prologue: ring 0 rows y0-2 .. y0+W-1 (wave w fills slots w and w + W < R).
  {
    double pa[16], pb[16], ea, eb = 0.0;
    const bool two = w < R - W;
    load_row(base0 + w, pa, ea);
    if (two) load_row(base0 + w + W, pb, eb);
    if (base0 + w <= ylast) enter_row(base0 + w, pa, ea);
    if (two && base0 + w + W <= ylast) enter_row(base0 + w + W, pb, eb);
  }
  // level-n row entering ring 0 at the end of iteration i: y0 + W + iW + w
  double fa[16], fb[16], xa, xb;
  load_row(y0 + W + w, fa, xa);

  bool ok = true;
  // Level n+1 at row `rs` from ring 0, for this lane's column.
  auto level1 = [&](int rs, double* out, double& ux, double& uy) {
    const int s0 = (unsigned)(rs - base0) % R, sp = (unsigned)(rs + 1 - base0) % R,
              sm = (unsigned)(rs - 1 - base0) % R;
    // the collision's long dependency chain first; the convection's LDS
    // reads and arithmetic can then fill its latencies
    double f[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) f[i] = ring0[s0][i][lane + 1];
    NbrVel nv;
    nv.ux_xp = ring0[s0][16][lane + 2];
    nv.uy_xp = ring0[s0][17][lane + 2];
    nv.ux_xm = ring0[s0][16][lane];
    nv.uy_xm = ring0[s0][17][lane];
    nv.ux_yp = ring0[sp][16][lane + 1];
    nv.uy_yp = ring0[sp][17][lane + 1];
    nv.ux_ym = ring0[sm][16][lane + 1];
    nv.uy_ym = ring0[sm][17][lane + 1];
    double df[16];
    const bool good = collide_delta<VER>(c, f, nv, df);
    ConvLds<0, C0>::run(c, ring0[s0], ring0[sp], ring0[sm], lane + 1, lane + 2, lane, out);
#pragma unroll
    for (int i = 0; i < 16; ++i) out[i] = f[i] + (out[i] + df[i]);
    ok &= good || X < 0 || X >= nx || rs < 0 || rs >= ny;
    velocity_of(out, ux, uy);
  };
  // Writes level n+1 of row `rs` (this lane's column) into ring-1 row `slot`
  // with y rule `ym`, plus the x ghost entries next to the domain's sides.
  auto put_row = [&](int slot, const double* v, double ux, double uy, int ym, int yside) {
    double(*row)[C1] = ring1[slot];
    const bool ghost_l = X == -1 && gxl >= 0, ghost_h = X == nx && gxh >= 0;
    if (!ghost_l && !ghost_h) put_entry<C1>(row, lane, v, ux, uy, ym < 0 ? 0 : ym, cold, yside);
    if (ym < 0) {
      // x ghosts of a node row (a ghost row's x ghosts are never read)
      if (X == 0 && gxl >= 0 && lane > 0) put_entry<C1>(row, lane - 1, v, ux, uy, gxl, cold, 0);
      if (X == nx - 1 && gxh >= 0 && lane < 63) put_entry<C1>(row, lane + 1, v, ux, uy, gxh, cold, 1);
    }
  };

  for (int i = 0; y0 - 2 + i * W < y1; ++i) {
    // next level-n row in flight while this iteration computes
    load_row(y0 + 2 * W + i * W + w, fb, xb);
    __syncthreads();
    // level n+1 at row a
    const int a = y0 - 1 + i * W + w;
    if (a <= y1) {
      double v[16] = {}, ux = 0.0, uy = 0.0;
      const int slot = (unsigned)(a - base1) % R;
      if (a >= 0 && a < ny) {
        level1(a, v, ux, uy);
        put_row(slot, v, ux, uy, -1, 0);
      } else if ((a < 0 ? gyl : gyh) < 0) {
        // periodic: a ghost row is an image of a node row, computed as one
        level1(a, v, ux, uy);
        put_row(slot, v, ux, uy, -1, 0);
      } else {
        // non-periodic ghost row from its boundary row rb
        const int rb = a < 0 ? 0 : ny - 1;
        const int ym = a < 0 ? gyl : gyh;
        if (ym != 3) {
          if (rb - 1 >= base0 + i * W) {
            level1(rb, v, ux, uy);  // boundary row's inputs are in ring 0: compute it again
          } else {
            // computed in the previous iteration: read it back
            const int sb = (unsigned)(rb - base1) % R;
#pragma unroll
            for (int k = 0; k < 16; ++k) v[k] = ring1[sb][k][lane];
            ux = ring1[sb][16][lane];
            uy = ring1[sb][17][lane];
          }
        }
        put_row(slot, v, ux, uy, ym, a < 0 ? 2 : 3);
      }
    }
    __syncthreads();
    // ring 0 rows a-1 .. are no longer read: the row loaded last iteration enters
    {
      const int yn = y0 + W + i * W + w;
      if (yn <= ylast) enter_row(yn, fa, xa);
#pragma unroll
      for (int k = 0; k < 16; ++k) fa[k] = fb[k];
      xa = xb;
    }
    // level n+2 at row b = a - 1
    const int b = a - 1;
    if (b >= y0 && b < y1) {
      const int t0 = (unsigned)(b - base1) % R, tp = (unsigned)(b + 1 - base1) % R,
                tm = (unsigned)(b - 1 - base1) % R;
      const int cl = lane > 0 ? lane - 1 : 0, cr = lane < 63 ? lane + 1 : 63;
      double f[16];
#pragma unroll
      for (int k = 0; k < 16; ++k) f[k] = ring1[t0][k][lane];
      NbrVel nv;
      nv.ux_xp = ring1[t0][16][cr];
      nv.uy_xp = ring1[t0][17][cr];
      nv.ux_xm = ring1[t0][16][cl];
      nv.uy_xm = ring1[t0][17][cl];
      nv.ux_yp = ring1[tp][16][lane];
      nv.uy_yp = ring1[tp][17][lane];
      nv.ux_ym = ring1[tm][16][lane];
      nv.uy_ym = ring1[tm][17][lane];
      double df[16], out[16];
      const bool good = collide_delta<VER>(c, f, nv, df);
      ConvLds<0, C1>::run(c, ring1[t0], ring1[tp], ring1[tm], lane, cr, cl, out);
#pragma unroll
      for (int k = 0; k < 16; ++k) out[k] = f[k] + (out[k] + df[k]);
      const bool store = lane >= 1 && lane <= OSTRIP && X < nx;
      ok &= good || !store;
      if (store) {
        if constexpr (NT)
          store_node_stream(F, X, b, out);
        else
          store_node(F, X, b, out);
      }
    }
  }
  if (!ok) flag[0] = 1;
}

template <int VER, int W, bool NT>
__global__ __launch_bounds__(64 * W, 1) void k_step_fused2(Field F, const Hot* __restrict__ hot,
                                                            const Cold* __restrict__ cold, March2Geom g, int* flag) {
  const int tile = xcd_tile2(blockIdx.x, g);
  if (tile >= g.ntiles) return;  // whole workgroup leaves together
  fused2_tile<VER, W, NT>(F, hot, cold, g, tile, flag);
}

}  // namespace lbm
