// Batched form: many independent one-dimensional problems (a Riemann line
// along x with ny = 1, or a Couette column along y with nx = 1) advanced
// together. A workgroup owns one chunk of one instance, loads the chunk plus
// a halo of h nodes on each side into LDS and advances it h time steps
// there; the halo shrinks by one node per step (the stencil has radius 1), so
// after h steps the chunk itself is exact and is written back. Instances that
// fit one region need no halo at all (their ends are physical boundaries).
// Each node update is the same arithmetic as the single-problem kernels.
#pragma once

#include "lbm_kernels.h"

namespace lbm {

struct LineInst {
  long long off;  // offset (doubles) of plane 0 in each arena buffer
  int N;          // nodes along the line
  int stride;     // doubles between velocity planes
  int axis;       // 0: along x (ny == 1); 1: along y (nx == 1)
  int walls;      // 1 if an end is a NEQ wall
  Hot hot;
  Cold cold;
};

struct LineChunk {
  int inst;
  int start;
  int len;
  int pad;
};

// Ghost of line end `end` (0 low, 1 high) from the end node's distributions.
__device__ __forceinline__ void line_ghost(const LineInst& I, const Hot& c, int end, const double* fe, double* g) {
  const int side = 2 * I.axis + end;
  const int kind = c.bc[side];
  if (kind == BC_SPECULAR) {
#pragma unroll
    for (int i = 0; i < 16; ++i) g[i] = I.axis == 0 ? fe[MIRROR_X[i]] : fe[MIRROR_Y[i]];
  } else if (kind == BC_DIRICHLET_EQ) {
#pragma unroll
    for (int i = 0; i < 16; ++i) g[i] = I.cold.ghost[side][i];
  } else {  // zero-gradient (periodic lines are handled by wrapping inside the region)
#pragma unroll
    for (int i = 0; i < 16; ++i) g[i] = fe[i];
  }
}

template <int VER, int REGION>
__global__ __launch_bounds__(REGION, 2) void k_batch_line(const double* __restrict__ A, double* __restrict__ B,
                                                          const LineInst* __restrict__ insts,
                                                          const LineChunk* __restrict__ chunks,
                                                          const int* __restrict__ budget, int n0, int h,
                                                          int* flag) {
  __shared__ double buf[2][NV][REGION];
  __shared__ Hot hs;
  const LineChunk ch = chunks[blockIdx.x];
  const LineInst& I = insts[ch.inst];
  const int t = threadIdx.x;
  const int N = I.N;
  const long long off = I.off;
  const int stride = I.stride;
  int steps = budget[ch.inst] - n0;
  steps = steps < 0 ? 0 : (steps > h ? h : steps);
  if (steps == 0) {  // nothing to do this block: carry the chunk over to the output buffer
    for (int r = t; r < ch.len; r += REGION)
#pragma unroll
      for (int i = 0; i < 16; ++i) B[off + (long long)i * stride + ch.start + r] = A[off + (long long)i * stride + ch.start + r];
    return;
  }
  stage_hot(&I.hot, &hs);
  const Hot& c = hs;
  const bool periodic = c.bc[2 * I.axis] == BC_PERIODIC;  // then the chunk is the whole line
  const int lo = periodic ? 0 : max(ch.start - steps, 0);
  const int hi = periodic ? N : min(ch.start + ch.len + steps, N);
  const int R = hi - lo;  // <= REGION (guaranteed by the chunking)

  // load the region and its velocities
  if (t < R) {
    double f[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) f[i] = A[off + (long long)i * stride + lo + t];
    double ux, uy;
    velocity_of(f, ux, uy);
#pragma unroll
    for (int i = 0; i < 16; ++i) buf[0][i][t] = f[i];
    buf[0][16][t] = ux;
    buf[0][17][t] = uy;
  }
  __syncthreads();
  const int g = lo + t;  // line node of this thread
  const bool wall_lo = c.bc[2 * I.axis] == BC_NEQ_WALL, wall_hi = c.bc[2 * I.axis + 1] == BC_NEQ_WALL;
  bool ok = true;
  int P = 0;
  for (int s = 0; s < steps; ++s) {
    // nodes valid after this step: the region shrinks at ends that are not physical
    const int vlo = (lo == 0) ? 0 : lo + s + 1;
    const int vhi = (hi == N) ? N : hi - s - 1;
    const int Q = P ^ 1;
    const bool is_wall = (wall_lo && g == 0) || (wall_hi && g == N - 1);
    if (t < R && g >= vlo && g < vhi && !is_wall) {
      double f[16], fm[16], fp[16];
      double uxm, uym, uxp, uyp;
#pragma unroll
      for (int i = 0; i < 16; ++i) f[i] = buf[P][i][t];
      // neighbour below
      if (g > 0 || periodic) {
        const int r = (g > 0) ? t - 1 : R - 1;
#pragma unroll
        for (int i = 0; i < 16; ++i) fm[i] = buf[P][i][r];
        uxm = buf[P][16][r];
        uym = buf[P][17][r];
      } else {
        line_ghost(I, c, 0, f, fm);
        velocity_of(fm, uxm, uym);
      }
      if (g < N - 1 || periodic) {
        const int r = (g < N - 1) ? t + 1 : 0;
#pragma unroll
        for (int i = 0; i < 16; ++i) fp[i] = buf[P][i][r];
        uxp = buf[P][16][r];
        uyp = buf[P][17][r];
      } else {
        line_ghost(I, c, 1, f, fp);
        velocity_of(fp, uxp, uyp);
      }
      const double ux0 = buf[P][16][t], uy0 = buf[P][17][t];
      NbrVel nv;
      double out[16];
      if (I.axis == 0) {
        nv = NbrVel{uxp, uyp, uxm, uym, ux0, uy0, ux0, uy0};
        ok &= node_update<VER>(c, f, fp, fm, f, f, nv, out);
      } else {
        nv = NbrVel{ux0, uy0, ux0, uy0, uxp, uyp, uxm, uym};
        ok &= node_update<VER>(c, f, f, f, fp, fm, nv, out);
      }
      double ux, uy;
      velocity_of(out, ux, uy);
#pragma unroll
      for (int i = 0; i < 16; ++i) buf[Q][i][t] = out[i];
      buf[Q][16][t] = ux;
      buf[Q][17][t] = uy;
    }
    __syncthreads();
    if (I.walls) {  // wall nodes from their neighbour's new distributions
      if (t < R && is_wall) {
        const int r = (g == 0) ? t + 1 : t - 1;
        double fn[16], fw[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) fn[i] = buf[Q][i][r];
        neq_wall<VER>(I.cold.wall[2 * I.axis + (g == 0 ? 0 : 1)], fn, fw);
        double ux, uy;
        velocity_of(fw, ux, uy);
#pragma unroll
        for (int i = 0; i < 16; ++i) buf[Q][i][t] = fw[i];
        buf[Q][16][t] = ux;
        buf[Q][17][t] = uy;
      }
      __syncthreads();
    }
    P = Q;
  }
  // write the chunk back
  if (g >= ch.start && g < ch.start + ch.len && t < R) {
#pragma unroll
    for (int i = 0; i < 16; ++i) B[off + (long long)i * stride + g] = buf[P][i][t];
  }
  if (!ok) flag[0] = 1;
}

}  // namespace lbm

namespace lbm {

// A batch instance advanced tile by tile with the fused step kernel: the
// two-dimensional instances, and periodic lines too long for one line region.
// Its planes are pitched like a single problem's ([16][ny][pitch], pitch = nx
// rounded up to 64 doubles, 512-byte aligned).
struct TileInst {
  long long off;     // offset (doubles) of plane 0 in each arena buffer
  long long pitch, plane;
  int nx, ny;
  int gidx;          // index of the instance in the batch (budgets)
  int first_tile;    // index of its first tile in the batch's tile list
  MarchGeom geom;
  Hot hot;
  Cold cold;
};

// One time step of every tile of a group of tile instances (same
// equilibrium version and variant: NEQ walls, or the flux-limited scheme
// with its radius-2 stencil HR = 2); workgroup b takes tile
// (b mod 8) per_xcd + b / 8 of the group's list, so each XCD gets a
// contiguous run. An instance whose budget b is spent (step n >= b of a call
// of nsteps steps) idles: its final state stays where step b - 1 put it, and
// at n == b it is copied across once if the remaining nsteps - b steps are
// odd, so that after the call it sits in the same buffer as everyone else's.
template <int VER, bool WALLS, int HR>
__global__ __launch_bounds__(64 * WAVES, 2) void k_batch_tiles(const double* __restrict__ A, double* __restrict__ B,
                                                                const TileInst* __restrict__ insts,
                                                                const int* __restrict__ tile_inst, int ntiles,
                                                                int per_xcd, const int* __restrict__ budget, int n,
                                                                int nsteps, int* flag) {
  const int t = (blockIdx.x % 8) * per_xcd + blockIdx.x / 8;
  if (t >= ntiles) return;  // whole workgroup leaves together
  const TileInst& I = insts[tile_inst[t]];
  Field F;
  F.fin = A + I.off;
  F.fout = B + I.off;
  F.nx = I.nx;
  F.ny = I.ny;
  F.pitch = I.pitch;
  F.plane = I.plane;
  const int tile = t - I.first_tile;
  const int bud = budget[I.gidx];
  if (bud <= n) {
    if (n != bud || ((nsteps - bud) & 1) == 0) return;
    const int strip = tile % I.geom.nstrips, seg = tile / I.geom.nstrips;
    const int x = strip * STRIP + (threadIdx.x & 63);
    const int y1 = min((seg + 1) * I.geom.rows, I.ny);
    for (int y = seg * I.geom.rows + (threadIdx.x >> 6); y < y1; y += WAVES)
#pragma unroll
      for (int i = 0; i < 16; ++i) F.fout[i * F.plane + (long long)y * F.pitch + x] = F.fin[i * F.plane + (long long)y * F.pitch + x];
    return;
  }
  fused_tile<VER, WALLS, WAVES, HR>(F, &I.hot, &I.cold, I.geom, tile, flag);
}

}  // namespace lbm
