// Step kernels of one problem: the fused row-marching kernel and the plain
// one-thread-per-node reference kernel, plus init / moments kernels.
#pragma once

#include <type_traits>

#include "lbm_step.h"

namespace lbm {

// Launch-time view of one problem's distributions.
struct Field {
  const double* __restrict__ fin;
  double* __restrict__ fout;
  int nx, ny;
  long long pitch;  // doubles between rows
  long long plane;  // doubles between velocity planes
};

// Ghost-aware source of a stencil point along one axis: index actually read
// and how its velocities are treated (0 as stored, 1 mirrored, 2 replaced by
// the equilibrium ghost of side `side`).
struct Src {
  int idx;
  int mode;
  int side;
};

// Ghost layers are up to two deep (radius-2 scheme): a periodic ghost wraps,
// a zero-gradient ghost repeats the boundary node, a mirror ghost takes the
// mirror image about the wall half a spacing outside the boundary node
// (-1 -> 0, -2 -> 1), a fixed-state ghost is that state's equilibrium.
LBM_HD Src resolve(int i, int n, int bc_lo, int bc_hi, int side_lo) {
  Src s{i, 0, -1};
  if (i < 0) {
    s.side = side_lo;
    switch (bc_lo) {
      case BC_PERIODIC: s.idx = ((i % n) + n) % n; break;
      case BC_SPECULAR: s.idx = min(-1 - i, n - 1); s.mode = 1; break;
      case BC_DIRICHLET_EQ: s.idx = 0; s.mode = 2; break;
      default: s.idx = 0; break;  // zero-gradient; a NEQ-wall side's ghost is never used
    }
  } else if (i >= n) {
    s.side = side_lo + 1;
    switch (bc_hi) {
      case BC_PERIODIC: s.idx = i % n; break;
      case BC_SPECULAR: s.idx = max(2 * n - 1 - i, 0); s.mode = 1; break;
      case BC_DIRICHLET_EQ: s.idx = n - 1; s.mode = 2; break;
      default: s.idx = n - 1; break;
    }
  }
  return s;
}

// Raw distributions of stored node (col, row), no ghost treatment.
__device__ __forceinline__ void load_raw(const Field& F, int col, int row, double* f) {
  const double* p = F.fin + (long long)row * F.pitch + col;
#pragma unroll
  for (int i = 0; i < 16; ++i) f[i] = p[i * F.plane];
}

// Turns the raw values of the stored node a ghost point reads into the ghost
// values: mirrored velocities, or the fixed-state equilibrium.
__device__ __forceinline__ void fix_ghost(const Cold* __restrict__ cold, const Src& sx, const Src& sy, double* f) {
  if (__builtin_expect((sx.mode | sy.mode) != 0, 0)) {
    if (sx.mode == 2 || sy.mode == 2) {
      const int side = (sx.mode == 2) ? sx.side : sy.side;
#pragma unroll
      for (int i = 0; i < 16; ++i) f[i] = cold->ghost[side][i];
    } else {
      double t[16];
#pragma unroll
      for (int i = 0; i < 16; ++i) t[i] = f[i];
      if (sy.mode == 1) {
#pragma unroll
        for (int i = 0; i < 16; ++i) f[i] = t[MIRROR_Y[i]];
#pragma unroll
        for (int i = 0; i < 16; ++i) t[i] = f[i];
      }
      if (sx.mode == 1) {
#pragma unroll
        for (int i = 0; i < 16; ++i) f[i] = t[MIRROR_X[i]];
      }
    }
  }
}

// Distributions of the stencil point (column sx, row sy) after ghost resolution.
__device__ __forceinline__ void load_point(const Field& F, const Cold* __restrict__ cold, const Src& sx, const Src& sy,
                                           double* f) {
  load_raw(F, sx.idx, sy.idx, f);
  fix_ghost(cold, sx, sy, f);
}

LBM_HD bool is_wall_node(const Hot& c, int x, int y, int nx, int ny) {
  return (c.bc[0] == BC_NEQ_WALL && x == 0) || (c.bc[1] == BC_NEQ_WALL && x == nx - 1) ||
         (c.bc[2] == BC_NEQ_WALL && y == 0) || (c.bc[3] == BC_NEQ_WALL && y == ny - 1);
}

__device__ __forceinline__ void store_node(const Field& F, int x, int y, const double* v) {
  double* p = F.fout + (long long)y * F.pitch + x;
#pragma unroll
  for (int i = 0; i < 16; ++i) p[i * F.plane] = v[i];
}

// Streaming store of a node's new distributions: they are not read again in
// this launch, so keep them from displacing halo rows in the caches.
__device__ __forceinline__ void store_node_stream(const Field& F, int x, int y, const double* v) {
  double* p = F.fout + (long long)y * F.pitch + x;
#pragma unroll
  for (int i = 0; i < 16; ++i) __builtin_nontemporal_store(v[i], p + i * F.plane);
}

// Writes the NEQ wall node(s) fed by interior node (x, y) whose new
// distributions are `out`.
template <int VER>
__device__ __forceinline__ void walls_from(const Field& F, const Hot& c, const Cold* __restrict__ cold, int x, int y,
                                           const double* out) {
  const bool lo_y = c.bc[2] == BC_NEQ_WALL && y == 1;
  const bool hi_y = c.bc[3] == BC_NEQ_WALL && y == F.ny - 2;
  const bool lo_x = c.bc[0] == BC_NEQ_WALL && x == 1;
  const bool hi_x = c.bc[1] == BC_NEQ_WALL && x == F.nx - 2;
  if (__builtin_expect(lo_y | hi_y | lo_x | hi_x, 0)) {
    double fw[16];
    if (lo_y) {
      neq_wall<VER>(cold->wall[2], out, fw);
      store_node(F, x, 0, fw);
    }
    if (hi_y) {
      neq_wall<VER>(cold->wall[3], out, fw);
      store_node(F, x, F.ny - 1, fw);
    }
    if (lo_x) {
      neq_wall<VER>(cold->wall[0], out, fw);
      store_node(F, 0, y, fw);
    }
    if (hi_x) {
      neq_wall<VER>(cold->wall[1], out, fw);
      store_node(F, F.nx - 1, y, fw);
    }
  }
}

// Copies the problem coefficients into LDS. Reading them from LDS at each
// use (the row loop's barriers keep the compiler from hoisting the reads)
// keeps ~30 doubles out of the scalar register file.
__device__ __forceinline__ void stage_hot(const Hot* __restrict__ src, Hot* dst) {
  static_assert(sizeof(Hot) % 8 == 0, "Hot is copied as doubles");
  constexpr int n = sizeof(Hot) / 8;
  const double* s = reinterpret_cast<const double*>(src);
  double* d = reinterpret_cast<double*>(dst);
  for (int t = threadIdx.x; t < n; t += blockDim.x) d[t] = s[t];
  __syncthreads();
}

// ---------------------------------------------------------------------------
// Plain kernel: one thread per node, every stencil point read from global
// memory and its velocity recomputed. Reference for the fused kernel.
// ---------------------------------------------------------------------------
template <int VER>
__global__ __launch_bounds__(256) void k_step_plain(Field F, const Hot* __restrict__ hot,
                                                    const Cold* __restrict__ cold, int* flag) {
  __shared__ Hot hs;
  stage_hot(hot, &hs);
  const Hot& c = hs;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  if (x >= F.nx || y >= F.ny) return;
  if (is_wall_node(c, x, y, F.nx, F.ny)) return;
  const Src cx = resolve(x, F.nx, c.bc[0], c.bc[1], 0);
  const Src cy = resolve(y, F.ny, c.bc[2], c.bc[3], 2);
  double f[16], fxp[16], fxm[16], fyp[16], fym[16];
  load_point(F, cold, cx, cy, f);
  load_point(F, cold, resolve(x + 1, F.nx, c.bc[0], c.bc[1], 0), cy, fxp);
  load_point(F, cold, resolve(x - 1, F.nx, c.bc[0], c.bc[1], 0), cy, fxm);
  load_point(F, cold, cx, resolve(y + 1, F.ny, c.bc[2], c.bc[3], 2), fyp);
  load_point(F, cold, cx, resolve(y - 1, F.ny, c.bc[2], c.bc[3], 2), fym);
  NbrVel nv;
  velocity_of(fxp, nv.ux_xp, nv.uy_xp);
  velocity_of(fxm, nv.ux_xm, nv.uy_xm);
  velocity_of(fyp, nv.ux_yp, nv.uy_yp);
  velocity_of(fym, nv.ux_ym, nv.uy_ym);
  double out[16];
  bool ok;
  if (c.scheme == 1) {  // flux-limited: second neighbours too
    double fxp2[16], fxm2[16], fyp2[16], fym2[16];
    load_point(F, cold, resolve(x + 2, F.nx, c.bc[0], c.bc[1], 0), cy, fxp2);
    load_point(F, cold, resolve(x - 2, F.nx, c.bc[0], c.bc[1], 0), cy, fxm2);
    load_point(F, cold, cx, resolve(y + 2, F.ny, c.bc[2], c.bc[3], 2), fyp2);
    load_point(F, cold, cx, resolve(y - 2, F.ny, c.bc[2], c.bc[3], 2), fym2);
#pragma unroll
    for (int i = 0; i < 16; ++i)
      out[i] = convect_limited_i(c, i, f[i], fxm2[i], fxm[i], fxp[i], fxp2[i], fym2[i], fym[i], fyp[i], fyp2[i]);
    ok = collide_add<VER>(c, f, nv, out);
  } else {
    ok = node_update<VER>(c, f, fxp, fxm, fyp, fym, nv, out);
  }
  if (!ok) flag[0] = 1;
  store_node(F, x, y, out);
  walls_from<VER>(F, c, cold, x, y, out);
}

// ---------------------------------------------------------------------------
// Fused kernel. A workgroup of W wavefronts (2 or 4) owns a tile of STRIP =
// 64 columns (one per lane, 512-byte aligned rows) by `rows` rows and marches
// up it W rows at a time. With a stencil of radius HR (1: Lax-Wendroff; 2:
// its flux-limited form), rows y-HR .. y+W-1+HR live in a ring of W + 2 HR
// rows in LDS, each STRIP + 2 HR entries wide: the HR neighbour columns left
// of the strip, the 64 strip columns, the HR neighbour columns right of it,
// with 16 distributions and the velocity per entry. Each distribution is read
// from HBM about once and every lane stores a node (columns past nx land in
// the row padding), so the stores are full, aligned lines. Each wave keeps
// its next row in flight in registers while it computes the current one; the
// neighbour columns of a row come with one extra load (lane l holds plane
// l & 15 of neighbour column (l >> 4) mod 2 HR) and their velocities from a
// sum over the 16 lanes of a DPP row.
// ---------------------------------------------------------------------------
constexpr int STRIP = 64;
constexpr int WAVES = 4;  // wavefronts per workgroup of the default tile shape
constexpr int NV = 18;    // 16 distributions + u_x + u_y per ring entry

// Convection of all 16 velocities with the stencil values read from the LDS
// ring rows (current row r0, rows above/below rp/rm) as they are needed; c0,
// cp, cm are the ring columns of the node and its x+1 / x-1 neighbours.
template <int I, int RWT>
struct ConvLds {
  __device__ __forceinline__ static void run(const Hot& c, const double (*r0)[RWT], const double (*rp)[RWT],
                                             const double (*rm)[RWT], int c0, int cp, int cm, double* out) {
    out[I] = convect<I>(c, r0[I][c0], VX[I] ? r0[I][cp] : 0.0, VX[I] ? r0[I][cm] : 0.0,
                        VY[I] ? rp[I][c0] : 0.0, VY[I] ? rm[I][c0] : 0.0);
    ConvLds<I + 1, RWT>::run(c, r0, rp, rm, c0, cp, cm, out);
  }
};
template <int RWT>
struct ConvLds<16, RWT> {
  __device__ __forceinline__ static void run(const Hot&, const double (*)[RWT], const double (*)[RWT],
                                             const double (*)[RWT], int, int, int, double*) {}
};

// The same for the flux-limited scheme: rows y-2 .. y+2 (r2m .. r2p) and
// columns c0-2 .. c0+2.
template <int I, int RWT>
struct ConvLim {
  __device__ __forceinline__ static void run(const Hot& c, const double (*r2m)[RWT], const double (*r1m)[RWT],
                                             const double (*r0)[RWT], const double (*r1p)[RWT],
                                             const double (*r2p)[RWT], int c0, double* out) {
    out[I] = convect_limited<I>(c, r0[I][c0], VX[I] ? r0[I][c0 - 2] : 0.0, VX[I] ? r0[I][c0 - 1] : 0.0,
                                VX[I] ? r0[I][c0 + 1] : 0.0, VX[I] ? r0[I][c0 + 2] : 0.0,
                                VY[I] ? r2m[I][c0] : 0.0, VY[I] ? r1m[I][c0] : 0.0, VY[I] ? r1p[I][c0] : 0.0,
                                VY[I] ? r2p[I][c0] : 0.0);
    ConvLim<I + 1, RWT>::run(c, r2m, r1m, r0, r1p, r2p, c0, out);
  }
};
template <int RWT>
struct ConvLim<16, RWT> {
  __device__ __forceinline__ static void run(const Hot&, const double (*)[RWT], const double (*)[RWT],
                                             const double (*)[RWT], const double (*)[RWT], const double (*)[RWT], int,
                                             double*) {}
};

// Lane value from another lane of the same row of 16 (DPP control CTRL).
template <int CTRL>
__device__ __forceinline__ double dpp_move(double v) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_mov_dpp((int)b, CTRL, 0xF, 0xF, false);
  const int hi = __builtin_amdgcn_mov_dpp((int)(b >> 32), CTRL, 0xF, 0xF, false);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sum over each row of 16 lanes; every lane of the row gets the same value
// (xor-1 and xor-2 quad swaps, then half-row and row mirrors).
__device__ __forceinline__ double row16_sum(double v) {
  v += dpp_move<0xB1>(v);
  v += dpp_move<0x4E>(v);
  v += dpp_move<0x141>(v);
  v += dpp_move<0x140>(v);
  return v;
}

__device__ __forceinline__ int lane_table(const int (&t)[16], int i) {
  int r = 0;
#pragma unroll
  for (int k = 0; k < 16; ++k) r = (i == k) ? t[k] : r;
  return r;
}

struct MarchGeom {
  int nstrips;  // ceil(nx / STRIP)
  int rows;     // rows per tile (multiple of the workgroup's wavefront count)
  int nsegs;    // ceil(ny / rows)
  int ntiles;   // nstrips * nsegs
  int per_xcd;  // ceil(ntiles / 8)
};

// Workgroups are dealt to the 8 XCDs round-robin; give each XCD a contiguous
// run of tiles (x fastest) so tiles sharing halo rows and columns use the
// same L2.
__device__ __forceinline__ int xcd_tile(int b, const MarchGeom& g) { return (b % 8) * g.per_xcd + b / 8; }

// One tile (index `tile` < g.ntiles) of one problem, computed by a workgroup
// of W wavefronts (2 or 4); HR stencil radius (1: Lax-Wendroff, 2:
// flux-limited); the ring holds RING = W + 2 HR rows.
// NT: non-temporal stores (the new distributions are not kept in the caches;
// the better choice when the two buffers exceed the caches), else ordinary
// stores (a grid that fits the caches reads them back from there next step).
template <int VER, bool WALLS, int W, int HR, bool NT = true>
__device__ __forceinline__ void fused_tile(Field F, const Hot* __restrict__ hot, const Cold* __restrict__ cold,
                                           MarchGeom g, int tile, int* flag) {
  constexpr int WAVES = W;
  constexpr int RING = W + 2 * HR;
  constexpr int RWT = STRIP + 2 * HR;
  static_assert(HR == 1 || HR == 2, "stencil radius 1 or 2");
  static_assert(!WALLS || HR == 1, "NEQ walls with the radius-1 scheme only");
  __shared__ double ring[RING][NV][RWT];
  __shared__ Hot hs;
  stage_hot(hot, &hs);
  const Hot& c = hs;
  const int lane = threadIdx.x & 63;
  // wave index and everything derived from rows are wave-uniform: keep them
  // in scalar registers
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int strip = tile % g.nstrips, seg = tile / g.nstrips;
  const int x0 = strip * STRIP;
  const int x = x0 + lane;
  const int y0 = seg * g.rows;
  const int y1 = min(y0 + g.rows, F.ny);
  const int ylast = y1 - 1 + HR;  // last ring row the tile reads
  // this lane's column: x = nx .. nx+HR-1 are right ghosts; lanes past them
  // read column nx-1 and store into the row padding
  const Src sx = (x < F.nx + HR) ? resolve(x, F.nx, c.bc[0], c.bc[1], 0) : Src{F.nx - 1, 0, -1};
  const int c0 = lane + HR;  // ring column of this lane's node
  const int base = y0 - HR;  // row held in ring slot 0 at the start
  // ghost rows below and above the domain (scalar reads of the BC codes)
  const int bylo = __builtin_amdgcn_readfirstlane(hot->bc[2]);
  const int byhi = __builtin_amdgcn_readfirstlane(hot->bc[3]);
  // the (at most HR) ghost rows on each side, resolved once
  const Src ylo1 = resolve(-1, F.ny, bylo, byhi, 2), yhi1 = resolve(F.ny, F.ny, bylo, byhi, 2);
  const Src ylo2 = HR > 1 ? resolve(-2, F.ny, bylo, byhi, 2) : ylo1;
  const Src yhi2 = HR > 1 ? resolve(F.ny + 1, F.ny, bylo, byhi, 2) : yhi1;
  auto ysrc = [&](int yr) -> Src {
    if (yr < 0) return (HR > 1 && yr < -1) ? ylo2 : ylo1;
    if (yr >= F.ny) return (HR > 1 && yr > F.ny) ? yhi2 : yhi1;
    return Src{yr, 0, -1};
  };

  // neighbour-column value of this lane: plane ep of neighbour column e
  // (ring column ecol, grid column x0 - HR + ecol), with the x ghost rule
  // folded into the address (mirror: mirrored plane; fixed state: the ghost
  // value, same for every row). Only rows inside the domain use these
  // columns, so no y ghost rule is needed.
  const int ep = lane & 15, e = (lane >> 4) & (2 * HR - 1);
  const int ecol = (e < HR) ? e : STRIP + e;
  const double* eptr;
  long long estride;
  {
    const int ex = x0 - HR + ecol;
    const Src es = (ex < F.nx + HR) ? resolve(ex, F.nx, c.bc[0], c.bc[1], 0) : Src{F.nx - 1, 0, -1};
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

  auto to_ring = [&](int slot, const double* f, double ev) {
    double ux, uy;
    velocity_of(f, ux, uy);
#pragma unroll
    for (int i = 0; i < 16; ++i) ring[slot][i][c0] = f[i];
    ring[slot][16][c0] = ux;
    ring[slot][17][c0] = uy;
    // neighbour columns: every lane of a DPP row writes the same values
    ring[slot][ep][ecol] = ev;
    const double er = row16_sum(ev), ejx = row16_sum(evx * ev), ejy = row16_sum(evy * ev);
    const double ir = 1.0 / er;
    ring[slot][16][ecol] = ejx * ir;
    ring[slot][17][ecol] = ejy * ir;
  };

  // Prologue: ring rows y0-HR .. y0+W-1+HR (only those <= ylast are ever
  // read); wave w fills slots w and w + W (< RING). Every load of the
  // prologue and of the first prefetch row is issued before any is used.
  static_assert(RING - WAVES <= WAVES, "each wave fills at most two prologue slots");
  const bool two = w < RING - WAVES;
  const int ya = min(base + w, ylast), yb = min(base + w + WAVES, ylast);
  double pa[16], pb[16], pea, peb = 0.0;
  {
    const int ia = ysrc(ya).idx;
    load_raw(F, sx.idx, ia, pa);
    pea = eptr[ia * estride];
    if (two) {
      const int ib = ysrc(yb).idx;
      load_raw(F, sx.idx, ib, pb);
      peb = eptr[ib * estride];
    }
  }

  // Each wave keeps two rows in flight: `cur` (written to the ring at the
  // end of this iteration) and `nxt` (issued now, written next iteration).
  // Loads are plain (no ghost treatment, no branch: a row past the tile end
  // is clamped to the last row read); the ghost fix-up runs when the row
  // enters the ring, after its data has arrived. FULL iterations (every wave
  // has a row to compute and one to enter) have no branches around stores
  // and loads, so the waits before the ring entry cover only `cur`.
  double fa[16], fb[16], ea, eb;
  {
    const int yn = min(y0 + WAVES + HR + w, ylast);
    const int yi = ysrc(yn).idx;
    load_raw(F, sx.idx, yi, fa);
    ea = eptr[yi * estride];
  }
  if (base + w <= ylast) {
    fix_ghost(cold, sx, ysrc(base + w), pa);
    to_ring(w, pa, pea);
  }
  if (two && base + w + WAVES <= ylast) {
    fix_ghost(cold, sx, ysrc(base + w + WAVES), pb);
    to_ring(w + WAVES, pb, peb);
  }
  bool ok = true;
  auto iteration = [&](auto full, int Y, double* cur, double& ecur, double* nxt, double& enxt) {
    constexpr bool FULL = decltype(full)::value;
    {
      const int yi = ysrc(min(Y + 2 * WAVES + HR + w, ylast)).idx;
      load_raw(F, sx.idx, yi, nxt);
      enxt = eptr[yi * estride];
    }
    __syncthreads();
    const int y = Y + w;
    if (FULL || y < y1) {
      if (!WALLS || !is_wall_node(c, x, y, F.nx, F.ny)) {
        const int s0 = (y - base) % RING, sp = (y + 1 - base) % RING, sm = (y - 1 - base) % RING;
        double out[16];
        // convection first, reading each neighbour value from LDS as it is used
        if constexpr (HR == 1) {
          ConvLds<0, RWT>::run(c, ring[s0], ring[sp], ring[sm], c0, c0 + 1, c0 - 1, out);
        } else {
          const int sp2 = (y + 2 - base) % RING, sm2 = (y - 2 - base) % RING;
          ConvLim<0, RWT>::run(c, ring[sm2], ring[sm], ring[s0], ring[sp], ring[sp2], c0, out);
        }
        double f[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) f[i] = ring[s0][i][c0];
        NbrVel nv;
        nv.ux_xp = ring[s0][16][c0 + 1];
        nv.uy_xp = ring[s0][17][c0 + 1];
        nv.ux_xm = ring[s0][16][c0 - 1];
        nv.uy_xm = ring[s0][17][c0 - 1];
        nv.ux_yp = ring[sp][16][c0];
        nv.uy_yp = ring[sp][17][c0];
        nv.ux_ym = ring[sm][16][c0];
        nv.uy_ym = ring[sm][17][c0];
        ok &= collide_add<VER>(c, f, nv, out) || x >= F.nx;
        if constexpr (NT)
          store_node_stream(F, x, y, out);
        else
          store_node(F, x, y, out);
        if (WALLS) walls_from<VER>(F, c, cold, x, y, out);
      }
    }
    __syncthreads();
    const int yn = Y + WAVES + HR + w;
    if (FULL || yn <= ylast) {
      fix_ghost(cold, sx, ysrc(yn), cur);
      to_ring((yn - base) % RING, cur, ecur);
    }
  };
  using Full = std::integral_constant<bool, true>;
  using Part = std::integral_constant<bool, false>;
  int Y = y0;
  for (; Y + 3 * WAVES <= y1; Y += 2 * WAVES) {
    iteration(Full{}, Y, fa, ea, fb, eb);
    iteration(Full{}, Y + WAVES, fb, eb, fa, ea);
  }
  for (; Y < y1; Y += 2 * WAVES) {
    iteration(Part{}, Y, fa, ea, fb, eb);
    if (Y + WAVES >= y1) break;
    iteration(Part{}, Y + WAVES, fb, eb, fa, ea);
  }
  if (!ok) flag[0] = 1;
}

template <int VER, bool WALLS, int W, int HR, bool NT>
__global__ __launch_bounds__(64 * W, 2) void k_step_fused(Field F, const Hot* __restrict__ hot,
                                                           const Cold* __restrict__ cold, MarchGeom g, int* flag) {
  const int tile = xcd_tile(blockIdx.x, g);
  if (tile >= g.ntiles) return;  // whole workgroup leaves together
  fused_tile<VER, WALLS, W, HR, NT>(F, hot, cold, g, tile, flag);
}

// ---------------------------------------------------------------------------
// Streaming probe: copies 16 pitched planes with the fused kernel's access
// pattern (64-column strips, WAVES wavefronts on consecutive rows, the next
// row in flight, non-temporal stores) and no arithmetic; its bandwidth is
// what a kernel with this access pattern can reach.
// ---------------------------------------------------------------------------
// (template only so that every translation unit gets its own instance)
template <int U>
__global__ __launch_bounds__(64 * WAVES) void k_stream_copy(const double* __restrict__ src, double* __restrict__ dst,
                                                            int ny, long long pitch, int rows, int nstrips,
                                                            int ntiles) {
  const int tile = blockIdx.x;
  if (tile >= ntiles) return;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int strip = tile % nstrips, seg = tile / nstrips;
  const int y0 = seg * rows, y1 = min(y0 + rows, ny);
  const long long plane = (long long)ny * pitch;
  const int x = strip * STRIP + lane;
  double a[16], b[16];
  auto load = [&](int y, double* v) {
    const double* p = src + (long long)y * pitch + x;
#pragma unroll
    for (int i = 0; i < 16; ++i) v[i] = p[i * plane];
  };
  auto store = [&](int y, const double* v) {
    double* q = dst + (long long)y * pitch + x;
#pragma unroll
    for (int i = 0; i < 16; ++i) __builtin_nontemporal_store(v[i], q + i * plane);
  };
  load(min(y0 + w, y1 - 1), a);
  for (int y = y0 + w; y < y1; y += 2 * WAVES) {
    load(min(y + WAVES, y1 - 1), b);
    store(y, a);
    if (y + WAVES >= y1) break;
    load(min(y + 2 * WAVES, y1 - 1), a);
    store(y + WAVES, b);
  }
}

// ---------------------------------------------------------------------------
// Initial state and output moments.
// ---------------------------------------------------------------------------
template <int VER>
__global__ void k_init(Field F, const double* __restrict__ rho, const double* __restrict__ ux,
                       const double* __restrict__ uy, const double* __restrict__ T) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= F.nx) return;
  const long long k = (long long)y * F.nx + x;
  double f[16];
  equilibrium_f<VER>(rho[k], ux[k], uy[k], T[k], f);
  double* p = F.fout + (long long)y * F.pitch + x;
#pragma unroll
  for (int i = 0; i < 16; ++i) p[i * F.plane] = f[i];
}

// (template only so that every translation unit gets its own instance)
template <int U>
__global__ void k_moments(Field F, double* rho, double* ux, double* uy, double* T, double* P) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= F.nx) return;
  const double* p = F.fin + (long long)y * F.pitch + x;
  double f[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) f[i] = p[i * F.plane];
  double m[16];
  moments_from_f(f, m);
  const double r = m[0], ir = 1.0 / r;
  const double u = m[1] * ir, v = m[2] * ir;
  const double t = m[3] * ir - 0.5 * (u * u + v * v);
  const long long k = (long long)y * F.nx + x;
  if (rho) rho[k] = r;
  if (ux) ux[k] = u;
  if (uy) uy[k] = v;
  if (T) T[k] = t;
  if (P) P[k] = r * t;
}

}  // namespace lbm
