// Batched form: many independent one-dimensional problems (a Riemann line
// along x with ny = 1, or a Couette column along y with nx = 1) advanced
// together. A workgroup owns one chunk of one instance, loads the chunk plus
// a halo of h nodes on each side into LDS and advances it h time steps
// there; the halo shrinks by one node per step (the stencil has radius 1), so
// after h steps the chunk itself is exact and is written back. Instances that
// fit one region need no halo at all (their ends are physical boundaries).
// Each node update is the same arithmetic as the single-problem kernels.
#pragma once

#include "lbm_fused2.h"
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
  int dlo, dhi;  // chunks (list indices) whose output of a block this chunk's next block reads or overwrites
  int pad[3];
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

// One chunk (index ci of the chunk list) for up to h steps from step n0 of
// the call: A -> B. Every thread of the workgroup calls it (it holds
// barriers); returns false if a node lost positivity. With TICKET, thread 0
// also takes the workgroup's next ticket from *ctr once the chunk is loaded
// (so that the atomic's latency hides behind the time steps) and leaves it
// in *tk_out (LDS) at the end.
template <int VER, int REGION, bool TICKET = false>
__device__ __forceinline__ bool line_chunk(const double* __restrict__ A, double* __restrict__ B,
                                           const LineInst* __restrict__ insts, const LineChunk* __restrict__ chunks,
                                           int ci, const int* __restrict__ budget, int n0, int h,
                                           unsigned long long* ctr = nullptr, unsigned long long* tk_out = nullptr) {
  __shared__ double buf[2][NV][REGION];
  __shared__ Hot hs;
  const LineChunk ch = chunks[ci];
  const LineInst& I = insts[ch.inst];
  const int t = threadIdx.x;
  const int N = I.N;
  const long long off = I.off;
  const int stride = I.stride;
  int steps = budget[ch.inst] - n0;
  steps = steps < 0 ? 0 : (steps > h ? h : steps);
  if (steps == 0) {  // nothing to do this block: carry the chunk over to the output buffer
    if (TICKET && t == 0) *tk_out = __hip_atomic_fetch_add(ctr, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    for (int r = t; r < ch.len; r += REGION)
#pragma unroll
      for (int i = 0; i < 16; ++i) B[off + (long long)i * stride + ch.start + r] = A[off + (long long)i * stride + ch.start + r];
    return true;
  }
  stage_hot(&I.hot, &hs);
  const Hot& c = hs;
  const bool periodic = c.bc[2 * I.axis] == BC_PERIODIC;  // then the chunk is the whole line
  const int lo = periodic ? 0 : max(ch.start - steps, 0);
  const int hi = periodic ? N : min(ch.start + ch.len + steps, N);
  const int R = hi - lo;  // <= REGION (guaranteed by the chunking)

  // load the region and its velocities; each thread keeps its node's moments
  // (and 1 / rho) from one step to the next, for the collision and for the
  // velocity its neighbours read
  double m[16], ir = 0.0;
  if (t < R) {
    double f[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) f[i] = A[off + (long long)i * stride + lo + t];
    moments_from_f(f, m);
    ir = 1.0 / m[0];
#pragma unroll
    for (int i = 0; i < 16; ++i) buf[0][i][t] = f[i];
    buf[0][16][t] = m[1] * ir;
    buf[0][17][t] = m[2] * ir;
  }
  __syncthreads();
  unsigned long long next = 0;
  if (TICKET && t == 0) next = __hip_atomic_fetch_add(ctr, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
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
      // the step's arithmetic along the line's axis (the other axis's zero
      // convection terms left out), the collision from the kept moments
      double df[16], out[16];
      if (I.axis == 0) {
        ok &= collide_from_moments<VER>(c, m, ir, NbrVel{uxp, uyp, uxm, uym, ux0, uy0, ux0, uy0}, df);
        ConvAxis<0, 0>::run(c, f, fp, fm, out);
      } else {
        ok &= collide_from_moments<VER>(c, m, ir, NbrVel{ux0, uy0, ux0, uy0, uxp, uyp, uxm, uym}, df);
        ConvAxis<0, 1>::run(c, f, fp, fm, out);
      }
#pragma unroll
      for (int i = 0; i < 16; ++i) out[i] = f[i] + (out[i] + df[i]);
      moments_from_f(out, m);
      ir = 1.0 / m[0];
#pragma unroll
      for (int i = 0; i < 16; ++i) buf[Q][i][t] = out[i];
      buf[Q][16][t] = m[1] * ir;
      buf[Q][17][t] = m[2] * ir;
    }
    __syncthreads();
    if (I.walls) {  // wall nodes from their neighbour's new distributions
      if (t < R && is_wall) {
        const int r = (g == 0) ? t + 1 : t - 1;
        double fn[16], fw[16];
#pragma unroll
        for (int i = 0; i < 16; ++i) fn[i] = buf[Q][i][r];
        neq_wall<VER>(I.cold.wall[2 * I.axis + (g == 0 ? 0 : 1)], fn, fw);
        // its velocity as any node's (from its moments), so that it does not
        // depend on whether the next step reloads the node
        moments_from_f(fw, m);
        ir = 1.0 / m[0];
#pragma unroll
        for (int i = 0; i < 16; ++i) buf[Q][i][t] = fw[i];
        buf[Q][16][t] = m[1] * ir;
        buf[Q][17][t] = m[2] * ir;
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
  if (TICKET && t == 0) *tk_out = next;
  return ok;
}

template <int VER, int REGION>
__global__ __launch_bounds__(REGION, 2) void k_batch_line(const double* __restrict__ A, double* __restrict__ B,
                                                          const LineInst* __restrict__ insts,
                                                          const LineChunk* __restrict__ chunks,
                                                          const int* __restrict__ budget, int n0, int h,
                                                          int* flag) {
  if (!line_chunk<VER, REGION>(A, B, insts, chunks, blockIdx.x, budget, n0, h)) flag[0] = 1;
}

// A value every lane holds alike (read from LDS), marked workgroup-uniform
// so that what derives from it (the chunk and its instance) stays in scalar
// registers and uniform branches.
__device__ __forceinline__ unsigned long long uniform_u64(unsigned long long v) {
  const unsigned lo = __builtin_amdgcn_readfirstlane((unsigned)v);
  const unsigned hi = __builtin_amdgcn_readfirstlane((unsigned)(v >> 32));
  return ((unsigned long long)hi << 32) | lo;
}

// Start of a persistent launch: ticket counter 0, every chunk's epoch -1 (a
// kernel, so that it can sit in a captured graph).
__global__ void k_persist_reset(unsigned long long* ctr, int* epoch, int n) {
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i == 0) *ctr = 0ull;
  if (i < n) epoch[i] = -1;
}

// Persistent form of the line kernel: one launch advances every chunk of
// one equilibrium version through all the ceil(nsteps / h) blocks of h steps
// of a call. The grid holds at most as many workgroups as are resident at
// once. Chunks are handed out in ticket order from one counter (ticket k:
// chunk k mod nchunks of block k / nchunks), so the workgroups balance the
// load as the hardware dispatcher would; a workgroup fetches its next ticket
// while it works on a chunk. There is no grid-wide barrier between blocks:
// a workgroup starts chunk c of block k once the chunks dlo(c) .. dhi(c)
// have finished block k - 1 (their epoch >= k - 1): those wrote the region c
// reads in block k and read, as halo, the region c overwrites. Each finished
// chunk publishes its epoch after a release fence at device (agent) scope,
// which spans the L2 caches of all XCDs; the wait ends with an acquire fence.
// Tickets are handed out in order, so every chunk waited for is held by a
// running workgroup that waits only on earlier blocks, and the waits end.
// Each wait is bounded all the same: after `timeout` ticks of the
// constant-rate wall clock the workgroup raises the error word and leaves,
// and so does every workgroup that sees it raised (timeout 0: the first
// check of a chunk's dependencies raises it, met or not, for tests);
// the host reports the error and the state is then invalid.
// status: health flag at word 0, error word at 16, ticket counter at 32.
template <int VER, int REGION>
__global__ __launch_bounds__(REGION, 2) void k_batch_line_persistent(double* src, double* dst,
                                                               const LineInst* __restrict__ insts,
                                                               const LineChunk* __restrict__ chunks, int nchunks,
                                                               const int* __restrict__ budget, int nsteps, int h,
                                                               int* epoch, int* status, long long timeout) {
  unsigned long long* ctr = reinterpret_cast<unsigned long long*>(status + 32);
  int* err = status + 16;
  __shared__ unsigned long long tk_s[2];
  __shared__ int go_s;
  const unsigned long long nblocks = (unsigned long long)((nsteps + h - 1) / h);
  const unsigned long long last = nblocks * (unsigned long long)nchunks;
  bool ok = true;
  if (threadIdx.x == 0) tk_s[0] = __hip_atomic_fetch_add(ctr, 1ull, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
  __syncthreads();
  unsigned long long tk = uniform_u64(tk_s[0]);
  int par = 1;
  while (tk < last) {
    const int blk = (int)(tk / (unsigned long long)nchunks);
    const int ci = (int)(tk - (unsigned long long)blk * (unsigned long long)nchunks);
    if (threadIdx.x == 0) {
      int go = 1;
      if (blk > 0 && timeout <= 0) {  // no waiting allowed: the first check gives up
        __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
        go = 0;
      } else if (blk > 0) {
        const LineChunk& ch = chunks[ci];
        const long long t0 = wall_clock64();
        for (int d = ch.dlo; d <= ch.dhi && go; ++d) {
          for (unsigned n = 1; __hip_atomic_load(&epoch[d], __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) < blk - 1;
               ++n) {
            if ((n & 7) == 0 && (__hip_atomic_load(err, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT) ||
                                 wall_clock64() - t0 >= timeout)) {
              __hip_atomic_store(err, 1, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
              go = 0;
              break;
            }
            __builtin_amdgcn_s_sleep(1);
          }
        }
        __builtin_amdgcn_fence(__ATOMIC_ACQUIRE, "agent");
      }
      go_s = go;
    }
    __syncthreads();
    if (!go_s) break;
    const int n0 = blk * h;
    const int hb = min(h, nsteps - n0);
    const double* A = (blk & 1) ? dst : src;
    double* B = (blk & 1) ? src : dst;
    ok &= line_chunk<VER, REGION, true>(A, B, insts, chunks, ci, budget, n0, hb, ctr, &tk_s[par]);
    __syncthreads();  // the chunk's stores are issued and complete; LDS free for the next one
    if (threadIdx.x == 0) {
      __builtin_amdgcn_fence(__ATOMIC_RELEASE, "agent");
      __hip_atomic_store(&epoch[ci], blk, __ATOMIC_RELAXED, __HIP_MEMORY_SCOPE_AGENT);
    }
    tk = uniform_u64(tk_s[par]);
    par ^= 1;
  }
  if (!ok) status[0] = 1;
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
  int pad;
  MarchGeom geom;
  March2Geom geom2;  // its strips of the two-step kernel
  Hot hot;
  Cold cold;
};

// One time step of every tile of a group of tile instances (same
// equilibrium version and variant: NEQ walls, or the flux-limited scheme
// with its radius-2 stencil HR = 2); workgroup b takes entry
// (b mod 8) per_xcd + b / 8 of the group's list, (instance, tile of the
// instance) or instance -1 for a padding entry, so each XCD gets a run of
// its own.
//
// Budgets, one launch per step (pairs = 0): an instance whose budget b is
// spent (step n >= b of a call of nsteps steps) idles: its final state stays
// where step b - 1 put it, and at n == b it is copied across once if the
// remaining nsteps - b steps are odd, so that after the call it sits in the
// same buffer as everyone else's.
// Pairs of steps (pairs = 1, plain instances beside k_batch_tiles2): the
// launch for steps (n, n + 1) does the step only for an instance with just
// one step left (n + 1 == m, m = min(b, nsteps)); one with two left is
// k_batch_tiles2's; an idle one (n >= m) is copied across once, at the first
// pair after its last, if the pairs left in the call are odd (every active
// pair moves the state to the other buffer once).
template <int VER, bool WALLS, int HR>
__global__ __launch_bounds__(64 * WAVES, 2) void k_batch_tiles(const double* __restrict__ A, double* __restrict__ B,
                                                                const TileInst* __restrict__ insts,
                                                                const int2* __restrict__ tiles, int per_xcd,
                                                                const int* __restrict__ budget, int n, int nsteps,
                                                                int pairs, int* flag) {
  const int2 en = tiles[(blockIdx.x % 8) * per_xcd + blockIdx.x / 8];
  if (en.x < 0) return;  // whole workgroup leaves together
  const TileInst& I = insts[en.x];
  Field F;
  F.fin = A + I.off;
  F.fout = B + I.off;
  F.nx = I.nx;
  F.ny = I.ny;
  F.pitch = I.pitch;
  F.plane = I.plane;
  const int tile = en.y;
  const int bud = budget[I.gidx];
  bool copy;
  if (pairs) {
    const int m = min(bud, nsteps);
    if (n + 2 <= m) return;  // two steps: the two-step kernel's
    if (n + 1 == m) {
      copy = false;
    } else {
      const int done = (m + 1) / 2, total = (nsteps + 1) / 2;  // pairs active, pairs in the call
      if (n != 2 * done || ((total - done) & 1) == 0) return;
      copy = true;
    }
  } else {
    copy = bud <= n;
    if (copy && (n != bud || ((nsteps - bud) & 1) == 0)) return;
  }
  if (copy) {
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

// Steps (n, n + 1) of every two-step tile (`geom2`) of the plain instances
// of one equilibrium version that have both steps left in the call; the
// others are k_batch_tiles's (pairs = 1). Each instance's two steps are
// those of k_step_fused2 on it alone. Workgroup b takes entry
// (b mod 8) per_xcd + b / 8 of the list: (instance, tile of the instance),
// or instance -1 for a padding entry.
template <int VER>
__global__ __launch_bounds__(128, 1) void k_batch_tiles2(const double* __restrict__ A, double* __restrict__ B,
                                                         const TileInst* __restrict__ insts,
                                                         const int2* __restrict__ tiles, int per_xcd,
                                                         const int* __restrict__ budget, int n, int nsteps, int* flag) {
  const int2 e = tiles[(blockIdx.x % 8) * per_xcd + blockIdx.x / 8];
  if (e.x < 0) return;  // whole workgroup leaves together
  const TileInst& I = insts[e.x];
  if (min(budget[I.gidx], nsteps) < n + 2) return;
  Field F;
  F.fin = A + I.off;
  F.fout = B + I.off;
  F.nx = I.nx;
  F.ny = I.ny;
  F.pitch = I.pitch;
  F.plane = I.plane;
  fused2_tile<VER, 2, true>(F, &I.hot, &I.cold, I.geom2, e.y, flag);
}

}  // namespace lbm
