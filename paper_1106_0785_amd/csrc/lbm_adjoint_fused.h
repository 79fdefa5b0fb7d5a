// Adjoint step staged through an LDS ring (the layout of the fused forward
// kernel, lbm_kernels.h): a workgroup of W wavefronts owns a tile of 64
// columns x `rows` rows and marches up it W rows at a time. Each ring entry
// holds what the transposed step reads at a stencil point: the 16 planes of
// lambda^{n+1} and the point's record (dL/dA, dL/dB and its velocity), with
// the ghost rules of the transposed step already applied (mirror: mirrored
// planes and record; zero gradient: the record's dL/dA, dL/dB negated;
// fixed state: lambda 0, dL/dA = dL/dB = 0 and the state's velocity), so
// every lambda and record value is read from HBM about once per step. The
// node's own f^n (and f^{n-1} for the next step's records) go straight to
// the lane that needs them. The arithmetic is adj_node's, in the same order.
#pragma once

#include "lbm_adjoint_kernels.h"

namespace lbm {

constexpr int NA = 20;  // ring entry: 16 lambda planes + GA, GB, ux, uy
constexpr int RA = STRIP + 2;

// Ghost values of a ring entry read from stored node (sx, sy) (resolve):
// lambda as lam_src / lam_plane transform it, the record as rec_point does.
__device__ __forceinline__ void fix_ghost_adj(const Hot& c, const Cold* __restrict__ cold, const Src& sx,
                                              const Src& sy, double* l, double* r) {
  if (__builtin_expect(sx.side < 0 && sy.side < 0, 1)) return;
  const int side = sx.side >= 0 ? sx.side : sy.side;
  const int kind = c.bc[side];
  if (sx.mode == 2 || sy.mode == 2) {
#pragma unroll
    for (int i = 0; i < 16; ++i) l[i] = 0.0;
  } else if (sx.mode == 1 || sy.mode == 1) {
    double t[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) t[i] = l[i];
    if (sx.mode == 1) {
#pragma unroll
      for (int i = 0; i < 16; ++i) l[i] = t[MIRROR_X[i]];
    } else {
#pragma unroll
      for (int i = 0; i < 16; ++i) l[i] = t[MIRROR_Y[i]];
    }
  }
  if (kind == BC_DIRICHLET_EQ) {
    r[REC_GA] = r[REC_GB] = 0.0;
    velocity_of(cold->ghost[side], r[REC_UX], r[REC_UY]);
  } else if (kind == BC_SPECULAR) {
    r[REC_GB] = -r[REC_GB];
    if (side < 2)
      r[REC_UX] = -r[REC_UX];
    else
      r[REC_UY] = -r[REC_UY];
  } else if (kind == BC_ZERO_GRADIENT) {
    r[REC_GA] = -r[REC_GA];
    r[REC_GB] = -r[REC_GB];
  }
}

// Transposed convection and identity for velocity I at ring column c0, the
// new lambda stored at once (adj_node's AdjOut with ring reads).
template <int I>
struct AdjOutRing {
  __device__ __forceinline__ static void run(const Hot& c, const double (*r0)[RA], const double (*rp)[RA],
                                             const double (*rm)[RA], int c0, bool zxl, bool zxh, bool zyl,
                                             bool zyh, double* __restrict__ lo, long long plane, double* out) {
    const double l = r0[I][c0];
    double v = out[I];
    if (VX[I] != 0) v += conv_t_axis(VX[I], c.lx, r0[I][c0 - 1], r0[I][c0 + 1], l, zxl, zxh);
    if (VY[I] != 0) v += conv_t_axis(VY[I], c.ly, rm[I][c0], rp[I][c0], l, zyl, zyh);
    out[I] = l + v;
    lo[I * plane] = out[I];
    AdjOutRing<I + 1>::run(c, r0, rp, rm, c0, zxl, zxh, zyl, zyh, lo, plane, out);
  }
};
template <>
struct AdjOutRing<16> {
  __device__ __forceinline__ static void run(const Hot&, const double (*)[RA], const double (*)[RA],
                                             const double (*)[RA], int, bool, bool, bool, bool, double* __restrict__,
                                             long long, double*) {}
};

// adj_node with lambda and the records of the node and its four neighbours
// from ring rows r0 (the node's), rp (y+1), rm (y-1) at column c0; f is the
// node's f^n. Writes lambda^n through lo (the node's address in lam_out) and,
// when fp (the node's address in f^{n-1}) is given, the next step's record
// of the node through ro.
template <int VER, bool SERIAL>
__device__ __forceinline__ void adj_node_ring(const Hot& c, const AdjCoef* __restrict__ adj, const double (*r0)[RA],
                                              const double (*rp)[RA], const double (*rm)[RA], int c0,
                                              const double* f, bool zxl, bool zxh, bool zyl, bool zyh,
                                              double* __restrict__ lo, long long plane, const double* fp,
                                              double* __restrict__ ro, double* sg) {
  double m[16];
  moments_from_f(f, m);
  const double rho = m[0], ir = 1.0 / rho;
  const double ux = m[1] * ir, uy = m[2] * ir;
  const double T = m[3] * ir - 0.5 * (ux * ux + uy * uy);
  const double rT = rho * T;
  const double GAxp = r0[16 + REC_GA][c0 + 1], GBxp = r0[16 + REC_GB][c0 + 1];
  const double uxxp = r0[16 + REC_UX][c0 + 1], uyxp = r0[16 + REC_UY][c0 + 1];
  const double GAxm = r0[16 + REC_GA][c0 - 1], GBxm = r0[16 + REC_GB][c0 - 1];
  const double uxxm = r0[16 + REC_UX][c0 - 1], uyxm = r0[16 + REC_UY][c0 - 1];
  const double GAyp = rp[16 + REC_GA][c0], GByp = rp[16 + REC_GB][c0];
  const double uxyp = rp[16 + REC_UX][c0], uyyp = rp[16 + REC_UY][c0];
  const double GAym = rm[16 + REC_GA][c0], GBym = rm[16 + REC_GB][c0];
  const double uxym = rm[16 + REC_UX][c0], uyym = rm[16 + REC_UY][c0];
  const double A = (uxxp - uxxm) * c.inv2dx - (uyyp - uyym) * c.inv2dy;
  const double B = (uyxp - uyxm) * c.inv2dx + (uxyp - uxym) * c.inv2dy;
  double mu[16];
  {
    double l[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) l[i] = r0[i][c0];
    minvt_apply(l, mu);
  }
  {
    double q[16];
    equilibrium_moments<VER, double>(m[0], m[1], m[2], m[3], q);
#pragma unroll
    for (int k = 4; k < 16; ++k) sg[k - 4] += mu[k] * adj->mdt * (m[k] - q[k]);
    const double a7 = rT * ux * A, b7 = rT * uy * B, b8 = rT * ux * B, a8 = rT * uy * A;
    sg[0] += mu[6] * adj->dcm[0] * a7 + mu[7] * adj->dcm[6] * a8;
    sg[1] += mu[6] * adj->dcm[2] * b7 + mu[7] * adj->dcm[4] * b8;
    sg[2] += mu[6] * (adj->dcm[1] * a7 + adj->dcm[3] * b7);
    sg[3] += mu[7] * (adj->dcm[5] * b8 + adj->dcm[7] * a8);
  }
  double nu[16];
#pragma unroll
  for (int k = 4; k < 16; ++k) nu[k] = c.cq[k - 4] * mu[k];
  auto dual_dir = [&](int a) -> double {
    Dual cc[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) cc[b] = Dual(m[b], a == b ? 1.0 : 0.0);
    Dual qd[16];
    equilibrium_moments<VER, Dual>(cc[0], cc[1], cc[2], cc[3], qd);
    double s = 0.0;
#pragma unroll
    for (int k = 4; k < 16; ++k) s -= nu[k] * qd[k].d;
    const Dual iR = 1.0 / cc[0];
    const Dual vxd = cc[1] * iR, vyd = cc[2] * iR;
    const Dual Td = cc[3] * iR - 0.5 * (vxd * vxd + vyd * vyd);
    const Dual rTd = cc[0] * Td;
    const Dual g7 = c.cmod[0] * rTd * vxd * A + c.cmod[1] * rTd * vyd * B;
    const Dual g8 = c.cmod[2] * rTd * vxd * B + c.cmod[3] * rTd * vyd * A;
    return s + mu[6] * g7.d + mu[7] * g8.d;
  };
  double gc[4] = {0.0, 0.0, 0.0, 0.0};
  if constexpr (SERIAL) {
#pragma unroll 1
    for (int a = 0; a < 4; ++a) {
      const double g = dual_dir(a);
#pragma unroll
      for (int b = 0; b < 4; ++b) gc[b] = (a == b) ? g : gc[b];
    }
  } else {
#pragma unroll
    for (int a = 0; a < 4; ++a) gc[a] = dual_dir(a);
  }
  const double gux = (GAxm - GAxp) * c.inv2dx + (GBym - GByp) * c.inv2dy;
  const double guy = (GBxm - GBxp) * c.inv2dx - (GAym - GAyp) * c.inv2dy;
  gc[0] += -(ux * gux + uy * guy) * ir;
  gc[1] += gux * ir;
  gc[2] += guy * ir;
#pragma unroll
  for (int k = 0; k < 4; ++k) nu[k] = gc[k];
  double out[16];
  mt_apply(nu, out);
  AdjOutRing<0>::run(c, r0, rp, rm, c0, zxl, zxh, zyl, zyh, lo, plane, out);
  if (fp) {
    double r[NREC], fq[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) fq[i] = fp[i * plane];
    record_from(c, fq, out, r);
#pragma unroll
    for (int j = 0; j < NREC; ++j) ro[j * plane] = r[j];
  }
}

// One tile of the adjoint step. F.fin = f^n; lam_in = lambda^{n+1}; rec =
// the records of this step; lam_out = lambda^n; f_prev (may be NULL) =
// f^{n-1}, whose records rec_out receives. The tile's dL/ds contribution
// is added to partials[slot * 12 ..] (one slot per tile, fixed order).
template <int VER, int W, bool SERIAL>
__device__ __forceinline__ void adj_tile(Field F, const double* __restrict__ lam_in, double* __restrict__ lam_out,
                                         const double* __restrict__ rec, const Hot* __restrict__ hot,
                                         const Cold* __restrict__ cold, const AdjCoef* __restrict__ adj,
                                         double* __restrict__ partials, const double* __restrict__ f_prev,
                                         double* __restrict__ rec_out, MarchGeom g, int tile) {
  constexpr int RING = W + 2;
  __shared__ double ring[RING][NA][RA];
  __shared__ Hot hs;
  __shared__ double red[12][W];
  stage_hot(hot, &hs);
  const Hot& c = hs;
  const int lane = threadIdx.x & 63;
  const int w = __builtin_amdgcn_readfirstlane(threadIdx.x >> 6);
  const int strip = tile % g.nstrips, seg = tile / g.nstrips;
  const int nx = F.nx, ny = F.ny;
  const int x0 = strip * STRIP;
  const int x = x0 + lane;
  const int y0 = seg * g.rows;
  const int y1 = min(y0 + g.rows, ny);
  const int ylast = y1;  // last ring row the tile reads
  const int base = y0 - 1;
  const Src sx = (x < nx + 1) ? resolve(x, nx, c.bc[0], c.bc[1], 0) : Src{nx - 1, 0, -1};
  const int c0 = lane + 1;
  const int bylo = __builtin_amdgcn_readfirstlane(hot->bc[2]);
  const int byhi = __builtin_amdgcn_readfirstlane(hot->bc[3]);
  auto ysrc = [&](int yr) -> Src {
    if (yr < 0 || yr >= ny) return resolve(yr, ny, bylo, byhi, 2);
    return Src{yr, 0, -1};
  };
  // neighbour columns x0 - 1 (e = 0) and x0 + 64 (e = 1): lanes 0..31 hold
  // lambda plane ep of column e, lanes 32..63 with ep < 4 its record value
  // ep; the x ghost rule is folded into the address and an affine map
  const int ep = lane & 15, e = (lane >> 4) & 1;
  const bool erec = lane >= 32;
  const int ecol = e ? RA - 1 : 0;
  const double* eptr;
  long long estride;
  double escale = 1.0, eoff = 0.0;
  {
    const int ex = e ? x0 + STRIP : x0 - 1;
    const Src es = (ex < nx + 1) ? resolve(ex, nx, c.bc[0], c.bc[1], 0) : Src{nx - 1, 0, -1};
    const int kind = es.side >= 0 ? c.bc[es.side] : BC_PERIODIC;
    if (!erec) {
      const int pl = (es.mode == 1) ? lane_table(MIRROR_X, ep) : ep;
      eptr = lam_in + (long long)pl * F.plane + es.idx;
      if (es.mode == 2) escale = 0.0;
    } else {
      const int j = ep < NREC ? ep : 0;
      eptr = rec + (long long)j * F.plane + es.idx;
      if (kind == BC_DIRICHLET_EQ) {
        escale = 0.0;
        if (j >= REC_UX) {
          double gx, gy;
          velocity_of(cold->ghost[es.side], gx, gy);
          eoff = j == REC_UX ? gx : gy;
        }
      } else if (kind == BC_SPECULAR) {
        if (j == REC_GB || j == REC_UX) escale = -1.0;  // x side: dL/dB and u_x change sign
      } else if (kind == BC_ZERO_GRADIENT) {
        if (j == REC_GA || j == REC_GB) escale = -1.0;
      }
    }
    estride = F.pitch;
  }
  const bool ewrite = !erec || ep < NREC;
  const int eslot = erec ? 16 + ep : ep;

  auto load_row = [&](int yr, double* l, double* r, double& ev) {
    const int yi = ysrc(min(yr, ylast)).idx;
    const long long k = (long long)yi * F.pitch + sx.idx;
#pragma unroll
    for (int i = 0; i < 16; ++i) l[i] = lam_in[k + i * F.plane];
#pragma unroll
    for (int j = 0; j < NREC; ++j) r[j] = rec[k + j * F.plane];
    ev = eptr[yi * estride];
  };
  auto enter_row = [&](int yr, double* l, double* r, double ev) {
    fix_ghost_adj(c, cold, sx, ysrc(yr), l, r);
    const int slot = (unsigned)(yr - base) % RING;
#pragma unroll
    for (int i = 0; i < 16; ++i) ring[slot][i][c0] = l[i];
#pragma unroll
    for (int j = 0; j < NREC; ++j) ring[slot][16 + j][c0] = r[j];
    if (ewrite) ring[slot][eslot][ecol] = escale * ev + eoff;
  };

  // prologue: ring rows y0-1 .. y0+W (wave w fills slots w and w + W < RING)
  {
    double la[16], ra[NREC], lb[16], rb[NREC], ea, eb = 0.0;
    const bool two = w < RING - W;
    load_row(base + w, la, ra, ea);
    if (two) load_row(base + w + W, lb, rb, eb);
    if (base + w <= ylast) enter_row(base + w, la, ra, ea);
    if (two && base + w + W <= ylast) enter_row(base + w + W, lb, rb, eb);
  }
  double sg[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) sg[k] = 0.0;
  const bool zxl = x == 0 && c.bc[0] == BC_ZERO_GRADIENT, zxh = x == nx - 1 && c.bc[1] == BC_ZERO_GRADIENT;
  for (int Y = y0; Y < y1; Y += W) {
    const int y = Y + w;
    // the node's f^n, in flight across the barrier (the row entering the
    // ring next is loaded after the update, to keep registers for it)
    double f[16];
    const long long k0 = (long long)min(y, ny - 1) * F.pitch + min(x, nx - 1);
#pragma unroll
    for (int i = 0; i < 16; ++i) f[i] = F.fin[k0 + i * F.plane];
    __syncthreads();
    if (y < y1 && x < nx) {
      const int s0 = (unsigned)(y - base) % RING, sp = (unsigned)(y + 1 - base) % RING,
                sm = (unsigned)(y - 1 - base) % RING;
      const bool zyl = y == 0 && c.bc[2] == BC_ZERO_GRADIENT, zyh = y == ny - 1 && c.bc[3] == BC_ZERO_GRADIENT;
      adj_node_ring<VER, SERIAL>(c, adj, ring[s0], ring[sp], ring[sm], c0, f, zxl, zxh, zyl, zyh, lam_out + k0,
                                 F.plane, f_prev ? f_prev + k0 : nullptr, rec_out + k0, sg);
    }
    // the row entering the ring after this iteration's updates
    const int yn = Y + W + 1 + w;
    double ln[16], rn[NREC], en;
    load_row(yn, ln, rn, en);
    __syncthreads();
    if (yn <= ylast) enter_row(yn, ln, rn, en);
  }
  // deterministic tile sum: DPP/readlane within each wave, then the waves
  // in order; one slot per tile, accumulated over the steps
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    const double s = wave_sum(sg[k]);
    if (lane == 0) red[k][w] = s;
  }
  __syncthreads();
  if (threadIdx.x < 12) {
    double s = 0.0;
#pragma unroll
    for (int v = 0; v < W; ++v) s += red[threadIdx.x][v];
    partials[(long long)tile * 12 + threadIdx.x] += s;
  }
}

template <int VER, int W, bool SERIAL>
__global__ __launch_bounds__(64 * W, 2) void k_adj_fused(Field F, const double* __restrict__ lam_in,
                                                        double* __restrict__ lam_out, const double* __restrict__ rec,
                                                        const Hot* __restrict__ hot, const Cold* __restrict__ cold,
                                                        const AdjCoef* __restrict__ adj, double* __restrict__ partials,
                                                        const double* __restrict__ f_prev,
                                                        double* __restrict__ rec_out, MarchGeom g) {
  const int tile = xcd_tile(blockIdx.x, g);
  if (tile >= g.ntiles) return;  // whole workgroup leaves together
  adj_tile<VER, W, SERIAL>(F, lam_in, lam_out, rec, hot, cold, adj, partials, f_prev, rec_out, g, tile);
}

}  // namespace lbm
