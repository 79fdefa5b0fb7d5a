// Adjoint (reverse-mode) step of the MRT FD-LBM update, hand-written.
//
// One forward step is f^{n+1}(x) = f(x) + L(x) + M^-1 col(x), with the
// per-axis Lax-Wendroff increments L, col_k = -dt s_k (m_k - q_k(c)) for the
// non-conserved moments (c = rho, j_x, j_y, e) and the energy-flux
// modification g_7, g_8 added to col_7, col_8 (Sec. II); g depends on the
// node's c and on the central-difference velocity gradients A, B built from
// the four neighbours' velocities. Its amplification matrix G_ij (Sec. III)
// is this map's Jacobian in Fourier space. Given lambda = dL/df^{n+1}, the
// adjoint step returns dL/df^n:
//
//   lambda^n_i(x) = lambda_i(x) + sum_axes [ p_i (lambda_i(x-e) - lambda_i(x))
//                                          + m_i (lambda_i(x+e) - lambda_i(x)) ]
//                 + (M^T nu)_i + (M_{1..4}^T g_c)_i
//   mu  = M^-T lambda(x),   nu_k = -dt s_k mu_k  (k >= 5)
//   g_c = - J_q^T nu + mu_7 dg_7/dc + mu_8 dg_8/dc + (du/dc)^T g_u
//   g_u(x) = gathered from the neighbours' dL/dA, dL/dB (the modification's
//            coupling to the velocities of the four neighbours)
//
// and accumulates dL/ds_k = sum_n sum_x mu_k d col_k/d s_k. Ghost layers
// are transposed: a periodic ghost is the wrapped node, a mirror ghost
// returns the mirrored lambda and (dL/dA, -dL/dB), a zero-gradient ghost
// returns lambda with the Lax-Wendroff weights swapped and (-dL/dA, -dL/dB),
// a fixed-state ghost returns nothing.
#pragma once

#include "lbm_dual.h"
#include "lbm_kernels.h"

namespace lbm {

// Derivatives of the modification coefficients (Hot::cmod) w.r.t. the rates:
// d cm0/d s5, d cm0/d s7, d cm1/d s6, d cm1/d s7, d cm2/d s6, d cm2/d s8,
// d cm3/d s5, d cm3/d s8 (all 0 for the unmodified model).
struct AdjCoef {
  double dcm[8];
  double mdt;  // -dt: d col_k / d s_k = -dt (m_k - q_k)
};

// Per-node record written by the first pass: dL/dA, dL/dB and the velocity.
enum { REC_GA = 0, REC_GB = 1, REC_UX = 2, REC_UY = 3, NREC = 4 };

// Record of a node from its distributions f (the forward level the next
// adjoint step linearises about) and its lambda (that step's input).
LBM_HD void record_from(const Hot& c, const double* f, const double* l, double* r) {
  double m[16], mu[16];
  moments_from_f(f, m);
  minvt_apply(l, mu);
  const double rho = m[0], ir = 1.0 / rho;
  const double ux = m[1] * ir, uy = m[2] * ir;
  const double T = m[3] * ir - 0.5 * (ux * ux + uy * uy);
  const double rT = rho * T;
  double vx, vy;
  velocity_of(f, vx, vy);
  r[REC_GA] = mu[6] * c.cmod[0] * rT * ux + mu[7] * c.cmod[3] * rT * uy;
  r[REC_GB] = mu[6] * c.cmod[1] * rT * uy + mu[7] * c.cmod[2] * rT * ux;
  r[REC_UX] = vx;
  r[REC_UY] = vy;
}

LBM_HD void adj_record(const Field& F, const Hot& c, const double* __restrict__ lam, double* __restrict__ rec, int x,
                       int y) {
  const long long k = (long long)y * F.pitch + x;
  double f[16], l[16], r[NREC];
#pragma unroll
  for (int i = 0; i < 16; ++i) {
    f[i] = F.fin[k + i * F.plane];
    l[i] = lam[k + i * F.plane];
  }
  record_from(c, f, l, r);
#pragma unroll
  for (int j = 0; j < NREC; ++j) rec[k + j * F.plane] = r[j];
}

template <int VER>
__global__ __launch_bounds__(256) void k_adj_records(Field F, const double* __restrict__ lam,
                                                     double* __restrict__ rec, const Hot* __restrict__ hot) {
  __shared__ Hot hs;
  stage_hot(hot, &hs);
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  if (x >= F.nx || y >= F.ny) return;
  adj_record(F, hs, lam, rec, x, y);
}

// Record of stencil point (x + ox, y + oy) of node (x, y) as its ghost
// transposition requires; ux, uy are the velocity the forward step used.
LBM_HD void rec_point(const Field& F, const Hot& c, const Cold* __restrict__ cold,
                                          const double* __restrict__ rec, int x, int y, int ox, int oy, double& GA,
                                          double& GB, double& ux, double& uy) {
  const int xn = x + ox, yn = y + oy;
  const Src sx = resolve(xn, F.nx, c.bc[0], c.bc[1], 0);
  const Src sy = resolve(yn, F.ny, c.bc[2], c.bc[3], 2);
  // side whose ghost this stencil point is (-1: a stored node); periodic
  // ghosts are stored nodes after wrapping
  const int side = (xn < 0 || xn >= F.nx) ? sx.side : ((yn < 0 || yn >= F.ny) ? sy.side : -1);
  const int kind = side >= 0 ? c.bc[side] : BC_PERIODIC;
  if (kind == BC_DIRICHLET_EQ) {
    GA = GB = 0.0;
    velocity_of(cold->ghost[side], ux, uy);
    return;
  }
  const long long k = (long long)sy.idx * F.pitch + sx.idx;
  GA = rec[k + REC_GA * F.plane];
  GB = rec[k + REC_GB * F.plane];
  ux = rec[k + REC_UX * F.plane];
  uy = rec[k + REC_UY * F.plane];
  if (kind == BC_SPECULAR) {
    GB = -GB;
    if (side < 2)
      ux = -ux;
    else
      uy = -uy;
  } else if (kind == BC_ZERO_GRADIENT) {
    GA = -GA;
    GB = -GB;
  }
}

// Where the transposed convection finds lambda at stencil point (x + ox,
// y + oy): the stored node k and how plane i maps onto it (0: plane i;
// 1: mirror in x, mirrored plane; 3: mirror in y; 2: fixed-state ghost,
// value 0; a zero-gradient ghost gives the node's own lambda and the caller
// swaps the weights). Lets the caller load one plane at a time.
struct LamSrc {
  long long k;
  int mode;
};

LBM_HD LamSrc lam_src(const Field& F, const Hot& c, int x, int y, int ox, int oy) {
  const Src sx = resolve(x + ox, F.nx, c.bc[0], c.bc[1], 0);
  const Src sy = resolve(y + oy, F.ny, c.bc[2], c.bc[3], 2);
  LamSrc r;
  r.k = (long long)sy.idx * F.pitch + sx.idx;
  r.mode = (sx.mode == 2 || sy.mode == 2) ? 2 : (sx.mode == 1 ? 1 : (sy.mode == 1 ? 3 : 0));
  return r;
}

// Plane I of lambda at a stencil point described by lam_src.
template <int I>
LBM_HD double lam_plane(const Field& F, const double* __restrict__ lam, LamSrc s) {
  const int pl = (s.mode == 1) ? MIRROR_X[I] : ((s.mode == 3) ? MIRROR_Y[I] : I);
  const double v = lam[s.k + (long long)pl * F.plane];
  return (s.mode == 2) ? 0.0 : v;
}

// Transposed Lax-Wendroff increment of velocity I along one axis; v is the
// velocity component, (pm, mm) the weights as the forward step applies them
// to (f(x+e) - f, f(x-e) - f), zl/zh true when the low/high neighbour is a
// zero-gradient ghost.
LBM_HD double conv_t_axis(int v, const double* lc, double lo, double hi, double lam, bool zl,
                                              bool zh) {
  // weights of f(x+e) (p) and f(x-e) (m) for this velocity
  double p = 0.0, m = 0.0;
  if (v == 1) { p = lc[0]; m = lc[1]; }
  if (v == -1) { p = lc[1]; m = lc[0]; }
  if (v == 2) { p = lc[2]; m = lc[3]; }
  if (v == -2) { p = lc[3]; m = lc[2]; }
  // node x is the + neighbour of x-e (weight p) and the - neighbour of x+e (weight m)
  double r = p * (lo - lam) + m * (hi - lam);
  if (zl) r += (m - p) * lam;  // ghost x-e = f(x): node x itself used weight m on it
  if (zh) r += (p - m) * lam;  // ghost x+e = f(x): weight p
  return r;
}

// New adjoint lambda^n at node (x, y) into lam_out; adds this node's
// contribution to dL/ds_5..16 (index k - 5) into sg.
// With f_prev (the forward level of the next adjoint step, same layout as
// F.fin) also writes that step's record of this node into rec_out.
// Per-plane part of the transposed convection and identity for velocity I,
// with the new lambda stored at once (so no neighbour plane set is kept).
template <int I>
struct AdjOut {
  LBM_HD static void run(const Field& F, const Hot& c, const double* __restrict__ lam_in, double* __restrict__ lam_out,
                         long long k0, LamSrc sxp, LamSrc sxm, LamSrc syp, LamSrc sym, bool zxl, bool zxh, bool zyl,
                         bool zyh, double* out) {
    const double l = lam_in[k0 + (long long)I * F.plane];
    double v = out[I];
    if (VX[I] != 0) v += conv_t_axis(VX[I], c.lx, lam_plane<I>(F, lam_in, sxm), lam_plane<I>(F, lam_in, sxp), l, zxl, zxh);
    if (VY[I] != 0) v += conv_t_axis(VY[I], c.ly, lam_plane<I>(F, lam_in, sym), lam_plane<I>(F, lam_in, syp), l, zyl, zyh);
    out[I] = l + v;
    lam_out[k0 + (long long)I * F.plane] = out[I];
    AdjOut<I + 1>::run(F, c, lam_in, lam_out, k0, sxp, sxm, syp, sym, zxl, zxh, zyl, zyh, out);
  }
};
template <>
struct AdjOut<16> {
  LBM_HD static void run(const Field&, const Hot&, const double* __restrict__, double* __restrict__, long long, LamSrc,
                         LamSrc, LamSrc, LamSrc, bool, bool, bool, bool, double*) {}
};

// New adjoint lambda^n at node (x, y) into lam_out; adds this node's
// contribution to dL/ds_5..16 (index k - 5) into sg.
// With f_prev (the forward level of the next adjoint step, same layout as
// F.fin) also writes that step's record of this node into rec_out.
// Ordered so that few values are live at once: the distributions are
// dropped after their moments, dL/ds is formed as soon as mu is known, and
// the transposed convection loads one plane of each neighbour at a time.
template <int VER, bool SERIAL = false>
LBM_HD void adj_node(const Field& F, const Hot& c, const Cold* __restrict__ cold, const AdjCoef* __restrict__ adj,
                     const double* __restrict__ lam_in, double* __restrict__ lam_out, const double* __restrict__ rec,
                     const double* __restrict__ f_prev, double* __restrict__ rec_out, int x, int y, double* sg) {
  const long long k0 = (long long)y * F.pitch + x;
  // --- forward quantities at the node
  double m[16];
  {
    double f[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) f[i] = F.fin[k0 + i * F.plane];
    moments_from_f(f, m);
  }
  const double rho = m[0], ir = 1.0 / rho;
  const double ux = m[1] * ir, uy = m[2] * ir;
  const double T = m[3] * ir - 0.5 * (ux * ux + uy * uy);
  const double rT = rho * T;
  // --- neighbour records: velocities for A, B and dL/dA, dL/dB
  double GAxp, GBxp, uxxp, uyxp, GAxm, GBxm, uxxm, uyxm, GAyp, GByp, uxyp, uyyp, GAym, GBym, uxym, uyym;
  rec_point(F, c, cold, rec, x, y, +1, 0, GAxp, GBxp, uxxp, uyxp);
  rec_point(F, c, cold, rec, x, y, -1, 0, GAxm, GBxm, uxxm, uyxm);
  rec_point(F, c, cold, rec, x, y, 0, +1, GAyp, GByp, uxyp, uyyp);
  rec_point(F, c, cold, rec, x, y, 0, -1, GAym, GBym, uxym, uyym);
  const double A = (uxxp - uxxm) * c.inv2dx - (uyyp - uyym) * c.inv2dy;
  const double B = (uyxp - uyxm) * c.inv2dx + (uxyp - uxym) * c.inv2dy;
  // --- collision adjoint
  double mu[16];
  {
    double l[16];
#pragma unroll
    for (int i = 0; i < 16; ++i) l[i] = lam_in[k0 + i * F.plane];
    minvt_apply(l, mu);
  }
  // --- dL/ds: d col_k/d s_k = -dt (m_k - q_k), plus the modification's
  // coefficients (their s-derivatives already carry the factor dt)
  {
    double q[16];
    equilibrium_moments<VER, double>(m[0], m[1], m[2], m[3], q);
#pragma unroll
    for (int k = 4; k < 16; ++k) sg[k - 4] = mu[k] * adj->mdt * (m[k] - q[k]);
    const double a7 = rT * ux * A, b7 = rT * uy * B, b8 = rT * ux * B, a8 = rT * uy * A;
    sg[0] += mu[6] * adj->dcm[0] * a7 + mu[7] * adj->dcm[6] * a8;   // s5
    sg[1] += mu[6] * adj->dcm[2] * b7 + mu[7] * adj->dcm[4] * b8;   // s6
    sg[2] += mu[6] * (adj->dcm[1] * a7 + adj->dcm[3] * b7);          // s7
    sg[3] += mu[7] * (adj->dcm[5] * b8 + adj->dcm[7] * a8);          // s8
  }
  double nu[16];
#pragma unroll
  for (int k = 4; k < 16; ++k) nu[k] = c.cq[k - 4] * mu[k];
  // conserved-moment adjoint: -J_q^T nu + mu7 dg7/dc + mu8 dg8/dc, by dual
  // numbers, one derivative direction a at a time
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
    // not unrolled: interleaving the four evaluations would hold four times
    // the registers (this form runs two blocks per CU)
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
  // velocity adjoint from the neighbours' gradient terms, then du/dc
  const double gux = (GAxm - GAxp) * c.inv2dx + (GBym - GByp) * c.inv2dy;
  const double guy = (GBxm - GBxp) * c.inv2dx - (GAym - GAyp) * c.inv2dy;
  gc[0] += -(ux * gux + uy * guy) * ir;
  gc[1] += gux * ir;
  gc[2] += guy * ir;
#pragma unroll
  for (int k = 0; k < 4; ++k) nu[k] = gc[k];
  double out[16];
  mt_apply(nu, out);
  // --- transposed convection and identity, plane by plane
  const LamSrc sxp = lam_src(F, c, x, y, +1, 0), sxm = lam_src(F, c, x, y, -1, 0);
  const LamSrc syp = lam_src(F, c, x, y, 0, +1), sym = lam_src(F, c, x, y, 0, -1);
  const bool zxl = x == 0 && c.bc[0] == BC_ZERO_GRADIENT, zxh = x == F.nx - 1 && c.bc[1] == BC_ZERO_GRADIENT;
  const bool zyl = y == 0 && c.bc[2] == BC_ZERO_GRADIENT, zyh = y == F.ny - 1 && c.bc[3] == BC_ZERO_GRADIENT;
  AdjOut<0>::run(F, c, lam_in, lam_out, k0, sxp, sxm, syp, sym, zxl, zxh, zyl, zyh, out);
  if (f_prev) {
    double fp[16], r[NREC];
#pragma unroll
    for (int i = 0; i < 16; ++i) fp[i] = f_prev[k0 + i * F.plane];
    record_from(c, fp, out, r);
#pragma unroll
    for (int j = 0; j < NREC; ++j) rec_out[k0 + j * F.plane] = r[j];
  }
}

// Value of lane l (uniform) of a wave.
__device__ __forceinline__ double read_lane(double v, int l) {
  const long long b = __double_as_longlong(v);
  const int lo = __builtin_amdgcn_readlane((int)b, l);
  const int hi = __builtin_amdgcn_readlane((int)(b >> 32), l);
  return __longlong_as_double(((long long)hi << 32) | (long long)(unsigned)lo);
}

// Sum over the 64 lanes of a wave in a fixed order (rows of 16 by DPP, then
// the four row sums), so the result does not depend on timing.
__device__ __forceinline__ double wave_sum(double v) {
  v = row16_sum(v);
  return (read_lane(v, 0) + read_lane(v, 16)) + (read_lane(v, 32) + read_lane(v, 48));
}

// Launched with 64 x 4 threads per block. WIDE (large grids): two blocks per
// CU, so that each SIMD has two waves to hide the latency of ~100 loads per
// node (version 3 excepted: its Maxwellian terms would spill), at the cost of
// evaluating the four dual directions one after another; otherwise one block
// per CU with the four interleaved (small grids give each SIMD one wave
// anyway, and then instruction-level parallelism is what hides latency).
template <int VER, bool WIDE>
__global__ __launch_bounds__(256, (WIDE && VER != 3) ? 2 : 1) void k_adj_step(Field F, const double* __restrict__ lam_in,
                                                  double* __restrict__ lam_out, const double* __restrict__ rec,
                                                  const Hot* __restrict__ hot, const Cold* __restrict__ cold,
                                                  const AdjCoef* __restrict__ adj, double* __restrict__ partials,
                                                  const double* __restrict__ f_prev, double* __restrict__ rec_out) {
  __shared__ Hot hs;
  __shared__ double red[12][4];
  stage_hot(hot, &hs);
  const int t = threadIdx.y * blockDim.x + threadIdx.x;
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y * blockDim.y + threadIdx.y;
  double sg[12];
#pragma unroll
  for (int k = 0; k < 12; ++k) sg[k] = 0.0;
  if (x < F.nx && y < F.ny)
    adj_node<VER, WIDE && VER != 3>(F, hs, cold, adj, lam_in, lam_out, rec, f_prev, rec_out, x, y, sg);
  // deterministic block reduction, one slot per block, accumulated over steps
#pragma unroll
  for (int k = 0; k < 12; ++k) {
    const double w = wave_sum(sg[k]);
    if ((t & 63) == 0) red[k][t >> 6] = w;
  }
  __syncthreads();
  if (t < 12) {
    const long long slot = (long long)blockIdx.y * gridDim.x + blockIdx.x;
    partials[slot * 12 + t] += (red[t][0] + red[t][1]) + (red[t][2] + red[t][3]);
  }
}

}  // namespace lbm

namespace lbm {

// Transpose of a non-equilibrium extrapolation wall (Sec. IV.A): the step
// writes f_w = f^eq(rho_n, u_w, T_w) + f_n - f^eq(rho_n, u_n, T_n) from the
// fluid neighbour's new distributions f_n, so lambda_n += (d f_w / d f_n)^T
// lambda_w. With mu = M^-T lambda_w (f^eq = M^-1 q): the fixed-state
// equilibrium depends on f_n through rho only (d rho / d f_i = 1), the
// neighbour's through (rho, j, e) = the first four moments (M^T of their
// derivatives), both by dual numbers through the step's own equilibria.
template <int VER>
LBM_HD void wall_t_apply(const double* wall, const double* fn, const double* lw, double* ln) {
  double mu[16], m[16];
  minvt_apply(lw, mu);
  moments_from_f(fn, m);
  const double uwx = wall[1], uwy = wall[2], ew = wall[3] + 0.5 * (uwx * uwx + uwy * uwy);
  double g1 = 0.0;
  {
    const Dual r(m[0], 1.0);
    Dual q[16];
    equilibrium_moments<VER, Dual>(r, r * uwx, r * uwy, r * ew, q);
#pragma unroll
    for (int k = 0; k < 16; ++k) g1 += mu[k] * q[k].d;
  }
  double nu[16];
#pragma unroll
  for (int k = 4; k < 16; ++k) nu[k] = 0.0;
#pragma unroll 1
  for (int a = 0; a < 4; ++a) {
    Dual cc[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) cc[b] = Dual(m[b], a == b ? 1.0 : 0.0);
    Dual q[16];
    equilibrium_moments<VER, Dual>(cc[0], cc[1], cc[2], cc[3], q);
    double g = 0.0;
#pragma unroll
    for (int k = 0; k < 16; ++k) g += mu[k] * q[k].d;
#pragma unroll
    for (int b = 0; b < 4; ++b) nu[b] = (a == b) ? g : nu[b];
  }
  double t[16];
  mt_apply(nu, t);
#pragma unroll
  for (int i = 0; i < 16; ++i) ln[i] += lw[i] + g1 - t[i];
}

// Wall transposes of one adjoint step, applied to lambda^{n+1} before the
// step's transpose; F.fin = f^{n+1}. One thread per node along the walled
// sides (walls on one axis only); the wall node's own lambda is then 0 (the
// step overwrites it). With two walls 3 nodes apart both act on the same
// fluid node, in turn, in the same thread.
template <int VER>
__global__ __launch_bounds__(64) void k_adj_walls(Field F, double* __restrict__ lam, const Hot* __restrict__ hot,
                                                  const Cold* __restrict__ cold) {
  const bool ywalls = hot->bc[2] == BC_NEQ_WALL || hot->bc[3] == BC_NEQ_WALL;
  const int i = blockIdx.x * blockDim.x + threadIdx.x;
  if (i >= (ywalls ? F.nx : F.ny)) return;
  const int across = ywalls ? F.ny : F.nx;
  for (int side = 0; side < 2; ++side) {
    const int sd = (ywalls ? 2 : 0) + side;
    if (hot->bc[sd] != BC_NEQ_WALL) continue;
    const int wpos = side == 0 ? 0 : across - 1, npos = side == 0 ? 1 : across - 2;
    const long long kw = ywalls ? (long long)wpos * F.pitch + i : (long long)i * F.pitch + wpos;
    const long long kn = ywalls ? (long long)npos * F.pitch + i : (long long)i * F.pitch + npos;
    double lw[16], fn[16], ln[16];
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      lw[j] = lam[kw + j * F.plane];
      fn[j] = F.fin[kn + j * F.plane];
      ln[j] = lam[kn + j * F.plane];
    }
    wall_t_apply<VER>(cold->wall[sd], fn, lw, ln);
#pragma unroll
    for (int j = 0; j < 16; ++j) {
      lam[kn + j * F.plane] = ln[j];
      lam[kw + j * F.plane] = 0.0;
    }
  }
}

// lambda at the final level from dL/d(rho, u_x, u_y, T) of the final fields
// (any gradient pointer may be NULL); the fields are rho = m1, u = (m2, m3)/m1,
// T = m4/m1 - |u|^2/2 (R = 1).
LBM_HD void adj_final_node(const Field& F, const double* __restrict__ g_rho, const double* __restrict__ g_ux,
                           const double* __restrict__ g_uy, const double* __restrict__ g_T, double* __restrict__ lam,
                           int x, int y) {
  const long long k = (long long)y * F.pitch + x;
  const long long d = (long long)y * F.nx + x;
  double f[16], m[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) f[i] = F.fin[k + i * F.plane];
  moments_from_f(f, m);
  const double r = m[0], ir = 1.0 / r;
  const double gr = g_rho ? g_rho[d] : 0.0, gu = g_ux ? g_ux[d] : 0.0, gv = g_uy ? g_uy[d] : 0.0,
               gt = g_T ? g_T[d] : 0.0;
  double nu[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) nu[i] = 0.0;
  const double ux = m[1] * ir, uy = m[2] * ir;
  nu[0] = gr - (gu * ux + gv * uy) * ir + gt * (-m[3] * ir * ir + (ux * ux + uy * uy) * ir);
  nu[1] = gu * ir - gt * ux * ir;
  nu[2] = gv * ir - gt * uy * ir;
  nu[3] = gt * ir;
  double l[16];
  mt_apply(nu, l);
#pragma unroll
  for (int i = 0; i < 16; ++i) lam[k + i * F.plane] = l[i];
}

template <int U>
__global__ void k_adj_final(Field F, const double* __restrict__ g_rho, const double* __restrict__ g_ux,
                            const double* __restrict__ g_uy, const double* __restrict__ g_T, double* __restrict__ lam) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= F.nx) return;
  adj_final_node(F, g_rho, g_ux, g_uy, g_T, lam, x, y);
}

// dL/d(rho0, u0, T0) from lambda^0: f^0 = M^-1 q(rho, rho u, rho (T + u^2/2)).
template <int VER>
LBM_HD void adj_init_node(const Field& F, const double* __restrict__ lam, const double* __restrict__ rho,
                          const double* __restrict__ ux, const double* __restrict__ uy, const double* __restrict__ T,
                          double* g_rho, double* g_ux, double* g_uy, double* g_T, int x, int y) {
  const long long k = (long long)y * F.pitch + x;
  const long long d = (long long)y * F.nx + x;
  double l[16], mu[16];
#pragma unroll
  for (int i = 0; i < 16; ++i) l[i] = lam[k + i * F.plane];
  minvt_apply(l, mu);
  const double p0[4] = {rho[d], ux[d], uy[d], T[d]};
  double g[4];
#pragma unroll
  for (int a = 0; a < 4; ++a) {
    Dual pv[4];
#pragma unroll
    for (int b = 0; b < 4; ++b) pv[b] = Dual(p0[b], a == b ? 1.0 : 0.0);
    const Dual jx = pv[0] * pv[1], jy = pv[0] * pv[2];
    const Dual e = pv[0] * (pv[3] + 0.5 * (pv[1] * pv[1] + pv[2] * pv[2]));
    Dual q[16];
    equilibrium_moments<VER, Dual>(pv[0], jx, jy, e, q);
    double s = 0.0;
#pragma unroll
    for (int kk = 0; kk < 16; ++kk) s += mu[kk] * q[kk].d;
    g[a] = s;
  }
  if (g_rho) g_rho[d] = g[0];
  if (g_ux) g_ux[d] = g[1];
  if (g_uy) g_uy[d] = g[2];
  if (g_T) g_T[d] = g[3];
}

template <int VER>
__global__ void k_adj_init(Field F, const double* __restrict__ lam, const double* __restrict__ rho,
                           const double* __restrict__ ux, const double* __restrict__ uy, const double* __restrict__ T,
                           double* g_rho, double* g_ux, double* g_uy, double* g_T) {
  const int x = blockIdx.x * blockDim.x + threadIdx.x;
  const int y = blockIdx.y;
  if (x >= F.nx) return;
  adj_init_node<VER>(F, lam, rho, ux, uy, T, g_rho, g_ux, g_uy, g_T, x, y);
}

// One pass of the fixed-order reduction of per-block partials [nrows][12]:
// out row r = sum of input rows r*CHUNK .. r*CHUNK + CHUNK - 1 (in order).
constexpr int ADJ_CHUNK = 64;
template <int U>
__global__ void k_adj_reduce(const double* __restrict__ in, int nrows, double* __restrict__ out) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  const long long nout = ((long long)nrows + ADJ_CHUNK - 1) / ADJ_CHUNK;
  if (i >= nout * 12) return;
  const long long r = i / 12;
  const int comp = (int)(i % 12);
  const long long b0 = r * ADJ_CHUNK, b1 = min(b0 + ADJ_CHUNK, (long long)nrows);
  double s = 0.0;
  for (long long b = b0; b < b1; ++b) s += in[b * 12 + comp];
  out[i] = s;
}

// dL/ds_1..16 from the last reduction row (s_1..s_4 have no effect).
template <int U>
__global__ void k_adj_grad(const double* __restrict__ row, double* __restrict__ grad_s) {
  const int k = threadIdx.x;
  if (k < 16) grad_s[k] = (k >= 4) ? row[k - 4] : 0.0;
}

template <int U>
__global__ void k_zero(double* p, long long n) {
  const long long i = (long long)blockIdx.x * blockDim.x + threadIdx.x;
  if (i < n) p[i] = 0.0;
}

}  // namespace lbm
