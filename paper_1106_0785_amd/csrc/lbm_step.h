// Device-side description of one time step and the node update shared by
// every step kernel (plain, fused, batched). The update follows Eq. (3) with
// the scheme of Sec. III: explicit collision at the old level plus per-axis
// central Lax-Wendroff convection, and the energy-flux modification (Sec. II).
#pragma once

#include "lbm_node.h"

namespace lbm {

enum { BC_PERIODIC = 0, BC_ZERO_GRADIENT = 1, BC_SPECULAR = 2, BC_NEQ_WALL = 3, BC_DIRICHLET_EQ = 4 };

// Per-problem coefficients read in the inner loop (kept small: they live in
// scalar registers).
struct Hot {
  double cq[12];   // -dt s_k for k = 5..16 (index k-5)
  double cmod[4];  // -dt (s7/s5-1), -dt (s7/s6-1), -dt (s8/s6-1), -dt sgn (s8/s5-1); 0 if unmodified
  double inv2dx, inv2dy;
  // Lax-Wendroff along one axis for a velocity component v = +1 / +2 with
  // c = v dt/dx: coefficient of f(x+1) is p = (c^2 - c)/2 and of f(x-1) is
  // m = (c^2 + c)/2; for v = -1 / -2 the two swap. Stored as p1, m1, p2, m2.
  double lx[4], ly[4];
  // Flux-limited scheme (scheme 1) along one axis: for speeds 1 and 2,
  // a = |v| dt/dx and k = a (1 - a)/2. Stored as a1, k1, a2, k2.
  double tx[4], ty[4];
  int bc[4];
  int version;
  int modified;
  int scheme;  // 0 Lax-Wendroff (Sec. III); 1 its minmod flux-limited form
};

// Rarely read per-problem data.
struct Cold {
  double ghost[4][16];  // equilibrium ghosts of DIRICHLET_EQ sides
  double wall[4][4];    // (rho, ux, uy, T) per side for NEQ walls
};

// Neighbour velocities the modification needs.
struct NbrVel {
  double ux_xp, uy_xp, ux_xm, uy_xm;  // at x+1, x-1
  double ux_yp, uy_yp, ux_ym, uy_ym;  // at y+1, y-1
};

LBM_HD void velocity_of(const double* f, double& ux, double& uy) {
  double rho, jx, jy;
  density_momentum(f, rho, jx, jy);
  const double ir = 1.0 / rho;
  ux = jx * ir;
  uy = jy * ir;
}

// Lax-Wendroff convection increment of velocity I (Sec. III, G_ij):
// sum over axes of p (f(+1) - f) + m (f(-1) - f), with p = (c^2 - c)/2 and
// m = (c^2 + c)/2 for c = v dt/dx. Written with differences so that a
// uniform state is reproduced exactly and the grid totals of rho, j, e are
// conserved to rounding (a centre coefficient 1 - c^2 would scale every
// distribution by a rounding bias each step).
template <int I>
LBM_HD double convect(const Hot& c, double f, double fxp, double fxm, double fyp, double fym) {
  double v = 0.0;
  if (VX[I] == 1) v += c.lx[0] * (fxp - f) + c.lx[1] * (fxm - f);
  if (VX[I] == -1) v += c.lx[1] * (fxp - f) + c.lx[0] * (fxm - f);
  if (VX[I] == 2) v += c.lx[2] * (fxp - f) + c.lx[3] * (fxm - f);
  if (VX[I] == -2) v += c.lx[3] * (fxp - f) + c.lx[2] * (fxm - f);
  if (VY[I] == 1) v += c.ly[0] * (fyp - f) + c.ly[1] * (fym - f);
  if (VY[I] == -1) v += c.ly[1] * (fyp - f) + c.ly[0] * (fym - f);
  if (VY[I] == 2) v += c.ly[2] * (fyp - f) + c.ly[3] * (fym - f);
  if (VY[I] == -2) v += c.ly[3] * (fyp - f) + c.ly[2] * (fym - f);
  return v;
}

// minmod(a, b): the argument of smaller magnitude when both have the same
// sign, else 0.
LBM_HD double minmod(double a, double b) { return (a * b > 0.0) ? (fabs(a) < fabs(b) ? a : b) : 0.0; }

// Flux-limited convection increment along one axis (scheme 1): the
// Lax-Wendroff update of Sec. III whose anti-diffusive flux k (f(+1) - f) is
// limited by minmod of the two differences around it; POS: velocity
// component > 0; (a, k) from Hot::tx / Hot::ty for this speed; f2m .. f2p the
// values at -2 .. +2 along the axis. With minmod(d1, d2) replaced by d1 it is
// exactly convect() below.
template <bool POS>
LBM_HD double limited_axis(double a, double k, double f2m, double f1m, double f0, double f1p, double f2p) {
  const double dm = f0 - f1m, dp = f1p - f0;
  if (POS) return -a * dm - k * (minmod(dp, dm) - minmod(dm, f1m - f2m));
  return a * dp - k * (minmod(dp, f2p - f1p) - minmod(dm, dp));
}

// Both axes of velocity I with the flux-limited scheme.
template <int I>
LBM_HD double convect_limited(const Hot& c, double f, double x2m, double x1m, double x1p, double x2p, double y2m,
                              double y1m, double y1p, double y2p) {
  double v = 0.0;
  constexpr int ax = VX[I] < 0 ? -VX[I] : VX[I], ay = VY[I] < 0 ? -VY[I] : VY[I];
  if constexpr (ax != 0)
    v += limited_axis<(VX[I] > 0)>(c.tx[2 * (ax - 1)], c.tx[2 * (ax - 1) + 1], x2m, x1m, f, x1p, x2p);
  if constexpr (ay != 0)
    v += limited_axis<(VY[I] > 0)>(c.ty[2 * (ay - 1)], c.ty[2 * (ay - 1) + 1], y2m, y1m, f, y1p, y2p);
  return v;
}

// convect_limited<I> for a run-time velocity index (unrolled loops only).
LBM_HD double convect_limited_i(const Hot& c, int i, double f, double x2m, double x1m, double x1p, double x2p,
                                double y2m, double y1m, double y1p, double y2p) {
  double v = 0.0;
#define LBM_CASE(I) \
  case I: v = convect_limited<I>(c, f, x2m, x1m, x1p, x2p, y2m, y1m, y1p, y2p); break;
  switch (i) {
    LBM_CASE(0) LBM_CASE(1) LBM_CASE(2) LBM_CASE(3) LBM_CASE(4) LBM_CASE(5) LBM_CASE(6) LBM_CASE(7)
    LBM_CASE(8) LBM_CASE(9) LBM_CASE(10) LBM_CASE(11) LBM_CASE(12) LBM_CASE(13) LBM_CASE(14) LBM_CASE(15)
  }
#undef LBM_CASE
  return v;
}

template <int I>
struct ConvAll {
  LBM_HD static void run(const Hot& c, const double* f, const double* fxp, const double* fxm, const double* fyp,
                         const double* fym, double* out) {
    out[I] = convect<I>(c, f[I], fxp[I], fxm[I], fyp[I], fym[I]);
    ConvAll<I + 1>::run(c, f, fxp, fxm, fyp, fym, out);
  }
};
template <>
struct ConvAll<16> {
  LBM_HD static void run(const Hot&, const double*, const double*, const double*, const double*, const double*,
                         double*) {}
};

// The Lax-Wendroff increment of velocity I along one axis only (AXIS 0: x,
// 1: y), for a node whose neighbours along the other axis are itself (a
// one-dimensional problem: those terms are exact zeros, left out).
template <int I, int AXIS>
LBM_HD double convect_axis(const Hot& c, double f, double fp, double fm) {
  constexpr int v = AXIS == 0 ? VX[I] : VY[I];
  const double* l = AXIS == 0 ? c.lx : c.ly;
  if (v == 1) return l[0] * (fp - f) + l[1] * (fm - f);
  if (v == -1) return l[1] * (fp - f) + l[0] * (fm - f);
  if (v == 2) return l[2] * (fp - f) + l[3] * (fm - f);
  if (v == -2) return l[3] * (fp - f) + l[2] * (fm - f);
  return 0.0;
}

template <int I, int AXIS>
struct ConvAxis {
  LBM_HD static void run(const Hot& c, const double* f, const double* fp, const double* fm, double* out) {
    out[I] = convect_axis<I, AXIS>(c, f[I], fp[I], fm[I]);
    ConvAxis<I + 1, AXIS>::run(c, f, fp, fm, out);
  }
};
template <int AXIS>
struct ConvAxis<16, AXIS> {
  LBM_HD static void run(const Hot&, const double*, const double*, const double*, double*) {}
};

// Collision of one node in velocity space, -dt M^-1 Q (Sec. II), into df,
// from the node's moments m = M f and ir = 1 / m[0]. Returns false when
// rho <= 0, T <= 0 or a NaN appears.
template <int VER>
LBM_HD bool collide_from_moments(const Hot& c, const double* m, double ir, const NbrVel& nv, double* df) {
  const double rho = m[0], jx = m[1], jy = m[2], e = m[3];
  double q[16];
  equilibrium_moments<VER, double>(rho, jx, jy, e, q);
  double col[16];
#pragma unroll
  for (int k = 4; k < 16; ++k) col[k] = c.cq[k - 4] * (m[k] - q[k]);
  const double ux = jx * ir, uy = jy * ir;
  const double T = e * ir - 0.5 * (ux * ux + uy * uy);
  {
    // energy-flux modification; its coefficients are exactly 0 for the
    // unmodified model, so the terms then add exactly 0 (no branch)
    const double A = (nv.ux_xp - nv.ux_xm) * c.inv2dx - (nv.uy_yp - nv.uy_ym) * c.inv2dy;
    const double B = (nv.uy_xp - nv.uy_xm) * c.inv2dx + (nv.ux_yp - nv.ux_ym) * c.inv2dy;
    const double rT = rho * T;
    col[6] += c.cmod[0] * rT * ux * A + c.cmod[1] * rT * uy * B;
    col[7] += c.cmod[2] * rT * ux * B + c.cmod[3] * rT * uy * A;
  }
  f_from_nonconserved(col, df);
  return (rho > 0.0) && (T > 0.0);
}

// The same from the distributions f.
template <int VER>
LBM_HD bool collide_delta(const Hot& c, const double* f, const NbrVel& nv, double* df) {
  double m[16];
  moments_from_f(f, m);
  return collide_from_moments<VER>(c, m, 1.0 / m[0], nv, df);
}

// The collision added to the convection increments `acc`; the new
// distributions f + (acc + df) are written to `acc`.
template <int VER>
LBM_HD bool collide_add(const Hot& c, const double* f, const NbrVel& nv, double* acc) {
  double df[16];
  const bool ok = collide_delta<VER>(c, f, nv, df);
#pragma unroll
  for (int i = 0; i < 16; ++i) acc[i] = f[i] + (acc[i] + df[i]);
  return ok;
}

// New distributions at one interior node.
template <int VER>
LBM_HD bool node_update(const Hot& c, const double* f, const double* fxp, const double* fxm, const double* fyp,
                        const double* fym, const NbrVel& nv, double* out) {
  ConvAll<0>::run(c, f, fxp, fxm, fyp, fym, out);
  return collide_add<VER>(c, f, nv, out);
}

// Non-equilibrium extrapolation wall node from its fluid neighbour's new
// distributions fn (Sec. IV.A): f_w = f^eq(rho_n, u_w, T_w) + (f_n - f^eq(rho_n, u_n, T_n)).
template <int VER>
LBM_HD void neq_wall(const double* wall, const double* fn, double* fw) {
  double m[16];
  moments_from_f(fn, m);
  const double rho = m[0], ir = 1.0 / rho;
  const double ux = m[1] * ir, uy = m[2] * ir;
  const double T = m[3] * ir - 0.5 * (ux * ux + uy * uy);
  double ew[16], en[16];
  equilibrium_f<VER>(rho, wall[1], wall[2], wall[3], ew);
  equilibrium_f<VER>(rho, ux, uy, T, en);
#pragma unroll
  for (int i = 0; i < 16; ++i) fw[i] = ew[i] + (fn[i] - en[i]);
}

}  // namespace lbm
