// Plain FP64 CPU oracle for the compressible two-dimensional 16-velocity MRT
// finite-difference lattice Boltzmann model with the energy-flux collision
// modification (Chen, Xu, Zhang, Li, "Prandtl number effects in MRT lattice
// Boltzmann models for shocked and unshocked compressible fluids").
//
// TEST INFRASTRUCTURE ONLY. Only the test suite, the smoke check and the CPU
// baseline leg of the benchmark load this library. The product path (the HIP
// library) never calls it, and the two share no code, header, table or
// constant generator.
//
// The method is an explicit time-marching scheme, so this file takes the
// algorithm's steps in the paper's order and notation, one node at a time,
// with dense 16x16 matrix products and no blocking, fusion or reordering:
//   moments        f^ = M f                              (Sec. II, Eq. 3 and text)
//   macroscopic    rho, j, e -> u, T = e/rho - u^2/2      (Sec. II; R = 1, Sec. IV)
//   equilibria     f^eq_k, Eqs. (14a)-(14i); free moments 12, 15, 16 by version (Sec. II)
//   relaxation     Q_k = s_k (f^_k - f^eq_k), diagonal S^ (Sec. II, Eq. 3)
//   modification   extra terms in Q_7 and Q_8 (Sec. II, energy-flux modification)
//   collision      -dt M^-1 Q
//   convection     forward Euler in time, per-axis central Lax-Wendroff in
//                  space, read off the amplification matrix G_ij (Sec. III);
//                  optionally (scheme 1) the same Lax-Wendroff update with a
//                  minmod limiter on its anti-diffusive flux (flux-limited,
//                  total-variation-diminishing form; radius 2)
//   walls          non-equilibrium extrapolation (Sec. IV.A)
//
// Readings where the paper is silent (each listed in the design notes):
//   * velocity gradients in the modification are second-order central
//     differences of the nodal velocity at time level n;
//   * all right-hand-side terms are evaluated at level n (single stage);
//   * non-equilibrium extrapolation walls sit on the first/last node of the
//     walled axis, take rho from the adjacent fluid node and copy that node's
//     non-equilibrium part, evaluated after the interior update;
//   * ghost layers: periodic wrap, zero-gradient copy, specular mirror (the
//     normal velocity component negated), or the equilibrium of a fixed state;
//     two layers deep for the radius-2 scheme: the second zero-gradient layer
//     repeats the boundary node, the second mirror layer mirrors the node
//     next to it (reflection about the wall half a spacing outside the
//     boundary node).
//
// Parity status: the algorithm is pinned by the CPU tests (closed-form
// equilibria, transport coefficients, thermal Couette profile, gamma = 2
// Riemann solutions, conservation, symmetry). The free equilibrium moments
// of version 3 are pinned against the sampled Maxwellian's moments in closed
// form; those of version 2 only by their symmetry under reflection and
// rotation ("parity unpinned" beyond that: the paper gives no worked value).
//
// Scalar type is a template parameter so the same code runs in complex
// arithmetic for complex-step derivatives (every operation used is analytic).

#include <cmath>
#include <complex>
#include <cstdint>
#include <cstring>
#include <vector>

#ifdef _OPENMP
#include <omp.h>
#endif

namespace {

constexpr int NQ = 16;

// Discrete velocities (Sec. II, Fig. 1): i = 1..4 cyc(+-1, 0); 5..8 (+-1, +-1);
// 9..12 cyc(+-2, 0); 13..16 (+-2, +-2). The order within each group is the
// column order of rows m2 (v_x) and m3 (v_y) of M.
const int VEL[NQ][2] = {
    {1, 0},  {0, 1},  {-1, 0},  {0, -1},   //
    {1, 1},  {-1, 1}, {-1, -1}, {1, -1},   //
    {2, 0},  {0, 2},  {-2, 0},  {0, -2},   //
    {2, 2},  {-2, 2}, {-2, -2}, {2, -2}};

// Rows m1..m16 of the transformation matrix M exactly as printed (Sec. II).
const double MROWS[NQ][NQ] = {
    {1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1, 1},
    {1, 0, -1, 0, 1, -1, -1, 1, 2, 0, -2, 0, 2, -2, -2, 2},
    {0, 1, 0, -1, 1, 1, -1, -1, 0, 2, 0, -2, 2, 2, -2, -2},
    {0.5, 0.5, 0.5, 0.5, 1, 1, 1, 1, 2, 2, 2, 2, 4, 4, 4, 4},
    {1, -1, 1, -1, 0, 0, 0, 0, 4, -4, 4, -4, 0, 0, 0, 0},
    {0, 0, 0, 0, 1, -1, 1, -1, 0, 0, 0, 0, 4, -4, 4, -4},
    {0.5, 0, -0.5, 0, 1, -1, -1, 1, 4, 0, -4, 0, 8, -8, -8, 8},
    {0, 0.5, 0, -0.5, 1, 1, -1, -1, 0, 4, 0, -4, 8, 8, -8, -8},
    {1, 0, -1, 0, -2, 2, 2, -2, 8, 0, -8, 0, -16, 16, 16, -16},
    {0, -1, 0, 1, 2, 2, -2, -2, 0, -8, 0, 8, 16, 16, -16, -16},
    {0.25, 0.25, 0.25, 0.25, 1, 1, 1, 1, 4, 4, 4, 4, 16, 16, 16, 16},
    {1, 1, 1, 1, -4, -4, -4, -4, 16, 16, 16, 16, -64, -64, -64, -64},
    {1, -1, 1, -1, 0, 0, 0, 0, 16, -16, 16, -16, 0, 0, 0, 0},
    {0, 0, 0, 0, 2, -2, 2, -2, 0, 0, 0, 0, 32, -32, 32, -32},
    {1, 0, -1, 0, -4, 4, 4, -4, 32, 0, -32, 0, -128, 128, 128, -128},
    {0, -1, 0, 1, 4, 4, -4, -4, 0, -32, 0, 32, 128, 128, -128, -128}};

// Velocity permutations of the specular mirror: reflecting across a wall
// normal to x negates v_x; across a wall normal to y negates v_y.
int MIRROR_X[NQ];
int MIRROR_Y[NQ];

double MINV[NQ][NQ];
bool TABLES_READY = false;

// M^-1 by Gauss-Jordan elimination with partial pivoting in long double,
// rounded once to binary64.
void build_tables() {
  if (TABLES_READY) return;
  long double a[NQ][2 * NQ];
  for (int r = 0; r < NQ; ++r) {
    for (int c = 0; c < NQ; ++c) a[r][c] = MROWS[r][c];
    for (int c = 0; c < NQ; ++c) a[r][NQ + c] = (r == c) ? 1.0L : 0.0L;
  }
  for (int col = 0; col < NQ; ++col) {
    int piv = col;
    for (int r = col + 1; r < NQ; ++r)
      if (std::fabs(a[r][col]) > std::fabs(a[piv][col])) piv = r;
    if (piv != col)
      for (int c = 0; c < 2 * NQ; ++c) std::swap(a[piv][c], a[col][c]);
    long double d = a[col][col];
    for (int c = 0; c < 2 * NQ; ++c) a[col][c] /= d;
    for (int r = 0; r < NQ; ++r) {
      if (r == col) continue;
      long double m = a[r][col];
      if (m == 0.0L) continue;
      for (int c = 0; c < 2 * NQ; ++c) a[r][c] -= m * a[col][c];
    }
  }
  for (int r = 0; r < NQ; ++r)
    for (int c = 0; c < NQ; ++c) MINV[r][c] = (double)a[r][NQ + c];

  for (int i = 0; i < NQ; ++i) {
    for (int j = 0; j < NQ; ++j) {
      if (VEL[j][0] == -VEL[i][0] && VEL[j][1] == VEL[i][1]) MIRROR_X[i] = j;
      if (VEL[j][0] == VEL[i][0] && VEL[j][1] == -VEL[i][1]) MIRROR_Y[i] = j;
    }
  }
  TABLES_READY = true;
}

// Boundary kinds, one per side (x_lo, x_hi, y_lo, y_hi).
enum { BC_PERIODIC = 0, BC_ZERO_GRADIENT = 1, BC_SPECULAR = 2, BC_NEQ_WALL = 3, BC_DIRICHLET_EQ = 4 };
enum { SIDE_XLO = 0, SIDE_XHI = 1, SIDE_YLO = 2, SIDE_YHI = 3 };

}  // namespace

extern "C" {
// Problem description for the oracle (its own struct; the HIP library has its own).
typedef struct {
  int32_t nx, ny;
  double dx, dy, dt;
  double s[16];
  int32_t eq_version;  // 1, 2 or 3
  int32_t modified;    // 0 unmodified; 1 modified (Eq. 5 consistent); 2 modified, Q_8 sign as printed
  int32_t bc[4];       // x_lo, x_hi, y_lo, y_hi
  double wall[4][4];   // per side: rho, ux, uy, T
  int32_t scheme;      // 0 Lax-Wendroff (Sec. III); 1 the same with a minmod flux limiter
} oracle_params;
}

namespace {

template <class R>
struct Macro {
  R rho, jx, jy, e, ux, uy, T;
};

// Order in which the dense sums below run over their index. The default
// build sums in index order; ORACLE_REVERSED_SUMS builds the same arithmetic
// with every dense sum taken in reverse order: an equally valid evaluation
// of the same definition, used to measure a problem's FP64 noise floor.
#ifdef ORACLE_REVERSED_SUMS
inline int sum_index(int j) { return NQ - 1 - j; }
#else
inline int sum_index(int j) { return j; }
#endif

// f^ = M f, dense.
template <class R>
void to_moments(const R* f, R* fh) {
  for (int k = 0; k < NQ; ++k) {
    R acc = R(0);
    for (int j = 0; j < NQ; ++j) {
      const int i = sum_index(j);
      acc += MROWS[k][i] * f[i];
    }
    fh[k] = acc;
  }
}

// Conserved moments f^_1..f^_4 = rho, j_x, j_y, e = rho (T + u^2/2) with R = 1.
template <class R>
Macro<R> macro_of(const R* fh) {
  Macro<R> m;
  m.rho = fh[0];
  m.jx = fh[1];
  m.jy = fh[2];
  m.e = fh[3];
  m.ux = m.jx / m.rho;
  m.uy = m.jy / m.rho;
  m.T = m.e / m.rho - (m.ux * m.ux + m.uy * m.uy) / 2.0;
  return m;
}

// Equilibrium moments, Eqs. (14a)-(14i); k = 1..4 equal the conserved moments.
// Free moments 12, 15, 16: version 1 zeros, version 2 the printed polynomials,
// version 3 the M-moments of the sampled Maxwellian (Sec. II).
template <class R>
void feq_moments(int version, const Macro<R>& m, R* q) {
  const R rho = m.rho, jx = m.jx, jy = m.jy, e = m.e, T = m.T;
  q[0] = rho;
  q[1] = jx;
  q[2] = jy;
  q[3] = e;
  q[4] = (jx * jx - jy * jy) / rho;                                          // 14a
  q[5] = jx * jy / rho;                                                      // 14b
  q[6] = (e + rho * T) * jx / rho;                                           // 14c (R = 1)
  q[7] = (e + rho * T) * jy / rho;                                           // 14d
  q[8] = (jx * jx - 3.0 * jy * jy) * jx / (rho * rho);                       // 14e
  q[9] = (3.0 * jx * jx - jy * jy) * jy / (rho * rho);                       // 14f
  q[10] = 2.0 * e * e / rho - (jx * jx + jy * jy) * (jx * jx + jy * jy) / (4.0 * rho * rho * rho);  // 14g
  q[12] = (6.0 * rho * e - 2.0 * jx * jx - 2.0 * jy * jy) * (jx * jx - jy * jy) / (rho * rho * rho);  // 14h
  q[13] = (6.0 * rho * e - 2.0 * jx * jx - 2.0 * jy * jy) * jx * jy / (rho * rho * rho);             // 14i
  if (version == 2) {
    const R ux = m.ux, uy = m.uy;
    q[11] = R(0);
    q[14] = rho * ux * (-4.0 + 10.0 * T + 5.0 * ux * ux - 5.0 * uy * uy);
    q[15] = rho * uy * (4.0 - 10.0 * T + 5.0 * ux * ux - 5.0 * uy * uy);
  } else if (version == 3) {
    R fmax[NQ];
    for (int i = 0; i < NQ; ++i) {
      R cx = double(VEL[i][0]) - m.ux, cy = double(VEL[i][1]) - m.uy;
      fmax[i] = rho / (2.0 * M_PI * T) * std::exp(-(cx * cx + cy * cy) / (2.0 * T));
    }
    R a12 = R(0), a15 = R(0), a16 = R(0);
    for (int i = 0; i < NQ; ++i) {
      a12 += MROWS[11][i] * fmax[i];
      a15 += MROWS[14][i] * fmax[i];
      a16 += MROWS[15][i] * fmax[i];
    }
    q[11] = a12;
    q[14] = a15;
    q[15] = a16;
  } else {
    q[11] = R(0);
    q[14] = R(0);
    q[15] = R(0);
  }
}

// Equilibrium distribution f^eq = M^-1 f^eq(rho, u, T), used for the initial
// state, the fixed-state ghost and the non-equilibrium extrapolation walls.
template <class R>
void feq_distribution(int version, R rho, R ux, R uy, R T, R* f) {
  Macro<R> m;
  m.rho = rho;
  m.ux = ux;
  m.uy = uy;
  m.T = T;
  m.jx = rho * ux;
  m.jy = rho * uy;
  m.e = rho * (T + (ux * ux + uy * uy) / 2.0);
  R q[NQ];
  feq_moments(version, m, q);
  for (int i = 0; i < NQ; ++i) {
    R acc = R(0);
    for (int j = 0; j < NQ; ++j) {
      const int k = sum_index(j);
      acc += MINV[i][k] * q[k];
    }
    f[i] = acc;
  }
}

template <class R>
struct Grid {
  int nx, ny;
  std::vector<R> f;  // [y][x][q]
  R* at(int x, int y) { return &f[((size_t)y * nx + x) * NQ]; }
  const R* at(int x, int y) const { return &f[((size_t)y * nx + x) * NQ]; }
};

inline bool is_wall_node(const oracle_params& p, int x, int y) {
  if (p.bc[SIDE_XLO] == BC_NEQ_WALL && x == 0) return true;
  if (p.bc[SIDE_XHI] == BC_NEQ_WALL && x == p.nx - 1) return true;
  if (p.bc[SIDE_YLO] == BC_NEQ_WALL && y == 0) return true;
  if (p.bc[SIDE_YHI] == BC_NEQ_WALL && y == p.ny - 1) return true;
  return false;
}

// The distribution at grid point (xn, yn), which lies inside the domain or in
// a ghost layer of one side: a stored node, or a ghost built by that side's
// condition (periodic wrap, zero-gradient copy of the boundary node, mirror
// image about the wall half a spacing outside the boundary node with the
// normal velocity negated, or the equilibrium of the side's fixed state).
template <class R>
void point_value(const oracle_params& p, const Grid<R>& g, int xn, int yn, R* out) {
  int side = -1;
  if (xn < 0) side = SIDE_XLO;
  if (xn >= p.nx) side = SIDE_XHI;
  if (yn < 0) side = SIDE_YLO;
  if (yn >= p.ny) side = SIDE_YHI;
  if (side < 0) {
    const R* src = g.at(xn, yn);
    for (int i = 0; i < NQ; ++i) out[i] = src[i];
    return;
  }
  const int kind = p.bc[side];
  const bool xside = side == SIDE_XLO || side == SIDE_XHI;
  const int n = xside ? p.nx : p.ny;
  int k = xside ? xn : yn;
  if (kind == BC_DIRICHLET_EQ) {  // (a wall side never needs a ghost: its nodes are not stepped)
    const double* w = p.wall[side];
    feq_distribution<R>(p.eq_version, R(w[0]), R(w[1]), R(w[2]), R(w[3]), out);
    return;
  }
  if (kind == BC_PERIODIC) k = ((k % n) + n) % n;
  else if (kind == BC_ZERO_GRADIENT) k = (k < 0) ? 0 : n - 1;
  else k = (k < 0) ? -1 - k : 2 * n - 1 - k;  // specular mirror image
  if (k < 0) k = 0;
  if (k > n - 1) k = n - 1;
  const R* src = xside ? g.at(k, yn) : g.at(xn, k);
  if (kind == BC_SPECULAR) {
    const int* perm = xside ? MIRROR_X : MIRROR_Y;
    for (int i = 0; i < NQ; ++i) out[i] = src[perm[i]];
  } else {
    for (int i = 0; i < NQ; ++i) out[i] = src[i];
  }
}

// The distribution at the stencil point (x + ox, y + oy) of node (x, y).
template <class R>
void stencil_point(const oracle_params& p, const Grid<R>& g, int x, int y, int ox, int oy, R* out) {
  point_value(p, g, x + ox, y + oy, out);
}

inline double real_part(double v) { return v; }
inline double real_part(const std::complex<double>& v) { return v.real(); }

// minmod(a, b): the argument of smaller magnitude when both have the same
// sign, else 0 (decisions on the real part, so that the complex build takes
// the derivative of the branch the real computation takes).
template <class R>
R minmod(R a, R b) {
  const double ra = real_part(a), rb = real_part(b);
  if (!(ra * rb > 0.0)) return R(0);
  return (std::fabs(ra) < std::fabs(rb)) ? a : b;
}

// Convection increment of one distribution along one axis for the
// flux-limited scheme: Lax-Wendroff (Sec. III) whose anti-diffusive flux
// (c/2)(1-|c|)(f_{j+1} - f_j) is limited by minmod of the two adjacent
// differences; c = v dt / dx, f2m .. f2p the values at j-2 .. j+2. With the
// limiter replaced by its first argument it is exactly Sec. III's scheme.
template <class R>
R limited_lw(double c, R f2m, R f1m, R f0, R f1p, R f2p) {
  const R dm = f0 - f1m, dp = f1p - f0;
  if (c > 0.0) {
    const double k = 0.5 * c * (1.0 - c);
    const R dmm = f1m - f2m;
    return -c * dm - k * (minmod(dp, dm) - minmod(dm, dmm));
  }
  const double a = -c, k = 0.5 * a * (1.0 - a);
  const R dpp = f2p - f1p;
  return a * dp - k * (minmod(dp, dpp) - minmod(dm, dp));
}

template <class R>
void velocity_of(const R* f, R& ux, R& uy) {
  R fh[NQ];
  to_moments(f, fh);
  Macro<R> m = macro_of(fh);
  ux = m.ux;
  uy = m.uy;
}

// One time step f^n -> f^{n+1} at interior (non-wall) node (x, y).
template <class R>
void update_node(const oracle_params& p, const R* s, const Grid<R>& g, int x, int y, R* out) {
  const R* f = g.at(x, y);

  // Stencil points: +x, -x, +y, -y.
  R fxp[NQ], fxm[NQ], fyp[NQ], fym[NQ];
  stencil_point(p, g, x, y, +1, 0, fxp);
  stencil_point(p, g, x, y, -1, 0, fxm);
  stencil_point(p, g, x, y, 0, +1, fyp);
  stencil_point(p, g, x, y, 0, -1, fym);
  // Second neighbours, used by the flux-limited scheme only.
  R fxp2[NQ], fxm2[NQ], fyp2[NQ], fym2[NQ];
  if (p.scheme == 1) {
    stencil_point(p, g, x, y, +2, 0, fxp2);
    stencil_point(p, g, x, y, -2, 0, fxm2);
    stencil_point(p, g, x, y, 0, +2, fyp2);
    stencil_point(p, g, x, y, 0, -2, fym2);
  }

  // Moments and macroscopic variables at the node.
  R fh[NQ];
  to_moments(f, fh);
  Macro<R> m = macro_of(fh);
  R feq[NQ];
  feq_moments(p.eq_version, m, feq);

  // Relaxation Q_k = s_k (f^_k - f^eq_k); the conserved k = 1..4 give zero.
  R Q[NQ];
  for (int k = 0; k < NQ; ++k) Q[k] = (k < 4) ? R(0) : s[k] * (fh[k] - feq[k]);

  // Energy-flux modification of Q_7 and Q_8 with central-difference gradients.
  if (p.modified) {
    R uxp, uyp, uxm, uym, vxp, vyp, vxm, vym;
    velocity_of(fxp, uxp, uyp);
    velocity_of(fxm, uxm, uym);
    velocity_of(fyp, vxp, vyp);
    velocity_of(fym, vxm, vym);
    const R dux_dx = (uxp - uxm) / (2.0 * p.dx);
    const R duy_dx = (uyp - uym) / (2.0 * p.dx);
    const R dux_dy = (vxp - vxm) / (2.0 * p.dy);
    const R duy_dy = (vyp - vym) / (2.0 * p.dy);
    const R A = dux_dx - duy_dy;
    const R B = duy_dx + dux_dy;
    const R rT = m.rho * m.T;
    // s index k is s[k - 1]. The normal-stress term of Q_8 is taken with
    // u_y (d_y u_y - d_x u_x), the sign for which the recovered energy
    // equation is Eq. (5) (its y flux in Eq. (15d) carries -u_y A);
    // modified == 2 keeps the sign exactly as printed, u_y (d_x u_x - d_y u_y).
    const double sgn8 = (p.modified == 2) ? 1.0 : -1.0;
    Q[6] += (s[6] / s[4] - 1.0) * rT * m.ux * A + (s[6] / s[5] - 1.0) * rT * m.uy * B;
    Q[7] += (s[7] / s[5] - 1.0) * rT * m.ux * B + sgn8 * (s[7] / s[4] - 1.0) * rT * m.uy * A;
  }

  // Collision in velocity space: -dt M^-1 Q.
  for (int i = 0; i < NQ; ++i) {
    R coll = R(0);
    for (int j = 0; j < NQ; ++j) {
      const int k = sum_index(j);
      coll += MINV[i][k] * Q[k];
    }
    coll = -p.dt * coll;

    const double cx = VEL[i][0] * p.dt / p.dx;
    const double cy = VEL[i][1] * p.dt / p.dy;
    R conv;
    if (p.scheme == 0) {
      // Central Lax-Wendroff convection, axis by axis, as in G_ij (Sec. III).
      conv = -0.5 * cx * (fxp[i] - fxm[i]) + 0.5 * cx * cx * (fxp[i] - 2.0 * f[i] + fxm[i]) -
             0.5 * cy * (fyp[i] - fym[i]) + 0.5 * cy * cy * (fyp[i] - 2.0 * f[i] + fym[i]);
    } else {
      // The same scheme with a minmod-limited anti-diffusive flux, axis by axis.
      conv = R(0);
      if (VEL[i][0] != 0) conv += limited_lw(cx, fxm2[i], fxm[i], f[i], fxp[i], fxp2[i]);
      if (VEL[i][1] != 0) conv += limited_lw(cy, fym2[i], fym[i], f[i], fyp[i], fyp2[i]);
    }
    out[i] = f[i] + conv + coll;
  }
}

// Non-equilibrium extrapolation: the wall node takes the equilibrium of
// (rho of the adjacent fluid node, wall velocity, wall temperature) plus that
// node's non-equilibrium part, all at the new time level.
template <class R>
void neq_wall(const oracle_params& p, Grid<R>& g, int x, int y, int xn, int yn, int side) {
  const R* fn = g.at(xn, yn);
  R fh[NQ];
  to_moments(fn, fh);
  Macro<R> m = macro_of(fh);
  R eq_w[NQ], eq_n[NQ];
  const double* w = p.wall[side];
  feq_distribution<R>(p.eq_version, m.rho, R(w[1]), R(w[2]), R(w[3]), eq_w);
  feq_distribution<R>(p.eq_version, m.rho, m.ux, m.uy, m.T, eq_n);
  R* fw = g.at(x, y);
  for (int i = 0; i < NQ; ++i) fw[i] = eq_w[i] + (fn[i] - eq_n[i]);
}

template <class R>
void step(const oracle_params& p, const R* s, const Grid<R>& in, Grid<R>& out, int nthreads) {
  const long long n = (long long)p.nx * p.ny;
#pragma omp parallel for schedule(static) num_threads(nthreads)
  for (long long idx = 0; idx < n; ++idx) {
    const int x = (int)(idx % p.nx), y = (int)(idx / p.nx);
    if (is_wall_node(p, x, y)) continue;
    update_node(p, s, in, x, y, out.at(x, y));
  }
  if (p.bc[SIDE_YLO] == BC_NEQ_WALL)
    for (int x = 0; x < p.nx; ++x) neq_wall(p, out, x, 0, x, 1, SIDE_YLO);
  if (p.bc[SIDE_YHI] == BC_NEQ_WALL)
    for (int x = 0; x < p.nx; ++x) neq_wall(p, out, x, p.ny - 1, x, p.ny - 2, SIDE_YHI);
  if (p.bc[SIDE_XLO] == BC_NEQ_WALL)
    for (int y = 0; y < p.ny; ++y) neq_wall(p, out, 0, y, 1, y, SIDE_XLO);
  if (p.bc[SIDE_XHI] == BC_NEQ_WALL)
    for (int y = 0; y < p.ny; ++y) neq_wall(p, out, p.nx - 1, y, p.nx - 2, y, SIDE_XHI);
}

int check_params(const oracle_params* p) {
  if (!p || p->nx < 1 || p->ny < 1) return -1;
  if (!(p->dx > 0) || !(p->dy > 0) || !(p->dt > 0)) return -1;
  if (p->eq_version < 1 || p->eq_version > 3) return -1;
  if (p->modified < 0 || p->modified > 2) return -1;
  if (p->scheme < 0 || p->scheme > 1) return -1;
  for (int a = 0; a < 2; ++a) {
    int lo = p->bc[2 * a], hi = p->bc[2 * a + 1];
    if (lo < 0 || lo > 4 || hi < 0 || hi > 4) return -1;
    if ((lo == BC_PERIODIC) != (hi == BC_PERIODIC)) return -1;
  }
  const bool xwall = p->bc[0] == BC_NEQ_WALL || p->bc[1] == BC_NEQ_WALL;
  const bool ywall = p->bc[2] == BC_NEQ_WALL || p->bc[3] == BC_NEQ_WALL;
  if (xwall && ywall) return -1;
  if (xwall && p->nx < 3) return -1;
  if (ywall && p->ny < 3) return -1;
  if (p->nx == 1 && p->bc[0] != BC_PERIODIC) return -1;
  if (p->ny == 1 && p->bc[2] != BC_PERIODIC) return -1;
  return 0;
}

template <class R>
void load_soa(const oracle_params& p, Grid<R>& g, const double* re, const double* im) {
  const size_t n = (size_t)p.nx * p.ny;
  g.nx = p.nx;
  g.ny = p.ny;
  g.f.assign(n * NQ, R(0));
  for (int q = 0; q < NQ; ++q)
    for (size_t c = 0; c < n; ++c) {
      if constexpr (std::is_same<R, double>::value) {
        g.f[c * NQ + q] = re[q * n + c];
      } else {
        g.f[c * NQ + q] = R(re[q * n + c], im ? im[q * n + c] : 0.0);
      }
    }
}

template <class R>
void store_soa(const oracle_params& p, const Grid<R>& g, double* re, double* im) {
  const size_t n = (size_t)p.nx * p.ny;
  for (int q = 0; q < NQ; ++q)
    for (size_t c = 0; c < n; ++c) {
      if constexpr (std::is_same<R, double>::value) {
        re[q * n + c] = g.f[c * NQ + q];
      } else {
        re[q * n + c] = g.f[c * NQ + q].real();
        if (im) im[q * n + c] = g.f[c * NQ + q].imag();
      }
    }
}

template <class R>
void run(const oracle_params& p, const R* s, Grid<R>& g, int64_t nsteps, int nthreads) {
  Grid<R> other;
  other.nx = g.nx;
  other.ny = g.ny;
  other.f = g.f;  // wall nodes are overwritten each step; copying keeps them defined
  for (int64_t n = 0; n < nsteps; ++n) {
    step(p, s, g, other, nthreads);
    std::swap(g.f, other.f);
  }
}

template <class R>
void init_fields(const oracle_params& p, Grid<R>& g, const R* rho, const R* ux, const R* uy, const R* T) {
  const size_t n = (size_t)p.nx * p.ny;
  g.nx = p.nx;
  g.ny = p.ny;
  g.f.assign(n * NQ, R(0));
  for (size_t c = 0; c < n; ++c) feq_distribution<R>(p.eq_version, rho[c], ux[c], uy[c], T[c], &g.f[c * NQ]);
}

template <class R>
void fields_of(const oracle_params& p, const Grid<R>& g, R* rho, R* ux, R* uy, R* T, R* P) {
  const size_t n = (size_t)p.nx * p.ny;
  for (size_t c = 0; c < n; ++c) {
    R fh[NQ];
    to_moments(&g.f[c * NQ], fh);
    Macro<R> m = macro_of(fh);
    if (rho) rho[c] = m.rho;
    if (ux) ux[c] = m.ux;
    if (uy) uy[c] = m.uy;
    if (T) T[c] = m.T;
    if (P) P[c] = m.rho * m.T;
  }
}

int clamp_threads(int nthreads) {
  if (nthreads < 1) nthreads = 1;
  return nthreads;
}

}  // namespace

extern "C" {

// Velocity table [16][2], M [16][16] and the oracle's own M^-1 [16][16], row-major.
int oracle_matrices(double* vel, double* m, double* minv) {
  build_tables();
  for (int i = 0; i < NQ; ++i) {
    if (vel) {
      vel[2 * i] = VEL[i][0];
      vel[2 * i + 1] = VEL[i][1];
    }
    for (int k = 0; k < NQ; ++k) {
      if (m) m[i * NQ + k] = MROWS[i][k];
      if (minv) minv[i * NQ + k] = MINV[i][k];
    }
  }
  return 0;
}

// Equilibrium moments f^eq_1..16 at one state.
int oracle_feq_moments(int version, double rho, double ux, double uy, double T, double* out) {
  build_tables();
  if (version < 1 || version > 3) return -1;
  Macro<double> m;
  m.rho = rho;
  m.ux = ux;
  m.uy = uy;
  m.T = T;
  m.jx = rho * ux;
  m.jy = rho * uy;
  m.e = rho * (T + (ux * ux + uy * uy) / 2.0);
  feq_moments(version, m, out);
  return 0;
}

// For one node's distributions f (16 complex values): the equilibrium
// moments f^eq_1..16 and (rho, u_x, u_y, T), through the same moment and
// macroscopic steps as the time step (complex, so that a complex-step
// perturbation of f yields their derivatives with respect to f).
int oracle_node_equilibrium_complex(int version, const double* f_re, const double* f_im, double* q_re, double* q_im,
                                    double* mac) {
  build_tables();
  if (version < 1 || version > 3) return -1;
  using C = std::complex<double>;
  C f[NQ], fh[NQ], q[NQ];
  for (int i = 0; i < NQ; ++i) f[i] = C(f_re[i], f_im[i]);
  to_moments(f, fh);
  Macro<C> m = macro_of(fh);
  feq_moments(version, m, q);
  for (int k = 0; k < NQ; ++k) {
    q_re[k] = q[k].real();
    q_im[k] = q[k].imag();
  }
  const C v[4] = {m.rho, m.ux, m.uy, m.T};
  for (int k = 0; k < 4; ++k) {
    mac[2 * k] = v[k].real();
    mac[2 * k + 1] = v[k].imag();
  }
  return 0;
}

// Equilibrium moments f^eq_1..16 at one complex state (rho, u_x, u_y, T)
// ([4] real and imaginary parts), so that a complex-step perturbation of one
// of them yields the derivatives with respect to it.
int oracle_feq_moments_complex(int version, const double* v_re, const double* v_im, double* q_re, double* q_im) {
  build_tables();
  if (version < 1 || version > 3) return -1;
  using C = std::complex<double>;
  Macro<C> m;
  m.rho = C(v_re[0], v_im[0]);
  m.ux = C(v_re[1], v_im[1]);
  m.uy = C(v_re[2], v_im[2]);
  m.T = C(v_re[3], v_im[3]);
  m.jx = m.rho * m.ux;
  m.jy = m.rho * m.uy;
  m.e = m.rho * (m.T + (m.ux * m.ux + m.uy * m.uy) / 2.0);
  C q[NQ];
  feq_moments(version, m, q);
  for (int k = 0; k < NQ; ++k) {
    q_re[k] = q[k].real();
    q_im[k] = q[k].imag();
  }
  return 0;
}

// f = M^-1 f^eq(rho, u, T) at every node; fields [ny][nx], f [16][ny][nx].
int oracle_init(const oracle_params* p, const double* rho, const double* ux, const double* uy, const double* T,
                double* f) {
  build_tables();
  if (check_params(p)) return -1;
  Grid<double> g;
  init_fields<double>(*p, g, rho, ux, uy, T);
  store_soa(*p, g, f, nullptr);
  return 0;
}

// rho, u_x, u_y, T, p = rho T at every node (any output may be NULL).
int oracle_moments(const oracle_params* p, const double* f, double* rho, double* ux, double* uy, double* T,
                   double* P) {
  build_tables();
  if (check_params(p)) return -1;
  Grid<double> g;
  load_soa(*p, g, f, nullptr);
  fields_of<double>(*p, g, rho, ux, uy, T, P);
  return 0;
}

// nsteps time steps from f_in to f_out (both [16][ny][nx]; may alias).
int oracle_run(const oracle_params* p, const double* f_in, int64_t nsteps, double* f_out, int nthreads) {
  build_tables();
  if (check_params(p) || nsteps < 0) return -1;
  Grid<double> g;
  load_soa(*p, g, f_in, nullptr);
  run<double>(*p, p->s, g, nsteps, clamp_threads(nthreads));
  store_soa(*p, g, f_out, nullptr);
  return 0;
}

// Complex-step variants: every input carries an imaginary part (NULL = 0),
// including the relaxation rates (s_im, 16 values).
int oracle_init_complex(const oracle_params* p, const double* rho_re, const double* rho_im, const double* ux_re,
                        const double* ux_im, const double* uy_re, const double* uy_im, const double* T_re,
                        const double* T_im, double* f_re, double* f_im) {
  using C = std::complex<double>;
  build_tables();
  if (check_params(p)) return -1;
  const size_t n = (size_t)p->nx * p->ny;
  std::vector<C> rho(n), ux(n), uy(n), T(n);
  for (size_t c = 0; c < n; ++c) {
    rho[c] = C(rho_re[c], rho_im ? rho_im[c] : 0.0);
    ux[c] = C(ux_re[c], ux_im ? ux_im[c] : 0.0);
    uy[c] = C(uy_re[c], uy_im ? uy_im[c] : 0.0);
    T[c] = C(T_re[c], T_im ? T_im[c] : 0.0);
  }
  Grid<C> g;
  init_fields<C>(*p, g, rho.data(), ux.data(), uy.data(), T.data());
  store_soa(*p, g, f_re, f_im);
  return 0;
}

int oracle_run_complex(const oracle_params* p, const double* s_im, const double* f_re, const double* f_im,
                       int64_t nsteps, double* out_re, double* out_im, int nthreads) {
  using C = std::complex<double>;
  build_tables();
  if (check_params(p) || nsteps < 0) return -1;
  C s[NQ];
  for (int k = 0; k < NQ; ++k) s[k] = C(p->s[k], s_im ? s_im[k] : 0.0);
  Grid<C> g;
  load_soa(*p, g, f_re, f_im);
  run<C>(*p, s, g, nsteps, clamp_threads(nthreads));
  store_soa(*p, g, out_re, out_im);
  return 0;
}

int oracle_moments_complex(const oracle_params* p, const double* f_re, const double* f_im, double* rho_re,
                           double* rho_im, double* ux_re, double* ux_im, double* uy_re, double* uy_im,
                           double* T_re, double* T_im) {
  using C = std::complex<double>;
  build_tables();
  if (check_params(p)) return -1;
  Grid<C> g;
  load_soa(*p, g, f_re, f_im);
  const size_t n = (size_t)p->nx * p->ny;
  std::vector<C> rho(n), ux(n), uy(n), T(n);
  fields_of<C>(*p, g, rho.data(), ux.data(), uy.data(), T.data(), nullptr);
  for (size_t c = 0; c < n; ++c) {
    rho_re[c] = rho[c].real();
    if (rho_im) rho_im[c] = rho[c].imag();
    ux_re[c] = ux[c].real();
    if (ux_im) ux_im[c] = ux[c].imag();
    uy_re[c] = uy[c].real();
    if (uy_im) uy_im[c] = uy[c].imag();
    T_re[c] = T[c].real();
    if (T_im) T_im[c] = T[c].imag();
  }
  return 0;
}

int oracle_max_threads(void) {
#ifdef _OPENMP
  return omp_get_max_threads();
#else
  return 1;
#endif
}

}  // extern "C"
