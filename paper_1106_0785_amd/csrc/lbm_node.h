// Per-node arithmetic of the D2V16 MRT finite-difference lattice Boltzmann
// step (Sec. II): moment transform f^ = M f, equilibria f^eq, and the
// back-transform M^-1, in the shell-factorised form generated into
// lbm_consts.h. Host and device; no memory access, no state.
#pragma once

#include <hip/hip_runtime.h>

#include <cmath>

#include "lbm_consts.h"

namespace lbm {

#define LBM_HD __host__ __device__ __forceinline__

// Shell quantities (sigma, gx, gy, q) of the four shells of f (see lbm_consts.h).
template <class S>
LBM_HD void shell_quantities(const S* f, S* sig, S* gx, S* gy, S* q) {
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const S a = f[4 * s + 0], b = f[4 * s + 1], c = f[4 * s + 2], d = f[4 * s + 3];
    const S P = a + c, Q = b + d;
    sig[s] = P + Q;
    q[s] = P - Q;
    if (s == 0 || s == 2) {  // axis shell E, N, W, S
      gx[s] = a - c;
      gy[s] = b - d;
    } else {  // diagonal shell NE, NW, SW, SE
      const S R = a - c, W = b - d;
      gx[s] = R - W;
      gy[s] = R + W;
    }
  }
}

// All 16 moments f^_k = sum_i M_ki f_i (k = 1..16 stored at index k-1).
LBM_HD void moments_from_f(const double* f, double* m) {
  double sig[4], gx[4], gy[4], q[4];
  shell_quantities(f, sig, gx, gy, q);
  const int ks[4] = {0, 3, 10, 11};
  const int kx[4] = {1, 6, 8, 14};
  const int ky[4] = {2, 7, 9, 15};
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    double a = 0.0, b = 0.0, c = 0.0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      a += A_SIG[r][s] * sig[s];
      b += A_GX[r][s] * gx[s];
      c += A_GY[r][s] * gy[s];
    }
    m[ks[r]] = a;
    m[kx[r]] = b;
    m[ky[r]] = c;
  }
  m[4] = A_QA[0][0] * q[0] + A_QA[0][1] * q[2];
  m[12] = A_QA[1][0] * q[0] + A_QA[1][1] * q[2];
  m[5] = A_QD[0][0] * q[1] + A_QD[0][1] * q[3];
  m[13] = A_QD[1][0] * q[1] + A_QD[1][1] * q[3];
}

// rho, j_x, j_y only (the velocity of a neighbour node).
LBM_HD void density_momentum(const double* f, double& rho, double& jx, double& jy) {
  double sig[4], gx[4], gy[4], q[4];
  shell_quantities(f, sig, gx, gy, q);
  rho = (sig[0] + sig[1]) + (sig[2] + sig[3]);
  jx = (gx[0] + gx[1]) + 2.0 * (gx[2] + gx[3]);
  jy = (gy[0] + gy[1]) + 2.0 * (gy[2] + gy[3]);
}

// f = M^-1 m for a full moment vector m (index k-1 holds moment k).
LBM_HD void f_from_moments(const double* m, double* f) {
  double sig[4], gx[4], gy[4], qa[2], qd[2];
  const int ks[4] = {0, 3, 10, 11};
  const int kx[4] = {1, 6, 8, 14};
  const int ky[4] = {2, 7, 9, 15};
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    double a = 0.0, b = 0.0, c = 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      a += AINV_SIG[s][r] * m[ks[r]];
      b += AINV_GX[s][r] * m[kx[r]];
      c += AINV_GY[s][r] * m[ky[r]];
    }
    sig[s] = a;
    gx[s] = b;
    gy[s] = c;
  }
  qa[0] = AINV_QA[0][0] * m[4] + AINV_QA[0][1] * m[12];
  qa[1] = AINV_QA[1][0] * m[4] + AINV_QA[1][1] * m[12];
  qd[0] = AINV_QD[0][0] * m[5] + AINV_QD[0][1] * m[13];
  qd[1] = AINV_QD[1][0] * m[5] + AINV_QD[1][1] * m[13];
  const double q[4] = {qa[0], qd[0], qa[1], qd[1]};
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const double h = 0.25 * sig[s], r = 0.25 * q[s];
    if (s == 0 || s == 2) {  // E, N, W, S
      const double X = 0.5 * gx[s], Y = 0.5 * gy[s];
      f[4 * s + 0] = (h + r) + X;
      f[4 * s + 1] = (h - r) + Y;
      f[4 * s + 2] = (h + r) - X;
      f[4 * s + 3] = (h - r) - Y;
    } else {  // NE, NW, SW, SE
      const double X = 0.25 * gx[s], Y = 0.25 * gy[s];
      f[4 * s + 0] = (h + r) + (X + Y);
      f[4 * s + 1] = (h - r) - (X - Y);
      f[4 * s + 2] = (h + r) - (X + Y);
      f[4 * s + 3] = (h - r) + (X - Y);
    }
  }
}

// Transposed transforms, used by the adjoint.
//
// M^T nu: the transpose of moments_from_f. The block coefficients act on
// nu first (A^T), then each shell's four values are spread back to its
// points with the sign patterns of the shell quantities (S^T).
LBM_HD void mt_apply(const double* nu, double* out) {
  const int ks[4] = {0, 3, 10, 11};
  const int kx[4] = {1, 6, 8, 14};
  const int ky[4] = {2, 7, 9, 15};
  double sig[4], gx[4], gy[4], q[4];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    double a = 0.0, b = 0.0, c = 0.0;
#pragma unroll
    for (int r = 0; r < 4; ++r) {
      a += A_SIG[r][s] * nu[ks[r]];
      b += A_GX[r][s] * nu[kx[r]];
      c += A_GY[r][s] * nu[ky[r]];
    }
    sig[s] = a;
    gx[s] = b;
    gy[s] = c;
  }
  q[0] = A_QA[0][0] * nu[4] + A_QA[1][0] * nu[12];
  q[2] = A_QA[0][1] * nu[4] + A_QA[1][1] * nu[12];
  q[1] = A_QD[0][0] * nu[5] + A_QD[1][0] * nu[13];
  q[3] = A_QD[0][1] * nu[5] + A_QD[1][1] * nu[13];
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    if (s == 0 || s == 2) {  // E, N, W, S
      out[4 * s + 0] = (sig[s] + q[s]) + gx[s];
      out[4 * s + 1] = (sig[s] - q[s]) + gy[s];
      out[4 * s + 2] = (sig[s] + q[s]) - gx[s];
      out[4 * s + 3] = (sig[s] - q[s]) - gy[s];
    } else {  // NE, NW, SW, SE
      out[4 * s + 0] = (sig[s] + q[s]) + (gx[s] + gy[s]);
      out[4 * s + 1] = (sig[s] - q[s]) - (gx[s] - gy[s]);
      out[4 * s + 2] = (sig[s] + q[s]) - (gx[s] + gy[s]);
      out[4 * s + 3] = (sig[s] - q[s]) + (gx[s] - gy[s]);
    }
  }
}

// M^-T lambda: the transpose of f_from_moments. The per-shell
// reconstruction is transposed first (shell quantities of lambda with the
// reconstruction's 1/4 and 1/2 weights), then the inverse blocks.
LBM_HD void minvt_apply(const double* lam, double* mu) {
  double sig[4], gx[4], gy[4], q[4];
  shell_quantities(lam, sig, gx, gy, q);
#pragma unroll
  for (int s = 0; s < 4; ++s) {
    const double wg = (s == 0 || s == 2) ? 0.5 : 0.25;
    sig[s] *= 0.25;
    q[s] *= 0.25;
    gx[s] *= wg;
    gy[s] *= wg;
  }
  const int ks[4] = {0, 3, 10, 11};
  const int kx[4] = {1, 6, 8, 14};
  const int ky[4] = {2, 7, 9, 15};
#pragma unroll
  for (int r = 0; r < 4; ++r) {
    double a = 0.0, b = 0.0, c = 0.0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      a += AINV_SIG[s][r] * sig[s];
      b += AINV_GX[s][r] * gx[s];
      c += AINV_GY[s][r] * gy[s];
    }
    mu[ks[r]] = a;
    mu[kx[r]] = b;
    mu[ky[r]] = c;
  }
  // inverse quadrupole blocks: q of shells 0, 2 from m5, m13; of shells 1, 3 from m6, m14
  mu[4] = AINV_QA[0][0] * q[0] + AINV_QA[1][0] * q[2];
  mu[12] = AINV_QA[0][1] * q[0] + AINV_QA[1][1] * q[2];
  mu[5] = AINV_QD[0][0] * q[1] + AINV_QD[1][0] * q[3];
  mu[13] = AINV_QD[0][1] * q[1] + AINV_QD[1][1] * q[3];
}

// Velocity-space image of a moment vector with only the non-conserved
// components k = 5..16 set: f = M^-1 (0, 0, 0, 0, c_5, ..., c_16).
LBM_HD void f_from_nonconserved(const double* c, double* f) {
  double m[16];
  m[0] = m[1] = m[2] = m[3] = 0.0;
#pragma unroll
  for (int k = 4; k < 16; ++k) m[k] = c[k];
  f_from_moments(m, f);
}

LBM_HD double sexp(double x) { return ::exp(x); }

// Equilibrium moments, Eqs. (14a)-(14i); moments 1..4 are the conserved ones;
// free moments 12, 15, 16 by version VER (1: zero; 2: printed polynomials;
// 3: moments of the Maxwellian sampled at the velocities). S is double, or a
// dual number when the adjoint differentiates this very code.
template <int VER, class S>
LBM_HD void equilibrium_moments(S rho, S jx, S jy, S e, S* q) {
  const S ir = 1.0 / rho;
  const S ux = jx * ir, uy = jy * ir;
  const S jx2 = jx * jx, jy2 = jy * jy;
  const S u2 = ux * ux + uy * uy;
  const S T = e * ir - 0.5 * u2;
  q[0] = rho;
  q[1] = jx;
  q[2] = jy;
  q[3] = e;
  q[4] = (jx2 - jy2) * ir;
  q[5] = jx * jy * ir;
  const S h = (e + rho * T) * ir;  // (e + rho R T)/rho, R = 1
  q[6] = h * jx;
  q[7] = h * jy;
  q[8] = (jx2 - 3.0 * jy2) * ux * ir;
  q[9] = (3.0 * jx2 - jy2) * uy * ir;
  const S j2 = jx2 + jy2;
  q[10] = 2.0 * e * e * ir - 0.25 * j2 * j2 * ir * ir * ir;
  const S w = (6.0 * rho * e - 2.0 * j2) * ir * ir * ir;
  q[12] = w * (jx2 - jy2);
  q[13] = w * jx * jy;
  if constexpr (VER == 2) {
    const S d = 5.0 * ux * ux - 5.0 * uy * uy;
    q[11] = 0.0;
    q[14] = jx * (-4.0 + 10.0 * T + d);
    q[15] = jy * (4.0 - 10.0 * T + d);
  } else if constexpr (VER == 3) {
    S fm[16];
    const S pre = rho / (2.0 * M_PI * T), i2T = 0.5 / T;
#pragma unroll
    for (int i = 0; i < 16; ++i) {
      const S cx = (double)VX[i] - ux, cy = (double)VY[i] - uy;
      fm[i] = pre * sexp(-(cx * cx + cy * cy) * i2T);
    }
    S sig[4], gx[4], gy[4], qq[4];
    shell_quantities(fm, sig, gx, gy, qq);
    S a = 0.0, b = 0.0, c = 0.0;
#pragma unroll
    for (int s = 0; s < 4; ++s) {
      a += A_SIG[3][s] * sig[s];
      b += A_GX[3][s] * gx[s];
      c += A_GY[3][s] * gy[s];
    }
    q[11] = a;
    q[14] = b;
    q[15] = c;
  } else {
    q[11] = 0.0;
    q[14] = 0.0;
    q[15] = 0.0;
  }
}

// Equilibrium distribution f^eq = M^-1 f^eq(rho, u, T).
template <int VER>
LBM_HD void equilibrium_f(double rho, double ux, double uy, double T, double* f) {
  double q[16];
  const double jx = rho * ux, jy = rho * uy;
  const double e = rho * (T + 0.5 * (ux * ux + uy * uy));
  equilibrium_moments<VER, double>(rho, jx, jy, e, q);
  f_from_moments(q, f);
}

// Runtime-version form for set-up code.
LBM_HD void equilibrium_f(int version, double rho, double ux, double uy, double T, double* f) {
  if (version == 2)
    equilibrium_f<2>(rho, ux, uy, T, f);
  else if (version == 3)
    equilibrium_f<3>(rho, ux, uy, T, f);
  else
    equilibrium_f<1>(rho, ux, uy, T, f);
}

}  // namespace lbm
