"""Von Neumann stability of the step (Sec. III): the amplification matrix
G(theta) and its largest eigenvalue modulus |omega|_max.

TEST INFRASTRUCTURE ONLY: used by the test suite, the smoke check and the
benchmark's CPU baseline; the HIP library never calls it.

A Fourier mode f_i(x) = f_i e^{i (theta_x x / dx + theta_y y / dy)} around a
uniform state (rho, u_x, u_y, T) is mapped by one linearised step to G(theta)
times itself. G is the sum of
  * the convection symbol of the per-axis Lax-Wendroff update on the diagonal,
    with c = v_i,alpha dt / dx_alpha:
      1 - (c/2)(e^{i t} - e^{-i t}) + (c^2/2)(e^{i t} - 2 + e^{-i t}) per axis;
  * the collision term -dt M^-1 S (M - d f^eq / d f), the derivative of the
    equilibrium moments taken through rho, u, T (Sec. III, chain rule);
  * for the modified model, the derivative of the extra Q_7 and Q_8 terms
    (Sec. II), added to Q before -dt M^-1: at a uniform state only the
    velocity gradients vary, and the central difference of a Fourier mode has
    the symbol (e^{i t} - e^{-i t}) / (2 dx) (reading of the paper's silent
    gradient discretisation: the step's own central differences).

The derivative d f^eq / d f follows the paper's chain rule through (rho,
u, T): the oracle's equilibrium moments differentiated by complex step (no
subtraction, exact to rounding) at the state itself, times the derivatives
of (rho, u, T) with respect to f from their definitions. |omega|_max is the
largest modulus among numpy's eigenvalues of G (taken in the moment basis,
see radius()).
"""

import numpy as np

from . import oracle

H = 1e-30  # complex step


def derivatives(p, state):
    """(d f^eq_k / d f_j [16, 16], d u_x / d f_j [16], d u_y / d f_j [16]) at
    the uniform state, by the chain rule of Sec. III through rho, u and T:
    the derivatives of the equilibrium moments with respect to (rho, u_x,
    u_y, T) by complex step at the state itself, and those of (rho, u, T)
    with respect to f from their definitions rho = sum f, rho u = sum f v,
    rho (T + u^2/2) = sum f v^2/2 (moment rows 1..4 of M)."""
    _, M, _ = oracle.matrices()
    rho, ux, uy, T = (float(v) for v in state)
    dq = np.zeros((16, 4))
    for c in range(4):
        v = np.array([rho, ux, uy, T], dtype=np.complex128)
        v[c] += 1j * H
        dq[:, c] = oracle.feq_moments_complex(p["eq_version"], v).imag / H
    drho = M[0]
    dux = (M[1] - ux * M[0]) / rho
    duy = (M[2] - uy * M[0]) / rho
    dT = (M[3] - (T + 0.5 * (ux * ux + uy * uy)) * M[0]) / rho - ux * dux - uy * duy
    jeq = np.outer(dq[:, 0], drho) + np.outer(dq[:, 1], dux) + np.outer(dq[:, 2], duy) + np.outer(dq[:, 3], dT)
    return jeq, dux, duy


def amplification_matrix(p, state, theta_x, theta_y, derivs=None):
    """G(theta) [16, 16] complex for parameters p (dx, dy, dt, s, eq_version,
    modified) and the uniform state (rho, u_x, u_y, T)."""
    V, M, Mi = oracle.matrices()
    jeq, dux, duy = derivs if derivs is not None else derivatives(p, state)
    dt, dx, dy = p["dt"], p["dx"], p["dy"]
    s = np.asarray(p["s"], dtype=np.float64)
    ex, ey = np.exp(1j * theta_x), np.exp(1j * theta_y)
    G = np.zeros((16, 16), dtype=np.complex128)
    for i in range(16):
        g = 1.0 + 0j
        for c, e in ((V[i, 0] * dt / dx, ex), (V[i, 1] * dt / dy, ey)):
            g += -0.5 * c * (e - 1.0 / e) + 0.5 * c * c * (e - 2.0 + 1.0 / e)
        G[i, i] = g
    G += -dt * (Mi @ (np.diag(s) @ (M - jeq)))
    mod = int(p.get("modified", 1))
    if mod:
        rho, ux, uy, T = (float(v) for v in state)
        rT = rho * T
        gx = (ex - 1.0 / ex) / (2.0 * dx)  # central difference along x of a Fourier mode
        gy = (ey - 1.0 / ey) / (2.0 * dy)
        dA = gx * dux - gy * duy  # d(d_x u_x - d_y u_y) / d f_j
        dB = gx * duy + gy * dux  # d(d_x u_y + d_y u_x) / d f_j
        sgn8 = 1.0 if mod == 2 else -1.0
        m7 = (s[6] / s[4] - 1.0) * rT * ux * dA + (s[6] / s[5] - 1.0) * rT * uy * dB
        m8 = (s[7] / s[5] - 1.0) * rT * ux * dB + sgn8 * (s[7] / s[4] - 1.0) * rT * uy * dA
        G += -dt * (np.outer(Mi[:, 6], m7) + np.outer(Mi[:, 7], m8))
    return G


def radius(G):
    """|omega|_max: the largest eigenvalue modulus of G (velocity basis).
    The eigenvalues are taken of the similar matrix M G M^-1 (the oracle's
    M and M^-1): the same spectrum, but far less non-normal for these
    operators (the collision acts moment by moment), so numpy's
    double-precision eigenvalues are several times closer to exact ones
    (checked against 40-digit eigenvalues)."""
    _, M, Mi = oracle.matrices()
    return float(np.max(np.abs(np.linalg.eigvals(M @ G @ Mi))))


def omega_max(p, state, thetas):
    """|omega|_max at each (theta_x, theta_y) of thetas [n, 2]."""
    d = derivatives(p, state)
    return np.array([radius(amplification_matrix(p, state, tx, ty, d)) for tx, ty in np.asarray(thetas)])
