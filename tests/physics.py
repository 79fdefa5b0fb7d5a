"""Closed-form and exact reference solutions used to pin the oracle.

Written from textbook gas dynamics, independently of the oracle and of the
HIP path:
  * exact Riemann solver for an ideal gas (two-rarefaction / two-shock
    pressure function, Newton iteration, self-similar sampling);
  * thermal Couette temperature profile (Sec. IV.A);
  * Rankine-Hugoniot jump (for the shock/bubble state of Sec. IV.B(b)).
The paper's gas has e = rho (T + u^2/2) and p = rho R T with R = 1, i.e.
gamma = 2.
"""

import math

import numpy as np

GAMMA = 2.0


def _pressure_function(p, rho, pk, ck, g):
    if p > pk:  # shock
        A = 2.0 / ((g + 1.0) * rho)
        B = (g - 1.0) / (g + 1.0) * pk
        f = (p - pk) * math.sqrt(A / (p + B))
        df = math.sqrt(A / (B + p)) * (1.0 - 0.5 * (p - pk) / (B + p))
    else:  # rarefaction
        f = 2.0 * ck / (g - 1.0) * ((p / pk) ** ((g - 1.0) / (2.0 * g)) - 1.0)
        df = 1.0 / (rho * ck) * (p / pk) ** (-(g + 1.0) / (2.0 * g))
    return f, df


def riemann_star(left, right, g=GAMMA):
    """(p*, u*) for states (rho, u, p)."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    p = max(1e-10, 0.5 * (pl + pr) - 0.125 * (ur - ul) * (rl + rr) * (cl + cr))
    for _ in range(200):
        fl, dfl = _pressure_function(p, rl, pl, cl, g)
        fr, dfr = _pressure_function(p, rr, pr, cr, g)
        dp = (fl + fr + ur - ul) / (dfl + dfr)
        pn = max(1e-12, p - dp)
        if abs(pn - p) < 1e-14 * (pn + p):
            p = pn
            break
        p = pn
    fl, _ = _pressure_function(p, rl, pl, cl, g)
    fr, _ = _pressure_function(p, rr, pr, cr, g)
    u = 0.5 * (ul + ur) + 0.5 * (fr - fl)
    return p, u


def riemann_sample(left, right, xi, g=GAMMA):
    """Exact self-similar solution at xi = (x - x0)/t. Returns rho, u, p arrays."""
    rl, ul, pl = left
    rr, ur, pr = right
    cl = math.sqrt(g * pl / rl)
    cr = math.sqrt(g * pr / rr)
    ps, us = riemann_star(left, right, g)
    gm = (g - 1.0) / (g + 1.0)
    xi = np.asarray(xi, dtype=np.float64)
    rho = np.empty_like(xi)
    u = np.empty_like(xi)
    p = np.empty_like(xi)
    for n, s in enumerate(xi):
        if s <= us:  # left of contact
            if ps > pl:  # left shock
                sl = ul - cl * math.sqrt((g + 1.0) / (2.0 * g) * ps / pl + (g - 1.0) / (2.0 * g))
                if s <= sl:
                    rho[n], u[n], p[n] = rl, ul, pl
                else:
                    rho[n] = rl * (ps / pl + gm) / (gm * ps / pl + 1.0)
                    u[n], p[n] = us, ps
            else:  # left rarefaction
                shl = ul - cl
                cs = cl * (ps / pl) ** ((g - 1.0) / (2.0 * g))
                stl = us - cs
                if s <= shl:
                    rho[n], u[n], p[n] = rl, ul, pl
                elif s >= stl:
                    rho[n] = rl * (ps / pl) ** (1.0 / g)
                    u[n], p[n] = us, ps
                else:
                    c = 2.0 / (g + 1.0) * (cl + (g - 1.0) / 2.0 * (ul - s))
                    rho[n] = rl * (c / cl) ** (2.0 / (g - 1.0))
                    u[n] = 2.0 / (g + 1.0) * (cl + (g - 1.0) / 2.0 * ul + s)
                    p[n] = pl * (c / cl) ** (2.0 * g / (g - 1.0))
        else:  # right of contact
            if ps > pr:  # right shock
                sr = ur + cr * math.sqrt((g + 1.0) / (2.0 * g) * ps / pr + (g - 1.0) / (2.0 * g))
                if s >= sr:
                    rho[n], u[n], p[n] = rr, ur, pr
                else:
                    rho[n] = rr * (ps / pr + gm) / (gm * ps / pr + 1.0)
                    u[n], p[n] = us, ps
            else:  # right rarefaction
                shr = ur + cr
                cs = cr * (ps / pr) ** ((g - 1.0) / (2.0 * g))
                str_ = us + cs
                if s >= shr:
                    rho[n], u[n], p[n] = rr, ur, pr
                elif s <= str_:
                    rho[n] = rr * (ps / pr) ** (1.0 / g)
                    u[n], p[n] = us, ps
                else:
                    c = 2.0 / (g + 1.0) * (cr - (g - 1.0) / 2.0 * (ur - s))
                    rho[n] = rr * (c / cr) ** (2.0 / (g - 1.0))
                    u[n] = 2.0 / (g + 1.0) * (-cr + (g - 1.0) / 2.0 * ur + s)
                    p[n] = pr * (c / cr) ** (2.0 * g / (g - 1.0))
    return rho, u, p


def couette_profile(y, H, T0, T1, U, Pr, cp=2.0):
    """Steady thermal Couette temperature (Sec. IV.A): heating/conduction ratio
    mu/(2 lambda) = Pr/(2 c_p) with c_p = 2."""
    eta = np.asarray(y) / H
    return T0 + (T1 - T0) * eta + Pr * U * U / (2.0 * cp) * eta * (1.0 - eta)


def rankine_hugoniot(mach, rho1, p1, g=GAMMA):
    """Post-shock (rho2, |u2|, p2) and shock speed D for a shock of Mach
    `mach` running into gas at rest (standard normal-shock relations)."""
    c1 = math.sqrt(g * p1 / rho1)
    D = mach * c1
    # mass and momentum flux continuity in the shock frame, solved by the
    # textbook density ratio
    m2 = mach * mach
    r = (g + 1.0) * m2 / ((g - 1.0) * m2 + 2.0)
    rho2 = rho1 * r
    u2 = D * (1.0 - 1.0 / r)
    p2 = p1 + rho1 * D * u2
    return rho2, u2, p2, D
