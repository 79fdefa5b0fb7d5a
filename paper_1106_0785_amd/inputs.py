"""Seeded synthetic workloads shaped like the paper's test problems.

This module builds problem parameters (grid, dx, dt, relaxation rates,
boundary kinds) and initial macroscopic fields (rho, u_x, u_y, T) only. It
holds none of the lattice Boltzmann arithmetic: turning fields into
distributions is done separately by the HIP library and by the CPU oracle.

Conventions (the paper's non-dimensional units with R = 1, Sec. IV):
  * an ideal gas with e = rho (T + u^2/2) and p = rho T, i.e. gamma = 2;
  * node (i, j) sits at x = (i + 1/2) dx, y = (j + 1/2) dy unless a wall
    occupies the first/last node (thermal Couette, walls on nodes);
  * fields are numpy float64 arrays of shape [ny, nx];
  * a parameter dict has keys nx, ny, dx, dy, dt, s (16 rates), eq_version,
    modified, bc (x_lo, x_hi, y_lo, y_hi) and wall (4 x (rho, ux, uy, T)).
Sharp initial jumps are smoothed with a tanh profile a few cells wide: the
central Lax-Wendroff stencil of the method is non-dissipative and a sharp jump
excites grid-scale oscillations.
"""

import math

import numpy as np

GAMMA = 2.0  # e = rho (T + u^2/2), p = rho T (R = 1): c_v = 1, c_p = 2


def rates(s5, s7, s_other, s6=None, s8=None):
    """16 relaxation rates; s1..s4 act on conserved moments and have no effect."""
    s = [float(s_other)] * 16
    s[4] = float(s5)
    s[5] = float(s5 if s6 is None else s6)
    s[6] = float(s7)
    s[7] = float(s7 if s8 is None else s8)
    return s


def params(nx, ny, dx, dy, dt, s, bc, wall=None, eq_version=1, modified=1):
    if wall is None:
        wall = [[1.0, 0.0, 0.0, 1.0] for _ in range(4)]
    return {
        "nx": int(nx),
        "ny": int(ny),
        "dx": float(dx),
        "dy": float(dy),
        "dt": float(dt),
        "s": [float(v) for v in s],
        "eq_version": int(eq_version),
        "modified": int(modified),
        "bc": list(bc),
        "wall": [[float(v) for v in w] for w in wall],
    }


def smooth_step(x, x0, width):
    """0 -> 1 across x0 with a tanh profile of the given width."""
    return 0.5 * (1.0 + np.tanh((x - x0) / width))


# --------------------------------------------------------------------------
# Thermal Couette flow (Sec. IV.A): walls on the first and last node of y,
# periodic in x. Bottom wall at rest at T0, top wall moving at u0 at T1.
# --------------------------------------------------------------------------
def couette(Pr, nx=4, ny=64, T0=1.0, T1=1.01, u0=0.1, s5=50.0, s_other=100.0, dt_over_dy=0.25,
            modified=1, eq_version=1):
    H = 1.0
    dy = H / (ny - 1)
    dt = dt_over_dy * dy
    s_oth = float(s_other) * max(1.0, Pr * s5 / s_other * 1.0) if Pr * s5 > s_other else float(s_other)
    s = rates(s5, Pr * s5, s_oth)
    wall = [[1.0, 0.0, 0.0, 1.0] for _ in range(4)]
    wall[2] = [1.0, 0.0, 0.0, T0]
    wall[3] = [1.0, u0, 0.0, T1]
    p = params(nx, ny, dy, dy, dt, s, ["periodic", "periodic", "neq_wall", "neq_wall"], wall,
               eq_version=eq_version, modified=modified)
    y = np.arange(ny) * dy
    T = np.broadcast_to((T0 + (T1 - T0) * y / H)[:, None], (ny, nx)).copy()
    fields = {"rho": np.ones((ny, nx)), "ux": np.zeros((ny, nx)), "uy": np.zeros((ny, nx)), "T": T}
    meta = {"H": H, "T0": T0, "T1": T1, "u0": u0, "Pr": Pr, "y": y}
    return p, fields, meta


def couette_x(Pr, nx=64, ny=4, T0=1.0, T1=1.01, u0=0.1, s5=50.0, s_other=100.0, dt_over_dx=0.25, modified=1):
    """The same flow rotated: walls on the first/last node of x, the right wall
    moving along y (the orientation of the paper's own Couette runs)."""
    p, f, meta = couette(Pr, nx=ny, ny=nx, T0=T0, T1=T1, u0=u0, s5=s5, s_other=s_other,
                         dt_over_dy=dt_over_dx, modified=modified)
    wall = [[1.0, 0.0, 0.0, T0], [1.0, 0.0, u0, T1], [1.0, 0.0, 0.0, 1.0], [1.0, 0.0, 0.0, 1.0]]
    q = params(nx, ny, p["dx"], p["dy"], p["dt"], p["s"], ["neq_wall", "neq_wall", "periodic", "periodic"], wall,
               modified=modified)
    fields = {k: np.ascontiguousarray(v.T) for k, v in f.items()}
    fields["ux"], fields["uy"] = fields["uy"].copy(), fields["ux"].copy()
    return q, fields, meta


# --------------------------------------------------------------------------
# One-dimensional Riemann problems (Sec. IV.B(a)) on [0, 1] along x.
# --------------------------------------------------------------------------
RIEMANN_STATES = {
    # (rho, u, p) left | right
    "sod": ((1.0, 0.0, 1.0), (0.125, 0.0, 0.1)),
    "lax": ((0.445, 0.698, 3.528), (0.5, 0.0, 0.571)),
}


def riemann(kind="sod", Pr=1.0, nx=2000, ny=4, dt=1e-5, s5=1e4, s_other=1e5, width_cells=3.0, x0=0.5,
            modified=1, states=None):
    L, R = states if states is not None else RIEMANN_STATES[kind]
    dx = 1.0 / nx
    s = rates(s5, Pr * s5, max(s_other, Pr * s5))
    p = params(nx, ny, dx, dx, dt, s, ["zero_gradient", "zero_gradient", "periodic", "periodic"],
               modified=modified)
    x = (np.arange(nx) + 0.5) * dx
    w = smooth_step(x, x0, width_cells * dx)
    rho = L[0] + (R[0] - L[0]) * w
    u = L[1] + (R[1] - L[1]) * w
    pr = L[2] + (R[2] - L[2]) * w
    T = pr / rho
    f = {
        "rho": np.tile(rho, (ny, 1)),
        "ux": np.tile(u, (ny, 1)),
        "uy": np.zeros((ny, nx)),
        "T": np.tile(T, (ny, 1)),
    }
    meta = {"x": x, "left": L, "right": R, "x0": x0}
    return p, f, meta


# --------------------------------------------------------------------------
# Normal-shock jump for the gamma = 2 gas (Rankine-Hugoniot).
# --------------------------------------------------------------------------
def post_shock(mach, rho1=1.0, p1=1.0, u1=0.0, gamma=GAMMA):
    """State behind a shock of Mach `mach` running into (rho1, u1, p1).

    Returns (rho2, du, p2, D) with D the shock speed relative to the
    pre-shock gas and du = |u2 - u1| the speed the gas acquires."""
    c1 = math.sqrt(gamma * p1 / rho1)
    D = mach * c1
    m2 = mach * mach
    rho2 = rho1 * (gamma + 1.0) * m2 / ((gamma - 1.0) * m2 + 2.0)
    p2 = p1 * (2.0 * gamma * m2 - (gamma - 1.0)) / (gamma + 1.0)
    du = D * (1.0 - rho1 / rho2)
    return rho2, du, p2, D


# --------------------------------------------------------------------------
# Richtmyer-Meshkov: planar shock in the light gas running into a perturbed
# light/heavy interface (Sec. IV.B(b) in spirit). Reflecting x walls,
# periodic y.
# --------------------------------------------------------------------------
def rm(seed=0, nx=1024, ny=256, dx=0.003, dt=1e-5, Pr=0.71, s5=1e4, s_other=1e5, mach=None,
       heavy=3.0, amp_frac=0.05, max_modes=4, width_cells=3.0, shock_gap_cells=20, modified=1,
       interface_offset=None, wall_ramp_cells=12.0):
    """Returns (params, fields, meta). meta['a'] is the per-row interface
    displacement field a(y) (in units of dy) that shapes the interface; the
    initial fields are smooth functions of it."""
    rng = np.random.default_rng(seed)
    if mach is None:
        mach = float(rng.uniform(1.2, 2.0))
    K = int(rng.integers(1, max_modes + 1))
    phases = rng.uniform(0.0, 2.0 * math.pi, size=K)
    Ly = ny * dx
    y = (np.arange(ny) + 0.5) * dx
    a = np.zeros(ny)
    for m in range(1, K + 1):
        lam = Ly / m
        a += amp_frac * lam * np.cos(2.0 * math.pi * y / lam + phases[m - 1])
    a_cells = a / dx
    if interface_offset is not None:
        a_cells = a_cells + np.asarray(interface_offset)
    s = rates(s5, Pr * s5, s_other)
    p = params(nx, ny, dx, dx, dt, s, ["specular", "specular", "periodic", "periodic"], modified=modified)
    meta = {"mach": mach, "K": K, "phases": phases, "a": a_cells, "heavy": heavy, "seed": seed,
            "width_cells": width_cells}
    x0_cells = 0.35 * nx
    meta["x0_cells"] = x0_cells
    meta["shock_cells"] = x0_cells - np.max(np.abs(a_cells)) - shock_gap_cells
    meta["wall_ramp_cells"] = wall_ramp_cells
    fields = rm_fields(nx, ny, a_cells, mach, heavy, x0_cells, meta["shock_cells"], width_cells, wall_ramp_cells)
    return p, fields, meta


def rm_fields(nx, ny, a_cells, mach, heavy, x0_cells, shock_cells, width_cells, wall_ramp_cells=12.0, xp=np):
    """Initial fields of the shock/interface problem as smooth functions of the
    per-row interface displacement a (cells). `xp` may be numpy or torch; with
    complex or differentiable a the fields carry the perturbation. The driver
    gas behind the shock is brought smoothly to rest at the reflecting left
    wall (a sharp velocity jump against the mirror ghost would excite
    grid-scale oscillations of the central stencil)."""
    rho2, du, p2, _ = post_shock(mach)
    if xp is np:
        ii = (np.arange(nx) + 0.5)[None, :]
        aa = np.asarray(a_cells)[:, None]
    else:
        ii = (xp.arange(nx, dtype=a_cells.dtype, device=a_cells.device) + 0.5)[None, :]
        aa = a_cells[:, None]
    w_int = 0.5 * (1.0 + xp.tanh((ii - x0_cells - aa) / width_cells))    # 0 light -> 1 heavy
    w_sh = 0.5 * (1.0 + xp.tanh((ii - shock_cells) / width_cells)) + 0 * aa  # 0 shocked -> 1 quiet
    ramp = xp.tanh(ii / wall_ramp_cells) + 0 * aa
    rho_light = rho2 + (1.0 - rho2) * w_sh
    u_light = du * (1.0 - w_sh) * ramp
    p_light = p2 + (1.0 - p2) * w_sh
    rho = rho_light + (heavy - rho_light) * w_int
    ux = u_light * (1.0 - w_int)
    pr = p_light + (1.0 - p_light) * w_int
    T = pr / rho
    uy = 0.0 * rho
    return {"rho": rho, "ux": ux, "uy": uy, "T": T}


# --------------------------------------------------------------------------
# Shock-bubble interaction (Sec. IV.B(b), Figs. 7-8): a Mach 1.22 shock
# running in -x through gas at rest (1, 0, 0, p = 1) into a light cylindrical
# bubble (rho 0.1358, p = 1). Right side: inflow fixed at the post-shock
# state; left side: extrapolation (zero gradient); y sides: reflecting.
# --------------------------------------------------------------------------
def shock_bubble(s5=1e4, s7=1e5, nx=600, ny=100, dx=0.003, dt=1e-5, s_other=1e5, mach=1.22, bubble_rho=0.1358,
                 radius=None, center=None, shock_x=None, width_cells=3.0, modified=1):
    """Returns (params, fields, meta). Positions are node indices (0-based):
    by default the bubble is centred at (0.75 nx - 1, (ny - 1)/2) with radius
    0.2 ny nodes and the post-shock gas fills the nodes x >= 5 nx / 6; every
    jump is smoothed with tanh over `width_cells` nodes."""
    rho2, du, p2, D = post_shock(mach)
    post = [rho2, -du, 0.0, p2 / rho2]
    cx, cy = (0.75 * nx - 1.0, 0.5 * (ny - 1)) if center is None else center
    r0 = 0.2 * ny if radius is None else radius
    xs = 5.0 * nx / 6.0 - 0.5 if shock_x is None else shock_x
    x = np.arange(nx, dtype=np.float64)[None, :]
    y = np.arange(ny, dtype=np.float64)[:, None]
    w_sh = smooth_step(x, xs, width_cells) + 0.0 * y  # 0 at rest, 1 post-shock
    r = np.sqrt((x - cx) ** 2 + (y - cy) ** 2)
    in_b = 1.0 - smooth_step(r, r0, width_cells)  # 1 inside the bubble
    rho_bg = 1.0 + (rho2 - 1.0) * w_sh
    pr = 1.0 + (p2 - 1.0) * w_sh
    rho = rho_bg + (bubble_rho - rho_bg) * in_b
    ux = -du * w_sh * (1.0 - in_b)
    T = pr / rho
    s = rates(s5, s7, s_other)
    wall = [[1.0, 0.0, 0.0, 1.0] for _ in range(4)]
    wall[1] = post
    p = params(nx, ny, dx, dx, dt, s, ["zero_gradient", "dirichlet_eq", "specular", "specular"], wall,
               modified=modified)
    fields = {"rho": rho, "ux": ux, "uy": np.zeros_like(rho), "T": T}
    meta = {"mach": mach, "D": D, "post": post, "bubble_rho": bubble_rho, "radius": r0, "center": (cx, cy),
            "shock_x": xs, "width_cells": width_cells}
    return p, fields, meta


# --------------------------------------------------------------------------
# Uneven batch of independent 1-D instances: Riemann problems along x
# (ny = 1) and thermal Couette columns along y (nx = 1).
# --------------------------------------------------------------------------
def batch(seed=0, n=512, riemann_n=(256, 4096), couette_h=(32, 256), pr_range=(0.3, 3.0)):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        if rng.random() < 0.5:
            N = int(rng.integers(riemann_n[0], riemann_n[1] + 1))
            rho = rng.uniform(0.1, 1.0, size=2)
            pr = rng.uniform(0.1, 3.0, size=2)
            u = rng.uniform(-1.0, 1.0, size=2)
            Pr = float(rng.uniform(*pr_range))
            dx = 1.0 / N
            Tmax = float(np.max(pr / rho))
            s5 = math.sqrt(Tmax) / (0.3 * dx)
            s_oth = 10.0 * s5 * max(1.0, Pr)
            s = rates(s5, Pr * s5, s_oth)
            dt = min(1.0 / max(s), dx / 4.0)
            p = params(N, 1, dx, dx, dt, s, ["zero_gradient", "zero_gradient", "periodic", "periodic"])
            x = (np.arange(N) + 0.5) * dx
            w = smooth_step(x, 0.5, 3.0 * dx)
            r = rho[0] + (rho[1] - rho[0]) * w
            uu = u[0] + (u[1] - u[0]) * w
            pp = pr[0] + (pr[1] - pr[0]) * w
            fields = {"rho": r[None, :], "ux": uu[None, :], "uy": np.zeros((1, N)), "T": (pp / r)[None, :]}
            out.append(("riemann", p, fields))
        else:
            H = int(rng.integers(couette_h[0], couette_h[1] + 1))
            Pr = float(rng.uniform(*pr_range))
            s5 = 50.0
            s_oth = 100.0 * max(1.0, Pr)
            s = rates(s5, Pr * s5, s_oth)
            dy = 1.0 / (H - 1)
            dt = min(dy / 4.0, 0.5 / max(s))
            wall = [[1.0, 0.0, 0.0, 1.0] for _ in range(4)]
            wall[2] = [1.0, 0.0, 0.0, 1.0]
            wall[3] = [1.0, 0.1, 0.0, 1.01]
            p = params(1, H, dy, dy, dt, s, ["periodic", "periodic", "neq_wall", "neq_wall"], wall)
            y = np.arange(H) * dy
            fields = {"rho": np.ones((H, 1)), "ux": np.zeros((H, 1)), "uy": np.zeros((H, 1)),
                      "T": (1.0 + 0.01 * y)[:, None].copy()}
            out.append(("couette", p, fields))
    return out


# --------------------------------------------------------------------------
# Uneven batch mixing the 1-D instances above with 2-D ones: shock/interface
# (Richtmyer-Meshkov) set-ups of random size, shock-bubble set-ups,
# Couette channels with two-dimensional extent (NEQ walls), periodic smooth
# states under the three equilibrium versions, and periodic Riemann lines
# longer than one line region.
# --------------------------------------------------------------------------
def mixed_batch(seed=0, n=24, rm_nx=(64, 320), rm_ny=(8, 72), riemann_n=(200, 900), couette_h=(32, 120)):
    rng = np.random.default_rng(seed)
    lines = batch(seed=seed + 1000, n=n, riemann_n=riemann_n, couette_h=couette_h)
    out = []
    for i in range(n):
        kind = i % 6
        if kind == 0:
            out.append(lines[i])
        elif kind == 1:
            nx = int(rng.integers(rm_nx[0], rm_nx[1] + 1))
            ny = int(rng.integers(rm_ny[0], rm_ny[1] + 1))
            p, f, _ = rm(seed=int(rng.integers(0, 1 << 30)), nx=nx, ny=ny)
            out.append(("rm", p, f))
        elif kind == 2:
            nx = int(rng.integers(6, 13)) * 10
            p, f, _ = shock_bubble(nx=nx, ny=nx // 6, dx=0.003 * 600 / nx)
            out.append(("shock_bubble", p, f))
        elif kind == 3:
            p, f, _ = couette(float(rng.uniform(0.3, 3.0)), nx=int(rng.integers(2, 80)),
                              ny=int(rng.integers(couette_h[0], couette_h[1] + 1)),
                              eq_version=int(rng.integers(1, 4)))
            out.append(("couette2d", p, f))
        elif kind == 4:
            p, f = smooth_periodic(seed=int(rng.integers(0, 1 << 30)), nx=int(rng.integers(16, 200)),
                                   ny=int(rng.integers(3, 70)), eq_version=int(rng.integers(1, 4)))
            out.append(("periodic2d", p, f))
        else:
            N = int(rng.integers(max(129, riemann_n[0]), riemann_n[1] + 1))
            p, f = smooth_periodic(seed=int(rng.integers(0, 1 << 30)), nx=N, ny=1, dx=1.0 / N, dt=1e-4)
            out.append(("periodic_line", p, f))
    return out


# --------------------------------------------------------------------------
# Uneven batch of independent 2-D shock/interface problems (random size,
# Mach number, interface modes and Prandtl number per instance).
# --------------------------------------------------------------------------
def rm_batch(seed=0, n=96, nx=(128, 512), ny=(32, 128), pr_range=(0.3, 3.0)):
    rng = np.random.default_rng(seed)
    out = []
    for _ in range(n):
        p, f, _ = rm(seed=int(rng.integers(0, 1 << 30)), nx=int(rng.integers(nx[0], nx[1] + 1)),
                     ny=int(rng.integers(ny[0], ny[1] + 1)), Pr=float(rng.uniform(*pr_range)))
        out.append(("rm", p, f))
    return out


# --------------------------------------------------------------------------
# Von Neumann stability cases of Fig. 2 (Sec. III): base state (rho, u_x,
# u_y, T), dx = dy = 1e-3, dt = 1e-5, relaxation rates 1e5 except those
# listed (1-based index) for the paper's model ("three versions").
# --------------------------------------------------------------------------
FIG2_CASES = {
    "a": ((2.0, 2.0, 0.0, 2.0), {}),
    "b": ((2.0, 6.0, 0.0, 2.0), {9: 1e3}),
    "c": ((2.0, 10.0, 0.0, 2.0), {9: 1.2e4, 13: 1e2, 14: 5e4, 15: 1.5e3}),
    "d": ((2.0, 12.0, 0.0, 2.0), {9: 1e4, 13: 1e2, 14: 6e4, 15: 1.5e3}),
}


def fig2_stability_sets(versions=(1,), modified=1):
    """(params list, base-state list) for cases (a)-(d), each under every
    equilibrium version given."""
    params, states = [], []
    for case, (st, over) in FIG2_CASES.items():
        s = [1e5] * 16
        for k, v in over.items():
            s[k - 1] = v
        for ver in versions:
            params.append(params_of_stability(s, ver, modified))
            states.append(st)
    return params, states


# The high-Mach shock tube of Sec. IV.B(a), Fig. 6: uniform states (rho, u_x,
# u_y, T) on either side (Mach 10.1 and 6.3 with Ma = u / sqrt(2T)),
# dx = dy = 0.003, dt = 1e-5, s5 = s6 = 1.5e4, every other rate 1e5.
FIG6_STATES = {"left": (5.0, 45.0, 0.0, 10.0), "right": (6.0, -20.0, 0.0, 5.0)}


def fig6_stability_sets(versions=(1, 2), modified=(0, 1), dt=1e-5, at_rest=False):
    """(params list, base-state list, labels) for the two states of the
    Fig. 6 shock tube under every equilibrium version and modification mode
    given; at_rest: the same states with zero velocity."""
    s = [1e5] * 16
    s[4] = s[5] = 1.5e4
    params, states, labels = [], [], []
    for side, st in FIG6_STATES.items():
        if at_rest:
            st = (st[0], 0.0, 0.0, st[3])
        for ver in versions:
            for mod in modified:
                params.append(params_of_stability(s, ver, mod, dx=0.003, dy=0.003, dt=dt))
                states.append(st)
                labels.append("%s v%d mod%d" % (side, ver, mod))
    return params, states, labels


def riemann_stability_sets(kind="lax", Prs=(0.5, 1.0, 2.0)):
    """(params list, base-state list, labels): the two uniform states of a
    shock-tube configuration (riemann() above) at each Prandtl number."""
    L, R = RIEMANN_STATES[kind]
    params, states, labels = [], [], []
    for Pr in Prs:
        p, _, _ = riemann(kind, Pr=Pr, nx=2000, ny=1)
        q = params_of_stability(p["s"], 1, p["modified"], dx=p["dx"], dy=p["dy"], dt=p["dt"])
        for side, st in (("left", L), ("right", R)):
            params.append(q)
            states.append((st[0], st[1], 0.0, st[2] / st[0]))
            labels.append("%s Pr %g %s" % (kind, Pr, side))
    return params, states, labels


def params_of_stability(s, version=1, modified=1, dx=1e-3, dy=1e-3, dt=1e-5):
    return params(1, 1, dx, dy, dt, s, ["periodic"] * 4, eq_version=version, modified=modified)


def wavenumber_grid(n, lo=0.0, hi=math.pi):
    """[n*n, 2] grid of (theta_x, theta_y) over [lo, hi]^2, theta_x fastest."""
    g = np.linspace(lo, hi, n)
    tx, ty = np.meshgrid(g, g)
    return np.stack([tx.ravel(), ty.ravel()], 1)


# --------------------------------------------------------------------------
# Small smooth periodic states for invariants and wave tests.
# --------------------------------------------------------------------------
def smooth_periodic(seed=0, nx=32, ny=32, dx=0.01, dt=1e-4, s5=1e3, s7=1e3, s_other=2e3, amp=0.05,
                    modes=3, modified=1, eq_version=1):
    rng = np.random.default_rng(seed)
    x = (np.arange(nx) + 0.5) / nx
    y = (np.arange(ny) + 0.5) / ny
    X, Y = np.meshgrid(x, y)

    def field(base, a):
        g = np.full((ny, nx), base, dtype=np.float64)
        for _ in range(modes):
            kx = int(rng.integers(0, 3)) if nx > 1 else 0
            ky = int(rng.integers(0, 3)) if ny > 1 else 0
            ph = rng.uniform(0, 2 * math.pi)
            g += a * rng.uniform(0.3, 1.0) * np.cos(2 * math.pi * (kx * X + ky * Y) + ph)
        return g

    fields = {"rho": field(1.0, amp), "ux": field(0.1, amp), "uy": field(-0.05, amp), "T": field(1.0, amp)}
    p = params(nx, ny, dx, dx, dt, rates(s5, s7, s_other), ["periodic"] * 4, modified=modified,
               eq_version=eq_version)
    return p, fields
