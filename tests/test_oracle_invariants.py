"""Invariant pins of the oracle's time step (Sec. II-III).

  * the collision conserves rho, j, e and the Lax-Wendroff differences
    telescope, so totals are constant on a periodic grid;
  * a uniform equilibrium state is a fixed point;
  * a y-uniform state stays y-uniform, and ny = 1 equals ny = 4;
  * mirror (x -> -x) and quarter-turn rotation symmetry of the model: the
    velocity set, M, the equilibria and the modification are isotropic, so a
    mirrored or rotated initial state evolves into the mirrored or rotated
    solution. A dropped term or a transposed index in any stage breaks this.
"""

import numpy as np

import oracle
from paper_1106_0785_amd import inputs


def _totals(p, f):
    m = oracle.moments(p, f)
    rho, ux, uy, T = m["rho"], m["ux"], m["uy"], m["T"]
    return np.array([rho.sum(), (rho * ux).sum(), (rho * uy).sum(), (rho * (T + 0.5 * (ux * ux + uy * uy))).sum()])


def test_conservation_periodic():
    for modified in (0, 1):
        p, fl = inputs.smooth_periodic(seed=11, nx=32, ny=24, amp=0.08, modified=modified)
        f0 = oracle.init(p, **fl)
        f1 = oracle.run(p, f0, 300)
        assert np.abs(f1 - f0).max() > 1e-3  # the state really evolved
        t0, t1 = _totals(p, f0), _totals(p, f1)
        np.testing.assert_allclose(t1, t0, rtol=1e-13, atol=1e-12)


def test_uniform_state_is_fixed_point():
    for ver in (1, 2, 3):
        p, fl = inputs.smooth_periodic(seed=1, nx=8, ny=6, amp=0.0, eq_version=ver)
        f0 = oracle.init(p, **fl)
        f1 = oracle.run(p, f0, 200)
        assert np.abs(f1 - f0).max() < 1e-14


def test_one_dimensional_reduction():
    p4, fl = inputs.smooth_periodic(seed=5, nx=24, ny=1, amp=0.08)
    f1d = oracle.init(p4, **fl)
    r1 = oracle.run(p4, f1d, 150)
    p4["ny"] = 4
    f2d = np.repeat(f1d, 4, axis=1)
    r2 = oracle.run(p4, f2d, 150)
    for j in range(4):
        assert np.array_equal(r2[:, j], r1[:, 0])


def _mirror_x(f, v):
    perm = [int(np.where((v[:, 0] == -v[i, 0]) & (v[:, 1] == v[i, 1]))[0][0]) for i in range(16)]
    return f[perm][:, :, ::-1].copy()


def test_mirror_symmetry_with_walls():
    v, _, _ = oracle.matrices()
    p, fl = inputs.smooth_periodic(seed=7, nx=20, ny=12, amp=0.08)
    for bc in (["specular", "specular", "periodic", "periodic"], ["zero_gradient", "zero_gradient", "periodic", "periodic"]):
        p["bc"] = bc
        f0 = oracle.init(p, **fl)
        a = oracle.run(p, f0, 120)
        b = oracle.run(p, _mirror_x(f0, v), 120)
        np.testing.assert_allclose(_mirror_x(a, v), b, rtol=0, atol=1e-13)


def _rotate(f, v):
    """Quarter turn: position (x, y) -> (-y, x), velocity (vx, vy) -> (-vy, vx)."""
    perm = [int(np.where((v[:, 0] == -v[i, 1]) & (v[:, 1] == v[i, 0]))[0][0]) for i in range(16)]
    g = np.empty((16, f.shape[2], f.shape[1]))
    for i in range(16):
        # new[y'=x][x'=ny-1-y] = old[y][x]
        g[perm[i]] = f[i].T[:, ::-1]
    return g


def test_quarter_turn_symmetry():
    v, _, _ = oracle.matrices()
    p, fl = inputs.smooth_periodic(seed=9, nx=18, ny=14, amp=0.08)
    # isotropy needs s7 = s8, s9 = s10, s15 = s16; s5 and s6 may differ
    p["s"][4], p["s"][5], p["s"][6], p["s"][7] = 800.0, 1300.0, 1100.0, 1100.0
    for modified in (0, 1):
        p["modified"] = modified
        f0 = oracle.init(p, **fl)
        a = oracle.run(p, f0, 150)
        q = dict(p, nx=p["ny"], ny=p["nx"])
        b = oracle.run(q, _rotate(f0, v), 150)
        np.testing.assert_allclose(_rotate(a, v), b, rtol=0, atol=1e-13)


def test_printed_q8_sign_breaks_isotropy():
    """The Q_8 normal-stress term exactly as printed (modified = 2) is not the
    quarter-turn image of the Q_7 term, so the rotated run differs."""
    v, _, _ = oracle.matrices()
    p, fl = inputs.smooth_periodic(seed=9, nx=18, ny=14, amp=0.08)
    p["s"][4], p["s"][5], p["s"][6], p["s"][7] = 800.0, 1300.0, 1100.0, 1100.0
    p["modified"] = 2
    f0 = oracle.init(p, **fl)
    a = oracle.run(p, f0, 150)
    q = dict(p, nx=p["ny"], ny=p["nx"])
    b = oracle.run(q, _rotate(f0, v), 150)
    assert np.abs(_rotate(a, v) - b).max() > 1e-9


def test_equal_rates_reduce_to_single_relaxation():
    """Sec. II, the remark after the three equilibrium versions: with every
    rate equal (S = s I) the model is a single-relaxation (BGK) model. Then
    M^-1 S M = s I and the four modification terms vanish, so one step is
    the pure convection of f minus dt s (f - f^eq(f)), with f^eq = M^-1 f^eq^
    of f's own density, velocity and temperature. The convection-only step is
    the oracle with every rate zero and the unmodified model; f^eq comes from
    the oracle's initialiser. A wrong column of M^-1, a relaxed conserved
    moment, a sign or a misplaced dt fails it."""
    for version in (1, 2, 3):
        p, fl = inputs.smooth_periodic(seed=31 + version, nx=11, ny=9, amp=0.08, eq_version=version)
        f0 = oracle.run(p, oracle.init(p, **fl), 3)  # away from equilibrium
        s = 3.7e3
        conv = dict(p, s=[0.0] * 16, modified=0)
        c = oracle.run(conv, f0, 1)
        m = oracle.moments(p, f0)
        feq = oracle.init(p, m["rho"], m["ux"], m["uy"], m["T"])
        expect = c - p["dt"] * s * (f0 - feq)
        assert np.max(np.abs(f0 - feq)) > 1e-4 * np.max(np.abs(f0))  # the relaxation term is not trivial
        for modified in (0, 1, 2):
            srt = dict(p, s=[s] * 16, modified=modified)
            got = oracle.run(srt, f0, 1)
            err = np.max(np.abs(got - expect)) / np.max(np.abs(f0))
            assert err < 1e-13, (version, modified, err)


def test_neq_wall_nodes_carry_wall_velocity_and_temperature():
    """Sec. IV.A, non-equilibrium extrapolation: a wall node is the
    equilibrium at (fluid neighbour's density, wall velocity, wall
    temperature) plus the neighbour's non-equilibrium part f - f^eq(f). That
    part has no density, momentum or energy, so after every step each wall
    node's density equals its neighbour's and its velocity and temperature
    are exactly the wall's (to rounding), for every equilibrium version and
    modification mode, on walls normal to either axis."""
    for version in (1, 2, 3):
        for modified in (0, 1, 2):
            for axis in ("y", "x"):
                if axis == "y":
                    p, fl = inputs.smooth_periodic(seed=40 + version, nx=9, ny=12, amp=0.06, eq_version=version,
                                                   modified=modified)
                    p["bc"] = ["periodic", "periodic", "neq_wall", "neq_wall"]
                else:
                    p, fl = inputs.smooth_periodic(seed=50 + version, nx=12, ny=9, amp=0.06, eq_version=version,
                                                   modified=modified)
                    p["bc"] = ["neq_wall", "neq_wall", "periodic", "periodic"]
                lo, hi = (2, 3) if axis == "y" else (0, 1)
                p["wall"][lo] = [1.0, 0.03, -0.02, 0.98]
                p["wall"][hi] = [1.0, -0.05, 0.04, 1.03]
                f = oracle.run(p, oracle.init(p, **fl), 7)
                m = oracle.moments(p, f)
                for side, idx, nb in ((lo, 0, 1), (hi, -1, -2)):
                    take = (lambda a, i: a[i, :]) if axis == "y" else (lambda a, i: a[:, i])
                    _, ux, uy, T = p["wall"][side]
                    assert np.allclose(take(m["ux"], idx), ux, rtol=0, atol=1e-13)
                    assert np.allclose(take(m["uy"], idx), uy, rtol=0, atol=1e-13)
                    assert np.allclose(take(m["T"], idx), T, rtol=1e-13, atol=0)
                    assert np.allclose(take(m["rho"], idx), take(m["rho"], nb), rtol=1e-13, atol=0)


def test_uniform_states_are_fixed_points_of_every_boundary_kind():
    """A uniform equilibrium state is left unchanged (to rounding) by a step
    with each boundary kind under the conditions where that kind is
    compatible with it: zero-gradient for any velocity; specular walls when
    the velocity normal to them is zero; fixed-state ghosts equal to the
    state; NEQ walls moving with the fluid at its temperature (Sec. IV). A
    ghost built from the wrong node, a mirror of the wrong planes or a wall
    state taken from the wrong side moves the state."""
    rho, ux, uy, T = 1.1, 0.07, -0.04, 0.93
    cases = [
        (["zero_gradient"] * 4, (ux, uy)),
        (["specular", "specular", "periodic", "periodic"], (0.0, uy)),
        (["periodic", "periodic", "specular", "specular"], (ux, 0.0)),
        (["dirichlet_eq", "dirichlet_eq", "zero_gradient", "zero_gradient"], (ux, uy)),
        (["periodic", "periodic", "neq_wall", "neq_wall"], (ux, uy)),
        (["neq_wall", "neq_wall", "specular", "specular"], (ux, 0.0)),
    ]
    for version in (1, 2, 3):
        for bc, (u, v) in cases:
            p, _ = inputs.smooth_periodic(seed=1, nx=7, ny=6, eq_version=version)
            p["bc"] = bc
            for side in range(4):
                p["wall"][side] = [rho, u, v, T]
            fl = {k: np.full((6, 7), val) for k, val in (("rho", rho), ("ux", u), ("uy", v), ("T", T))}
            f0 = oracle.init(p, **fl)
            f1 = oracle.run(p, f0, 3)
            err = float(np.max(np.abs(f1 - f0)) / np.max(np.abs(f0)))
            assert err < 1e-14, (version, bc, err)
    # and a specular wall with a normal velocity is not a fixed point
    p, _ = inputs.smooth_periodic(seed=1, nx=7, ny=6)
    p["bc"] = ["specular", "specular", "periodic", "periodic"]
    fl = {k: np.full((6, 7), val) for k, val in (("rho", rho), ("ux", ux), ("uy", uy), ("T", T))}
    f0 = oracle.init(p, **fl)
    assert np.max(np.abs(oracle.run(p, f0, 3) - f0)) > 1e-6
