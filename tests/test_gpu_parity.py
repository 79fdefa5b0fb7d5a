"""Parity of the HIP path (through the C ABI) with the CPU oracle on the
paper-shaped workloads, plus edge cases. Tolerance: 1e-11 per moment field
(definition in gpu_util)."""

import numpy as np
import pytest

import oracle
from gpu_util import assert_parity, gpu_run, log, oracle_run
from paper_1106_0785_amd import inputs

pytestmark = pytest.mark.gpu


@pytest.mark.parametrize("Pr", [0.5, 1.0, 2.0])
def test_couette_full_run(Pr):
    """Thermal Couette 4 x 64, walls on the first/last row, 20000 steps."""
    p, fl, _ = inputs.couette(Pr)
    log("couette Pr=%g 4x64 20000 steps" % Pr)
    g, gf = gpu_run(p, fl, 20000)
    o, _ = oracle_run(p, fl, 20000)
    assert_parity(g, o, what="couette Pr=%g" % Pr)


@pytest.mark.parametrize("kind,steps,Pr", [("sod", 20000, 0.5), ("sod", 20000, 1.0), ("sod", 20000, 2.0),
                                           ("lax", 14000, 1.0), ("lax", 14000, 2.0)])
def test_riemann_full_run(kind, steps, Pr):
    """2000 x 4 Riemann problems for their full run at each configured
    Prandtl number (the Lax tube at Pr = 0.5 is unstable: next test); the
    oracle runs the y-uniform problem on one row (its rows are bitwise equal,
    pinned on CPU)."""
    p, fl, _ = inputs.riemann(kind, Pr=Pr, nx=2000, ny=4)
    log("riemann %s Pr=%g 2000x4 %d steps" % (kind, Pr, steps))
    g, _ = gpu_run(p, fl, steps)
    p1, fl1, _ = inputs.riemann(kind, Pr=Pr, nx=2000, ny=1)
    o, _ = oracle_run(p1, fl1, steps)
    for j in range(4):
        gj = {k: v[j:j + 1] for k, v in g.items()}
        assert_parity(gj, o, what="riemann %s Pr=%g row %d" % (kind, Pr, j))


def test_lax_prandtl_half_loses_positivity_on_both_sides():
    """The Lax tube at Pr = 0.5 (s7 = s8 = s5 / 2) is not stable with the
    central scheme: the oracle's temperature turns negative between steps
    2700 and 2720 (a grid-scale oscillation behind the contact grows from
    step ~2000). Both sides agree to 1e-11 at step 1500, and both lose
    positivity by step 3000: the GPU path reports it through the health
    flag."""
    from paper_1106_0785_amd import lbm

    p, fl, _ = inputs.riemann("lax", Pr=0.5, nx=2000, ny=4)
    p1, fl1, _ = inputs.riemann("lax", Pr=0.5, nx=2000, ny=1)
    g, _ = gpu_run(p, fl, 1500)
    o, _ = oracle_run(p1, fl1, 1500)
    for j in range(4):
        assert_parity({k: v[j:j + 1] for k, v in g.items()}, o, what="lax Pr=0.5 1500 steps row %d" % j)
    o3, _ = oracle_run(p1, fl1, 3000)
    assert not (np.all(np.isfinite(o3["T"])) and o3["T"].min() > 0 and o3["rho"].min() > 0)
    sim = lbm.Simulation(p)
    sim.init(**fl)
    sim.step(3000)
    with pytest.raises(lbm.LbmError) as err:
        sim.check()
    assert err.value.status == -5
    sim.close()


def test_rm_small_ragged():
    p, fl, _ = inputs.rm(seed=4, nx=200, ny=42)
    log("rm 200x42 300 steps")
    g, _ = gpu_run(p, fl, 300)
    o, _ = oracle_run(p, fl, 300)
    assert_parity(g, o, what="rm 200x42")


def test_rm_full_size_short_run():
    p, fl, _ = inputs.rm(seed=0, nx=1024, ny=256)
    log("rm 1024x256 60 steps")
    g, _ = gpu_run(p, fl, 60)
    o, _ = oracle_run(p, fl, 60)
    assert_parity(g, o, what="rm 1024x256")


def _kernel_diff(a, b):
    return float(np.max(np.abs(a - b) / np.abs(b).max(axis=(1, 2), keepdims=True)))


def test_fused_matches_plain_kernel():
    """Same node arithmetic, different data movement: the results agree to
    a few ulps (the compiler may contract multiply-adds differently)."""
    p, fl, _ = inputs.rm(seed=2, nx=300, ny=100)
    _, f0 = gpu_run(p, fl, 50, variant=0)
    _, f1 = gpu_run(p, fl, 50, variant=1)
    d = _kernel_diff(f0, f1)
    log("fused vs plain 300x100 50 steps: max diff %.2e (bitwise equal: %s)" % (d, np.array_equal(f0, f1)))
    assert d <= 1e-13


@pytest.mark.parametrize("rows,waves", [(4, 4), (8, 4), (16, 4), (64, 4), (2, 2), (6, 2), (16, 2), (64, 2)])
def test_tile_shape_does_not_change_result(rows, waves):
    """The tile shape changes only which workgroup computes a node: bitwise
    equal results."""
    p, fl, _ = inputs.rm(seed=3, nx=190, ny=77)
    _, f = gpu_run(p, fl, 30, rows=rows, waves=waves)
    _, ref = gpu_run(p, fl, 30, rows=4, waves=4)
    log("tile %d rows x %d waves 190x77: bitwise equal to 4 x 4: %s" % (rows, waves, np.array_equal(f, ref)))
    assert np.array_equal(f, ref)


def test_conservation_periodic():
    """Totals of rho, j, e on a periodic grid are conserved to rounding."""
    from paper_1106_0785_amd import lbm

    p, fl = inputs.smooth_periodic(seed=11, nx=200, ny=120, amp=0.08)
    sim = lbm.Simulation(p)
    sim.init(**fl)

    def totals():
        m = {k: v.cpu().numpy() for k, v in sim.moments().items()}
        r, u, v, T = m["rho"], m["ux"], m["uy"], m["T"]
        return np.array([r.sum(), (r * u).sum(), (r * v).sum(), (r * (T + 0.5 * (u * u + v * v))).sum()])

    t0 = totals()
    sim.step(1000)
    t1 = totals()
    sim.check()
    sim.close()
    rel = np.abs(t1 - t0) / np.abs(t0)
    log("conservation 200x120 1000 steps: relative drift %s" % rel)
    assert np.all(rel <= 1e-13)


def test_rm_5000_steps_reduced_grid():
    """The shock/interface problem for its full 5000 steps on a 256 x 64 grid."""
    p, fl, _ = inputs.rm(seed=6, nx=256, ny=64)
    g, _ = gpu_run(p, fl, 5000)
    o, _ = oracle_run(p, fl, 5000)
    assert_parity(g, o, what="rm 256x64 5000 steps")


def _small(seed, nx, ny, bc, **kw):
    p, fl = inputs.smooth_periodic(seed=seed, nx=nx, ny=ny, amp=0.06, **kw)
    p["bc"] = bc
    return p, fl


CASES = {
    "zero_gradient_x_specular_y": (["zero_gradient", "zero_gradient", "specular", "specular"], {}),
    "specular_x_periodic_y": (["specular", "specular", "periodic", "periodic"], {}),
    "periodic_both_v2": (["periodic"] * 4, {"eq_version": 2}),
    "periodic_both_v3": (["periodic"] * 4, {"eq_version": 3}),
    "unmodified": (["periodic"] * 4, {"modified": 0}),
    "printed_q8_sign": (["periodic"] * 4, {"modified": 2}),
}


@pytest.mark.parametrize("waves", [4, 2])
@pytest.mark.parametrize("name", sorted(CASES))
def test_boundary_and_model_variants(name, waves):
    bc, kw = CASES[name]
    p, fl = _small(7, 70, 23, bc, **kw)
    log("variant %s 70x23 200 steps, %d-wave tiles" % (name, waves))
    g, _ = gpu_run(p, fl, 200, waves=waves)
    o, _ = oracle_run(p, fl, 200)
    assert_parity(g, o, what=name)


@pytest.mark.parametrize("waves", [4, 2])
def test_dirichlet_ghost(waves):
    p, fl = _small(8, 66, 9, ["dirichlet_eq", "zero_gradient", "periodic", "periodic"])
    p["wall"][0] = [1.05, 0.02, 0.0, 1.02]
    log("dirichlet x_lo 66x9 200 steps, %d-wave tiles" % waves)
    g, _ = gpu_run(p, fl, 200, waves=waves)
    o, _ = oracle_run(p, fl, 200)
    assert_parity(g, o, what="dirichlet")


def test_neq_walls_on_x():
    p, fl, _ = inputs.couette_x(2.0, nx=40, ny=3)
    log("neq walls on x 40x3 2000 steps")
    g, _ = gpu_run(p, fl, 2000)
    o, _ = oracle_run(p, fl, 2000)
    assert_parity(g, o, what="neq x walls")


@pytest.mark.parametrize("waves", [4, 2])
@pytest.mark.parametrize("shape", [(1, 1), (2, 2), (1, 37), (300, 1), (63, 5), (125, 3), (64, 7), (129, 6)])
def test_degenerate_shapes(shape, waves):
    nx, ny = shape
    p, fl = _small(5, nx, ny, ["periodic"] * 4)
    log("shape %dx%d, %d-wave tiles" % (shape + (waves,)))
    g, _ = gpu_run(p, fl, 100, waves=waves)
    o, _ = oracle_run(p, fl, 100)
    assert_parity(g, o, what="shape %dx%d" % shape)


def test_couette_column_nx1():
    p, fl, _ = inputs.couette(0.7, nx=1, ny=50)
    g, _ = gpu_run(p, fl, 3000)
    o, _ = oracle_run(p, fl, 3000)
    assert_parity(g, o, what="couette nx=1")


def test_zero_steps_returns_initial_state():
    p, fl, _ = inputs.rm(seed=5, nx=64, ny=16)
    g, _ = gpu_run(p, fl, 0)
    o, _ = oracle_run(p, fl, 0)
    assert_parity(g, o, tol=1e-14, what="zero steps")


def test_health_flag_reports_blow_up():
    """A sharp (unsmoothed) jump with the central stencil overflows within a
    few hundred steps; lbm_check reports it."""
    from paper_1106_0785_amd import lbm

    p, fl, _ = inputs.riemann("sod", Pr=1.0, nx=400, ny=1, width_cells=1e-3)
    sim = lbm.Simulation(p)
    sim.init(**fl)
    sim.step(3000)
    with pytest.raises(lbm.LbmError) as e:
        sim.check()
    assert e.value.status == -5
    sim.close()


@pytest.mark.parametrize("shape", [(4096, 64), (100, 37), (1, 5)])
def test_stream_copy_probe_copies_exactly(shape):
    """The bandwidth probe copies every pitched plane (padding included)."""
    import torch

    from paper_1106_0785_amd import lbm

    nx, ny = shape
    pitch = (nx + 63) // 64 * 64
    n = 16 * ny * pitch
    a = torch.arange(n, dtype=torch.float64, device="cuda") * 0.5 + 1.0
    b = torch.zeros_like(a)
    lbm.lbm_stream_copy(a, b, nx, ny)
    torch.cuda.synchronize()
    assert torch.equal(a, b)


@pytest.mark.parametrize("waves", [4, 2])
def test_shock_bubble_small(waves):
    """Shock-bubble set-up (Sec. IV.B(b)) at 120 x 40: fixed-state inflow on
    the right, extrapolation on the left, reflecting y sides."""
    p, fl, _ = inputs.shock_bubble(nx=120, ny=40)
    log("shock-bubble 120x40 2000 steps, %d-wave tiles" % waves)
    g, _ = gpu_run(p, fl, 2000, waves=waves)
    o, _ = oracle_run(p, fl, 2000)
    assert_parity(g, o, what="shock-bubble 120x40")


# Grids of at most 512 nodes run by default in the one-workgroup kernel that
# keeps the grid in LDS and takes many steps per launch (variant 2).
SMALL = {
    "periodic_v1": (["periodic"] * 4, {}, (23, 19)),
    "periodic_v2": (["periodic"] * 4, {"eq_version": 2}, (23, 19)),
    "periodic_v3": (["periodic"] * 4, {"eq_version": 3}, (23, 19)),
    "unmodified": (["periodic"] * 4, {"modified": 0}, (23, 19)),
    "printed_q8_sign": (["periodic"] * 4, {"modified": 2}, (23, 19)),
    "zero_gradient_x_specular_y": (["zero_gradient", "zero_gradient", "specular", "specular"], {}, (31, 16)),
    "specular_x_periodic_y": (["specular", "specular", "periodic", "periodic"], {}, (16, 31)),
    "dirichlet_x": (["dirichlet_eq", "zero_gradient", "periodic", "periodic"], {}, (66, 7)),
    "line_512": (["periodic"] * 4, {}, (512, 1)),
    "column_512": (["periodic"] * 4, {}, (1, 512)),
    "one_node": (["periodic"] * 4, {}, (1, 1)),
    "ragged_wave": (["periodic"] * 4, {}, (5, 13)),
}


@pytest.mark.parametrize("name", sorted(SMALL))
def test_small_grid_kernel(name):
    bc, kw, (nx, ny) = SMALL[name]
    p, fl = _small(9, nx, ny, bc, **kw)
    if bc[0] == "dirichlet_eq":
        p["wall"][0] = [1.05, 0.02, 0.0, 1.02]
    log("small-grid kernel %s %dx%d 500 steps" % (name, nx, ny))
    g, f2 = gpu_run(p, fl, 500, variant=2)
    o, _ = oracle_run(p, fl, 500)
    assert_parity(g, o, what="small-grid " + name)
    _, f0 = gpu_run(p, fl, 500, variant=0)
    d = _kernel_diff(f2, f0)
    log("small-grid vs fused kernel: max diff %.2e" % d)
    assert d <= 1e-13


@pytest.mark.parametrize("axis", ["y", "x"])
def test_small_grid_kernel_walls(axis):
    """NEQ walls in the small-grid kernel, on either axis, with a step count
    above one launch's chunk (65536) so the hand-over between launches is
    exercised."""
    if axis == "y":
        p, fl, _ = inputs.couette(0.7, nx=4, ny=64)
    else:
        p, fl, _ = inputs.couette_x(2.0, nx=40, ny=3)
    steps = 70000
    log("small-grid kernel, NEQ walls on %s, %dx%d, %d steps" % (axis, p["nx"], p["ny"], steps))
    g, f2 = gpu_run(p, fl, steps, variant=2)
    _, f0 = gpu_run(p, fl, steps, variant=0)
    d = _kernel_diff(f2, f0)
    log("small-grid vs fused kernel after %d steps: max diff %.2e" % (steps, d))
    assert d <= 1e-11
    o, _ = oracle_run(p, fl, 3000)
    g3, _ = gpu_run(p, fl, 3000, variant=2)
    assert_parity(g3, o, what="small-grid walls on " + axis)


def test_small_grid_variant_is_rejected_for_larger_grids():
    from paper_1106_0785_amd import lbm

    p, fl = _small(9, 33, 16, ["periodic"] * 4)  # 528 nodes
    sim = lbm.Simulation(p)
    with pytest.raises(lbm.LbmError):
        sim.set_variant(2)
    p, fl = _small(9, 32, 16, ["periodic"] * 4)
    p["scheme"] = 1
    sim2 = lbm.Simulation(p)
    with pytest.raises(lbm.LbmError):
        sim2.set_variant(2)
    sim.close()
    sim2.close()


@pytest.mark.parametrize("version", [1, 2, 3])
def test_equal_rates_single_relaxation(version):
    """Every rate equal (the single-relaxation limit of the three versions)."""
    p, fl = _small(12, 70, 23, ["periodic"] * 4, eq_version=version)
    p["s"] = [2.0e3] * 16
    log("equal rates, version %d, 70x23 300 steps" % version)
    g, _ = gpu_run(p, fl, 300)
    o, _ = oracle_run(p, fl, 300)
    assert_parity(g, o, what="equal rates v%d" % version)


@pytest.mark.parametrize("bc", [["periodic"] * 4, ["specular", "zero_gradient", "periodic", "periodic"],
                                ["dirichlet_eq", "specular", "zero_gradient", "specular"]])
def test_state_changes_between_steps(bc):
    """Everything that writes the distributions between steps (init,
    restore from a checkpoint, a step of another kernel variant, the tuner's
    probes and restore) leaves the next step a consistent state. Three
    strips (nx = 150), several x boundary kinds."""
    from paper_1106_0785_amd import lbm

    p, fl = _small(13, 150, 21, bc)
    if bc[0] == "dirichlet_eq":
        p["wall"][0] = [1.04, 0.03, 0.0, 1.01]
    f0 = oracle.init(p, **fl)
    f20 = oracle.run(p, f0, 20)
    sim = lbm.Simulation(p)
    sim.init(**fl)
    sim.step(7)
    sim.set_f(f20)  # restore: the next step must not use the edges of step 7
    sim.step(5)
    sim.set_variant(1)
    sim.step(4)  # plain kernel: leaves the edge copies stale
    sim.set_variant(0)
    sim.step(6)
    sim.tune(probe_steps=2)  # probes, then restores the state
    sim.step(5)
    got = sim.get_f().cpu().numpy()
    sim.check()
    sim.close()
    ref = oracle.run(p, f20, 20)
    err = float(np.max(np.abs(got - ref)) / np.max(np.abs(ref)))
    log("state changes between steps, bc %s: max rel diff %.2e" % (bc, err))
    assert err <= 1e-12


# Narrow grids (at most 16 rows, more than 512 nodes) can run in the band
# kernel (variant 3): LDS windows of all rows, several steps per launch.
BAND = {
    "periodic_2000x4": (["periodic"] * 4, {}, (2000, 4)),
    "line_700": (["periodic"] * 4, {}, (700, 1)),
    "specular_x_333x16": (["specular", "specular", "periodic", "periodic"], {}, (333, 16)),
    "zero_gradient_x_specular_y_130x9": (["zero_gradient", "zero_gradient", "specular", "specular"], {}, (130, 9)),
    "dirichlet_x_200x5": (["dirichlet_eq", "zero_gradient", "periodic", "periodic"], {}, (200, 5)),
    "periodic_40x13_v2": (["periodic"] * 4, {"eq_version": 2}, (40, 13)),
    "periodic_97x8_v3": (["periodic"] * 4, {"eq_version": 3}, (97, 8)),
    "unmodified_515x1": (["periodic"] * 4, {"modified": 0}, (515, 1)),
    "printed_q8_sign_90x7": (["periodic"] * 4, {"modified": 2}, (90, 7)),
}


@pytest.mark.parametrize("name", sorted(BAND))
def test_band_kernel(name):
    bc, kw, (nx, ny) = BAND[name]
    p, fl = _small(14, nx, ny, bc, **kw)
    if bc[0] == "dirichlet_eq":
        p["wall"][0] = [1.05, 0.02, 0.0, 1.02]
    steps = 203  # not a multiple of the steps per launch
    log("band kernel %s %dx%d %d steps" % (name, nx, ny, steps))
    g, f3 = gpu_run(p, fl, steps, variant=3)
    o, _ = oracle_run(p, fl, steps)
    assert_parity(g, o, what="band " + name)
    _, f0 = gpu_run(p, fl, steps, variant=0)
    d = _kernel_diff(f3, f0)
    log("band vs fused kernel: max diff %.2e" % d)
    assert d <= 1e-13


@pytest.mark.parametrize("axis", ["y", "x"])
def test_band_kernel_walls(axis):
    """NEQ walls in the band kernel: on the rows of a 600 x 5 channel, or on
    the first and last columns of a 700 x 3 one."""
    if axis == "y":
        p, fl, _ = inputs.couette(0.7, nx=600, ny=5, dt_over_dy=0.05)
    else:
        p, fl, _ = inputs.couette_x(2.0, nx=700, ny=3)
    steps = 1001
    log("band kernel, NEQ walls on %s, %dx%d, %d steps" % (axis, p["nx"], p["ny"], steps))
    g, f3 = gpu_run(p, fl, steps, variant=3)
    o, _ = oracle_run(p, fl, steps)
    assert_parity(g, o, what="band walls on " + axis)
    _, f0 = gpu_run(p, fl, steps, variant=0)
    d = _kernel_diff(f3, f0)
    log("band vs fused kernel: max diff %.2e" % d)
    assert d <= 1e-12


def test_window_variant_is_rejected_where_it_does_not_apply():
    """Variant 3 needs scheme 0 and more than 512 nodes."""
    from paper_1106_0785_amd import lbm

    for nx, ny, scheme in [(16, 32, 0), (20, 20, 0), (300, 4, 1)]:
        p, fl = _small(9, nx, ny, ["periodic"] * 4)
        p["scheme"] = scheme
        sim = lbm.Simulation(p)
        with pytest.raises(lbm.LbmError):
            sim.set_variant(3)
        sim.close()


WINDOWS = {
    "periodic_200x77_32x16h2": (["periodic"] * 4, {}, (200, 77), (32, 16, 2)),
    "specular_130x60_16x32h3": (["specular", "specular", "zero_gradient", "zero_gradient"], {}, (130, 60), (16, 32, 3)),
    "dirichlet_150x45_64x8h1": (["dirichlet_eq", "zero_gradient", "specular", "specular"], {}, (150, 45), (64, 8, 1)),
    "periodic_v3_99x99_8x8h3": (["periodic"] * 4, {"eq_version": 3}, (99, 99), (8, 8, 3)),
    "mixed_x_periodic_y_70x200_32x16h4": (["zero_gradient", "specular", "periodic", "periodic"], {"modified": 2},
                                          (70, 200), (32, 16, 4)),
}


@pytest.mark.parametrize("name", sorted(WINDOWS))
def test_window_kernel_cut_both_axes(name):
    """The windowed kernel with windows cut along both axes."""
    bc, kw, (nx, ny), (wc, wr, h) = WINDOWS[name]
    p, fl = _small(15, nx, ny, bc, **kw)
    if bc[0] == "dirichlet_eq":
        p["wall"][0] = [1.05, 0.02, 0.0, 1.02]
    from paper_1106_0785_amd import lbm

    steps = 101
    sim = lbm.Simulation(p)
    sim.set_variant(3)
    sim.set_window(wc, wr, h)
    sim.init(**fl)
    sim.step(steps)
    g = {k: v.cpu().numpy() for k, v in sim.moments().items()}
    f3 = sim.get_f().cpu().numpy()
    sim.check()
    sim.close()
    o, _ = oracle_run(p, fl, steps)
    assert_parity(g, o, what="windows %s" % name)
    _, f0 = gpu_run(p, fl, steps, variant=0)
    d = _kernel_diff(f3, f0)
    log("windows %s vs fused kernel: max diff %.2e" % (name, d))
    assert d <= 1e-13


@pytest.mark.parametrize("axis", ["y", "x"])
def test_window_kernel_walls_on_a_cut_axis(axis):
    """NEQ walls on an axis cut into windows (only the end windows hold
    wall nodes)."""
    from paper_1106_0785_amd import lbm

    if axis == "y":
        p, fl, _ = inputs.couette(0.7, nx=40, ny=64)
    else:
        p, fl, _ = inputs.couette_x(2.0, nx=64, ny=40)
    steps = 1001
    sim = lbm.Simulation(p)
    sim.set_variant(3)
    sim.set_window(16, 32, 3)
    sim.init(**fl)
    sim.step(steps)
    g = {k: v.cpu().numpy() for k, v in sim.moments().items()}
    sim.check()
    sim.close()
    o, _ = oracle_run(p, fl, steps)
    assert_parity(g, o, what="windows, walls on " + axis)


def test_window_shapes_are_checked():
    from paper_1106_0785_amd import lbm

    p, fl = _small(9, 100, 50, ["periodic"] * 4)
    sim = lbm.Simulation(p)
    for bad in [(32, 16, 0), (32, 32, 2), (4, 16, 2), (600, 1, 1)]:
        with pytest.raises(lbm.LbmError):
            sim.set_window(*bad)
    sim.set_window(32, 16, 2)
    assert sim.window() == (32, 16, 2)
    sim.close()


@pytest.mark.parametrize("case", ["sod_2000x4", "rm_256x64", "rm_300x100"])
def test_tuner_picks_a_kernel_and_keeps_the_state(case):
    """The tuner times fused tile shapes, window shapes and two-step tile
    shapes, keeps the fastest kernel (variant 0, 3 or 4), and restores the
    state; the run that follows matches the oracle."""
    from paper_1106_0785_amd import lbm

    if case == "sod_2000x4":
        p, fl, _ = inputs.riemann("sod", Pr=1.0, nx=2000, ny=4)
    else:
        nx, ny = (256, 64) if case == "rm_256x64" else (300, 100)
        p, fl, _ = inputs.rm(seed=8, nx=nx, ny=ny)
    sim = lbm.Simulation(p)
    sim.init(**fl)
    f0 = sim.get_f().cpu().numpy()
    sim.tune(probe_steps=8)
    variant = sim.variant()
    log("tuner on %s: variant %d, window %s, tile %s" % (case, variant, sim.window(), sim.tile()))
    assert variant in (0, 3, 4)
    assert np.array_equal(sim.get_f().cpu().numpy(), f0)
    sim.step(100)
    g = {k: v.cpu().numpy() for k, v in sim.moments().items()}
    sim.check()
    sim.close()
    o, _ = oracle_run(p, fl, 100)
    assert_parity(g, o, what="after tuning, " + case)


def test_random_configurations_all_kernels():
    """40 seeded random problems (shape, boundary kinds on each axis,
    equilibrium version, modification, kernel variant and window shape)
    against the oracle."""
    from paper_1106_0785_amd import lbm

    rng = np.random.default_rng(2024)
    kinds = ["periodic", "zero_gradient", "specular", "dirichlet_eq", "neq_wall"]
    done = 0
    while done < 40:
        nx = int(rng.integers(1, 120))
        ny = int(rng.integers(1, 60)) if rng.random() < 0.7 else int(rng.integers(1, 9))
        bx = kinds[int(rng.integers(0, 5))]
        by = kinds[int(rng.integers(0, 5))]
        if bx == "neq_wall" and by == "neq_wall":
            continue
        if (nx == 1 and bx != "periodic") or (ny == 1 and by != "periodic"):
            continue
        if (bx == "neq_wall" and nx < 3) or (by == "neq_wall" and ny < 3):
            continue
        version, modified = int(rng.integers(1, 4)), int(rng.integers(0, 3))
        p, fl = _small(int(rng.integers(0, 10 ** 6)), nx, ny, [bx, bx, by, by], eq_version=version,
                       modified=modified)
        for side in range(4):
            p["wall"][side] = [1.0 + 0.05 * rng.random(), 0.05 * rng.standard_normal(), 0.05 * rng.standard_normal(),
                               1.0 + 0.05 * rng.random()]
        choices = [0, 1]
        if nx * ny <= 512:
            choices.append(2)
        else:
            choices.append(3)
        variant = int(rng.choice(choices))
        steps = int(rng.integers(1, 60))
        sim = lbm.Simulation(p)
        sim.set_variant(variant)
        window = None
        if variant == 3 and rng.random() < 0.5:
            for _ in range(10):
                cand = (int(rng.choice([8, 16, 32, 64])), int(rng.choice([4, 8, 16, 32])), int(rng.integers(1, 4)))
                try:
                    sim.set_window(*cand)
                    window = cand
                    break
                except lbm.LbmError:
                    pass
        sim.init(**fl)
        sim.step(steps)
        g = {k: v.cpu().numpy() for k, v in sim.moments().items()}
        sim.check()
        sim.close()
        o, _ = oracle_run(p, fl, steps)
        assert_parity(g, o, what="random %d: %dx%d bc (%s, %s) v%d m%d variant %d window %s, %d steps"
                      % (done, nx, ny, bx, by, version, modified, variant, window, steps))
        done += 1


@pytest.mark.parametrize("case", ["periodic", "walls", "limited"])
def test_store_modes_give_identical_results(case):
    """Non-temporal and ordinary stores in the fused kernel: the same
    results bit for bit (a cache hint only)."""
    from paper_1106_0785_amd import lbm

    if case == "periodic":
        p, fl = _small(16, 300, 100, ["periodic"] * 4)
    elif case == "walls":
        p, fl, _ = inputs.couette(0.7, nx=40, ny=64)
    else:
        p, fl, _ = inputs.rm(seed=9, nx=200, ny=60, width_cells=0.5)
        p["scheme"] = 1
    f = []
    for nt in (1, 0):
        sim = lbm.Simulation(p)
        sim.set_variant(0)
        sim.set_store_mode(nt)
        assert sim.store_mode() == nt
        sim.init(**fl)
        sim.step(41)
        f.append(sim.get_f().cpu().numpy())
        sim.check()
        sim.close()
    log("store modes, %s: bitwise equal %s" % (case, np.array_equal(f[0], f[1])))
    assert np.array_equal(f[0], f[1])
    sim = lbm.Simulation(p)
    with pytest.raises(lbm.LbmError):
        sim.set_store_mode(2)
    sim.close()


@pytest.mark.parametrize("case", ["y_walls_23x37", "x_walls_193x3", "x_walls_193x5"])
def test_window_kernel_wall_node_written_alone(case):
    """Shapes where a window's written part is (almost) only a wall node:
    the wall takes its fluid neighbour's value of the same step, so cut sides
    on a walled axis overlap by one node more."""
    from paper_1106_0785_amd import lbm

    if case == "y_walls_23x37":
        p, fl = _small(21, 23, 37, ["periodic", "periodic", "neq_wall", "neq_wall"], eq_version=2, modified=0)
    else:
        nx, ny = (193, 3) if case == "x_walls_193x3" else (193, 5)
        p, fl = _small(22, nx, ny, ["neq_wall", "neq_wall", "periodic", "periodic"])
    for side in range(4):
        p["wall"][side] = [1.0, 0.02 * side, -0.01 * side, 1.0 + 0.01 * side]
    steps = 38
    sim = lbm.Simulation(p)
    sim.set_variant(3)
    sim.init(**fl)
    sim.step(steps)
    g = {k: v.cpu().numpy() for k, v in sim.moments().items()}
    log("%s: window %s" % (case, sim.window()))
    sim.check()
    sim.close()
    o, _ = oracle_run(p, fl, steps)
    assert_parity(g, o, what="wall node written alone, " + case)
