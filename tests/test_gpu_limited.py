"""The flux-limited scheme (scheme 1: Lax-Wendroff with a minmod limiter on
its anti-diffusive flux, radius 2, two ghost layers) on the GPU against the
oracle, including sharp jumps that the central scheme does not survive."""

import numpy as np
import pytest

from gpu_util import assert_parity, gpu_run, log, oracle_run
from paper_1106_0785_amd import inputs
from physics import riemann_sample

pytestmark = pytest.mark.gpu


def _kernel_diff(a, b):
    """Max difference of two distribution arrays, relative per plane."""
    return float(np.max(np.abs(a - b) / np.abs(b).max(axis=(1, 2), keepdims=True)))


def test_sharp_sod_full_run():
    """Sharp Sod tube, 2000 x 4. At 2000 steps the GPU path is within 1e-11 of
    the oracle. Over the full 20 000 steps the limiter's switching amplifies
    FP64 rounding: two equally valid evaluations of the oracle (plain and with
    fused multiply-adds) already differ by ~5e-8, so the full run is held to
    20 x that measured noise floor, and to the exact solution."""
    import oracle

    from gpu_util import field_errors

    nx = 2000
    p, fl, _ = inputs.riemann("sod", Pr=1.0, nx=nx, ny=4, width_cells=0.01)
    p["scheme"] = 1
    log("limited scheme, sharp Sod 2000x4, 2000 steps")
    g, _ = gpu_run(p, fl, 2000)
    o, _ = oracle_run(p, fl, 2000)
    assert_parity(g, o, what="limited sharp sod 2000 steps")
    steps = 20000
    log("limited scheme, sharp Sod 2000x4, 20000 steps")
    g, _ = gpu_run(p, fl, steps)
    f0 = oracle.init(p, **fl)
    o = oracle.moments(p, oracle.run(p, f0, steps))
    o_fma = oracle.moments(p, oracle.run(p, f0, steps, variant="fma"))
    floor = field_errors(o_fma, o)
    err = field_errors(g, o)
    log("noise floor (oracle fma vs plain): %s" % ", ".join("%s %.1e" % kv for kv in floor.items()))
    log("gpu vs oracle: %s" % ", ".join("%s %.1e" % kv for kv in err.items()))
    for k in err:
        assert err[k] <= max(20.0 * floor[k], 1e-11), (k, err[k], floor[k])
    x = (np.arange(nx) + 0.5) / nx
    rho_e, u_e, p_e = riemann_sample((1.0, 0.0, 1.0), (0.125, 0.0, 0.1), (x - 0.5) / (steps * p["dt"]))
    l1 = float(np.mean(np.abs(g["rho"][0] - rho_e)) / np.mean(rho_e))
    log("limited sharp Sod: L1 relative error of rho vs exact %.4f" % l1)
    assert l1 < 0.006


CASES = {
    "zero_gradient_x_specular_y": ["zero_gradient", "zero_gradient", "specular", "specular"],
    "specular_x_periodic_y": ["specular", "specular", "periodic", "periodic"],
    "periodic_both": ["periodic"] * 4,
    "dirichlet_x_zero_gradient": ["dirichlet_eq", "zero_gradient", "periodic", "periodic"],
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_boundary_kinds(name):
    p, fl = inputs.smooth_periodic(seed=7, nx=70, ny=23, amp=0.06)
    p["bc"] = CASES[name]
    p["wall"][0] = [1.05, 0.02, 0.0, 1.02]
    p["scheme"] = 1
    log("limited scheme %s 70x23 200 steps" % name)
    g, _ = gpu_run(p, fl, 200)
    o, _ = oracle_run(p, fl, 200)
    assert_parity(g, o, what="limited " + name)


@pytest.mark.parametrize("shape", [(1, 1), (2, 2), (3, 5), (5, 3), (1, 37), (300, 1), (64, 7), (129, 6), (66, 9)])
def test_shapes(shape):
    nx, ny = shape
    p, fl = inputs.smooth_periodic(seed=5, nx=nx, ny=ny, amp=0.06)
    p["scheme"] = 1
    log("limited scheme shape %dx%d" % shape)
    g, _ = gpu_run(p, fl, 100)
    o, _ = oracle_run(p, fl, 100)
    assert_parity(g, o, what="limited shape %dx%d" % shape)


def test_sharp_shock_bubble():
    p, fl, _ = inputs.shock_bubble(nx=120, ny=40, width_cells=0.01)
    p["scheme"] = 1
    log("limited scheme, sharp shock-bubble 120x40 2000 steps")
    g, _ = gpu_run(p, fl, 2000)
    o, _ = oracle_run(p, fl, 2000)
    assert_parity(g, o, what="limited sharp shock-bubble")


def test_fused_matches_plain_kernel():
    p, fl, _ = inputs.rm(seed=2, nx=300, ny=100, width_cells=0.5)
    p["scheme"] = 1
    _, f0 = gpu_run(p, fl, 50, variant=0)
    _, f1 = gpu_run(p, fl, 50, variant=1)
    d = _kernel_diff(f0, f1)
    log("limited scheme fused vs plain 300x100 50 steps: max diff %.2e" % d)
    assert d <= 1e-13


@pytest.mark.parametrize("rows", [4, 16, 64])
def test_tile_rows_do_not_change_result(rows):
    p, fl, _ = inputs.rm(seed=3, nx=190, ny=77, width_cells=0.5)
    p["scheme"] = 1
    _, f = gpu_run(p, fl, 30, rows=rows)
    _, ref = gpu_run(p, fl, 30, rows=8)
    assert np.array_equal(f, ref)
