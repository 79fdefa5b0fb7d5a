"""The two-steps-per-launch kernel (variant 4) against the oracle and against
the one-step kernel: every boundary kind it takes, the three equilibrium
versions and the modification modes, ragged and narrow shapes (strips of 62
columns cut anywhere), odd step counts (the last step then takes the
one-step kernel), tile shapes, and the 4096 x 1024 problem at full size."""

import numpy as np
import pytest

from gpu_util import assert_parity, gpu_run, log, oracle_run
from paper_1106_0785_amd import inputs

pytestmark = pytest.mark.gpu


def _small(seed, nx, ny, bc, **kw):
    p, fl = inputs.smooth_periodic(seed=seed, nx=nx, ny=ny, amp=0.06, **kw)
    p["bc"] = bc
    p["wall"][0] = [1.03, 0.02, 0.01, 1.01]
    p["wall"][1] = [0.98, -0.01, 0.03, 1.04]
    p["wall"][2] = [1.01, -0.03, 0.02, 0.97]
    p["wall"][3] = [1.0, 0.05, -0.02, 1.02]
    return p, fl


CASES = {
    "periodic_v1": (["periodic"] * 4, {}),
    "periodic_v2": (["periodic"] * 4, {"eq_version": 2}),
    "periodic_v3": (["periodic"] * 4, {"eq_version": 3}),
    "unmodified": (["periodic"] * 4, {"modified": 0}),
    "printed_sign": (["specular", "specular", "periodic", "periodic"], {"modified": 2}),
    "specular_both": (["specular", "specular", "specular", "specular"], {}),
    "zero_gradient_both": (["zero_gradient", "zero_gradient", "zero_gradient", "zero_gradient"], {}),
    "fixed_state_x": (["dirichlet_eq", "zero_gradient", "periodic", "periodic"], {}),
    "fixed_state_y": (["periodic", "periodic", "dirichlet_eq", "specular"], {"eq_version": 3}),
    "mixed_sides": (["dirichlet_eq", "specular", "zero_gradient", "dirichlet_eq"], {"eq_version": 2}),
}

SHAPES = [(70, 20), (130, 37), (40, 30), (124, 9), (125, 8), (63, 64), (200, 3), (1, 50), (187, 1)]


def _ok(p, shape):
    nx, ny = shape
    if nx == 1 and p["bc"][0] != "periodic":
        return False
    if ny == 1 and p["bc"][2] != "periodic":
        return False
    return True


@pytest.mark.parametrize("name", sorted(CASES))
def test_two_step_kernel_matches_oracle(name):
    bc, kw = CASES[name]
    worst = 0
    for k, shape in enumerate(SHAPES):
        p, fl = _small(100 + k, shape[0], shape[1], bc, **kw)
        if not _ok(p, shape):
            continue
        steps = 31 if k % 2 else 40
        for waves, rows in ((4, 8), (2, 6)):
            g, _ = gpu_run(p, fl, steps, variant=4, rows=rows, waves=waves)
            o, _ = oracle_run(p, fl, steps)
            assert_parity(g, o, what="two-step %s %dx%d %d steps (%d waves, %d rows)"
                          % (name, shape[0], shape[1], steps, waves, rows))


def test_two_step_equals_one_step_to_rounding():
    """Same node arithmetic, other strips: the two kernels agree to rounding."""
    p, fl, _ = inputs.rm(seed=3, nx=700, ny=190)
    g4, f4 = gpu_run(p, fl, 60, variant=4)
    g0, f0 = gpu_run(p, fl, 60, variant=0)
    d = float(np.max(np.abs(f4 - f0) / np.abs(f0).max(axis=(1, 2), keepdims=True)))
    log("two-step vs one-step kernel, 700x190 shock/interface, 60 steps: %.2e" % d)
    assert d <= 1e-13


@pytest.mark.parametrize("rows,waves", [(2, 2), (4, 4), (8, 2), (16, 4), (64, 4), (128, 2)])
def test_two_step_tile_shape_does_not_change_result(rows, waves):
    """Tiles of other heights cut the same strips: bitwise the same result."""
    p, fl, _ = inputs.rm(seed=5, nx=300, ny=77)
    ref, fr = gpu_run(p, fl, 24, variant=4, rows=8, waves=4)
    g, f = gpu_run(p, fl, 24, variant=4, rows=rows, waves=waves)
    assert np.array_equal(f, fr), (rows, waves)


def test_two_step_headline_size_every_node():
    p, fl, _ = inputs.rm(seed=0, nx=4096, ny=1024)
    g, _ = gpu_run(p, fl, 6, variant=4)
    o, _ = oracle_run(p, fl, 6)
    assert_parity(g, o, what="two-step rm 4096x1024 6 steps")


def test_two_step_rm_1024x256_full_run():
    p, fl, _ = inputs.rm(seed=0, nx=1024, ny=256)
    g, _ = gpu_run(p, fl, 5000, variant=4)
    o, _ = oracle_run(p, fl, 5000)
    assert_parity(g, o, what="two-step rm 1024x256 5000 steps")


def test_two_step_health_flag():
    from paper_1106_0785_amd import lbm

    p, fl = _small(7, 90, 40, ["periodic"] * 4)
    fl["T"][11, 33] = -0.2
    sim = lbm.Simulation(p)
    sim.set_variant(4)
    sim.init(**fl)
    sim.step(2)
    with pytest.raises(lbm.LbmError) as err:
        sim.check()
    assert err.value.status == -5
    sim.close()


def test_two_step_rejects_walls_and_limited_scheme():
    from paper_1106_0785_amd import lbm

    p, fl, _ = inputs.couette(1.0)
    sim = lbm.Simulation(p)
    with pytest.raises(lbm.LbmError):
        sim.set_variant(4)
    sim.close()
    q, _ = _small(1, 80, 20, ["periodic"] * 4)
    q["scheme"] = 1
    sim = lbm.Simulation(q)
    with pytest.raises(lbm.LbmError):
        sim.set_variant(4)
    sim.close()
