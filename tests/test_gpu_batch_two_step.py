"""Two-step mode of the batched form: the plain tiled instances (Lax-Wendroff,
no NEQ walls) advance two steps per launch through the two-step kernel
(mode 1), one step when only one is left in the call or in their budget. Each such
instance must end bitwise where lbm_step with the two-step kernel (variant
4) puts it alone, the other instances where they always did, every instance
within 1e-11 of the oracle; graph replays, budgets, mode changes between
calls and two-step tile heights must not change results."""

import numpy as np
import pytest

from gpu_util import assert_parity, gpu_run, log, oracle_run
from paper_1106_0785_amd import inputs

pytestmark = pytest.mark.gpu

# A persistent form of the two-step tiles (every pair of a call in one launch,
# mode 2) was tried and taken out: its first GPU run went silent in the first
# mode-2 case, and reading the code found no cause. set_two_step rejects 2;
# the mode-2 cases stay here, skipped, as the record of it.
_MODE2_GONE = pytest.mark.skip(reason="persistent two-step form (mode 2) taken out: its first GPU run "
                                      "hung with no cause found by reading the code")
MODES = [1, pytest.param(2, marks=_MODE2_GONE)]


def _mixed(seed, n):
    from paper_1106_0785_amd.batch import Batch

    items = inputs.mixed_batch(seed=seed, n=n)
    b = Batch([p for _, p, _ in items])
    b.init([f for _, _, f in items])
    return items, b


def _plain_tiled(p):
    tiled = (p["nx"] > 1 and p["ny"] > 1) or (p["ny"] == 1 and p["bc"][0] == "periodic" and p["nx"] > 128)
    return tiled and p.get("scheme", 0) == 0 and "neq_wall" not in p["bc"]


def _rel(a, b):
    return float(np.max(np.abs(a - b) / np.abs(b).max(axis=(1, 2), keepdims=True)))


def _check_against_single(items, b, fb, steps_of):
    m = {k: v.cpu().numpy() for k, v in b.moments().items()}
    plain = 0
    for i, (kind, p, fl) in enumerate(items):
        n = steps_of(i)
        fi = b.f_of(fb, i)
        if _plain_tiled(p):
            plain += 1
            _, g4 = gpu_run(p, fl, n, variant=4)
            assert np.array_equal(fi, g4), (i, kind, n, _rel(fi, g4))
        else:
            _, g0 = gpu_run(p, fl, n, variant=0)
            if p["nx"] > 1 and p["ny"] > 1:
                assert np.array_equal(fi, g0), (i, kind, n)
            else:
                assert _rel(fi, g0) <= 1e-12, (i, kind, n)
        o, _ = oracle_run(p, fl, n)
        assert_parity({k: b.split(v, i) for k, v in m.items()}, o,
                      what="two-step batch instance %d (%s, %dx%d, %d steps)" % (i, kind, p["nx"], p["ny"], n))
    return plain


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("steps", [150, 151])
def test_two_step_mode_matches_single_problem_paths_and_oracle(steps, mode):
    items, b = _mixed(3, 18)
    b.set_two_step(mode, 16)
    b.step(steps)
    b.check()
    fb = b.get_f().cpu().numpy()
    plain = _check_against_single(items, b, fb, lambda i: steps)
    log("two-step mode, %d steps: %d plain tiled instances bitwise equal to variant 4" % (steps, plain))
    assert plain >= 4
    b.close()


@pytest.mark.parametrize("mode", MODES)
def test_two_step_mode_with_budgets(mode):
    """Budgets of both parities, below and above the call's length, and 0."""
    items, b = _mixed(8, 18)
    budgets = [11 * (i + 1) + (i % 3) for i in range(len(items))]
    budgets[5] = 0
    b.set_budgets(budgets)
    b.set_two_step(mode, 8)
    b.step(101)
    b.check()
    fb = b.get_f().cpu().numpy()
    _check_against_single(items, b, fb, lambda i: min(101, budgets[i]))
    b.close()


@pytest.mark.parametrize("mode", MODES)
@pytest.mark.parametrize("rows", [2, 8, 32, 128])
def test_two_step_tile_heights_agree(rows, mode):
    items, b = _mixed(13, 12)
    items, r = _mixed(13, 12)
    budgets = [7 * (i + 2) + (i % 2) for i in range(len(items))]
    b.set_budgets(budgets)
    r.set_budgets(budgets)
    b.set_two_step(mode, rows)
    r.set_two_step(1, 16)
    info = b.two_step()
    assert info["two_step"] == mode and info["tile_rows2"] == rows and info["tiles2"] > 0
    b.step(61)
    r.step(61)
    assert np.array_equal(b.get_f().cpu().numpy(), r.get_f().cpu().numpy())
    b.close()
    r.close()


@pytest.mark.parametrize("mode", MODES)
def test_two_step_graph_replays_match_eager_runs(mode):
    import torch

    items, g = _mixed(9, 12)
    items, e = _mixed(9, 12)
    g.set_schedule(256, 16, use_graph=True)
    e.set_schedule(256, 16, use_graph=False)
    g.set_two_step(mode, 16)
    e.set_two_step(1, 16)
    for rep, k in enumerate((47, 47, 30, 47, 1)):
        g.step(k)
        e.step(k)
        torch.cuda.synchronize()
        _ = torch.ones(1000, device="cuda").sum().item()
        fg, fe = g.get_f().cpu().numpy(), e.get_f().cpu().numpy()
        log("two-step graph replay %d (%d steps) bitwise equal to eager: %s" % (rep, k, np.array_equal(fg, fe)))
        assert np.array_equal(fg, fe)
    g.close()
    e.close()


def test_mode_changes_between_calls():
    """One-step and two-step calls in turn (odd lengths, so the kinds of
    instance sit in different buffers at each change): the result is that of
    the same calls made by lbm_step on each instance (variant 0, 4, ...),
    and within 1e-11 of the oracle."""
    from paper_1106_0785_amd import lbm

    items, b = _mixed(5, 12)
    plan = ((0, 33), (1, 41), (0, 17), (1, 29), (1, 6), (0, 1), (1, 1))
    for mode, k in plan:
        b.set_two_step(mode, 16)
        b.step(k)
    b.check()
    fb = b.get_f().cpu().numpy()
    total = sum(k for _, k in plan)
    m = {k: v.cpu().numpy() for k, v in b.moments().items()}
    for i, (kind, p, fl) in enumerate(items):
        if _plain_tiled(p):
            sim = lbm.Simulation(p)
            sim.init(**fl)
            for mode, k in plan:
                sim.set_variant(4 if mode else 0)
                sim.step(k)
            ref = sim.get_f().cpu().numpy()
            sim.close()
            assert np.array_equal(b.f_of(fb, i), ref), (i, kind)
        o, _ = oracle_run(p, fl, total)
        assert_parity({k: b.split(v, i) for k, v in m.items()}, o, what="mode changes, instance %d (%s)" % (i, kind))
    b.close()


def test_tuner_with_two_step_candidates_keeps_state():
    items, b = _mixed(11, 12)
    b.step(17)
    f0 = b.get_f().cpu().numpy()
    s = b.tune(probe_steps=16, use_cache=False)
    log("tuner choice with two-step candidates: %s" % s)
    assert np.array_equal(f0, b.get_f().cpu().numpy())
    assert "two_step" in s and "tile_rows2" in s
    b.close()


def test_set_two_step_rejects_bad_arguments():
    from paper_1106_0785_amd import lbm

    items, b = _mixed(1, 6)
    for args in ((2, 16), (3, 16), (-1, 16), (1, 3), (1, 0), (1, 8192)):
        with pytest.raises(lbm.LbmError):
            b.set_two_step(*args)
    b.close()
