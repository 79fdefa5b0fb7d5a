"""Persistent form of the batched line kernel: one launch per equilibrium
version runs every block of h steps of a call, each chunk starting a block
once the chunks it depends on have finished the block before. It must give
bitwise the result of one launch per block, in and out of a hipGraph, with
budgets, mixed versions and tiled instances, at schedules whose halo spans
several chunks, and its bounded waits must end every launch and be reported
when they run out (forced from the host with a zero time limit)."""

import numpy as np
import pytest

from gpu_util import assert_parity, log, oracle_run
from paper_1106_0785_amd import inputs

pytestmark = pytest.mark.gpu


def _make(items):
    from paper_1106_0785_amd.batch import Batch

    b = Batch([p for _, p, _ in items])
    b.init([f for _, _, f in items])
    return b


def _lines(seed, n, **kw):
    return inputs.batch(seed=seed, n=n, **kw)


def _run(items, steps, region, h, persistent, use_graph=True, budgets=None, calls=1):
    b = _make(items)
    b.set_schedule(region, h, use_graph=use_graph)
    b.set_persistent(persistent)
    if budgets is not None:
        b.set_budgets(budgets)
    for _ in range(calls):
        b.step(steps)
    b.check()
    f = b.get_f().cpu().numpy()
    info = b.persistent()
    b.close()
    return f, info


@pytest.mark.parametrize("region,h,steps", [(128, 8, 100), (256, 16, 100), (256, 32, 37), (128, 1, 5),
                                            (256, 24, 24), (128, 4, 3), (256, 112, 230), (128, 48, 100)])
def test_persistent_equals_block_launches(region, h, steps):
    items = _lines(21, 40, riemann_n=(256, 2500), couette_h=(32, 256))
    ref, _ = _run(items, steps, region, h, False, use_graph=False)
    for use_graph in (False, True):
        f, info = _run(items, steps, region, h, True, use_graph=use_graph)
        log("persistent (%d, %d) %d steps, graph %s, grid %d: bitwise %s"
            % (region, h, steps, use_graph, info["grid"], np.array_equal(f, ref)))
        assert info["persistent"] and info["grid"] > 0
        assert np.array_equal(f, ref)


def test_persistent_grid_exceeds_one_wave_of_chunks():
    """More chunks than resident workgroups: each workgroup takes several
    chunks per block (the 512-instance batch)."""
    items = _lines(0, 512)
    f, info = _run(items, 40, 256, 16, True)
    ref, _ = _run(items, 40, 256, 16, False)
    from paper_1106_0785_amd.batch import Batch

    b = Batch([p for _, p, _ in items])
    b.set_schedule(256, 16)
    chunks = b.schedule()["chunks"]
    b.close()
    log("512 instances: %d chunks on a persistent grid of %d workgroups" % (chunks, info["grid"]))
    assert chunks > info["grid"]
    assert np.array_equal(f, ref)


def test_persistent_mixed_versions_tiles_and_budgets():
    items = inputs.mixed_batch(seed=4, n=24)
    budgets = [13 * (i % 7) + 5 for i in range(len(items))]
    ref, _ = _run(items, 70, 256, 12, False, budgets=budgets, use_graph=False)
    f, _ = _run(items, 70, 256, 12, True, budgets=budgets)
    assert np.array_equal(f, ref)


def test_persistent_matches_oracle():
    items = _lines(23, 10, riemann_n=(256, 900), couette_h=(32, 120))
    b = _make(items)
    b.set_schedule(256, 16)
    b.set_persistent(True)
    b.step(150)
    b.check()
    m = {k: v.cpu().numpy() for k, v in b.moments().items()}
    for i, (kind, p, fl) in enumerate(items):
        o, _ = oracle_run(p, fl, 150)
        assert_parity({k: b.split(v, i) for k, v in m.items()}, o,
                      what="persistent batch instance %d (%s, %dx%d)" % (i, kind, p["nx"], p["ny"]))
    b.close()


def test_persistent_graph_replays_match_eager_runs():
    import torch

    items = _lines(25, 16, riemann_n=(256, 1200), couette_h=(32, 150))
    g, e = _make(items), _make(items)
    g.set_schedule(256, 16, use_graph=True)
    e.set_schedule(256, 16, use_graph=False)
    g.set_persistent(True)
    for rep in range(4):
        g.step(48)
        e.step(48)
        torch.cuda.synchronize()
        _ = torch.ones(1000, device="cuda").sum().item()
        fg, fe = g.get_f().cpu().numpy(), e.get_f().cpu().numpy()
        log("persistent graph replay %d bitwise equal to block launches: %s" % (rep, np.array_equal(fg, fe)))
        assert np.array_equal(fg, fe)
    g.check()
    g.close()
    e.close()


def test_wait_timeout_is_reported_and_cleared():
    """A zero time limit makes the first check of a chunk's dependencies
    (block 1 on) give up: every workgroup leaves, the launch ends, the batch
    reports LBM_ETIMEOUT once, and after re-initialisation the persistent
    form is exact again."""
    from paper_1106_0785_amd import lbm

    items = _lines(27, 24, riemann_n=(600, 2000), couette_h=(32, 200))
    b = _make(items)
    b.set_schedule(256, 16)
    b.set_persistent(True, timeout_ms=0.0)
    assert b.persistent()["grid"] >= 2
    b.step(64)  # 4 blocks
    with pytest.raises(lbm.LbmError) as err:
        b.check()
    assert err.value.status == -6
    b.check()  # cleared
    b.set_persistent(True)  # default limit
    b.init([f for _, _, f in items])
    b.step(64)
    b.check()
    f = b.get_f().cpu().numpy()
    b.close()
    ref, _ = _run(items, 64, 256, 16, False)
    assert np.array_equal(f, ref)


def test_persistent_health_flag():
    from paper_1106_0785_amd import lbm

    items = _lines(29, 8, riemann_n=(300, 600), couette_h=(32, 64))
    items[2][2]["T"][:] = -1.0
    b = _make(items)
    b.set_persistent(True)
    b.step(40)
    with pytest.raises(lbm.LbmError) as err:
        b.check()
    assert err.value.status == -5
    b.close()


def test_set_persistent_rejects_bad_arguments():
    from paper_1106_0785_amd import lbm

    b = _make(_lines(31, 4))
    for args in ((2, 100.0), (1, -1.0), (1, 1e9), (1, float("nan"))):
        with pytest.raises(lbm.LbmError):
            b.set_persistent(*args)
    b.close()


def test_persistent_with_every_budget_zero():
    """Budgets of 0 for every instance: each chunk only carries its nodes over
    block after block, in ticket order, and the state comes out unchanged."""
    items = _lines(33, 12, riemann_n=(256, 1500), couette_h=(32, 120))
    b = _make(items)
    f0 = b.get_f().cpu().numpy()
    b.close()
    for steps in (50, 51):
        f, info = _run(items, steps, 256, 16, True, budgets=[0] * len(items))
        assert info["grid"] > 0
        assert np.array_equal(f, f0)


def test_persistent_form_without_line_instances():
    """A batch of two-dimensional instances only: there is no line chunk to
    launch persistently (grid 0) and the tiled instances advance as before."""
    from paper_1106_0785_amd.batch import Batch

    items = inputs.rm_batch(seed=2, n=4)
    out = []
    for pers in (False, True):
        b = Batch([p for _, p, _ in items])
        b.init([f for _, _, f in items])
        b.set_persistent(pers)
        assert b.persistent()["grid"] == 0
        b.step(9)
        b.check()
        out.append(b.get_f().cpu().numpy())
        b.close()
    assert np.array_equal(out[0], out[1])
