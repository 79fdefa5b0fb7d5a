"""Batched form: every instance of an uneven batch ends where the
single-problem path and the oracle put it; budgets, schedules and graph
replays do not change results."""

import numpy as np
import pytest

from gpu_util import assert_parity, field_errors, gpu_run, log, oracle_run
from paper_1106_0785_amd import inputs

pytestmark = pytest.mark.gpu


def _batch(seed, n, **kw):
    from paper_1106_0785_amd.batch import Batch

    items = inputs.batch(seed=seed, n=n, **kw)
    b = Batch([p for _, p, _ in items])
    b.init([f for _, _, f in items])
    return items, b


def _moments_of(b, i):
    m = {k: v.cpu().numpy() for k, v in b.moments().items()}
    return {k: b.split(v, i) for k, v in m.items()}


def test_batch_matches_single_problem_path_and_oracle():
    """Every instance: moments within 1e-11 of the oracle; distributions within
    rounding of the single-problem kernel (the two kernels contract
    multiply-adds differently, and shock-tube runs amplify ulp differences)."""
    items, b = _batch(3, 24, riemann_n=(200, 900), couette_h=(32, 120))
    steps = 300
    b.step(steps)
    b.check()
    fb = b.get_f().cpu().numpy()
    worst = 0.0
    for i, (kind, p, fl) in enumerate(items):
        g, gf = gpu_run(p, fl, steps, variant=0)
        d = float(np.max(np.abs(b.f_of(fb, i) - gf) / np.abs(gf).max(axis=(1, 2), keepdims=True)))
        worst = max(worst, d)
        assert d <= 1e-12, (i, kind, d)
        o, _ = oracle_run(p, fl, steps)
        assert_parity(_moments_of(b, i), o, what="batch instance %d (%s, %dx%d)" % (i, kind, p["nx"], p["ny"]))
    log("batch vs single-problem kernels: max diff %.2e over %d instances" % (worst, len(items)))
    b.close()


@pytest.mark.parametrize("region,h", [(128, 8), (256, 16), (256, 32), (128, 1)])
def test_schedules_agree(region, h):
    items, b = _batch(5, 12, riemann_n=(300, 1500), couette_h=(40, 200))
    b.set_schedule(region, h)
    b.step(100)
    f = b.get_f().cpu().numpy()
    b.close()
    items, r = _batch(5, 12, riemann_n=(300, 1500), couette_h=(40, 200))
    r.set_schedule(256, 4, use_graph=False)
    r.step(100)
    ref = r.get_f().cpu().numpy()
    r.close()
    log("schedule (%d, %d) vs (256, 4): bitwise %s" % (region, h, np.array_equal(f, ref)))
    assert np.array_equal(f, ref)


def test_budgets():
    items, b = _batch(7, 10, riemann_n=(256, 700), couette_h=(32, 90))
    budgets = [17 * (i + 1) for i in range(len(items))]
    b.set_budgets(budgets)
    b.step(200)
    fb = b.get_f().cpu().numpy()
    m = {k: v.cpu().numpy() for k, v in b.moments().items()}
    for i, (kind, p, fl) in enumerate(items):
        n = min(200, budgets[i])
        _, gf = gpu_run(p, fl, n, variant=0)
        d = float(np.max(np.abs(b.f_of(fb, i) - gf) / np.abs(gf).max(axis=(1, 2), keepdims=True)))
        assert d <= 1e-12, (i, budgets[i], d)
        o, _ = oracle_run(p, fl, n)
        assert_parity({k: b.split(v, i) for k, v in m.items()}, o, what="budget %d instance %d" % (n, i))
    b.close()


def test_graph_replays_match_eager_runs():
    """The captured graph replayed several times, with eager work and
    synchronisations in between, equals the same steps without a graph."""
    import torch

    items, g = _batch(9, 16, riemann_n=(256, 1200), couette_h=(32, 150))
    items, e = _batch(9, 16, riemann_n=(256, 1200), couette_h=(32, 150))
    g.set_schedule(256, 16, use_graph=True)
    e.set_schedule(256, 16, use_graph=False)
    for rep in range(4):
        g.step(48)  # 3 launches: odd, so the graph alternates between buffers
        e.step(48)
        torch.cuda.synchronize()
        _ = torch.ones(1000, device="cuda").sum().item()  # unrelated eager work
        fg = g.get_f().cpu().numpy()
        fe = e.get_f().cpu().numpy()
        log("graph replay %d bitwise equal to eager: %s" % (rep, np.array_equal(fg, fe)))
        assert np.array_equal(fg, fe)
    g.close()
    e.close()


def test_tuner_keeps_state_and_picks_a_schedule():
    items, b = _batch(11, 20)
    f0 = b.get_f().cpu().numpy()
    s = b.tune(probe_steps=32, use_cache=False)
    log("tuner choice: %s" % s)
    f1 = b.get_f().cpu().numpy()
    assert np.array_equal(f0, f1)
    assert s["region"] in (128, 256)
    b.close()


def test_tuner_reports_an_earlier_health_error_first():
    """A step that went non-finite before the tuner is called: the tuner
    returns LBM_ENONFINITE (as lbm_batch_check would) instead of tuning and
    clearing the flag with its own trials."""
    from paper_1106_0785_amd import lbm

    items, b = _batch(12, 8)
    items[3][2]["T"][:] = -1.0
    b.init([f for _, _, f in items])
    b.step(8)
    with pytest.raises(lbm.LbmError) as err:
        b.tune(probe_steps=8, use_cache=False)
    assert err.value.status == -5
    b.close()


# ---------------------------------------------------------------------------
# Batches mixing one-dimensional lines with two-dimensional (tiled) instances.
# ---------------------------------------------------------------------------
def _mixed(seed, n):
    from paper_1106_0785_amd.batch import Batch

    items = inputs.mixed_batch(seed=seed, n=n)
    b = Batch([p for _, p, _ in items])
    b.init([f for _, _, f in items])
    return items, b


def _rel(a, b):
    return float(np.max(np.abs(a - b) / np.abs(b).max(axis=(1, 2), keepdims=True)))


def test_mixed_batch_matches_single_problem_path_and_oracle():
    """Every instance of a batch of lines, shock/interface and shock-bubble
    set-ups, Couette channels, periodic states (three equilibrium versions)
    and long periodic lines: tiled instances bitwise equal to the
    single-problem kernel (same fused step), lines within rounding of it, and
    moments of all within 1e-11 of the oracle. An odd step count leaves the
    two kinds of instance in different buffers."""
    items, b = _mixed(3, 18)
    steps = 151
    b.step(steps)
    b.check()
    fb = b.get_f().cpu().numpy()
    kinds = set()
    for i, (kind, p, fl) in enumerate(items):
        _, gf = gpu_run(p, fl, steps, variant=0)
        fi = b.f_of(fb, i)
        if p["nx"] > 1 and p["ny"] > 1 or kind == "periodic_line":
            assert np.array_equal(fi, gf), (i, kind, _rel(fi, gf))
        else:
            assert _rel(fi, gf) <= 1e-12, (i, kind)
        o, _ = oracle_run(p, fl, steps)
        assert_parity(_moments_of(b, i), o, what="mixed instance %d (%s, %dx%d)" % (i, kind, p["nx"], p["ny"]))
        kinds.add(kind)
    assert {"rm", "shock_bubble", "couette2d", "periodic2d", "periodic_line"} <= kinds
    b.close()


def test_mixed_batch_budgets():
    items, b = _mixed(8, 12)
    budgets = [13 * (i + 1) + (i % 2) for i in range(len(items))]
    b.set_budgets(budgets)
    b.step(101)
    fb = b.get_f().cpu().numpy()
    m = {k: v.cpu().numpy() for k, v in b.moments().items()}
    for i, (kind, p, fl) in enumerate(items):
        n = min(101, budgets[i])
        _, gf = gpu_run(p, fl, n, variant=0)
        assert _rel(b.f_of(fb, i), gf) <= 1e-12, (i, kind, budgets[i])
        o, _ = oracle_run(p, fl, n)
        assert_parity({k: b.split(v, i) for k, v in m.items()}, o, what="budget %d mixed instance %d" % (n, i))
    b.close()


def test_mixed_graph_replays_match_eager_runs():
    import torch

    items, g = _mixed(9, 12)
    items, e = _mixed(9, 12)
    g.set_schedule(256, 16, use_graph=True)
    e.set_schedule(256, 16, use_graph=False)
    for rep, k in enumerate((47, 47, 30, 47)):
        g.step(k)
        e.step(k)
        torch.cuda.synchronize()
        _ = torch.ones(1000, device="cuda").sum().item()
        fg = g.get_f().cpu().numpy()
        fe = e.get_f().cpu().numpy()
        log("mixed graph replay %d (%d steps) bitwise equal to eager: %s" % (rep, k, np.array_equal(fg, fe)))
        assert np.array_equal(fg, fe)
    g.close()
    e.close()


def test_mixed_tuner_keeps_state():
    items, b = _mixed(11, 12)
    b.step(17)  # two line launches (h = 16), 17 tile steps: the kinds end in different buffers
    f0 = b.get_f().cpu().numpy()
    s = b.tune(probe_steps=16, use_cache=False)
    f1 = b.get_f().cpu().numpy()
    assert np.array_equal(f0, f1), s
    b.step(5)
    items2, r = _mixed(11, 12)
    r.step(17)
    t = b.two_step()
    r.set_two_step(t["two_step"], t["tile_rows2"])  # the plain 2-D instances as the tuner left them
    r.step(5)
    assert np.array_equal(b.get_f().cpu().numpy(), r.get_f().cpu().numpy())
    b.close()
    r.close()


@pytest.mark.parametrize("rows", [4, 8, 64, 128])
def test_mixed_tile_heights_agree(rows):
    """Tile height of the tiled instances changes the work split, not the
    result (bitwise), also with budgets."""
    items, b = _mixed(13, 12)
    items, r = _mixed(13, 12)
    budgets = [7 * (i + 2) for i in range(len(items))]
    b.set_budgets(budgets)
    r.set_budgets(budgets)
    b.set_tile_rows(rows)
    info = b.tile_rows()
    assert info["tile_rows"] == rows and info["tiles"] > 0
    b.step(61)
    r.step(61)
    f, ref = b.get_f().cpu().numpy(), r.get_f().cpu().numpy()
    log("tile rows %d (%d tiles) vs default %s: bitwise %s" % (rows, info["tiles"], r.tile_rows(), np.array_equal(f, ref)))
    assert np.array_equal(f, ref)
    b.close()
    r.close()


def test_batch_with_the_flux_limited_scheme():
    """Instances with the flux-limited scheme (2-D set-ups and lines, which
    then run tile by tile) beside Lax-Wendroff ones: bitwise equal to the
    single-problem path, and within 1e-11 of the oracle."""
    from paper_1106_0785_amd.batch import Batch

    items = inputs.mixed_batch(seed=4, n=12)
    for i, (kind, p, fl) in enumerate(items):
        if "neq_wall" not in p["bc"] and (i % 2 == 1 or i == 0):
            p["scheme"] = 1
    assert sum(p.get("scheme", 0) for _, p, _ in items) >= 4
    b = Batch([p for _, p, _ in items])
    b.init([f for _, _, f in items])
    b.step(61)
    b.check()
    fb = b.get_f().cpu().numpy()
    m = {k: v.cpu().numpy() for k, v in b.moments().items()}
    for i, (kind, p, fl) in enumerate(items):
        _, gf = gpu_run(p, fl, 61, variant=0)
        fi = b.f_of(fb, i)
        if p.get("scheme", 0) == 1 or (p["nx"] > 1 and p["ny"] > 1) or kind == "periodic_line":
            assert np.array_equal(fi, gf), (i, kind, p.get("scheme", 0), _rel(fi, gf))
        else:
            assert _rel(fi, gf) <= 1e-12, (i, kind)
        o, _ = oracle_run(p, fl, 61)
        assert_parity({k: b.split(v, i) for k, v in m.items()}, o,
                      what="batch instance %d (%s, scheme %d)" % (i, kind, p.get("scheme", 0)))
    b.close()


@pytest.mark.parametrize("region,h", [(128, 16), (256, 16), (128, 8)])
def test_wall_lines_whose_last_chunk_would_be_one_node(region, h):
    """Couette columns longer than a line region, with lengths N = k C + 1
    (C = region - 2 h nodes per chunk), so that plain chunking would leave
    the wall node alone in the last chunk: the chunk that writes the wall
    also writes its fluid neighbour, whose value the wall takes in the same
    step. Against the oracle after a number of steps that is not a
    multiple of h."""
    from paper_1106_0785_amd.batch import Batch

    C = region - 2 * h
    items = []
    for k, pr in ((1, 0.7), (2, 1.5)):
        p, fl, _ = inputs.couette(pr, nx=1, ny=k * C + 1)
        items.append((p, fl))
    p, fl, _ = inputs.riemann("sod", Pr=1.0, nx=k * C + 1, ny=1)
    items.append((p, fl))
    b = Batch([p for p, _ in items])
    b.init([f for _, f in items])
    b.set_schedule(region, h)
    steps = 5 * h + 3
    b.step(steps)
    b.check()
    for i, (p, fl) in enumerate(items):
        o, _ = oracle_run(p, fl, steps)
        assert_parity(_moments_of(b, i), o, what="wall line %d (N = %d), schedule (%d, %d)" % (i, p["nx"] * p["ny"], region, h))
    b.close()


def test_random_batches():
    """8 seeded random batches: Couette columns and channels (NEQ walls,
    some longer than a line region), Riemann lines, periodic lines and 2-D
    states, with a random line schedule, tile height, step count and
    per-instance budgets; every instance against the oracle."""
    from paper_1106_0785_amd import lbm
    from paper_1106_0785_amd.batch import Batch

    rng = np.random.default_rng(99)
    for trial in range(8):
        items = []
        for _ in range(int(rng.integers(2, 9))):
            kind = int(rng.integers(0, 5))
            if kind == 0:
                p, fl, _ = inputs.couette(float(rng.uniform(0.4, 2.5)), nx=1, ny=int(rng.integers(3, 600)))
            elif kind == 1:
                p, fl, _ = inputs.couette_x(float(rng.uniform(0.4, 2.5)), nx=int(rng.integers(3, 600)), ny=1)
            elif kind == 2:
                p, fl, _ = inputs.riemann("sod", Pr=1.0, nx=int(rng.integers(16, 700)), ny=1)
            elif kind == 3:
                p, fl = inputs.smooth_periodic(seed=int(rng.integers(0, 10 ** 6)), nx=int(rng.integers(2, 300)), ny=1,
                                               amp=0.05)
            else:
                p, fl = inputs.smooth_periodic(seed=int(rng.integers(0, 10 ** 6)), nx=int(rng.integers(2, 70)),
                                               ny=int(rng.integers(3, 40)), amp=0.05, eq_version=int(rng.integers(1, 4)))
            if lbm.lbm_workspace_bytes(p) > 0:
                items.append((p, fl))
        b = Batch([p for p, _ in items])
        b.init([f for _, f in items])
        region = int(rng.choice([128, 256]))
        h = int(rng.choice([4, 8, 16, 32]))
        b.set_schedule(region, h)
        b.set_tile_rows(int(rng.choice([4, 16, 64])))
        steps = int(rng.integers(1, 100))
        budgets = [int(rng.integers(0, steps + 5)) for _ in items] if rng.random() < 0.5 else None
        if budgets:
            b.set_budgets(budgets)
        b.step(steps)
        b.check()
        m = {k: v.cpu().numpy() for k, v in b.moments().items()}
        for i, (p, fl) in enumerate(items):
            n = steps if budgets is None else min(steps, budgets[i])
            o, _ = oracle_run(p, fl, n)
            assert_parity({k: b.split(v, i) for k, v in m.items()}, o,
                          what="random batch %d instance %d (%dx%d, %s), schedule (%d, %d), %d steps"
                          % (trial, i, p["nx"], p["ny"], p["bc"][0], region, h, n))
        b.close()


def test_library_loaded_before_any_tensor():
    """A process whose first call into the library is a host-only one (the
    workspace size) and that creates tensors only afterwards: the binding
    loads PyTorch's HIP runtime before the library, so both share one
    runtime and the batch runs. Run in a fresh process, where nothing has
    imported PyTorch yet."""
    import os
    import subprocess
    import sys

    root = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
    script = (
        "import sys; sys.path.insert(0, %r)\n"
        "from paper_1106_0785_amd import inputs, lbm\n"
        "p, fl, _ = inputs.couette(1.0, nx=1, ny=300)\n"
        "assert lbm.lbm_workspace_bytes(p) > 0\n"
        "from paper_1106_0785_amd.batch import Batch\n"
        "b = Batch([p]); b.init([fl]); b.step(10); b.check(); b.close()\n"
        "print('ok')\n" % root)
    r = subprocess.run([sys.executable, "-c", script], capture_output=True, text=True, timeout=100)
    log("fresh process: rc %d, %s" % (r.returncode, (r.stdout + r.stderr).strip()[-300:]))
    assert r.returncode == 0 and "ok" in r.stdout
