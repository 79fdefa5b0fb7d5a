"""Parity at the full sizes of the measured workloads, in the launch
configuration the benchmark times (tile shape or schedule picked by the
tuners), against the oracle:

  * the 4096 x 1024 shock/interface problem (the HBM-resident step), every
    node after a few steps;
  * the 1024 x 256 shock/interface configuration for its full 5000 steps;
  * the same configuration at the fast end of its Mach range (seed 4:
    Mach 1.95, four interface modes) for its full 5000 steps;
  * the 512-instance uneven batch for 1000 steps, every instance;
  * the adjoint of 2000 steps at 512 x 128, against the oracle's complex-step
    directional derivative (exact up to rounding).
"""

import numpy as np
import pytest

import oracle
from gpu_util import assert_parity, log, oracle_run
from paper_1106_0785_amd import inputs

pytestmark = pytest.mark.gpu


def _tuned_run(p, fl, steps):
    from paper_1106_0785_amd import lbm

    sim = lbm.Simulation(p)
    sim.init(**fl)
    tile = sim.tune(probe_steps=4)
    # the kernel and shape the tuner kept
    shape = ("window", sim.window()) if sim.variant() == 3 else ("tile", tile[:2])
    sim.step(steps)
    out = {k: v.cpu().numpy() for k, v in sim.moments().items()}
    sim.check()
    sim.close()
    return out, shape


def test_headline_size_every_node():
    p, fl, _ = inputs.rm(seed=0, nx=4096, ny=1024)
    g, shape = _tuned_run(p, fl, 6)
    o, _ = oracle_run(p, fl, 6)
    log("4096x1024, tuned %s %s, 6 steps" % shape)
    assert_parity(g, o, what="rm 4096x1024 6 steps")


def test_rm_1024x256_full_run():
    p, fl, _ = inputs.rm(seed=0, nx=1024, ny=256)
    g, shape = _tuned_run(p, fl, 5000)
    o, _ = oracle_run(p, fl, 5000)
    log("1024x256, tuned %s %s, 5000 steps" % shape)
    assert_parity(g, o, what="rm 1024x256 5000 steps")


def test_rm_1024x256_fast_shock_full_run():
    p, fl, meta = inputs.rm(seed=4, nx=1024, ny=256)
    assert meta["mach"] > 1.9 and meta["K"] == 4
    g, shape = _tuned_run(p, fl, 5000)
    o, _ = oracle_run(p, fl, 5000)
    log("1024x256 Mach %.3f, %d modes, tuned %s %s, 5000 steps" % (meta["mach"], meta["K"], shape[0], shape[1]))
    assert_parity(g, o, what="rm 1024x256 seed 4 5000 steps")


def _oracle_instances(items, steps):
    """Oracle results of every instance, one thread each, instances in
    parallel (the oracle's foreign calls release the interpreter lock)."""
    import os
    from concurrent.futures import ThreadPoolExecutor

    def one(item):
        _, p, fl = item
        return oracle.moments(p, oracle.run(p, oracle.init(p, **fl), steps, nthreads=1))

    with ThreadPoolExecutor(max_workers=min(16, os.cpu_count() or 1)) as ex:
        return list(ex.map(one, items))


def test_batch_512_every_instance():
    from paper_1106_0785_amd.batch import Batch

    items = inputs.batch(seed=0, n=512)
    b = Batch([p for _, p, _ in items])
    b.init([f for _, _, f in items])
    sched = b.tune(probe_steps=32, use_cache=False)
    b.step(1000)
    b.check()
    m = {k: v.cpu().numpy() for k, v in b.moments().items()}
    b_split = [{k: b.split(v, i) for k, v in m.items()} for i in range(len(items))]
    b.close()
    log("batch512: 1000 steps, schedule %s; oracle on every instance" % (sched,))
    refs = _oracle_instances(items, 1000)
    for i, ((kind, p, _), o) in enumerate(zip(items, refs)):
        assert_parity(b_split[i], o, what="batch512 instance %d (%s, %dx%d)" % (i, kind, p["nx"], p["ny"]))


def test_adjoint_512x128_2000_steps_against_complex_step():
    import torch

    from paper_1106_0785_amd.autograd import Adjoint

    nx, ny, steps = 512, 128, 2000
    p, fl, _ = inputs.rm(seed=0, nx=nx, ny=ny)
    rng = np.random.default_rng(21)
    w = rng.standard_normal((ny, nx))
    d_fields = [1e-3 * rng.standard_normal((ny, nx)) for _ in range(4)]
    d_logs = rng.standard_normal(16)
    a = Adjoint(p, steps)
    f0 = [torch.from_numpy(np.ascontiguousarray(fl[k])).cuda() for k in ("rho", "ux", "uy", "T")]
    a.forward(*f0)
    grads, gs = a.backward(torch.from_numpy(w).cuda(), None, None, None)
    grads = [g.cpu().numpy() for g in grads]
    gs = gs.cpu().numpy()
    a.close()
    s = np.array(p["s"])
    got = sum(float(np.sum(g * d)) for g, d in zip(grads, d_fields)) + float(np.sum(gs * s * d_logs))
    h = 1e-30
    keys = ("rho", "ux", "uy", "T")
    cf = {k: fl[k] + 1j * h * d for k, d in zip(keys, d_fields)}
    f = oracle.init_complex(p, cf["rho"], cf["ux"], cf["uy"], cf["T"])
    f = oracle.run_complex(p, f, steps, s_im=h * s * d_logs)
    ref = float(np.sum(w * oracle.moments_complex(p, f)["rho"].imag)) / h
    rel = abs(got - ref) / abs(ref)
    log("adjoint 512x128x2000 vs oracle complex step: %.6e vs %.6e, rel %.2e" % (got, ref, rel))
    # both are exact derivatives of the step as each side rounds it (measured
    # 9e-13 apart after 2000 steps); the bound leaves room for the growth of
    # rounding differences along the shocked trajectory
    assert rel <= 1e-10


def test_grid_beyond_32_bit_offsets():
    """A periodic 64 x 40 field tiled 257 x 410 times (16448 x 16400 nodes,
    16 planes = 4.3e9 doubles per buffer, past 2^32 elements; 69 GB of
    distributions): by translation invariance every node after 3 steps
    equals the node of the 64 x 40 problem run alone, which matches the
    oracle."""
    import torch

    from paper_1106_0785_amd import lbm

    p, fl = inputs.smooth_periodic(seed=17, nx=64, ny=40, amp=0.07)
    steps = 3
    small = lbm.Simulation(p)
    small.init(**fl)
    small.step(steps)
    gs = {k: v.cpu().numpy() for k, v in small.moments().items()}
    small.check()
    small.close()
    o, _ = oracle_run(p, fl, steps)
    assert_parity(gs, o, what="64x40 tile")

    rx, ry = 257, 410
    big = dict(p, nx=64 * rx, ny=40 * ry)
    log("16448 x 16400 tiled periodic grid: %d steps" % steps)
    sim = lbm.Simulation(big)
    sim.init(**{k: torch.from_numpy(np.tile(v, (ry, rx))) for k, v in fl.items()})
    sim.step(steps)
    m = sim.moments()
    sim.check()
    for k in ("rho", "ux", "uy", "T", "p"):
        got = m[k].cpu().numpy().reshape(ry, 40, rx, 64)
        same = bool(np.array_equal(got, np.broadcast_to(gs[k][None, :, None, :], got.shape)))
        log("  %s: every node equals its tile node: %s" % (k, same))
        assert same, k
    del m
    sim.close()
    torch.cuda.empty_cache()


def test_sod_2000x4_tuned_full_run():
    """The 2000 x 4 Sod tube for its full 20 000 steps in the kernel and
    shape the tuner picks (the benchmark's configuration: windows of all
    rows, several steps per launch); the oracle runs the y-uniform problem
    on one row."""
    p, fl, _ = inputs.riemann("sod", Pr=1.0, nx=2000, ny=4)
    g, shape = _tuned_run(p, fl, 20000)
    p1, fl1, _ = inputs.riemann("sod", Pr=1.0, nx=2000, ny=1)
    o, _ = oracle_run(p1, fl1, 20000)
    log("sod 2000x4, tuned %s %s, 20000 steps" % shape)
    for j in range(4):
        assert_parity({k: v[j:j + 1] for k, v in g.items()}, o, what="sod 2000x4 row %d" % j)


def test_limited_scheme_headline_size_every_node():
    """The flux-limited scheme on the 4096 x 1024 sharp-interface problem
    (the benchmark's side measurement), tuned tile, every node after 4
    steps."""
    p, fl, _ = inputs.rm(seed=0, nx=4096, ny=1024, width_cells=0.5)
    p["scheme"] = 1
    g, shape = _tuned_run(p, fl, 4)
    o, _ = oracle_run(p, fl, 4)
    log("limited 4096x1024, tuned %s %s, 4 steps" % shape)
    assert_parity(g, o, what="limited 4096x1024 4 steps")
