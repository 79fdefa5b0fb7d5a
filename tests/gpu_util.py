"""Helpers of the GPU parity tests: run the HIP path and the oracle on the
same seeded inputs and compare per moment field.

Tolerance (per field, after the stated number of steps): for rho, T and p
the max over cells of |g - o|/|o|; for u_x and u_y the max of |g - o|
divided by the max over cells of sqrt(u_x^2 + u_y^2 + 2T) (velocity scaled by
the flow's speed plus sound speed, so near-zero components do not divide by
zero). Both sides are FP64; they differ only in rounding order (structured vs
dense transforms, fused multiply-adds), which grows roughly linearly with the
number of steps.
"""

import sys

import numpy as np

import oracle

TOL = 1e-11


def log(msg):
    print(msg, flush=True)
    sys.stdout.flush()


def gpu_run(p, fields, steps, variant=None, rows=None, waves=None):
    """Runs the HIP path. variant None keeps the library's default kernel,
    except that a tile shape (rows, waves) selects the fused kernel."""
    from paper_1106_0785_amd import lbm

    sim = lbm.Simulation(p)
    if variant is None and (rows or waves):
        variant = 0
    if variant is not None:
        sim.set_variant(variant)
    if rows or waves:
        sim.set_tile(rows or 16, waves or 4)
    sim.init(**fields)
    sim.step(steps)
    out = {k: v.cpu().numpy() for k, v in sim.moments().items()}
    f = sim.get_f().cpu().numpy()
    sim.check()
    sim.close()
    return out, f


def oracle_run(p, fields, steps):
    f = oracle.run(p, oracle.init(p, **fields), steps)
    return oracle.moments(p, f), f


def field_errors(g, o):
    scale_u = np.max(np.sqrt(o["ux"] ** 2 + o["uy"] ** 2 + 2.0 * o["T"]))
    e = {}
    for k in ("rho", "T", "p"):
        e[k] = float(np.max(np.abs(g[k] - o[k]) / np.abs(o[k])))
    for k in ("ux", "uy"):
        e[k] = float(np.max(np.abs(g[k] - o[k])) / scale_u)
    return e


def assert_parity(g, o, tol=TOL, what=""):
    e = field_errors(g, o)
    log("%s max rel errors: %s" % (what, ", ".join("%s %.2e" % kv for kv in e.items())))
    bad = {k: v for k, v in e.items() if not (v <= tol)}
    assert not bad, (what, bad)
