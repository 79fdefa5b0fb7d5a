"""Shocked-flow pins of the oracle (Sec. IV.B(a)): one-dimensional Riemann
problems against the exact solution of the gamma = 2 gas, and the paper's
observation that the modification hardly matters under shocks.

The initial jumps are smoothed over three cells (the central Lax-Wendroff
stencil needs it); the L1 bound reflects the viscous smearing of the shock
and contact over a few cells at 2000 nodes.
"""

import numpy as np
import pytest

import oracle
from paper_1106_0785_amd import inputs
from physics import riemann_sample


def _l1(a, b):
    return np.abs(a - b).sum() / np.abs(b).sum()


def _run(kind, Pr, steps, modified=1):
    p, f, meta = inputs.riemann(kind, Pr=Pr, nx=2000, ny=1, modified=modified)
    m = oracle.moments(p, oracle.run(p, oracle.init(p, **f), steps))
    t = steps * p["dt"]
    r, u, pr = riemann_sample(meta["left"], meta["right"], (meta["x"] - meta["x0"]) / t)
    return m, (r, u, pr)


@pytest.mark.parametrize("kind,steps,bound", [("sod", 20000, 0.008), ("lax", 14000, 0.015)])
def test_riemann_matches_gamma2_exact_solution(kind, steps, bound):
    m, (r, u, pr) = _run(kind, 1.0, steps)
    assert _l1(m["rho"][0], r) < bound
    assert _l1(m["ux"][0], u) < bound
    assert _l1(m["p"][0], pr) < bound
    # a gamma = 1.4 solution is far off: the gas really has gamma = 2
    r14, _, _ = riemann_sample(inputs.RIEMANN_STATES[kind][0], inputs.RIEMANN_STATES[kind][1],
                               (np.arange(2000) + 0.5) / 2000 / (steps * 1e-5) - 0.5 / (steps * 1e-5), g=1.4)
    assert _l1(m["rho"][0], r14) > 3 * bound


def test_modification_negligible_under_shock():
    """Sec. IV.B(a): modified and unmodified results hardly differ."""
    m1, ex = _run("sod", 2.0, 20000, modified=1)
    m0, _ = _run("sod", 2.0, 20000, modified=0)
    assert _l1(m1["rho"][0], m0["rho"][0]) < 0.1 * 0.008
    assert abs(_l1(m1["rho"][0], ex[0]) - _l1(m0["rho"][0], ex[0])) < 0.002
