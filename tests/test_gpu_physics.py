"""Trends the paper reports for the shock-bubble runs (Sec. IV.B(b),
Figs. 7-8), on the full 600 x 100 set-up at the three snapshot times of the
figures, t = 0.5, 0.7 and 1: at fixed viscosity a smaller thermal
conductivity (larger s7 = s8), and at fixed conductivity a smaller viscosity
(larger s5 = s6), leave the flow less smoothed (the paper: both favour the
development of the instability). The measure is the total variation of the
density field. The paper also finds the modified and the unmodified model
give the same picture. Parity for these trends is unpinned (the paper prints
no values); the GPU path itself is checked against the oracle on the same
set-up in test_gpu_parity.py."""

import numpy as np
import pytest

from gpu_util import log
from paper_1106_0785_amd import inputs

pytestmark = pytest.mark.gpu

DT = 1e-5
TIMES = (0.5, 0.7, 1.0)


def _run(s5, s7, modified=1):
    """Density at each snapshot time of TIMES."""
    from paper_1106_0785_amd import lbm

    p, fl, _ = inputs.shock_bubble(s5=s5, s7=s7, modified=modified)
    assert p["dt"] == DT
    sim = lbm.Simulation(p)
    sim.init(**fl)
    out, done = {}, 0
    for t in TIMES:
        n = int(round(t / DT))
        sim.step(n - done)
        done = n
        out[t] = sim.moments()["rho"].cpu().numpy()
    sim.check()
    sim.close()
    return out


def _tv(rho):
    return float(np.abs(np.diff(rho, axis=0)).sum() + np.abs(np.diff(rho, axis=1)).sum())


def test_conductivity_and_viscosity_trends():
    tv = {}
    for s5 in (1e4, 1e3):
        for s7 in (1e5, 1e4, 1e3):
            rho = _run(s5, s7)
            for t in TIMES:
                tv[(t, s5, s7)] = _tv(rho[t])
            log("shock-bubble s5=%g s7=%g: total variation of rho at t=0.5/0.7/1: %s"
                % (s5, s7, " ".join("%.4f" % tv[(t, s5, s7)] for t in TIMES)))
    for t in TIMES:
        for s5 in (1e4, 1e3):  # Figs. 7 and 8 across: conductivity at fixed viscosity
            assert tv[(t, s5, 1e5)] > tv[(t, s5, 1e4)] > tv[(t, s5, 1e3)], (t, s5)
        for s7 in (1e5, 1e4, 1e3):  # Fig. 7 against Fig. 8: viscosity at fixed conductivity
            assert tv[(t, 1e4, s7)] > tv[(t, 1e3, s7)], (t, s7)


def test_modified_and_unmodified_agree_under_shock():
    a = _run(1e4, 1e5, modified=1)
    b = _run(1e4, 1e5, modified=0)
    for t in TIMES:
        d = float(np.linalg.norm(a[t] - b[t]) / np.linalg.norm(a[t]))
        log("shock-bubble t=%g s5=1e4 s7=1e5: modified vs unmodified relative L2 difference of rho %.2e" % (t, d))
        assert d < 0.05, t
