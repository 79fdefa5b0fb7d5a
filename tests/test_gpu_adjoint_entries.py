"""Single components of the adjoint's gradient against the oracle's
complex-step derivative (exact up to rounding), one component per oracle run:

  * each of the 16 dL/dlog s_k on every boundary/model variant of the small
    problems (s_1..s_4 act on conserved moments: exactly 0 on both sides);
  * dL/d(initial rho, u_x, u_y, T) at single nodes of a problem whose four
    sides are four different boundary kinds (fixed-state ghost, specular
    mirror, non-equilibrium extrapolation wall, zero-gradient ghost):
    interior nodes, nodes on and next to each side, and the four corners.

A directional check (a random projection of the whole gradient) could hide
an error in a component that carries little weight in the projection; these
compare every rate and the boundary nodes one at a time.
"""

import numpy as np
import pytest

import oracle
from gpu_util import log
from paper_1106_0785_amd import inputs
from test_gpu_adjoint import CASES

pytestmark = pytest.mark.gpu

NX, NY, STEPS, CKPT = 23, 17, 40, 7
H = 1e-30
KEYS = ("rho", "ux", "uy", "T")


def _setup(bc, **kw):
    p, fl = inputs.smooth_periodic(seed=13, nx=NX, ny=NY, amp=0.06, **kw)
    p["bc"] = bc
    p["wall"][0] = [1.03, 0.02, 0.0, 1.01]
    p["wall"][1] = [1.0, 0.0, 0.05, 1.04]
    p["wall"][2] = [1.0, -0.03, 0.0, 0.97]
    p["wall"][3] = [1.0, 0.06, 0.0, 1.02]
    p["s"][4], p["s"][5], p["s"][6], p["s"][7] = 700.0, 900.0, 1200.0, 1500.0
    rng = np.random.default_rng(1)
    w_rho = rng.standard_normal((NY, NX))
    w_T = rng.standard_normal((NY, NX))
    return p, fl, w_rho, w_T


def _adjoint(p, fl, w_rho, w_T):
    """Full gradient from the library: dL/d(rho0, ux0, uy0, T0) and dL/dlog s."""
    import torch

    from paper_1106_0785_amd.autograd import Adjoint

    a = Adjoint(p, STEPS, CKPT)
    a.forward(*[torch.from_numpy(np.ascontiguousarray(fl[k])).cuda() for k in KEYS])
    grads, gs = a.backward(torch.from_numpy(w_rho).cuda(), None, None, torch.from_numpy(w_T).cuda())
    a.close()
    return [g.cpu().numpy() for g in grads], gs.cpu().numpy() * np.array(p["s"])


def _complex_step(p, fl, w_rho, w_T, field=None, node=None, rate=None):
    """Oracle derivative of L = sum(w_rho rho_T) + sum(w_T T_T) along one
    unit direction: initial field `field` at node (y, x), or log s_rate."""
    cf = {k: fl[k].astype(np.complex128) for k in KEYS}
    if field is not None:
        cf[field][node] += 1j * H
    s_im = np.zeros(16)
    if rate is not None:
        s_im[rate] = H * p["s"][rate]
    f = oracle.init_complex(p, cf["rho"], cf["ux"], cf["uy"], cf["T"])
    f = oracle.run_complex(p, f, STEPS, s_im=s_im)
    m = oracle.moments_complex(p, f)
    return float(np.sum(w_rho * m["rho"].imag) + np.sum(w_T * m["T"].imag)) / H


MIXED = ["dirichlet_eq", "specular", "neq_wall", "zero_gradient"]
CASES_ALL = dict(CASES, mixed_sides=(MIXED, {}))


@pytest.mark.parametrize("name", sorted(CASES_ALL))
def test_each_rate_against_complex_step(name):
    bc, kw = CASES_ALL[name]
    p, fl, w_rho, w_T = _setup(bc, **kw)
    _, g = _adjoint(p, fl, w_rho, w_T)
    worst = 0.0
    for k in range(16):
        ref = _complex_step(p, fl, w_rho, w_T, rate=k)
        if k < 4:
            assert g[k] == 0.0 and ref == 0.0, (k, g[k], ref)
            continue
        rel = abs(g[k] - ref) / abs(ref)
        log("%s: dL/dlog s_%d adjoint %+.12e complex step %+.12e rel %.1e" % (name, k + 1, g[k], ref, rel))
        worst = max(worst, rel)
        assert rel <= 1e-9, (name, k + 1, g[k], ref, rel)
    log("%s: every dL/dlog s_k within %.1e" % (name, worst))


# (field, (y, x)) on the 23 x 17 problem with sides x_lo fixed state,
# x_hi specular, y_lo NEQ wall (row 0 is the wall row), y_hi zero gradient
ENTRIES = [
    ("rho", (8, 11)), ("T", (8, 11)), ("ux", (3, 5)), ("uy", (13, 17)),
    ("rho", (8, 0)), ("ux", (8, 0)), ("T", (9, 1)),                     # fixed-state side and next to it
    ("uy", (8, 22)), ("ux", (6, 22)), ("rho", (10, 21)),                # specular side and next to it
    ("rho", (0, 10)), ("T", (0, 10)), ("ux", (1, 10)), ("uy", (1, 4)),  # wall row and the fluid row above it
    ("T", (16, 10)), ("uy", (16, 12)), ("rho", (15, 10)),               # zero-gradient side and next to it
    ("rho", (0, 0)), ("T", (0, 22)), ("ux", (16, 0)), ("uy", (16, 22)),  # corners
    ("T", (1, 0)), ("rho", (15, 22)), ("ux", (1, 21)),                  # next to corners
]


def test_single_field_entries_against_complex_step():
    p, fl, w_rho, w_T = _setup(MIXED)
    grads, _ = _adjoint(p, fl, w_rho, w_T)
    worst = 0.0
    for field, node in ENTRIES:
        got = grads[KEYS.index(field)][node]
        ref = _complex_step(p, fl, w_rho, w_T, field=field, node=node)
        rel = abs(got - ref) / abs(ref)
        log("dL/d%s0%s adjoint %+.12e complex step %+.12e rel %.1e" % (field, node, got, ref, rel))
        worst = max(worst, rel)
        assert rel <= 1e-9, (field, node, got, ref, rel)
    log("%d single entries: worst rel %.1e" % (len(ENTRIES), worst))
