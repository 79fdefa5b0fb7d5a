"""Pins of the synthetic workload generators against values the paper prints.

  * Sec. IV.B(b): a Mach 1.22 shock (D = 1.725) into (rho, u, p) = (1, 0, 1)
    leaves (1.28, -0.3774, 1.6512) behind it; this holds for gamma = 2.
  * Sec. III and IV.B(a): Ma = u / sqrt(2 T), e.g. 45/sqrt(20) = 10.1.
"""

import json
import math
import os

import numpy as np

from paper_1106_0785_amd import inputs
from physics import rankine_hugoniot

GOLD = os.path.join(os.path.dirname(__file__), "golden")


def test_post_shock_state_matches_paper():
    g = json.load(open(os.path.join(GOLD, "rm_post_shock.json")))
    rho2, du, p2, D = inputs.post_shock(g["mach"], g["pre"][0], g["pre"][3])
    assert abs(D - g["D"]) < 5e-4
    assert abs(rho2 - g["post"][0]) < 5e-3
    assert abs(-du - g["post"][1]) < 5e-5
    assert abs(p2 - g["post"][3]) < 5e-5
    # the generator agrees with an independent textbook jump relation
    r, u, p, d = rankine_hugoniot(g["mach"], 1.0, 1.0)
    assert abs(r - rho2) < 1e-12 and abs(u - du) < 1e-12 and abs(p - p2) < 1e-12 and abs(d - D) < 1e-12


def test_mach_numbers_match_paper():
    g = json.load(open(os.path.join(GOLD, "mach_numbers.json")))
    for c in g["cases"]:
        ma = abs(c["u"]) / math.sqrt(inputs.GAMMA * c["T"])
        assert abs(ma - c["Ma"]) <= 0.051 * max(1.0, c["Ma"] / 10), c


def test_generators_are_seeded_and_shaped():
    p1, f1, m1 = inputs.rm(seed=3, nx=128, ny=32)
    p2, f2, m2 = inputs.rm(seed=3, nx=128, ny=32)
    for k in f1:
        assert f1[k].shape == (32, 128)
        np.testing.assert_array_equal(f1[k], f2[k])
    assert 1.2 <= m1["mach"] <= 2.0 and 1 <= m1["K"] <= 4
    # shock sits in the light gas, left of the whole interface
    assert m1["shock_cells"] < m1["x0_cells"] - np.max(np.abs(m1["a"]))
    b = inputs.batch(seed=0, n=64)
    assert len(b) == 64
    for kind, p, f in b:
        assert f["rho"].shape == (p["ny"], p["nx"])
        assert max(p["s"]) * p["dt"] <= 1.0 + 1e-12
        if kind == "riemann":
            assert p["ny"] == 1 and 256 <= p["nx"] <= 4096
        else:
            assert p["nx"] == 1 and 32 <= p["ny"] <= 256


def test_rm_fields_torch_matches_numpy():
    """The differentiable (torch) form of the shock/interface generator gives
    the same fields as the numpy form, on the device of its argument."""
    import torch

    p, f, m = inputs.rm(seed=4, nx=64, ny=16)
    a = torch.tensor(m["a"], dtype=torch.float64)
    g = inputs.rm_fields(64, 16, a, m["mach"], m["heavy"], m["x0_cells"], m["shock_cells"], m["width_cells"],
                         m["wall_ramp_cells"], xp=torch)
    for k in f:
        assert g[k].device == a.device
        np.testing.assert_allclose(g[k].numpy(), f[k], rtol=0, atol=1e-14)


def test_shock_bubble_states_match_paper():
    """Sec. IV.B(b): the shock-bubble set-up's pre-shock, post-shock and
    bubble states, the inflow state on the right side and the positions
    (post-shock region x >= 5/6 of the domain, bubble at 3/4 of the length
    and mid height)."""
    g = json.load(open(os.path.join(GOLD, "rm_post_shock.json")))
    p, f, m = inputs.shock_bubble(nx=600, ny=100)
    rho, ux, T = f["rho"], f["ux"], f["T"]
    pr = rho * T
    # far right: post-shock state; also the fixed inflow state of the x_hi side
    post = [rho[50, 599], ux[50, 599], 0.0, pr[50, 599]]
    for got, want, tol in zip(post, g["post"], (5e-3, 5e-5, 0, 5e-5)):
        assert abs(got - want) <= tol
    w = p["wall"][1]
    assert abs(w[0] - rho[50, 599]) < 1e-12 and abs(w[1] - ux[50, 599]) < 1e-12 and abs(w[3] - T[50, 599]) < 1e-12
    assert p["bc"] == ["zero_gradient", "dirichlet_eq", "specular", "specular"]
    # far left: gas at rest; bubble centre: the light gas at the same pressure
    assert abs(rho[50, 0] - g["pre"][0]) < 1e-12 and abs(pr[50, 0] - g["pre"][3]) < 1e-12 and ux[50, 0] == 0.0
    assert abs(rho[49, 449] - g["bubble"][0]) < 1e-5 and abs(pr[49, 449] - g["bubble"][3]) < 1e-5
    # the shock sits between nodes 499 and 500 (the paper's 1-based [501, 600])
    assert rho[10, 497] < 1.05 and rho[10, 502] > 1.23
    assert m["radius"] == 20.0 and m["center"] == (449.0, 49.5)


def test_mixed_and_2d_batches_are_seeded_and_shaped():
    a = inputs.mixed_batch(seed=5, n=12)
    b = inputs.mixed_batch(seed=5, n=12)
    kinds = set()
    for (ka, pa, fa), (kb, pb, fb) in zip(a, b):
        assert ka == kb and pa == pb
        for k in fa:
            assert fa[k].shape == (pa["ny"], pa["nx"])
            np.testing.assert_array_equal(fa[k], fb[k])
        assert max(pa["s"]) * pa["dt"] <= 1.0 + 1e-12
        kinds.add(ka)
    assert {"rm", "shock_bubble", "couette2d", "periodic2d", "periodic_line"} <= kinds
    assert {p["eq_version"] for _, p, _ in inputs.mixed_batch(seed=1, n=36)} == {1, 2, 3}
    r = inputs.rm_batch(seed=0, n=8)
    for kind, p, f in r:
        assert 128 <= p["nx"] <= 512 and 32 <= p["ny"] <= 128 and f["rho"].shape == (p["ny"], p["nx"])
