"""The oracle's complex-step mode (the reference for adjoint gradients) agrees
with real-arithmetic central differences of the same oracle.

Every operation of the step is analytic in f and s, so Im L(x + i h d)/h is the
exact directional derivative up to O(h^2) with no cancellation.
"""

import numpy as np

import oracle
from paper_1106_0785_amd import inputs


def _loss_real(p, fields, steps, target):
    f = oracle.run(p, oracle.init(p, **fields), steps)
    rho = oracle.moments(p, f)["rho"]
    return 0.5 * np.sum((rho - target) ** 2)


def test_complex_step_matches_central_differences():
    p, fl = inputs.smooth_periodic(seed=21, nx=12, ny=10, amp=0.06)
    p["bc"] = ["specular", "specular", "periodic", "periodic"]
    steps = 40
    rng = np.random.default_rng(0)
    target = oracle.moments(p, oracle.init(p, **fl))["rho"] + 0.01 * rng.standard_normal((10, 12))
    d_logs = rng.standard_normal(16)
    d_rho = rng.standard_normal((10, 12))
    h = 1e-30
    s = np.array(p["s"])
    # complex step along (log s, rho0)
    fc = oracle.init_complex(p, fl["rho"] + 1j * h * d_rho, fl["ux"], fl["uy"], fl["T"])
    fc = oracle.run_complex(p, fc, steps, s_im=h * s * d_logs)
    rc = oracle.moments_complex(p, fc)["rho"]
    dl_cs = np.sum((rc.real - target) * rc.imag) / h
    # central differences with the same direction
    hf = 1e-6
    vals = []
    for sgn in (1, -1):
        q = dict(p, s=list(s * np.exp(sgn * hf * d_logs)))
        f2 = dict(fl, rho=fl["rho"] + sgn * hf * d_rho)
        vals.append(_loss_real(q, f2, steps, target))
    dl_fd = (vals[0] - vals[1]) / (2 * hf)
    assert abs(dl_cs - dl_fd) <= 1e-6 * abs(dl_cs), (dl_cs, dl_fd)
