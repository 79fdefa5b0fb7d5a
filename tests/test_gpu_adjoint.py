"""The hand-written adjoint against the oracle's complex-step derivatives
(exact up to rounding) and against central finite differences of the GPU
forward path, on small problems with every supported boundary kind and on
the 512 x 128, 2000-step shock/interface configuration."""

import math

import numpy as np
import pytest

import oracle
from gpu_util import log
from paper_1106_0785_amd import inputs

pytestmark = pytest.mark.gpu


def _torch():
    import torch

    return torch


def _adjoint_directional(p, fl, steps, w_rho, w_T, d_fields, d_logs, ckpt=0):
    """dL along (d_fields, d_logs) for L = sum(w_rho * rho_T) + sum(w_T * T_T)."""
    from paper_1106_0785_amd.autograd import Adjoint

    torch = _torch()
    a = Adjoint(p, steps, ckpt)
    f0 = [torch.from_numpy(np.ascontiguousarray(fl[k])).cuda() for k in ("rho", "ux", "uy", "T")]
    a.forward(*f0)
    grads, gs = a.backward(torch.from_numpy(w_rho).cuda(), None, None, torch.from_numpy(w_T).cuda())
    grads = [g.cpu().numpy() for g in grads]
    gs = gs.cpu().numpy()
    s = np.array(p["s"])
    a.close()
    dl = sum(float(np.sum(g * d)) for g, d in zip(grads, d_fields))
    return dl + float(np.sum(gs * s * d_logs)), gs


def _complex_step(p, fl, steps, w_rho, w_T, d_fields, d_logs):
    h = 1e-30
    keys = ("rho", "ux", "uy", "T")
    cf = {k: fl[k] + 1j * h * d for k, d in zip(keys, d_fields)}
    f = oracle.init_complex(p, cf["rho"], cf["ux"], cf["uy"], cf["T"])
    s = np.array(p["s"])
    f = oracle.run_complex(p, f, steps, s_im=h * s * d_logs)
    m = oracle.moments_complex(p, f)
    return float(np.sum(w_rho * m["rho"].imag) + np.sum(w_T * m["T"].imag)) / h


CASES = {
    "specular_x_periodic_y": (["specular", "specular", "periodic", "periodic"], {}),
    "zero_gradient_x_specular_y": (["zero_gradient", "zero_gradient", "specular", "specular"], {}),
    "dirichlet_x": (["dirichlet_eq", "zero_gradient", "periodic", "periodic"], {}),
    "unmodified_periodic": (["periodic"] * 4, {"modified": 0}),
    "version2_periodic": (["periodic"] * 4, {"eq_version": 2}),
    "printed_sign": (["specular", "specular", "periodic", "periodic"], {"modified": 2}),
    "neq_walls_y": (["periodic", "periodic", "neq_wall", "neq_wall"], {}),
    "neq_walls_x_version3": (["neq_wall", "neq_wall", "specular", "specular"], {"eq_version": 3}),
}


@pytest.mark.parametrize("name", sorted(CASES))
def test_adjoint_matches_complex_step(name):
    bc, kw = CASES[name]
    p, fl = inputs.smooth_periodic(seed=13, nx=23, ny=17, amp=0.06, **kw)
    p["bc"] = bc
    p["wall"][0] = [1.03, 0.02, 0.0, 1.01]
    p["wall"][1] = [1.0, 0.0, 0.05, 1.04]
    p["wall"][2] = [1.0, -0.03, 0.0, 0.97]
    p["wall"][3] = [1.0, 0.06, 0.0, 1.02]
    p["s"][4], p["s"][5], p["s"][6], p["s"][7] = 700.0, 900.0, 1200.0, 1500.0
    steps = 40
    rng = np.random.default_rng(1)
    w_rho = rng.standard_normal((17, 23))
    w_T = rng.standard_normal((17, 23))
    worst = 0.0
    for trial in range(3):
        d_fields = [rng.standard_normal((17, 23)) for _ in range(4)]
        d_logs = rng.standard_normal(16)
        got, gs = _adjoint_directional(p, fl, steps, w_rho, w_T, d_fields, d_logs, ckpt=7)
        ref = _complex_step(p, fl, steps, w_rho, w_T, d_fields, d_logs)
        rel = abs(got - ref) / abs(ref)
        worst = max(worst, rel)
        assert np.all(gs[:4] == 0.0)
    log("adjoint vs complex step (%s): max rel diff %.2e" % (name, worst))
    assert worst <= 1e-9


@pytest.mark.parametrize("ny", [3, 5])
def test_adjoint_walls_three_and_five_nodes_apart(ny):
    """Walls on both ends of a short column: with ny = 3 both walls take
    their values from the same fluid node."""
    p, fl = inputs.smooth_periodic(seed=5, nx=9, ny=ny, amp=0.04)
    p["bc"] = ["periodic", "periodic", "neq_wall", "neq_wall"]
    p["wall"][2] = [1.0, 0.01, 0.0, 1.0]
    p["wall"][3] = [1.0, 0.08, 0.0, 1.03]
    rng = np.random.default_rng(ny)
    w = rng.standard_normal((ny, 9))
    d_fields = [rng.standard_normal((ny, 9)) for _ in range(4)]
    d_logs = rng.standard_normal(16)
    got, gs = _adjoint_directional(p, fl, 30, w, np.zeros((ny, 9)), d_fields, d_logs, ckpt=4)
    ref = _complex_step(p, fl, 30, w, np.zeros((ny, 9)), d_fields, d_logs)
    rel = abs(got - ref) / abs(ref)
    log("adjoint with walls %d nodes apart vs complex step: rel diff %.2e" % (ny, rel))
    assert rel <= 1e-9


def test_couette_prandtl_sensitivity():
    """The thermal Couette configuration (4 x 64, NEQ walls, Pr = 1) run to
    steady state (20000 steps): d/d log(s7 s8) of the mid-channel temperature
    bump (the Pr-dependent viscous heating of Sec. IV.A) against the oracle's
    complex-step derivative."""
    p, fl, meta = inputs.couette(1.0)
    steps = 20000
    ny, nx = 64, 4
    w = np.zeros((ny, nx))
    w[ny // 2, :] = 1.0 / nx  # mean temperature of the middle row
    d_logs = np.zeros(16)
    d_logs[6] = d_logs[7] = 1.0  # Pr = s7 / s5 up by the same factor in s7 and s8
    zeros = [np.zeros((ny, nx)) for _ in range(4)]
    got, gs = _adjoint_directional(p, fl, steps, np.zeros((ny, nx)), w, zeros, d_logs)
    ref = _complex_step(p, fl, steps, np.zeros((ny, nx)), w, zeros, d_logs)
    rel = abs(got - ref) / abs(ref)
    log("Couette dT_mid/dlog Pr: adjoint %.6e, complex step %.6e, rel %.2e" % (got, ref, rel))
    assert rel <= 1e-9
    # a larger Pr (less conduction against the same viscous heating) raises the bump
    assert got > 0.0


def test_wide_grid_adjoint_matches_complex_step():
    """A grid of more than 2048 adjoint blocks (2112 x 260) takes the
    two-blocks-per-CU form of the adjoint step; same check as above."""
    nx, ny = 2112, 260
    p, fl = inputs.smooth_periodic(seed=17, nx=nx, ny=ny, amp=0.06)
    p["bc"] = ["specular", "specular", "periodic", "periodic"]
    p["s"][4], p["s"][5], p["s"][6], p["s"][7] = 700.0, 900.0, 1200.0, 1500.0
    steps = 6
    rng = np.random.default_rng(3)
    w_rho = rng.standard_normal((ny, nx))
    w_T = rng.standard_normal((ny, nx))
    d_fields = [rng.standard_normal((ny, nx)) for _ in range(4)]
    d_logs = rng.standard_normal(16)
    got, gs = _adjoint_directional(p, fl, steps, w_rho, w_T, d_fields, d_logs, ckpt=2)
    ref = _complex_step(p, fl, steps, w_rho, w_T, d_fields, d_logs)
    rel = abs(got - ref) / abs(ref)
    log("wide-grid adjoint vs complex step: rel diff %.2e" % rel)
    assert rel <= 1e-9
    assert np.all(gs[:4] == 0.0)


def _rm_loss_setup(nx=512, ny=128, steps=2000):
    torch = _torch()
    p, fl, meta = inputs.rm(seed=0, nx=nx, ny=ny)
    p_t, fl_t, meta_t = inputs.rm(seed=101, nx=nx, ny=ny, mach=meta["mach"])
    from paper_1106_0785_amd import lbm

    sim = lbm.Simulation(p_t)
    sim.init(**fl_t)
    sim.step(steps)
    target = sim.moments()["rho"].clone()
    sim.close()
    return p, meta, target


def _fields_of(a, meta, nx, ny):
    torch = _torch()
    return inputs.rm_fields(nx, ny, a, meta["mach"], meta["heavy"], meta["x0_cells"], meta["shock_cells"],
                            meta["width_cells"], meta["wall_ramp_cells"], xp=torch)


def _rho_forward(p, meta, a, log_s, steps):
    """Final density of the plain forward path (no adjoint)."""
    from paper_1106_0785_amd import lbm

    nx, ny = p["nx"], p["ny"]
    f = _fields_of(a, meta, nx, ny)
    q = dict(p, s=[math.exp(v) for v in log_s.tolist()])
    sim = lbm.Simulation(q)
    sim.init(f["rho"], f["ux"], f["uy"], f["T"])
    sim.step(steps)
    rho = sim.moments()["rho"].clone()
    sim.close()
    return rho


def _loss_difference(rho_p, rho_m, target):
    """L(+) - L(-) for L = 1/2 sum (rho - target)^2, written as
    1/2 sum (rho+ - rho-)(rho+ + rho- - 2 target) so that the two losses are
    not formed separately (their difference is ~1e-6 of either, and each is
    a sum over 65536 nodes), then summed exactly on the host."""
    t = 0.5 * (rho_p - rho_m) * (rho_p + rho_m - 2.0 * target)
    return math.fsum(t.cpu().numpy().ravel().tolist())


def test_rm_adjoint_finite_differences_and_timing():
    """512 x 128 shock/interface, 2000 steps, sqrt(T) checkpoints; gradient
    w.r.t. all log s_i and the per-row interface displacement a(y), checked by
    central differences (h = 1e-6) along 8 seeded directions."""
    import time

    from paper_1106_0785_amd.autograd import simulate

    torch = _torch()
    nx, ny, steps = 512, 128, 2000
    p, meta, target = _rm_loss_setup(nx, ny, steps)
    a = torch.tensor(meta["a"], dtype=torch.float64, device="cuda", requires_grad=True)
    log_s = torch.tensor(np.log(p["s"]), dtype=torch.float64, device="cuda", requires_grad=True)
    torch.cuda.synchronize()
    t0 = time.perf_counter()
    f = _fields_of(a, meta, nx, ny)
    rho, ux, uy, T = simulate(f["rho"], f["ux"], f["uy"], f["T"], log_s, p, steps)
    loss = 0.5 * torch.sum((rho - target) ** 2)
    torch.cuda.synchronize()
    t1 = time.perf_counter()
    loss.backward()
    torch.cuda.synchronize()
    t2 = time.perf_counter()
    log("rm 512x128x2000: forward (checkpointed) %.3f s, backward %.3f s, ratio %.2f"
        % (t1 - t0, t2 - t1, (t2 - t1) / (t1 - t0)))
    ga = a.grad.detach().cpu().numpy()
    gs = log_s.grad.detach().cpu().numpy()
    a0 = a.detach().clone()
    s0 = log_s.detach().clone()
    rng = np.random.default_rng(8)
    h = 1e-6
    worst = 0.0
    for k in range(8):
        d = rng.standard_normal(ny + 16)
        d /= np.linalg.norm(d)
        da, ds = d[:ny], d[ny:]
        adj = float(np.sum(ga * da) + np.sum(gs * ds))
        dat = torch.tensor(da, dtype=torch.float64, device="cuda")
        dst = torch.tensor(ds, dtype=torch.float64, device="cuda")
        rp = _rho_forward(p, meta, a0 + h * dat, s0 + h * dst, steps)
        rm = _rho_forward(p, meta, a0 - h * dat, s0 - h * dst, steps)
        fd = _loss_difference(rp, rm, target) / (2 * h)
        rel = abs(adj - fd) / max(abs(fd), 1e-300)
        worst = max(worst, rel)
        log("direction %d: adjoint %.10e  central FD %.10e  rel %.2e" % (k, adj, fd, rel))
    assert worst <= 1e-6


def test_random_problems_against_complex_step():
    """20 seeded random problems (shape, boundary kinds including NEQ walls,
    equilibrium version, modification, rates, step count, checkpoint
    interval): the adjoint's directional derivative against the oracle's
    complex step."""
    rng = np.random.default_rng(404)
    kinds = ["periodic", "zero_gradient", "specular", "dirichlet_eq", "neq_wall"]
    done = 0
    worst = 0.0
    while done < 20:
        nx, ny = int(rng.integers(1, 60)), int(rng.integers(1, 40))
        bx, by = kinds[int(rng.integers(0, 5))], kinds[int(rng.integers(0, 5))]
        if bx == "neq_wall" and by == "neq_wall":
            continue
        if (nx == 1 and bx != "periodic") or (ny == 1 and by != "periodic"):
            continue
        if (bx == "neq_wall" and nx < 3) or (by == "neq_wall" and ny < 3):
            continue
        p, fl = inputs.smooth_periodic(seed=int(rng.integers(0, 10 ** 6)), nx=nx, ny=ny, amp=0.06,
                                       eq_version=int(rng.integers(1, 4)), modified=int(rng.integers(0, 3)))
        p["bc"] = [bx, bx, by, by]
        for side in range(4):
            p["wall"][side] = [1.0 + 0.05 * rng.random(), 0.05 * rng.standard_normal(), 0.05 * rng.standard_normal(),
                               1.0 + 0.05 * rng.random()]
        p["s"][4], p["s"][5], p["s"][6], p["s"][7] = [float(x) for x in rng.uniform(500, 1900, 4)]
        steps, ckpt = int(rng.integers(1, 50)), int(rng.integers(0, 9))
        w_rho, w_T = rng.standard_normal((ny, nx)), rng.standard_normal((ny, nx))
        d_fields = [rng.standard_normal((ny, nx)) for _ in range(4)]
        d_logs = rng.standard_normal(16)
        got, _ = _adjoint_directional(p, fl, steps, w_rho, w_T, d_fields, d_logs, ckpt=ckpt)
        ref = _complex_step(p, fl, steps, w_rho, w_T, d_fields, d_logs)
        rel = abs(got - ref) / abs(ref)
        log("random adjoint %d: %dx%d (%s, %s), %d steps, ckpt %d: rel diff %.2e" % (done, nx, ny, bx, by, steps, ckpt, rel))
        assert rel <= 1e-9
        worst = max(worst, rel)
        done += 1
    log("random adjoint problems: worst rel diff %.2e" % worst)


def test_forward_reports_lost_positivity():
    """A trajectory that loses positivity (here: one node starts at T < 0)
    raises instead of returning gradients; the handle's flag is cleared, so
    the next valid run of the same size passes."""
    import torch

    from paper_1106_0785_amd import lbm
    from paper_1106_0785_amd.autograd import Adjoint

    p, fl = inputs.smooth_periodic(seed=3, nx=16, ny=8, amp=0.05)
    bad = {k: v.copy() for k, v in fl.items()}
    bad["T"][4, 7] = -0.5
    a = Adjoint(p, 5, 2)
    with pytest.raises(lbm.LbmError) as err:
        a.forward(*[torch.from_numpy(bad[k]).cuda() for k in ("rho", "ux", "uy", "T")])
    assert err.value.status == -5, str(err.value)
    out = a.forward(*[torch.from_numpy(fl[k]).cuda() for k in ("rho", "ux", "uy", "T")])
    assert torch.isfinite(out["rho"]).all()
    a.close()


@pytest.mark.parametrize("shape", [(23, 17), (70, 9), (1, 13), (130, 1), (64, 4), (129, 33)])
@pytest.mark.parametrize("name", ["specular_x_periodic_y", "dirichlet_x", "neq_walls_y", "neq_walls_x_version3",
                                  "zero_gradient_x_specular_y"])
def test_lds_step_matches_gather_step(name, shape):
    """The LDS-staged adjoint step against the one-thread-per-node form on
    the same problem: every gradient entry to rounding (the per-tile
    s-gradient sums run in another order). The other adjoint tests run
    whichever form is the default for their grid."""
    import torch

    from paper_1106_0785_amd.autograd import Adjoint

    bc, kw = CASES[name]
    nx, ny = shape
    if (nx == 1 and bc[0] != "periodic") or (ny == 1 and bc[2] != "periodic"):
        pytest.skip("an axis of extent 1 must be periodic")
    if ("neq_wall" in bc[:2] and nx < 3) or ("neq_wall" in bc[2:] and ny < 3):
        pytest.skip("walls need 3 nodes")
    p, fl = inputs.smooth_periodic(seed=31, nx=nx, ny=ny, amp=0.06, **kw)
    p["bc"] = bc
    p["wall"][0] = [1.03, 0.02, 0.0, 1.01]
    p["wall"][1] = [1.0, 0.0, 0.05, 1.04]
    p["wall"][2] = [1.0, -0.03, 0.0, 0.97]
    p["wall"][3] = [1.0, 0.06, 0.0, 1.02]
    rng = np.random.default_rng(7)
    w_rho = torch.from_numpy(rng.standard_normal((ny, nx))).cuda()
    w_T = torch.from_numpy(rng.standard_normal((ny, nx))).cuda()
    f0 = [torch.from_numpy(np.ascontiguousarray(fl[k])).cuda() for k in ("rho", "ux", "uy", "T")]
    res = []
    for v in (0, 1):
        a = Adjoint(p, 25, 6)
        a.set_variant(v)
        a.forward(*f0)
        grads, gs = a.backward(w_rho, None, None, w_T)
        res.append(([g.cpu().numpy() for g in grads], gs.cpu().numpy()))
        a.close()
    for k in range(4):
        g0, g1 = res[0][0][k], res[1][0][k]
        err = np.max(np.abs(g0 - g1)) / max(np.max(np.abs(g1)), 1e-300)
        assert err <= 1e-12, (name, shape, k, err)
    es = np.max(np.abs(res[0][1] - res[1][1])) / np.max(np.abs(res[1][1]))
    assert es <= 1e-12, (name, shape, es)
