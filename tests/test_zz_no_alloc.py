"""The allocation-free entry point (lbm_run_noalloc) through the C ABI,
against the workspace path (lbm_create / lbm_set_f / lbm_step / lbm_get_f)
on the same input: two calls in a row, the second with a smaller grid (the
array then still holds the first call's larger state), and the size limit."""

import ctypes

import numpy as np
import pytest

from gpu_util import log
from paper_1106_0785_amd import inputs

pytestmark = pytest.mark.gpu

TOL = 1e-11


def _lib():
    from paper_1106_0785_amd import lbm

    lib = lbm.load()
    P = ctypes.c_void_p
    lib.lbm_run_noalloc.argtypes = [ctypes.POINTER(lbm.LbmParams), P, P, ctypes.c_int64, P, P]
    lib.lbm_run_noalloc.restype = ctypes.c_int
    return lib, lbm


def _reference(p, f0, steps):
    """The existing entry points on the same distributions."""
    import torch

    from paper_1106_0785_amd import lbm

    sim = lbm.Simulation(p)
    sim.set_f(torch.from_numpy(f0).cuda())
    sim.step(steps)
    out = sim.get_f().cpu().numpy()
    sim.check()
    sim.close()
    return out


def _noalloc(p, f0, steps):
    import torch

    lib, lbm = _lib()
    fin = torch.from_numpy(f0).cuda()
    fout = torch.full_like(fin, float("nan"))
    status = torch.full((1,), 99, dtype=torch.int32, device="cuda")
    stream = torch.cuda.current_stream().cuda_stream
    q = lbm.LbmParams.from_dict(p)
    rc = lib.lbm_run_noalloc(ctypes.byref(q), ctypes.c_void_p(fin.data_ptr()), ctypes.c_void_p(fout.data_ptr()),
                             int(steps), ctypes.c_void_p(status.data_ptr()), ctypes.c_void_p(stream))
    assert rc == 0, lib.lbm_last_error().decode()
    torch.cuda.synchronize()
    assert int(status.item()) == 0
    return fout.cpu().numpy()


def _initial(p, fl):
    import torch

    from paper_1106_0785_amd import lbm

    sim = lbm.Simulation(p)
    sim.init(**fl)
    f0 = sim.get_f().cpu().numpy()
    sim.close()
    return f0


def _compare(got, ref, what):
    scale = np.abs(ref).max(axis=(1, 2), keepdims=True)
    err = float(np.max(np.abs(got - ref) / scale))
    log("%s: max difference / plane scale %.2e (bitwise equal: %s)" % (what, err, bool(np.array_equal(got, ref))))
    assert err <= TOL, (what, err)


def test_noalloc_matches_workspace_path_twice_then_smaller():
    # first call: the largest shape the array holds (1024 x 256, fused kernel)
    p1, fl1, _ = inputs.rm(seed=2, nx=1024, ny=256)
    f1 = _initial(p1, fl1)
    _compare(_noalloc(p1, f1, 12), _reference(p1, f1, 12), "noalloc 1024x256 x 12 steps")
    # second call, smaller and with NEQ walls, on the array the first call left
    p2, fl2, _ = inputs.couette(2.0, nx=37, ny=30)
    f2 = _initial(p2, fl2)
    _compare(_noalloc(p2, f2, 300), _reference(p2, f2, 300), "noalloc 37x30 Couette x 300 steps")
    # a narrow grid (windowed kernel) and a tiny one (small-grid kernel)
    p3, fl3, _ = inputs.riemann("lax", Pr=0.5, nx=700, ny=2)
    f3 = _initial(p3, fl3)
    _compare(_noalloc(p3, f3, 50), _reference(p3, f3, 50), "noalloc 700x2 Lax x 50 steps")
    p4, fl4 = inputs.smooth_periodic(seed=9, nx=13, ny=11, amp=0.05)
    f4 = _initial(p4, fl4)
    _compare(_noalloc(p4, f4, 70), _reference(p4, f4, 70), "noalloc 13x11 periodic x 70 steps")


def test_noalloc_reports_lost_positivity_and_rejects_large_grids():
    import torch

    lib, lbm = _lib()
    p, fl = inputs.smooth_periodic(seed=3, nx=70, ny=20, amp=0.05)
    bad = {k: v.copy() for k, v in fl.items()}
    bad["T"][4, 7] = -0.5
    f0 = _initial(p, bad)
    fin = torch.from_numpy(f0).cuda()
    status = torch.zeros(1, dtype=torch.int32, device="cuda")
    q = lbm.LbmParams.from_dict(p)
    stream = torch.cuda.current_stream().cuda_stream
    rc = lib.lbm_run_noalloc(ctypes.byref(q), ctypes.c_void_p(fin.data_ptr()), ctypes.c_void_p(fin.data_ptr()), 3,
                             ctypes.c_void_p(status.data_ptr()), ctypes.c_void_p(stream))
    assert rc == 0
    torch.cuda.synchronize()
    assert int(status.item()) == -5
    # one row more than the array holds: rejected before anything is enqueued
    big = lbm.LbmParams.from_dict(dict(p, nx=1024, ny=257))
    rc = lib.lbm_run_noalloc(ctypes.byref(big), ctypes.c_void_p(fin.data_ptr()), ctypes.c_void_p(fin.data_ptr()), 1,
                             None, ctypes.c_void_p(stream))
    assert rc == -1
    assert "at most 262144" in lib.lbm_last_error().decode()
