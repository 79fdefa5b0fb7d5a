"""Binding of the von Neumann stability tool (include/lbm_stability.h):
argument marshalling only; G(theta) and |omega|_max are computed by the
library's kernels."""

import ctypes

from . import lbm

_sig_done = False


class LbmState(ctypes.Structure):
    _fields_ = [("rho", ctypes.c_double), ("ux", ctypes.c_double), ("uy", ctypes.c_double), ("T", ctypes.c_double)]


def _lib():
    global _sig_done
    lib = lbm.load()
    if not _sig_done:
        P = ctypes.c_void_p
        pp = ctypes.POINTER(lbm.LbmParams)
        ps = ctypes.POINTER(LbmState)
        sigs = {
            "lbm_stability_workspace_bytes": ([ctypes.c_int32], ctypes.c_size_t),
            "lbm_stability_matrix": ([pp, ps, ctypes.c_int32, P, ctypes.c_int32, P, ctypes.c_size_t, P, P],
                                     ctypes.c_int),
            "lbm_stability_radius": ([pp, ps, ctypes.c_int32, P, ctypes.c_int32, ctypes.c_int32, P,
                                      ctypes.c_size_t, P, P], ctypes.c_int),
        }
        for name, (args, res) in sigs.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _sig_done = True
    return lib


def _sets(params, states):
    if len(params) != len(states):
        raise ValueError("one base state per parameter set")
    n = len(params)
    ps = (lbm.LbmParams * n)()
    ss = (LbmState * n)()
    for k, (p, s) in enumerate(zip(params, states)):
        q = dict(p)
        q.setdefault("nx", 1)
        q.setdefault("ny", 1)
        q.setdefault("bc", ["periodic"] * 4)
        ps[k] = lbm.LbmParams.from_dict(q)
        ss[k] = LbmState(*[float(v) for v in s])
    return ps, ss, n


def lbm_stability_workspace_bytes(nsets):
    return int(_lib().lbm_stability_workspace_bytes(int(nsets)))


def _workspace(n, device):
    import torch

    nbytes = lbm_stability_workspace_bytes(n)
    if nbytes == 0:
        raise lbm.LbmError(-1, "no parameter sets")
    ws = torch.empty(nbytes, dtype=torch.uint8, device=device)
    assert ws.data_ptr() % 256 == 0
    return ws


def amplification_matrix(params, states, theta):
    """G(theta) in the moment basis: complex tensor [nsets, npts, 16, 16].
    params: list of parameter dicts; states: list of (rho, ux, uy, T);
    theta: float64 CUDA tensor [npts, 2] of (k_x dx, k_y dy)."""
    import torch

    ps, ss, n = _sets(params, states)
    theta = theta.contiguous()
    npts = theta.shape[0]
    ws = _workspace(n, theta.device)
    out = torch.empty((n, npts, 2, 16, 16), dtype=torch.float64, device=theta.device)
    lbm._check(_lib().lbm_stability_matrix(ps, ss, n, lbm._ptr(theta), npts, ctypes.c_void_p(ws.data_ptr()),
                                           ws.numel(), lbm._ptr(out), lbm._stream()))
    return torch.complex(out[:, :, 0], out[:, :, 1])


def omega_max(params, states, theta, squarings=0):
    """|omega|_max: float64 tensor [nsets, npts] (arguments as above)."""
    import torch

    ps, ss, n = _sets(params, states)
    theta = theta.contiguous()
    npts = theta.shape[0]
    ws = _workspace(n, theta.device)
    out = torch.empty((n, npts), dtype=torch.float64, device=theta.device)
    lbm._check(_lib().lbm_stability_radius(ps, ss, n, lbm._ptr(theta), npts, int(squarings),
                                           ctypes.c_void_p(ws.data_ptr()), ws.numel(), lbm._ptr(out),
                                           lbm._stream()))
    return out
