"""Differentiable simulation: a torch.autograd.Function whose forward runs the
checkpointed forward sweep of liblbm's adjoint form and whose backward runs
the hand-written adjoint kernels (include/lbm_adjoint.h). Gradients flow to
the initial fields (rho, u_x, u_y, T) and to log s_1..s_16 (s_1..s_4 get 0).
This module only marshals arguments; all arithmetic runs in the library."""

import ctypes
import math

import torch

from . import lbm

_sig_done = False


def _lib():
    global _sig_done
    lib = lbm.load()
    if not _sig_done:
        P = ctypes.c_void_p
        pp = ctypes.POINTER(lbm.LbmParams)
        sigs = {
            "lbm_adjoint_workspace_bytes": ([pp, ctypes.c_int64, ctypes.c_int32], ctypes.c_size_t),
            "lbm_adjoint_create": ([pp, ctypes.c_int64, ctypes.c_int32, P, ctypes.c_size_t, P, ctypes.POINTER(P)],
                                   ctypes.c_int),
            "lbm_adjoint_forward": ([P, P, P, P, P], ctypes.c_int),
            "lbm_adjoint_final_moments": ([P, P, P, P, P, P], ctypes.c_int),
            "lbm_adjoint_backward": ([P] + [P] * 13, ctypes.c_int),
            "lbm_adjoint_check": ([P], ctypes.c_int),
            "lbm_adjoint_set_variant": ([P, ctypes.c_int32], ctypes.c_int),
            "lbm_adjoint_destroy": ([P], None),
        }
        for name, (args, res) in sigs.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _sig_done = True
    return lib


def _check(rc):
    if rc != 0:
        raise lbm.LbmError(rc, lbm.load().lbm_last_error().decode())


def _p(t):
    return None if t is None else ctypes.c_void_p(t.data_ptr())


class Adjoint:
    """Owner of one adjoint context (workspace + handle)."""

    def __init__(self, params, nsteps, ckpt_interval=0, device="cuda"):
        self.params = dict(params)
        self.nx, self.ny = int(params["nx"]), int(params["ny"])
        p = lbm.LbmParams.from_dict(params)
        nbytes = int(_lib().lbm_adjoint_workspace_bytes(ctypes.byref(p), int(nsteps), int(ckpt_interval)))
        if nbytes == 0:
            raise lbm.LbmError(-1, lbm.load().lbm_last_error().decode())
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        assert self.workspace.data_ptr() % 256 == 0
        self.device = self.workspace.device
        h = ctypes.c_void_p()
        stream = ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)
        _check(_lib().lbm_adjoint_create(ctypes.byref(p), int(nsteps), int(ckpt_interval),
                                         ctypes.c_void_p(self.workspace.data_ptr()), nbytes, stream, ctypes.byref(h)))
        self.handle = h

    def set_variant(self, v):
        """0: the LDS-staged adjoint step (default on large grids); 1: one
        thread per node (default on small grids)."""
        _check(_lib().lbm_adjoint_set_variant(self.handle, int(v)))

    def _f(self, a):
        return a.detach().to(self.device, dtype=torch.float64).contiguous()

    def forward(self, rho0, ux0, uy0, T0):
        self._init = [self._f(a) for a in (rho0, ux0, uy0, T0)]
        _check(_lib().lbm_adjoint_forward(self.handle, *[_p(t) for t in self._init]))
        out = {k: torch.empty((self.ny, self.nx), dtype=torch.float64, device=self.device)
               for k in ("rho", "ux", "uy", "T", "p")}
        _check(_lib().lbm_adjoint_final_moments(self.handle, *[_p(out[k]) for k in ("rho", "ux", "uy", "T", "p")]))
        # a trajectory that lost positivity has no meaningful gradient
        _check(_lib().lbm_adjoint_check(self.handle))
        return out

    def backward(self, g_rho=None, g_ux=None, g_uy=None, g_T=None):
        g = [None if x is None else self._f(x) for x in (g_rho, g_ux, g_uy, g_T)]
        grads = [torch.empty((self.ny, self.nx), dtype=torch.float64, device=self.device) for _ in range(4)]
        grad_s = torch.empty(16, dtype=torch.float64, device=self.device)
        _check(_lib().lbm_adjoint_backward(self.handle, *[_p(t) for t in self._init], *[_p(t) for t in g],
                                           *[_p(t) for t in grads], _p(grad_s)))
        self._keep = g
        _check(_lib().lbm_adjoint_check(self.handle))
        return grads, grad_s

    def close(self):
        if getattr(self, "handle", None) is not None:
            _lib().lbm_adjoint_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass


class LBMSimulate(torch.autograd.Function):
    """(rho0, ux0, uy0, T0, log_s) -> final (rho, ux, uy, T) after nsteps."""

    @staticmethod
    def forward(ctx, rho0, ux0, uy0, T0, log_s, params, nsteps, ckpt_interval):
        s = [math.exp(v) for v in log_s.detach().cpu().tolist()]
        q = dict(params, s=s)
        adj = Adjoint(q, nsteps, ckpt_interval, device=rho0.device)
        out = adj.forward(rho0, ux0, uy0, T0)
        ctx.adj = adj
        ctx.s = torch.tensor(s, dtype=torch.float64, device=rho0.device)
        return out["rho"], out["ux"], out["uy"], out["T"]

    @staticmethod
    def backward(ctx, g_rho, g_ux, g_uy, g_T):
        grads, grad_s = ctx.adj.backward(g_rho, g_ux, g_uy, g_T)
        ctx.adj.close()
        grad_log_s = grad_s * ctx.s
        return grads[0], grads[1], grads[2], grads[3], grad_log_s, None, None, None


def simulate(rho0, ux0, uy0, T0, log_s, params, nsteps, ckpt_interval=0):
    """Differentiable nsteps-step simulation; returns final (rho, ux, uy, T)."""
    return LBMSimulate.apply(rho0, ux0, uy0, T0, log_s, params, int(nsteps), int(ckpt_interval))
