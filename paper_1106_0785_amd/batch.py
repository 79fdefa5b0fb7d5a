"""Binding of the batched form (include/lbm_batch.h): argument marshalling,
plus a small on-disk cache of the autotuner's choice per batch signature and
device. All stepping runs in the library's kernels."""

import ctypes
import hashlib
import json
import os

import numpy as np

from . import lbm

_sig_done = False


def _lib():
    global _sig_done
    lib = lbm.load()
    if not _sig_done:
        P = ctypes.c_void_p
        pp = ctypes.POINTER(lbm.LbmParams)
        sigs = {
            "lbm_batch_workspace_bytes": ([pp, ctypes.c_int32], ctypes.c_size_t),
            "lbm_batch_create": ([pp, ctypes.c_int32, P, ctypes.c_size_t, P, ctypes.POINTER(P)], ctypes.c_int),
            "lbm_batch_offset": ([P, ctypes.c_int32], ctypes.c_int64),
            "lbm_batch_init": ([P, P, P, P, P], ctypes.c_int),
            "lbm_batch_set_budgets": ([P, ctypes.POINTER(ctypes.c_int64)], ctypes.c_int),
            "lbm_batch_step": ([P, ctypes.c_int64], ctypes.c_int),
            "lbm_batch_moments": ([P, P, P, P, P, P], ctypes.c_int),
            "lbm_batch_get_f": ([P, P], ctypes.c_int),
            "lbm_batch_set_schedule": ([P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32], ctypes.c_int),
            "lbm_batch_get_schedule": ([P] + [ctypes.POINTER(ctypes.c_int32)] * 3, ctypes.c_int),
            "lbm_batch_set_persistent": ([P, ctypes.c_int32, ctypes.c_double], ctypes.c_int),
            "lbm_batch_get_persistent": ([P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)],
                                         ctypes.c_int),
            "lbm_batch_set_tile_rows": ([P, ctypes.c_int32], ctypes.c_int),
            "lbm_batch_set_two_step": ([P, ctypes.c_int32, ctypes.c_int32], ctypes.c_int),
            "lbm_batch_get_two_step": ([P] + [ctypes.POINTER(ctypes.c_int32)] * 3, ctypes.c_int),
            "lbm_batch_get_tile_rows": ([P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)],
                                        ctypes.c_int),
            "lbm_batch_tune": ([P, ctypes.c_int64, ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
            "lbm_batch_check": ([P], ctypes.c_int),
            "lbm_batch_destroy": ([P], None),
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


def _param_array(params):
    arr = (lbm.LbmParams * len(params))()
    for i, p in enumerate(params):
        arr[i] = lbm.LbmParams.from_dict(p)
    return arr


def lbm_batch_workspace_bytes(params):
    return int(_lib().lbm_batch_workspace_bytes(_param_array(params), len(params)))


CACHE = os.path.join(os.path.expanduser("~"), ".cache", "paper_1106_0785_amd", "batch_schedule.json")


def signature(params):
    h = hashlib.sha256()
    for p in params:
        h.update(json.dumps(p, sort_keys=True).encode())
    return h.hexdigest()[:20]


class Batch:
    """Owner of one batch: workspace tensor + handle. `params` is a list of
    parameter dicts (one- or two-dimensional problems, scheme 0)."""

    def __init__(self, params, device="cuda"):
        import torch

        self.params = [dict(p) for p in params]
        self.n = len(params)
        arr = _param_array(params)
        nbytes = int(_lib().lbm_batch_workspace_bytes(arr, self.n))
        if nbytes == 0:
            raise lbm.LbmError(-1, lbm.load().lbm_last_error().decode())
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        assert self.workspace.data_ptr() % 256 == 0
        self.device = self.workspace.device
        h = ctypes.c_void_p()
        stream = ctypes.c_void_p(torch.cuda.current_stream(self.device).cuda_stream)
        _check(_lib().lbm_batch_create(arr, self.n, ctypes.c_void_p(self.workspace.data_ptr()), nbytes, stream,
                                       ctypes.byref(h)))
        self.handle = h
        self.offsets = [int(_lib().lbm_batch_offset(h, i)) for i in range(self.n + 1)]
        self.total_nodes = self.offsets[-1]

    def concat(self, fields_list, key):
        import torch

        a = np.concatenate([np.ascontiguousarray(f[key], dtype=np.float64).ravel() for f in fields_list])
        return torch.from_numpy(a).to(self.device)

    def init(self, fields_list):
        t = [self.concat(fields_list, k) for k in ("rho", "ux", "uy", "T")]
        _check(_lib().lbm_batch_init(self.handle, *[ctypes.c_void_p(x.data_ptr()) for x in t]))
        self._keep = t

    def set_budgets(self, steps):
        if steps is None:
            _check(_lib().lbm_batch_set_budgets(self.handle, None))
        else:
            arr = (ctypes.c_int64 * self.n)(*[int(s) for s in steps])
            _check(_lib().lbm_batch_set_budgets(self.handle, arr))

    def step(self, nsteps):
        _check(_lib().lbm_batch_step(self.handle, int(nsteps)))

    def moments(self):
        import torch

        out = {k: torch.empty(self.total_nodes, dtype=torch.float64, device=self.device)
               for k in ("rho", "ux", "uy", "T", "p")}
        _check(_lib().lbm_batch_moments(self.handle, *[ctypes.c_void_p(out[k].data_ptr())
                                                       for k in ("rho", "ux", "uy", "T", "p")]))
        return out

    def split(self, flat, i):
        p = self.params[i]
        a, b = self.offsets[i], self.offsets[i + 1]
        return flat[a:b].reshape(p["ny"], p["nx"])

    def get_f(self):
        import torch

        f = torch.empty(16 * self.total_nodes, dtype=torch.float64, device=self.device)
        _check(_lib().lbm_batch_get_f(self.handle, ctypes.c_void_p(f.data_ptr())))
        return f

    def f_of(self, flat_f, i):
        p = self.params[i]
        a, b = 16 * self.offsets[i], 16 * self.offsets[i + 1]
        return flat_f[a:b].reshape(16, p["ny"], p["nx"])

    def set_schedule(self, region, steps_per_launch, use_graph=True):
        _check(_lib().lbm_batch_set_schedule(self.handle, int(region), int(steps_per_launch), int(bool(use_graph))))

    def schedule(self):
        r, h, c = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(_lib().lbm_batch_get_schedule(self.handle, ctypes.byref(r), ctypes.byref(h), ctypes.byref(c)))
        return {"region": r.value, "steps_per_launch": h.value, "chunks": c.value}

    def set_persistent(self, persistent, timeout_ms=2000.0):
        """Line instances: one persistent launch per equilibrium version for a
        whole call (True) or one launch per block of h steps (False);
        timeout_ms bounds each wait of the persistent launch for the chunks a
        chunk depends on."""
        _check(_lib().lbm_batch_set_persistent(self.handle, int(persistent), float(timeout_ms)))

    def persistent(self):
        p, g = ctypes.c_int32(), ctypes.c_int32()
        _check(_lib().lbm_batch_get_persistent(self.handle, ctypes.byref(p), ctypes.byref(g)))
        return {"persistent": bool(p.value), "grid": g.value}

    def set_tile_rows(self, rows):
        _check(_lib().lbm_batch_set_tile_rows(self.handle, int(rows)))

    def tile_rows(self):
        r, t = ctypes.c_int32(), ctypes.c_int32()
        _check(_lib().lbm_batch_get_tile_rows(self.handle, ctypes.byref(r), ctypes.byref(t)))
        return {"tile_rows": r.value, "tiles": t.value}

    def set_two_step(self, on, rows=32):
        """Plain tiled instances: two steps per launch (on) with `rows`
        output rows per two-step tile, or one step per launch."""
        _check(_lib().lbm_batch_set_two_step(self.handle, int(on), int(rows)))

    def two_step(self):
        o, r, t = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
        _check(_lib().lbm_batch_get_two_step(self.handle, ctypes.byref(o), ctypes.byref(r), ctypes.byref(t)))
        return {"two_step": bool(o.value), "tile_rows2": r.value, "tiles2": t.value}

    def tune(self, probe_steps=64, use_cache=True):
        """Run the library's autotuner (or reuse a cached choice for this batch
        signature and device). Returns the chosen schedule."""
        import torch

        key = signature(self.params) + ":" + torch.cuda.get_device_name(self.device)
        cache = {}
        if use_cache and os.path.exists(CACHE):
            try:
                cache = json.load(open(CACHE))
            except ValueError:
                cache = {}
        if use_cache and key in cache and all(k in cache[key] for k in ("tile_rows", "persistent", "two_step")):
            c = cache[key]
            self.set_schedule(c["region"], c["steps_per_launch"])
            self.set_persistent(c["persistent"])
            self.set_tile_rows(c["tile_rows"])
            self.set_two_step(c["two_step"], c["tile_rows2"])
            return dict(c, cached=True)
        best = ctypes.c_double()
        _check(_lib().lbm_batch_tune(self.handle, int(probe_steps), ctypes.byref(best)))
        s = self.schedule()
        s.update(self.tile_rows())
        s["persistent"] = self.persistent()["persistent"]
        s.update(self.two_step())
        s["probe_ms"] = best.value
        if use_cache:
            os.makedirs(os.path.dirname(CACHE), exist_ok=True)
            cache[key] = s
            with open(CACHE, "w") as fh:
                json.dump(cache, fh)
        return dict(s, cached=False)

    def check(self):
        _check(_lib().lbm_batch_check(self.handle))

    def close(self):
        if getattr(self, "handle", None) is not None:
            _lib().lbm_batch_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
