"""Python binding of liblbm (include/lbm.h): argument marshalling only.

Every function here calls the C ABI of the HIP library with the same name;
all arithmetic of the method runs in the library's kernels. PyTorch provides
device memory and the stream. There is no fallback: if the library is not
built, or no GPU is present, calls fail loudly.
"""

import ctypes
import os

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
LIB_PATH = os.path.join(_HERE, "liblbm.so")

BC = {"periodic": 0, "zero_gradient": 1, "specular": 2, "neq_wall": 3, "dirichlet_eq": 4}
STATUS = {0: "LBM_OK", -1: "LBM_EINVAL", -2: "LBM_ENOMEM", -3: "LBM_EHIP", -4: "LBM_ESTATE", -5: "LBM_ENONFINITE",
          -6: "LBM_ETIMEOUT"}


class LbmError(RuntimeError):
    def __init__(self, status, msg):
        super().__init__("%s: %s" % (STATUS.get(status, status), msg))
        self.status = status


class LbmParams(ctypes.Structure):
    _fields_ = [
        ("nx", ctypes.c_int32),
        ("ny", ctypes.c_int32),
        ("dx", ctypes.c_double),
        ("dy", ctypes.c_double),
        ("dt", ctypes.c_double),
        ("s", ctypes.c_double * 16),
        ("eq_version", ctypes.c_int32),
        ("modified", ctypes.c_int32),
        ("bc", ctypes.c_int32 * 4),
        ("wall", (ctypes.c_double * 4) * 4),
        ("scheme", ctypes.c_int32),
    ]

    @classmethod
    def from_dict(cls, d):
        p = cls()
        p.nx, p.ny = int(d["nx"]), int(d["ny"])
        p.dx, p.dy, p.dt = float(d["dx"]), float(d["dy"]), float(d["dt"])
        for k in range(16):
            p.s[k] = float(d["s"][k])
        p.eq_version = int(d.get("eq_version", 1))
        p.modified = int(d.get("modified", 1))
        for k, b in enumerate(d["bc"]):
            p.bc[k] = BC[b] if isinstance(b, str) else int(b)
        wall = d.get("wall", [[1.0, 0.0, 0.0, 1.0]] * 4)
        for a in range(4):
            for b in range(4):
                p.wall[a][b] = float(wall[a][b])
        p.scheme = int(d.get("scheme", 0))
        return p


_lib = None


def load():
    """Load liblbm.so (raises if it has not been built).

    PyTorch is imported first: it brings its own HIP runtime, and the
    library must bind to that same runtime (loaded before PyTorch, the
    library would pull in a second runtime, whose streams do not see the
    device memory PyTorch allocates)."""
    global _lib
    if _lib is None:
        if not os.path.exists(LIB_PATH):
            raise RuntimeError("liblbm.so is not built: run __graft_entry__.build() (hipcc, gfx950)")
        import torch  # noqa: F401  (the HIP runtime the library shares)

        lib = ctypes.CDLL(LIB_PATH)
        P = ctypes.c_void_p
        pp = ctypes.POINTER(LbmParams)
        sigs = {
            "lbm_workspace_bytes": ([pp], ctypes.c_size_t),
            "lbm_create": ([pp, P, ctypes.c_size_t, P, ctypes.POINTER(P)], ctypes.c_int),
            "lbm_init": ([P, P, P, P, P], ctypes.c_int),
            "lbm_step": ([P, ctypes.c_int64], ctypes.c_int),
            "lbm_moments": ([P, P, P, P, P, P], ctypes.c_int),
            "lbm_get_f": ([P, P], ctypes.c_int),
            "lbm_set_f": ([P, P], ctypes.c_int),
            "lbm_check": ([P], ctypes.c_int),
            "lbm_set_variant": ([P, ctypes.c_int32], ctypes.c_int),
            "lbm_set_tile": ([P, ctypes.c_int32, ctypes.c_int32], ctypes.c_int),
            "lbm_tune": ([P, ctypes.c_int64, P, ctypes.c_size_t, ctypes.POINTER(ctypes.c_int32),
                          ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_double)], ctypes.c_int),
            "lbm_get_tile": ([P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
            "lbm_get_variant": ([P, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
            "lbm_set_store_mode": ([P, ctypes.c_int32], ctypes.c_int),
            "lbm_get_store_mode": ([P, ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
            "lbm_set_window": ([P, ctypes.c_int32, ctypes.c_int32, ctypes.c_int32], ctypes.c_int),
            "lbm_get_window": ([P, ctypes.POINTER(ctypes.c_int32), ctypes.POINTER(ctypes.c_int32),
                                ctypes.POINTER(ctypes.c_int32)], ctypes.c_int),
            "lbm_last_error": ([], ctypes.c_char_p),
            "lbm_destroy": ([P], None),
            "lbm_stream_copy": ([P, P, ctypes.c_int32, ctypes.c_int32, P], ctypes.c_int),
        }
        for name, (args, res) in sigs.items():
            fn = getattr(lib, name)
            fn.argtypes = args
            fn.restype = res
        _lib = lib
    return _lib


def _check(rc):
    if rc != 0:
        msg = load().lbm_last_error().decode()
        raise LbmError(rc, msg)


def _params(p):
    return p if isinstance(p, LbmParams) else LbmParams.from_dict(p)


def _ptr(t):
    if t is None:
        return None
    import torch

    assert t.is_cuda and t.dtype == torch.float64 and t.is_contiguous(), "expected a contiguous float64 CUDA tensor"
    return ctypes.c_void_p(t.data_ptr())


def _stream():
    import torch

    return ctypes.c_void_p(torch.cuda.current_stream().cuda_stream)


# ---------------------------------------------------------------------------
# The C ABI, one Python function per entry point.
# ---------------------------------------------------------------------------
def lbm_workspace_bytes(p):
    return int(load().lbm_workspace_bytes(ctypes.byref(_params(p))))


def lbm_create(p, workspace, stream=None):
    """workspace: uint8/float64 CUDA tensor of >= lbm_workspace_bytes(p) bytes."""
    p = _params(p)
    h = ctypes.c_void_p()
    nbytes = workspace.numel() * workspace.element_size()
    s = _stream() if stream is None else ctypes.c_void_p(stream)
    _check(load().lbm_create(ctypes.byref(p), ctypes.c_void_p(workspace.data_ptr()), nbytes, s, ctypes.byref(h)))
    return h


def lbm_init(h, rho, ux, uy, T):
    _check(load().lbm_init(h, _ptr(rho), _ptr(ux), _ptr(uy), _ptr(T)))


def lbm_step(h, nsteps):
    _check(load().lbm_step(h, int(nsteps)))


def lbm_moments(h, rho=None, ux=None, uy=None, T=None, p=None):
    _check(load().lbm_moments(h, _ptr(rho), _ptr(ux), _ptr(uy), _ptr(T), _ptr(p)))


def lbm_get_f(h, f):
    _check(load().lbm_get_f(h, _ptr(f)))


def lbm_set_f(h, f):
    _check(load().lbm_set_f(h, _ptr(f)))


def lbm_check(h):
    _check(load().lbm_check(h))


def lbm_set_variant(h, variant):
    _check(load().lbm_set_variant(h, int(variant)))


def lbm_set_tile(h, rows, waves=4):
    _check(load().lbm_set_tile(h, int(rows), int(waves)))


def lbm_tune(h, probe_steps, scratch=None):
    """Returns (rows, waves, best_ms)."""
    rows = ctypes.c_int32()
    waves = ctypes.c_int32()
    ms = ctypes.c_double()
    sp = ctypes.c_void_p(scratch.data_ptr()) if scratch is not None else None
    nbytes = scratch.numel() * scratch.element_size() if scratch is not None else 0
    _check(load().lbm_tune(h, int(probe_steps), sp, nbytes, ctypes.byref(rows), ctypes.byref(waves),
                           ctypes.byref(ms)))
    return rows.value, waves.value, ms.value


def lbm_get_tile(h):
    """Returns (rows, waves)."""
    rows = ctypes.c_int32()
    waves = ctypes.c_int32()
    _check(load().lbm_get_tile(h, ctypes.byref(rows), ctypes.byref(waves)))
    return rows.value, waves.value


def lbm_get_variant(h):
    v = ctypes.c_int32()
    _check(load().lbm_get_variant(h, ctypes.byref(v)))
    return v.value


def lbm_set_store_mode(h, nontemporal):
    _check(load().lbm_set_store_mode(h, int(nontemporal)))


def lbm_get_store_mode(h):
    v = ctypes.c_int32()
    _check(load().lbm_get_store_mode(h, ctypes.byref(v)))
    return v.value


def lbm_set_window(h, cols, rows, steps):
    _check(load().lbm_set_window(h, int(cols), int(rows), int(steps)))


def lbm_get_window(h):
    """Returns (cols, rows, steps) of the windowed kernel (variant 3)."""
    c, r, st = ctypes.c_int32(), ctypes.c_int32(), ctypes.c_int32()
    _check(load().lbm_get_window(h, ctypes.byref(c), ctypes.byref(r), ctypes.byref(st)))
    return c.value, r.value, st.value


def lbm_destroy(h):
    load().lbm_destroy(h)


def lbm_stream_copy(src, dst, nx, ny):
    """Diagnostic copy of 16 pitched planes with the step kernel's access
    pattern (src, dst: float64 device tensors of 16 * ny * pitch doubles)."""
    pitch = (int(nx) + 63) // 64 * 64
    n = 16 * int(ny) * pitch
    assert src.numel() >= n and dst.numel() >= n, "buffers need 16 * ny * pitch doubles"
    _check(load().lbm_stream_copy(_ptr(src), _ptr(dst), int(nx), int(ny), _stream()))


# ---------------------------------------------------------------------------
# Convenience owner of one problem: workspace tensor + handle.
# ---------------------------------------------------------------------------
class Simulation:
    def __init__(self, params, device="cuda"):
        import torch

        self.params = dict(params)
        self.nx, self.ny = int(params["nx"]), int(params["ny"])
        nbytes = lbm_workspace_bytes(params)
        if nbytes == 0:
            load()
            raise LbmError(-1, load().lbm_last_error().decode())
        # torch's caching allocator returns 512-byte aligned blocks
        self.workspace = torch.empty(nbytes, dtype=torch.uint8, device=device)
        assert self.workspace.data_ptr() % 256 == 0
        self.device = self.workspace.device
        self.handle = lbm_create(params, self.workspace)

    def _field(self, a):
        import torch

        if isinstance(a, np.ndarray):
            a = torch.from_numpy(np.ascontiguousarray(a, dtype=np.float64))
        return a.to(self.device, dtype=torch.float64).contiguous()

    def init(self, rho, ux, uy, T):
        tensors = [self._field(a) for a in (rho, ux, uy, T)]
        lbm_init(self.handle, *tensors)
        self._keep = tensors  # alive until the stream has consumed them

    def step(self, nsteps):
        lbm_step(self.handle, nsteps)

    def moments(self):
        import torch

        out = {k: torch.empty((self.ny, self.nx), dtype=torch.float64, device=self.device)
               for k in ("rho", "ux", "uy", "T", "p")}
        lbm_moments(self.handle, out["rho"], out["ux"], out["uy"], out["T"], out["p"])
        return out

    def get_f(self):
        import torch

        f = torch.empty((16, self.ny, self.nx), dtype=torch.float64, device=self.device)
        lbm_get_f(self.handle, f)
        return f

    def set_f(self, f):
        f = self._field(f)
        lbm_set_f(self.handle, f)
        self._keep = [f]

    def check(self):
        lbm_check(self.handle)

    def set_variant(self, v):
        lbm_set_variant(self.handle, v)

    def set_tile(self, rows, waves=4):
        lbm_set_tile(self.handle, rows, waves)

    def tile(self):
        return lbm_get_tile(self.handle)

    def variant(self):
        return lbm_get_variant(self.handle)

    def set_store_mode(self, nontemporal):
        lbm_set_store_mode(self.handle, nontemporal)

    def store_mode(self):
        return lbm_get_store_mode(self.handle)

    def set_window(self, cols, rows, steps):
        lbm_set_window(self.handle, cols, rows, steps)

    def window(self):
        return lbm_get_window(self.handle)

    def tune(self, probe_steps=20, keep_state=True):
        """Time the fused kernel's tile shapes and store modes and, where it
        applies, the windowed kernel's window shapes; keep the fastest
        (variant(), tile(), store_mode(), window() report the choice). With
        keep_state the state is saved to a scratch tensor and restored.
        Returns (rows, waves, best_ms) of the fastest fused tile and the best
        time over all candidates."""
        import torch

        scratch = None
        if keep_state:
            scratch = torch.empty(16 * self.ny * ((self.nx + 63) // 64 * 64), dtype=torch.float64, device=self.device)
        return lbm_tune(self.handle, probe_steps, scratch)

    def close(self):
        if getattr(self, "handle", None) is not None:
            lbm_destroy(self.handle)
            self.handle = None

    def __del__(self):
        try:
            self.close()
        except Exception:
            pass
