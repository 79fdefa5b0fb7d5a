"""ctypes wrapper of the C++ oracle library (test infrastructure only).

Every array crossing this wrapper is a host numpy float64 array. Fields are
[ny][nx]; distributions are [16][ny][nx] in the paper's velocity order.
"""

import ctypes
import os
import subprocess

import numpy as np

_HERE = os.path.dirname(os.path.abspath(__file__))
_SRC = os.path.join(_HERE, "lbm_oracle.cpp")
_LIB = os.path.join(_HERE, "liblbm_oracle.so")
# The same source built with fused multiply-adds: a second rounding of the
# same arithmetic, used only to measure how strongly a problem amplifies
# rounding differences (the noise floor of any parity comparison).
_LIB_FMA = os.path.join(_HERE, "liblbm_oracle_fma.so")
# ... and with every dense sum taken in reverse index order.
_LIB_REV = os.path.join(_HERE, "liblbm_oracle_rev.so")
# ... and built -O3 -march=native for the host it runs on: the CPU baseline
# of the benchmark times this variant (the parity reference stays the -O2 one).
_LIB_NATIVE = os.path.join(_HERE, "liblbm_oracle_native.so")
_VARIANTS = {"plain": _LIB, "fma": _LIB_FMA, "reversed": _LIB_REV, "native": _LIB_NATIVE}
_EXTRA = {"plain": [], "fma": ["-mfma", "-ffp-contract=fast"], "reversed": ["-DORACLE_REVERSED_SUMS"],
          "native": ["-O3", "-march=native"]}

BC_CODES = {"periodic": 0, "zero_gradient": 1, "specular": 2, "neq_wall": 3, "dirichlet_eq": 4}


class OracleParams(ctypes.Structure):
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
            p.bc[k] = BC_CODES[b] if isinstance(b, str) else int(b)
        wall = d.get("wall", [[1.0, 0.0, 0.0, 1.0]] * 4)
        for a in range(4):
            for b in range(4):
                p.wall[a][b] = float(wall[a][b])
        p.scheme = int(d.get("scheme", 0))
        return p


def lib_path():
    return _LIB


def build(force=False, variants=("plain", "fma", "reversed")):
    """Compile the oracle with g++ (plain -O2, OpenMP over nodes), and the
    other builds of the same source (fused multiply-adds, reversed sums; the
    -O3 -march=native build is made where it is first used, on the host that
    runs it)."""
    for v in variants:
        path = _VARIANTS[v]
        if force or not os.path.exists(path) or os.path.getmtime(path) < os.path.getmtime(_SRC):
            tmp = path + ".tmp%d" % os.getpid()
            cmd = ["g++", "-O2", "-std=c++17", "-fopenmp", "-fPIC", "-shared"] + _EXTRA[v] + [_SRC, "-o", tmp]
            subprocess.check_call(cmd)
            os.replace(tmp, path)
    return _LIB


_libs = {}
# A different build of the same source to load in place of the plain one
# (a path; used to run the oracle's tests against an instrumented build).
_OVERRIDE = os.environ.get("LBM_ORACLE_LIB")


def _load(variant="plain"):
    if variant not in _libs:
        if variant == "plain" and _OVERRIDE:
            path = _OVERRIDE
        else:
            build(variants=(variant,), force=(variant == "native"))
            path = _VARIANTS[variant]
        lib = ctypes.CDLL(path)
        P = ctypes.POINTER(ctypes.c_double)
        pp = ctypes.POINTER(OracleParams)
        lib.oracle_matrices.argtypes = [P, P, P]
        lib.oracle_feq_moments.argtypes = [ctypes.c_int] + [ctypes.c_double] * 4 + [P]
        lib.oracle_node_equilibrium_complex.argtypes = [ctypes.c_int, P, P, P, P, P]
        lib.oracle_feq_moments_complex.argtypes = [ctypes.c_int, P, P, P, P]
        lib.oracle_init.argtypes = [pp, P, P, P, P, P]
        lib.oracle_moments.argtypes = [pp, P, P, P, P, P, P]
        lib.oracle_run.argtypes = [pp, P, ctypes.c_int64, P, ctypes.c_int]
        lib.oracle_init_complex.argtypes = [pp] + [P] * 10
        lib.oracle_run_complex.argtypes = [pp, P, P, P, ctypes.c_int64, P, P, ctypes.c_int]
        lib.oracle_moments_complex.argtypes = [pp, P, P] + [P] * 8
        lib.oracle_max_threads.argtypes = []
        _libs[variant] = lib
    return _libs[variant]


def _ptr(a):
    if a is None:
        return None
    assert a.dtype == np.float64 and a.flags["C_CONTIGUOUS"]
    return a.ctypes.data_as(ctypes.POINTER(ctypes.c_double))


def _f64(a):
    return np.ascontiguousarray(a, dtype=np.float64)


def _params(p):
    return p if isinstance(p, OracleParams) else OracleParams.from_dict(p)


def max_threads():
    return int(_load().oracle_max_threads())


def matrices():
    """(V [16,2], M [16,16], M^-1 [16,16]) as used by the oracle."""
    lib = _load()
    v = np.zeros((16, 2))
    m = np.zeros((16, 16))
    mi = np.zeros((16, 16))
    lib.oracle_matrices(_ptr(v), _ptr(m), _ptr(mi))
    return v, m, mi


def feq_moments(version, rho, ux, uy, T):
    out = np.zeros(16)
    rc = _load().oracle_feq_moments(int(version), float(rho), float(ux), float(uy), float(T), _ptr(out))
    if rc:
        raise ValueError("oracle_feq_moments rejected its arguments")
    return out


def node_equilibrium_complex(version, f):
    """For one node's complex distributions f (16): (complex f^eq moments
    [16], complex (rho, u_x, u_y, T))."""
    f = np.asarray(f, dtype=np.complex128)
    fr, fi = _f64(f.real), _f64(f.imag)
    qr, qi, mac = np.zeros(16), np.zeros(16), np.zeros(8)
    if _load().oracle_node_equilibrium_complex(int(version), _ptr(fr), _ptr(fi), _ptr(qr), _ptr(qi), _ptr(mac)):
        raise ValueError("oracle_node_equilibrium_complex rejected its arguments")
    return qr + 1j * qi, mac[0::2] + 1j * mac[1::2]


def feq_moments_complex(version, state):
    """Equilibrium moments [16] (complex) at a complex state (rho, u_x, u_y, T)."""
    v = np.asarray(state, dtype=np.complex128)
    vr, vi = _f64(v.real), _f64(v.imag)
    qr, qi = np.zeros(16), np.zeros(16)
    if _load().oracle_feq_moments_complex(int(version), _ptr(vr), _ptr(vi), _ptr(qr), _ptr(qi)):
        raise ValueError("oracle_feq_moments_complex rejected its arguments")
    return qr + 1j * qi


def init(p, rho, ux, uy, T):
    p = _params(p)
    rho, ux, uy, T = (_f64(a) for a in (rho, ux, uy, T))
    f = np.zeros((16, p.ny, p.nx))
    if _load().oracle_init(ctypes.byref(p), _ptr(rho), _ptr(ux), _ptr(uy), _ptr(T), _ptr(f)):
        raise ValueError("oracle_init rejected its arguments")
    return f


def moments(p, f):
    """dict with rho, ux, uy, T, p."""
    p = _params(p)
    f = _f64(f)
    out = {k: np.zeros((p.ny, p.nx)) for k in ("rho", "ux", "uy", "T", "p")}
    rc = _load().oracle_moments(
        ctypes.byref(p), _ptr(f), _ptr(out["rho"]), _ptr(out["ux"]), _ptr(out["uy"]), _ptr(out["T"]), _ptr(out["p"])
    )
    if rc:
        raise ValueError("oracle_moments rejected its arguments")
    return out


def run(p, f, nsteps, nthreads=None, variant="plain"):
    """variant "fma" / "reversed": the same arithmetic rounded differently
    (fused multiply-adds / dense sums in reverse order), to measure how far
    FP64 rounding alone moves a problem's result."""
    p = _params(p)
    f = _f64(f)
    out = np.empty_like(f)
    nt = max_threads() if nthreads is None else int(nthreads)
    if _load(variant).oracle_run(ctypes.byref(p), _ptr(f), int(nsteps), _ptr(out), nt):
        raise ValueError("oracle_run rejected its arguments")
    return out


def init_complex(p, rho, ux, uy, T):
    p = _params(p)
    args = []
    for a in (rho, ux, uy, T):
        a = np.asarray(a)
        args += [_f64(a.real), _f64(a.imag)]
    fr = np.zeros((16, p.ny, p.nx))
    fi = np.zeros((16, p.ny, p.nx))
    if _load().oracle_init_complex(ctypes.byref(p), *[_ptr(a) for a in args], _ptr(fr), _ptr(fi)):
        raise ValueError("oracle_init_complex rejected its arguments")
    return fr + 1j * fi


def run_complex(p, f, nsteps, s_im=None, nthreads=None, variant="plain"):
    p = _params(p)
    f = np.asarray(f)
    fr, fi = _f64(f.real), _f64(f.imag)
    sim = _f64(np.zeros(16) if s_im is None else s_im)
    outr = np.empty_like(fr)
    outi = np.empty_like(fr)
    nt = max_threads() if nthreads is None else int(nthreads)
    if _load(variant).oracle_run_complex(ctypes.byref(p), _ptr(sim), _ptr(fr), _ptr(fi), int(nsteps), _ptr(outr),
                                         _ptr(outi), nt):
        raise ValueError("oracle_run_complex rejected its arguments")
    return outr + 1j * outi


def moments_complex(p, f):
    p = _params(p)
    f = np.asarray(f)
    fr, fi = _f64(f.real), _f64(f.imag)
    bufs = [np.zeros((p.ny, p.nx)) for _ in range(8)]
    if _load().oracle_moments_complex(ctypes.byref(p), _ptr(fr), _ptr(fi), *[_ptr(b) for b in bufs]):
        raise ValueError("oracle_moments_complex rejected its arguments")
    names = ("rho", "ux", "uy", "T")
    return {n: bufs[2 * i] + 1j * bufs[2 * i + 1] for i, n in enumerate(names)}
