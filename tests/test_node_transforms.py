"""CPU checks of the HIP library's per-node arithmetic (host build of the same
header): the shell-factorised transforms and their transposes equal the
oracle's dense M and M^-1, and the dual-number derivative of the equilibrium
moments equals central differences."""

import ctypes
import os
import subprocess

import numpy as np
import pytest

import oracle

HERE = os.path.dirname(os.path.abspath(__file__))
SRC = os.path.join(HERE, "native", "node_host.cpp")
OUT = os.path.join(HERE, "native", "_build", "libnode_host.so")


@pytest.fixture(scope="module")
def lib():
    os.makedirs(os.path.dirname(OUT), exist_ok=True)
    if not os.path.exists(OUT) or os.path.getmtime(OUT) < max(
            os.path.getmtime(SRC), *[os.path.getmtime(os.path.join(HERE, "..", "paper_1106_0785_amd", "csrc", h))
                                     for h in ("lbm_node.h", "lbm_dual.h", "lbm_consts.h")]):
        subprocess.check_call(["/opt/rocm/bin/hipcc", "--offload-arch=gfx950", "-O2", "-std=c++17", "-fPIC", "-shared",
                               "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops", SRC, "-o", OUT],
                              stderr=subprocess.DEVNULL)
    L = ctypes.CDLL(OUT)
    return L


def _call(fn, *arrays):
    return fn(*[a.ctypes.data_as(ctypes.c_void_p) if isinstance(a, np.ndarray) else a for a in arrays])


def test_transforms_match_dense_matrices(lib):
    _, M, Minv = oracle.matrices()
    rng = np.random.default_rng(0)
    for _ in range(20):
        x = rng.standard_normal(16)
        out = np.zeros(16)
        _call(lib.host_moments, x, out)
        np.testing.assert_allclose(out, M @ x, rtol=0, atol=1e-12 * np.abs(M).max())
        _call(lib.host_f_from_moments, x, out)
        np.testing.assert_allclose(out, Minv @ x, rtol=0, atol=1e-13)
        _call(lib.host_mt, x, out)
        np.testing.assert_allclose(out, M.T @ x, rtol=0, atol=1e-12 * np.abs(M).max())
        _call(lib.host_minvt, x, out)
        np.testing.assert_allclose(out, Minv.T @ x, rtol=0, atol=1e-13)


@pytest.mark.parametrize("version", [1, 2, 3])
def test_equilibrium_derivatives_match_central_differences(lib, version):
    rng = np.random.default_rng(version)
    for _ in range(5):
        rho = rng.uniform(0.3, 3.0)
        u = rng.uniform(-0.8, 0.8, 2)
        T = rng.uniform(0.4, 2.5)
        c = np.array([rho, rho * u[0], rho * u[1], rho * (T + 0.5 * (u @ u))])
        q0 = np.zeros(16)
        _call(lib.host_feq, ctypes.c_int(version), c, q0)
        # the library's equilibria equal the oracle's
        np.testing.assert_allclose(q0, oracle.feq_moments(version, rho, u[0], u[1], T), rtol=1e-13, atol=1e-13)
        for a in range(4):
            dq = np.zeros(16)
            _call(lib.host_feq_dir, ctypes.c_int(version), c, ctypes.c_int(a), dq)
            h = 1e-6 * max(1.0, abs(c[a]))
            cp, cm = c.copy(), c.copy()
            cp[a] += h
            cm[a] -= h
            qp, qm = np.zeros(16), np.zeros(16)
            _call(lib.host_feq, ctypes.c_int(version), cp, qp)
            _call(lib.host_feq, ctypes.c_int(version), cm, qm)
            fd = (qp - qm) / (2 * h)
            np.testing.assert_allclose(dq, fd, rtol=1e-6, atol=1e-7 * (1 + np.abs(fd).max()))
