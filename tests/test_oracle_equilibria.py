"""Pins of the equilibrium moments, Eqs. (14a)-(14i), and of the initial state.

Each printed equilibrium moment equals the moment of the continuous 2-D
Maxwellian with density rho, velocity u and temperature T (R = 1):
f^eq_k = rho E[psi_k(u + sqrt(T) xi)], xi ~ N(0, I). The expectation is
computed here by tensor Gauss-Hermite quadrature, exact for polynomials of
degree < 2n. A dropped term, wrong power or transposed component in any of
the nine printed formulas fails this.
"""

import math

import numpy as np
import pytest

import oracle
from test_oracle_constants import _polys


def _maxwell_moments(rho, ux, uy, T, n=12):
    x, w = np.polynomial.hermite_e.hermegauss(n)
    w = w / math.sqrt(2.0 * math.pi)
    acc = np.zeros(16)
    for a, wa in zip(x, w):
        for b, wb in zip(x, w):
            acc += wa * wb * np.array(_polys(ux + math.sqrt(T) * a, uy + math.sqrt(T) * b))
    return rho * acc


STATES = [(1.0, 0.0, 0.0, 1.0), (1.0, 0.1, -0.05, 1.1), (0.37, -0.8, 0.45, 2.3), (5.0, 45.0, 0.0, 10.0),
          (0.1358, 0.0, 0.0, 1.0 / 0.1358), (2.0, 6.0, -1.5, 2.0)]


@pytest.mark.parametrize("state", STATES)
def test_printed_equilibria_are_maxwellian_moments(state):
    rho, ux, uy, T = state
    got = oracle.feq_moments(1, rho, ux, uy, T)
    want = _maxwell_moments(rho, ux, uy, T)
    degree = [0, 1, 1, 2, 2, 2, 3, 3, 3, 3, 4, 4, 4, 4, 5, 5]
    speed = 1.0 + abs(ux) + abs(uy) + math.sqrt(T)
    for k in [0, 1, 2, 3, 4, 5, 6, 7, 8, 9, 10, 12, 13]:
        scale = rho * speed ** degree[k]  # size of the terms that cancel in the moment
        assert abs(got[k] - want[k]) <= 1e-13 * scale, (k + 1, got[k], want[k])
    # version 1 leaves the three free moments at zero
    assert got[11] == 0.0 and got[14] == 0.0 and got[15] == 0.0


def test_free_moments_versions_2_and_3_symmetry():
    """Parity unpinned beyond symmetry: versions 2 and 3 differ only in the
    free moments 12, 15, 16; 15 and 16 are odd in (u_x, u_y) and vanish at rest."""
    for ver in (2, 3):
        q = oracle.feq_moments(ver, 1.3, 0.0, 0.0, 0.9)
        assert abs(q[14]) < 1e-14 and abs(q[15]) < 1e-14
        q1 = oracle.feq_moments(1, 1.3, 0.2, -0.1, 0.9)
        qv = oracle.feq_moments(ver, 1.3, 0.2, -0.1, 0.9)
        same = [k for k in range(16) if k not in (11, 14, 15)]
        np.testing.assert_array_equal(q1[same], qv[same])
    # version 2 at u_y = 0 has no f^16 (odd in u_y)
    assert oracle.feq_moments(2, 1.0, 0.3, 0.0, 1.0)[15] == 0.0


def test_init_reproduces_fields():
    rng = np.random.default_rng(3)
    ny, nx = 5, 7
    rho = rng.uniform(0.2, 3.0, (ny, nx))
    ux = rng.uniform(-1, 1, (ny, nx))
    uy = rng.uniform(-1, 1, (ny, nx))
    T = rng.uniform(0.3, 4.0, (ny, nx))
    from paper_1106_0785_amd import inputs

    for ver in (1, 2, 3):
        p = inputs.params(nx, ny, 0.01, 0.01, 1e-4, [1e3] * 16, ["periodic"] * 4, eq_version=ver)
        f = oracle.init(p, rho, ux, uy, T)
        np.testing.assert_allclose(f.sum(axis=0), rho, rtol=1e-13)
        m = oracle.moments(p, f)
        np.testing.assert_allclose(m["rho"], rho, rtol=1e-13)
        np.testing.assert_allclose(m["ux"], ux, atol=1e-13)
        np.testing.assert_allclose(m["uy"], uy, atol=1e-13)
        np.testing.assert_allclose(m["T"], T, rtol=1e-12)
        np.testing.assert_allclose(m["p"], rho * T, rtol=1e-12)


@pytest.mark.parametrize("state", STATES[:4] + [(0.8, 1.3, -0.7, 0.6)])
def test_version3_free_moments_are_sampled_maxwellian_moments(state):
    """Version 3 (Sec. II): f^eq_12, 15, 16 are the moments of f^max_i =
    rho/(2 pi T) exp(-|v_i - u|^2 / (2T)) sampled at the 16 velocities,
    computed here with the closed-form polynomials Re z^4, Re z^5, -Im z^5
    (z = v_x + i v_y) instead of the oracle's table of M."""
    rho, ux, uy, T = state
    V, _, _ = oracle.matrices()
    want = np.zeros(16)
    for vx, vy in V:
        fmax = rho / (2.0 * math.pi * T) * math.exp(-((vx - ux) ** 2 + (vy - uy) ** 2) / (2.0 * T))
        z = complex(vx, vy)
        want += fmax * np.array([0.0] * 11 + [(z ** 4).real, 0.0, 0.0, (z ** 5).real, -(z ** 5).imag])
    got = oracle.feq_moments(3, rho, ux, uy, T)
    scale = max(1e-300, rho / T)
    for k in (11, 14, 15):
        assert abs(got[k] - want[k]) <= 1e-13 * scale * 32 ** 2, (k + 1, got[k], want[k])


@pytest.mark.parametrize("version", [2, 3])
def test_free_moments_rotate_with_the_velocity(version):
    """A quarter turn u -> (-u_y, u_x) maps z -> i z, so the free moments must
    satisfy f^12(Ru) = f^12(u), f^15(Ru) = f^16(u), f^16(Ru) = -f^15(u): a
    wrong sign or coefficient in one of the printed version-2 forms fails."""
    for rho, ux, uy, T in [(1.3, 0.2, -0.1, 0.9), (0.6, -1.1, 0.7, 2.2), (2.0, 3.0, 1.0, 1.5)]:
        q = oracle.feq_moments(version, rho, ux, uy, T)
        r = oracle.feq_moments(version, rho, -uy, ux, T)
        tol = 1e-12 * max(1.0, np.max(np.abs(q)))
        assert abs(r[11] - q[11]) <= tol
        assert abs(r[14] - q[15]) <= tol
        assert abs(r[15] + q[14]) <= tol
