"""Pins of the oracle's constant tables (Sec. II: velocity set, matrix M).

The velocity set and the rows of M are checked against their closed-form
definitions (the SO(2) polynomial basis the paper says M is built from), and
M^-1 against an exact rational inverse computed here with fractions.
"""

from fractions import Fraction

import numpy as np

import oracle


def _polys(vx, vy):
    """The 16 basis polynomials psi_k(v) whose values at the velocities form
    the rows m1..m16 (z = vx + i vy)."""
    z = complex(vx, vy)
    v2 = vx * vx + vy * vy
    return [
        1.0,
        vx,
        vy,
        v2 / 2.0,
        vx * vx - vy * vy,
        vx * vy,
        vx * v2 / 2.0,
        vy * v2 / 2.0,
        (z ** 3).real,
        (z ** 3).imag,
        v2 * v2 / 4.0,
        (z ** 4).real,
        (vx * vx - vy * vy) * v2,
        vx * vy * v2,
        (z ** 5).real,
        -(z ** 5).imag,
    ]


def test_velocity_set_is_fig1():
    v, m, _ = oracle.matrices()
    # cyc(+-1,0), (+-1,+-1), cyc(+-2,0), (+-2,+-2) in groups of four
    groups = [set(map(tuple, v[4 * g: 4 * g + 4].astype(int).tolist())) for g in range(4)]
    assert groups[0] == {(1, 0), (0, 1), (-1, 0), (0, -1)}
    assert groups[1] == {(1, 1), (-1, 1), (-1, -1), (1, -1)}
    assert groups[2] == {(2, 0), (0, 2), (-2, 0), (0, -2)}
    assert groups[3] == {(2, 2), (-2, 2), (-2, -2), (2, -2)}
    # the order is the one the rows m2 (v_x) and m3 (v_y) print
    np.testing.assert_array_equal(m[1], v[:, 0])
    np.testing.assert_array_equal(m[2], v[:, 1])


def test_rows_are_so2_polynomials():
    v, m, _ = oracle.matrices()
    for i in range(16):
        np.testing.assert_allclose(m[:, i], _polys(v[i, 0], v[i, 1]), rtol=0, atol=1e-12)


def test_inverse_is_exact_rational_inverse():
    v, m, minv = oracle.matrices()
    n = 16
    a = [[Fraction(m[r, c]).limit_denominator(8) for c in range(n)] + [Fraction(int(r == c)) for c in range(n)]
         for r in range(n)]
    for col in range(n):
        piv = next(r for r in range(col, n) if a[r][col] != 0)
        a[col], a[piv] = a[piv], a[col]
        d = a[col][col]
        a[col] = [x / d for x in a[col]]
        for r in range(n):
            if r != col and a[r][col] != 0:
                f = a[r][col]
                a[r] = [x - f * y for x, y in zip(a[r], a[col])]
    exact = np.array([[float(a[r][n + c]) for c in range(n)] for r in range(n)])
    # the oracle's long-double Gauss-Jordan rounds to within one ulp of each
    # non-zero entry and leaves at most long-double residue in the exact zeros
    assert np.all(np.abs(minv - exact) <= np.maximum(np.spacing(np.abs(exact)), 1e-18))
    np.testing.assert_allclose(m @ minv, np.eye(n), atol=5e-15)
    # denominators divide 960
    assert all((a[r][n + c] * 960).denominator == 1 for r in range(n) for c in range(n))


def test_mirror_symmetry_of_tables():
    """Negating v_x permutes the velocities and flips the sign of exactly the
    rows odd in v_x (m2, m7, m9, m15; m6, m14 and m10, m16 mix components)."""
    v, m, _ = oracle.matrices()
    perm = [int(np.where((v[:, 0] == -v[i, 0]) & (v[:, 1] == v[i, 1]))[0][0]) for i in range(16)]
    for k in range(16):
        row = m[k]
        mirrored = row[perm]
        assert np.array_equal(mirrored, row) or np.array_equal(mirrored, -row)
