"""Generate lbm_consts.h: the velocity set and the shell-factorised moment
transform of the D2V16 model (Sec. II), as exact rationals.

The 16 velocities form four shells of four points each: axis shells of radius
1 and 2 (cyc(+-1,0), cyc(+-2,0)) and diagonal shells (+-1,+-1), (+-2,+-2).
On each shell, four "shell quantities" capture everything the moment basis
can see:
    sigma = sum of the four values,
    gx, gy = the v_x- and v_y-odd (dipole) combinations,
    q     = the quadrupole combination (v_x^2 - v_y^2 sign on axis shells,
            v_x v_y sign on diagonal shells).
Every row of M (the SO(2) polynomial basis psi_k evaluated at the
velocities) is then a combination of one kind of shell quantity across the
four shells, so f^ = M f splits into
    sigma-block (m1, m4, m11, m12), gx-block (m2, m7, m9, m15),
    gy-block (m3, m8, m10, m16), and two 2x2 quadrupole blocks
    (m5, m13 | axis shells) and (m6, m14 | diagonal shells).
M^-1 is the inverse of each block followed by the per-shell 4-point inverse.
This script derives the blocks from the polynomial basis, inverts them with
fractions, checks that the factorisation reproduces M and M^-1 exactly, and
writes the header. Run: python gen_consts.py [output]
"""

import os
import sys
from fractions import Fraction as F

# velocity order of Sec. II (columns of rows m2, m3)
VEL = [(1, 0), (0, 1), (-1, 0), (0, -1),
       (1, 1), (-1, 1), (-1, -1), (1, -1),
       (2, 0), (0, 2), (-2, 0), (0, -2),
       (2, 2), (-2, 2), (-2, -2), (2, -2)]


def psi(vx, vy):
    vx, vy = F(vx), F(vy)
    v2 = vx * vx + vy * vy
    # z^n = (vx + i vy)^n, real/imag parts by binomial expansion
    def zpow(n):
        re, im = F(1), F(0)
        for _ in range(n):
            re, im = re * vx - im * vy, re * vy + im * vx
        return re, im
    z3, z4, z5 = zpow(3), zpow(4), zpow(5)
    return [F(1), vx, vy, v2 / 2, vx * vx - vy * vy, vx * vy, vx * v2 / 2, vy * v2 / 2, z3[0], z3[1],
            v2 * v2 / 4, z4[0], (vx * vx - vy * vy) * v2, vx * vy * v2, z5[0], -z5[1]]


def matmul(a, b):
    return [[sum(a[i][k] * b[k][j] for k in range(len(b))) for j in range(len(b[0]))] for i in range(len(a))]


def inverse(a):
    n = len(a)
    m = [list(r) + [F(int(i == j)) for j in range(n)] for i, r in enumerate(a)]
    for c in range(n):
        p = next(r for r in range(c, n) if m[r][c] != 0)
        m[c], m[p] = m[p], m[c]
        d = m[c][c]
        m[c] = [x / d for x in m[c]]
        for r in range(n):
            if r != c and m[r][c] != 0:
                f = m[r][c]
                m[r] = [x - f * y for x, y in zip(m[r], m[c])]
    return [r[n:] for r in m]


M = [[psi(*VEL[i])[k] for i in range(16)] for k in range(16)]
MINV = inverse(M)

# Shell quantity transform S: f -> (sigma_s, gx_s, gy_s, q_s) for shells s = 0..3.
# Rows ordered: sigma0..3, gx0..3, gy0..3, q0..3.
SHELL_AXIS = [True, False, True, False]
S = [[F(0)] * 16 for _ in range(16)]
for s in range(4):
    base = 4 * s
    for j in range(4):
        vx, vy = VEL[base + j]
        sx = (vx > 0) - (vx < 0)
        sy = (vy > 0) - (vy < 0)
        S[0 + s][base + j] = F(1)
        S[4 + s][base + j] = F(sx)
        S[8 + s][base + j] = F(sy)
        S[12 + s][base + j] = F(sx * sx - sy * sy) if SHELL_AXIS[s] else F(sx * sy)
SINV = inverse(S)
A = matmul(M, SINV)  # moments = A * shell quantities

BLOCKS = {
    "SIG": ([0, 3, 10, 11], [0, 1, 2, 3]),
    "GX": ([1, 6, 8, 14], [4, 5, 6, 7]),
    "GY": ([2, 7, 9, 15], [8, 9, 10, 11]),
    "QA": ([4, 12], [12, 14]),  # axis-shell quadrupole: m5, m13 <- q of shells 0, 2
    "QD": ([5, 13], [13, 15]),  # diagonal-shell quadrupole: m6, m14 <- q of shells 1, 3
}

# check A is exactly block-structured
covered = set()
for name, (rows, cols) in BLOCKS.items():
    for r in rows:
        for c in range(16):
            if c not in cols:
                assert A[r][c] == 0, (name, r, c, A[r][c])
        covered.add(r)
assert covered == set(range(16))

blk = {}
blkinv = {}
for name, (rows, cols) in BLOCKS.items():
    b = [[A[r][c] for c in cols] for r in rows]
    blk[name] = b
    blkinv[name] = inverse(b)

# Reconstruct M^-1 from the factorisation and compare exactly.
AINV = [[F(0)] * 16 for _ in range(16)]
for name, (rows, cols) in BLOCKS.items():
    bi = blkinv[name]
    for a, c in enumerate(cols):
        for b_, r in enumerate(rows):
            AINV[c][r] = bi[a][b_]
assert matmul(SINV, AINV) == MINV
assert matmul(M, MINV) == [[F(int(i == j)) for j in range(16)] for i in range(16)]


def lit(x):
    x = F(x)
    if x.denominator == 1:
        return "%d.0" % x.numerator
    v = x.numerator / x.denominator
    assert F(v) == x, x  # every entry is dyadic or has an exact binary64 form
    return repr(v)


def lit_any(x):
    """Correctly rounded binary64 literal of a rational (17 significant digits)."""
    x = F(x)
    if x.denominator == 1:
        return "%d.0" % x.numerator
    # Python's true division of big ints is correctly rounded
    return "%.17g" % (x.numerator / x.denominator)


def emit_matrix(name, m, comment):
    rows = ",\n    ".join("{" + ", ".join(lit_any(v) for v in r) + "}" for r in m)
    return "// %s\nconstexpr double %s[%d][%d] = {\n    %s};\n" % (comment, name, len(m), len(m[0]), rows)


def main(out):
    mirror_x = [VEL.index((-vx, vy)) for vx, vy in VEL]
    mirror_y = [VEL.index((vx, -vy)) for vx, vy in VEL]
    lines = []
    lines.append("// Generated by gen_consts.py from the velocity set and the SO(2) polynomial\n"
                 "// basis of the D2V16 MRT model (Sec. II). Do not edit by hand.\n"
                 "#pragma once\n\nnamespace lbm {\n")
    lines.append("// Discrete velocities in the paper's order (columns of rows m2, m3 of M).\n")
    lines.append("constexpr int VX[16] = {%s};\n" % ", ".join(str(v[0]) for v in VEL))
    lines.append("constexpr int VY[16] = {%s};\n" % ", ".join(str(v[1]) for v in VEL))
    lines.append("// Velocity index after negating v_x (MIRROR_X) or v_y (MIRROR_Y).\n")
    lines.append("constexpr int MIRROR_X[16] = {%s};\n" % ", ".join(map(str, mirror_x)))
    lines.append("constexpr int MIRROR_Y[16] = {%s};\n\n" % ", ".join(map(str, mirror_y)))
    lines.append("// Shells: 0 axis r=1 (i=0..3), 1 diagonal r=1 (4..7), 2 axis r=2 (8..11),\n"
                 "// 3 diagonal r=2 (12..15). Within a shell the points run E,N,W,S (axis) or\n"
                 "// NE,NW,SW,SE (diagonal). Shell quantities: sigma = sum, gx/gy = dipole\n"
                 "// combinations (sign of v_x / v_y), q = quadrupole (sign of v_x^2-v_y^2 on\n"
                 "// axis shells, of v_x v_y on diagonal shells).\n\n")
    names = {"SIG": "moments m1, m4, m11, m12 <- sigma of shells 0..3",
             "GX": "moments m2, m7, m9, m15 <- gx of shells 0..3",
             "GY": "moments m3, m8, m10, m16 <- gy of shells 0..3",
             "QA": "moments m5, m13 <- q of shells 0, 2",
             "QD": "moments m6, m14 <- q of shells 1, 3"}
    for k in ["SIG", "GX", "GY", "QA", "QD"]:
        lines.append(emit_matrix("A_" + k, blk[k], "forward block: " + names[k]))
    lines.append("\n")
    for k in ["SIG", "GX", "GY", "QA", "QD"]:
        lines.append(emit_matrix("AINV_" + k, blkinv[k], "inverse block of A_" + k))
    lines.append("\n// Full M^-1 (row = velocity, column = moment), for host-side checks.\n")
    lines.append(emit_matrix("MINV_FULL", MINV, "M^-1, correctly rounded"))
    lines.append("\n}  // namespace lbm\n")
    text = "".join(lines)
    with open(out, "w") as fh:
        fh.write(text)


if __name__ == "__main__":
    here = os.path.dirname(os.path.abspath(__file__))
    main(sys.argv[1] if len(sys.argv) > 1 else os.path.join(here, "lbm_consts.h"))
