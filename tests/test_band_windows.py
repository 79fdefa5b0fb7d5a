"""Host-side check of the narrow-grid kernel's window indexing (no GPU).

The kernel gives each workgroup a window of wc columns by all ny rows in LDS
(wc = 64 for ny <= 8, else 32; h = wc / 8 steps per launch; v = wc - 2 h
columns written per window). This walks every window and thread of the
kernel's index arithmetic, restated here, for narrow shapes and every x
boundary kind, and checks: LDS and stored indices in range, the thread count
within the launch bound, each column written by exactly one window, and every
written node at least h columns from a cut side (so it is exact after up to h
steps)."""

import pytest

PER, ZG, SPEC, NEQ, DIR = 0, 1, 2, 3, 4
SMALL_NODES = 512


def _resolve(i, n, lo, hi):
    """Source index of stencil point i on an axis of n nodes (ghost rules)."""
    if i < 0:
        if lo == PER:
            return ((i % n) + n) % n
        if lo == SPEC:
            return min(-1 - i, n - 1)
        return 0
    if i >= n:
        if hi == PER:
            return i % n
        if hi == SPEC:
            return max(2 * n - 1 - i, 0)
        return n - 1
    return i


def _geom(nx, ny):
    wc = 64 if ny <= 8 else 32
    h = wc // 8
    v = wc - 2 * h
    return wc, h, v, (nx + v - 1) // v


def _check(nx, ny, bx):
    wc, h, v, nwin = _geom(nx, ny)
    xper = bx[0] == PER
    threads = (wc * ny + 63) // 64 * 64
    assert threads <= SMALL_NODES
    written = [0] * nx
    for win in range(nwin):
        x0 = win * v
        xs, xe = x0 - h, x0 + v + h
        if not xper:
            xs, xe = max(xs, 0), min(xe, nx)
        ncols = xe - xs
        assert 1 <= ncols <= wc
        lo_cut, hi_cut = xper or xs > 0, xper or xe < nx
        for t in range(ncols * ny):
            xw, y = t % ncols, t // ncols
            xv = xs + xw
            xg = ((xv % nx) + nx) % nx if xper else xv
            assert 0 <= xg < nx
            for d in (1, -1):
                w2 = xw + d
                if 0 <= w2 < ncols:
                    col = w2
                elif (d < 0 and lo_cut) or (d > 0 and hi_cut):
                    col = xw
                else:
                    col = _resolve(xg + d, nx, bx[0], bx[1]) - xs
                assert 0 <= col < ncols
                for yy in (y - 1, y + 1):
                    assert 0 <= _resolve(yy, ny, SPEC, SPEC) * ncols + col < ncols * ny
            if bx[0] == NEQ and xg in (0, nx - 1):
                assert 0 <= (xw + 1 if xg == 0 else xw - 1) < ncols
            if x0 <= xv < x0 + v and 0 <= xv < nx:
                if y == 0:
                    written[xg] += 1
                assert not (lo_cut and xw < h) and not (hi_cut and xw >= ncols - h)
    assert written == [1] * nx


BCS = [(PER, PER), (ZG, ZG), (SPEC, SPEC), (DIR, ZG), (NEQ, NEQ), (SPEC, DIR)]


@pytest.mark.parametrize("ny", [1, 2, 3, 4, 7, 8, 9, 13, 16])
def test_band_windows(ny):
    n_min = SMALL_NODES // ny + 1  # the narrow-grid kernel takes nx ny > 512
    for nx in sorted({n_min, n_min + 1, n_min + 17, n_min + 47, 2 * n_min + 5, 2000, 4097}):
        for bx in BCS:
            _check(nx, ny, bx)
