"""Host-side check of the windowed kernel's index arithmetic (no GPU).

Each workgroup holds a window of the grid in LDS (one thread per node) and
advances it up to h steps per launch. An axis no longer than the window is
held whole; a longer one is cut into windows overlapping by h nodes on each
cut side (periodic: periodic images; otherwise clipped to the domain), each
writing its middle w - 2 h nodes. This restates that arithmetic and walks
every window and thread for narrow grids (the default shapes) and for cut
two-dimensional shapes, with every boundary kind, and checks: LDS and stored
indices in range, the thread count within the launch bound, every node
written by exactly one window, and every written node at least h nodes from
a cut side (exact after up to h steps); a written NEQ wall node's fluid
neighbour too, since the wall takes its value of the same step (cut sides
on a walled axis overlap by h + 1)."""

import itertools

import pytest

PER, ZG, SPEC, NEQ, DIR = 0, 1, 2, 3, 4
SMALL_NODES = 512


def _resolve(i, n, lo, hi):
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


def _axis(length, w, h, walls):
    halo = h + (1 if walls else 0)  # a wall node takes its neighbour's value of the same step
    if length <= w:
        return dict(w=length, v=length, nwin=1, whole=True, halo=halo)
    v = w - 2 * halo
    if v < 1:
        return None  # the library rejects the shape
    return dict(w=w, v=v, nwin=(length + v - 1) // v, whole=False, halo=halo)


def _span(a, win, length, per):
    if a["whole"]:
        return dict(s=0, n=length, o=0, v=length, lo=False, hi=False)
    o = win * a["v"]
    s, e = o - a["halo"], o + a["v"] + a["halo"]
    if not per:
        s, e = max(s, 0), min(e, length)
    return dict(s=s, n=e - s, o=o, v=a["v"], lo=per or s > 0, hi=per or e < length)


def _nbr(sp, w, g, d, length, bc):
    w2 = w + d
    if 0 <= w2 < sp["n"]:
        return w2
    if (d < 0 and sp["lo"]) or (d > 0 and sp["hi"]):
        return w
    return _resolve(g + d, length, bc[0], bc[1]) - sp["s"]


def _check(nx, ny, wc, wr, h, bx, by):
    ax, ay = _axis(nx, wc, h, bx[0] == NEQ), _axis(ny, wr, h, by[0] == NEQ)
    if ax is None or ay is None:
        return
    assert ax["w"] * ay["w"] <= SMALL_NODES
    xper, yper = bx[0] == PER, by[0] == PER
    written = {}
    for b in range(ax["nwin"] * ay["nwin"]):
        sx = _span(ax, b % ax["nwin"], nx, xper)
        sy = _span(ay, b // ax["nwin"], ny, yper)
        assert 1 <= sx["n"] <= ax["w"] and 1 <= sy["n"] <= ay["w"]
        for t in range(sx["n"] * sy["n"]):
            xw, yw = t % sx["n"], t // sx["n"]
            xv, yv = sx["s"] + xw, sy["s"] + yw
            xg = xv % nx if xper else xv
            yg = yv % ny if yper else yv
            assert 0 <= xg < nx and 0 <= yg < ny
            for d in (1, -1):
                lx = _nbr(sx, xw, xg, d, nx, bx)
                ly = _nbr(sy, yw, yg, d, ny, by)
                assert 0 <= lx < sx["n"] and 0 <= ly < sy["n"]
            # a wall node's value comes from its fluid neighbour in the same step
            nbx, nby = xw, yw
            if by[0] == NEQ and yg in (0, ny - 1):
                nby = yw + 1 if yg == 0 else yw - 1
                assert 0 <= nby < sy["n"]
            elif bx[0] == NEQ and xg in (0, nx - 1):
                nbx = xw + 1 if xg == 0 else xw - 1
                assert 0 <= nbx < sx["n"]
            if sx["o"] <= xv < sx["o"] + sx["v"] and 0 <= xv < nx and sy["o"] <= yv < sy["o"] + sy["v"] and 0 <= yv < ny:
                written[(xg, yg)] = written.get((xg, yg), 0) + 1
                for lx, ly in ((xw, yw), (nbx, nby)):  # the node, and the node its value comes from
                    assert not (sx["lo"] and lx < h) and not (sx["hi"] and lx >= sx["n"] - h)
                    assert not (sy["lo"] and ly < h) and not (sy["hi"] and ly >= sy["n"] - h)
    assert len(written) == nx * ny and set(written.values()) == {1}


BCS = [(PER, PER), (ZG, ZG), (SPEC, SPEC), (DIR, ZG), (NEQ, NEQ), (SPEC, DIR)]


@pytest.mark.parametrize("ny", [1, 2, 3, 4, 7, 8, 9, 13, 16])
def test_narrow_default_windows(ny):
    """The default shape of grids with <= 16 rows: every row, 64 columns
    (32 when ny > 8), h = columns / 8."""
    wc = 64 if ny <= 8 else 32
    n_min = SMALL_NODES // ny + 1  # the windowed kernel takes nx ny > 512
    for nx in sorted({n_min, n_min + 1, n_min + 47, 2 * n_min + 5, 2000}):
        for bx in BCS:
            by = (PER, PER) if bx[0] == NEQ else (SPEC, SPEC)
            if ny < 3 and by[0] != PER:
                by = (PER, PER)
            _check(nx, ny, wc, ny, wc // 8, bx, by)


@pytest.mark.parametrize("wc,wr,h", [(32, 16, 2), (16, 32, 3), (64, 8, 1), (8, 8, 3)])
def test_cut_windows(wc, wr, h):
    """Windows cut along both axes, every pair of boundary kinds (NEQ walls
    on one axis only)."""
    for (nx, ny), bx, by in itertools.product([(100, 41), (37, 90), (64, 64)], BCS, BCS):
        if bx[0] == NEQ and by[0] == NEQ:
            continue
        _check(nx, ny, wc, wr, h, bx, by)


@pytest.mark.parametrize("shape", [(23, 37, 32, 16, 2, "y"), (193, 3, 64, 3, 8, "x"), (193, 5, 64, 5, 8, "x")])
def test_written_wall_nodes_have_exact_neighbours(shape):
    """Shapes where a window writes a wall node whose fluid neighbour lies h
    nodes from a cut side: exact only with the extra node of overlap."""
    nx, ny, wc, wr, h, axis = shape
    walls, other = (NEQ, NEQ), (PER, PER)
    if axis == "y":
        _check(nx, ny, wc, wr, h, other, walls)
    else:
        _check(nx, ny, wc, wr, h, walls, other)
