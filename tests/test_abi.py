"""The C-ABI library loads without a GPU, exports every entry point that
include/*.h declares, and validates problem descriptions on the host."""

import ctypes
import glob
import os
import re

import pytest

from paper_1106_0785_amd import inputs, lbm

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def _declared():
    names = []
    for h in glob.glob(os.path.join(ROOT, "include", "*.h")):
        text = open(h).read()
        text = re.sub(r"/\*.*?\*/", "", text, flags=re.S)
        names += re.findall(r"\b(lbm_[a-z0-9_]+)\s*\(", text)
    return sorted(set(names))


def test_every_declared_symbol_is_exported():
    lib = ctypes.CDLL(lbm.LIB_PATH)
    names = _declared()
    assert len(names) >= 10
    missing = [n for n in names if not hasattr(lib, n)]
    assert not missing, missing


def _bytes(p):
    return lbm.lbm_workspace_bytes(p)


def test_valid_problem_sizes_workspace():
    p, _, _ = inputs.couette(1.0)
    n = _bytes(p)
    pitch = 64
    assert n >= 2 * 16 * pitch * 64 * 8


@pytest.mark.parametrize(
    "change,needle",
    [
        ({"nx": 0}, "nx and ny"),
        ({"dt": 0.0}, "dt"),
        ({"dt": 1.0}, "unstable"),
        ({"eq_version": 4}, "eq_version"),
        ({"modified": 3}, "modified"),
        ({"bc": ["periodic", "specular", "periodic", "periodic"]}, "paired"),
        ({"bc": ["neq_wall", "neq_wall", "neq_wall", "neq_wall"]}, "both axes"),
        ({"nx": 1, "bc": ["specular", "specular", "neq_wall", "neq_wall"]}, "extent 1"),
        ({"scheme": 2}, "scheme"),
        ({"scheme": 1}, "scheme 1"),  # the Couette problem has NEQ walls
    ],
)
def test_invalid_problems_are_rejected(change, needle):
    p, _, _ = inputs.couette(1.0)
    p = dict(p, **change)
    assert _bytes(p) == 0
    assert needle in lbm.load().lbm_last_error().decode()


def test_rate_must_be_positive():
    p, _, _ = inputs.couette(1.0)
    s = list(p["s"])
    s[9] = 0.0
    assert _bytes(dict(p, s=s)) == 0
    assert "s_10" in lbm.load().lbm_last_error().decode()


def test_adjoint_form_rejects_the_limited_scheme():
    """The adjoint needs a differentiable step (minmod is not); the batched
    form takes the limited scheme (tile by tile, even for lines)."""
    import ctypes

    from paper_1106_0785_amd import autograd, batch

    p, _ = inputs.smooth_periodic(seed=1, nx=40, ny=1)
    p["scheme"] = 1
    assert lbm.lbm_workspace_bytes(p) > 0  # valid for the plain path
    q0 = dict(p, scheme=0)
    # a limited line is laid out like a tiled instance (pitched rows), a Lax-Wendroff one as a line
    assert batch.lbm_batch_workspace_bytes([p]) > batch.lbm_batch_workspace_bytes([q0]) > 0
    q = lbm.LbmParams.from_dict(p)
    assert autograd._lib().lbm_adjoint_workspace_bytes(ctypes.byref(q), 10, 0) == 0
    assert "scheme 0" in lbm.load().lbm_last_error().decode()


def test_batch_workspace_covers_lines_and_tiled_instances():
    """Host-side layout of the batched form: lines take 16 planes of their
    length rounded to 16 nodes, tiled (2-D, or periodic lines over 128 nodes)
    instances 16 planes of ny rows of nx rounded to 64 nodes; both arenas,
    the tuner's backup and the descriptors must fit."""
    from paper_1106_0785_amd import batch

    items = inputs.mixed_batch(seed=2, n=12)
    params = [p for _, p, _ in items]
    need = 0
    for p in params:
        tiled = (p["nx"] > 1 and p["ny"] > 1) or (p["ny"] == 1 and p["bc"][0] == "periodic" and p["nx"] > 128)
        need += 16 * 8 * (p["ny"] * ((p["nx"] + 63) // 64 * 64) if tiled else (p["nx"] * p["ny"] + 15) // 16 * 16)
    got = batch.lbm_batch_workspace_bytes(params)
    assert got >= 3 * need
    assert got < 3 * need + 4 * 1024 * 1024
    assert batch.lbm_batch_workspace_bytes([]) == 0


@pytest.mark.parametrize(
    "change,squarings,needle",
    [
        ({"scheme": 1}, 0, "scheme 0"),
        ({"eq_version": 0}, 0, "eq_version"),
        ({"modified": 5}, 0, "modified"),
        ({"dt": -1.0}, 0, "dt"),
        ({}, 61, "squarings"),
        ({}, -2, "squarings"),
    ],
)
def test_stability_tool_rejects_bad_sets_on_the_host(change, squarings, needle):
    """Rejected before any device work (the pointers are never touched)."""
    from paper_1106_0785_amd import stability

    lib = stability._lib()
    p = dict(inputs.params(1, 1, 1e-3, 1e-3, 1e-5, [1e5] * 16, ["periodic"] * 4), **change)
    ps, ss, n = stability._sets([p], [(1.0, 0.1, 0.0, 1.0)])
    fake = ctypes.c_void_p(1 << 20)  # 256-aligned, never dereferenced
    nbytes = stability.lbm_stability_workspace_bytes(1)
    rc = lib.lbm_stability_radius(ps, ss, 1, fake, 4, squarings, fake, nbytes, fake, None)
    assert rc == -1
    assert needle in lbm.load().lbm_last_error().decode()
    if not change:
        return
    rc = lib.lbm_stability_matrix(ps, ss, 1, fake, 4, fake, nbytes, fake, None)
    assert rc == -1


def test_stability_workspace_and_state_checks():
    from paper_1106_0785_amd import stability

    lib = stability._lib()
    assert stability.lbm_stability_workspace_bytes(0) == 0
    assert stability.lbm_stability_workspace_bytes(3) >= 3 * 5 * 256 * 8
    p = inputs.params(1, 1, 1e-3, 1e-3, 1e-5, [1e5] * 16, ["periodic"] * 4)
    fake = ctypes.c_void_p(1 << 20)
    ps, ss, n = stability._sets([p], [(1.0, 0.1, 0.0, -1.0)])
    assert lib.lbm_stability_radius(ps, ss, 1, fake, 4, 0, fake, 1 << 20, fake, None) == -1
    assert "T > 0" in lbm.load().lbm_last_error().decode()
    ps, ss, n = stability._sets([p], [(1.0, 0.1, 0.0, 1.0)])
    assert lib.lbm_stability_radius(ps, ss, 1, fake, 4, 0, fake, 16, fake, None) == -2
