"""Build liblbm.so (HIP, gfx950) in-tree with hipcc.

The constants header is regenerated from the velocity set and polynomial
basis first (gen_consts.py checks the factorisation exactly)."""

import os
import subprocess
import sys

HERE = os.path.dirname(os.path.abspath(__file__))
CSRC = os.path.join(HERE, "csrc")
ROOT = os.path.dirname(HERE)
LIB = os.path.join(HERE, "liblbm.so")
SOURCES = ["lbm_api.hip", "lbm_batch.hip", "lbm_adjoint.hip", "lbm_stability.hip"]

HIPCC = os.environ.get("HIPCC", "/opt/rocm/bin/hipcc")
FLAGS = [
    "--offload-arch=gfx950",
    "-O3",
    "-std=c++17",
    "-fPIC",
    "-shared",
    "-Xclang", "-target-feature", "-Xclang", "-packed-fp32-ops",
    "-I", os.path.join(ROOT, "include"),
]


def sources():
    return [os.path.join(CSRC, s) for s in SOURCES]


def build(verbose=False, extra=()):
    subprocess.check_call([sys.executable, os.path.join(CSRC, "gen_consts.py")])
    tmp = LIB + ".tmp"
    cmd = [HIPCC] + FLAGS + list(extra) + sources() + ["-o", tmp]
    if verbose:
        print(" ".join(cmd), flush=True)
    subprocess.check_call(cmd)
    os.replace(tmp, LIB)
    return LIB


if __name__ == "__main__":
    build(verbose=True, extra=sys.argv[1:])
