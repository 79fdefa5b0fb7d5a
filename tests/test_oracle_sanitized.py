"""The oracle's own tests against a build of the oracle instrumented with
AddressSanitizer and UndefinedBehaviorSanitizer (host code; g++). Any
out-of-bounds access, use of freed memory or undefined arithmetic in the
oracle ends the run with the sanitizer's report. The long physics runs (the
shock-tube exact solutions, the Couette refinement study) are left out: they
exercise the same code paths as the short tests for many more steps."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SRC = os.path.join(ROOT, "oracle", "lbm_oracle.cpp")
LIB = os.path.join(ROOT, "oracle", "liblbm_oracle_sanitized.so")

FILES = ["test_oracle_constants.py", "test_oracle_equilibria.py", "test_oracle_invariants.py",
         "test_oracle_complex_step.py", "test_oracle_limited.py", "test_oracle_modification.py",
         "test_oracle_stability.py", "test_oracle_transport.py"]
SKIP = "not sharp_sod and not couette and not matches_exact"


def _build():
    if not os.path.exists(LIB) or os.path.getmtime(LIB) < os.path.getmtime(SRC):
        flags = ["-O1", "-g", "-fno-omit-frame-pointer", "-fsanitize=" + "address,undefined",
                 "-fno-sanitize-recover=undefined"]
        tmp = LIB + ".tmp%d" % os.getpid()
        subprocess.check_call(["g++", "-std=c++17", "-fopenmp", "-fPIC", "-shared"] + flags + [SRC, "-o", tmp])
        os.replace(tmp, LIB)


def test_oracle_tests_pass_under_sanitizers():
    _build()
    runtime = subprocess.check_output(["g++", "-print-file-name=libasan.so"], text=True).strip()
    assert os.path.exists(runtime), runtime
    env = dict(os.environ)
    env.update({"LD_PRELOAD": runtime, "LBM_ORACLE_LIB": LIB, "OMP_NUM_THREADS": "4",
                "ASAN_OPTIONS": "detect_leaks=0:halt_on_error=1",
                "UBSAN_OPTIONS": "halt_on_error=1:print_stacktrace=1"})
    cmd = [sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu", "-k", SKIP]
    cmd += [os.path.join(ROOT, "tests", f) for f in FILES]
    r = subprocess.run(cmd, env=env, cwd=ROOT, capture_output=True, text=True, timeout=900)
    tail = (r.stdout + r.stderr)[-4000:]
    assert r.returncode == 0, tail
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr, tail
    assert " passed" in r.stdout, tail
