"""The library's host code under AddressSanitizer and UndefinedBehaviorSanitizer (CPU only):
the C ABI's argument checks (tests/test_abi.py, run against the sanitized build in a child
process with the sanitizer runtimes preloaded) and the NNQP of the LASSO weight step on random
problems (tests/host/nnqp_check.cpp, which also checks the KKT conditions). Any sanitizer report
aborts the child and fails the test."""
import os
import shutil
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST = os.path.join(ROOT, "tests", "host")
LIB = os.path.join(ROOT, "paper_2009_05473_amd", "libsfw.so")

pytestmark = pytest.mark.skipif(shutil.which("g++") is None or not os.path.exists(LIB),
                                reason="needs g++ and a built libsfw")


def _env(extra):
    env = dict(os.environ)
    env.update(extra)
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["UBSAN_OPTIONS"] = "halt_on_error=1:print_stacktrace=1"
    return env


def _san():
    sys.path.insert(0, HOST)
    import build_sanitized
    return build_sanitized


def test_nnqp_under_sanitizers():
    exe = _san().build_nnqp_check()
    r = subprocess.run([exe], capture_output=True, text=True, timeout=300, env=_env({}))
    assert r.returncode == 0, r.stdout + r.stderr
    assert r.stdout.startswith("ok ")


def test_abi_checks_under_sanitizers():
    san = _san()
    lib = san.build_library()
    env = _env({"SFW_LIB_PATH": lib, "LD_PRELOAD": " ".join(san.runtimes())})
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-p", "no:cacheprovider",
                        os.path.join(ROOT, "tests", "test_abi.py")],
                       capture_output=True, text=True, timeout=600, env=env, cwd=ROOT)
    assert r.returncode == 0, (r.stdout + r.stderr)[-4000:]
    assert "ERROR: AddressSanitizer" not in r.stderr and "runtime error" not in r.stderr
