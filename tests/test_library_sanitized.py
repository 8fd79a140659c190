"""The library's host tests again, against a build whose host code runs under
AddressSanitizer and UndefinedBehaviorSanitizer (tests/sanitized_build.py):
an out-of-bounds access, a use after free, a signed overflow or a bad shift
in plan lowering, the planner, the variant space and search, the cost
model's host side or the run-time source generation aborts the run. No GPU
is used (planning contexts)."""
import os
import subprocess
import sys

import pytest

import sanitized_build

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
HOST_TESTS = ["test_library_host.py", "test_planner_host.py", "test_jit_host.py", "test_optimizer_host.py"]


def test_library_host_code_under_sanitizers():
    rt = sanitized_build.asan_runtime()
    if rt is None:
        pytest.skip("no clang ASan runtime in the ROCm toolchain here")
    lib = sanitized_build.build()
    env = dict(os.environ, LD_PRELOAD=rt, HAWK_LIBRARY=lib, ASAN_OPTIONS="detect_leaks=0:abort_on_error=1",
               UBSAN_OPTIONS="halt_on_error=1:print_stacktrace=1")
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider"] +
                       [os.path.join(ROOT, "tests", t) for t in HOST_TESTS],
                       cwd=ROOT, env=env, capture_output=True, text=True, timeout=900)
    out = r.stdout + r.stderr
    assert r.returncode == 0, out[-4000:]
    assert "AddressSanitizer" not in out and "runtime error" not in out, out[-4000:]
    assert " passed" in out
