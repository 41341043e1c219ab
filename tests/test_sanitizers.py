"""The library's host code under AddressSanitizer and ThreadSanitizer, on the CPU: argument checks,
plans' host state, the serving loop with its arrival thread, first-fit arena, slots and staging
(virtual-clock executor), through the same tests as the plain build (test_server_fake.py,
test_abi.py). Each variant is built with host-only instrumentation (build.py --sanitize) and loaded
into a fresh interpreter with the clang runtime preloaded; any sanitizer report fails the run."""

import os
import subprocess
import sys

import pytest

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))
SUITES = [os.path.join(ROOT, "tests", "test_server_fake.py"), os.path.join(ROOT, "tests", "test_abi.py")]


@pytest.mark.parametrize("kind", ["address", "thread"])
def test_host_code_under_sanitizer(kind):
    sys.path.insert(0, ROOT)
    from paper_1802_06130_amd import build as B
    lib = B.build(sanitize=kind)
    env = dict(os.environ)
    env["MDN_LIB"] = lib
    env["LD_PRELOAD"] = B.sanitizer_runtime(kind)
    # the interpreter itself is not instrumented and keeps memory until exit by design
    env["ASAN_OPTIONS"] = "detect_leaks=0:abort_on_error=1"
    env["TSAN_OPTIONS"] = "halt_on_error=1:exitcode=66"
    r = subprocess.run([sys.executable, "-m", "pytest", "-q", "-x", "-p", "no:cacheprovider", "-m", "not gpu", *SUITES],
                       capture_output=True, text=True, timeout=900, cwd=ROOT, env=env)
    out = r.stdout + r.stderr
    assert "Sanitizer" not in out, out[-4000:]
    assert r.returncode == 0, out[-4000:]
    assert " passed" in out
