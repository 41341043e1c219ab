"""The benchmark's command line on the CPU: a request for more than one GPU ends at once with a message
(the library has no multi-GPU path) and a non-zero status, before anything touches a device."""

import os
import subprocess
import sys

ROOT = os.path.dirname(os.path.dirname(os.path.abspath(__file__)))


def test_more_than_one_gpu_is_refused():
    r = subprocess.run([sys.executable, os.path.join(ROOT, "bench.py"), "--gpus", "2"], capture_output=True,
                       text=True, timeout=120, cwd=ROOT)
    assert r.returncode != 0
    assert "multi-GPU" in (r.stdout + r.stderr)
