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


def test_paper_configuration_table_matches_the_oracle():
    """The frame probe's table of the paper's configuration (Section 5) is the oracle's paper_setup."""
    sys.path.insert(0, ROOT)
    import bench
    import oracle as O
    for sigma, (L, rf, rg) in bench.PAPER_CONFIG.items():
        assert O.paper_setup(sigma) == (L, rf, rg, (16, 16, 16))


def test_gram_mfma_flop_counts_the_upper_triangle_tiles():
    """D = 98 plus the target pads to 4 tiles of 32; 10 of the 16 tiles are on or above the diagonal."""
    sys.path.insert(0, ROOT)
    import bench
    assert bench.gram_mfma_flop(98, 3, 1) == 2.0 * 10 * 32 * 32 * 3
    assert bench.gram_mfma_flop(25, 1, 7) == 2.0 * 1 * 32 * 32 * 7
    assert bench.gram_mfma_flop(147, 1, 1) == 2.0 * 15 * 32 * 32
