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


def test_spread_reports_the_percentiles_of_the_timings():
    sys.path.insert(0, ROOT)
    import bench
    d = bench.spread(list(range(101)), "t")
    assert d == {"p10": 10.0, "p50": 50.0, "p90": 90.0, "p99": 99.0, "what": "t"}


def test_quality_items_are_8bit_noisy_views_of_one_scene():
    """A quality-run item: the clean scene in [0, 1] and one noisy observation per noise level, each a
    multiple of 1/255 in [0, 1] (to float32 rounding) whose error against the scene has about the level's deviation."""
    sys.path.insert(0, ROOT)
    import numpy as np
    import bench
    u, zs = bench._make_quality_item((8001, 321, 481))
    assert u.shape == (3, 321, 481) and float(u.min()) >= 0.0 and float(u.max()) <= 1.0
    assert len(zs) == len(bench.QUALITY_SIGMAS)
    for g, z in zip(bench.QUALITY_SIGMAS, zs):
        q = z.astype(np.float64) * 255.0
        assert np.abs(q - np.round(q)).max() < 1e-4 and q.min() >= 0 and q.max() <= 255   # float32 k / 255
        inner = (u > 0.25) & (u < 0.75)          # away from the clamp
        sd = float(np.std((z.astype(np.float64) - u)[inner])) * 255.0
        assert abs(sd - g) < 0.05 * g + 0.5, (g, sd)
    noisy_psnr = [bench._psnr(z, u) for z in zs]
    assert noisy_psnr[0] > noisy_psnr[1] > noisy_psnr[2]
