"""Seeded synthetic inputs shared by the tests, the smoke check and the benchmark.

This package only draws and renders test data (scenes, noise, image-size mixes,
arrival times, stand-in filter banks). It holds none of the denoiser's own
arithmetic, so both the FP64 oracle and the GPU library can be fed from it
without sharing any method code.
"""

from .scenes import (  # noqa: F401
    synth_scene,
    add_noise,
    noisy_pair,
    ragged_sizes,
    poisson_arrivals,
    random_bank_coeffs,
    SIGMAS_8BIT,
)
