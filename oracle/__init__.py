"""FP64 CPU oracle for the trainable multiscale denoiser (arXiv 1802.06130).

TEST INFRASTRUCTURE ONLY. This package is a plain, slow, obviously-correct
NumPy float64 implementation of what the GPU library computes. Only the tests,
the smoke check and the CPU-baseline leg of the benchmark may import it; the
GPU library never imports, links or calls it, and it shares no code with the
GPU library (no kernels, headers, tables or constant generators).
"""

from .mdn_oracle import *  # noqa: F401,F403
from .mdn_oracle import __all__  # noqa: F401
