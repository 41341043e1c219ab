"""MI355X (gfx950) implementation of the trainable multiscale adaptive-filter denoiser
(arXiv 1802.06130): HIP kernels behind the C ABI in include/mdn.h, bound here with ctypes."""

from ._lib import (  # noqa: F401
    F16, F32, GRAY, RGB, YCC,
    Bank, Level, MdnError,
    apply_level, denoise, denoise_workspace_size, header_functions, image, lib,
    pyramid_build, select_filters,
    GRAM_BF16X3, GRAM_F32, X_CROSS_CHANNEL, X_PER_CHANNEL, Gram, level_features, level_thresholds,
    quantiles, train_accumulate, train_multiscale, train_single, train_solve, Plan,
)
