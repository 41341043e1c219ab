"""MI355X (gfx950) implementation of the trainable multiscale adaptive-filter denoiser
(arXiv 1802.06130): HIP kernels behind the C ABI in include/mdn.h, bound here with ctypes."""

from ._lib import (  # noqa: F401
    F16, F32, GRAY, RGB, YCC, SELECT_COARSE, SELECT_LUMA, SELECT_RGB,
    Bank, Level, MdnError,
    apply_level, denoise, denoise_noalloc, denoise_workspace_size, NOALLOC_SCRATCH_BYTES, header_functions, image, lib,
    pyramid_build, select_filters, selector_dtype, dihedral, augment_pairs,
    GRAM_BF16X3, GRAM_F32, X_CROSS_CHANNEL, X_PER_CHANNEL, Gram, level_features, level_thresholds,
    quantiles, train_accumulate, train_multiscale, train_single, train_solve, Plan,
    EXEC_FAKE, EXEC_HIP, FAKE_FAIL_DOWNLOAD, FAKE_FAIL_LAUNCH, FAKE_FAIL_TICK, FAKE_FAIL_UPLOAD, FAKE_STALL,
    MDN_ECANCELED, MDN_EDEVICE, MDN_EINVAL, MDN_ENOMEM, MDN_ENOTSUP, MDN_ETIMEOUT, MDN_OK, Server,
)
