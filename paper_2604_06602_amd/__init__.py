"""UMI sliding-window asymmetric robust detrending on MI355X (gfx950).

The estimate of arXiv 2604.06602 (Section 2) -- window median, upper-RMS
scale, asymmetric Tukey-bisquare iterations -- at every sample of every light
curve, computed by hand-written HIP kernels behind a small C ABI
(include/umi.h).  This package is the thin Python binding over that library
plus the batching helpers and the serving loop built on it.
"""
from ._lib import (  # noqa: F401
    MAX_WINDOW,
    MODE_PER_CURVE,
    MODE_PERSISTENT,
    PRESETS,
    SCALES,
    LaunchOptions,
    Plan,
    UmiError,
    debug_inject_error,
    detrend,
    detrend_batch,
    detrend_batch_into,
    detrend_batch_noalloc_into,
    detrend_gather_into,
    host_copy_many,
    copy_async,
    COPY_H2D,
    COPY_D2H,
    COPY_KERNEL,
    last_error,
    release,
    set_tuning,
    version,
    window_from_cadence,
)
