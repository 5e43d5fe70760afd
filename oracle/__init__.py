"""UMI oracle -- TEST INFRASTRUCTURE ONLY.

A plain FP64 CPU implementation of the UMI estimate (arXiv 2604.06602,
Section 2) used to check the GPU library.  Only the tests, the smoke check and
the benchmark's CPU-baseline leg may import it; the product path never does.
It shares no code with the GPU library.
"""
from .oracle import (  # noqa: F401
    build,
    detrend,
    detrend_at,
    detrend_batch,
    mad_scale,
    median,
    normalise,
    SCALES,
    segments,
    upper_scale,
    weight,
    window,
    window_from_cadence,
)
