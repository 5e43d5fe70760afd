"""Seeded synthetic light curves shaped like the paper's TESS and Kepler data.

This module generates inputs only: it holds none of the estimator's
arithmetic, and both the GPU path and the oracle's tests draw from it.
"""
from .lightcurves import (  # noqa: F401
    CONFIGS,
    Batch,
    config_batch,
    curve_config0,
    curve_for,
    draw_config3_curve,
    poisson_arrivals,
    white_noise_windows,
)
