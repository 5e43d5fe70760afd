"""White-noise bias check of Sections 2.4 and 4.1, shared by the oracle pin
and the GPU test: the mean trend offset, in units of the noise, over many
independent full windows of a flat white-noise star."""
from __future__ import annotations

import math

import numpy as np

# Monte-Carlo trend offsets on white noise (W = 361, 5 iterations, sigma =
# 1000 ppm), in units of sigma, from an independent Monte-Carlo of Eqs. 1-4:
# +0.41 (alpha 2, c 5), +1.63 (alpha 10, c 2.5), about +0.002 (alpha 1).  The
# paper's own offsets on flat TESS-like stars (Section 2.4: about 451 ppm at
# the default, Section 3.1: 1857 ppm at the aggressive setting, Section 4.1:
# -2 ppm symmetric) sit at 1.10 and 1.14 times these at sigma = 1000 ppm, i.e.
# one common per-star noise near 1.1e-3.  `printed` is the precision the
# values are quoted to.
BIAS_MC = [  # alpha, c, offset / sigma, printed
    (1.0, 5.0, 0.002, 0.0005),
    (2.0, 5.0, 0.41, 0.005),
    (10.0, 2.5, 1.63, 0.005),
]
BIAS_WINDOWS = 40000


def bias_offsets(detrend_at):
    """Mean trend offset and its standard error (units of sigma) over
    BIAS_WINDOWS disjoint, hence independent, full windows of white noise."""
    import synth
    sigma = 1e-3
    flux, time, idx = synth.white_noise_windows(BIAS_WINDOWS, 361, sigma)
    out = {}
    for a, c, _, _ in BIAS_MC:
        d = (np.asarray(detrend_at(flux, time, 361, idx, a, c), np.float64) - 1.0) / sigma
        out[a] = (float(d.mean()), float(d.std(ddof=1) / np.sqrt(d.size)))
    return out


def assert_offsets_match(got):
    """Each offset within half a unit of the printed last digit plus three
    combined standard errors (this run's and, at equal size, the reference
    Monte-Carlo's) of its value; the ordering of Section 3.1."""
    for a, c, want, printed in BIAS_MC:
        mean, se = got[a]
        assert abs(mean - want) <= printed + 3 * math.sqrt(2) * se, (a, c, mean, se, want)
    assert got[10.0][0] > 3.5 * got[2.0][0] > 0
