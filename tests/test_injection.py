"""Host logic of the injection-recovery harness (CPU): the depth read-off,
the error metric, and a small end-to-end run with the FP64 oracle as the
detrender (Section 3.2 protocol)."""
from __future__ import annotations

import numpy as np
import pytest

from paper_2604_06602_amd import injection as inj
from synth import injection as si


def test_recovered_depth_is_exact_on_a_noiseless_star_with_its_true_trend():
    t = np.arange(5000) * (2 / 1440)
    mask = si.in_transit(t, 0.7)
    level = 1.0 + 0.01 * np.sin(t)
    flux = level * np.where(mask, 1 - 500e-6, 1.0)
    d = inj.recovered_depth(flux / level, mask)
    assert d == pytest.approx(500e-6, rel=1e-9)
    assert inj.percent_error(d, 500) == pytest.approx(0.0, abs=1e-6)
    # an overall offset of the detrended flux is not a depth error
    assert inj.recovered_depth(1.003 * flux / level, mask) == pytest.approx(500e-6, rel=1e-9)


def test_transit_geometry():
    t = np.arange(0, 30, 1 / 1440)
    mask = si.in_transit(t, 1.0)
    # 10 transits of 3 h in 30 days, centred on 1 + 3k
    assert mask.sum() == pytest.approx(10 * 180, abs=10)
    assert mask[np.searchsorted(t, 1.0)] and not mask[np.searchsorted(t, 1.1)]


def test_stars_are_seeded_and_shaped():
    f1, t1, W1, m1 = si.injected("tess", 3, 200)
    f2, t2, W2, m2 = si.injected("tess", 3, 200)
    assert np.array_equal(f1, f2, equal_nan=True) and W1 == 361 and f1.size == 19440
    assert np.isnan(f1).sum() == 720                      # the mid-sector gap
    fk, tk, Wk, mk = si.injected("kepler", 3, 200)
    assert Wk == 25 and fk.size == 4408 and not np.isnan(fk).any()
    # the injected dip is multiplicative with the given depth
    base, _, _, _ = si.star("kepler", 3)
    assert np.allclose(fk[mk], (base[mk] * (1 - 200e-6)).astype(np.float32))


def test_harness_with_the_oracle_small(oracle_lib):
    """A few Kepler-like stars end to end with the oracle as detrender: at a
    signal-dominated depth every setting recovers it to tens of percent, at
    5 ppm all are noise-limited."""
    def detrend(flux, time, lengths, W, alpha, c, scale):
        tr, _ = oracle_lib.detrend_batch(flux, time, lengths, W, alpha=alpha, c=c, scale=scale)
        return flux / tr
    table, errors = inj.run("kepler", 8, depths=(5, 1000), detrend=detrend)
    for m in inj.METHODS:
        assert table[m][1000] < 20.0
        assert table[m][5] > 50.0
