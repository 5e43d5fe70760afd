"""Injection-recovery on the GPU path (Section 3.2 protocol, Tables 1-2):
the qualitative claims the paper draws from its tables, checked on seeded
synthetic TESS- and Kepler-like stars.  The assertions are orderings the
paper states, never stored numbers:

  * far below the per-cadence noise (5 ppm) every setting is noise-limited;
  * well above it the asymmetric default beats the symmetric reference, and
    the aggressive setting (alpha 10, c 2.5) recovers deep transits best.
"""
from __future__ import annotations

import pytest

pytestmark = pytest.mark.gpu

STARS = 400


@pytest.fixture(scope="module")
def tables():
    import torch
    if not torch.cuda.is_available():
        pytest.skip("no GPU")
    from paper_2604_06602_amd import injection as inj
    return {m: inj.run(m, STARS)[0] for m in ("tess", "kepler")}


def test_noise_limited_at_5ppm(tables):
    for mission, table in tables.items():
        for m, row in table.items():
            assert row[5] > 100.0, (mission, m, row[5])


def test_tess_asymmetry_helps_deep_transits(tables):
    t = tables["tess"]
    assert t["umi_default"][1000] < t["symmetric"][1000]
    assert t["umi_default"][1000] < t["symmetric_mad"][1000]
    assert t["umi_aggressive"][1000] < t["umi_default"][1000]
    assert t["umi_aggressive"][500] < t["symmetric"][500]


def test_kepler_asymmetry_helps_from_200ppm(tables):
    k = tables["kepler"]
    for d in (200, 500):
        assert k["umi_aggressive"][d] < k["umi_default"][d] < k["symmetric"][d], (d, k)
        assert k["umi_default"][d] < k["symmetric_mad"][d]


def test_errors_fall_with_depth_above_the_noise(tables):
    for mission, table in tables.items():
        for m, row in table.items():
            assert row[1000] < row[200] < row[50], (mission, m, row)


def test_long_transits_need_a_longer_window():
    """Section 4.2: with the 0.5-day window (W = 361 at 2 min) the depth of a
    transit longer than about 5 hours is underestimated; a 1.5-day
    window_length (W = 1081 by the rule of Section 2) recovers a 10-hour
    transit far better."""
    from paper_2604_06602_amd import _lib
    from paper_2604_06602_amd import injection as inj
    W_long = _lib.window_from_cadence(2 / 1440, 1.5)
    assert W_long == 1081
    default = {"umi_default": inj.METHODS["umi_default"]}
    short, _ = inj.run("tess", 200, depths=(1000,), methods=default, duration_d=10 / 24)
    long_, _ = inj.run("tess", 200, depths=(1000,), methods=default, duration_d=10 / 24,
                       W=W_long)
    three_h, _ = inj.run("tess", 200, depths=(1000,), methods=default)
    assert short["umi_default"][1000] > 2 * long_["umi_default"][1000]
    assert short["umi_default"][1000] > 2 * three_h["umi_default"][1000]
