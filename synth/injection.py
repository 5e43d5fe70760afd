"""Seeded synthetic stars and box-transit injection for injection-recovery
tests (the paper's Section 3.2 protocol: period 3 d, duration 3 h, depths
5 to 1000 ppm), standing in for its TESS sector 6 and Kepler Q5 stars, which
are not available here.  Input generation only: nothing of the estimate.

TESS-like stars: 27 d at 2-min cadence (19,440 samples) with a 1-day NaN gap
at mid-sector, white noise of 600-2000 ppm per cadence (around the paper's
quoted ~1000 ppm floor) and two starspot-like sinusoids (amplitude 0.1-5 ppt,
period 0.5-10 d).  Kepler-like stars: 90 d at 29.4-min cadence (4,408
samples), white noise of 50-200 ppm (around its quoted ~100 ppm floor), AR(1)
red noise (2-day correlation, 0.1-1 ppt) and one sinusoid (0.1-3 ppt, 5-30 d).
Every star has its own generator, SeedSequence([2604066020, 5 or 6, star]).
"""
from __future__ import annotations

import numpy as np
from scipy.signal import lfilter

from .lightcurves import HOUR, MIN, ROOT_SEED, _log_uniform

DEPTHS_PPM = (5, 50, 100, 200, 500, 1000)   # Tables 1-2
PERIOD_D = 3.0
DURATION_D = 3 * HOUR
MISSIONS = {
    "tess": dict(cfg=5, n=19440, dt=2 * MIN, W=361),
    "kepler": dict(cfg=6, n=4408, dt=29.4 * MIN, W=25),
}


def _rng(mission: str, star: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([ROOT_SEED, MISSIONS[mission]["cfg"], star]))


def star(mission: str, i: int):
    """(flux float32 without transits, time float64, W, transit epoch)."""
    m = MISSIONS[mission]
    rng = _rng(mission, i)
    n, dt = m["n"], m["dt"]
    t = np.arange(n, dtype=np.float64) * dt
    f = np.ones(n)
    if mission == "tess":
        sigma = _log_uniform(rng, 6e-4, 2e-3)
        for _ in range(2):
            f += _log_uniform(rng, 1e-4, 5e-3) * np.sin(2 * np.pi * t / rng.uniform(0.5, 10.0)
                                                       + rng.uniform(0, 2 * np.pi))
        f += rng.normal(0.0, sigma, n)
        gap = (t > t[-1] / 2 - 0.5) & (t < t[-1] / 2 + 0.5)
        f[gap] = np.nan
    else:
        sigma = _log_uniform(rng, 5e-5, 2e-4)
        phi = np.exp(-dt / 2.0)
        red_std = _log_uniform(rng, 1e-4, 1e-3)
        e = rng.normal(0.0, red_std * np.sqrt(1 - phi * phi), n)
        e[0] = rng.normal(0.0, red_std)
        f += lfilter([1.0], [1.0, -phi], e)
        f += _log_uniform(rng, 1e-4, 3e-3) * np.sin(2 * np.pi * t / rng.uniform(5.0, 30.0)
                                                    + rng.uniform(0, 2 * np.pi))
        f += rng.normal(0.0, sigma, n)
    epoch = rng.uniform(0.0, PERIOD_D)
    return f, t, m["W"], epoch


def in_transit(t, epoch, period=PERIOD_D, duration=DURATION_D):
    """Samples inside the box transits (centred at epoch + k * period)."""
    ph = np.mod(t - epoch + duration / 2, period)
    return ph < duration


def injected(mission: str, i: int, depth_ppm: float, duration_d: float = DURATION_D,
             period_d: float = PERIOD_D):
    """(flux float32 with the transits multiplied in, time, W, in-transit mask)."""
    f, t, W, epoch = star(mission, i)
    mask = in_transit(t, epoch, period_d, duration_d)
    g = f * np.where(mask, 1.0 - depth_ppm * 1e-6, 1.0)
    return g.astype(np.float32), t, W, mask
