"""Seeded synthetic light-curve workloads.

Each curve is drawn from its own generator,
``np.random.default_rng(SeedSequence([2604066020, config, curve_id]))``, so any
subset of a workload is reproducible on its own.  Time is in days from 0 at a
uniform cadence; flux is float32 around 1.0, time is float64.  Invalid samples
are NaN in the flux (time stays finite).

The five workloads stand in for the paper's TESS sector 6 and Kepler Q5 data
(Sections 3.2 and 3.5), which are not available here:

  0  one TESS-like curve, 20,000 samples at 2 min, W=361;
  1  1,000 TESS-sector curves of 18,000 samples at 2 min, W=361, each with a
     1-day NaN gap in the middle;
  2  2,000 Kepler-like curves at 29.4 min, lengths U[40k, 70k], W=25, white
     plus AR(1) red noise;
  3  10,000 mixed curves at 2 min, lengths log-uniform 1,000..120,000, W drawn
     from {25, 121, 361, 721}, 5 % of samples NaN in 1-48 h gaps;
  4  a serving stream: Poisson arrivals of curves drawn like workload 3.
"""
from __future__ import annotations

from dataclasses import dataclass, field

import numpy as np
from scipy.signal import lfilter

ROOT_SEED = 2604066020
MIN = 1.0 / 1440.0
HOUR = 1.0 / 24.0

CONFIGS = {
    0: dict(name="tess_single_20k_w361", n_curves=1, dt=2 * MIN),
    1: dict(name="tess_batch_1000x18k_w361", n_curves=1000, dt=2 * MIN),
    2: dict(name="kepler_ragged_2000x40k-70k_w25", n_curves=2000, dt=29.4 * MIN),
    3: dict(name="mixed_ragged_10000x1k-120k_wmix", n_curves=10000, dt=2 * MIN),
    4: dict(name="serving_poisson_mixed", n_curves=None, dt=2 * MIN),
}
MIXED_W = (25, 121, 361, 721)


def _rng(cfg: int, curve_id: int) -> np.random.Generator:
    return np.random.default_rng(np.random.SeedSequence([ROOT_SEED, cfg, curve_id]))


def _log_uniform(rng, lo, hi, size=None):
    return np.exp(rng.uniform(np.log(lo), np.log(hi), size))


def _sinusoids(rng, t, n_terms=3, amp=1e-3, pmin=1.0, pmax=5.0):
    out = np.zeros_like(t)
    for _ in range(n_terms):
        period = rng.uniform(pmin, pmax)
        phase = rng.uniform(0.0, 2 * np.pi)
        out += amp * np.sin(2 * np.pi * t / period + phase)
    return out


def _flares(rng, t, n=5, amp=5e-3, tau=10 * MIN):
    out = np.zeros_like(t)
    t0s = rng.uniform(t[0], t[-1], n) if t.size else []
    for t0 in t0s:
        m = t >= t0
        out[m] += amp * np.exp(-(t[m] - t0) / tau)
    return out


def _periodic_box(rng, t, depth_lo, depth_hi, dur_h=(1.0, 8.0), per_d=(1.0, 13.0)):
    depth = _log_uniform(rng, depth_lo, depth_hi)
    dur = rng.uniform(*dur_h) * HOUR
    period = rng.uniform(*per_d)
    epoch = rng.uniform(0.0, period)
    in_tr = np.mod(t - epoch, period) < dur
    return -depth * in_tr


def curve_config0() -> tuple[np.ndarray, np.ndarray, int]:
    """Workload 0: flux, time, W."""
    rng = _rng(0, 0)
    n, dt = 20000, CONFIGS[0]["dt"]
    t = np.arange(n, dtype=np.float64) * dt
    f = 1.0 + _sinusoids(rng, t) + rng.normal(0.0, 1e-3, n)
    centre = rng.uniform(t[0], t[-1])
    f -= 1e-3 * (np.abs(t - centre) < 1.5 * HOUR)
    f += _flares(rng, t)
    return f.astype(np.float32), t, 361


def _tess_like(rng, n, dt, depth_lo, depth_hi):
    t = np.arange(n, dtype=np.float64) * dt
    f = 1.0 + _sinusoids(rng, t) + rng.normal(0.0, 1e-3, n)
    f += _periodic_box(rng, t, depth_lo, depth_hi)
    f += _flares(rng, t)
    return f, t


def curve_config1(i: int):
    rng = _rng(1, i)
    n, dt = 18000, CONFIGS[1]["dt"]
    f, t = _tess_like(rng, n, dt, 1e-4, 5e-2)
    gap = 720  # one day at 2-min cadence, centred mid-sector
    g0 = n // 2 - gap // 2
    f[g0:g0 + gap] = np.nan
    return f.astype(np.float32), t, 361


def curve_config2(i: int):
    rng = _rng(2, i)
    dt = CONFIGS[2]["dt"]
    n = int(rng.integers(40000, 70001))
    t = np.arange(n, dtype=np.float64) * dt
    sigma_w = _log_uniform(rng, 5e-5, 1e-3)
    phi = np.exp(-dt / 2.0)  # AR(1) with a 2-day correlation time
    red_std = 1e-3
    e = rng.normal(0.0, red_std * np.sqrt(1 - phi * phi), n)
    e[0] = rng.normal(0.0, red_std)
    red = lfilter([1.0], [1.0, -phi], e)
    f = 1.0 + red + rng.normal(0.0, sigma_w, n)
    f += _periodic_box(rng, t, 1e-4, 1e-2)
    # W for a 0.5-day window at 29.4 min cadence (the rule gives 25)
    return f.astype(np.float32), t, 25


def _nan_gaps(rng, f, frac=0.05, dur_h=(1.0, 48.0), dt=2 * MIN):
    n = f.size
    target = int(round(frac * n))
    mask = np.zeros(n, bool)
    guard = 0
    while mask.sum() < target and guard < 10000:
        guard += 1
        length = max(1, int(round(rng.uniform(*dur_h) * HOUR / dt)))
        start = int(rng.integers(0, n))
        seg = np.arange(start, min(n, start + length))
        new = seg[~mask[seg]]
        need = target - int(mask.sum())
        mask[new[:need]] = True
    f[mask] = np.nan
    return f


def draw_config3_curve(rng: np.random.Generator):
    dt = CONFIGS[3]["dt"]
    n = int(round(_log_uniform(rng, 1000, 120000)))
    W = int(MIXED_W[int(rng.integers(0, len(MIXED_W)))])
    f, t = _tess_like(rng, n, dt, 1e-4, 5e-2)
    f = _nan_gaps(rng, f, dt=dt)
    return f.astype(np.float32), t, W


def curve_config3(i: int):
    return draw_config3_curve(_rng(3, i))


_CURVE_FN = {1: curve_config1, 2: curve_config2, 3: curve_config3}


def curve_for(cfg: int, i: int):
    """Curve ``i`` of workload ``cfg``: (flux float32, time float64, W)."""
    if cfg == 0:
        if i != 0:
            raise IndexError("workload 0 has one curve")
        return curve_config0()
    if cfg == 4:
        return draw_config3_curve(_rng(4, i))
    return _CURVE_FN[cfg](i)


@dataclass
class Batch:
    """A packed ragged batch: curve b is [offsets[b], offsets[b] + lengths[b])."""
    flux: np.ndarray
    time: np.ndarray
    lengths: np.ndarray
    W: np.ndarray
    name: str = ""
    curve_ids: list = field(default_factory=list)

    @property
    def offsets(self) -> np.ndarray:
        return np.concatenate([[0], np.cumsum(self.lengths)[:-1]]).astype(np.int64)

    @property
    def n_curves(self) -> int:
        return int(self.lengths.size)

    @property
    def n_samples(self) -> int:
        return int(self.flux.size)

    def curve(self, b: int):
        o = int(self.offsets[b])
        L = int(self.lengths[b])
        return self.flux[o:o + L], self.time[o:o + L], int(self.W[b])


def pack(curves, name="", ids=None) -> Batch:
    fl = [c[0] for c in curves]
    tl = [c[1] for c in curves]
    lengths = np.array([x.size for x in fl], dtype=np.int64)
    W = np.array([c[2] for c in curves], dtype=np.int32)
    flux = np.concatenate(fl).astype(np.float32) if fl else np.zeros(0, np.float32)
    time = np.concatenate(tl).astype(np.float64) if tl else np.zeros(0, np.float64)
    return Batch(flux, time, lengths, W, name, list(ids or range(len(curves))))


def config_batch(cfg: int, n_curves: int | None = None, first: int = 0) -> Batch:
    """Workload ``cfg`` as a packed batch; ``n_curves`` takes a prefix subset."""
    if cfg == 0:
        return pack([curve_config0()], CONFIGS[0]["name"], [0])
    total = CONFIGS[cfg]["n_curves"]
    if n_curves is None:
        if total is None:
            raise ValueError("workload 4 is a stream; give n_curves")
        n_curves = total
    ids = list(range(first, first + n_curves))
    return pack([curve_for(cfg, i) for i in ids], CONFIGS[cfg]["name"], ids)


def poisson_arrivals(rate_hz: float, duration_s: float, seed: int = 0) -> np.ndarray:
    """Open-loop Poisson arrival times (seconds) for the serving stream."""
    rng = np.random.default_rng(np.random.SeedSequence([ROOT_SEED, 4, 10**6 + seed]))
    n_max = int(rate_hz * duration_s * 1.5 + 50)
    gaps = rng.exponential(1.0 / rate_hz, n_max)
    t = np.cumsum(gaps)
    while t[-1] < duration_s:
        t = np.concatenate([t, t[-1] + np.cumsum(rng.exponential(1.0 / rate_hz, n_max))])
    return t[t < duration_s]


def white_noise_windows(n_windows: int, W: int = 361, sigma: float = 1e-3, seed: int = 0):
    """Flat white-noise star for the bias check of Sections 2.4 and 4.1: one
    float32 curve 1 + N(0, sigma^2) of n_windows * W samples (2-min cadence),
    and the centres of its n_windows disjoint full windows of W samples,
    which are therefore independent draws.  Returns (flux, time, centres)."""
    rng = np.random.default_rng(np.random.SeedSequence([ROOT_SEED, 7, seed]))
    n = n_windows * W
    f = (1.0 + rng.normal(0.0, sigma, n)).astype(np.float32)
    t = np.arange(n, dtype=np.float64) * (2 * MIN)
    centres = (W - 1) // 2 + W * np.arange(n_windows, dtype=np.int64)
    return f, t, centres
