"""Brute-force restatement of the method for tiny inputs (test use only).

Pure-Python loops, written separately from the C oracle in a different way:
the median is found by counting ranks (no sort), windows are gathered by
scanning every index, and segments by a second independent scan.  It pins the
oracle's window geometry, gap handling and median selection on small cases.
Section references are to arXiv 2604.06602.
"""
from __future__ import annotations

import math
import struct

GAP_DAYS = 0.5
SCALE = 0.6745


def f32(v: float) -> float:
    return struct.unpack("<f", struct.pack("<f", v))[0]


def bits(v: float) -> int:
    return struct.unpack("<I", struct.pack("<f", v))[0]


def order_key(v: float) -> int:
    """IEEE-754 totalOrder position of a float32 value (no NaNs here)."""
    b = bits(v)
    return (~b & 0xFFFFFFFF) if b & 0x80000000 else (b | 0x80000000)


def rank_median(xs):
    """Lower median: the element with exactly floor((n-1)/2) elements before
    it when ties are broken by list position (Section 2.1)."""
    n = len(xs)
    k = (n - 1) // 2
    keys = [order_key(x) for x in xs]
    for i in range(n):
        before = sum(1 for j in range(n) if keys[j] < keys[i] or (keys[j] == keys[i] and j < i))
        if before == k:
            return xs[i]
    raise AssertionError("no element has the median rank")


def valid(flux, time, j):
    if not math.isfinite(flux[j]):
        return False
    if time is not None and not math.isfinite(time[j]):
        return False
    return True


def segment_of(flux, time, W):
    """For each index: (lo, hi) of its live segment, or None."""
    n = len(flux)
    m_min = max(1, W // 3)
    seg_id = [None] * n
    sid = -1
    prev = None
    for j in range(n):
        if not valid(flux, time, j):
            continue
        if prev is None or (time is not None and time[j] - time[prev] > GAP_DAYS):
            sid += 1
        seg_id[j] = sid
        prev = j
    members = {}
    for j in range(n):
        if seg_id[j] is not None:
            members.setdefault(seg_id[j], []).append(j)
    out = [None] * n
    for sid, idx in members.items():
        if len(idx) >= m_min:
            for j in idx:
                out[j] = (idx[0], idx[-1])
    return out


def count_mad(xs, m):
    """MAD ablation scale: the smallest deviation |x - m| that at least
    floor((n-1)/2) + 1 deviations do not exceed (the lower median of the
    deviations, found by counting)."""
    k = (len(xs) - 1) // 2
    devs = [abs(x - m) for x in xs]
    return min(d for d in devs if sum(1 for e in devs if e <= d) >= k + 1)


def estimate(xs, alpha, c, iters, scale="upper_rms"):
    m = rank_median(xs)
    if scale == "mad":
        s = count_mad(xs, m)
    else:
        up = [x - m for x in xs if x > m]
        s = SCALE * math.sqrt(sum(d * d for d in up) / len(up)) if up else 0.0
    mu = m
    if s > 0:
        for _ in range(iters):
            num = den = 0.0
            for x in xs:
                u = (x - mu) / (c * s)
                ue = alpha * u if u < 0 else u
                w = (1 - ue * ue) ** 2 if abs(ue) < 1 else 0.0
                num += w * x
                den += w
            if den == 0:
                break
            mu = num / den
    return mu, m


def detrend(flux, time, W, alpha=2.0, c=5.0, iters=5, scale="upper_rms", window_days=0.0):
    flux = [f32(float(v)) for v in flux]
    time = None if time is None else [float(v) for v in time]
    n = len(flux)
    h = (W - 1) // 2
    seg = segment_of(flux, time, W)
    trend = [math.nan] * n
    med = [math.nan] * n
    for i in range(n):
        if seg[i] is None:
            continue
        lo, hi = seg[i]
        xs = [flux[j] for j in range(n)
              if lo <= j <= hi and i - h <= j <= i + h and valid(flux, time, j)
              and (window_days <= 0 or 2 * abs(time[j] - time[i]) <= window_days)]
        trend[i], med[i] = estimate(xs, alpha, c, iters, scale)
    return trend, med
