"""Synthetic injection-recovery harness (the protocol of Section 3.2).

Box transits (period 3 d, duration 3 h) at depths from 5 to 1000 ppm are
multiplied into synthetic TESS- and Kepler-like stars (``synth.injection``),
every star is detrended on the GPU with each parameter setting, and the
recovered depth is compared with the injected one.  The score is the
paper's: the median over stars of the absolute percentage depth error.

The recovered depth is read off the detrended flux d = flux / trend as
(mean of d out of transit - mean of d in transit) / mean of d out of transit,
over valid samples; referencing the out-of-transit level removes the
estimator's overall offset (Section 2.4), which is not a depth error.

Settings: the paper's default (alpha 2, c 5) and aggressive (alpha 10, c 2.5)
ones, and two symmetric references under this library's conventions (alpha
1 with the upper-RMS scale, and alpha 1 with the MAD scale).  They stand in
for the qualitative comparison of Tables 1-2; the paper's comparison
packages and real stars are not available, so its absolute numbers are not
expected here.

Usage on a GPU:  python -m paper_2604_06602_amd.injection [--stars N]
"""
from __future__ import annotations

import argparse
import json
import sys

import numpy as np

METHODS = {
    "umi_default": dict(alpha=2.0, c=5.0, scale="upper_rms"),
    "umi_aggressive": dict(alpha=10.0, c=2.5, scale="upper_rms"),
    "symmetric": dict(alpha=1.0, c=5.0, scale="upper_rms"),
    "symmetric_mad": dict(alpha=1.0, c=5.0, scale="mad"),
}


def recovered_depth(detrended: np.ndarray, in_mask: np.ndarray) -> float:
    ok = np.isfinite(detrended)
    out = detrended[ok & ~in_mask]
    inn = detrended[ok & in_mask]
    if out.size == 0 or inn.size == 0:
        return float("nan")
    base = float(out.astype(np.float64).mean())
    return (base - float(inn.astype(np.float64).mean())) / base


def percent_error(recovered: float, depth_ppm: float) -> float:
    d = depth_ppm * 1e-6
    return abs(recovered - d) / d * 100.0


def _batch(mission, n_stars, depth_ppm, first=0, duration_d=None, W=None):
    from synth import injection as si
    kw = {} if duration_d is None else {"duration_d": duration_d}
    curves = [si.injected(mission, first + i, depth_ppm, **kw) for i in range(n_stars)]
    flux = np.concatenate([c[0] for c in curves])
    time = np.concatenate([c[1] for c in curves])
    lengths = np.array([c[0].size for c in curves], np.int64)
    W = np.array([c[2] if W is None else W for c in curves], np.int32)
    masks = [c[3] for c in curves]
    return flux, time, lengths, W, masks


def run(mission: str, n_stars: int, depths=None, methods=None, first: int = 0, detrend=None,
        duration_d=None, W=None):
    """Median per-star absolute % depth error for each method and depth.

    ``detrend(flux, time, lengths, W, alpha, c, scale) -> detrended flux`` (host
    arrays) defaults to the GPU library; tests may pass another one.
    ``duration_d`` overrides the 3-hour transit duration and ``W`` the
    mission's window (e.g. the window of a longer ``window_length``)."""
    from synth import injection as si
    depths = si.DEPTHS_PPM if depths is None else depths
    methods = METHODS if methods is None else methods
    detrend = _gpu_detrend if detrend is None else detrend
    table = {m: {} for m in methods}
    errors = {m: {} for m in methods}
    for d in depths:
        flux, time, lengths, Ws, masks = _batch(mission, n_stars, d, first, duration_d, W)
        off = np.concatenate([[0], np.cumsum(lengths)])
        for name, p in methods.items():
            det = detrend(flux, time, lengths, Ws, p["alpha"], p["c"], p["scale"])
            errs = [percent_error(recovered_depth(det[off[i]:off[i + 1]], masks[i]), d)
                    for i in range(len(masks))]
            errors[name][d] = errs
            table[name][d] = float(np.nanmedian(errs))
    return table, errors


def _gpu_detrend(flux, time, lengths, W, alpha, c, scale):
    import torch

    from . import _lib
    f = torch.from_numpy(np.ascontiguousarray(flux)).cuda()
    t = torch.from_numpy(np.ascontiguousarray(time)).cuda()
    _, _, det = _lib.detrend_batch(f, t, lengths, W, alpha=alpha, c=c, scale=scale,
                                   with_detrended=True)
    return det.cpu().numpy()


def format_table(table) -> str:
    from synth import injection as si
    depths = sorted(next(iter(table.values())).keys()) if table else si.DEPTHS_PPM
    lines = ["%-16s" % "method" + "".join("%9d" % d for d in depths)]
    for m, row in table.items():
        lines.append("%-16s" % m + "".join("%9.1f" % row[d] for d in depths))
    return "\n".join(lines)


def main(argv=None):
    ap = argparse.ArgumentParser(description="synthetic injection-recovery (Section 3.2 protocol)")
    ap.add_argument("--stars", type=int, default=1000)
    ap.add_argument("--missions", default="tess,kepler")
    args = ap.parse_args(argv)
    out = {}
    for mission in args.missions.split(","):
        table, _ = run(mission, args.stars)
        print("%s, %d stars: median per-star absolute depth error (%%)" % (mission, args.stars),
              file=sys.stderr)
        print(format_table(table), file=sys.stderr, flush=True)
        out[mission] = {m: {str(d): v for d, v in row.items()} for m, row in table.items()}
    print(json.dumps({"injection_recovery": out, "stars": args.stars}))
    return 0


if __name__ == "__main__":
    sys.exit(main())
