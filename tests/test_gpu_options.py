"""GPU parity of the optional paths against the FP64 oracle: the MAD scale
ablation (Sections 1, 2.2 and 3.1), per-curve alpha and c (the use-case
settings of Table 4) mixed in one batch, and the detrended flux (flux /
trend, the normalisation stage of Table 3).  Every call goes through the C
ABI (umi_detrend_gather_ex, umi_plan_run_ex).

Acceptance as for the main path: median bit-exact, trend within 1e-5 of the
oracle relative to max(|trend|, the window's sample magnitude); the detrended
flux within the error that bound implies for flux / trend plus two float32
roundings.
"""
from __future__ import annotations

import numpy as np
import pytest

import synth
from tests.test_gpu_parity import (REL_TOL, assert_parity, edge_case_batch, run_batch, to_dev,
                                   window_magnitude)

pytestmark = pytest.mark.gpu

PRESETS = [(2.0, 5.0), (3.0, 5.0), (1.0, 5.0), (10.0, 2.5)]  # Table 4


@pytest.fixture(scope="module")
def torch():
    import torch as _t
    if not _t.cuda.is_available():
        pytest.skip("no GPU")
    return _t


@pytest.fixture(scope="module")
def umi(torch):
    import paper_2604_06602_amd as _u
    return _u


def assert_detrended(g_det, o_tr, flux, mag, what=""):
    o_det = flux.astype(np.float64) / o_tr
    o_nan = np.isnan(o_tr)
    assert np.array_equal(np.isnan(g_det), o_nan), what
    ok = ~o_nan
    if not ok.any():
        return
    t = np.abs(o_tr[ok])
    bound = (REL_TOL * np.maximum(1.0, mag[ok] / np.maximum(t, 1e-30)) + 2.4e-7) * np.abs(o_det[ok])
    err = np.abs(g_det[ok].astype(np.float64) - o_det[ok])
    worst = np.argmax(err - bound)
    assert (err <= bound).all(), "%s: detrended err %.3e > bound %.3e" % (what, err[worst], bound[worst])


def test_mad_scale_config0(torch, umi, oracle_lib):
    flux, time, W = synth.curve_config0()
    g_tr, g_md = run_batch(torch, umi, flux, time, [flux.size], [W], scale="mad")
    o_tr, o_md = oracle_lib.detrend(flux, time, W, scale="mad")
    assert_parity(g_tr, g_md, o_tr, o_md, what="config0 MAD")
    # the ablation really changes the estimate
    u_tr, _ = run_batch(torch, umi, flux, time, [flux.size], [W])
    assert not np.array_equal(u_tr, g_tr)


def test_mad_scale_edge_cases(torch, umi, oracle_lib):
    packed = edge_case_batch()
    mag = window_magnitude(packed.flux, packed.time, packed.lengths, packed.W, oracle_lib)
    for a, c, it in [(2.0, 5.0, 5), (1.0, 5.0, 5), (10.0, 2.5, 5), (0.5, 5.0, 3)]:
        g_tr, g_md = run_batch(torch, umi, packed.flux, packed.time, packed.lengths, packed.W,
                               alpha=a, c=c, iters=it, scale="mad")
        o_tr, o_md = oracle_lib.detrend_batch(packed.flux, packed.time, packed.lengths, packed.W,
                                              alpha=a, c=c, iters=it, scale="mad")
        assert_parity(g_tr, g_md, o_tr, o_md, what="MAD edge cases a=%g c=%g" % (a, c), scale=mag)


def _mixed_batch(n=12):
    ids = [i for i in range(80) if synth.curve_for(3, i)[0].size < 12000][:n]
    return synth.lightcurves.pack([synth.curve_for(3, i) for i in ids])


def test_table4_presets_mixed_in_one_batch(torch, umi, oracle_lib):
    b = _mixed_batch()
    alphas = np.array([PRESETS[i % 4][0] for i in range(b.n_curves)], np.float32)
    cs = np.array([PRESETS[i % 4][1] for i in range(b.n_curves)], np.float32)
    g_tr, g_md = run_batch(torch, umi, b.flux, b.time, b.lengths, b.W, alpha=alphas, c=cs)
    o_tr, o_md = oracle_lib.detrend_batch(b.flux, b.time, b.lengths, b.W, alpha=alphas, c=cs)
    assert_parity(g_tr, g_md, o_tr, o_md, what="per-curve presets")
    # each curve equals that curve run alone with its own scalar pair, bit
    # for bit at one tile size
    fixed = umi.LaunchOptions(tile=1024)
    f_tr, _ = run_batch(torch, umi, b.flux, b.time, b.lengths, b.W, alpha=alphas, c=cs,
                        launch=fixed)
    off = b.offsets
    for ci in [0, 1, 2, 3]:
        f, t, W = b.curve(ci)
        a_tr, _ = run_batch(torch, umi, f, t, [f.size], [W], alpha=float(alphas[ci]),
                            c=float(cs[ci]), launch=fixed)
        assert np.array_equal(a_tr.view(np.uint32), f_tr[off[ci]:off[ci] + f.size].view(np.uint32))


def test_detrended_flux(torch, umi, oracle_lib):
    b = _mixed_batch(8)
    f = to_dev(torch, b.flux)
    t = to_dev(torch, b.time)
    tr, md, det = umi.detrend_batch(f, t, b.lengths, b.W, with_median=True, with_detrended=True)
    torch.cuda.synchronize()
    o_tr, o_md = oracle_lib.detrend_batch(b.flux, b.time, b.lengths, b.W)
    assert_parity(tr.cpu().numpy(), md.cpu().numpy(), o_tr, o_md, what="with detrended")
    mag = window_magnitude(b.flux, b.time, b.lengths, b.W, oracle_lib)
    assert_detrended(det.cpu().numpy(), o_tr, b.flux, mag, "detrended")
    # same as dividing the library's own trend in float32
    g = b.flux / tr.cpu().numpy()
    assert np.array_equal(np.nan_to_num(det.cpu().numpy(), nan=7.0), np.nan_to_num(g, nan=7.0))


def test_options_default_equal_plain_call(torch, umi):
    b = _mixed_batch(6)
    ref, _ = run_batch(torch, umi, b.flux, b.time, b.lengths, b.W)
    same, _ = run_batch(torch, umi, b.flux, b.time, b.lengths, b.W,
                        alpha=np.full(b.n_curves, 2.0, np.float32),
                        c=np.full(b.n_curves, 5.0, np.float32))
    assert np.array_equal(ref.view(np.uint32), same.view(np.uint32))


def test_plan_run_ex_equals_gather_ex(torch, umi):
    """A plan replay with per-curve parameters, the MAD scale and a detrended
    output equals the direct call; replays in between use other options."""
    b = _mixed_batch(10)
    cap = b.flux.size + 5000
    flux = torch.zeros(cap, dtype=torch.float32, device="cuda")
    time = torch.zeros(cap, dtype=torch.float64, device="cuda")
    flux[:b.flux.size] = to_dev(torch, b.flux)
    time[:b.flux.size] = to_dev(torch, b.time)
    offs = b.offsets.astype(np.int64)
    alphas = np.array([PRESETS[i % 4][0] for i in range(b.n_curves)], np.float32)
    cs = np.array([PRESETS[i % 4][1] for i in range(b.n_curves)], np.float32)
    trend = torch.zeros(cap, dtype=torch.float32, device="cuda")
    det = torch.zeros(cap, dtype=torch.float32, device="cuda")
    stream = torch.cuda.Stream()
    plan = umi.Plan(flux, time, trend, None, max_curves=64, max_W=721, stream=stream)
    try:
        for rep in range(3):
            for sc in ["mad", "upper_rms"]:
                trend.fill_(-1.0)
                det.fill_(-1.0)
                torch.cuda.synchronize()
                wd = np.where(np.arange(b.n_curves) % 3 == 0, 0.4, 0.0) if rep == 2 else None
                plan.run(offs, b.lengths, b.W, alpha=alphas, c=cs, scale=sc, detrended=det,
                         window_days=wd)
                stream.synchronize()
                p_tr, p_det = trend.cpu().numpy(), det.cpu().numpy()
                r_tr = torch.full((cap,), -1.0, dtype=torch.float32, device="cuda")
                r_det = torch.full((cap,), -1.0, dtype=torch.float32, device="cuda")
                umi.detrend_gather_into(flux, time, offs, b.lengths, b.W, r_tr, alpha=alphas,
                                        c=cs, scale=sc, detrended=r_det, window_days=wd)
                torch.cuda.synchronize()
                assert np.array_equal(p_tr.view(np.uint32), r_tr.cpu().numpy().view(np.uint32)), (rep, sc)
                assert np.array_equal(p_det.view(np.uint32), r_det.cpu().numpy().view(np.uint32)), (rep, sc)
                # samples beyond the curves are untouched
                assert (p_tr[b.flux.size:] == -1.0).all() and (p_det[b.flux.size:] == -1.0).all()
    finally:
        plan.destroy()


def _irregular_batch(n_curves=8, seed=77):
    """Irregular cadence (exponential steps, mean 2 min), pauses shorter than
    a segment break, isolated NaNs: non-decreasing times throughout."""
    rng = np.random.default_rng(seed)
    curves = []
    for i in range(n_curves):
        n = int(rng.integers(1500, 4000))
        t = np.cumsum(rng.exponential(2 / 1440, n))
        for _ in range(2):
            k = int(rng.integers(1, n))
            t[k:] += rng.uniform(0.01, 0.3)
        f = 1 + 1e-3 * rng.normal(size=n) + 2e-3 * np.sin(2 * np.pi * t / 1.7)
        f[rng.random(n) < 0.03] = np.nan
        curves.append((f.astype(np.float32), t, 1441))
    return synth.lightcurves.pack(curves)


def test_time_windows_irregular_cadence(torch, umi, oracle_lib):
    b = _irregular_batch()
    for L, sc in [(0.5, "upper_rms"), (0.25, "mad"), (1.0, "upper_rms")]:
        g_tr, g_md = run_batch(torch, umi, b.flux, b.time, b.lengths, b.W, window_days=L, scale=sc)
        o_tr, o_md = oracle_lib.detrend_batch(b.flux, b.time, b.lengths, b.W, window_days=L,
                                              scale=sc)
        assert_parity(g_tr, g_md, o_tr, o_md, what="time windows L=%g %s" % (L, sc))
    # a mixed batch: some curves with time windows, some with index windows
    wd = np.array([0.5 if i % 2 else 0.0 for i in range(b.n_curves)])
    g_tr, g_md = run_batch(torch, umi, b.flux, b.time, b.lengths, b.W, window_days=wd)
    o_tr, o_md = oracle_lib.detrend_batch(b.flux, b.time, b.lengths, b.W, window_days=wd)
    assert_parity(g_tr, g_md, o_tr, o_md, what="mixed time/index windows")


def test_time_windows_equal_index_windows_at_regular_cadence(torch, umi):
    b = _mixed_batch(8)
    dt = 2 / 1440
    ref, ref_md = run_batch(torch, umi, b.flux, b.time, b.lengths, b.W)
    wd = (np.asarray(b.W, np.float64) - 1) * dt * 1.0000001
    tw, tw_md = run_batch(torch, umi, b.flux, b.time, b.lengths, b.W, window_days=wd)
    assert np.array_equal(ref.view(np.uint32), tw.view(np.uint32))
    assert np.array_equal(ref_md.view(np.uint32), tw_md.view(np.uint32))
